// Pattern-specialised solve kernels compiled at plan creation with hipRTC.
//
// The precompiled variants read a pattern's slot segment boundaries at run
// time, which costs a scalar test and branch on every SpMV step and pads every
// lane to the variant's step count.  A plan instead compiles the same kernel
// body with its exact segment lengths as template constants, so that each SpMV
// is straight-line code.  Compiled code objects are cached in memory for the
// process and on disk (directory $BCS_JIT_CACHE, else $HOME/.cache/bcs_jit,
// else /tmp/bcs_jit), keyed by a hash of the generated source, the compile
// options and the device architecture.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "bcs_internal.h"
#include "bcs_jit_sources.inc"  // kJitHeaderCount, kJitHeaderNames[], kJitHeaderSources[], kJitSourceHash

namespace bcs {
namespace {

std::mutex g_mu;
std::map<std::string, JitKernel> g_cache;

// Options of every kernel compile (after --offload-arch), then the scheduling
// option of the FP64 bodies.  Those are long straight-line bodies whose
// occupancy is fixed by their register use, so the scheduler is asked to
// order them for instruction-level parallelism (max-ilp) rather than for the
// default occupancy/latency balance: with it, the n = 80 FP64 kernel at 32
// lanes per cell runs 4% faster and the adjoint 3% faster, at the same
// occupancy and with bitwise the same results.  The FP32 inner solve of the
// mixed body ran 1.5% slower with it and keeps the default.
const char* const kJitOptions[] = {"-O3",     "-std=c++17", "-Xclang", "-target-feature",
                                   "-Xclang", "-packed-fp32-ops"};
constexpr int kJitOptionCount = (int)(sizeof(kJitOptions) / sizeof(kJitOptions[0]));
const char* const kIlpOptions[] = {"-mllvm", "-amdgpu-sched-strategy=max-ilp"};
constexpr int kIlpOptionCount = (int)(sizeof(kIlpOptions) / sizeof(kIlpOptions[0]));

std::string jit_options_key(bool ilp) {
  std::string k;
  for (int i = 0; i < kJitOptionCount; ++i) k += std::string(kJitOptions[i]) + " ";
  if (ilp)
    for (int i = 0; i < kIlpOptionCount; ++i) k += std::string(kIlpOptions[i]) + " ";
  return k;
}

uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull) {
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

std::string cache_dir() {
  if (const char* d = std::getenv("BCS_JIT_CACHE")) return d;
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/bcs_jit";
  return "/tmp/bcs_jit";
}

void mkdirs(const std::string& path) {
  std::string cur;
  std::stringstream ss(path);
  std::string part;
  if (!path.empty() && path[0] == '/') cur = "/";
  while (std::getline(ss, part, '/')) {
    if (part.empty()) continue;
    cur += part + "/";
    mkdir(cur.c_str(), 0755);
  }
}

bool read_file(const std::string& path, std::vector<char>* out) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  out->assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
  return !out->empty();
}

void write_file_atomic(const std::string& path, const std::vector<char>& data) {
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return;
    f.write(data.data(), (std::streamsize)data.size());
    if (!f) return;
  }
  std::rename(tmp.c_str(), path.c_str());
}

int compile(const std::string& src, const std::string& arch, bool ilp, std::vector<char>* code, std::string* log) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "bcs_jit.hip", kJitHeaderCount, kJitHeaderSources,
                          kJitHeaderNames) != HIPRTC_SUCCESS) {
    *log = "hiprtcCreateProgram failed";
    return -1;
  }
  const std::string arch_opt = "--offload-arch=" + arch;
  const char* opts[1 + kJitOptionCount + kIlpOptionCount] = {arch_opt.c_str()};
  int nopt = 1;
  for (int i = 0; i < kJitOptionCount; ++i) opts[nopt++] = kJitOptions[i];
  if (ilp)
    for (int i = 0; i < kIlpOptionCount; ++i) opts[nopt++] = kIlpOptions[i];
  const hiprtcResult r = hiprtcCompileProgram(prog, nopt, opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(prog, &ls);
  if (ls > 1) {
    std::vector<char> buf(ls + 1, 0);
    hiprtcGetProgramLog(prog, buf.data());
    *log = buf.data();
  }
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return -1;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  code->resize(cs);
  hiprtcGetCode(prog, code->data());
  hiprtcDestroyProgram(&prog);
  return 0;
}

}  // namespace

namespace {

// Compile (or load from the caches) `source`, whose kernel is `name`;
// `ilp` adds the FP64 bodies' scheduling option.
int load_source(const std::string& source, const char* name, bool ilp, size_t lds_bytes, JitKernel* out, char* err,
                size_t errlen, int threads = kWgThreads) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    snprintf(err, errlen, "no HIP device");
    return BCS_ERR_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    snprintf(err, errlen, "cannot query device properties");
    return BCS_ERR_HIP;
  }
  std::string arch = prop.gcnArchName;
  const std::string base_arch = arch.substr(0, arch.find(':'));
  const std::string key = std::string(kJitSourceHash) + "|" + arch + "|" + jit_options_key(ilp) + "|" + source;

  std::lock_guard<std::mutex> lock(g_mu);
  const std::string mkey = std::to_string(dev) + "|" + key;
  auto it = g_cache.find(mkey);
  if (it == g_cache.end()) {
    char fname[64];
    snprintf(fname, sizeof(fname), "%016llx.co", (unsigned long long)fnv1a(key));
    const std::string dir = cache_dir();
    const std::string path = dir + "/" + fname;
    std::vector<char> code;
    if (std::getenv("BCS_VERBOSE")) std::fprintf(stderr, "[bcs] jit %s %s\n", name, path.c_str());
    if (const char* dump = std::getenv("BCS_JIT_DUMP")) {
      // debug aid: the kernel's source beside its cache name, to rebuild it offline
      mkdirs(dump);
      std::vector<char> text(source.begin(), source.end());
      write_file_atomic(std::string(dump) + "/" + fname + ".hip", text);
    }
    if (!read_file(path, &code)) {
      std::string log;
      if (compile(source, base_arch, ilp, &code, &log) != 0) {
        snprintf(err, errlen, "hipRTC compile failed: %.400s", log.c_str());
        return BCS_ERR_HIP;
      }
      mkdirs(dir);
      write_file_atomic(path, code);
    }
    hipModule_t mod;
    if (hipModuleLoadData(&mod, code.data()) != hipSuccess) {
      snprintf(err, errlen, "hipModuleLoadData failed for the compiled kernel");
      return BCS_ERR_HIP;
    }
    JitKernel k;
    if (hipModuleGetFunction(&k.fn, mod, name) != hipSuccess) {
      snprintf(err, errlen, "compiled kernel not found in module");
      return BCS_ERR_HIP;
    }
    it = g_cache.emplace(mkey, k).first;
  }
  JitKernel k = it->second;
  int nb = 0;
  if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k.fn, threads, lds_bytes) != hipSuccess) {
    snprintf(err, errlen, "occupancy query failed");
    return BCS_ERR_HIP;
  }
  k.max_blocks = nb > 0 ? nb : 1;
  int local = 0;
  if (hipFuncGetAttribute(&local, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, k.fn) == hipSuccess) k.scratch = local;
  *out = k;
  return BCS_OK;
}

// First lines of every kernel source: the device-source version (no
// compiler cache may reuse code across header versions) and, with
// BCS_DEBUG_VISITS set (not "0") in the environment, the per-cell output
// counter of bcs_debug_count_visits, which costs registers and is left out
// otherwise.
void preamble(std::ostringstream& src, int wg_waves = kWavesPerWg) {
  src << "// device sources " << kJitSourceHash << "\n";
  if (wg_waves != kWavesPerWg) src << "#define BCS_WG_WAVES " << wg_waves << "\n";
  const char* v = std::getenv("BCS_DEBUG_VISITS");
  if (v && std::string(v) != "0") src << "#define BCS_COUNT_VISITS 1\n";
}

void sched_type(std::ostringstream& src, int lanes, int flags, const int* seg, int rpl) {
  src << "bcs::dev::StaticSched<" << lanes << ", " << flags;
  for (int j = 0; j < rpl; ++j) src << ", " << seg[j];
  src << ">";
}

}  // namespace

int jit_kernel(const char* body, int adjoint, int grouped, int lanes, int flags, const int* seg, int rpl,
               int waves_per_eu,
               size_t lds_bytes, JitKernel* out, char* err, size_t errlen, const std::vector<int>* mech_terms,
               int wg_waves) {
  const bool mech = mech_terms != nullptr;
  std::ostringstream src;
  preamble(src, wg_waves);
  src << "#include \"bcs_fp64.h\"\n#include \"bcs_mixed.h\"\n"
      << "extern \"C\" __global__ void __launch_bounds__(bcs::kWgThreads";
  if (waves_per_eu > 0) src << ", " << waves_per_eu;
  // kernel names tell the forms apart in profiles
  const bool fp64 = std::string(body) == "fp64_body";
  const char* name = fp64 ? (adjoint ? "bcs_solve_adjoint"
                                     : (grouped ? "bcs_solve_fp64_grouped" : (mech ? "bcs_solve_fp64_mech" : "bcs_solve_fp64")))
                          : "bcs_solve_mixed";
  src << ") " << name << "(bcs::KParams P) {\n  bcs::" << body << "<";
  sched_type(src, lanes, flags, seg, rpl);
  if (fp64) {
    src << ", " << (adjoint ? 1 : 0) << ", " << (grouped ? "true" : "false") << ", ";
    if (mech) {
      src << "bcs::dev::MechTerms<";
      for (size_t q = 0; q < mech_terms->size(); ++q) src << (q ? ", " : "") << (*mech_terms)[q];
      src << ">";
    } else {
      src << "bcs::dev::NoMechTerms";
    }
  }
  src << ">(P);\n}\n";
  return load_source(src.str(), name, fp64, lds_bytes, out, err, errlen, 64 * wg_waves);
}

int jit_ilu_kernel(int lanes, const int* flags, const int* const* seg, const int* rpl, int nnz,
                   const int* widths, int nstep, int waves_per_eu, size_t lds_bytes, JitKernel* out, char* err,
                   size_t errlen) {
  std::ostringstream src;
  preamble(src);
  src << "#include \"bcs_ilu.h\"\n"
      << "extern \"C\" __global__ void __launch_bounds__(bcs::kWgThreads";
  if (waves_per_eu > 0) src << ", " << waves_per_eu;
  src << ") bcs_solve_ilu0(bcs::KParams P) {\n"
      << "  bcs::ilu_body<";
  for (int m = 0; m < 3; ++m) {
    sched_type(src, lanes, flags[m], seg[m], rpl[m]);
    src << ", ";
  }
  src << "bcs::dev::FactProg<" << nnz;
  for (int q = 0; q < nstep; ++q) src << ", " << widths[q];
  src << ">>(P);\n}\n";
  return load_source(src.str(), "bcs_solve_ilu0", true, lds_bytes, out, err, errlen);
}

int jit_multi_kernel(int nmech, const int* lanes, const int* flags, const int* const* seg, const int* rpl,
                     size_t lds_bytes,
                     JitKernel* out, char* err, size_t errlen) {
  std::ostringstream src;
  preamble(src);
  src << "#include \"bcs_fp64.h\"\n"
      << "extern \"C\" __global__ void __launch_bounds__(bcs::kWgThreads) bcs_solve_multi(bcs::MultiParams P) {\n"
      << "  bcs::multi_body<";
  for (int m = 0; m < nmech; ++m) {
    if (m) src << ", ";
    sched_type(src, lanes[m], flags[m], seg[m], rpl[m]);
  }
  src << ">(P);\n}\n";
  return load_source(src.str(), "bcs_solve_multi", true, lds_bytes, out, err, errlen);
}

}  // namespace bcs
