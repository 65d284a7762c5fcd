"""Debug builds on the CPU: the oracle and the host side of the HIP library
(pattern validation, gather schedules, the ILU(0) factorisation program, the
mass-action tables, plan option checks) run under AddressSanitizer and
UndefinedBehaviorSanitizer, in a child process that preloads the ASan
runtime.  Any report fails the test (UBSan errors are made fatal).  No GPU
is involved: only code paths that return before the first device call run."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run_child(code, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], capture_output=True, text=True, env=env,
                       cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


@pytest.fixture(scope="module")
def asan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime for gcc")
    return rt


def test_oracle_under_asan_and_ubsan(asan, tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", *SAN, "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", lib,
                    os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    out = _run_child("""
        import numpy as np, oracle
        from workload import config_inputs, gen_mechanism
        m, c = config_inputs(1, ncells=40)[0]
        rp, ci, V, G, B = m.row_ptr, m.col_idx, c["values"], c["gamma"], c["b"]
        for pc in (0, 1, 2):
            oracle.solve_batch(rp, ci, V, G, B, precond=pc)
        oracle.solve_batch(rp, ci, V, G, B, x0=0.5 * B)
        oracle.lu_batch(rp, ci, V, G, B)
        oracle.lu_batch(rp, ci, V, G, B, transpose=True)
        x, _, _, _ = oracle.solve_batch(rp, ci, V, G, B)
        oracle.adjoint_batch(rp, ci, V, G, x, B)
        for budget in ("inner", "cell"):
            oracle.mixed_batch(rp, ci, V, G, B, budget=budget)
        oracle.solve_groups(rp, ci, V, G, B, 4)
        f, J = oracle.assemble(m.reactants, m.products, m.k, rp, ci, c["y"])
        oracle.assemble(m.reactants, m.products, np.tile(m.k, (40, 1)), rp, ci, c["y"])
        print("oracle ok")
    """, {"LD_PRELOAD": asan, "ORACLE_LIB": lib, "OMP_NUM_THREADS": "2"})
    assert "oracle ok" in out


def _clang_asan_runtime():
    import glob

    paths = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return paths[-1] if paths else None


def test_library_host_code_under_asan(tmp_path):
    """libbcs.so built with host-side ASan/UBSan by hipcc (clang; device code
    unchanged), run with clang's ASan runtime (which carries the UBSan
    handlers) preloaded; only host paths that end before any HIP device call
    run."""
    from paper_2405_17363_amd import build as hip_build

    asan = _clang_asan_runtime()
    if asan is None:
        pytest.skip("no clang ASan runtime")

    lib = str(tmp_path / "libbcs_san.so")
    objs = []
    inc = os.path.join(hip_build.BUILD, "")
    hip_build._write_jit_sources()
    host_san = []
    for flag in SAN[:3]:
        host_san += ["-Xarch_host", flag]
    import concurrent.futures as cf

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        subprocess.run([hip_build.HIPCC, *hip_build.FLAGS, *host_san, f"-I{inc}", "-x", "hip", "-c",
                        os.path.join(hip_build.CSRC, src), "-o", obj], check=True, capture_output=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, hip_build.SOURCES))
    subprocess.run([hip_build.HIPCC, "-shared", f"--offload-arch={hip_build.ARCH}", "-fPIC", "-o", lib, *objs,
                    "-lhiprtc", "-Xarch_host", "-fsanitize=address,undefined"], check=True, capture_output=True)
    out = _run_child("""
        import ctypes, numpy as np
        import paper_2405_17363_amd._binding as b
        b._LIB_PATH = %r
        import paper_2405_17363_amd as bcs
        from workload import gen_mechanism
        for n, R in ((30, 50), (80, 150), (200, 400)):
            m = gen_mechanism(n, R)
            for lanes in (16, 32, 64):
                for part in (0, 1, 2, 3):
                    try:
                        bcs.schedule_describe(m.row_ptr, m.col_idx, lanes, transpose=part, shapes=3 if part < 2 else 1)
                    except bcs.BcsError:
                        pass
                try:
                    bcs.ilu_describe(m.row_ptr, m.col_idx, lanes)
                except bcs.BcsError:
                    pass
        L = bcs.lib()
        # plan and mechanism validation (rejected before any device call)
        from paper_2405_17363_amd._binding import _Options
        o = _Options(); L.bcs_options_default(ctypes.byref(o))
        h = ctypes.c_void_p()
        rp = np.array([0, 2, 3], np.int32); ci = np.array([1, 0, 1], np.int32)
        assert L.bcs_plan_create(2, 3, rp.ctypes.data, ci.ctypes.data, ctypes.byref(o), ctypes.byref(h)) < 0
        m = gen_mechanism(30, 50)
        ci2 = np.delete(m.col_idx, 1); rp2 = m.row_ptr.copy(); rp2[1:] -= 1
        re = np.ascontiguousarray(m.reactants, np.int32); pr = np.ascontiguousarray(m.products, np.int32)
        assert L.bcs_mechanism_create(30, len(ci2), rp2.ctypes.data, ci2.ctypes.data, 50, re.ctypes.data,
                                      pr.ctypes.data, ctypes.byref(h)) == -2
        print("host ok")
    """ % lib, {"LD_PRELOAD": asan})
    assert "host ok" in out
