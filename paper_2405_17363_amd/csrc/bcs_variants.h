// Compiled kernel variants.  Each translation unit bcs_l<LANES>.hip defines
// BCS_LANES and includes this file, which instantiates the solve kernels for
// every (rows per lane, max steps per lane) pair below and exports them.
#pragma once

#include "bcs_internal.h"
#include "bcs_fp64.h"

#ifndef BCS_LANES
#error "define BCS_LANES"
#endif

// (row slots per lane, max schedule steps per lane)
#define BCS_RPL_KMAX_LIST(X)                                                       \
  X(1, 16) X(1, 32) X(2, 16) X(2, 32) X(2, 48) X(3, 32) X(3, 48) X(3, 64)           \
  X(4, 32) X(4, 48) X(4, 64) X(4, 96) X(5, 48) X(5, 64) X(5, 96) X(6, 64) X(6, 96)  \
  X(6, 128) X(7, 64) X(7, 96) X(7, 128) X(8, 64) X(8, 96) X(8, 128)

#define BCS_VARIANT_ENTRY(R, K)                                                      \
  {BCS_LANES, R, K, &bcs::launch_fp64<BCS_LANES, R, K>, nullptr,                     \
   (const void*)&bcs::k_fp64<BCS_LANES, R, K>},
