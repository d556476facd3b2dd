// Host launch and attribute entry points of the register-resident element kernel k_level0r and
// the chain kernel k_chain for one thread grid TS x TS (TS * TS threads) with NB register blocks
// per side, in FP64 and FP32 factors.  Every (TS, NB) pair is instantiated in one of the
// k_level0_*.hip units: each pair takes minutes to compile, so the units build in parallel.
#pragma once
#include "level0_impl.h"
#include "chain_impl.h"

#define CL_LEVEL0_INSTANCE(TS, NB)                                                                        \
  void launch_level0_##TS##_##NB(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused,        \
                                  hipStream_t st) {                                                       \
    if (prec)                                                                                             \
      hipLaunchKernelGGL((k_level0r<float, TS, NB>), dim3((unsigned)tb.n_elem), dim3(TS * TS),            \
                         level0r_lds_bytes(S), st, S, tb, ws, fused);                                     \
    else                                                                                                  \
      hipLaunchKernelGGL((k_level0r<double, TS, NB>), dim3((unsigned)tb.n_elem), dim3(TS * TS),           \
                         level0r_lds_bytes(S), st, S, tb, ws, fused);                                     \
  }                                                                                                       \
  int attrs_level0_##TS##_##NB(size_t bytes) {                                                            \
    const hipFuncAttribute a = hipFuncAttributeMaxDynamicSharedMemorySize;                                \
    if (hipFuncSetAttribute((const void*)k_level0r<double, TS, NB>, a, (int)bytes) != hipSuccess) return -1; \
    if (hipFuncSetAttribute((const void*)k_level0r<float, TS, NB>, a, (int)bytes) != hipSuccess) return -1;  \
    if (hipFuncSetAttribute((const void*)k_chain<double, TS, NB>, a, (int)bytes) != hipSuccess) return -1;   \
    if (hipFuncSetAttribute((const void*)k_chain<float, TS, NB>, a, (int)bytes) != hipSuccess) return -1;    \
    return 0;                                                                                             \
  }                                                                                                       \
  void launch_chain_##TS##_##NB(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, \
                                unsigned grid, size_t lds, hipStream_t st) {                              \
    if (prec)                                                                                             \
      hipLaunchKernelGGL((k_chain<float, TS, NB>), dim3(grid), dim3(TS * TS), lds, st, S, tb, ws, mode, level); \
    else                                                                                                  \
      hipLaunchKernelGGL((k_chain<double, TS, NB>), dim3(grid), dim3(TS * TS), lds, st, S, tb, ws, mode, level); \
  }
