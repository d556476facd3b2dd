// Instantiations of the register-resident element and chain kernels for thread grids
// TS x TS with NB register blocks per side: 8x8/1, 8x8/2, 8x8/3, 8x8/4.
// Every block index of the register array is a compile-time constant for these NB.
#include "level0_impl.h"
#include "chain_impl.h"

namespace cl {
void launch_level0_8_1(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 8, 1>), dim3((unsigned)tb.n_elem), dim3(64), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 8, 1>), dim3((unsigned)tb.n_elem), dim3(64), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_8_1(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 8, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 8, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 8, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 8, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_8_1(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 8, 1>), dim3(grid), dim3(64), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 8, 1>), dim3(grid), dim3(64), lds, st, S, tb, ws, mode, level);
}
void launch_level0_8_2(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 8, 2>), dim3((unsigned)tb.n_elem), dim3(64), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 8, 2>), dim3((unsigned)tb.n_elem), dim3(64), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_8_2(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 8, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 8, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 8, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 8, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_8_2(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 8, 2>), dim3(grid), dim3(64), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 8, 2>), dim3(grid), dim3(64), lds, st, S, tb, ws, mode, level);
}
void launch_level0_8_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 8, 3>), dim3((unsigned)tb.n_elem), dim3(64), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 8, 3>), dim3((unsigned)tb.n_elem), dim3(64), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_8_3(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 8, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 8, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 8, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 8, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_8_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 8, 3>), dim3(grid), dim3(64), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 8, 3>), dim3(grid), dim3(64), lds, st, S, tb, ws, mode, level);
}
void launch_level0_8_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 8, 4>), dim3((unsigned)tb.n_elem), dim3(64), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 8, 4>), dim3((unsigned)tb.n_elem), dim3(64), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_8_4(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 8, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 8, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 8, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 8, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_8_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 8, 4>), dim3(grid), dim3(64), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 8, 4>), dim3(grid), dim3(64), lds, st, S, tb, ws, mode, level);
}
}  // namespace cl
