// Instantiations of the register-resident element and chain kernels for thread grids
// TS x TS with NB register blocks per side: 16x16/1, 16x16/2, 24x24/2, 24x24/3.
// Every block index of the register array is a compile-time constant for these NB.
#include "level0_impl.h"
#include "chain_impl.h"

namespace cl {
void launch_level0_16_1(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 16, 1>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 16, 1>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_16_1(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 16, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 16, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 16, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 16, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_16_1(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 16, 1>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 16, 1>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
}
void launch_level0_16_2(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 16, 2>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 16, 2>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_16_2(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 16, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 16, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 16, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 16, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_16_2(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 16, 2>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 16, 2>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
}
void launch_level0_24_2(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 24, 2>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 24, 2>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_24_2(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 24, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 24, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 24, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 24, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_24_2(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 24, 2>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 24, 2>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
}
void launch_level0_24_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 24, 3>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 24, 3>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_24_3(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 24, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 24, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 24, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 24, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_24_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 24, 3>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 24, 3>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
}
}  // namespace cl
