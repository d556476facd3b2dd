// Instantiations of the register-resident element and chain kernels for thread grids
// TS x TS with NB register blocks per side: 16x16/3, 16x16/4, 16x16/5, 16x16/6.
// Every block index of the register array is a compile-time constant for these NB.
#include "level0_impl.h"
#include "chain_impl.h"

namespace cl {
void launch_level0_16_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 16, 3>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 16, 3>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_16_3(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 16, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 16, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 16, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 16, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_16_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 16, 3>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 16, 3>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
}
void launch_level0_16_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 16, 4>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 16, 4>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_16_4(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 16, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 16, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 16, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 16, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_16_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 16, 4>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 16, 4>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
}
void launch_level0_16_5(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 16, 5>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 16, 5>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_16_5(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 16, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 16, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 16, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 16, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_16_5(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 16, 5>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 16, 5>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
}
void launch_level0_16_6(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 16, 6>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 16, 6>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_16_6(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 16, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 16, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 16, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 16, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_16_6(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 16, 6>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 16, 6>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
}
}  // namespace cl
