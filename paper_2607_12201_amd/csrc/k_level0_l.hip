// Instantiations of the register-resident element and chain kernels for thread grids
// TS x TS with NB register blocks per side: 16x16/7, 16x16/8.
// Every block index of the register array is a compile-time constant for these NB.
#include "level0_impl.h"
#include "chain_impl.h"

namespace cl {
void launch_level0_16_7(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 16, 7>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 16, 7>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_16_7(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 16, 7>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 16, 7>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 16, 7>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 16, 7>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_16_7(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 16, 7>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 16, 7>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
}
void launch_level0_16_8(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 16, 8>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 16, 8>), dim3((unsigned)tb.n_elem), dim3(256), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_16_8(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 16, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 16, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 16, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 16, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_16_8(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 16, 8>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 16, 8>), dim3(grid), dim3(256), lds, st, S, tb, ws, mode, level);
}
}  // namespace cl
