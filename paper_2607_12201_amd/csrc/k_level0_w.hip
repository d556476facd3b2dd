// Instantiations of the register-resident element and chain kernels for thread grids
// TS x TS with NB register blocks per side: 24x24/4, 24x24/5.
// Every block index of the register array is a compile-time constant for these NB.
#include "level0_impl.h"
#include "chain_impl.h"

namespace cl {
void launch_level0_24_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 24, 4>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 24, 4>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_24_4(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 24, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 24, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 24, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 24, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_24_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 24, 4>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 24, 4>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
}
void launch_level0_24_5(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 24, 5>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 24, 5>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
int attrs_level0_24_5(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 24, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 24, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<double, 24, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_chain<float, 24, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
void launch_chain_24_5(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 24, 5>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 24, 5>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
}
}  // namespace cl
