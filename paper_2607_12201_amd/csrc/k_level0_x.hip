// Instantiations of the level-0 element kernel and the chain kernel for the largest shapes:
// a 24 x 24 thread grid keeps the register block count at 6-7, where every block index is
// resolved at compile time (larger counts on a 16 x 16 grid spill the register array).
#include "level0_impl.h"
#include "chain_impl.h"

namespace cl {
void launch_level0_24_6(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 24, 6>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 24, 6>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
}
void launch_level0_24_7(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_level0r<float, 24, 7>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
  else hipLaunchKernelGGL((k_level0r<double, 24, 7>), dim3((unsigned)tb.n_elem), dim3(576), level0r_lds_bytes(S), st, S, tb, ws, fused);
}

int attrs_level0_24_6(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 24, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 24, 6>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}
int attrs_level0_24_7(size_t bytes) {
  if (hipFuncSetAttribute((const void*)k_level0r<double, 24, 7>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  if (hipFuncSetAttribute((const void*)k_level0r<float, 24, 7>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return -1;
  return 0;
}

void launch_chain_24_6(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 24, 6>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 24, 6>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
}
void launch_chain_24_7(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st) {
  if (prec) hipLaunchKernelGGL((k_chain<float, 24, 7>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
  else hipLaunchKernelGGL((k_chain<double, 24, 7>), dim3(grid), dim3(576), lds, st, S, tb, ws, mode, level);
}
}  // namespace cl
