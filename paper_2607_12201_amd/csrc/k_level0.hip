// Level-0 dispatch: picks the thread-grid size and register block count for the shape.
#include "kernels.h"

namespace cl {
void launch_level0_8_1(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_8_2(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_8_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_8_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_16_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_16_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_16_5(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_16_6(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_16_7(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_16_8(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_24_6(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);
void launch_level0_24_7(const Shape& S, const Tab& tb, const Ws& ws, int prec, int fused, hipStream_t st);

int attrs_level0_8_1(size_t bytes);
int attrs_level0_8_2(size_t bytes);
int attrs_level0_8_3(size_t bytes);
int attrs_level0_8_4(size_t bytes);
int attrs_level0_16_3(size_t bytes);
int attrs_level0_16_4(size_t bytes);
int attrs_level0_16_5(size_t bytes);
int attrs_level0_16_6(size_t bytes);
int attrs_level0_16_7(size_t bytes);
int attrs_level0_16_8(size_t bytes);
int attrs_level0_24_6(size_t bytes);
int attrs_level0_24_7(size_t bytes);

void launch_chain_8_1(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_8_2(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_8_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_8_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_16_3(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_16_4(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_16_5(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_16_6(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_16_7(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_16_8(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_24_6(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);
void launch_chain_24_7(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, size_t lds, hipStream_t st);

size_t level0r_lds_bytes(const Shape& S) {
  const size_t ns = S.ns, np = S.np, jl = (size_t)S.K * S.nr;
  size_t nd = 8 * (size_t)S.R + 8 + S.b + 7 * jl + ns + 3 * ns * ns + 3 * ns * np + np + np * np +
              S.lsp + (size_t)S.mmax * (S.K + 1);
  size_t ni = 3 * (size_t)S.nr + 2 * (ns + 1) + (np + 1) + S.lsp + 2 * (size_t)S.lrq + S.lpc +
              S.mmax + S.R;
  return sizeof(double) * nd + sizeof(int) * ni;
}

bool level0r_supported(const Shape& S) { return S.R <= 160 && 3 * S.ns + S.np <= 160; }

int launch_level0(const Shape& S, const Tab& tb, const Ws& ws, int prec, bool fused, hipStream_t st) {
  const int f = fused ? 1 : 0;
  if (S.R <= 32) {
    switch ((int)cl_ceil_div(S.R, 8)) {
      case 1: launch_level0_8_1(S, tb, ws, prec, f, st); return 0;
      case 2: launch_level0_8_2(S, tb, ws, prec, f, st); return 0;
      case 3: launch_level0_8_3(S, tb, ws, prec, f, st); return 0;
      case 4: launch_level0_8_4(S, tb, ws, prec, f, st); return 0;
    }
  }
  if (S.R > 128) {
    switch ((int)cl_ceil_div(S.R, 24)) {
      case 6: launch_level0_24_6(S, tb, ws, prec, f, st); return 0;
      case 7: launch_level0_24_7(S, tb, ws, prec, f, st); return 0;
    }
    return -1;
  }
  switch ((int)cl_ceil_div(S.R, 16)) {
    case 3: launch_level0_16_3(S, tb, ws, prec, f, st); return 0;
    case 4: launch_level0_16_4(S, tb, ws, prec, f, st); return 0;
    case 5: launch_level0_16_5(S, tb, ws, prec, f, st); return 0;
    case 6: launch_level0_16_6(S, tb, ws, prec, f, st); return 0;
    case 7: launch_level0_16_7(S, tb, ws, prec, f, st); return 0;
    case 8: launch_level0_16_8(S, tb, ws, prec, f, st); return 0;
  }
  return -1;
}

int level0_prepare_attrs(const Shape& S) {
  const size_t by = level0r_lds_bytes(S);
  if (by <= 64 * 1024) return 0;
  if (S.R <= 32) {
    switch ((int)cl_ceil_div(S.R, 8)) {
      case 1: return attrs_level0_8_1(by);
      case 2: return attrs_level0_8_2(by);
      case 3: return attrs_level0_8_3(by);
      case 4: return attrs_level0_8_4(by);
    }
  }
  if (S.R > 128) {
    switch ((int)cl_ceil_div(S.R, 24)) {
      case 6: return attrs_level0_24_6(by);
      case 7: return attrs_level0_24_7(by);
    }
    return -1;
  }
  switch ((int)cl_ceil_div(S.R, 16)) {
    case 3: return attrs_level0_16_3(by);
    case 4: return attrs_level0_16_4(by);
    case 5: return attrs_level0_16_5(by);
    case 6: return attrs_level0_16_6(by);
    case 7: return attrs_level0_16_7(by);
    case 8: return attrs_level0_16_8(by);
  }
  return -1;
}
// mode: 0 first chain level, 1 chain step `level`, 2 border; grid = work items.
int launch_chain(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level, unsigned grid, hipStream_t st) {
  if (grid == 0) return 0;
  const int Rl = mode == 2 ? S.ns + S.np : 3 * S.ns + S.np;
  const size_t lds = sizeof(double) * (8 * (size_t)Rl + 8);
  if (Rl <= 32) {
    switch ((int)cl_ceil_div(Rl, 8)) {
      case 1: launch_chain_8_1(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
      case 2: launch_chain_8_2(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
      case 3: launch_chain_8_3(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
      case 4: launch_chain_8_4(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
    }
  }
  if (Rl > 128) {
    switch ((int)cl_ceil_div(Rl, 24)) {
      case 6: launch_chain_24_6(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
      case 7: launch_chain_24_7(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
    }
    return -1;
  }
  switch ((int)cl_ceil_div(Rl, 16)) {
    case 3: launch_chain_16_3(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
    case 4: launch_chain_16_4(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
    case 5: launch_chain_16_5(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
    case 6: launch_chain_16_6(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
    case 7: launch_chain_16_7(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
    case 8: launch_chain_16_8(S, tb, ws, prec, mode, level, grid, lds, st); return 0;
  }
  return -1;
}
}  // namespace cl
