// Dispatch of the register-resident elimination kernels: thread grid TS x TS (TS in 8, 16,
// 20, 24) with NB = ceil(rows / TS) register blocks per side.  The built-in rule picks the smallest
// grid whose block count stays within the instantiated range; a handle may override the grid
// per kernel (tuning).
#include "kernels.h"
#include "chain_impl.h"

namespace cl {
void launch_level0_8_1(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_8_1(size_t);
void launch_chain_8_1(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_8_2(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_8_2(size_t);
void launch_chain_8_2(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_8_3(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_8_3(size_t);
void launch_chain_8_3(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_8_4(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_8_4(size_t);
void launch_chain_8_4(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_16_1(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_16_1(size_t);
void launch_chain_16_1(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_16_2(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_16_2(size_t);
void launch_chain_16_2(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_24_2(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_24_2(size_t);
void launch_chain_24_2(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_24_3(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_24_3(size_t);
void launch_chain_24_3(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_16_3(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_16_3(size_t);
void launch_chain_16_3(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_16_4(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_16_4(size_t);
void launch_chain_16_4(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_16_5(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_16_5(size_t);
void launch_chain_16_5(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_16_6(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_16_6(size_t);
void launch_chain_16_6(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_16_7(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_16_7(size_t);
void launch_chain_16_7(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_16_8(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_16_8(size_t);
void launch_chain_16_8(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_24_4(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_24_4(size_t);
void launch_chain_24_4(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_24_5(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_24_5(size_t);
void launch_chain_24_5(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_24_6(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_24_6(size_t);
void launch_chain_24_6(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_24_7(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_24_7(size_t);
void launch_chain_24_7(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_20_5(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_20_5(size_t);
void launch_chain_20_5(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_20_6(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_20_6(size_t);
void launch_chain_20_6(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_20_7(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_20_7(size_t);
void launch_chain_20_7(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
void launch_level0_20_8(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
int attrs_level0_20_8(size_t);
void launch_chain_20_8(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);

namespace {
struct Variant {
  int ts, nb;
  void (*level0)(const Shape&, const Tab&, const Ws&, int, int, hipStream_t);
  int (*attrs)(size_t);
  void (*chain)(const Shape&, const Tab&, const Ws&, int, int, int, unsigned, size_t, hipStream_t);
};
const Variant kVariants[] = {
    {8, 1, launch_level0_8_1, attrs_level0_8_1, launch_chain_8_1},
    {8, 2, launch_level0_8_2, attrs_level0_8_2, launch_chain_8_2},
    {8, 3, launch_level0_8_3, attrs_level0_8_3, launch_chain_8_3},
    {8, 4, launch_level0_8_4, attrs_level0_8_4, launch_chain_8_4},
    {16, 1, launch_level0_16_1, attrs_level0_16_1, launch_chain_16_1},
    {16, 2, launch_level0_16_2, attrs_level0_16_2, launch_chain_16_2},
    {24, 2, launch_level0_24_2, attrs_level0_24_2, launch_chain_24_2},
    {24, 3, launch_level0_24_3, attrs_level0_24_3, launch_chain_24_3},
    {16, 3, launch_level0_16_3, attrs_level0_16_3, launch_chain_16_3},
    {16, 4, launch_level0_16_4, attrs_level0_16_4, launch_chain_16_4},
    {16, 5, launch_level0_16_5, attrs_level0_16_5, launch_chain_16_5},
    {16, 6, launch_level0_16_6, attrs_level0_16_6, launch_chain_16_6},
    {16, 7, launch_level0_16_7, attrs_level0_16_7, launch_chain_16_7},
    {16, 8, launch_level0_16_8, attrs_level0_16_8, launch_chain_16_8},
    {24, 4, launch_level0_24_4, attrs_level0_24_4, launch_chain_24_4},
    {24, 5, launch_level0_24_5, attrs_level0_24_5, launch_chain_24_5},
    {24, 6, launch_level0_24_6, attrs_level0_24_6, launch_chain_24_6},
    {24, 7, launch_level0_24_7, attrs_level0_24_7, launch_chain_24_7},
    {20, 5, launch_level0_20_5, attrs_level0_20_5, launch_chain_20_5},
    {20, 6, launch_level0_20_6, attrs_level0_20_6, launch_chain_20_6},
    {20, 7, launch_level0_20_7, attrs_level0_20_7, launch_chain_20_7},
    {20, 8, launch_level0_20_8, attrs_level0_20_8, launch_chain_20_8}
};

const Variant* find_variant(int ts, int rows) {
  const int nb = (int)cl_ceil_div(rows, ts);
  for (const Variant& v : kVariants)
    if (v.ts == ts && v.nb == nb) return &v;
  return nullptr;
}

// Built-in rule: 8 x 8 up to 32 rows, 16 x 16 up to 128, 20 x 20 up to 160 (seven waves and
// at most 128 registers, so two elements share a compute unit), 24 x 24 above.
int default_ts(int rows) { return rows <= 32 ? 8 : (rows <= 128 ? 16 : (rows <= 160 ? 20 : 24)); }

const Variant* pick(int ts, int rows) {
  return find_variant(ts > 0 ? ts : default_ts(rows), rows);
}
}  // namespace

size_t level0r_lds_bytes(const Shape& S) {
  const size_t ns = S.ns, np = S.np, jl = (size_t)S.K * S.nr;
  size_t nd = (size_t)elim_lds_doubles(S.R) + 8 + S.b + (CL_KMAX + 1) * (CL_KMAX + 1) + 1 + 7 * jl + ns +
              3 * ns * ns + 3 * ns * np + np + np * np + 3 * (size_t)S.lsp + 2 * (size_t)S.lrq +
              S.lsp + (size_t)S.mmax * (S.K + 1);
  size_t ni = 3 * (size_t)S.nr + 2 * (ns + 1) + (np + 1) + S.lsp + 2 * (size_t)S.lrq + S.lpc +
              S.mmax + S.R + 1 + 3 * (size_t)S.lsp + 2 * (size_t)S.lrq;
  return sizeof(double) * nd + sizeof(int) * ni;
}

bool level0r_supported(const Shape& S) { return S.R <= 160 && 3 * S.ns + S.np <= 160; }

int chain_rows(const Shape& S, int which) { return which == 2 ? S.ns + S.np : 3 * S.ns + S.np; }

// Chain kernels: the elimination buffers, flags, the staged separator columns (R x ns) and a
// dummy slot.
size_t chain_lds_bytes(const Shape& S, int which) {
  const size_t Rl = chain_rows(S, which);
  return sizeof(double) * (elim_lds_doubles((int)Rl) + 8 + Rl * S.ns + 1);
}

int tile_rows(const Shape& S, int which) { return which == 0 ? S.R : chain_rows(S, which); }

size_t chain_blk_lds_bytes(const Shape& S) {
  const size_t ns = S.ns, Rt = 2 * (size_t)S.ns + S.np;
  return sizeof(double) * (ns * ns + Rt * ns + ns + 8);
}

// The blocked LDS variant of the chain kernel (selected as TS = 1, FP64 factors only).
bool chain_blk_ok(const Shape& S) { return chain_blk_lds_bytes(S) <= 64 * 1024 && S.ns <= 64; }

int tile_options(const Shape& S, int which, int* ts, int cap) {
  const int rows = tile_rows(S, which);
  int n = 0;
  if (which == 1 && chain_blk_ok(S)) {
    if (n < cap) ts[n] = 1;
    ++n;
  }
  for (int t : {8, 16, 20, 24})
    if (find_variant(t, rows)) {
      if (n < cap) ts[n] = t;
      ++n;
    }
  return n;
}

bool tile_valid(const Shape& S, int which, int ts) {
  if (ts == 1) return which == 1 && chain_blk_ok(S);
  return ts == 0 || find_variant(ts, tile_rows(S, which)) != nullptr;
}

int launch_level0(const Shape& S, const Tab& tb, const Ws& ws, int prec, bool fused, int ts,
                  hipStream_t st) {
  const Variant* v = pick(ts, S.R);
  if (!v) return -1;
  v->level0(S, tb, ws, prec, fused ? 1 : 0, st);
  return 0;
}

// Dynamic LDS above 64 KB needs the kernel attribute; it is set on every grid that the element
// or chain kernels may use for this shape.
int level0_prepare_attrs(const Shape& S) {
  const size_t by = std::max(level0r_lds_bytes(S), std::max(chain_lds_bytes(S, 1), chain_lds_bytes(S, 2)));
  if (by <= 64 * 1024) return 0;
  for (int rows : {S.R, chain_rows(S, 1), chain_rows(S, 2)})
    for (int t : {8, 16, 20, 24})
      if (const Variant* v = find_variant(t, rows))
        if (v->attrs(by)) return -1;
  return 0;
}

// mode: 0 first chain level, 1 chain step `level`, 2 border; grid = work items.
int launch_chain(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level,
                 unsigned grid, int ts, hipStream_t st) {
  if (grid == 0) return 0;
  // the blocked LDS variant of the FP64 chain levels when chosen (TS = 1)
  if (prec == 0 && mode != 2 && ts == 1 && chain_blk_ok(S)) {
    hipLaunchKernelGGL(k_chain_blk<double>, dim3(grid), dim3(256), chain_blk_lds_bytes(S), st, S, tb,
                       ws, mode, level);
    return 0;
  }
  const int Rl = chain_rows(S, mode == 2 ? 2 : 1);
  const size_t lds = chain_lds_bytes(S, mode == 2 ? 2 : 1);
  const Variant* v = pick(ts == 1 ? 0 : ts, Rl);
  if (!v) return -1;
  v->chain(S, tb, ws, prec, mode, level, grid, lds, st);
  return 0;
}
}  // namespace cl
