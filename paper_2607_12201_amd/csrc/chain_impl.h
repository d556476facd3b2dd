// Separator-chain and border elimination kernels (included by the k_level0*.hip units).
//
// Eliminating separator s of the chain (node K of element s) is a partial Cholesky of its
// local matrix over [s | left neighbour | right neighbour | theta]: the s block T_s, the
// couplings to the neighbours and the theta border G_s in the first n_s columns, zeros in the
// trailing block.  After the n_s columns are eliminated (eliminate_regs), the rows below hold
// the transformed couplings U_L^T, U_R^T, U_B^T (kept for the solve) and the trailing block
// holds exactly the Schur contributions to the neighbours: -U_L^T U_L, -U_R^T U_L (the new
// coupling between the neighbours), -U_R^T U_R, -U_B^T U_L, -U_B^T U_R and -U_B^T U_B.
// A survivor later adds the contributions of its two eliminated neighbours.  The border is the
// full Cholesky of [separator 0 | theta] with the reduced parameter block.
#pragma once
#include "kernels.h"
#include "regchol.h"

namespace cl {

enum { CH_FIRST = 0, CH_STEP = 1, CH_BORDER = 2 };

template <typename T>
__device__ inline double ld(const void* base, int64_t i) {
  return (double)((const T*)base)[i];
}

// Value of the current separator block T_s(a, b) and border G_s(a, c) before elimination.
struct SepSrc {
  int64_t es;          // global index of separator s
  bool add_next;       // add the next element's level-0 part (first touch)
  int64_t j1, j2;      // eliminated neighbours whose contributions are added (-1 if none)
};

template <typename T>
__device__ inline double sep_T(const Shape& S, const Ws& ws, const SepSrc& c, int a, int b) {
  const int ns = S.ns;
  double v = ld<T>(ws.dss, c.es * ns * ns + a * ns + b);
  if (c.add_next) v += ld<T>(ws.tprev, (c.es + 1) * ns * ns + a * ns + b);
  if (c.j1 >= 0) v += ld<T>(ws.cTr, c.j1 * ns * ns + a * ns + b);
  if (c.j2 >= 0) v += ld<T>(ws.cTl, c.j2 * ns * ns + a * ns + b);
  return v;
}
template <typename T>
__device__ inline double sep_G(const Shape& S, const Ws& ws, const SepSrc& c, int a, int col) {
  const int ns = S.ns, np = S.np;
  double v = ld<T>(ws.bs, c.es * ns * np + a * np + col);
  if (c.add_next) v += ld<T>(ws.gprev, (c.es + 1) * ns * np + a * np + col);
  if (c.j1 >= 0) v += ld<T>(ws.cGr, c.j1 * ns * np + a * np + col);
  if (c.j2 >= 0) v += ld<T>(ws.cGl, c.j2 * ns * np + a * np + col);
  return v;
}

// One separator of a chain level (or the border item): which instance and separator, whether it
// is eliminated at this level, and where its current blocks come from.
struct ChainItem {
  bool valid, elim;
  int inst, s, N;
  int64_t e0, es;
  SepSrc src;
  int64_t eL, eR;             // coupling sources (E1 rows or stored Schur couplings), -1 = none
  bool eL_is_e1, eR_is_e1;
};

__device__ inline ChainItem chain_item(const Tab& tb, int mode, int level) {
  ChainItem c;
  c.valid = true;
  c.elim = true;
  if (mode == CH_FIRST) {
    const int it = tb.cr_ptr[0] + blockIdx.x;
    if (it >= tb.cr_ptr[1]) {
      c.valid = false;
      return c;
    }
    c.inst = tb.cr_inst[it];
    c.s = tb.cr_j[it];
  } else if (mode == CH_STEP) {
    const int it = tb.st_ptr[level - 1] + blockIdx.x;
    if (it >= tb.st_ptr[level]) {
      c.valid = false;
      return c;
    }
    c.inst = tb.st_inst[it];
    c.s = tb.st_s[it];
    c.elim = ((c.s >> level) & 1) != 0;
  } else {
    c.inst = blockIdx.x;
    c.s = 0;
  }
  const int s = c.s;
  c.N = tb.inst_N[c.inst];
  const int N = c.N;
  c.e0 = tb.inst_e0[c.inst];
  c.es = c.e0 + s;
  c.src.es = c.es;
  c.src.j1 = -1;
  c.src.j2 = -1;
  c.eL = c.eR = -1;
  c.eL_is_e1 = c.eR_is_e1 = false;
  if (mode == CH_FIRST) {
    c.src.add_next = s + 1 < N;
    c.eL = c.es;
    c.eL_is_e1 = true;
    if (s + 1 < N) {
      c.eR = c.es + 1;
      c.eR_is_e1 = true;
    }
  } else if (mode == CH_STEP) {
    const int half = 1 << (level - 1);
    c.src.add_next = (level == 1) && (s + 1 < N);
    if (s > 0) c.src.j1 = c.e0 + s - half;
    if (s + half < N) c.src.j2 = c.e0 + s + half;
    if (c.elim) {
      c.eL = c.src.j1;
      if (s + 2 * half < N) c.eR = c.src.j2;
    }
  } else {
    const int L = tb.L;
    c.src.add_next = (L <= 1) && (N > 1);
    const int jl = L >= 1 ? (1 << (L - 1)) : N;
    if (jl < N) c.src.j2 = c.e0 + jl;
  }
  return c;
}

// A separator that survives this level: add the contributions, keep the block for later.
template <typename T>
__device__ inline void chain_survivor(const Shape& S, const Ws& ws, const SepSrc& src) {
  const int ns = S.ns, np = S.np;
  T* dss = (T*)ws.dss + src.es * ns * ns;
  T* bsv = (T*)ws.bs + src.es * ns * np;
  for (int t = tid(); t < ns * ns; t += nthr()) dss[t] = (T)sep_T<T>(S, ws, src, t / ns, t % ns);
  for (int t = tid(); t < ns * np; t += nthr()) bsv[t] = (T)sep_G<T>(S, ws, src, t / np, t % np);
}

// Off-diagonal row a of a separator's local matrix in pivot column q: left neighbour rows
// (E_L[q][a] = K(s_q, l_a)), right neighbour rows (E_R[a][q] = K(r_a, s_q)), parameter rows.
template <typename T>
__device__ inline double chain_offdiag(const Shape& S, const Ws& ws, const ChainItem& c, int a, int q) {
  const int ns = S.ns;
  if (a < ns) {
    if (c.eL < 0) return 0.0;
    return c.eL_is_e1 ? ld<T>(ws.e1, c.eL * ns * ns + q * ns + a) : ld<T>(ws.cE, c.eL * ns * ns + q * ns + a);
  }
  if (a < 2 * ns) {
    const int b = a - ns;
    if (c.eR < 0) return 0.0;
    return c.eR_is_e1 ? ld<T>(ws.e1, c.eR * ns * ns + b * ns + q) : ld<T>(ws.cE, c.eR * ns * ns + b * ns + q);
  }
  return sep_G<T>(S, ws, c.src, q, a - 2 * ns);
}

// The separator columns of a chain item's local matrix (its first ns columns, all Rl rows),
// gathered into X (row-major, Rl x ns) by all threads.  In each pass a thread loads one entry
// of every row group (T_s with its added terms, the neighbour couplings, G_s with its added
// terms) from valid addresses (the separator's own block where a term does not apply), then
// selects and stores them, so a pass costs one memory latency.  X[Rl * ns] is a dummy slot for
// threads past the end of a group.  Terms are added in the order of sep_T / sep_G.
template <typename T>
__device__ inline void chain_stage(const Shape& S, const Ws& ws, const ChainItem& c, bool border,
                                   int Rl, int th0, double* X) {
  const int ns = S.ns, np = S.np;
  const int64_t n2 = (int64_t)ns * ns, ng = (int64_t)ns * np;
  const bool an = c.src.add_next, h1 = c.src.j1 >= 0, h2 = c.src.j2 >= 0;
  const bool hL = !border && c.eL >= 0, hR = !border && c.eR >= 0;
  const T* tw = (const T*)ws.dss + c.es * n2;
  const T* t1 = an ? (const T*)ws.tprev + (c.es + 1) * n2 : tw;
  const T* t2 = h1 ? (const T*)ws.cTr + c.src.j1 * n2 : tw;
  const T* t3 = h2 ? (const T*)ws.cTl + c.src.j2 * n2 : tw;
  const T* gw = (const T*)ws.bs + c.es * ng;
  const T* g1 = an ? (const T*)ws.gprev + (c.es + 1) * ng : gw;
  const T* g2 = h1 ? (const T*)ws.cGr + c.src.j1 * ng : gw;
  const T* g3 = h2 ? (const T*)ws.cGl + c.src.j2 * ng : gw;
  const T* pl = hL ? (const T*)(c.eL_is_e1 ? ws.e1 : ws.cE) + c.eL * n2 : tw;
  const T* pr = hR ? (const T*)(c.eR_is_e1 ? ws.e1 : ws.cE) + c.eR * n2 : tw;
  const int nT = ns * ns, nG = np * ns, nmax = nT > nG ? nT : nG, dummy = Rl * ns;
  for (int t0 = 0; t0 < nmax; t0 += nthr()) {
    const int t = t0 + tid();
    const bool vT = t < nT, vG = t < nG;
    const int tT = vT ? t : 0, tG = vG ? t : 0;
    const int a = tT / ns, q = tT - a * ns;       // separator-column entry (a, q)
    const int cg = tG / ns, qg = tG - cg * ns;    // theta row cg, separator column qg
    const int iG = qg * np + cg;
    const double xT0 = (double)tw[tT], xT1 = (double)t1[tT], xT2 = (double)t2[tT], xT3 = (double)t3[tT];
    const double xL = (double)pl[q * ns + a], xR = (double)pr[a * ns + q];
    const double xG0 = (double)gw[iG], xG1 = (double)g1[iG], xG2 = (double)g2[iG], xG3 = (double)g3[iG];
    double vt = xT0;
    vt += an ? xT1 : 0.0;
    vt += h1 ? xT2 : 0.0;
    vt += h2 ? xT3 : 0.0;
    double vg = xG0;
    vg += an ? xG1 : 0.0;
    vg += h1 ? xG2 : 0.0;
    vg += h2 ? xG3 : 0.0;
    X[vT ? a * ns + q : dummy] = vt;
    X[vG ? (th0 + cg) * ns + qg : dummy] = vg;
    X[vT && !border ? (ns + a) * ns + q : dummy] = hL ? xL : 0.0;
    X[vT && !border ? (2 * ns + a) * ns + q : dummy] = hR ? xR : 0.0;
  }
}

// Elimination of one separator by blocks, in LDS (FP64): Cholesky of the separator block T_s
// by one wave, then U = L_s^{-1} [E_L E_R G]^T row by row (one thread per row), then the Schur
// contributions -U^T U as register-blocked dot products over the ns pivot columns.  It needs few
// workgroup barriers but has long dependent chains in its serial parts; the autotuner times it
// against the register-resident grids (at 20 species it is the slower one).  Outputs are those
// of k_chain (lsep, ul, ur, ub and the contributions cTl, cE, cTr, cGl, cGr, thcr).
// LDS: Tm (ns x ns) | X (Rt x ns, Rt = 2 ns + np) | rd (ns) | misc (8)
template <typename T>
__global__ void __launch_bounds__(256) k_chain_blk(Shape S, Tab tb, Ws ws, int mode, int level) {
  static_assert(sizeof(T) == 8, "FP64 only");
  extern __shared__ double lds[];
  const ChainItem c = chain_item(tb, mode, level);
  if (!c.valid) return;
  if (block_flag(&ws.flag[c.inst])) return;
  if (!c.elim) {
    chain_survivor<double>(S, ws, c.src);
    return;
  }
  const int ns = S.ns, np = S.np, Rt = 2 * ns + np;
  double* Tm = lds;
  double* X = Tm + ns * ns;
  double* rd = X + Rt * ns;
  double* misc = rd + ns;
  for (int t = tid(); t < ns * ns; t += nthr()) {
    const int a = t / ns, b = t - a * ns;
    Tm[t] = b <= a ? sep_T<double>(S, ws, c.src, a, b) : 0.0;
  }
  for (int t = tid(); t < Rt * ns; t += nthr()) {
    const int a = t / ns, q = t - a * ns;
    X[t] = chain_offdiag<double>(S, ws, c, a, q);
  }
  __syncthreads();
  if (tid() < 64) {   // Cholesky of T_s: lane i keeps row i
    const int lane = tid();
    for (int k = 0; k < ns; ++k) {
      if (lane == 0) {
        const double piv = Tm[k * ns + k];
        const bool good = piv > 0.0 && isfinite(piv);
        const double sq = good ? sqrt(piv) : 1.0;
        Tm[k * ns + k] = sq;
        misc[0] = good ? 1.0 : 0.0;
        misc[1] = 1.0 / sq;
      }
      __builtin_amdgcn_wave_barrier();
      if (misc[0] == 0.0) break;
      const double inv = misc[1];
      if (lane > k && lane < ns) Tm[lane * ns + k] *= inv;
      __builtin_amdgcn_wave_barrier();
      if (lane > k && lane < ns) {
        const double lik = Tm[lane * ns + k];
        for (int j = k + 1; j <= lane; ++j) Tm[lane * ns + j] -= lik * Tm[j * ns + k];
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (lane < ns) rd[lane] = 1.0 / Tm[lane * ns + lane];
  }
  __syncthreads();
  if (misc[0] == 0.0) {
    if (tid() == 0) atomicOr(&ws.flag[c.inst], 1);
    return;
  }
  for (int a = tid(); a < Rt; a += nthr()) {   // U row a = L_s^{-1} x_a
    double* xa = X + a * ns;
    for (int j = 0; j < ns; ++j) {
      double v = xa[j];
      for (int k = 0; k < j; ++k) v -= xa[k] * Tm[j * ns + k];
      xa[j] = v * rd[j];
    }
  }
  __syncthreads();
  const int64_t es = c.es;
  double* lsep = (double*)ws.lsep + es * ns * ns;
  double* ul = (double*)ws.ul + es * ns * ns;
  double* ur = (double*)ws.ur + es * ns * ns;
  double* ub = (double*)ws.ub + es * ns * np;
  for (int t = tid(); t < ns * ns; t += nthr()) {
    const int a = t / ns, q = t - a * ns;
    if (q <= a) lsep[t] = Tm[t];
  }
  for (int t = tid(); t < Rt * ns; t += nthr()) {
    const int a = t / ns, q = t - a * ns;
    const double v = X[t];
    if (a < ns) ul[q * ns + a] = v;
    else if (a < 2 * ns) ur[q * ns + (a - ns)] = v;
    else ub[q * np + (a - 2 * ns)] = v;
  }
  // Schur contributions -U_a^T U_b (b <= a), 2 x 2 row blocks per thread
  double* cTl = (double*)ws.cTl + es * ns * ns;
  double* cTr = (double*)ws.cTr + es * ns * ns;
  double* cE = (double*)ws.cE + es * ns * ns;
  double* cGl = (double*)ws.cGl + es * ns * np;
  double* cGr = (double*)ws.cGr + es * ns * np;
  double* th = ws.thcr + es * np * np;
  const int nb2 = (Rt + 1) / 2, nblk = nb2 * (nb2 + 1) / 2;
  for (int t = tid(); t < nblk; t += nthr()) {
    int bi = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    while (bi * (bi + 1) / 2 > t) --bi;
    const int bj = t - bi * (bi + 1) / 2;
    const int a0 = 2 * bi, b0 = 2 * bj;
    const double* x0 = X + a0 * ns;
    const double* x1 = X + (a0 + 1 < Rt ? a0 + 1 : a0) * ns;
    const double* y0 = X + b0 * ns;
    const double* y1 = X + (b0 + 1 < Rt ? b0 + 1 : b0) * ns;
    double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
    for (int q = 0; q < ns; ++q) {
      const double u0 = x0[q], u1 = x1[q], w0 = y0[q], w1 = y1[q];
      s00 += u0 * w0;
      s01 += u0 * w1;
      s10 += u1 * w0;
      s11 += u1 * w1;
    }
    const double vals[4] = {s00, s01, s10, s11};
    for (int k = 0; k < 4; ++k) {
      const int a = a0 + (k >> 1), b = b0 + (k & 1);
      if (a >= Rt || b >= Rt || b > a) continue;
      const double v = -vals[k];
      const int ag = a < ns ? 1 : (a < 2 * ns ? 2 : 3);
      const int bg = b < ns ? 1 : (b < 2 * ns ? 2 : 3);
      const int aa = a - (ag - 1) * ns, bb = b - (bg - 1) * ns;
      if (ag == 1) cTl[aa * ns + bb] = v;
      else if (ag == 2 && bg == 1) cE[aa * ns + bb] = v;
      else if (ag == 2) cTr[aa * ns + bb] = v;
      else if (bg == 1) cGl[bb * np + (a - 2 * ns)] = v;
      else if (bg == 2) cGr[bb * np + (a - 2 * ns)] = v;
      else th[(a - 2 * ns) * np + (b - 2 * ns)] = v;
    }
  }
}

template <typename T, int TS, int NB>
__global__ void __launch_bounds__(TS* TS) k_chain(Shape S, Tab tb, Ws ws, int mode, int level) {
  extern __shared__ double lds[];
  constexpr int NBLK = NB * (NB + 1) / 2;
  const int ns = S.ns, np = S.np;
  const ChainItem ci = chain_item(tb, mode, level);
  if (!ci.valid) return;
  const int inst = ci.inst;
  if (block_flag(&ws.flag[inst])) return;
  const int64_t es = ci.es;
  if (!ci.elim) {
    chain_survivor<T>(S, ws, ci.src);
    return;
  }

  const int Rl = (mode == CH_BORDER) ? ns + np : 3 * ns + np;
  const int ne = (mode == CH_BORDER) ? Rl : ns;
  const int th0 = (mode == CH_BORDER) ? ns : 3 * ns;   // first theta row
  const int ty = threadIdx.x / TS, tx = threadIdx.x % TS;
  double* pbuf = lds;
  double* misc = pbuf + elim_lds_doubles(Rl);
  const bool border = mode == CH_BORDER;
  double* X = misc + 8;                                 // Rl x ns separator columns + 1
  chain_stage<T>(S, ws, ci, border, Rl, th0, X);
  __syncthreads();
  double av[NBLK];
  if (border) {
    // separator columns from X, the reduced parameter block straight from memory
    const double* Sg = ws.S + (int64_t)inst * np * np;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const int r = I * TS + ty, q = J * TS + tx;
        const bool in = r < Rl && q <= r, qs = q < ns;
        const double xs = Sg[in && !qs ? (r - ns) * np + (q - ns) : 0];
        const double xx = X[in && qs ? r * ns + q : 0];
        av[I * (I + 1) / 2 + J] = pick(in, pick(qs, xx, xs), 0.0);
      }
  } else {
    // column block 0 holds separator columns; the blocks right of it only when the separator
    // is wider than the grid
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      const int r = I * TS + ty, q = tx;
      const bool in = r < Rl && q <= r && q < ns;
      const double xx = X[in ? r * ns + q : 0];
      av[I * (I + 1) / 2] = in ? xx : 0.0;
    }
#pragma unroll
    for (int I = 1; I < NB; ++I)
#pragma unroll
      for (int J = 1; J <= I; ++J) {
        const int r = I * TS + ty, q = J * TS + tx;
        const bool in = r < Rl && q <= r && q < ns;
        const double xx = X[in ? r * ns + q : 0];
        av[I * (I + 1) / 2 + J] = in ? xx : 0.0;
      }
  }

  bool ok;
  if constexpr (sizeof(T) == 8) {
    ok = eliminate_regs<double, TS, NB>(av, ne, Rl, ty, tx, pbuf, misc);
  } else {
    // FP32 block factors: the separator columns in FP32; the theta-theta trailing block is
    // formed below in FP64 from the stored FP32 border rows
    float af[NBLK];
#pragma unroll
    for (int B = 0; B < NBLK; ++B) af[B] = (float)av[B];
    if (mode == CH_BORDER) {
      ok = eliminate_regs<double, TS, NB>(av, ne, Rl, ty, tx, pbuf, misc);
    } else {
      ok = eliminate_regs<float, TS, NB>(af, ne, Rl, ty, tx, pbuf, misc);
#pragma unroll
      for (int B = 0; B < NBLK; ++B) av[B] = (double)af[B];
    }
  }
  if (!ok) {
    if (tid() == 0) atomicOr(&ws.flag[inst], 1);
    return;
  }

  T* lsep = (T*)ws.lsep + es * ns * ns;
  T* ub = (T*)ws.ub + es * ns * np;
  if (mode == CH_BORDER) {
    double* Sg = ws.S + (int64_t)inst * np * np;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const int r = I * TS + ty, q = J * TS + tx;
        if (!(r < Rl && q <= r)) continue;
        const double v = av[I * (I + 1) / 2 + J];
        if (q < ns) {
          if (r < ns) lsep[r * ns + q] = (T)v;
          else ub[q * np + (r - ns)] = (T)v;
        } else {
          Sg[(r - ns) * np + (q - ns)] = v;
        }
      }
    return;
  }
  T* ul = (T*)ws.ul + es * ns * ns;
  T* ur = (T*)ws.ur + es * ns * ns;
  T* cTl = (T*)ws.cTl + es * ns * ns;
  T* cTr = (T*)ws.cTr + es * ns * ns;
  T* cE = (T*)ws.cE + es * ns * ns;
  T* cGl = (T*)ws.cGl + es * ns * np;
  T* cGr = (T*)ws.cGr + es * ns * np;
  double* th = ws.thcr + es * np * np;
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J <= I; ++J) {
      const int r = I * TS + ty, q = J * TS + tx;
      if (!(r < Rl && q <= r)) continue;
      const T v = (T)av[I * (I + 1) / 2 + J];
      const int rg = r < ns ? 0 : (r < 2 * ns ? 1 : (r < 3 * ns ? 2 : 3));
      const int ra = r - rg * ns;
      if (q < ns) {
        if (rg == 0) lsep[r * ns + q] = v;
        else if (rg == 1) ul[q * ns + ra] = v;
        else if (rg == 2) ur[q * ns + ra] = v;
        else ub[q * np + (r - 3 * ns)] = v;
      } else {
        const int qg = q < 2 * ns ? 1 : (q < 3 * ns ? 2 : 3);
        const int qa = q - qg * ns;
        if (rg == 1) cTl[ra * ns + qa] = v;                  // (l, l)
        else if (rg == 2 && qg == 1) cE[ra * ns + qa] = v;   // (r, l): new coupling
        else if (rg == 2) cTr[ra * ns + qa] = v;             // (r, r)
        else if (qg == 1) cGl[qa * np + (r - 3 * ns)] = v;   // (theta, l)
        else if (qg == 2) cGr[qa * np + (r - 3 * ns)] = v;   // (theta, r)
        else if (sizeof(T) == 8) th[(r - 3 * ns) * np + (q - 3 * ns)] = (double)v;
      }
    }
  if (sizeof(T) == 4) {
    // FP64 theta-theta contribution -U_B^T U_B from the stored FP32 border rows
    __syncthreads();
    for (int t = tid(); t < np * np; t += nthr()) {
      const int r = t / np, q = t % np;
      if (q > r) continue;
      double sum = 0.0;
      for (int p = 0; p < ns; ++p) sum += (double)ub[p * np + r] * (double)ub[p * np + q];
      th[t] = -sum;
    }
  }
}

}  // namespace cl
