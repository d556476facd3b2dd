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

template <typename T, int TS, int NB>
__global__ void __launch_bounds__(TS* TS) k_chain(Shape S, Tab tb, Ws ws, int mode, int level) {
  extern __shared__ double lds[];
  constexpr int NBLK = NB * (NB + 1) / 2;
  const int ns = S.ns, np = S.np;
  int inst, s;
  bool elim = true;
  if (mode == CH_FIRST) {
    const int it = tb.cr_ptr[0] + blockIdx.x;
    if (it >= tb.cr_ptr[1]) return;
    inst = tb.cr_inst[it];
    s = tb.cr_j[it];
  } else if (mode == CH_STEP) {
    const int it = tb.st_ptr[level - 1] + blockIdx.x;
    if (it >= tb.st_ptr[level]) return;
    inst = tb.st_inst[it];
    s = tb.st_s[it];
    elim = ((s >> level) & 1) != 0;
  } else {
    inst = blockIdx.x;
    s = 0;
  }
  if (block_flag(&ws.flag[inst])) return;
  const int N = tb.inst_N[inst];
  const int64_t e0 = tb.inst_e0[inst], es = e0 + s;

  // sources of the separator's current block
  SepSrc src;
  src.es = es;
  src.j1 = -1;
  src.j2 = -1;
  int64_t eL = -1, eR = -1;     // coupling sources (E1 rows or stored Schur couplings)
  bool eL_is_e1 = false, eR_is_e1 = false;
  if (mode == CH_FIRST) {
    src.add_next = s + 1 < N;
    eL = es;
    eL_is_e1 = true;
    if (s + 1 < N) {
      eR = es + 1;
      eR_is_e1 = true;
    }
  } else if (mode == CH_STEP) {
    const int half = 1 << (level - 1);
    src.add_next = (level == 1) && (s + 1 < N);
    if (s > 0) src.j1 = e0 + s - half;
    if (s + half < N) src.j2 = e0 + s + half;
    if (elim) {
      eL = src.j1;
      if (s + 2 * half < N) eR = src.j2;
    }
  } else {
    const int L = tb.L;
    src.add_next = (L <= 1) && (N > 1);
    const int jl = L >= 1 ? (1 << (L - 1)) : N;
    if (jl < N) src.j2 = e0 + jl;
  }

  if (!elim) {   // survivor: add the contributions and keep the block for a later level
    T* dss = (T*)ws.dss + es * ns * ns;
    T* bsv = (T*)ws.bs + es * ns * np;
    for (int t = tid(); t < ns * ns; t += nthr()) dss[t] = (T)sep_T<T>(S, ws, src, t / ns, t % ns);
    for (int t = tid(); t < ns * np; t += nthr()) bsv[t] = (T)sep_G<T>(S, ws, src, t / np, t % np);
    return;
  }

  const int Rl = (mode == CH_BORDER) ? ns + np : 3 * ns + np;
  const int ne = (mode == CH_BORDER) ? Rl : ns;
  const int th0 = (mode == CH_BORDER) ? ns : 3 * ns;   // first theta row
  const int ty = threadIdx.x / TS, tx = threadIdx.x % TS;
  double* pbuf = lds;
  double* misc = pbuf + 8 * Rl;
  double av[NBLK];
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J <= I; ++J) {
      const int r = I * TS + ty, q = J * TS + tx;
      double v = 0.0;
      if (r < Rl && q <= r) {
        if (q < ns) {
          if (r < ns) {
            v = sep_T<T>(S, ws, src, r, q);
          } else if (r >= th0) {
            v = sep_G<T>(S, ws, src, q, r - th0);
          } else if (r < 2 * ns) {          // left neighbour row a: E_L[q][a] = K(s_q, l_a)
            const int a = r - ns;
            if (eL >= 0) v = eL_is_e1 ? ld<T>(ws.e1, eL * ns * ns + q * ns + a) : ld<T>(ws.cE, eL * ns * ns + q * ns + a);
          } else {                          // right neighbour row a: E_R[a][q] = K(r_a, s_q)
            const int a = r - 2 * ns;
            if (eR >= 0) v = eR_is_e1 ? ld<T>(ws.e1, eR * ns * ns + a * ns + q) : ld<T>(ws.cE, eR * ns * ns + a * ns + q);
          }
        } else if (mode == CH_BORDER) {     // theta-theta: reduced parameter block
          v = ws.S[(int64_t)inst * np * np + (r - ns) * np + (q - ns)];
        }
      }
      av[I * (I + 1) / 2 + J] = v;
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
