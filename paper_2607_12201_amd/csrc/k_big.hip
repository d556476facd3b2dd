// Tiled (matrix-core) factorization and solve of the condensed KKT matrix for element blocks too
// large for the register-resident kernels.  Same elimination order as the register path (every
// element's interior collocation nodes, then cyclic reduction of the element-end separators,
// then the border [separator 0 | theta]), with every dense block in global memory:
//
//   assembly   k_big_asm       one workgroup per element writes the lower triangle of its
//                              matrix over [z | theta | P] (eq. 2b-2d through J^T Ds J + W) from
//                              the per-pattern derivative values, the theta-theta block in FP64
//   level 0    k_pchol_diag / k_pchol_strip  left-looking partial Cholesky of the interior
//                              columns in 32-column panels: the diagonal block (one wave per
//                              matrix), then the strips below it (one wave per 32 rows), updates
//                              and solves as 16x16x4 matrix-core products
//              k_pchol_trail   trailing Schur complement (all rows below the interior block)
//                              as 32 x 64 matrix-core blocks, the blocks of one element on one XCD
//   chain      k_sep_init / k_sep_step gather each separator's local matrix; the same two
//                              kernels eliminate the separators of every cyclic-reduction level
//   border     k_big_theta     theta-theta Schur complement in FP64 on matrix cores, split over
//                              16-element chunks (fixed order); k_border_build sums the chunks
//                              into the border matrix, the same panel kernels factor it
//   solve      blocked forward/backward substitution through the same levels (FP64 vectors)
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>

#include "../../include/colloc.h"
#include "big.h"
#include "elem.h"
#include "kernels.h"

namespace cl {

// ---------------------------------------------------------------- item addressing
// mode 0: element e (matrix e of ebuf), mode 1: separator eliminated at cyclic-reduction level
// `level` (matrix = its global index in sbuf), mode 2: instance border (matrix = instance).
struct PArgs {
  void* base;
  int64_t stride;   // elements between matrices
  int ld, n, m, count, mode, level;
  int zero;         // trailing update: the trailing block starts at zero (not read)
  int skip0, skip1; // trailing update: blocks inside [skip0, skip1)^2 are not computed
};

__device__ inline void pitem(const Tab& tb, const PArgs& a, int k, int64_t& mat, int& inst) {
  if (a.mode == 0) {
    mat = k;
    inst = tb.elem_inst[k];
  } else if (a.mode == 1) {
    const int it = tb.cr_ptr[a.level - 1] + k;
    inst = tb.cr_inst[it];
    mat = tb.inst_e0[inst] + tb.cr_j[it];
  } else {
    mat = k;
    inst = k;
  }
}

// ---------------------------------------------------------------- assembly
// LDS layout of k_big_asm (doubles, then ints).
struct AsmLds {
  double *D;            // (K + 1) x ns row weights Ds of the element (node-major)
  double *vF, *vT;      // K x lnf nonzeros of F (pair order), K x lct list values of Fth
  double *mw;           // element measurements' weights (mmax x (K + 1))
  double *a;            // collocation weights a[j * 8 + k] = l_j'(tau_k)
  const double* hes;    // the element's weighted second-derivative values (global, K nr 4)
  int *fcp, *fqs, *frp, *frq, *fru, *ctp, *cts, *zsp, *zsk, *zst, *ztc, *pcp, *pcr, *msp;
  int nmeas;
};

// Per-wave scratch of one column (doubles): wv the dense weights, ext the column's sparse terms
// by target row (ns entries for the rows of its own node, np for the theta rows), dg the diagonal
// terms of rows of its own species at every node.
__host__ __device__ inline int asm_wave_doubles(const Shape& S) { return (S.K + 1) * S.ns + S.ns + S.np + 8; }

size_t big_asm_lds(const Shape& S) {
  const size_t nd = (size_t)(S.K + 1) * S.ns + (size_t)S.K * (S.lnf + S.lct) + (size_t)S.mmax * (S.K + 1) + 64 +
                    16 * (size_t)asm_wave_doubles(S);
  const size_t ni = 2 * (S.ns + 1) + 3 * (size_t)S.lnf + (S.np + 1) + S.lct + (S.ns + 1) + 2 * (size_t)S.lzs + 1 +
                    S.lzt + (S.np + 1) + S.lpc + S.mmax + 8;
  return sizeof(double) * nd + sizeof(int) * ni;
}

// sum of term(o) over o in [b, e) with four independent partial sums, so that the LDS loads of
// four terms are in flight together
template <typename F>
__device__ inline double sum4(int b, int e, F term) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int o = b;
  for (; o + 4 <= e; o += 4) {
    a0 += term(o);
    a1 += term(o + 1);
    a2 += term(o + 2);
    a3 += term(o + 3);
  }
  for (; o < e; ++o) a0 += term(o);
  return (a0 + a1) + (a2 + a3);
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Element i's matrix over [z (b) | theta (np) | P (ns)] (eq. 2b-2d through J^T Ds J + W): for
// every collocation point k the rows a_jk e_(j,s) - h F_k on node k - h Fth_k on theta, weighted
// by Ds, the node-0 rows (initial condition / continuity), the measurement Hessian and dw on z,
// and the reaction second derivatives.  A column is assembled by one wave: its dense weights
// first (column_prep), then one lane per row, so the products F^T Ds F, Fth^T Ds F and
// Fth^T Ds Fth take one pass over the row's column list.
//
// Dense weights of z column (j, s2): wv[s] = Ds_(j,s) F_j[s][s2] (j >= 1) and
// wv[ns + (k-1) ns + u] = F_k[s2][u], scattered from the nonzeros of F (distinct targets, one
// lane each); ext the sums of its term groups by target row (one lane per group, terms in
// order); dg[j1] the diagonal part of row (j1, s2): sum_k Ds_(k,s2) a_(j1,k) a_(j,k), the
// measurements of s2 in the element, and Ds of node 0 on the (0, 0) block.  Theta column th:
// wv[(k-1) ns + s] = Ds_(k,s) Fth_k[s][th] (a parameter's list may name a species more than once,
// so one lane per point adds its list in order).
__device__ inline void column_prep(const Shape& S, const AsmLds& L, double h, int c, int lane, double* wv) {
  const int ns = S.ns, np = S.np, nr = S.nr, b = S.b, K = S.K;
  double* ext = wv + (K + 1) * ns;
  double* dg = ext + ns + np;
  if (c < b) {
    const int j = c / ns, s2 = c - j * ns;
    for (int s = lane; s < (K + 1) * ns + ns + np; s += 64) wv[s] = 0.0;
    wave_sync();
    if (j >= 1) {
      const double* vf = L.vF + (j - 1) * S.lnf;
      for (int q = L.fcp[s2] + lane; q < L.fcp[s2 + 1]; q += 64) {
        const int s = L.fqs[q];
        wv[s] = L.D[j * ns + s] * vf[q];
      }
    }
    const int r0 = L.frp[s2], nrow = L.frp[s2 + 1] - r0;
    for (int t = lane; t < K * nrow; t += 64) {   // row s2 of F_k
      const int k = t / nrow, o = r0 + t - k * nrow;
      wv[ns + k * ns + L.fru[o]] = L.vF[k * S.lnf + L.frq[o]];
    }
    for (int g = L.zsp[s2] + lane; g < L.zsp[s2 + 1]; g += 64) {
      double v = 0.0;
      for (int t = L.zst[g]; t < L.zst[g + 1]; ++t) {
        const int code = L.ztc[t];
        if (code >= 0) {
          double q = 0.0;
          for (int k = 1; k <= K; ++k) q += L.a[j * 8 + k] * L.D[k * ns + s2] * L.vT[(k - 1) * S.lct + code];
          v += -h * q;
        } else if (j >= 1) {
          const int x = -1 - code, rr = x >> 2, sl = (x >> 1) & 1;
          v += L.hes[((j - 1) * nr + rr) * 4 + ((x & 1) ? 1 + sl : 0)];
        }
      }
      ext[L.zsk[g]] = v;
    }
    if (lane <= K) {
      const int j1 = lane;
      double v = (j1 == 0 && j == 0) ? L.D[s2] : 0.0;
      for (int q = 0; q < L.nmeas; ++q)
        if (L.msp[q] == s2) v += L.mw[q * (K + 1) + j1] * L.mw[q * (K + 1) + j];
      for (int k = 1; k <= K; ++k) v += L.D[k * ns + s2] * L.a[j1 * 8 + k] * L.a[j * 8 + k];
      dg[j1] = v;
    }
  } else if (c < b + np) {
    const int th = c - b;
    for (int t = lane; t < K * ns; t += 64) wv[t] = 0.0;
    wave_sync();
    if (lane < K) {
      const int k = lane + 1;
      const double* vt = L.vT + (k - 1) * S.lct;
      for (int o = L.ctp[th]; o < L.ctp[th + 1]; ++o) {
        const int s = L.cts[o];
        wv[(k - 1) * ns + s] += L.D[k * ns + s] * vt[o];
      }
    }
  }
  wave_sync();
}

// Theta-theta entry (th, th2), th2 <= th: h^2 sum_k (Fth_k^T Ds_k Fth_k)[th][th2] plus, on the
// diagonal, the reactions' second derivatives in their parameter; wv holds the weights of column
// th, so the entry is one pass over th2's column list (the block is symmetric).  Sx + dw are added
// once per instance at the border.
__device__ inline double theta_entry(const Shape& S, const AsmLds& L, double h, int th, int th2, const double* wv) {
  const int ns = S.ns, K = S.K, nr = S.nr;
  double v = 0.0;
  for (int k = 1; k <= K; ++k) {
    const double* vt = L.vT + (k - 1) * S.lct;
    const double* w = wv + (k - 1) * ns;
    v += h * h * sum4(L.ctp[th2], L.ctp[th2 + 1], [&](int o) { return vt[o] * w[L.cts[o]]; });
    if (th == th2)
      for (int o = L.pcp[th]; o < L.pcp[th + 1]; ++o) v += L.hes[((k - 1) * nr + L.pcr[o]) * 4 + 3];
  }
  return v;
}

// One workgroup of 16 waves per element; each wave assembles whole columns (column c by wave
// c mod 16), its lanes on consecutive rows (coalesced stores), after building the column's dense
// weights.  The theta-theta block goes to an FP64 side array, row-major, written by rows.
template <typename T>
__global__ void __launch_bounds__(1024) k_big_asm(Shape S, Tab tb, Ws ws) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, nr = S.nr, K = S.K, b = S.b, R = S.R;
  const BigGeom G = big_geom(S);
  const double h = tb.elem_h[e], dw = ws.dw[inst];
  const int WD = asm_wave_doubles(S);
  AsmLds L;
  L.D = lds;
  L.vF = L.D + (K + 1) * ns;
  L.vT = L.vF + K * S.lnf;
  L.mw = L.vT + K * S.lct;
  L.a = L.mw + S.mmax * (K + 1);
  double* wscr = L.a + 64;   // 16 wave slices of WD doubles
  int* ip = (int*)(wscr + 16 * WD);
  L.fcp = ip; ip += ns + 1;
  L.fqs = ip; ip += S.lnf;
  L.frp = ip; ip += ns + 1;
  L.frq = ip; ip += S.lnf;
  L.fru = ip; ip += S.lnf;
  L.ctp = ip; ip += np + 1;
  L.cts = ip; ip += S.lct;
  L.zsp = ip; ip += ns + 1;
  L.zsk = ip; ip += S.lzs;
  L.zst = ip; ip += S.lzs + 1;
  L.ztc = ip; ip += S.lzt;
  L.pcp = ip; ip += np + 1;
  L.pcr = ip; ip += S.lpc;
  L.msp = ip;
  // instance tables (relative list offsets), element values
  const int fq0 = tb.fq_ptr[inst * (ns + 1)], fr0 = tb.fr_ptr[inst * (ns + 1)], ct0 = tb.ct_ptr[inst * (np + 1)];
  const int zs0 = tb.zs_ptr[inst * (ns + 1)], pc0 = tb.pc_ptr[inst * (np + 1)];
  const int nfq = tb.fq_ptr[inst * (ns + 1) + ns] - fq0, nct = tb.ct_ptr[inst * (np + 1) + np] - ct0;
  const int nzs = tb.zs_ptr[inst * (ns + 1) + ns] - zs0, zt0 = tb.zs_t[zs0];
  const int nzt = tb.zs_t[zs0 + nzs] - zt0, npc = tb.pc_ptr[inst * (np + 1) + np] - pc0;
  const int m0 = tb.elem_mptr[e], nm = tb.elem_mptr[e + 1] - m0;
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  const int64_t jl = (int64_t)K * nr;
  const double* jac = ws.jac + e * jl * 3;
  L.hes = ws.hess + e * jl * 4;
  for (int t = tid(); t <= ns; t += nthr()) {
    L.fcp[t] = tb.fq_ptr[inst * (ns + 1) + t] - fq0;
    L.frp[t] = tb.fr_ptr[inst * (ns + 1) + t] - fr0;
    L.zsp[t] = tb.zs_ptr[inst * (ns + 1) + t] - zs0;
  }
  for (int t = tid(); t <= np; t += nthr()) {
    L.ctp[t] = tb.ct_ptr[inst * (np + 1) + t] - ct0;
    L.pcp[t] = tb.pc_ptr[inst * (np + 1) + t] - pc0;
  }
  for (int t = tid(); t < nfq; t += nthr()) {
    L.fqs[t] = tb.fq_s[fq0 + t];
    L.frq[t] = tb.fr_q[fr0 + t];
    L.fru[t] = tb.fr_u[fr0 + t];
  }
  for (int t = tid(); t < nct; t += nthr()) L.cts[t] = tb.ct_s[ct0 + t];
  for (int t = tid(); t <= nzs; t += nthr()) {
    if (t < nzs) L.zsk[t] = tb.zs_key[zs0 + t];
    L.zst[t] = tb.zs_t[zs0 + t] - zt0;
  }
  for (int t = tid(); t < nzt; t += nthr()) L.ztc[t] = tb.zt_code[zt0 + t];
  for (int t = tid(); t < npc; t += nthr()) L.pcr[t] = tb.pc_r[pc0 + t];
  for (int t = tid(); t < nm; t += nthr()) L.msp[t] = tb.meas_sp[m0 + t];
  for (int t = tid(); t < nm * (K + 1); t += nthr()) L.mw[t] = tb.meas_w[(int64_t)m0 * (K + 1) + t];
  for (int t = tid(); t < b; t += nthr()) L.D[t] = ws.Ds[gi + t];
  for (int t = tid(); t < 64; t += nthr()) L.a[t] = ((t >> 3) <= K && (t & 7) <= K) ? S.a[t >> 3][t & 7] : 0.0;
  for (int t = tid(); t < K * nfq; t += nthr()) {   // nonzeros of F_k, each summed in term order
    const int k = t / nfq, q = t - k * nfq;
    double v = 0.0;
    for (int o = tb.fq_o[fq0 + q]; o < tb.fq_o[fq0 + q + 1]; ++o)
      v += tb.cf_nu[o] * jac[(k * nr + tb.cf_r[o]) * 3 + tb.cf_t[o]];
    L.vF[k * S.lnf + q] = v;
  }
  for (int t = tid(); t < K * nct; t += nthr()) {
    const int k = t / nct, o = t - k * nct;
    L.vT[k * S.lct + o] = tb.ct_nu[ct0 + o] * jac[(k * nr + tb.ct_r[ct0 + o]) * 3 + 2];
  }
  L.nmeas = nm;
  __syncthreads();
  T* A = (T*)ws.ebuf + e * (int64_t)G.Rp * G.Rp;
  double* ath = ws.ath + e * (int64_t)np * np;
  const int wid = tid() >> 6, lane = tid() & 63;
  double* wv = wscr + wid * WD;
  const double* ext = wv + (K + 1) * ns;
  const double* dg = ext + ns + np;
  const double* d0 = L.D;
  for (int c = wid; c < R; c += 16) {
    column_prep(S, L, h, c, lane, wv);
    T* col = A + (int64_t)c * G.Rp;
    if (c < b) {
      const int j2 = c / ns, s2 = c - j2 * ns;
      int r = c + lane, j1 = r / ns, s1 = r - j1 * ns;
      for (; r < b; r += 64) {   // z rows (j1, s1)
        double v = (r == c) ? dw : 0.0;
        if (s1 == s2) v += dg[j1];
        if (j2 >= 1) v -= h * L.a[j1 * 8 + j2] * wv[s1];   // wv[s] = Ds_(j2,s) F_j2[s][s2]
        if (j1 >= 1) v -= h * L.a[j2 * 8 + j1] * L.D[j1 * ns + s2] * wv[ns + (j1 - 1) * ns + s1];   // F_j1[s2][s1]
        if (j1 == j2 && j1 >= 1) {
          // (F^T Ds F)[s1][s2] = sum over column s1's nonzeros of F[s][s1] wv[s]
          const double* vf = L.vF + (j1 - 1) * S.lnf;
          v += h * h * sum4(L.fcp[s1], L.fcp[s1 + 1], [&](int q) { return vf[q] * wv[L.fqs[q]]; }) + ext[s1];
        }
        col[r] = (T)v;
        s1 += 64;
        while (s1 >= ns) {
          s1 -= ns;
          ++j1;
        }
      }
      const double* vt = L.vT + (j2 >= 1 ? j2 - 1 : 0) * S.lct;
      for (int th = lane; th < np; th += 64) {   // theta rows: for j2 >= 1 (Fth_j^T Ds_j F_j)[th][s2]
        double v = ext[ns + th];
        if (j2 >= 1) v += h * h * sum4(L.ctp[th], L.ctp[th + 1], [&](int o) { return vt[o] * wv[L.cts[o]]; });
        col[b + th] = (T)v;
      }
      for (int p = lane; p < ns; p += 64)   // P rows: the previous separator through eq. 2c
        col[b + np + p] = (T)((i != 0 && c == p) ? -d0[p] : 0.0);
    } else if (c < b + np) {
      // theta column th: row th of the theta-theta block (th2 <= th, consecutive lanes on
      // consecutive entries), zeros in the P rows
      const int th = c - b;
      for (int t2 = lane; t2 <= th; t2 += 64) ath[th * np + t2] = theta_entry(S, L, h, th, t2, wv);
      for (int p = lane; p < ns; p += 64) col[b + np + p] = (T)0;
    } else {
      const int pc = c - b - np;
      for (int r = c + lane; r < R; r += 64) col[r] = (T)((i != 0 && r == c) ? d0[pc] : 0.0);
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------- partial Cholesky
// Left-looking partial Cholesky of the first m columns of an n x n SPD matrix (lower triangle,
// column-major, leading dimension ld), for every matrix of a batch.  Columns are eliminated in
// panels of 32, each in two launches:
//   k_pchol_diag   one wave per matrix brings the panel's 32 x 32 diagonal block up to date with
//                  the earlier columns, factors it (each lane one row in registers) and writes the
//                  factor, and its inverse (FP64, row-major) to ws.linv
//   k_pchol_strip  one wave per 32-row strip below: C = A - L_strip L_panel^T, then X = C L^-T,
//                  both as 16x16x4 matrix-core products, with no LDS: the update is formed
//                  transposed (L_panel L_strip^T), and that accumulator is already laid out as
//                  the operand of the solve X^T = L^-1 C^T
// A non-positive or non-finite pivot sets the instance's flag; later launches skip the instance.

// Update products of a 32-row strip (rows r0..) with NP panels of 32 rows (rows pr, pr + 32, ..)
// over the columns [kb, ke): acc[q][jt][rt] element v of the lane = sum_k L[pr + 32 q + 16 jt + i][k]
// L[r0 + 16 rt + li][k], i = Mma<T>::row(lane, v): the (panel, strip) blocks of L L^T transposed.
// Operands are loaded from memory straight into the product's register layout (32-bit byte
// offsets from the matrix base, rows clamped to the matrix: rows past its end give products that
// are never used), the next columns in flight while the current ones are multiplied.  Bit
// 4 q + 2 jt + rt of `skip` (the same in every lane) leaves the 16 x 16 product c[q][jt][rt] out.
template <typename T, int NP>
__device__ inline void panel_products(const T* A, int ld, int n, int kb, int ke, int pr, int r0, int lane,
                                      typename Mma<T>::acc (&c)[NP][2][2], uint32_t skip = 0) {
  constexpr int KU = NP == 1 ? 4 : 2;
  const int li = lane & 15, lk = lane >> 4;
  const char* base = (const char*)A;
  const uint32_t cs = (uint32_t)ld * sizeof(T);
  uint32_t op[NP][2];
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int h = 0; h < 2; ++h) op[q][h] = (uint32_t)min(pr + 32 * q + 16 * h + li, n - 1) * sizeof(T) + lk * cs;
  const uint32_t os0 = (uint32_t)min(r0 + li, n - 1) * sizeof(T) + lk * cs;
  const uint32_t os1 = (uint32_t)min(r0 + 16 + li, n - 1) * sizeof(T) + lk * cs;
  T cp[NP][2][KU], cs0[KU], cs1[KU], np_[NP][2][KU], ns0[KU], ns1[KU];
  auto load = [&](int kc, T (&p)[NP][2][KU], T* s0, T* s1) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const uint32_t off = (uint32_t)(kc + 4 * u) * cs;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        p[q][0][u] = *(const T*)(base + (op[q][0] + off));
        p[q][1][u] = *(const T*)(base + (op[q][1] + off));
      }
      s0[u] = *(const T*)(base + (os0 + off));
      s1[u] = *(const T*)(base + (os1 + off));
    }
  };
  auto mult = [&](const T (&p)[NP][2][KU], const T* s0, const T* s1) {
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        if (!(skip >> (4 * q) & 1)) c[q][0][0] = Mma<T>::mma(p[q][0][u], s0[u], c[q][0][0]);
        if (!(skip >> (4 * q + 1) & 1)) c[q][0][1] = Mma<T>::mma(p[q][0][u], s1[u], c[q][0][1]);
        if (!(skip >> (4 * q + 2) & 1)) c[q][1][0] = Mma<T>::mma(p[q][1][u], s0[u], c[q][1][0]);
        if (!(skip >> (4 * q + 3) & 1)) c[q][1][1] = Mma<T>::mma(p[q][1][u], s1[u], c[q][1][1]);
      }
  };
  const int kfull = kb + (ke > kb ? (ke - kb) / (8 * KU) * (8 * KU) : 0);
  if (kfull > kb) {
    load(kb, cp, cs0, cs1);
    for (int kc = kb; kc < kfull; kc += 8 * KU) {
      load(kc + 4 * KU, np_, ns0, ns1);
      mult(cp, cs0, cs1);
      if (kc + 8 * KU < kfull) load(kc + 8 * KU, cp, cs0, cs1);
      mult(np_, ns0, ns1);
    }
  }
  // ragged end (the trailing update's K = m): columns at or past ke read as zero
  for (int kc = kfull; kc < ke; kc += 4) {
    const bool ok = kc + lk < ke;
    const uint32_t off = (uint32_t)(ok ? kc : ke - 1 - lk) * cs;
    T p[NP][2][1], s0[1], s1[1];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      p[q][0][0] = ok ? *(const T*)(base + (op[q][0] + off)) : (T)0;
      p[q][1][0] = ok ? *(const T*)(base + (op[q][1] + off)) : (T)0;
    }
    s0[0] = ok ? *(const T*)(base + (os0 + off)) : (T)0;
    s1[0] = ok ? *(const T*)(base + (os1 + off)) : (T)0;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      if (!(skip >> (4 * q) & 1)) c[q][0][0] = Mma<T>::mma(p[q][0][0], s0[0], c[q][0][0]);
      if (!(skip >> (4 * q + 1) & 1)) c[q][0][1] = Mma<T>::mma(p[q][0][0], s1[0], c[q][0][1]);
      if (!(skip >> (4 * q + 2) & 1)) c[q][1][0] = Mma<T>::mma(p[q][1][0], s0[0], c[q][1][0]);
      if (!(skip >> (4 * q + 3) & 1)) c[q][1][1] = Mma<T>::mma(p[q][1][0], s1[0], c[q][1][1]);
    }
  }
}

// threadIdx.x % 64 through an empty asm: values derived from it are neither hoisted out of
// loops nor kept alive between the points where it is re-read (register pressure in long
// unrolled code)
__device__ inline int opaque_lane() {
  int l = threadIdx.x & 63;
  __asm__ volatile("" : "+v"(l));
  return l;
}

// One wave per matrix: the diagonal block of the panel at column k0 (wd = min(32, m - k0)
// columns, padded with the identity) brought up to date with the columns [kb, k0) (the earlier
// ones are already applied), its factor into the matrix and its inverse into ws.linv[item]
// (32 x 32, row-major).
template <typename T>
__global__ void __launch_bounds__(64) k_pchol_diag(Tab tb, Ws ws, PArgs a, int k0, int kb) {
  constexpr int NB = 32, PC = NB + 1;
  __shared__ double sC[NB * PC];   // the updated block, then the factor, then its inverse
  __shared__ double sR[NB];        // reciprocals of the pivots' square roots
  typedef typename Mma<T>::acc acc_t;
  if ((int)blockIdx.x >= a.count) return;
  int64_t mat;
  int inst;
  pitem(tb, a, blockIdx.x, mat, inst);
  if (block_flag(&ws.flag[inst])) return;
  T* A = (T*)a.base + mat * a.stride;
  const int n = a.n, ld = a.ld, wd = min(NB, a.m - k0);
  int lane = opaque_lane();
  {
    acc_t c[1][2][2] = {{{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}}};
    panel_products<T, 1>(A, ld, n, kb, k0, k0, k0, lane, c);
    const int li = lane & 15;
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = 16 * jt + Mma<T>::row(lane, v), r = 16 * rt + li;
          const int hi = min(max(r, j), wd - 1), lo = min(min(r, j), wd - 1);   // lower triangle, clamped
          sC[r * PC + j] = (double)A[k0 + hi + (int64_t)(k0 + lo) * ld] - (double)c[0][jt][rt][v];
        }
  }
  wave_sync();
  lane = opaque_lane();
  const int r = lane & 31;
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = (r < wd) ? (j < wd ? sC[r * PC + j] : 0.0) : (r == j ? 1.0 : 0.0);
  wave_sync();
  bool good = true;
  // column j of the updated block passes through row j of sC; lane r keeps row r
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (lane < NB) sC[j * PC + lane] = x[j];
    wave_sync();
    const double piv = sC[j * PC + j];
    if (j < wd) good = good && piv > 0.0 && isfinite(piv);
    const double d = sqrt(piv), inv = 1.0 / d, l = x[j] * inv;
#pragma unroll
    for (int k = j + 1; k < NB; ++k) x[k] -= l * (sC[j * PC + k] * inv);
    x[j] = (r == j) ? d : l;
    if (lane == 0) sR[j] = inv;
    // the updates happen at this step (not sunk towards their use, which would keep every
    // step's multipliers alive)
#pragma unroll
    for (int k = j + 1; k < NB; ++k) __asm__ volatile("" : "+v"(x[k]));
  }
  if (!good) {
    if (lane == 0) atomicOr(&ws.flag[inst], 1);
    return;
  }
  wave_sync();
  if (lane < NB) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      sC[r * PC + j] = j <= r ? x[j] : 0.0;
      if (j <= r && r < wd) A[k0 + r + (int64_t)(k0 + j) * ld] = (T)x[j];
    }
  }
  wave_sync();
  // inverse: lane c forms column c by forward substitution; every lane reads row i of the
  // factor before row i of the inverse replaces it
  double* Li = ws.linv + (int64_t)blockIdx.x * NB * NB;
  double y[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double sum = (i == r) ? 1.0 : 0.0;
#pragma unroll
    for (int p = 0; p < i; ++p) sum -= sC[i * PC + p] * y[p];
    y[i] = sum * sR[i];
    if (lane < NB) Li[i * NB + r] = y[i];
    __asm__ volatile("" ::: "memory");   // row by row: keeps the factor reads from piling up in registers
  }
}

// Strips below the diagonal block of the panel at column k0: grid = items x groups of four
// strips (one per wave), the groups of one item on one XCD (block id mod 8) in consecutive
// dispatch order so that its panel rows and inverse factor are shared through that XCD's L2.
// The strips are brought up to date with the columns [kb, k0) and solved.  Strips start at s0
// (0 when the panel is narrower than 32 and its diagonal strip holds rows below the block); only
// rows at or below k0 + wd are written.  LOOK: the same pass over the strip rows also applies
// the columns [kb, k0) to the next panel's columns (k0 + 32..), which then need only this panel.
template <typename T, int LOOK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LOOK ? 3 : 4)))
k_pchol_strip(Tab tb, Ws ws, PArgs a, int k0, int kb, int s0, int groups) {
  constexpr int NB = 32, NP = LOOK ? 2 : 1;
  typedef typename Mma<T>::acc acc_t;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int item = (slot / groups) * 8 + xcd, g = slot % groups;
  if (item >= a.count) return;
  int64_t mat;
  int inst;
  pitem(tb, a, item, mat, inst);
  if (block_flag(&ws.flag[inst])) return;
  const int n = a.n, ld = a.ld, wd = min(NB, a.m - k0);
  const int r0 = k0 + NB * (s0 + 4 * g + (int)(threadIdx.x >> 6));
  if (r0 >= n) return;
  T* A = (T*)a.base + mat * a.stride;
  int lane = opaque_lane();
  acc_t c[NP][2][2];
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int h = 0; h < 2; ++h) c[q][h][0] = c[q][h][1] = acc_t{0, 0, 0, 0};
  panel_products<T, NP>(A, ld, n, kb, k0, k0, r0, lane, c);
  lane = opaque_lane();
  const int li = lane & 15, lk = lane >> 4;
  if (LOOK) {
    // next panel (columns k1..): A -= products, rows at or below the diagonal
    const int k1 = k0 + NB, wd1 = min(NB, a.m - k1);
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = 16 * jt + Mma<T>::row(lane, v), r = r0 + 16 * rt + li;
          if (j < wd1 && r < n && r >= k1 + j) {
            T* p = A + r + (int64_t)(k1 + j) * ld;
            *p = (T)((double)*p - (double)c[NP - 1][jt][rt][v]);
          }
        }
  }
  // C^T = A^T - products (FP64), in the accumulators' layout; 0 right of the panel
  double ct[2][2][4];
#pragma unroll
  for (int jt = 0; jt < 2; ++jt)
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 16 * jt + Mma<T>::row(lane, v), r = min(r0 + 16 * rt + li, n - 1);
        const double av = (double)A[r + (int64_t)(k0 + min(j, wd - 1)) * ld];
        ct[jt][rt][v] = j < wd ? av - (double)c[0][jt][rt][v] : 0.0;
      }
  // X^T = L^-1 C^T on matrix cores: K index j of step (jt, v) for lane group lk is
  // 16 jt + Mma<T>::row(lane, v), the layout the update products left C^T in; the inverse is
  // lower triangular, so rows [0, 16) of X^T need only j < 16
  const double* Li = ws.linv + (int64_t)item * NB * NB;
  dvec4 x[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
#pragma unroll
  for (int jt = 0; jt < 2; ++jt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = 16 * jt + Mma<T>::row(lane, v);
      const double a1 = Li[(16 + li) * NB + j];
      x[1][0] = Mma<double>::mma(a1, ct[jt][0][v], x[1][0]);
      x[1][1] = Mma<double>::mma(a1, ct[jt][1][v], x[1][1]);
      if (jt == 0) {
        const double a0 = Li[li * NB + j];
        x[0][0] = Mma<double>::mma(a0, ct[0][0][v], x[0][0]);
        x[0][1] = Mma<double>::mma(a0, ct[0][1][v], x[0][1]);
      }
    }
  // element v of x[ct][rt]: X[r0 + 16 rt + li][k0 + 16 ct + lk + 4 v]
#pragma unroll
  for (int ctl = 0; ctl < 2; ++ctl)
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * rt + li, j = 16 * ctl + lk + 4 * v;
        if (j < wd && r < n && r >= k0 + wd) A[r + (int64_t)(k0 + j) * ld] = (T)x[ctl][rt][v];
      }
}

// Trailing update C = C - X X^T (or -X X^T when the block starts at zero) of the rows and columns
// [m, n), X = L[m:n, 0:m], in blocks of 32 rows x 64 columns of the lower triangle, one per wave:
// the strip products above with the block's columns in the place of the panel rows.  Blocks
// inside [skip0, skip1)^2 are left out.  The blocks of one matrix go to one XCD (block id mod 8)
// in consecutive dispatch order, so its X rows are read from HBM into that XCD's L2 once.
__host__ __device__ inline bool trail_skipped(const PArgs& a, int s, int cb) {
  const int r0 = a.m + 32 * s, c0 = a.m + 64 * cb;
  return r0 >= a.skip0 && min(r0 + 32, a.n) <= a.skip1 && c0 >= a.skip0 && min(c0 + 64, a.n) <= a.skip1;
}
// Block bi of the enumeration (strips in order, then column blocks): s, cb; false past the end.
__host__ __device__ inline bool trail_block(const PArgs& a, int bi, int& s, int& cb) {
  const int t = a.n - a.m, nst = (t + 31) / 32, ncb = (t + 63) / 64;
  int k = 0;
  for (int ss = 0; ss < nst; ++ss) {
    const int cmax = min(ncb - 1, (32 * ss + 31) / 64);
    for (int cc = 0; cc <= cmax; ++cc) {
      if (trail_skipped(a, ss, cc)) continue;
      if (k == bi) {
        s = ss;
        cb = cc;
        return true;
      }
      ++k;
    }
  }
  return false;
}

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_pchol_trail(Tab tb, Ws ws, PArgs a, int groups) {
  typedef typename Mma<T>::acc acc_t;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int item = (slot / groups) * 8 + xcd, g = slot % groups;
  if (item >= a.count) return;
  int s, cb;
  if (!trail_block(a, 4 * g + (int)(threadIdx.x >> 6), s, cb)) return;
  int64_t mat;
  int inst;
  pitem(tb, a, item, mat, inst);
  if (block_flag(&ws.flag[inst])) return;
  const int n = a.n, ld = a.ld, r0 = a.m + 32 * s, c0 = a.m + 64 * cb;
  T* A = (T*)a.base + mat * a.stride;
  int lane = opaque_lane();
  acc_t c[2][2][2];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int h = 0; h < 2; ++h) c[q][h][0] = c[q][h][1] = acc_t{0, 0, 0, 0};
  // 16 x 16 products not stored: wholly above the diagonal, past the matrix, or inside the
  // square left out [skip0, skip1)^2
  uint32_t skip = 0;
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const int cs = c0 + 32 * q + 16 * jt, rs = r0 + 16 * rt;
        const bool above = cs >= rs + 16, past = rs >= n || cs >= n;
        const bool inner = rs >= a.skip0 && rs + 16 <= a.skip1 && cs >= a.skip0 && cs + 16 <= a.skip1;
        if (above || past || inner) skip |= 1u << (4 * q + 2 * jt + rt);
      }
  panel_products<T, 2>(A, ld, n, 0, a.m, c0, r0, lane, c, skip);
  lane = opaque_lane();
  const int li = lane & 15;
  // element v of c[q][jt][rt]: column c0 + 32 q + 16 jt + row(lane, v), row r0 + 16 rt + li
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = c0 + 32 * q + 16 * jt + Mma<T>::row(lane, v), row = r0 + 16 * rt + li;
          if (row < n && row >= col) {
            T* p = A + row + (int64_t)col * ld;
            *p = a.zero ? -c[q][jt][rt][v] : *p - c[q][jt][rt][v];
          }
        }
}

// ---------------------------------------------------------------- cyclic reduction gathers
// Separator s's local matrix (sbuf, ld Lp): rows [0, ns) its block T_s, [ns, 2 ns) the coupling to
// its left neighbour E_L(a, q) = K(left_a, s_q), [2 ns, 3 ns) to its right neighbour, [3 ns, Lr) the
// theta border G_s; columns [0, ns).  After elimination the trailing block (rows and columns from
// ns) holds -X X^T: C_LL, C_RL (the new coupling between the neighbours), C_RR, C_thL, C_thR.
template <typename T>
__device__ inline T& sep_at(const Ws& ws, const BigGeom& G, int64_t es, int r, int c) {
  return ((T*)ws.sbuf)[es * (int64_t)G.Lp * G.Lp + r + (int64_t)c * G.Lp];
}
template <typename T>
__device__ inline T elem_at(const Ws& ws, const BigGeom& G, int64_t e, int r, int c) {
  return ((const T*)ws.ebuf)[e * (int64_t)G.Rp * G.Rp + r + (int64_t)c * G.Rp];
}

// One band of 32 rows of a destination block (rows x cols, column-major, ld ldd) filled in 32 x 32
// tiles: v = (add ? dst : 0) + s1 + s2, summed in that order, lower triangle only if `lower`.  A
// source is read straight (src[r + c ld]) or transposed (src[c + r ld]); a transposed one is
// staged through LDS, so every read and write is coalesced.  Absent sources (p == nullptr) add
// nothing.
struct GSrc {
  const void* p;
  int ld, tr;
};
template <typename T>
__device__ inline double gsrc(const GSrc& g, int r, int c) {
  const T* q = (const T*)g.p;
  return g.tr ? (double)q[c + (int64_t)r * g.ld] : (double)q[r + (int64_t)c * g.ld];
}
template <typename T>
__device__ void gather_band(T* dst, int ldd, int rows, int cols, int r0, bool add, bool lower, GSrc s1,
                            GSrc s2, double* tiles) {
  // four groups of 256 threads take four column tiles at a time
  const int t = threadIdx.x & 255, grp = threadIdx.x >> 8;
  double* tile = tiles + grp * 32 * 33;
  const bool tr = (s1.p && s1.tr) || (s2.p && s2.tr);
  for (int cg = 0; cg < cols; cg += 128) {
    const int c0 = cg + 32 * grp;
    const bool act = c0 < cols && !(lower && c0 > r0 + 31);
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int idx = t + 256 * k, r = r0 + (idx & 31), c = c0 + (idx >> 5);
      double x = 0.0;
      if (act && r < rows && c < cols) {
        if (add) x = (double)dst[r + (int64_t)c * ldd];
        if (s1.p && !s1.tr) x += gsrc<T>(s1, r, c);
        if (s2.p && !s2.tr) x += gsrc<T>(s2, r, c);
      }
      v[k] = x;
    }
    if (tr) {
      __syncthreads();   // the previous tiles' reads are done
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int idx = t + 256 * k, c = c0 + (idx & 31), rr = idx >> 5, r = r0 + rr;
        double x = 0.0;
        if (act && r < rows && c < cols) {
          if (s1.p && s1.tr) x += gsrc<T>(s1, r, c);
          if (s2.p && s2.tr) x += gsrc<T>(s2, r, c);
        }
        tile[rr * 33 + (idx & 31)] = x;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int idx = t + 256 * k;
        v[k] += tile[(idx & 31) * 33 + (idx >> 5)];
      }
    }
    if (act) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int idx = t + 256 * k, r = r0 + (idx & 31), c = c0 + (idx >> 5);
        if (r < rows && c < cols && (!lower || r >= c)) dst[r + (int64_t)c * ldd] = (T)v[k];
      }
    }
  }
}

// Bands of a separator's gathers: T (ns rows), E_L (ns), E_R (ns), G (np), 32 rows each.
__host__ __device__ inline int gather_bands(const Shape& S) {
  return 3 * (int)cl_ceil_div(S.ns, 32) + (int)cl_ceil_div(S.np, 32);
}
__device__ inline void gather_op(const Shape& S, int band, int& op, int& r0) {
  const int bs = (int)cl_ceil_div(S.ns, 32);
  op = band < 3 * bs ? band / bs : 3;
  r0 = 32 * (op < 3 ? band - op * bs : band - 3 * bs);
}

// After level 0: every separator's T_s and G_s from the Schur complements of element s (its S
// block) and element s + 1 (its P block); the couplings of the separators eliminated at level 1.
// grid (element, band).
template <typename T>
__global__ void __launch_bounds__(1024) k_sep_init(Shape S, Tab tb, Ws ws) {
  __shared__ double tile[4 * 32 * 33];
  const int64_t es = blockIdx.x;
  const int inst = tb.elem_inst[es], s = tb.elem_loc[es];
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, b = S.b, mI = S.mI, N = tb.inst_N[inst];
  const BigGeom G = big_geom(S);
  const bool nxt = s + 1 < N, elim1 = (s & 1) != 0;
  const int P0 = b + np;   // first P row of an element
  int op, r0;
  gather_op(S, blockIdx.y, op, r0);
  if ((op == 1 || op == 2) && !elim1) return;
  const T* e = (const T*)ws.ebuf + es * (int64_t)G.Rp * G.Rp;
  const T* en = e + (int64_t)G.Rp * G.Rp;   // element s + 1 (read only when it exists)
  T* d = &sep_at<T>(ws, G, es, 0, 0);
  const GSrc none = {nullptr, 0, 0};
  if (op == 0)   // T_s = S block of element s + P block of element s + 1
    gather_band<T>(d, G.Lp, ns, ns, r0, false, true, GSrc{e + mI + (int64_t)mI * G.Rp, G.Rp, 0},
                   nxt ? GSrc{en + P0 + (int64_t)P0 * G.Rp, G.Rp, 0} : none, tile);
  else if (op == 1)   // E_L(a, q) = K(P_a of element s, S_q)
    gather_band<T>(d + ns, G.Lp, ns, ns, r0, false, false, GSrc{e + P0 + (int64_t)mI * G.Rp, G.Rp, 0}, none, tile);
  else if (op == 2)   // E_R(a, q) = K(P_q of element s + 1, S_a of element s + 1)
    gather_band<T>(d + 2 * ns, G.Lp, ns, ns, r0, false, false,
                   nxt ? GSrc{en + P0 + (int64_t)mI * G.Rp, G.Rp, 1} : none, none, tile);
  else   // G_s(c, q) = K(theta_c, S_q) of element s + K(P_q, theta_c) of element s + 1
    gather_band<T>(d + 3 * ns, G.Lp, np, ns, r0, false, false, GSrc{e + b + (int64_t)mI * G.Rp, G.Rp, 0},
                   nxt ? GSrc{en + P0 + (int64_t)b * G.Rp, G.Rp, 1} : none, tile);
}

// Step l (1..L-1): separators t that are multiples of 2^l add the contributions of the
// separators eliminated at level l on either side (u1 = t - 2^(l-1): t is its right neighbour;
// u2 = t + 2^(l-1): t is its left neighbour), in that order; those eliminated at level l+1 also
// take their new couplings.  grid (separator, band).
template <typename T>
__global__ void __launch_bounds__(1024) k_sep_step(Shape S, Tab tb, Ws ws, int level) {
  __shared__ double tile[4 * 32 * 33];
  const int it = tb.st_ptr[level - 1] + blockIdx.x;
  if (it >= tb.st_ptr[level]) return;
  const int inst = tb.st_inst[it], t = tb.st_s[it];
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, N = tb.inst_N[inst];
  const BigGeom G = big_geom(S);
  const int64_t e0 = tb.inst_e0[inst], et = e0 + t;
  const int half = 1 << (level - 1);
  const bool h1 = t > 0, h2 = t + half < N;
  const int64_t u1 = e0 + t - half, u2 = e0 + t + half;
  const bool elim = ((t >> level) & 1) != 0;
  const bool right = elim && h2 && t + 2 * half < N;
  int op, r0;
  gather_op(S, blockIdx.y, op, r0);
  if ((op == 1 || op == 2) && !elim) return;
  T* d = &sep_at<T>(ws, G, et, 0, 0);
  const T* a1 = h1 ? &sep_at<T>(ws, G, u1, 0, 0) : nullptr;
  const T* a2 = h2 ? &sep_at<T>(ws, G, u2, 0, 0) : nullptr;
  const GSrc none = {nullptr, 0, 0};
  if (op == 0)   // T_t += C_RR of u1 + C_LL of u2
    gather_band<T>(d, G.Lp, ns, ns, r0, true, true,
                   h1 ? GSrc{a1 + 2 * ns + (int64_t)2 * ns * G.Lp, G.Lp, 0} : none,
                   h2 ? GSrc{a2 + ns + (int64_t)ns * G.Lp, G.Lp, 0} : none, tile);
  else if (op == 1)   // E_L(a, q) = C_RL of u1 at (q, a)
    gather_band<T>(d + ns, G.Lp, ns, ns, r0, false, false, GSrc{a1 + 2 * ns + (int64_t)ns * G.Lp, G.Lp, 1},
                   none, tile);
  else if (op == 2)   // E_R(a, q) = C_RL of u2 at (a, q) when t + 2^l is a separator
    gather_band<T>(d + 2 * ns, G.Lp, ns, ns, r0, false, false,
                   right ? GSrc{a2 + 2 * ns + (int64_t)ns * G.Lp, G.Lp, 0} : none, none, tile);
  else   // G_t += C_thR of u1 + C_thL of u2
    gather_band<T>(d + 3 * ns, G.Lp, np, ns, r0, true, false,
                   h1 ? GSrc{a1 + 3 * ns + (int64_t)2 * ns * G.Lp, G.Lp, 0} : none,
                   h2 ? GSrc{a2 + 3 * ns + (int64_t)ns * G.Lp, G.Lp, 0} : none, tile);
}

// ---------------------------------------------------------------- border
// theta-theta partials of one 16-element chunk and one 64 x 64 lower tile of the parameter
// block, in FP64 on matrix cores: sum of the elements' assembled theta blocks minus the products of
// their transformed theta rows (elements: mI columns each; separators 1.. of the chunk: ns
// columns each).  grid (chunk-tile slots, instance): the tiles of one chunk go to one XCD (block id
// mod 8) in consecutive dispatch order, so each theta row is read from HBM once and shared by the
// chunk's tiles through that XCD's L2.
template <typename T>
__global__ void __launch_bounds__(256) k_big_theta(Shape S, Tab tb, Ws ws, int ntile) {
  constexpr int TM = 64, KC = 32, NL = KC * TM / 256;
  __shared__ double sA[KC * TM];
  __shared__ double sB[KC * TM];
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int inst = blockIdx.y, chunk = (slot / ntile) * 8 + xcd, tile = slot % ntile;
  if (chunk >= ws.nchunk) return;
  if (block_flag(&ws.flag[inst])) return;
  const int np = S.np, ns = S.ns, b = S.b, mI = S.mI, N = tb.inst_N[inst];
  const BigGeom G = big_geom(S);
  const int i0 = chunk * CL_THCHUNK, i1 = min(N, i0 + CL_THCHUNK);
  if (i0 >= N) return;
  int ti = (int)((sqrtf(8.0f * (float)tile + 1.0f) - 1.0f) * 0.5f);
  while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
  while (ti * (ti + 1) / 2 > tile) --ti;
  const int tj = tile - ti * (ti + 1) / 2;
  const int R0 = TM * ti, C0 = TM * tj;
  const int64_t e0 = tb.inst_e0[inst];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wr = w >> 1, wc = w & 1;
  dvec4 c00 = {0, 0, 0, 0}, c01 = {0, 0, 0, 0}, c10 = {0, 0, 0, 0}, c11 = {0, 0, 0, 0};
  for (int ii = i0; ii < i1; ++ii) {
    for (int src = 0; src < 2; ++src) {   // the element's theta rows, then separator ii's
      if (src == 1 && ii == 0) continue;
      const T* X = src == 0 ? (const T*)ws.ebuf + (e0 + ii) * (int64_t)G.Rp * G.Rp + b
                            : (const T*)ws.sbuf + (e0 + ii) * (int64_t)G.Lp * G.Lp + 3 * ns;
      const int ldx = src == 0 ? G.Rp : G.Lp, kn = src == 0 ? mI : ns;
      double ra[NL], rb[NL];
      auto load = [&](int kc) {
#pragma unroll
        for (int q = 0; q < NL; ++q) {
          const int r = t & (TM - 1), kk = (t >> 6) + 4 * q, k = kc + kk;
          ra[q] = (R0 + r < np && k < kn) ? (double)X[R0 + r + (int64_t)k * ldx] : 0.0;
          rb[q] = (C0 + r < np && k < kn) ? (double)X[C0 + r + (int64_t)k * ldx] : 0.0;
        }
      };
      load(0);
      for (int kc = 0; kc < kn; kc += KC) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NL; ++q) {
          sA[((t >> 6) + 4 * q) * TM + (t & (TM - 1))] = ra[q];
          sB[((t >> 6) + 4 * q) * TM + (t & (TM - 1))] = rb[q];
        }
        __syncthreads();
        if (kc + KC < kn) load(kc + KC);
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
          const int kk = 4 * s + (lane >> 4), li = lane & 15;
          const double a0 = sA[kk * TM + 32 * wr + li], a1 = sA[kk * TM + 32 * wr + 16 + li];
          const double b0 = sB[kk * TM + 32 * wc + li], b1 = sB[kk * TM + 32 * wc + 16 + li];
          c00 = Mma<double>::mma(a0, b0, c00);
          c01 = Mma<double>::mma(a0, b1, c01);
          c10 = Mma<double>::mma(a1, b0, c10);
          c11 = Mma<double>::mma(a1, b1, c11);
        }
      }
    }
  }
  double* out = ws.thred + ((int64_t)inst * ws.nchunk + chunk) * np * np;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rb = R0 + 32 * wr + Mma<double>::row(lane, v), cb = C0 + 32 * wc + (lane & 15);
    const double vals[4] = {c00[v], c01[v], c10[v], c11[v]};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = rb + 16 * (q >> 1), c = cb + 16 * (q & 1);
      if (r < np && c < np && r >= c) {
        double acc = 0.0;   // the chunk's assembled blocks, element order
        for (int ii = i0; ii < i1; ++ii) acc += ws.ath[(e0 + ii) * (int64_t)np * np + r * np + c];
        out[r * np + c] = acc - vals[q];
      }
    }
  }
}

// Border matrix of each instance (FP64, ld Bp): [T_0 | G_0^T; G_0 | S_thth], where separator 0
// takes the contributions of the separator eliminated at the last level (its theta-theta block is
// written by k_border_theta).
template <typename T>
__global__ void __launch_bounds__(256) k_border_build(Shape S, Tab tb, Ws ws) {
  const int inst = blockIdx.x;
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, N = tb.inst_N[inst], L = tb.L;
  const BigGeom G = big_geom(S);
  const int64_t e0 = tb.inst_e0[inst];
  const int u = L >= 1 ? (1 << (L - 1)) : N;
  const bool hu = u < N;
  double* B = ws.bbuf + (int64_t)inst * G.Bp * G.Bp;
  for (int idx = tid(); idx < ns * ns; idx += nthr()) {
    const int q = idx / ns, a = idx - q * ns;
    if (a < q) continue;
    double v = (double)sep_at<T>(ws, G, e0, a, q);
    if (hu) v += (double)sep_at<T>(ws, G, e0 + u, ns + a, ns + q);
    B[a + (int64_t)q * G.Bp] = v;
  }
  for (int idx = tid(); idx < np * ns; idx += nthr()) {
    const int q = idx / np, c = idx - q * np;
    double v = (double)sep_at<T>(ws, G, e0, 3 * ns + c, q);
    if (hu) v += (double)sep_at<T>(ws, G, e0 + u, 3 * ns + c, ns + q);
    B[ns + c + (int64_t)q * G.Bp] = v;
  }
}

// theta-theta block of the border matrix: sum of the chunk partials in chunk order + Sx + dw;
// grid (entry tile of 256, instance).
__global__ void __launch_bounds__(256) k_border_theta(Shape S, Tab tb, Ws ws) {
  const int inst = blockIdx.y;
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, N = tb.inst_N[inst];
  const BigGeom G = big_geom(S);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= np * np) return;
  const int r = idx / np, c = idx - r * np;
  if (c > r) return;
  const int nch = (int)cl_ceil_div(N, CL_THCHUNK);
  const double* src = ws.thred + (int64_t)inst * ws.nchunk * np * np + idx;
  double a0 = 0.0, a1 = 0.0;   // two interleaved partial sums, combined in a fixed order
  int ch = 0;
  for (; ch + 2 <= nch; ch += 2) {
    a0 += src[(int64_t)ch * np * np];
    a1 += src[(int64_t)(ch + 1) * np * np];
  }
  if (ch < nch) a0 += src[(int64_t)ch * np * np];
  double acc = a0 + a1;
  if (r == c) acc += ws.sxdw[inst * np + r];
  ws.bbuf[(int64_t)inst * G.Bp * G.Bp + ns + r + (int64_t)(ns + c) * G.Bp] = acc;
}

// ---------------------------------------------------------------- solves
// Workgroup-cooperative substitutions with an n x n column-major factor whose first m columns are
// eliminated: v (LDS, n doubles).  fwd: v[0:m] <- L11^-1 v[0:m], v[m:n] <- v[m:n] - L21 v[0:m].
// bwd: v[0:m] <- L11^-T (v[0:m] - L21^T v[m:n]).  Diagonal blocks of 64 are staged in LDS and
// solved by wave 0 with the right-hand side in registers; the other rows or columns are updated
// by all threads with four independent partial sums.  blk: 64 x 65 doubles of LDS.
template <typename T>
__device__ inline void stage_diag(const T* L, int ld, int c0, int bw, double* blk) {
  for (int idx = tid(); idx < 64 * 64; idx += nthr()) {
    const int c = idx >> 6, r = idx & 63;
    blk[r * 65 + c] = (r < bw && c < bw && r >= c) ? (double)L[(c0 + r) + (int64_t)(c0 + c) * ld] : 0.0;
  }
}

template <typename T>
__device__ void blocked_fwd(const T* L, int ld, int m, int n, double* v, double* blk) {
  for (int c0 = 0; c0 < m; c0 += 64) {
    const int bw = min(64, m - c0);
    __syncthreads();
    stage_diag(L, ld, c0, bw, blk);
    __syncthreads();
    if (tid() < 64) {
      const int lane = tid();
      double x = lane < bw ? v[c0 + lane] : 0.0;
      for (int j = 0; j < bw; ++j) {
        const double xj = __shfl(x, j) / blk[j * 65 + j];
        if (lane == j) x = xj;
        if (lane > j && lane < bw) x -= blk[lane * 65 + j] * xj;
      }
      if (lane < bw) v[c0 + lane] = x;
    }
    __syncthreads();
    for (int r = c0 + bw + tid(); r < n; r += nthr()) {
      const T* row = L + r + (int64_t)c0 * ld;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int c = 0;
      for (; c + 4 <= bw; c += 4) {
        s0 += (double)row[(int64_t)c * ld] * v[c0 + c];
        s1 += (double)row[(int64_t)(c + 1) * ld] * v[c0 + c + 1];
        s2 += (double)row[(int64_t)(c + 2) * ld] * v[c0 + c + 2];
        s3 += (double)row[(int64_t)(c + 3) * ld] * v[c0 + c + 3];
      }
      for (; c < bw; ++c) s0 += (double)row[(int64_t)c * ld] * v[c0 + c];
      v[r] -= (s0 + s1) + (s2 + s3);
    }
  }
  __syncthreads();
}

// sum over rows r in [r0, r1) of L[r, c] v[r] for columns c in [c0, c0 + cw), subtracted from
// v[c]: four threads per column (rows interleaved by 4), partial sums combined in a fixed order.
template <typename T>
__device__ inline void col_update(const T* L, int ld, int c0, int cw, int r0, int r1, double* v, double* red) {
  for (int cb = 0; cb < cw; cb += 64) {
    const int c = cb + (tid() >> 2), part = tid() & 3;
    double s = 0.0;
    if (c < cw) {
      const T* col = L + (int64_t)(c0 + c) * ld;
      for (int r = r0 + part; r < r1; r += 4) s += (double)col[r] * v[r];
    }
    red[tid()] = s;
    __syncthreads();
    if (part == 0 && c < cw) v[c0 + c] -= (red[tid()] + red[tid() + 1]) + (red[tid() + 2] + red[tid() + 3]);
    __syncthreads();
  }
}

template <typename T>
__device__ void blocked_bwd(const T* L, int ld, int m, int n, double* v, double* blk, double* red) {
  __syncthreads();
  col_update(L, ld, 0, m, m, n, v, red);
  for (int c0 = ((m - 1) / 64) * 64; c0 >= 0; c0 -= 64) {
    const int bw = min(64, m - c0);
    col_update(L, ld, c0, bw, c0 + bw, m, v, red);
    stage_diag(L, ld, c0, bw, blk);
    __syncthreads();
    if (tid() < 64) {
      const int lane = tid();
      double x = lane < bw ? v[c0 + lane] : 0.0;
      for (int j = bw - 1; j >= 0; --j) {
        const double xj = __shfl(x, j) / blk[j * 65 + j];
        if (lane == j) x = xj;
        if (lane < j) x -= blk[j * 65 + lane] * xj;
      }
      if (lane < bw) v[c0 + lane] = x;
    }
    __syncthreads();
  }
}

// Element forward: v = [r_I | 0] -> [y_I | -X y_I] kept in evec (theta and P parts included).
template <typename T>
__global__ void __launch_bounds__(256) k_big_fwd(Shape S, Tab tb, Ws ws, const double* __restrict__ rhs) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const BigGeom G = big_geom(S);
  const int R = S.R, mI = S.mI;
  double* v = lds;
  double* blk = v + G.Rp;
  const double* r = rhs + tb.inst_x[inst] + (int64_t)i * S.b;
  for (int q = tid(); q < R; q += nthr()) v[q] = q < mI ? r[q] : 0.0;
  blocked_fwd((const T*)ws.ebuf + e * (int64_t)G.Rp * G.Rp, G.Rp, mI, R, v, blk);
  for (int q = tid(); q < R; q += nthr()) ws.evec[e * (int64_t)G.Rp + q] = v[q];
}

// Separator right-hand sides after level 0: r_s = rhs(node K of element s) - X_S y (element s)
// - X_P y (element s + 1).
__global__ void k_big_seprhs(Shape S, Tab tb, Ws ws, const double* __restrict__ rhs) {
  const int64_t es = blockIdx.x;
  const int inst = tb.elem_inst[es], s = tb.elem_loc[es];
  if (block_flag(&ws.flag[inst])) return;
  const BigGeom G = big_geom(S);
  const int ns = S.ns, N = tb.inst_N[inst], P0 = S.b + S.np;
  for (int a = tid(); a < ns; a += nthr()) {
    double v = rhs[tb.inst_x[inst] + (int64_t)s * S.b + S.mI + a] + ws.evec[es * (int64_t)G.Rp + S.mI + a];
    if (s + 1 < N) v += ws.evec[(es + 1) * (int64_t)G.Rp + P0 + a];
    ws.rcur[es * ns + a] = v;
  }
}

// Cyclic-reduction forward of the separators eliminated at `level`: y = L_s^-1 r_s and their
// contributions -X y to the neighbours and theta (svec).
template <typename T>
__global__ void __launch_bounds__(256) k_big_crf(Shape S, Tab tb, Ws ws, int level) {
  extern __shared__ double lds[];
  const int it = tb.cr_ptr[level - 1] + blockIdx.x;
  if (it >= tb.cr_ptr[level]) return;
  const int inst = tb.cr_inst[it];
  if (block_flag(&ws.flag[inst])) return;
  const BigGeom G = big_geom(S);
  const int ns = S.ns;
  const int64_t es = tb.inst_e0[inst] + tb.cr_j[it];
  double* v = lds;
  double* blk = v + G.Lp;
  for (int q = tid(); q < G.Lr; q += nthr()) v[q] = q < ns ? ws.rcur[es * ns + q] : 0.0;
  blocked_fwd((const T*)ws.sbuf + es * (int64_t)G.Lp * G.Lp, G.Lp, ns, G.Lr, v, blk);
  for (int q = tid(); q < G.Lr; q += nthr()) ws.svec[es * (int64_t)G.Lp + q] = v[q];
}

// Right-hand sides of the separators that are multiples of 2^l after level l: add the
// contributions of the separators eliminated at level l on either side.
__global__ void k_big_crs(Shape S, Tab tb, Ws ws, int level) {
  const int it = tb.st_ptr[level - 1] + blockIdx.x;
  if (it >= tb.st_ptr[level]) return;
  const int inst = tb.st_inst[it], t = tb.st_s[it];
  if (block_flag(&ws.flag[inst])) return;
  const BigGeom G = big_geom(S);
  const int ns = S.ns, N = tb.inst_N[inst], half = 1 << (level - 1);
  const int64_t e0 = tb.inst_e0[inst], et = e0 + t;
  for (int a = tid(); a < ns; a += nthr()) {
    double v = ws.rcur[et * ns + a];
    if (t > 0) v += ws.svec[(et - half) * (int64_t)G.Lp + 2 * ns + a];
    if (t + half < N) v += ws.svec[(et + half) * (int64_t)G.Lp + ns + a];
    ws.rcur[et * ns + a] = v;
  }
}

// theta right-hand-side partials over 16-element chunks (fixed order): the elements'
// contributions, the eliminated separators' contributions and the optional per-element partials.
__global__ void k_big_thv(Shape S, Tab tb, Ws ws, const double* __restrict__ rthp) {
  const int inst = blockIdx.y, chunk = blockIdx.x;
  if (block_flag(&ws.flag[inst])) return;
  const BigGeom G = big_geom(S);
  const int np = S.np, ns = S.ns, N = tb.inst_N[inst];
  const int i0 = chunk * CL_THCHUNK, i1 = min(N, i0 + CL_THCHUNK);
  const int64_t e0 = tb.inst_e0[inst];
  for (int c = tid(); c < np; c += nthr()) {
    double acc = 0.0;
    for (int ii = i0; ii < i1; ++ii) {
      acc += ws.evec[(e0 + ii) * (int64_t)G.Rp + S.b + c];
      if (rthp) acc += rthp[(e0 + ii) * np + c];
      if (ii > 0) acc += ws.svec[(e0 + ii) * (int64_t)G.Lp + 3 * ns + c];
    }
    ws.thv[((int64_t)inst * ws.nchunk + chunk) * np + c] = acc;
  }
}

// Border solve: [separator 0 | theta] with the border factor; x_theta into dx, x_0 into xsep.
__global__ void __launch_bounds__(256) k_big_border_solve(Shape S, Tab tb, Ws ws, const double* __restrict__ rhs,
                                                          double* __restrict__ dx) {
  extern __shared__ double lds[];
  const int inst = blockIdx.x;
  if (block_flag(&ws.flag[inst])) return;
  const BigGeom G = big_geom(S);
  const int ns = S.ns, np = S.np, N = tb.inst_N[inst], L = tb.L;
  const int64_t e0 = tb.inst_e0[inst], xt = tb.inst_x[inst] + (int64_t)N * S.b;
  const int u = L >= 1 ? (1 << (L - 1)) : N;
  double* v = lds;
  double* blk = v + G.Bp;
  double* red = blk + 64 * 65;
  const int nch = (int)cl_ceil_div(N, CL_THCHUNK);
  for (int q = tid(); q < G.Br; q += nthr()) {
    double x;
    if (q < ns) {
      x = ws.rcur[e0 * ns + q];
      if (u < N) x += ws.svec[(e0 + u) * (int64_t)G.Lp + ns + q];
    } else {
      const int c = q - ns;
      x = rhs[xt + c];
      for (int ch = 0; ch < nch; ++ch) x += ws.thv[((int64_t)inst * ws.nchunk + ch) * np + c];
    }
    v[q] = x;
  }
  const double* B = ws.bbuf + (int64_t)inst * G.Bp * G.Bp;
  blocked_fwd(B, G.Bp, G.Br, G.Br, v, blk);
  blocked_bwd(B, G.Bp, G.Br, G.Br, v, blk, red);
  for (int q = tid(); q < G.Br; q += nthr()) {
    if (q < ns) ws.xsep[e0 * ns + q] = v[q];
    else dx[xt + q - ns] = v[q];
  }
}

// Cyclic-reduction backward of level l: x_s = L_s^-T (y_s - X^T [x_left; x_right; x_theta]).
template <typename T>
__global__ void __launch_bounds__(256) k_big_crb(Shape S, Tab tb, Ws ws, int level, const double* __restrict__ dx) {
  extern __shared__ double lds[];
  const int it = tb.cr_ptr[level - 1] + blockIdx.x;
  if (it >= tb.cr_ptr[level]) return;
  const int inst = tb.cr_inst[it], s = tb.cr_j[it];
  if (block_flag(&ws.flag[inst])) return;
  const BigGeom G = big_geom(S);
  const int ns = S.ns, np = S.np, N = tb.inst_N[inst], half = 1 << (level - 1);
  const int64_t e0 = tb.inst_e0[inst], es = e0 + s;
  const int64_t xt = tb.inst_x[inst] + (int64_t)N * S.b;
  double* v = lds;
  double* blk = v + G.Lp;
  double* red = blk + 64 * 65;
  for (int q = tid(); q < G.Lr; q += nthr()) {
    double x;
    if (q < ns) x = ws.svec[es * (int64_t)G.Lp + q];
    else if (q < 2 * ns) x = ws.xsep[(es - half) * ns + q - ns];
    else if (q < 3 * ns) x = (s + half < N) ? ws.xsep[(es + half) * ns + q - 2 * ns] : 0.0;
    else x = dx[xt + q - 3 * ns];
    v[q] = x;
  }
  blocked_bwd((const T*)ws.sbuf + es * (int64_t)G.Lp * G.Lp, G.Lp, ns, G.Lr, v, blk, red);
  for (int q = tid(); q < ns; q += nthr()) ws.xsep[es * ns + q] = v[q];
}

// Element backward: x_I = L_II^-T (y_I - X^T [x_S; x_theta; x_P]); dx of the element's nodes.
template <typename T>
__global__ void __launch_bounds__(256) k_big_bwd(Shape S, Tab tb, Ws ws, double* __restrict__ dx) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const BigGeom G = big_geom(S);
  const int ns = S.ns, np = S.np, b = S.b, mI = S.mI, R = S.R, N = tb.inst_N[inst];
  const int64_t xo = tb.inst_x[inst], xt = xo + (int64_t)N * b;
  double* v = lds;
  double* blk = v + G.Rp;
  double* red = blk + 64 * 65;
  for (int q = tid(); q < R; q += nthr()) {
    double x;
    if (q < mI) x = ws.evec[e * (int64_t)G.Rp + q];
    else if (q < b) x = ws.xsep[e * ns + q - mI];
    else if (q < b + np) x = dx[xt + q - b];
    else x = i > 0 ? ws.xsep[(e - 1) * ns + q - b - np] : 0.0;
    v[q] = x;
  }
  blocked_bwd((const T*)ws.ebuf + e * (int64_t)G.Rp * G.Rp, G.Rp, mI, R, v, blk, red);
  double* out = dx + xo + (int64_t)i * b;
  for (int q = tid(); q < b; q += nthr()) out[q] = v[q];
}

// ---------------------------------------------------------------- launches
static inline int ok_or() { return hipGetLastError() == hipSuccess ? 0 : -3; }

static PArgs pargs(void* base, int64_t stride, int ld, int n, int m, int count, int mode, int level) {
  PArgs a;
  a.base = base;
  a.stride = stride;
  a.ld = ld;
  a.n = n;
  a.m = m;
  a.count = count;
  a.mode = mode;
  a.level = level;
  a.zero = 0;
  a.skip0 = a.skip1 = 0;
  return a;
}

template <typename T>
static void trail(const Tab& tb, const Ws& ws, const PArgs& a, hipStream_t st) {
  if (a.count == 0 || a.n <= a.m) return;
  int nblk = 0, s, cb;
  while (trail_block(a, nblk, s, cb)) ++nblk;
  if (nblk == 0) return;
  const int groups = (int)cl_ceil_div(nblk, 4);
  const unsigned grid = (unsigned)(cl_ceil_div(a.count, 8) * 8 * groups);
  hipLaunchKernelGGL(k_pchol_trail<T>, dim3(grid), dim3(256), 0, st, tb, ws, a, groups);
}

// Partial Cholesky of the first a.m columns of every matrix of the batch: two launches per panel
// of 32 columns (the diagonal block, then the strips below it).  Panels go in pairs: from column
// kLookMin on, the first panel's strip pass also applies every earlier column to the second
// panel, so the second panel's launches need only the first panel's columns and the strip rows
// are read once per pair.  (Before that, the extra read and write of the second panel's columns
// costs more than the earlier columns it saves reading.)
constexpr int kLookMin = 128;
template <typename T>
static void pchol(const Tab& tb, const Ws& ws, const PArgs& a, hipStream_t st) {
  if (a.count == 0) return;
  for (int p = 0, k0 = 0; k0 < a.m; ++p, k0 += 32) {
    const int wd = std::min(32, a.m - k0);
    // columns not yet applied to this panel: all earlier ones, or only the previous panel's
    // when that panel's pass looked ahead
    const bool prev_look = (p & 1) && k0 - 32 >= kLookMin;
    const int kb = prev_look ? k0 - 32 : 0;
    const bool look = !(p & 1) && k0 >= kLookMin && k0 + 32 < a.m;
    hipLaunchKernelGGL(k_pchol_diag<T>, dim3(a.count), dim3(64), 0, st, tb, ws, a, k0, kb);
    if (a.n <= k0 + wd) continue;   // no rows below the block
    const int s0 = wd < 32 ? 0 : 1;
    const int nstrip = (int)cl_ceil_div(a.n - k0, 32) - s0;
    const int groups = (int)cl_ceil_div(nstrip, 4);
    const unsigned grid = (unsigned)(cl_ceil_div(a.count, 8) * 8 * groups);
    if (look)
      hipLaunchKernelGGL((k_pchol_strip<T, 1>), dim3(grid), dim3(256), 0, st, tb, ws, a, k0, kb, s0, groups);
    else
      hipLaunchKernelGGL((k_pchol_strip<T, 0>), dim3(grid), dim3(256), 0, st, tb, ws, a, k0, kb, s0, groups);
  }
}

template <typename T>
static int big_factor_t(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, phase_cb cb,
                        void* ctx, hipStream_t st) {
  const BigGeom G = big_geom(S);
  const int E = (int)tb.n_elem;
  const int64_t esz = (int64_t)G.Rp * G.Rp, ssz = (int64_t)G.Lp * G.Lp;
  if (cb) cb(ctx, COLLOC_PH_ASSEMBLY, 1, st);
  hipLaunchKernelGGL(k_big_asm<T>, dim3(E), dim3(1024), big_asm_lds(S), st, S, tb, ws);
  if (cb) cb(ctx, COLLOC_PH_ASSEMBLY, 0, st);
  if (cb) cb(ctx, COLLOC_PH_LEVEL0, 1, st);
  PArgs ea = pargs(ws.ebuf, esz, G.Rp, S.R, S.mI, E, 0, 0);
  pchol<T>(tb, ws, ea, st);
  if (cb) cb(ctx, COLLOC_PH_LEVEL0, 0, st);
  if (cb) cb(ctx, COLLOC_PH_SCHUR, 1, st);
  // the theta-theta block is formed by k_big_theta; its blocks here are skipped
  ea.skip0 = S.b;
  ea.skip1 = S.b + S.np;
  trail<T>(tb, ws, ea, st);
  if (cb) cb(ctx, COLLOC_PH_SCHUR, 0, st);
  if (cb) cb(ctx, 2, 1, st);
  hipLaunchKernelGGL(k_sep_init<T>, dim3(E, gather_bands(S)), dim3(1024), 0, st, S, tb, ws);
  for (int l = 1; l <= tb.L; ++l) {
    if (l > 1 && hp.st[l - 1] > 0)
      hipLaunchKernelGGL(k_sep_step<T>, dim3(hp.st[l - 1], gather_bands(S)), dim3(1024), 0, st, S, tb, ws, l - 1);
    const int cnt = hp.lvl[l];
    if (cnt == 0) continue;
    PArgs ca = pargs(ws.sbuf, ssz, G.Lp, G.Lr, S.ns, cnt, 1, l);
    pchol<T>(tb, ws, ca, st);
    ca.zero = 1;
    ca.skip0 = 3 * S.ns;
    ca.skip1 = G.Lr;
    trail<T>(tb, ws, ca, st);
  }
  if (cb) cb(ctx, 2, 0, st);
  if (cb) cb(ctx, 3, 1, st);
  const int nt = (int)cl_ceil_div(S.np, 64);
  if (nt > 0)
    hipLaunchKernelGGL(k_big_theta<T>, dim3((unsigned)(cl_ceil_div(ws.nchunk, 8) * 8 * (nt * (nt + 1) / 2)), tb.n_inst),
                       dim3(256), 0, st, S, tb, ws, nt * (nt + 1) / 2);
  hipLaunchKernelGGL(k_border_build<T>, dim3(tb.n_inst), dim3(256), 0, st, S, tb, ws);
  if (S.np > 0)
    hipLaunchKernelGGL(k_border_theta, dim3((unsigned)cl_ceil_div(S.np * S.np, 256), tb.n_inst), dim3(256), 0, st,
                       S, tb, ws);
  PArgs ba = pargs(ws.bbuf, (int64_t)G.Bp * G.Bp, G.Bp, G.Br, G.Br, tb.n_inst, 2, 0);
  pchol<double>(tb, ws, ba, st);
  if (cb) cb(ctx, 3, 0, st);
  return ok_or();
}

int launch_factor_big(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, int prec,
                      phase_cb cb, void* ctx, hipStream_t st) {
  return prec ? big_factor_t<float>(S, tb, hp, ws, cb, ctx, st) : big_factor_t<double>(S, tb, hp, ws, cb, ctx, st);
}

size_t big_solve_lds(const Shape& S) {
  const BigGeom G = big_geom(S);
  const int nv = std::max(G.Rp, std::max(G.Lp, G.Bp));
  return sizeof(double) * ((size_t)nv + 64 * 65 + 256);
}

template <typename T>
static int big_solve_t(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, const double* rhs,
                       const double* rthp, double* dx, phase_cb cb, void* ctx, hipStream_t st) {
  const size_t lds = big_solve_lds(S);
  const int E = (int)tb.n_elem;
  if (cb) cb(ctx, 4, 1, st);
  hipLaunchKernelGGL(k_big_fwd<T>, dim3(E), dim3(256), lds, st, S, tb, ws, rhs);
  hipLaunchKernelGGL(k_big_seprhs, dim3(E), dim3(64), 0, st, S, tb, ws, rhs);
  for (int l = 1; l <= tb.L; ++l) {
    if (l > 1 && hp.st[l - 1] > 0)
      hipLaunchKernelGGL(k_big_crs, dim3(hp.st[l - 1]), dim3(64), 0, st, S, tb, ws, l - 1);
    if (hp.lvl[l] > 0) hipLaunchKernelGGL(k_big_crf<T>, dim3(hp.lvl[l]), dim3(256), lds, st, S, tb, ws, l);
  }
  hipLaunchKernelGGL(k_big_thv, dim3(ws.nchunk, tb.n_inst), dim3(64), 0, st, S, tb, ws, rthp);
  hipLaunchKernelGGL(k_big_border_solve, dim3(tb.n_inst), dim3(256), lds, st, S, tb, ws, rhs, dx);
  for (int l = tb.L; l >= 1; --l)
    if (hp.lvl[l] > 0) hipLaunchKernelGGL(k_big_crb<T>, dim3(hp.lvl[l]), dim3(256), lds, st, S, tb, ws, l, dx);
  hipLaunchKernelGGL(k_big_bwd<T>, dim3(E), dim3(256), lds, st, S, tb, ws, dx);
  if (cb) cb(ctx, 4, 0, st);
  return ok_or();
}

int launch_solve_big(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, const double* rhs,
                     const double* rthp, double* dx, phase_cb cb, void* ctx, hipStream_t st) {
  return ws.prec ? big_solve_t<float>(S, tb, hp, ws, rhs, rthp, dx, cb, ctx, st)
                 : big_solve_t<double>(S, tb, hp, ws, rhs, rthp, dx, cb, ctx, st);
}

// Dynamic LDS above 64 KiB must be declared per kernel.
int big_prepare_attrs(const Shape& S) {
  const size_t a = big_asm_lds(S), s = big_solve_lds(S);
  int rc = 0;
  auto set = [&](const void* fn, size_t bytes) {
    if (bytes > 64 * 1024 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
      rc = -1;
  };
  set((const void*)k_big_asm<double>, a);
  set((const void*)k_big_asm<float>, a);
  for (const void* fn : {(const void*)k_big_fwd<double>, (const void*)k_big_fwd<float>, (const void*)k_big_crf<double>,
                         (const void*)k_big_crf<float>, (const void*)k_big_crb<double>, (const void*)k_big_crb<float>,
                         (const void*)k_big_bwd<double>, (const void*)k_big_bwd<float>, (const void*)k_big_border_solve})
    set(fn, s);
  return rc;
}

}  // namespace cl
