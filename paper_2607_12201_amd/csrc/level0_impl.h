// Level-0 element kernel template (included by the k_level0*.hip translation units).
#pragma once
// Level 0 of the factorization: every finite element, in parallel, assembles its block of the
// condensed KKT matrix and eliminates its interior collocation nodes 0..K-1.
//
// The element's symmetric matrix over [I (nodes 0..K-1) | S (node K) | theta | P (previous
// element's node K)] lives in registers: a TS x TS thread grid owns the lower-triangle
// entries block-cyclically (thread (ty, tx) owns rows ty + TS*I and columns tx + TS*J), so the
// assembly accumulates every entry in a register and the right-looking elimination of the mI
// interior columns only exchanges one column per step through LDS.  After the mI steps the
// remaining entries are the Schur complement on (S, theta, P): the separator-chain blocks and
// the element's parameter-border contribution.  Panel (L_I and the eliminated rows) is stored
// column-major with ld = R for the solve.
#include "kernels.h"
#include "elem.h"
#include "regchol.h"

namespace cl {

// Per-instance tables and the element's measurements staged in LDS (relative list offsets).
struct LTab {
  int *react, *param, *sp_ptr, *sp_r, *rq_ptr, *rq_r, *rq_t, *pc_ptr, *pc_r, *msp, *jdiv;
  double *sp_nu, *mw;
  int nmeas;
};

// Stage the element's inputs in LDS: Ds of its rows (d0), the reaction partials (jv, hv), the
// instance tables, its measurements, the collocation weights (La, row j = a[j][.]) and the
// row -> node map.  One flat pass per nthr entries: every thread loads entry t of each array
// (index 0 past an array's end, a valid fallback address for an empty array), and only then
// stores, to a dummy slot past the end, so a pass costs one memory latency.
__device__ inline void stage_element(const Shape& S, const Tab& tb, const Ws& ws, int inst,
                                     int64_t e, int i, LTab& L, double* d0, double* jv, double* hv,
                                     double* La, double* ddum, int* idum) {
  const int ns = S.ns, np = S.np, nr = S.nr, K = S.K, b = S.b, jl = K * nr;
  constexpr int NA = (CL_KMAX + 1) * (CL_KMAX + 1);
  const int* spp = tb.sp_ptr + inst * (ns + 1);
  const int* rqp = tb.rq_ptr + inst * (ns + 1);
  const int* pcp = tb.pc_ptr + inst * (np + 1);
  const int sp0 = spp[0], rq0 = rqp[0], pc0 = pcp[0];
  const int nsp = spp[ns] - sp0, nrq = rqp[ns] - rq0, npc = pcp[np] - pc0;
  const int m0 = tb.elem_mptr[e], nm = tb.elem_mptr[e + 1] - m0, nmw = nm * (K + 1);
  L.nmeas = nm;
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  const int* ifb = tb.elem_inst + e;       // valid fallbacks for empty lists
  const double* dfb = tb.elem_h + e;
  const int* spr = nsp > 0 ? tb.sp_r + sp0 : ifb;
  const double* spn = nsp > 0 ? tb.sp_nu + sp0 : dfb;
  const int* rqr = nrq > 0 ? tb.rq_r + rq0 : ifb;
  const int* rqt = nrq > 0 ? tb.rq_t + rq0 : ifb;
  const int* pcr = npc > 0 ? tb.pc_r + pc0 : ifb;
  const int* msp = nm > 0 ? tb.meas_sp + m0 : ifb;
  const double* mw = nm > 0 ? tb.meas_w + (int64_t)m0 * (K + 1) : dfb;
  const double* Ds = ws.Ds + gi;
  const double* jac = ws.jac + e * 3 * jl;
  const double* hes = ws.hess + e * 4 * jl;
  const int* rea = tb.react + inst * nr * 2;
  const int* par = tb.param + inst * nr;
  int nmax = b;
  for (int n : {4 * jl, 2 * nr, ns + 1, np + 1, nsp, nrq, npc, nmw, S.R, NA}) nmax = n > nmax ? n : nmax;
  for (int t0 = 0; t0 < nmax; t0 += nthr()) {
    const int t = t0 + tid();
    auto ix = [t](int n) { return t < n ? t : 0; };
    const double xd = Ds[ix(b)], xj = jac[ix(3 * jl)], xh = hes[ix(4 * jl)], xn = spn[ix(nsp)],
                 xw = mw[ix(nmw)];
    const int xre = rea[ix(2 * nr)], xpa = par[ix(nr)], xsp = spp[ix(ns + 1)], xrq = rqp[ix(ns + 1)],
              xpc = pcp[ix(np + 1)], xsr = spr[ix(nsp)], xqr = rqr[ix(nrq)], xqt = rqt[ix(nrq)],
              xpr = pcr[ix(npc)], xms = msp[ix(nm)];
    const int ta = ix(NA);
    const double xa = S.a[ta / (CL_KMAX + 1)][ta % (CL_KMAX + 1)];
    *(t < b ? d0 + t : ddum) = xd;
    *(t < 3 * jl ? jv + t : ddum) = xj;
    *(t < 4 * jl ? hv + t : ddum) = xh;
    *(t < nsp ? L.sp_nu + t : ddum) = xn;
    *(t < nmw ? L.mw + t : ddum) = xw;
    *(t < NA ? La + t : ddum) = xa;
    *(t < 2 * nr ? L.react + t : idum) = xre;
    *(t < nr ? L.param + t : idum) = xpa;
    *(t <= ns ? L.sp_ptr + t : idum) = xsp - sp0;
    *(t <= ns ? L.rq_ptr + t : idum) = xrq - rq0;
    *(t <= np ? L.pc_ptr + t : idum) = xpc - pc0;
    *(t < nsp ? L.sp_r + t : idum) = xsr;
    *(t < nrq ? L.rq_r + t : idum) = xqr;
    *(t < nrq ? L.rq_t + t : idum) = xqt;
    *(t < npc ? L.pc_r + t : idum) = xpr;
    *(t < nm ? L.msp + t : idum) = xms;
    *(t < S.R ? L.jdiv + t : idum) = t / ns;
  }
}

// node-0 rows (initial condition / continuity), measurement Hessian, dw on z; P couplings.
__device__ inline double base_entry(const Shape& S, const LTab& L, int i, double dw,
                                    const double* d0, int r, int q) {
  const int ns = S.ns, b = S.b, K = S.K, bp = S.b + S.np;
  if (r >= bp) {  // P row: previous separator, coupled by the continuity rows (eq. 2c)
    const int s = r - bp;
    if (i == 0) return 0.0;
    if (q < bp) return (q == s) ? -d0[s] : 0.0;
    return (q == r) ? d0[s] : 0.0;
  }
  if (r >= b) return 0.0;   // theta rows: parameter bounds and dw are added once per instance
  const int j1 = L.jdiv[r], s1 = r - j1 * ns, j2 = L.jdiv[q], s2 = q - j2 * ns;
  double v = (r == q) ? dw : 0.0;
  if (s1 != s2) return v;
  if (j1 == 0 && j2 == 0) v += d0[s1];
  for (int m = 0; m < L.nmeas; ++m)
    if (L.msp[m] == s1) {
      const double* w = L.mw + m * (K + 1);
      v += w[j1] * w[j2];
    }
  return v;
}

// Per-point tables of the collocation rows of point k (eq. 2b / 3).  The rows are
// a_jk e_(j,s) - h (F_k)_(s,.) on node k and -h (Fth_k)_(s,.) on theta, weighted by d_(k,s);
// with the products Q1 = h^2 F^T D F + Wzz, Q2 = h^2 F^T D Fth + Wzt and
// Q3 = h^2 Fth^T D Fth + diag(Wtt), each entry of their contribution needs a few lookups.
struct NodeTab {
  double *d, *F, *Fth, *Wzz, *Wzt, *Wtt, *Q1, *Q2, *Q3;
  // per list entry of the point: species-reaction entries (slot columns u1, u2 and parameter
  // column with their values nu * d rate / d .) and reactant-slot entries (partner column and
  // parameter column with the second-derivative values)
  double *sv1, *sv2, *svp, *qv, *qvp;
  int *su1, *su2, *sup, *qu, *qup;
};

__device__ inline double node_entry(const Shape& S, const LTab& L, const double* La, int k, double h,
                                    const NodeTab& nt, int r, int q) {
  const int ns = S.ns, np = S.np, b = S.b;
  if (r < b) {
    const int j1 = L.jdiv[r], s1 = r - j1 * ns, j2 = L.jdiv[q], s2 = q - j2 * ns;
    const double a1 = La[j1 * (CL_KMAX + 1) + k], a2 = La[j2 * (CL_KMAX + 1) + k];
    double v = 0.0;
    if (s1 == s2) v += nt.d[s1] * a1 * a2;
    if (j2 == k) v -= a1 * (h * nt.d[s1] * nt.F[s1 * ns + s2]);
    if (j1 == k) v -= a2 * (h * nt.d[s2] * nt.F[s2 * ns + s1]);
    if (j1 == k && j2 == k) v += nt.Q1[s1 * ns + s2];
    return v;
  }
  if (q < b) {
    const int c = r - b, j1 = L.jdiv[q], s1 = q - j1 * ns;
    double v = -La[j1 * (CL_KMAX + 1) + k] * (h * nt.d[s1] * nt.Fth[s1 * np + c]);
    if (j1 == k) v += nt.Q2[s1 * np + c];
    return v;
  }
  return nt.Q3[(r - b) * np + (q - b)];
}

// Lower-triangle index t -> (row, column) of an n x n triangle stored row by row.
__device__ inline void tri_rc(int t, int& r, int& c) {
  r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  c = t - r * (r + 1) / 2;
}

// Build the tables of point k from the element's staged derivative values (jv, hv) and Ds.
// First every list entry gets its contributions (one thread each); then each F / Wzz entry
// sums the entries of its row with selects (no branches, independent loads), in list order;
// then the products Q, one entry per thread.
__device__ inline void node_tables(const Shape& S, const LTab& L, int k, double h,
                                   const double* jv, const double* hv, const double* Ds_e,
                                   const NodeTab& nt) {
  const int ns = S.ns, np = S.np, nr = S.nr, nw = ns + np;
  const int nsp = L.sp_ptr[ns], nrq = L.rq_ptr[ns];
  for (int s = tid(); s < ns; s += nthr()) nt.d[s] = Ds_e[k * ns + s];
  for (int c = tid(); c < np; c += nthr()) {
    double acc = 0.0;
    for (int o = L.pc_ptr[c]; o < L.pc_ptr[c + 1]; ++o) acc += hv[((k - 1) * nr + L.pc_r[o]) * 4 + 3];
    nt.Wtt[c] = acc;
  }
  for (int o = tid(); o < nsp; o += nthr()) {
    const int r = L.sp_r[o];
    const double nu = L.sp_nu[o];
    const double* jr = jv + ((k - 1) * nr + r) * 3;
    nt.su1[o] = L.react[2 * r];
    nt.su2[o] = L.react[2 * r + 1];
    nt.sup[o] = L.param[r];
    nt.sv1[o] = nu * jr[0];
    nt.sv2[o] = nu * jr[1];
    nt.svp[o] = nu * jr[2];
  }
  for (int o = tid(); o < nrq; o += nthr()) {
    const int r = L.rq_r[o], sl = L.rq_t[o];
    const double* H = hv + ((k - 1) * nr + r) * 4;
    nt.qu[o] = L.react[2 * r + (1 - sl)];
    nt.qup[o] = L.param[r];
    nt.qv[o] = H[0];
    nt.qvp[o] = H[1 + sl];
  }
  __syncthreads();
  // F | Fth: row s = sum over the reactions of species s of nu_sr times the slot / theta partials
  for (int t = tid(); t < ns * nw; t += nthr()) {
    const int s = t / nw, u = t - s * nw;
    const bool isz = u < ns;
    const int uc = u - ns;
    double v = 0.0;
#pragma unroll 2
    for (int o = L.sp_ptr[s]; o < L.sp_ptr[s + 1]; ++o) {
      const int u1 = nt.su1[o], u2 = nt.su2[o], up = nt.sup[o];
      const double v1 = nt.sv1[o], v2 = nt.sv2[o], vp = nt.svp[o];
      v += pick(isz && u1 == u, v1, 0.0);
      v += pick(isz && u2 == u, v2, 0.0);
      v += pick(!isz && up == uc, vp, 0.0);
    }
    if (isz) nt.F[s * ns + u] = v;
    else nt.Fth[s * np + uc] = v;
  }
  // Wzz | Wzt: row q = the weighted second derivatives of the reactions with q in a slot
  for (int t = tid(); t < ns * nw; t += nthr()) {
    const int q = t / nw, u = t - q * nw;
    const bool isz = u < ns;
    const int uc = u - ns;
    double v = 0.0;
#pragma unroll 2
    for (int o = L.rq_ptr[q]; o < L.rq_ptr[q + 1]; ++o) {
      const int qu = nt.qu[o], qp = nt.qup[o];
      const double qv = nt.qv[o], qvp = nt.qvp[o];
      v += pick(isz && qu == u, qv, 0.0);
      v += pick(!isz && qp == uc, qvp, 0.0);
    }
    if (isz) nt.Wzz[q * ns + u] = v;
    else nt.Wzt[q * np + uc] = v;
  }
  __syncthreads();
  // Q entries: lower triangle of the (ns + np) x (ns + np) product, four partial sums each
  const double h2 = h * h;
  const int ntri = nw * (nw + 1) / 2;
  for (int t = tid(); t < ntri; t += nthr()) {
    int u1, u2;
    tri_rc(t, u1, u2);
    const double* c1 = u1 < ns ? nt.F + u1 : nt.Fth + (u1 - ns);
    const double* c2 = u2 < ns ? nt.F + u2 : nt.Fth + (u2 - ns);
    const int ld1 = u1 < ns ? ns : np, ld2 = u2 < ns ? ns : np;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int s = 0;
    for (; s + 4 <= ns; s += 4) {
      a0 += nt.d[s] * c1[s * ld1] * c2[s * ld2];
      a1 += nt.d[s + 1] * c1[(s + 1) * ld1] * c2[(s + 1) * ld2];
      a2 += nt.d[s + 2] * c1[(s + 2) * ld1] * c2[(s + 2) * ld2];
      a3 += nt.d[s + 3] * c1[(s + 3) * ld1] * c2[(s + 3) * ld2];
    }
    for (; s < ns; ++s) a0 += nt.d[s] * c1[s * ld1] * c2[s * ld2];
    const double acc = h2 * ((a0 + a1) + (a2 + a3));
    if (u1 < ns) {                       // u2 <= u1 < ns
      nt.Q1[u1 * ns + u2] = acc + nt.Wzz[u1 * ns + u2];
    } else if (u2 < ns) {                // theta row, species column
      nt.Q2[u2 * np + (u1 - ns)] = acc + nt.Wzt[u2 * np + (u1 - ns)];
    } else {
      const int c1i = u1 - ns, c2i = u2 - ns;
      nt.Q3[c1i * np + c2i] = acc + (c1i == c2i ? nt.Wtt[c1i] : 0.0);
    }
  }
}

// Stored value of entry (r, q) of the assembled matrix (kkt_assemble's block storage).
template <typename T>
__device__ inline double stored_entry(const Shape& S, const Ws& ws, int64_t e, int r, int q) {
  const int ns = S.ns, np = S.np, b = S.b, mI = S.mI, R = S.R, bp = S.b + S.np;
  if (q < mI) return (double)((const T*)ws.panel)[e * (int64_t)R * mI + (int64_t)q * R + r];
  if (r < b) return (double)((const T*)ws.dss)[e * ns * ns + (r - mI) * ns + (q - mI)];
  if (r < bp) {
    if (q < b) return (double)((const T*)ws.bs)[e * ns * np + (q - mI) * np + (r - b)];
    return ws.ath[e * np * np + (r - b) * np + (q - b)];
  }
  return (r == q) ? ws.dcont[e * ns + (r - bp)] : 0.0;
}

// Panel columns and the Schur complement on (S, theta, P) from the register entries.
template <typename T, int TS, int NB>
__device__ inline void store_regs(const Shape& S, const Ws& ws, int64_t e, int i, const T* acc,
                                  int ty, int tx) {
  const int ns = S.ns, np = S.np, b = S.b, mI = S.mI, R = S.R, bp = S.b + S.np;
  T* Qg = (T*)ws.panel + e * (int64_t)R * mI;
  T* dss = (T*)ws.dss + e * ns * ns;
  T* bsv = (T*)ws.bs + e * ns * np;
  T* tprev = (T*)ws.tprev + e * ns * ns;
  T* e1 = (T*)ws.e1 + e * ns * ns;
  T* gprev = (T*)ws.gprev + e * ns * np;
  double* ath = ws.ath + e * np * np;
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J <= I; ++J) {
      const int r = I * TS + ty, q = J * TS + tx;
      if (!(r < R && q <= r)) continue;
      const T v = acc[I * (I + 1) / 2 + J];
      if (q < mI) {
        Qg[(int64_t)q * R + r] = v;
      } else if (r < b) {
        dss[(r - mI) * ns + (q - mI)] = v;
      } else if (r < bp) {
        if (q < b) bsv[(q - mI) * np + (r - b)] = v;
        else if (sizeof(T) == 8) ath[(r - b) * np + (q - b)] = (double)v;
      } else if (i > 0) {
        const int pr = r - bp;
        if (q < b) e1[(q - mI) * ns + pr] = v;
        else if (q < bp) gprev[pr * np + (q - b)] = v;
        else tprev[pr * ns + (q - bp)] = v;
      }
    }
}

// The 20 x 20 grid (seven waves) is held to four waves per SIMD (at most 128 registers) so two
// elements share a compute unit.
template <typename T, int TS, int NB>
__global__ void __launch_bounds__(TS* TS) __attribute__((amdgpu_waves_per_eu(TS == 20 ? 4 : 1))) k_level0r(Shape S, Tab tb, Ws ws, int fused) {
  extern __shared__ double lds[];
  constexpr int NBLK = NB * (NB + 1) / 2;
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, b = S.b, R = S.R, bp = S.b + S.np;
  const int ty = threadIdx.x / TS, tx = threadIdx.x % TS;
  const int jl = S.K * S.nr;
  double* pbuf = lds;                 // elimination buffers
  double* misc = pbuf + elim_lds_doubles(R);   // 8
  double* d0 = misc + 8;              // b (Ds of the element's rows)
  double* La = d0 + b;                // (KMAX + 1)^2 collocation weights, then a dummy slot
  double* jv = La + (CL_KMAX + 1) * (CL_KMAX + 1) + 1;   // 3 K nr
  double* hv = jv + 3 * jl;           // 4 K nr
  NodeTab nt;
  nt.d = hv + 4 * jl;
  nt.F = nt.d + ns;
  nt.Fth = nt.F + ns * ns;
  nt.Wzz = nt.Fth + ns * np;
  nt.Wzt = nt.Wzz + ns * ns;
  nt.Wtt = nt.Wzt + ns * np;
  nt.Q1 = nt.Wtt + np;
  nt.Q2 = nt.Q1 + ns * ns;
  nt.Q3 = nt.Q2 + ns * np;
  nt.sv1 = nt.Q3 + np * np;
  nt.sv2 = nt.sv1 + S.lsp;
  nt.svp = nt.sv2 + S.lsp;
  nt.qv = nt.svp + S.lsp;
  nt.qvp = nt.qv + S.lrq;
  LTab L;
  L.sp_nu = nt.qvp + S.lrq;
  L.mw = L.sp_nu + S.lsp;
  int* ib = (int*)(L.mw + S.mmax * (S.K + 1));
  L.react = ib;
  L.param = L.react + 2 * S.nr;
  L.sp_ptr = L.param + S.nr;
  L.rq_ptr = L.sp_ptr + ns + 1;
  L.pc_ptr = L.rq_ptr + ns + 1;
  L.sp_r = L.pc_ptr + np + 1;
  L.rq_r = L.sp_r + S.lsp;
  L.rq_t = L.rq_r + S.lrq;
  L.pc_r = L.rq_t + S.lrq;
  L.msp = L.pc_r + S.lpc;
  L.jdiv = L.msp + S.mmax;
  int* idum = L.jdiv + R;
  nt.su1 = idum + 1;
  nt.su2 = nt.su1 + S.lsp;
  nt.sup = nt.su2 + S.lsp;
  nt.qu = nt.sup + S.lsp;
  nt.qup = nt.qu + S.lrq;
  double av[NBLK];

  if (fused) {
    const double h = tb.elem_h[e], dw = ws.dw[inst];
    stage_element(S, tb, ws, inst, e, i, L, d0, jv, hv, La, La + (CL_KMAX + 1) * (CL_KMAX + 1), idum);
    __syncthreads();
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const int r = I * TS + ty, q = J * TS + tx;
        av[I * (I + 1) / 2 + J] = (r < R && q <= r) ? base_entry(S, L, i, dw, d0, r, q) : 0.0;
      }
    for (int k = 1; k <= S.K; ++k) {
      __syncthreads();
      node_tables(S, L, k, h, jv, hv, d0, nt);
      __syncthreads();
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) {
          const int r = I * TS + ty, q = J * TS + tx;
          if (r < bp && q <= r) av[I * (I + 1) / 2 + J] += node_entry(S, L, La, k, h, nt, r, q);
        }
    }
    if (sizeof(T) == 4) {  // FP32 factors: keep the assembled theta-theta block in FP64
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) {
          const int r = I * TS + ty, q = J * TS + tx;
          if (r >= b && r < bp && q >= b && q <= r)
            ws.ath[e * np * np + (r - b) * np + (q - b)] = av[I * (I + 1) / 2 + J];
        }
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const int r = I * TS + ty, q = J * TS + tx;
        av[I * (I + 1) / 2 + J] = (r < R && q <= r) ? stored_entry<T>(S, ws, e, r, q) : 0.0;
      }
  }
  const int mI = S.mI;

  bool ok;
  if constexpr (sizeof(T) == 8) {
    ok = eliminate_regs<double, TS, NB>(av, mI, R, ty, tx, pbuf, misc);
    if (ok) store_regs<double, TS, NB>(S, ws, e, i, av, ty, tx);
  } else {
    float af[NBLK];
#pragma unroll
    for (int B = 0; B < NBLK; ++B) af[B] = (float)av[B];
    ok = eliminate_regs<float, TS, NB>(af, mI, R, ty, tx, pbuf, misc);
    if (ok) store_regs<float, TS, NB>(S, ws, e, i, af, ty, tx);
  }
  if (!ok) {
    if (tid() == 0) atomicOr(&ws.flag[inst], 1);
    return;
  }
  if (sizeof(T) == 4) {
    // FP64 parameter Schur part from the FP32 eliminated rows: ath -= X_B^T X_B
    const T* Qg = (const T*)ws.panel + e * (int64_t)R * mI;
    double* ath = ws.ath + e * np * np;
    __syncthreads();
    for (int t = tid(); t < np * np; t += nthr()) {
      int r = t / np, q = t % np;
      if (q > r) continue;
      double sum = 0.0;
      for (int k = 0; k < mI; ++k) sum += (double)Qg[(int64_t)k * R + b + r] * (double)Qg[(int64_t)k * R + b + q];
      ath[t] -= sum;
    }
  }
}

}  // namespace cl
