// a3-a5: condensed KKT assembly, pivoting-free factorization and solve.
//
// Matrix K = W + Sx + dw I + J^T Ds J of one instance is block tridiagonal over the finite
// elements (element i couples to element i-1 only through the continuity rows, eq. 2c) with a
// dense border in theta.  Elimination order (a nested-dissection ordering of the time chain):
//   level 0   every element eliminates its interior collocation nodes 0..K-1 (all elements in
//             parallel, one workgroup each, dense LDS panel), leaving a chain of separators
//             S_i = node K of element i (n_s each) with a theta border;
//   levels 1..L  cyclic reduction of that chain: at level l the separators j = q 2^(l-1), q odd,
//             are eliminated in parallel; each update of a survivor is gathered by the
//             workgroup that eliminates it later, in a fixed order (no atomics);
//   border    separator 0 last, then the dense parameter Schur complement (FP64) and its
//             Cholesky factor.
// The solve walks the same levels forward and backward.  Block data is FP64 or FP32 (T); the
// parameter Schur complement, its right-hand side and all vectors are FP64.
#include <stdio.h>
#include <stdlib.h>

#include "kernels.h"
#include "elem.h"

namespace cl {

template <typename T>
struct L0Lds {
  double *ath, *dcont, *d, *d0, *F, *Fth, *Wzz, *Wzt, *Wtt, *misc;
  T *Q, *dss, *bs;
};

template <typename T>
__device__ inline L0Lds<T> l0_carve(const Shape& S, void* base) {
  L0Lds<T> L;
  double* p = (double*)base;
  L.ath = p; p += S.np * S.np;
  L.dcont = p; p += S.ns;
  L.d = p; p += S.ns;
  L.d0 = p; p += S.ns;
  L.F = p; p += S.ns * S.ns;
  L.Fth = p; p += S.ns * S.np;
  L.Wzz = p; p += S.ns * S.ns;
  L.Wzt = p; p += S.ns * S.np;
  L.Wtt = p; p += S.np;
  L.misc = p; p += 8;
  T* q = (T*)p;
  L.Q = q; q += S.R * S.mI;
  L.dss = q; q += S.ns * S.ns;
  L.bs = q;
  return L;
}

size_t level0_lds_bytes(const Shape& S, int prec) {
  size_t nd = (size_t)S.np * S.np + 3 * S.ns + 2 * S.ns * S.ns + 2 * S.ns * S.np + S.np + 8;
  size_t nt = (size_t)S.R * S.mI + S.ns * S.ns + S.ns * S.np;
  return nd * 8 + nt * (prec ? 4 : 8);
}

__device__ inline void tri_index(int t, int& r1, int& r2) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  r1 = r;
  r2 = t - r * (r + 1) / 2;
}

// Value of K's lower-triangle entry (r1 >= r2, element-local natural indices: z (j,s) at
// j*ns+s, theta c at b+c) contributed by the collocation rows of point k.
__device__ inline double node_contrib(const Shape& S, int k, double h, const double* d,
                                      const double* F, const double* Fth, const double* Wzz,
                                      const double* Wzt, const double* Wtt, int r1, int r2) {
  const int ns = S.ns, np = S.np, b = S.b;
  double v = 0.0;
  if (r1 < b) {
    int j1 = r1 / ns, s1 = r1 - j1 * ns, j2 = r2 / ns, s2 = r2 - j2 * ns;
    double a1 = S.a[j1][k], a2 = S.a[j2][k];
    if (s1 == s2) v += d[s1] * a1 * a2;
    if (j2 == k) v -= h * d[s1] * a1 * F[s1 * ns + s2];
    if (j1 == k) v -= h * d[s2] * a2 * F[s2 * ns + s1];
    if (j1 == k && j2 == k) {
      double acc = 0.0;
      for (int s = 0; s < ns; ++s) acc += d[s] * F[s * ns + s1] * F[s * ns + s2];
      v += h * h * acc + Wzz[s1 * ns + s2];
    }
  } else if (r2 < b) {
    int c = r1 - b, j1 = r2 / ns, s1 = r2 - j1 * ns;
    v -= h * d[s1] * S.a[j1][k] * Fth[s1 * np + c];
    if (j1 == k) {
      double acc = 0.0;
      for (int s = 0; s < ns; ++s) acc += d[s] * F[s * ns + s1] * Fth[s * np + c];
      v += h * h * acc + Wzt[s1 * np + c];
    }
  } else {
    int c1 = r1 - b, c2 = r2 - b;
    double acc = 0.0;
    for (int s = 0; s < ns; ++s) acc += d[s] * Fth[s * np + c1] * Fth[s * np + c2];
    v = h * h * acc + (c1 == c2 ? Wtt[c1] : 0.0);
  }
  return v;
}

// Node-0 rows (initial condition / continuity), the measurement Hessian and dw on z.
__device__ inline double base_contrib(const Shape& S, const Tab& tb, int64_t e, double dw,
                                      const double* d0, int r1, int r2) {
  const int ns = S.ns, b = S.b, K = S.K;
  if (r1 >= b) return 0.0;
  int j1 = r1 / ns, s1 = r1 - j1 * ns, j2 = r2 / ns, s2 = r2 - j2 * ns;
  double v = 0.0;
  if (r1 == r2) v += dw;
  if (s1 != s2) return v;
  if (j1 == 0 && j2 == 0) v += d0[s1];
  int m0 = tb.elem_mptr[e], m1 = tb.elem_mptr[e + 1];
  for (int m = m0; m < m1; ++m)
    if (tb.meas_sp[m] == s1) {
      const double* w = tb.meas_w + (int64_t)m * (K + 1);
      v += w[j1] * w[j2];
    }
  return v;
}

// Storage of a lower-triangle entry in the level-0 LDS blocks.
template <typename T>
__device__ inline void entry_store(const Shape& S, L0Lds<T>& L, int r1, int r2, double v,
                                   bool add) {
  const int ns = S.ns, np = S.np, b = S.b, mI = S.mI, R = S.R;
  if (r2 < mI) {
    T* p = &L.Q[r2 * R + r1];   // panel rows [I | S | theta | P]: natural order up to b + np
    *p = add ? (T)((double)*p + v) : (T)v;
  } else if (r2 < b) {
    T* p = (r1 < b) ? &L.dss[(r1 - mI) * ns + (r2 - mI)] : &L.bs[(r2 - mI) * np + (r1 - b)];
    *p = add ? (T)((double)*p + v) : (T)v;
  } else {
    double* p = &L.ath[(r1 - b) * np + (r2 - b)];
    *p = add ? *p + v : v;
  }
}

// Assemble element e's blocks of K into LDS.  Inputs: derivative values of the element
// (jac_e, hess_e), Ds of its rows (Ds_e), dw.  Accumulation is in FP64 per entry; with T =
// float each addition rounds into the FP32 panel.
template <typename T>
__device__ void assemble_element(const Shape& S, const Tab& tb, int64_t e, int inst, int i,
                                 double h, const double* jac_e, const double* hess_e,
                                 const double* Ds_e, double dw, L0Lds<T>& L) {
  const int ns = S.ns, np = S.np, nr = S.nr, b = S.b, mI = S.mI, R = S.R;
  const int nb = b + np, ntri = nb * (nb + 1) / 2;
  for (int t = tid(); t < ns; t += nthr()) {
    L.d0[t] = Ds_e[t];
    L.dcont[t] = i > 0 ? Ds_e[t] : 0.0;
  }
  __syncthreads();
  for (int t = tid(); t < ntri; t += nthr()) {
    int r1, r2;
    tri_index(t, r1, r2);
    entry_store(S, L, r1, r2, base_contrib(S, tb, e, dw, L.d0, r1, r2), false);
  }
  // coupling of node-0 rows to the previous separator (continuity, eq. 2c): P rows last
  for (int t = tid(); t < ns * mI; t += nthr()) {
    int col = t / ns, s = t - col * ns;
    L.Q[col * R + b + np + s] = (T)((i > 0 && col == s) ? -L.d0[s] : 0.0);
  }
  for (int k = 1; k <= S.K; ++k) {
    __syncthreads();
    for (int s = tid(); s < ns; s += nthr()) {
      L.d[s] = Ds_e[k * ns + s];
      for (int q = 0; q < ns; ++q) L.F[s * ns + q] = 0.0;
      for (int c = 0; c < np; ++c) L.Fth[s * np + c] = 0.0;
      int p0 = tb.sp_ptr[inst * (ns + 1) + s], p1 = tb.sp_ptr[inst * (ns + 1) + s + 1];
      for (int q = p0; q < p1; ++q) {
        int r = tb.sp_r[q];
        double nu = tb.sp_nu[q];
        const double* jr = jac_e + ((k - 1) * nr + r) * 3;
        int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
        int c = tb.param[inst * nr + r];
        if (q0 >= 0) L.F[s * ns + q0] += nu * jr[0];
        if (q1 >= 0) L.F[s * ns + q1] += nu * jr[1];
        if (c >= 0) L.Fth[s * np + c] += nu * jr[2];
      }
    }
    for (int q = tid(); q < ns; q += nthr()) {
      for (int s2 = 0; s2 < ns; ++s2) L.Wzz[q * ns + s2] = 0.0;
      for (int c = 0; c < np; ++c) L.Wzt[q * np + c] = 0.0;
      for (int r = 0; r < nr; ++r) {
        int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
        if (q0 != q && q1 != q) continue;
        int c = tb.param[inst * nr + r];
        const double* H = hess_e + ((k - 1) * nr + r) * 4;
        if (q0 == q) {
          if (q1 >= 0) L.Wzz[q * ns + q1] += H[0];
          if (c >= 0) L.Wzt[q * np + c] += H[1];
        }
        if (q1 == q) {
          if (q0 >= 0) L.Wzz[q * ns + q0] += H[0];
          if (c >= 0) L.Wzt[q * np + c] += H[2];
        }
      }
    }
    for (int c = tid(); c < np; c += nthr()) {
      double acc = 0.0;
      for (int r = 0; r < nr; ++r)
        if (tb.param[inst * nr + r] == c) acc += hess_e[((k - 1) * nr + r) * 4 + 3];
      L.Wtt[c] = acc;
    }
    __syncthreads();
    for (int t = tid(); t < ntri; t += nthr()) {
      int r1, r2;
      tri_index(t, r1, r2);
      double v = node_contrib(S, k, h, L.d, L.F, L.Fth, L.Wzz, L.Wzt, L.Wtt, r1, r2);
      entry_store(S, L, r1, r2, v, true);
    }
  }
  __syncthreads();
}

// kkt_assemble: blocks to the workspace (unfactored), derivative copies, Ds, rhs.
template <typename T>
__global__ void __launch_bounds__(256) k_assemble(Shape S, Tab tb, Ws ws, const double* __restrict__ jac,
                                                  const double* __restrict__ hess, const double* __restrict__ sigma_s,
                                                  const double* __restrict__ delta_w, const double* __restrict__ r_x,
                                                  const double* __restrict__ r_s, const double* __restrict__ r_y,
                                                  double* __restrict__ rhs) {
  extern __shared__ double lds_raw[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  const int N = tb.inst_N[inst];
  const double h = tb.elem_h[e];
  const int ns = S.ns, np = S.np, b = S.b, R = S.R, mI = S.mI;
  const double dw = delta_w[inst];
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  const int64_t xi = tb.inst_x[inst] + (int64_t)i * b;
  const int64_t jl = (int64_t)S.K * S.nr;
  // copies used later by the factor and the matrix-free residual
  for (int t = tid(); t < jl * 3; t += nthr()) ws.jac[e * jl * 3 + t] = jac[e * jl * 3 + t];
  for (int t = tid(); t < jl * 4; t += nthr()) ws.hess[e * jl * 4 + t] = hess[e * jl * 4 + t];
  for (int t = tid(); t < b; t += nthr()) ws.Ds[gi + t] = sigma_s[gi + t] + dw;
  if (i == 0 && tid() == 0) ws.dw[inst] = dw;
  L0Lds<T> L = l0_carve<T>(S, lds_raw);
  __syncthreads();
  assemble_element<T>(S, tb, e, inst, i, h, ws.jac + e * jl * 3, ws.hess + e * jl * 4,
                      ws.Ds + gi, dw, L);
  // store blocks
  T* Qg = (T*)ws.panel + e * (int64_t)R * mI;
  for (int t = tid(); t < R * mI; t += nthr()) Qg[t] = L.Q[t];
  T* dssg = (T*)ws.dss + e * ns * ns;
  T* bsg = (T*)ws.bs + e * ns * np;
  for (int t = tid(); t < ns * ns; t += nthr()) dssg[t] = L.dss[t];
  for (int t = tid(); t < ns * np; t += nthr()) bsg[t] = L.bs[t];
  for (int t = tid(); t < np * np; t += nthr()) ws.ath[e * np * np + t] = L.ath[t];
  for (int t = tid(); t < ns; t += nthr()) ws.dcont[e * ns + t] = L.dcont[t];
  __syncthreads();
  // rhs = -r_x - J^T w, w = Ds r_y + r_s (element rows; next element's node-0 rows).
  // The blocks are stored, so the LDS is reused from its start (size checked at launch).
  double* w = lds_raw;
  double* wn = w + b;
  double* phi = wn + ns;
  double* outz = phi + S.K * S.nr;
  double* outth = outz + b;
  for (int t = tid(); t < b; t += nthr()) w[t] = (sigma_s[gi + t] + dw) * r_y[gi + t] + r_s[gi + t];
  if (i + 1 < N)
    for (int t = tid(); t < ns; t += nthr()) wn[t] = (sigma_s[gi + b + t] + dw) * r_y[gi + b + t] + r_s[gi + b + t];
  __syncthreads();
  reaction_weights(S, tb, inst, w, phi);
  __syncthreads();
  jtu_rows(S, tb, inst, h, ws.jac + e * jl * 3, w, (i + 1 < N) ? wn : nullptr, phi, outz, outth);
  __syncthreads();
  for (int t = tid(); t < b; t += nthr()) rhs[xi + t] = -r_x[xi + t] - outz[t];
  for (int t = tid(); t < np; t += nthr()) ws.rthp[e * np + t] = -outth[t];
}

// kkt_assemble on the tiled path: the derivative values, Ds and dw are stored for the factor
// (which assembles the element matrices from them) and the matrix-free product; the z part of the
// right-hand side per element, its theta partials to rthp.
__global__ void __launch_bounds__(256) k_assemble_rhs(Shape S, Tab tb, Ws ws, const double* __restrict__ jac,
                                                      const double* __restrict__ hess, const double* __restrict__ sigma_s,
                                                      const double* __restrict__ delta_w, const double* __restrict__ r_x,
                                                      const double* __restrict__ r_s, const double* __restrict__ r_y,
                                                      double* __restrict__ rhs) {
  extern __shared__ double lds_raw[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  const int N = tb.inst_N[inst];
  const double h = tb.elem_h[e];
  const int ns = S.ns, np = S.np, b = S.b;
  const double dw = delta_w[inst];
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  const int64_t xi = tb.inst_x[inst] + (int64_t)i * b;
  const int64_t jl = (int64_t)S.K * S.nr;
  for (int t = tid(); t < jl * 3; t += nthr()) ws.jac[e * jl * 3 + t] = jac[e * jl * 3 + t];
  for (int t = tid(); t < jl * 4; t += nthr()) ws.hess[e * jl * 4 + t] = hess[e * jl * 4 + t];
  for (int t = tid(); t < b; t += nthr()) ws.Ds[gi + t] = sigma_s[gi + t] + dw;
  if (i == 0 && tid() == 0) ws.dw[inst] = dw;
  double* w = lds_raw;
  double* wn = w + b;
  double* phi = wn + ns;
  double* outz = phi + S.K * S.nr;
  double* outth = outz + b;
  for (int t = tid(); t < b; t += nthr()) w[t] = (sigma_s[gi + t] + dw) * r_y[gi + t] + r_s[gi + t];
  if (i + 1 < N)
    for (int t = tid(); t < ns; t += nthr()) wn[t] = (sigma_s[gi + b + t] + dw) * r_y[gi + b + t] + r_s[gi + b + t];
  __syncthreads();
  reaction_weights(S, tb, inst, w, phi);
  __syncthreads();
  jtu_rows(S, tb, inst, h, jac + e * jl * 3, w, (i + 1 < N) ? wn : nullptr, phi, outz, outth);
  __syncthreads();
  for (int t = tid(); t < b; t += nthr()) rhs[xi + t] = -r_x[xi + t] - outz[t];
  for (int t = tid(); t < np; t += nthr()) ws.rthp[e * np + t] = -outth[t];
}

// rhs theta part: -r_x(theta) + sum_e partials (fixed order); sigma_x + dw kept for the border.
__global__ void k_rhs_theta(Shape S, Tab tb, Ws ws, const double* __restrict__ r_x,
                            const double* __restrict__ sigma_x, const double* __restrict__ delta_w,
                            double* __restrict__ rhs) {
  const int inst = blockIdx.x;
  const int N = tb.inst_N[inst];
  const int64_t e0 = tb.inst_e0[inst];
  const int64_t xt = tb.inst_x[inst] + (int64_t)N * S.b;
  (void)e0;
  for (int c = tid(); c < S.np; c += nthr()) {
    const double acc = thpart_sum(ws, ws.thv, inst, N, S.np, c);
    rhs[xt + c] = -r_x[xt + c] + acc;
    ws.sxdw[inst * S.np + c] = sigma_x[inst * S.np + c] + delta_w[inst];
  }
}

// ---------------------------------------------------------------- wave triangular solves
// One full wave (the calling workgroup's threads 0..63) solves with a lower-triangular L of
// order n <= 256 in place on the LDS vector x.  Column oriented: lane t keeps rows t, t+64,
// t+128, t+192 in registers; the pivot value x_c is broadcast from its owner lane by a
// shuffle, so no workgroup barrier is needed inside the solve.  Lrc(r, c) returns L(r, c)
// for r >= c.  The caller synchronises before (x written by other threads) and after.
template <class F>
__device__ inline void wave_trsv_l(const F& Lrc, int n, double* x) {
  const int lane = threadIdx.x & 63;
  double v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = (lane + 64 * k < n) ? x[lane + 64 * k] : 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int cend = min(n, 64 * k + 64);
    for (int c = 64 * k; c < cend; ++c) {
      const double xc = __shfl(v[k], c - 64 * k) / Lrc(c, c);
      if (lane == c - 64 * k) v[k] = xc;
#pragma unroll
      for (int k2 = k; k2 < 4; ++k2) {
        const int r = lane + 64 * k2;
        if (r > c && r < n) v[k2] -= Lrc(r, c) * xc;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (lane + 64 * k < n) x[lane + 64 * k] = v[k];
}

// Same with L^T: x <- L^{-T} x, columns taken from the last one down.
template <class F>
__device__ inline void wave_trsv_lt(const F& Lrc, int n, double* x) {
  const int lane = threadIdx.x & 63;
  double v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = (lane + 64 * k < n) ? x[lane + 64 * k] : 0.0;
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    for (int c = min(n, 64 * k + 64) - 1; c >= 64 * k; --c) {
      const double xc = __shfl(v[k], c - 64 * k) / Lrc(c, c);
      if (lane == c - 64 * k) v[k] = xc;
#pragma unroll
      for (int k2 = 0; k2 <= k; ++k2) {
        const int r = lane + 64 * k2;
        if (r < c) v[k2] -= Lrc(c, r) * xc;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (lane + 64 * k < n) x[lane + 64 * k] = v[k];
}

// Row-major dense block in LDS (L(r, c) at M[r * n + c]).
struct RowMajor {
  const double* M;
  int n;
  __device__ double operator()(int r, int c) const { return M[r * n + c]; }
};
// Packed lower triangle, column-major: column c holds rows c..n-1.
struct PackedCol {
  const double* M;
  int n;
  __device__ int off(int c) const { return c * n - (c * (c - 1)) / 2; }
  __device__ double operator()(int r, int c) const { return M[off(c) + (r - c)]; }
};


// ---------------------------------------------------------------- cyclic reduction levels
// The chain eliminations themselves run in the k_chain kernels (register partial Cholesky of
// each separator's local matrix, chain_impl.h); here only the parameter-block reductions.

// Theta-theta reduction, stage 1: partial sums over chunks of CL_THCHUNK elements of the
// element Schur parts and separator parts; grid (chunk, entry tile, instance).
__global__ void k_thred(Shape S, Tab tb, Ws ws) {
  const int inst = blockIdx.z, chunk = blockIdx.x;
  const int t = blockIdx.y * blockDim.x + threadIdx.x;
  const int np = S.np, N = tb.inst_N[inst];
  if (t >= np * np || ws.flag[inst]) return;
  const int i0 = chunk * CL_THCHUNK, i1 = min(N, i0 + CL_THCHUNK);
  if (i0 >= N) return;
  const int r = t / np, q = t % np;
  if (q > r) return;
  const int64_t e0 = tb.inst_e0[inst];
  // all loads of the chunk issued together (the last valid element stands in past the end;
  // separator 0 has no chain part), then added in element order
  double xa[CL_THCHUNK], xc[CL_THCHUNK];
#pragma unroll
  for (int u = 0; u < CL_THCHUNK; ++u) {
    const int64_t ei = e0 + min(i0 + u, i1 - 1);
    xa[u] = ws.ath[ei * np * np + t];
    xc[u] = ws.thcr[ei * np * np + t];
  }
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < CL_THCHUNK; ++u) {
    const int i = i0 + u;
    acc += pick(i < i1, xa[u], 0.0);
    acc += pick(i < i1 && i > 0, xc[u], 0.0);
  }
  ws.thred[((int64_t)inst * ws.nchunk + chunk) * np * np + t] = acc;
}

// Theta-theta reduction, stage 2: the reduced parameter block S = sum of the chunk partials
// + Sx + dw on the diagonal (lower triangle); grid (entry tile, instance).
__global__ void k_thred2(Shape S, Tab tb, Ws ws) {
  const int inst = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = S.np;
  if (t >= np * np || ws.flag[inst]) return;
  const int r = t / np, q = t % np;
  if (q > r) return;
  const int nch = (int)cl_ceil_div(tb.inst_N[inst], CL_THCHUNK);
  const double* src = ws.thred + (int64_t)inst * ws.nchunk * np * np + t;
  double acc = 0.0;
#pragma unroll 8
  for (int c = 0; c < nch; ++c) acc += src[(int64_t)c * np * np];
  ws.S[(int64_t)inst * np * np + t] = acc + (r == q ? ws.sxdw[inst * np + r] : 0.0);
}

__global__ void k_clear_flags(Ws ws, int n) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) ws.flag[t] = 0;
}
__global__ void k_copy_flags(Ws ws, int* info, int n) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) info[t] = ws.flag[t];
}

// ---------------------------------------------------------------- solve

// Stage the lower triangle of the leading mI x mI block of a column-major panel (ld R) into
// LDS as a packed lower triangle; eight independent loads in flight per thread.
template <typename T>
__device__ inline void stage_tri(double* dst, const T* Q, int R, int mI) {
  const int nn = mI * mI;
  for (int t0 = 0; t0 < nn; t0 += 8 * nthr()) {
    double tmp[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * nthr() + tid();
      const int c = t / mI, r = t - c * mI;
      tmp[u] = (t < nn && r >= c) ? (double)Q[c * R + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + u * nthr() + tid();
      const int c = t / mI, r = t - c * mI;
      if (t < nn && r >= c) dst[c * mI - (c * (c - 1)) / 2 + (r - c)] = tmp[u];
    }
  }
}

// sum_k a[k * sa] * b[k] over k < n with four independent partial sums.
template <typename T>
__device__ inline double dot4(const T* a, int sa, const double* b, int n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    s0 += (double)a[k * sa] * b[k];
    s1 += (double)a[(k + 1) * sa] * b[k + 1];
    s2 += (double)a[(k + 2) * sa] * b[k + 2];
    s3 += (double)a[(k + 3) * sa] * b[k + 3];
  }
  for (; k < n; ++k) s0 += (double)a[k * sa] * b[k];
  return (s0 + s1) + (s2 + s3);
}
// Level-0 forward, one wave per element: the element's interior factor L_I is staged in LDS as
// a packed lower triangle, y_I = L_I^{-1} r_I by the wave solve, then the tail contributions
// X^T y_I for the rows [S | theta | P].  LDS: packed L_I (mI (mI+1) / 2) + y (mI).
template <typename T>
__global__ void __launch_bounds__(64) k_l0_fwd(Shape S, Tab tb, Ws ws, const double* __restrict__ rhs) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, R = S.R, mI = S.mI;
  const T* Q = (const T*)ws.panel + e * (int64_t)R * mI;
  const PackedCol Lp{lds, mI};
  double* y = lds + mI * (mI + 1) / 2;
  stage_tri(lds, Q, R, mI);
  const double* r = rhs + tb.inst_x[inst] + (int64_t)i * S.b;
  for (int t = tid(); t < mI; t += nthr()) y[t] = r[t];
  __syncthreads();
  wave_trsv_l(Lp, mI, y);
  __syncthreads();
  for (int t = tid(); t < mI; t += nthr()) ws.yI[e * mI + t] = y[t];
  for (int a = tid(); a < S.Rt; a += nthr()) {   // tail rows [S | theta | P]
    const double acc = dot4(Q + mI + a, R, y, mI);
    if (a < ns) ws.cS[e * ns + a] = acc;
    else if (a < ns + np) ws.cB[e * np + (a - ns)] = acc;
    else ws.cP[e * ns + (a - ns - np)] = (i > 0) ? acc : 0.0;
  }
}

// LDS of the separator solve kernels: three ns x ns blocks, the ns x np border rows, four
// ns-vectors, an np-vector and a dummy slot.
size_t sep_solve_lds(const Shape& S) {
  const size_t ns = S.ns, np = S.np;
  return sizeof(double) * (3 * ns * ns + ns * np + 4 * ns + np + 1);
}
constexpr int kSepThreads = 256;    // most threads per item
constexpr int kSepUnroll = 4;       // block entries per thread per staging pass
// Threads per item: enough for one staging pass over the largest block, in whole waves.
static int sep_solve_threads(const Shape& S) {
  const int n2 = S.ns * S.ns, ng = S.ns * S.np;
  const int need = ((n2 > ng ? n2 : ng) + kSepUnroll - 1) / kSepUnroll;
  return need <= 64 ? 64 : (need <= 128 ? 128 : kSepThreads);
}

// One forward step of the separator chain (the first level when `first`): gathers everything
// the item needs in one flat pass per 256 entries (every load issued before the first store,
// index 0 past a block's end, a valid address for absent terms, a dummy LDS slot as the store
// target), then r = rhs_s - U_R(j1)^T y(j1) - U_L(j2)^T y(j2); an eliminated separator solves
// y_s = L_s^{-1} r and forms its border term U_B^T y_s, a survivor keeps r for the next level.
// An item's instance data, read before the skip-flag barrier so the loads overlap.
struct SepInst {
  int N;
  int64_t e0, x;
};
__device__ inline SepInst sep_inst(const Tab& tb, int inst) {
  return SepInst{tb.inst_N[inst], tb.inst_e0[inst], tb.inst_x[inst]};
}

template <typename T>
__device__ inline void sep_forward(const Shape& S, const Tab& tb, const Ws& ws, const double* rhs,
                                   int inst, const SepInst& si, int s, int level, bool first) {
  extern __shared__ double lds[];
  const int ns = S.ns, np = S.np, N = si.N;
  const int n2 = ns * ns, ng = ns * np;
  const int64_t e0 = si.e0, es = e0 + s;
  const int half = first ? 1 : 1 << (level - 1);
  const bool h1 = !first && s > 0, h2 = !first && s + half < N;
  const bool elim = first || ((s >> level) & 1) != 0;
  const bool init = first || level == 1, has_next = s + 1 < N;
  const int64_t e1 = h1 ? es - half : es, e2 = h2 ? es + half : es;
  double* Lm = lds;
  double* U1 = Lm + n2;
  double* U2 = U1 + n2;
  double* UB = U2 + n2;
  double* y1 = UB + ng;
  double* y2 = y1 + ns;
  double* r = y2 + ns;
  double* dum = r + 2 * ns + np;
  const T* lsrc = (const T*)ws.lsep + es * n2;
  const T* u1src = (const T*)ws.ur + e1 * n2;
  const T* u2src = (const T*)ws.ul + e2 * n2;
  const T* ubsrc = (const T*)ws.ub + es * ng;
  const double* rh = rhs + si.x + (int64_t)s * S.b + S.mI;
  const double* cs = ws.cS + es * ns;
  const double* cp = ws.cP + (has_next ? es + 1 : es) * ns;
  const double* rc = ws.rcur + es * ns;
  const int nmax = n2 > ng ? n2 : ng;
  for (int t0 = 0; t0 < nmax; t0 += kSepUnroll * nthr()) {
    double xl[kSepUnroll], xu1[kSepUnroll], xu2[kSepUnroll], xb[kSepUnroll];
#pragma unroll
    for (int u = 0; u < kSepUnroll; ++u) {
      const int t = t0 + u * nthr() + tid();
      const int i2 = t < n2 ? t : 0, ig = t < ng ? t : 0;
      xl[u] = (double)lsrc[i2];
      xu1[u] = (double)u1src[i2];
      xu2[u] = (double)u2src[i2];
      xb[u] = (double)ubsrc[ig];
    }
    const int t = t0 + tid(), iv = t < ns ? t : 0;
    const double xy1 = ws.ysep[e1 * ns + iv], xy2 = ws.ysep[e2 * ns + iv];
    const double xr = rh[iv], xs = cs[iv], xp = cp[iv], xc = rc[iv];
    const double r0 = pick(init, (xr - xs) - pick(has_next, xp, 0.0), xc);
#pragma unroll
    for (int u = 0; u < kSepUnroll; ++u) {
      const int tu = t0 + u * nthr() + tid();
      *(tu < n2 ? Lm + tu : dum) = xl[u];
      *(tu < n2 ? U1 + tu : dum) = xu1[u];
      *(tu < n2 ? U2 + tu : dum) = xu2[u];
      *(tu < ng ? UB + tu : dum) = xb[u];
    }
    *(t < ns ? y1 + t : dum) = xy1;
    *(t < ns ? y2 + t : dum) = xy2;
    *(t < ns ? r + t : dum) = r0;
  }
  __syncthreads();
  for (int a = tid(); a < ns; a += nthr()) {
    double v = r[a];
    if (h1) v -= dot4(U1 + a, ns, y1, ns);
    if (h2) v -= dot4(U2 + a, ns, y2, ns);
    r[a] = v;
  }
  __syncthreads();
  if (!elim) {
    for (int a = tid(); a < ns; a += nthr()) ws.rcur[es * ns + a] = r[a];
    return;
  }
  if (tid() < 64) wave_trsv_l(RowMajor{Lm, ns}, ns, r);
  __syncthreads();
  for (int t = tid(); t < ns; t += nthr()) ws.ysep[es * ns + t] = r[t];
  for (int c = tid(); c < np; c += nthr()) ws.cBsep[es * np + c] = dot4(UB + c, np, r, ns);
}

template <typename T>
__global__ void __launch_bounds__(kSepThreads) k_crf_first(Shape S, Tab tb, Ws ws, const double* __restrict__ rhs) {
  const int it = tb.cr_ptr[0] + blockIdx.x;
  if (it >= tb.cr_ptr[1]) return;
  const int inst = tb.cr_inst[it], j = tb.cr_j[it];
  const SepInst si = sep_inst(tb, inst);
  if (block_flag(&ws.flag[inst])) return;
  sep_forward<T>(S, tb, ws, rhs, inst, si, j, 1, true);
}

template <typename T>
__global__ void __launch_bounds__(kSepThreads) k_crf_step(Shape S, Tab tb, Ws ws, const double* __restrict__ rhs, int level) {
  const int it = tb.st_ptr[level - 1] + blockIdx.x;
  if (it >= tb.st_ptr[level]) return;
  const int inst = tb.st_inst[it], s = tb.st_s[it];
  const SepInst si = sep_inst(tb, inst);
  if (block_flag(&ws.flag[inst])) return;
  sep_forward<T>(S, tb, ws, rhs, inst, si, s, level, false);
}

// Theta partial sums of an instance over chunks of CL_THCHUNK elements, in element order:
// out[inst][chunk][c] = sum_i (a[e_i][c] + [i > 0] b[e_i][c] - d[e_i][c]) with b and d optional
// (null).  All loads of a chunk are issued together (the chunk's last element stands in past
// the instance's end).  Grid (chunk, instance).
__global__ void k_thpart(Shape S, Tab tb, Ws ws, const double* __restrict__ a,
                         const double* __restrict__ b, const double* __restrict__ d,
                         double* __restrict__ out) {
  const int inst = blockIdx.y, chunk = blockIdx.x;
  const int N = tb.inst_N[inst], np = S.np;
  const int i0 = chunk * CL_THCHUNK;
  if (i0 >= N) return;
  const int i1 = min(N, i0 + CL_THCHUNK);
  const int64_t e0 = tb.inst_e0[inst];
  const double* bb = b ? b : a;
  const double* dd = d ? d : a;
  double* o = out + ((int64_t)inst * ws.nchunk + chunk) * np;
  for (int c = tid(); c < np; c += nthr()) {
    double xa[CL_THCHUNK], xb[CL_THCHUNK], xd[CL_THCHUNK];
#pragma unroll
    for (int u = 0; u < CL_THCHUNK; ++u) {
      const int64_t ei = (e0 + min(i0 + u, i1 - 1)) * np + c;
      xa[u] = a[ei];
      xb[u] = bb[ei];
      xd[u] = dd[ei];
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < CL_THCHUNK; ++u) {
      const int i = i0 + u;
      acc += pick(i < i1, xa[u], 0.0);
      acc += pick(b != nullptr && i < i1 && i > 0, xb[u], 0.0);
      acc -= pick(d != nullptr && i < i1, xd[u], 0.0);
    }
    o[c] = acc;
  }
}

// LDS of the border solve: L_0 and the upper coupling block (ns x ns each), the parameter
// factor (np x np), the border rows (ns x np), y, r (ns), rt (np), the group sums (1024) and a
// dummy slot.
size_t border_solve_lds(const Shape& S) {
  const size_t ns = S.ns, np = S.np;
  return sizeof(double) * (2 * ns * ns + np * np + ns * np + 2 * ns + np + 1024 + 1);
}

// Border solve: separator 0, theta, back to separator 0.  Everything the instance needs is
// gathered in one staging phase (two entries of each block per thread and pass); the theta
// right-hand side sums the chunk partials of k_thpart (thread (c, g) takes chunks g, g + G, ...;
// the G group sums are added in group order).
template <typename T>
__global__ void __launch_bounds__(1024) k_border_solve(Shape S, Tab tb, Ws ws, const double* __restrict__ rhs,
                                                      double* __restrict__ dx) {
  extern __shared__ double lds[];
  const int inst = blockIdx.x;
  const SepInst si = sep_inst(tb, inst);
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, N = si.N;
  const int n2 = ns * ns, ng = ns * np, nq = np * np;
  const int64_t e0 = si.e0, xoff = si.x;
  const int L = tb.L;
  const int jl = L >= 1 ? (1 << (L - 1)) : N;
  const bool hj = jl < N, init = L <= 1, has_next = N > 1;
  double* Lm = lds;
  double* U = Lm + n2;
  double* Sm = U + n2;
  double* UB = Sm + nq;
  double* y = UB + ng;
  double* r = y + ns;
  double* rt = r + ns;
  double* red = rt + np;
  double* dum = red + 1024;
  const T* lsrc = (const T*)ws.lsep + e0 * n2;
  const T* usrc = (const T*)ws.ul + (hj ? e0 + jl : e0) * n2;
  const double* ssrc = ws.S + (int64_t)inst * nq;
  const T* ubsrc = (const T*)ws.ub + e0 * ng;
  const double* ys = ws.ysep + (hj ? e0 + jl : e0) * ns;
  const double* rh = rhs + xoff + S.mI;
  const double* cs = ws.cS + e0 * ns;
  const double* cp = ws.cP + (has_next ? e0 + 1 : e0) * ns;
  const double* rc = ws.rcur + e0 * ns;
  const double* rth = rhs + xoff + (int64_t)N * S.b;
  int nmax = n2 > ng ? n2 : ng;
  nmax = nq > nmax ? nq : nmax;
  for (int t0 = 0; t0 < nmax; t0 += 2 * nthr()) {
    double xl[2], xu[2], xs[2], xb[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = t0 + u * nthr() + tid();
      const int i2 = t < n2 ? t : 0, ig = t < ng ? t : 0, iq = t < nq ? t : 0;
      xl[u] = (double)lsrc[i2];
      xu[u] = (double)usrc[i2];
      xs[u] = ssrc[iq];
      xb[u] = (double)ubsrc[ig];
    }
    const int t = t0 + tid(), iv = t < ns ? t : 0, ip = t < np ? t : 0;
    const double xy = ys[iv], xr = rh[iv], xc = cs[iv], xp = cp[iv], xcur = rc[iv], xt = rth[ip];
    const double r0 = pick(init, (xr - xc) - pick(has_next, xp, 0.0), xcur);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int tu = t0 + u * nthr() + tid();
      *(tu < n2 ? Lm + tu : dum) = xl[u];
      *(tu < n2 ? U + tu : dum) = xu[u];
      *(tu < nq ? Sm + tu : dum) = xs[u];
      *(tu < ng ? UB + tu : dum) = xb[u];
    }
    *(t < ns ? y + t : dum) = xy;
    *(t < ns ? r + t : dum) = r0;
    *(t < np ? rt + t : dum) = xt;
  }
  // theta right-hand side: chunk partials, G = threads / np groups
  const int G = nthr() / np;
  const int c0 = tid() % np, g0 = tid() / np;
  const int nch = (int)cl_ceil_div(N, CL_THCHUNK);
  double acc = 0.0;
  if (g0 < G) {
    const double* p = ws.thv + (int64_t)inst * ws.nchunk * np + c0;
#pragma unroll 4
    for (int ch = g0; ch < nch; ch += G) acc += p[(int64_t)ch * np];
  }
  red[tid()] = acc;
  __syncthreads();
  for (int a = tid(); a < ns; a += nthr()) {
    double v = r[a];
    if (hj) v -= dot4(U + a, ns, y, ns);
    r[a] = v;
  }
  __syncthreads();
  if (tid() < 64) wave_trsv_l(RowMajor{Lm, ns}, ns, r);
  __syncthreads();
  for (int c = tid(); c < np; c += nthr()) {
    double sum = 0.0;
    for (int g = 0; g < G; ++g) sum += red[g * np + c];
    const double u = dot4(UB + c, np, r, ns);
    rt[c] = rt[c] - sum - u;
  }
  __syncthreads();
  if (tid() < 64) {
    wave_trsv_l(RowMajor{Sm, np}, np, rt);
    wave_trsv_lt(RowMajor{Sm, np}, np, rt);
  }
  __syncthreads();
  for (int a = tid(); a < ns; a += nthr()) {
    double v = r[a];
    v -= dot4(UB + a * np, 1, rt, np);
    r[a] = v;
  }
  __syncthreads();
  if (tid() < 64) wave_trsv_lt(RowMajor{Lm, ns}, ns, r);
  __syncthreads();
  for (int c = tid(); c < np; c += nthr()) {
    ws.xth[inst * np + c] = rt[c];
    dx[xoff + (int64_t)N * S.b + c] = rt[c];
  }
  for (int a = tid(); a < ns; a += nthr()) ws.xsep[e0 * ns + a] = r[a];
}

// Backward step of the separator chain: x_j = L_j^{-T} (y_j - U_L x(j - half) - U_R x(j + half)
// - U_B x_theta), with the item's blocks and vectors gathered in one staging phase as in the
// forward step.
template <typename T>
__global__ void __launch_bounds__(kSepThreads) k_cr_bwd(Shape S, Tab tb, Ws ws, int level) {
  extern __shared__ double lds[];
  const int it = tb.cr_ptr[level - 1] + blockIdx.x;
  if (it >= tb.cr_ptr[level]) return;
  const int inst = tb.cr_inst[it], j = tb.cr_j[it];
  const SepInst si = sep_inst(tb, inst);
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, N = si.N;
  const int n2 = ns * ns, ng = ns * np;
  const int64_t e0 = si.e0, ej = e0 + j;
  const int half = 1 << (level - 1);
  const bool hr = j + half < N;
  double* Lm = lds;
  double* UL = Lm + n2;
  double* UR = UL + n2;
  double* UB = UR + n2;
  double* xl = UB + ng;
  double* xr = xl + ns;
  double* r = xr + ns;
  double* xt = r + 2 * ns;
  double* dum = xt + np;
  const T* lsrc = (const T*)ws.lsep + ej * n2;
  const T* ulsrc = (const T*)ws.ul + ej * n2;
  const T* ursrc = (const T*)ws.ur + ej * n2;
  const T* ubsrc = (const T*)ws.ub + ej * ng;
  const double* xls = ws.xsep + (ej - half) * ns;
  const double* xrs = ws.xsep + (hr ? ej + half : ej) * ns;
  const double* ys = ws.ysep + ej * ns;
  const double* xts = ws.xth + inst * np;
  const int nmax = n2 > ng ? n2 : ng;
  for (int t0 = 0; t0 < nmax; t0 += kSepUnroll * nthr()) {
    double xlm[kSepUnroll], xul[kSepUnroll], xur[kSepUnroll], xub[kSepUnroll];
#pragma unroll
    for (int u = 0; u < kSepUnroll; ++u) {
      const int t = t0 + u * nthr() + tid();
      const int i2 = t < n2 ? t : 0, ig = t < ng ? t : 0;
      xlm[u] = (double)lsrc[i2];
      xul[u] = (double)ulsrc[i2];
      xur[u] = (double)ursrc[i2];
      xub[u] = (double)ubsrc[ig];
    }
    const int t = t0 + tid(), iv = t < ns ? t : 0, ip = t < np ? t : 0;
    const double vl = xls[iv], vr = xrs[iv], vy = ys[iv], vt = xts[ip];
#pragma unroll
    for (int u = 0; u < kSepUnroll; ++u) {
      const int tu = t0 + u * nthr() + tid();
      *(tu < n2 ? Lm + tu : dum) = xlm[u];
      *(tu < n2 ? UL + tu : dum) = xul[u];
      *(tu < n2 ? UR + tu : dum) = xur[u];
      *(tu < ng ? UB + tu : dum) = xub[u];
    }
    *(t < ns ? xl + t : dum) = vl;
    *(t < ns ? xr + t : dum) = vr;
    *(t < ns ? r + t : dum) = vy;
    *(t < np ? xt + t : dum) = vt;
  }
  __syncthreads();
  for (int a = tid(); a < ns; a += nthr()) {
    double v = r[a];
    v -= dot4(UL + a * ns, 1, xl, ns);
    if (hr) v -= dot4(UR + a * ns, 1, xr, ns);
    v -= dot4(UB + a * np, 1, xt, np);
    r[a] = v;
  }
  __syncthreads();
  if (tid() < 64) wave_trsv_lt(RowMajor{Lm, ns}, ns, r);
  __syncthreads();
  for (int a = tid(); a < ns; a += nthr()) ws.xsep[ej * ns + a] = r[a];
}

// Level-0 backward, one wave per element: x_I = L_I^{-T} (y_I - X_S x_S(i) - X_P x_S(i-1) -
// X_B x_theta); writes dx.  LDS: packed L_I + t (mI) + xs (ns) + xp (ns) + xt (np)
template <typename T>
__global__ void __launch_bounds__(64) k_l0_bwd(Shape S, Tab tb, Ws ws, double* __restrict__ dx) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, R = S.R, mI = S.mI;
  const T* Q = (const T*)ws.panel + e * (int64_t)R * mI;
  const PackedCol Lp{lds, mI};
  double* tv = lds + mI * (mI + 1) / 2;
  double* xs = tv + mI;
  double* xp = xs + ns;
  double* xt = xp + ns;
  stage_tri(lds, Q, R, mI);
  for (int a = tid(); a < ns; a += nthr()) {
    xs[a] = ws.xsep[e * ns + a];
    xp[a] = i > 0 ? ws.xsep[(e - 1) * ns + a] : 0.0;
  }
  for (int c = tid(); c < np; c += nthr()) xt[c] = ws.xth[inst * np + c];
  __syncthreads();
  for (int k = tid(); k < mI; k += nthr()) {
    const T* col = Q + k * R + mI;
    double v = ws.yI[e * mI + k] - dot4(col, 1, xs, ns) - dot4(col + ns, 1, xt, np);
    if (i > 0) v -= dot4(col + ns + np, 1, xp, ns);
    tv[k] = v;
  }
  __syncthreads();
  wave_trsv_lt(Lp, mI, tv);
  __syncthreads();
  double* out = dx + tb.inst_x[inst] + (int64_t)i * S.b;
  for (int k = tid(); k < mI; k += nthr()) out[k] = tv[k];
  for (int a = tid(); a < ns; a += nthr()) out[mI + a] = xs[a];
}

// ---------------------------------------------------------------- matrix-free K v (FP64)
// u = Ds (J v) for the element's rows.  LDS: v (b) vp (ns) vt (np) out (b)
template <bool AB>
__global__ void k_mv1(Shape S, Tab tb, Ws ws, const double* __restrict__ v, double* __restrict__ u,
                      const int* skip) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (skip && block_flag(&skip[inst])) return;
  const int N = tb.inst_N[inst];
  const int b = S.b, ns = S.ns, np = S.np;
  const double* vb = v + tb.inst_x[inst];
  double* vl = lds;
  double* vp = vl + b;
  double* vt = vp + ns;
  double* o = vt + np;
  // AB: v is the vector of ones (not read)
  for (int t = tid(); t < b; t += nthr()) vl[t] = AB ? 1.0 : vb[(int64_t)i * b + t];
  if (i > 0)
    for (int t = tid(); t < ns; t += nthr()) vp[t] = AB ? 1.0 : vb[(int64_t)(i - 1) * b + S.K * ns + t];
  for (int t = tid(); t < np; t += nthr()) vt[t] = AB ? 1.0 : vb[(int64_t)N * b + t];
  __syncthreads();
  const int64_t jl = (int64_t)S.K * S.nr;
  jv_rows<AB>(S, tb, inst, i, tb.elem_h[e], ws.jac + e * jl * 3, vl, vp, vt, o);
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  __syncthreads();
  for (int t = tid(); t < b; t += nthr()) u[gi + t] = ws.Ds[gi + t] * o[t];
}

// out_z = J^T u + W v + dw v ; theta partials to ws.rthp.  LDS: u (b) un (ns) phi (K nr)
// v (b) vt (np) oz (b) ot (np) wz (b) wt (np)
template <bool AB>
__global__ void k_mv2(Shape S, Tab tb, Ws ws, const double* __restrict__ v,
                      const double* __restrict__ u, double* __restrict__ out, const int* skip) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (skip && block_flag(&skip[inst])) return;
  const int N = tb.inst_N[inst];
  const int b = S.b, ns = S.ns, np = S.np;
  double* ul = lds;
  double* un = ul + b;
  double* phi = un + ns;
  double* vl = phi + S.K * S.nr;
  double* vt = vl + b;
  double* oz = vt + np;
  double* ot = oz + b;
  double* wz = ot + np;
  double* wt = wz + b;
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  const double* vb = v + tb.inst_x[inst];
  for (int t = tid(); t < b; t += nthr()) {
    ul[t] = u[gi + t];
    vl[t] = AB ? 1.0 : vb[(int64_t)i * b + t];
  }
  if (i + 1 < N)
    for (int t = tid(); t < ns; t += nthr()) un[t] = u[gi + b + t];
  for (int t = tid(); t < np; t += nthr()) vt[t] = AB ? 1.0 : vb[(int64_t)N * b + t];
  __syncthreads();
  reaction_weights<AB>(S, tb, inst, ul, phi);
  __syncthreads();
  const int64_t jl = (int64_t)S.K * S.nr;
  const double h = tb.elem_h[e];
  jtu_rows<AB>(S, tb, inst, h, ws.jac + e * jl * 3, ul, (i + 1 < N) ? un : nullptr, phi, oz, ot);
  wv_rows<AB>(S, tb, inst, e, ws.hess + e * jl * 4, vl, vt, wz, wt);
  __syncthreads();
  const double dw = ws.dw[inst];
  double* ob = out + tb.inst_x[inst] + (int64_t)i * b;
  for (int t = tid(); t < b; t += nthr()) ob[t] = oz[t] + wz[t] + dw * vl[t];
  for (int t = tid(); t < np; t += nthr()) ws.rthp[e * np + t] = ot[t] + wt[t];
}

template <bool AB>
__global__ void k_mv3(Shape S, Tab tb, Ws ws, const double* __restrict__ v, double* __restrict__ out,
                      const int* skip) {
  const int inst = blockIdx.x;
  if (skip && block_flag(&skip[inst])) return;
  const int N = tb.inst_N[inst];
  const int64_t e0 = tb.inst_e0[inst];
  const int64_t xt = tb.inst_x[inst] + (int64_t)N * S.b;
  (void)e0;
  for (int c = tid(); c < S.np; c += nthr()) {
    const double acc = thpart_sum(ws, ws.thv, inst, N, S.np, c);
    out[xt + c] = acc + ws.sxdw[inst * S.np + c] * (AB ? 1.0 : v[xt + c]);
  }
}

// ---------------------------------------------------------------- launches
static inline int ok_or() { return hipGetLastError() == hipSuccess ? 0 : -3; }

void launch_thpart(const Shape& S, const Tab& tb, const Ws& ws, const double* a, const double* b,
                   const double* d, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_thpart, dim3(ws.nchunk, tb.n_inst), dim3(64), 0, st, S, tb, ws, a, b, d, out);
}

int launch_assemble(const Shape& S, const Tab& tb, const Ws& ws, const double* jac,
                    const double* hess, const double* sigma_x, const double* sigma_s,
                    const double* delta_w, const double* r_x, const double* r_s,
                    const double* r_y, double* rhs, hipStream_t st) {
  int nt = elem_threads(S);
  size_t lds = level0_lds_bytes(S, ws.prec);
  size_t lds_rhs = sizeof(double) * (2 * S.b + S.ns + S.K * S.nr + S.np);
  if (lds_rhs > lds) lds = lds_rhs;
  if (S.big)
    hipLaunchKernelGGL(k_assemble_rhs, dim3((unsigned)tb.n_elem), dim3(256), lds_rhs, st, S, tb, ws, jac, hess,
                       sigma_s, delta_w, r_x, r_s, r_y, rhs);
  else if (ws.prec)
    hipLaunchKernelGGL(k_assemble<float>, dim3((unsigned)tb.n_elem), dim3(nt), lds, st, S, tb, ws,
                       jac, hess, sigma_s, delta_w, r_x, r_s, r_y, rhs);
  else
    hipLaunchKernelGGL(k_assemble<double>, dim3((unsigned)tb.n_elem), dim3(nt), lds, st, S, tb, ws,
                       jac, hess, sigma_s, delta_w, r_x, r_s, r_y, rhs);
  launch_thpart(S, tb, ws, ws.rthp, nullptr, nullptr, ws.thv, st);
  hipLaunchKernelGGL(k_rhs_theta, dim3(tb.n_inst), dim3(64), 0, st, S, tb, ws, r_x, sigma_x,
                     delta_w, rhs);
  return ok_or();
}

template <typename T>
static int factor_t(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, bool fused,
                    phase_cb cb, void* ctx, hipStream_t st) {
  if (cb) cb(ctx, 1, 1, st);
  if (launch_level0(S, tb, ws, sizeof(T) == 4 ? 1 : 0, fused, hp.ts[0], st)) return -4;
  if (cb) cb(ctx, 1, 0, st);
  const int np = S.np;
  const int prec = sizeof(T) == 4 ? 1 : 0;
  if (cb) cb(ctx, 2, 1, st);
  int rc = 0;
  if (tb.L >= 1) rc |= launch_chain(S, tb, ws, prec, 0, 1, hp.lvl[1], hp.ts[1], st);
  for (int l = 1; l < tb.L; ++l) rc |= launch_chain(S, tb, ws, prec, 1, l, hp.st[l], hp.ts[1], st);
  if (cb) cb(ctx, 2, 0, st);
  if (cb) cb(ctx, 3, 1, st);
  const unsigned tiles = (unsigned)cl_ceil_div(np * np, 256);
  hipLaunchKernelGGL(k_thred, dim3(ws.nchunk, tiles, tb.n_inst), dim3(256), 0, st, S, tb, ws);
  hipLaunchKernelGGL(k_thred2, dim3(tiles, tb.n_inst), dim3(256), 0, st, S, tb, ws);
  rc |= launch_chain(S, tb, ws, prec, 2, 0, tb.n_inst, hp.ts[2], st);
  if (rc) return -4;
  if (cb) cb(ctx, 3, 0, st);
  return ok_or();
}

int launch_factor_nc(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, int prec,
                     bool fused, phase_cb cb, void* ctx, hipStream_t st) {
  // the tiled path always assembles from the stored derivative values (its own kernel)
  if (S.big) return launch_factor_big(S, tb, hp, ws, prec, cb, ctx, st);
  return prec ? factor_t<float>(S, tb, hp, ws, fused, cb, ctx, st)
              : factor_t<double>(S, tb, hp, ws, fused, cb, ctx, st);
}

int launch_factor(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, int prec,
                  bool fused, phase_cb cb, void* ctx, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(256), 0, st, ws, tb.n_inst);
  return launch_factor_nc(S, tb, hp, ws, prec, fused, cb, ctx, st);
}

template <typename T>
static int solve_t(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws,
                   const double* rhs, const double* rthp, double* dx, phase_cb cb, void* ctx,
                   hipStream_t st) {
  if (cb) cb(ctx, 4, 1, st);
  const size_t tri = (size_t)S.mI * (S.mI + 1) / 2;
  hipLaunchKernelGGL(k_l0_fwd<T>, dim3((unsigned)tb.n_elem), dim3(64), sizeof(double) * (tri + S.mI),
                     st, S, tb, ws, rhs);
  const size_t clds = sep_solve_lds(S);
  const int snt = sep_solve_threads(S);
  if (tb.L >= 1 && hp.lvl[1] > 0)
    hipLaunchKernelGGL(k_crf_first<T>, dim3(hp.lvl[1]), dim3(snt), clds, st, S, tb, ws, rhs);
  for (int l = 1; l < tb.L; ++l)
    if (hp.st[l] > 0)
      hipLaunchKernelGGL(k_crf_step<T>, dim3(hp.st[l]), dim3(snt), clds, st, S, tb, ws, rhs, l);
  launch_thpart(S, tb, ws, ws.cB, ws.cBsep, rthp, ws.thv, st);
  hipLaunchKernelGGL(k_border_solve<T>, dim3(tb.n_inst), dim3(1024), border_solve_lds(S), st, S,
                     tb, ws, rhs, dx);
  for (int l = tb.L; l >= 1; --l) {
    int n = hp.lvl[l];
    if (n > 0) hipLaunchKernelGGL(k_cr_bwd<T>, dim3(n), dim3(snt), clds, st, S, tb, ws, l);
  }
  hipLaunchKernelGGL(k_l0_bwd<T>, dim3((unsigned)tb.n_elem), dim3(64),
                     sizeof(double) * (tri + S.mI + 2 * S.ns + S.np), st, S, tb, ws, dx);
  if (cb) cb(ctx, 4, 0, st);
  return ok_or();
}

int launch_solve_p(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws,
                   const double* rhs, const double* rthp, double* dx, phase_cb cb, void* ctx,
                   hipStream_t st) {
  if (S.big) return launch_solve_big(S, tb, hp, ws, rhs, rthp, dx, cb, ctx, st);
  return ws.prec ? solve_t<float>(S, tb, hp, ws, rhs, rthp, dx, cb, ctx, st)
                 : solve_t<double>(S, tb, hp, ws, rhs, rthp, dx, cb, ctx, st);
}

// K v (AB: an upper bound of the row sums of |K|, every coefficient in absolute value applied to
// the vector of ones; v is not read)
template <bool AB>
static int matvec_masked(const Shape& S, const Tab& tb, const Ws& ws, const double* v, double* out,
                         const int* skip, hipStream_t st) {
  int nt = elem_threads(S);
  hipLaunchKernelGGL(k_mv1<AB>, dim3((unsigned)tb.n_elem), dim3(nt),
                     sizeof(double) * (2 * S.b + S.ns + S.np), st, S, tb, ws, v, ws.vtmp2, skip);
  hipLaunchKernelGGL(k_mv2<AB>, dim3((unsigned)tb.n_elem), dim3(nt),
                     sizeof(double) * (4 * S.b + S.ns + S.K * S.nr + 3 * S.np), st, S, tb, ws, v,
                     ws.vtmp2, out, skip);
  launch_thpart(S, tb, ws, ws.rthp, nullptr, nullptr, ws.thv, st);
  hipLaunchKernelGGL(k_mv3<AB>, dim3(tb.n_inst), dim3(64), 0, st, S, tb, ws, v, out, skip);
  return ok_or();
}

int launch_matvec(const Shape& S, const Tab& tb, const Ws& ws, const double* v, double* out,
                  hipStream_t st) {
  return matvec_masked<false>(S, tb, ws, v, out, nullptr, st);
}

// ---------------------------------------------------------------- FP64 iterative refinement
// Per sweep: r = rhs - K dx (matrix-free FP64 product), d = K_factor^{-1} r, dx += d.  An instance
// stops as converged once the dx the residual was taken at has normwise backward error
// ||r|| <= ir_tol (||K|| ||dx|| + ||rhs||) (infinity norms; ||K|| bounded above by the largest row
// sum of |J|^T Ds |J| + |W| + the diagonal terms, formed once per call), and as failed when
// ir_max sweeps are spent or the correction stops contracting (||d|| > ||d_prev|| / 2).
// ws.irflag masks finished instances out of every kernel of the sweep.  Per element, ws.irpart
// holds six partial maxima: |d|, |dx| after, |r|, |rhs|, |dx| before, the row-sum bound.
constexpr int kIrPart = 6;

__global__ void k_ir_init(Ws ws, int n) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    ws.irflag[t] = ws.flag[t];
    ws.ircount[t] = 0;
    ws.irnorm[2 * t + 1] = INFINITY;   // previous correction
  }
}

// Row-sum bound partials: the largest entry of out (= |K| 1) over the element's z rows, the
// theta rows with element 0.
__global__ void k_ir_kpart(Shape S, Tab tb, Ws ws, const double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.irflag[inst])) return;
  const int64_t o = tb.inst_x[inst] + (int64_t)i * S.b;
  double km = 0.0;
  for (int t = tid(); t < S.b; t += nthr()) km = fmax(km, out[o + t]);
  if (i == 0) {
    const int64_t xt = tb.inst_x[inst] + (int64_t)tb.inst_N[inst] * S.b;
    for (int c = tid(); c < S.np; c += nthr()) km = fmax(km, out[xt + c]);
  }
  km = block_max(km, red);
  if (tid() == 0) ws.irpart[e * kIrPart + 5] = km;
}

__global__ void k_ir_knorm(Tab tb, Ws ws) {
  __shared__ double red[256];
  const int inst = blockIdx.x;
  if (block_flag(&ws.irflag[inst])) return;
  const int N = tb.inst_N[inst];
  const int64_t e0 = tb.inst_e0[inst];
  double km = 0.0;
  for (int i = tid(); i < N; i += nthr()) km = fmax(km, ws.irpart[(e0 + i) * kIrPart + 5]);
  km = block_max(km, red);
  if (tid() == 0) ws.irnorm[2 * inst] = km;
}

__global__ void k_ir_resid(Shape S, Tab tb, Ws ws, const double* __restrict__ rhs) {
  __shared__ double red[256];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.irflag[inst])) return;
  const int64_t o = tb.inst_x[inst] + (int64_t)i * S.b;
  double rm = 0.0, bm = 0.0;
  for (int t = tid(); t < S.b; t += nthr()) {
    const double r = rhs[o + t] - ws.vtmp[o + t];
    ws.vtmp[o + t] = r;
    rm = fmax(rm, fabs(r));
    bm = fmax(bm, fabs(rhs[o + t]));
  }
  if (i == 0) {
    const int64_t xt = tb.inst_x[inst] + (int64_t)tb.inst_N[inst] * S.b;
    for (int c = tid(); c < S.np; c += nthr()) {
      const double r = rhs[xt + c] - ws.vtmp[xt + c];
      ws.vtmp[xt + c] = r;
      rm = fmax(rm, fabs(r));
      bm = fmax(bm, fabs(rhs[xt + c]));
    }
  }
  rm = block_max(rm, red);
  bm = block_max(bm, red);
  if (tid() == 0) {
    ws.irpart[e * kIrPart + 2] = rm;
    ws.irpart[e * kIrPart + 3] = bm;
  }
}

__global__ void k_ir_update(Shape S, Tab tb, Ws ws, double* __restrict__ dx) {
  __shared__ double red[256];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.irflag[inst])) return;
  const int64_t o = tb.inst_x[inst] + (int64_t)i * S.b;
  double dm = 0.0, xm = 0.0, xo = 0.0;
  for (int t = tid(); t < S.b; t += nthr()) {
    const double d = ws.vtmp2[o + t], x0 = dx[o + t], x = x0 + d;
    dx[o + t] = x;
    dm = fmax(dm, fabs(d));
    xm = fmax(xm, fabs(x));
    xo = fmax(xo, fabs(x0));
  }
  dm = block_max(dm, red);
  xm = block_max(xm, red);
  xo = block_max(xo, red);
  if (tid() == 0) {
    ws.irpart[e * kIrPart] = dm;
    ws.irpart[e * kIrPart + 1] = xm;
    ws.irpart[e * kIrPart + 4] = xo;
  }
}

__global__ void k_ir_decide(Shape S, Tab tb, Ws ws, double* __restrict__ dx, int ir_max,
                            double ir_tol) {
  __shared__ double red[256];
  const int inst = blockIdx.x;
  if (block_flag(&ws.irflag[inst])) return;
  const int N = tb.inst_N[inst];
  const int64_t e0 = tb.inst_e0[inst];
  const int64_t xt = tb.inst_x[inst] + (int64_t)N * S.b;
  double dm = 0.0, xm = 0.0, xo = 0.0, rm = 0.0, bm = 0.0;
  for (int c = tid(); c < S.np; c += nthr()) {
    const double d = ws.vtmp2[xt + c], x0 = dx[xt + c], x = x0 + d;
    dx[xt + c] = x;
    dm = fmax(dm, fabs(d));
    xm = fmax(xm, fabs(x));
    xo = fmax(xo, fabs(x0));
  }
  for (int i = tid(); i < N; i += nthr()) {
    const double* p = ws.irpart + (e0 + i) * kIrPart;
    dm = fmax(dm, p[0]);
    xm = fmax(xm, p[1]);
    rm = fmax(rm, p[2]);
    bm = fmax(bm, p[3]);
    xo = fmax(xo, p[4]);
  }
  dm = block_max(dm, red);
  xm = block_max(xm, red);
  rm = block_max(rm, red);
  bm = block_max(bm, red);
  xo = block_max(xo, red);
  if (tid() == 0) {
    const int cnt = ws.ircount[inst] + 1;
    const double knorm = ws.irnorm[2 * inst], dprev = ws.irnorm[2 * inst + 1];
    (void)xm;
    if (rm <= ir_tol * (knorm * xo + bm)) {   // the iterate before this sweep was accurate
      ws.ircount[inst] = cnt;
      ws.irflag[inst] = 1;
    } else if (cnt >= ir_max || dm > 0.5 * dprev) {   // out of sweeps, or no longer contracting
      ws.ircount[inst] = -cnt;
      ws.irflag[inst] = 1;
    } else {
      ws.ircount[inst] = cnt;
      ws.irnorm[2 * inst + 1] = dm;
    }
  }
}

__global__ void k_ir_report(Ws ws, int* out, int n) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    out[t] = ws.flag[t] ? 0 : ws.ircount[t];
}

int launch_refine(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, const double* rhs,
                  double* dx, int ir_max, double ir_tol, phase_cb cb, void* ctx, hipStream_t st) {
  const unsigned gi = (unsigned)cl_ceil_div(tb.n_inst, 256);
  hipLaunchKernelGGL(k_ir_init, dim3(gi), dim3(256), 0, st, ws, tb.n_inst);
  Ws wm = ws;
  wm.flag = ws.irflag;
  const int nt = elem_threads(S);
  if (ir_max > 0) {   // the row-sum bound of |K|, once
    if (matvec_masked<true>(S, tb, ws, nullptr, ws.vtmp, ws.irflag, st)) return -3;
    hipLaunchKernelGGL(k_ir_kpart, dim3((unsigned)tb.n_elem), dim3(nt), 0, st, S, tb, ws, ws.vtmp);
    hipLaunchKernelGGL(k_ir_knorm, dim3(tb.n_inst), dim3(256), 0, st, tb, ws);
  }
  for (int s = 0; s < ir_max; ++s) {
    if (matvec_masked<false>(S, tb, ws, dx, ws.vtmp, ws.irflag, st)) return -3;
    hipLaunchKernelGGL(k_ir_resid, dim3((unsigned)tb.n_elem), dim3(nt), 0, st, S, tb, ws, rhs);
    if (launch_solve_p(S, tb, hp, wm, ws.vtmp, nullptr, ws.vtmp2, cb, ctx, st)) return -3;
    hipLaunchKernelGGL(k_ir_update, dim3((unsigned)tb.n_elem), dim3(nt), 0, st, S, tb, ws, dx);
    hipLaunchKernelGGL(k_ir_decide, dim3(tb.n_inst), dim3(256), 0, st, S, tb, ws, dx, ir_max, ir_tol);
  }
  return ok_or();
}

int launch_refine_report(const Tab& tb, const Ws& ws, int* ir_sweeps, hipStream_t st) {
  hipLaunchKernelGGL(k_ir_report, dim3((unsigned)cl_ceil_div(tb.n_inst, 256)), dim3(256), 0, st, ws,
                     ir_sweeps, tb.n_inst);
  return ok_or();
}

int launch_copy_flags(const Tab& tb, const Ws& ws, int* info, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_flags, dim3(1), dim3(256), 0, st, ws, info, tb.n_inst);
  return ok_or();
}

}  // namespace cl

namespace cl {
// Dynamic LDS above the default limit must be declared per kernel: request exactly what this
// shape class needs (static LDS of the kernel comes on top), bounded by the device's limit.
static int set_lds(const void* fn, size_t bytes, const char* name) {
  if (bytes <= 64 * 1024) return 0;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) {
    if (getenv("COLLOC_DEBUG"))
      fprintf(stderr, "colloc: hipFuncSetAttribute(%s, %zu) -> %s\n", name, bytes, hipGetErrorString(e));
    return -1;
  }
  return 0;
}

int kkt_prepare_attrs(const Shape& S) {
  size_t l64 = level0_lds_bytes(S, 0), l32 = level0_lds_bytes(S, 1);
  size_t r = sizeof(double) * (2 * S.b + S.ns + S.K * S.nr + S.np);
  int rc = 0;
  rc |= set_lds((const void*)k_assemble<double>, l64 > r ? l64 : r, "k_assemble<double>");
  rc |= set_lds((const void*)k_assemble<float>, l32 > r ? l32 : r, "k_assemble<float>");
  const size_t c = sep_solve_lds(S);
  rc |= set_lds((const void*)k_crf_first<double>, c, "k_crf_first<double>");
  rc |= set_lds((const void*)k_crf_first<float>, c, "k_crf_first<float>");
  rc |= set_lds((const void*)k_crf_step<double>, c, "k_crf_step<double>");
  rc |= set_lds((const void*)k_crf_step<float>, c, "k_crf_step<float>");
  rc |= set_lds((const void*)k_cr_bwd<double>, c, "k_cr_bwd<double>");
  rc |= set_lds((const void*)k_cr_bwd<float>, c, "k_cr_bwd<float>");
  const size_t bl = border_solve_lds(S);
  rc |= set_lds((const void*)k_border_solve<double>, bl, "k_border_solve<double>");
  rc |= set_lds((const void*)k_border_solve<float>, bl, "k_border_solve<float>");
  return rc;
}
}  // namespace cl
