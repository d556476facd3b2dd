// Per-element device helpers: mass-action rates, J v, J^T u and W v for one finite element,
// executed cooperatively by the threads of one workgroup on LDS-resident vectors.
#pragma once
#include "common.h"

namespace cl {

__device__ inline int tid() { return threadIdx.x; }
__device__ inline int nthr() { return blockDim.x; }

// c ? a : b kept as a select.  A plain conditional whose operand is a single-use load may be
// turned into a branch around that load, which then waits for it inside the branch; gathers
// that issue several loads before using any of them pick their results with this.
__device__ inline double pick(bool c, double a, double b) { return __builtin_unpredictable(c) ? a : b; }

// Per-instance skip flag read once per workgroup: other workgroups of the same launch may set
// it concurrently, so every wave takes the decision from one LDS copy (uniform control flow
// around the barriers that follow).
__device__ inline bool block_flag(const int* f) {
  __shared__ int sflag;
  if (threadIdx.x == 0) sflag = __atomic_load_n(f, __ATOMIC_RELAXED);
  __syncthreads();
  return sflag != 0;
}

// kappa_r = exp(theta[param_r]) or exp(logk_r)
__device__ inline void load_kappa(const Shape& S, const Tab& tb, int inst, const double* th,
                                  double* kap) {
  for (int r = tid(); r < S.nr; r += nthr()) {
    int c = tb.param[inst * S.nr + r];
    kap[r] = exp(c >= 0 ? th[c] : tb.logk[inst * S.nr + r]);
  }
}

// rho[k-1][r] and slot partials at collocation points k = 1..K of an element (z in LDS).
__device__ inline void rates(const Shape& S, const Tab& tb, int inst, const double* z,
                             const double* kap, double* rho, double* d0, double* d1) {
  const int nr = S.nr, ns = S.ns;
  for (int t = tid(); t < S.K * nr; t += nthr()) {
    int k = t / nr + 1, r = t - (k - 1) * nr;
    int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
    double u0 = q0 >= 0 ? z[k * ns + q0] : 1.0;
    double u1 = q1 >= 0 ? z[k * ns + q1] : 1.0;
    double kk = kap[r];
    rho[t] = kk * u0 * u1;
    if (d0) {
      d0[t] = q0 >= 0 ? kk * u1 : 0.0;
      d1[t] = q1 >= 0 ? kk * u0 : 0.0;
    }
  }
}

// Collocation/continuity residual rows of element i (b rows, LDS out).
__device__ inline void residual_rows(const Shape& S, const Tab& tb, int inst, int i, double h,
                                     const double* z, const double* zprevK, const double* rho,
                                     double* g) {
  const int ns = S.ns, nr = S.nr;
  for (int t = tid(); t < S.b; t += nthr()) {
    int j = t / ns, s = t - j * ns;
    double v;
    if (j == 0) {
      v = z[s] - (i == 0 ? tb.z0[inst * ns + s] : zprevK[s]);
    } else {
      double acc = 0.0;
      for (int jj = 0; jj <= S.K; ++jj) acc += S.a[jj][j] * z[jj * ns + s];
      double f = 0.0;
      int p0 = tb.sp_ptr[inst * (ns + 1) + s], p1 = tb.sp_ptr[inst * (ns + 1) + s + 1];
      for (int q = p0; q < p1; ++q) f += tb.sp_nu[q] * rho[(j - 1) * nr + tb.sp_r[q]];
      v = acc - h * f;
    }
    g[t] = v;
  }
}

// (J v) for the b rows of element i.  v: element's z (LDS, b), vprevK: node-K values of the
// previous element (ns) or unused for i == 0, vth: theta part (np), jac: element's values.
template <bool AB = false>
__device__ inline void jv_rows(const Shape& S, const Tab& tb, int inst, int i, double h,
                               const double* jac, const double* v, const double* vprevK,
                               const double* vth, double* out) {
  // AB: every coefficient taken in absolute value and every term added (v >= 0 expected), an
  // upper bound of |J| v
  const int ns = S.ns, nr = S.nr;
  auto ab = [](double x) { return AB ? fabs(x) : x; };
  for (int t = tid(); t < S.b; t += nthr()) {
    int j = t / ns, s = t - j * ns;
    double acc;
    if (j == 0) {
      const double pv = i == 0 ? 0.0 : vprevK[s];
      acc = AB ? v[s] + pv : v[s] - pv;
    } else {
      acc = 0.0;
      for (int jj = 0; jj <= S.K; ++jj) acc += ab(S.a[jj][j]) * v[jj * ns + s];
      double f = 0.0;
      int p0 = tb.sp_ptr[inst * (ns + 1) + s], p1 = tb.sp_ptr[inst * (ns + 1) + s + 1];
      for (int q = p0; q < p1; ++q) {
        int r = tb.sp_r[q];
        const double* jr = jac + ((j - 1) * nr + r) * 3;
        int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
        int c = tb.param[inst * nr + r];
        double dr = 0.0;
        if (q0 >= 0) dr += ab(jr[0]) * v[j * ns + q0];
        if (q1 >= 0) dr += ab(jr[1]) * v[j * ns + q1];
        if (c >= 0) dr += ab(jr[2]) * vth[c];
        f += ab(tb.sp_nu[q]) * dr;
      }
      acc = AB ? acc + fabs(h) * f : acc - h * f;
    }
    out[t] = acc;
  }
}

// phi[k-1][r] = sum_s nu_sr u[k][s]: reaction-space projection of row weights (LDS).
template <bool AB = false>
__device__ inline void reaction_weights(const Shape& S, const Tab& tb, int inst, const double* u,
                                        double* phi) {
  const int nr = S.nr, ns = S.ns;
  for (int t = tid(); t < S.K * nr; t += nthr()) {
    int k = t / nr + 1, r = t - (k - 1) * nr;
    double acc = 0.0;
    for (int q = 0; q < 4; ++q) {
      int sp = tb.rx_sp[(inst * nr + r) * 4 + q];
      const double nu = tb.rx_nu[(inst * nr + r) * 4 + q];
      if (sp >= 0) acc += (AB ? fabs(nu) : nu) * u[k * ns + sp];
    }
    phi[t] = acc;
  }
}

// (J^T u) restricted to element i's z variables (b outputs) given the element's row weights
// u (b), the next element's node-0 row weights unext0 (ns; nullptr for the last element), and
// phi from reaction_weights.  Theta contributions are returned per parameter (np partials).
template <bool AB = false>
__device__ inline void jtu_rows(const Shape& S, const Tab& tb, int inst, double h,
                                const double* jac, const double* u, const double* unext0,
                                const double* phi, double* outz, double* outth) {
  const int ns = S.ns, nr = S.nr, K = S.K;
  auto ab = [](double x) { return AB ? fabs(x) : x; };
  for (int t = tid(); t < S.b; t += nthr()) {
    int j = t / ns, s = t - j * ns;
    double acc = (j == 0) ? u[s] : 0.0;
    for (int k = 1; k <= K; ++k) acc += ab(S.a[j][k]) * u[k * ns + s];
    if (j >= 1) {   // reactant slots of species s (a 2A reaction lists both slots)
      double f = 0.0;
      const int o0 = tb.rq_ptr[inst * (ns + 1) + s], o1 = tb.rq_ptr[inst * (ns + 1) + s + 1];
      for (int o = o0; o < o1; ++o) {
        const int r = tb.rq_r[o];
        f += ab(jac[((j - 1) * nr + r) * 3 + tb.rq_t[o]]) * phi[(j - 1) * nr + r];
      }
      acc = AB ? acc + fabs(h) * f : acc - h * f;
    }
    if (j == K && unext0) acc = AB ? acc + unext0[s] : acc - unext0[s];
    outz[t] = acc;
  }
  if (outth) {
    for (int c = tid(); c < S.np; c += nthr()) {   // reactions of parameter c
      double acc = 0.0;
      const int o0 = tb.pc_ptr[inst * (S.np + 1) + c], o1 = tb.pc_ptr[inst * (S.np + 1) + c + 1];
      for (int k = 1; k <= K; ++k)
        for (int o = o0; o < o1; ++o) {
          const int r = tb.pc_r[o];
          acc += ab(jac[((k - 1) * nr + r) * 3 + 2]) * phi[(k - 1) * nr + r];
        }
      outth[c] = AB ? fabs(h) * acc : -h * acc;
    }
  }
}

// (W v) for element i: z outputs (b) and theta partials (np).  W = sum of the reaction
// second-derivative patterns (hess values) plus the measurement Hessian of the element.
template <bool AB = false>
__device__ inline void wv_rows(const Shape& S, const Tab& tb, int inst, int64_t e,
                               const double* hess, const double* v, const double* vth,
                               double* outz, double* outth) {
  const int ns = S.ns, nr = S.nr, K = S.K;
  auto ab = [](double x) { return AB ? fabs(x) : x; };
  for (int t = tid(); t < S.b; t += nthr()) {
    int j = t / ns, s = t - j * ns;
    double acc = 0.0;
    if (j >= 1) {   // reactant slots of species s
      const int o0 = tb.rq_ptr[inst * (ns + 1) + s], o1 = tb.rq_ptr[inst * (ns + 1) + s + 1];
      for (int o = o0; o < o1; ++o) {
        const int r = tb.rq_r[o], sl = tb.rq_t[o];
        const int other = tb.react[(inst * nr + r) * 2 + (1 - sl)];
        const int c = tb.param[inst * nr + r];
        const double* H = hess + ((j - 1) * nr + r) * 4;
        if (other >= 0) acc += ab(H[0]) * v[j * ns + other];
        if (c >= 0) acc += ab(H[1 + sl]) * vth[c];
      }
    }
    int m0 = tb.elem_mptr[e], m1 = tb.elem_mptr[e + 1];
    for (int m = m0; m < m1; ++m) {
      if (tb.meas_sp[m] != s) continue;
      const double* w = tb.meas_w + (int64_t)m * (K + 1);
      double dot = 0.0;
      for (int jj = 0; jj <= K; ++jj) dot += ab(w[jj]) * v[jj * ns + s];
      acc += ab(w[j]) * dot;
    }
    outz[t] = acc;
  }
  if (outth) {
    for (int c = tid(); c < S.np; c += nthr()) {   // reactions of parameter c
      double acc = 0.0;
      const int o0 = tb.pc_ptr[inst * (S.np + 1) + c], o1 = tb.pc_ptr[inst * (S.np + 1) + c + 1];
      for (int k = 1; k <= K; ++k)
        for (int o = o0; o < o1; ++o) {
          const int r = tb.pc_r[o];
          int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
          const double* H = hess + ((k - 1) * nr + r) * 4;
          if (q0 >= 0) acc += ab(H[1]) * v[k * ns + q0];
          if (q1 >= 0) acc += ab(H[2]) * v[k * ns + q1];
          acc += ab(H[3]) * vth[c];
        }
      outth[c] = acc;
    }
  }
}

// Objective residuals r_m of the element's measurements and grad Phi on its z (owner per var).
__device__ inline double obj_element(const Shape& S, const Tab& tb, int64_t e, const double* z,
                                     double* gradz) {
  const int ns = S.ns, K = S.K;
  int m0 = tb.elem_mptr[e], m1 = tb.elem_mptr[e + 1];
  if (gradz) {
    for (int t = tid(); t < S.b; t += nthr()) {
      int j = t / ns, s = t - j * ns;
      double acc = 0.0;
      for (int m = m0; m < m1; ++m) {
        if (tb.meas_sp[m] != s) continue;
        const double* w = tb.meas_w + (int64_t)m * (K + 1);
        double pr = -tb.meas_ys[m];
        for (int jj = 0; jj <= K; ++jj) pr += w[jj] * z[jj * ns + s];
        acc += pr * w[j];
      }
      gradz[t] = acc;
    }
  }
  // objective: sequential over the element's measurements (fixed order, few per element)
  double phi = 0.0;
  for (int m = m0; m < m1; ++m) {
    const double* w = tb.meas_w + (int64_t)m * (K + 1);
    int s = tb.meas_sp[m];
    double pr = -tb.meas_ys[m];
    for (int jj = 0; jj <= K; ++jj) pr += w[jj] * z[jj * ns + s];
    phi += 0.5 * pr * pr;
  }
  return phi;
}

// out[c] = sum over the instance's elements i < N of part[(e0 + i) * np + c].  Thread t covers
// parameter t % np over the elements t / np, t / np + G, ... (G = threads / np groups); the
// groups are then added in order, so the result depends only on N, np and the block size.
// red: nthr() doubles of LDS; out: np doubles of LDS.
// NS sums, then NM maxima, then NN minima, reduced together over the workgroup: a butterfly
// over each wave (every lane ends with the same value: each pairwise step is commutative), then
// the wave results combined in wave order.  red: at least (NS + NM + NN) * waves doubles.
template <int NS, int NM, int NN>
__device__ inline void block_reduce_multi(double* v, double* red) {
  constexpr int NV = NS + NM + NN;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double o = __shfl_xor(v[k], off);
      v[k] = k < NS ? v[k] + o : (k < NS + NM ? fmax(v[k], o) : fmin(v[k], o));
    }
  }
  const int nw = (nthr() + 63) / 64;
  if ((tid() & 63) == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[(tid() / 64) * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double a = red[k];
    for (int w = 1; w < nw; ++w) {
      const double o = red[w * NV + k];
      a = k < NS ? a + o : (k < NS + NM ? fmax(a, o) : fmin(a, o));
    }
    v[k] = a;
  }
  __syncthreads();
}

__device__ inline void theta_sum(const double* part, int64_t e0, int N, int np, double* out,
                                 double* red) {
  const int G = nthr() / np;
  if (G >= 1) {
    const int c = tid() % np, g = tid() / np;
    double acc = 0.0, acc2 = 0.0;
    if (g < G) {
      int i = g;
      for (; i + G < N; i += 2 * G) {
        acc += part[(e0 + i) * np + c];
        acc2 += part[(e0 + i + G) * np + c];
      }
      for (; i < N; i += G) acc += part[(e0 + i) * np + c];
    }
    red[tid()] = acc + acc2;
    __syncthreads();
    for (int c2 = tid(); c2 < np; c2 += nthr()) {
      double sum = 0.0;
      for (int gg = 0; gg < G; ++gg) sum += red[gg * np + c2];
      out[c2] = sum;
    }
  } else {
    for (int c2 = tid(); c2 < np; c2 += nthr()) {
      double sum = 0.0;
      for (int i = 0; i < N; ++i) sum += part[(e0 + i) * np + c2];
      out[c2] = sum;
    }
  }
  __syncthreads();
}

// Deterministic block reductions (fixed pairing for a given blockDim).
__device__ inline double block_sum(double v, double* red) {
  red[tid()] = v;
  __syncthreads();
  for (int w = nthr() / 2; w > 0; w >>= 1) {
    if (tid() < w) red[tid()] += red[tid() + w];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}
__device__ inline double block_max(double v, double* red) {
  red[tid()] = v;
  __syncthreads();
  for (int w = nthr() / 2; w > 0; w >>= 1) {
    if (tid() < w) red[tid()] = fmax(red[tid()], red[tid() + w]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}
__device__ inline double block_min(double v, double* red) {
  red[tid()] = v;
  __syncthreads();
  for (int w = nthr() / 2; w > 0; w >>= 1) {
    if (tid() < w) red[tid()] = fmin(red[tid()], red[tid() + w]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Sum of the chunk partials of parameter c of an instance, in chunk order.
__device__ inline double thpart_sum(const Ws& ws, const double* part, int inst, int N, int np, int c) {
  const int nch = (int)cl_ceil_div(N, CL_THCHUNK);
  const double* p = part + (int64_t)inst * ws.nchunk * np + c;
  double acc = 0.0;
#pragma unroll 8
  for (int ch = 0; ch < nch; ++ch) acc += p[(int64_t)ch * np];
  return acc;
}

}  // namespace cl
