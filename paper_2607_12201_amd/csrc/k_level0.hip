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

namespace cl {

__device__ inline double base_entry(const Shape& S, const Tab& tb, int64_t e, int i, double dw,
                                    const double* d0, int r, int q);
__device__ inline double node_entry(const Shape& S, int k, double h, const double* d,
                                    const double* F, const double* Fth, const double* Wzz,
                                    const double* Wzt, const double* Wtt, int r, int q);

// node-0 rows (initial condition / continuity), measurement Hessian, dw on z; P couplings.
__device__ inline double base_entry(const Shape& S, const Tab& tb, int64_t e, int i, double dw,
                                    const double* d0, int r, int q) {
  const int ns = S.ns, b = S.b, K = S.K, bp = S.b + S.np;
  if (r >= bp) {  // P row: previous separator, coupled by the continuity rows (eq. 2c)
    const int s = r - bp;
    if (i == 0) return 0.0;
    if (q < bp) return (q == s) ? -d0[s] : 0.0;
    return (q == r) ? d0[s] : 0.0;
  }
  if (r >= b) return 0.0;   // theta rows: parameter bounds and dw are added once per instance
  int j1 = r / ns, s1 = r - j1 * ns, j2 = q / ns, s2 = q - j2 * ns;
  double v = (r == q) ? dw : 0.0;
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

// Contribution of the collocation rows of point k (eq. 2b / 3) to entry (r, q), r >= q, both in
// the element's natural order (z (j, s) at j*ns + s, theta c at b + c): the rows are
// a_jk e_(j,s) - h (F_k)_(s,.) on node k and -h (Fth_k)_(s,.) on theta, weighted by d_(k,s).
__device__ inline double node_entry(const Shape& S, int k, double h, const double* d,
                                    const double* F, const double* Fth, const double* Wzz,
                                    const double* Wzt, const double* Wtt, int r, int q) {
  const int ns = S.ns, np = S.np, b = S.b;
  double v = 0.0;
  if (r < b) {
    int j1 = r / ns, s1 = r - j1 * ns, j2 = q / ns, s2 = q - j2 * ns;
    double a1 = S.a[j1][k], a2 = S.a[j2][k];
    if (s1 == s2) v += d[s1] * a1 * a2;
    if (j2 == k) v -= h * d[s1] * a1 * F[s1 * ns + s2];
    if (j1 == k) v -= h * d[s2] * a2 * F[s2 * ns + s1];
    if (j1 == k && j2 == k) {
      double acc = 0.0;
      for (int s = 0; s < ns; ++s) acc += d[s] * F[s * ns + s1] * F[s * ns + s2];
      v += h * h * acc + Wzz[s1 * ns + s2];
    }
  } else if (q < b) {
    int c = r - b, j1 = q / ns, s1 = q - j1 * ns;
    v -= h * d[s1] * S.a[j1][k] * Fth[s1 * np + c];
    if (j1 == k) {
      double acc = 0.0;
      for (int s = 0; s < ns; ++s) acc += d[s] * F[s * ns + s1] * Fth[s * np + c];
      v += h * h * acc + Wzt[s1 * np + c];
    }
  } else {
    int c1 = r - b, c2 = q - b;
    double acc = 0.0;
    for (int s = 0; s < ns; ++s) acc += d[s] * Fth[s * np + c1] * Fth[s * np + c2];
    v = h * h * acc + (c1 == c2 ? Wtt[c1] : 0.0);
  }
  return v;
}

// F_k, Fth_k (species rows of d f / d (u, theta) at point k) and the second-derivative
// patterns W at point k, from the per-reaction values; one thread per species row.
__device__ inline void node_data(const Shape& S, const Tab& tb, int inst, int k,
                                 const double* jac_e, const double* hess_e, const double* Ds_e,
                                 double* d, double* F, double* Fth, double* Wzz, double* Wzt,
                                 double* Wtt) {
  const int ns = S.ns, np = S.np, nr = S.nr;
  for (int s = tid(); s < ns; s += nthr()) {
    d[s] = Ds_e[k * ns + s];
    for (int q = 0; q < ns; ++q) F[s * ns + q] = 0.0;
    for (int c = 0; c < np; ++c) Fth[s * np + c] = 0.0;
    int p0 = tb.sp_ptr[inst * (ns + 1) + s], p1 = tb.sp_ptr[inst * (ns + 1) + s + 1];
    for (int q = p0; q < p1; ++q) {
      int r = tb.sp_r[q];
      double nu = tb.sp_nu[q];
      const double* jr = jac_e + ((k - 1) * nr + r) * 3;
      int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
      int c = tb.param[inst * nr + r];
      if (q0 >= 0) F[s * ns + q0] += nu * jr[0];
      if (q1 >= 0) F[s * ns + q1] += nu * jr[1];
      if (c >= 0) Fth[s * np + c] += nu * jr[2];
    }
  }
  for (int q = tid(); q < ns; q += nthr()) {
    for (int s2 = 0; s2 < ns; ++s2) Wzz[q * ns + s2] = 0.0;
    for (int c = 0; c < np; ++c) Wzt[q * np + c] = 0.0;
    for (int r = 0; r < nr; ++r) {
      int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
      if (q0 != q && q1 != q) continue;
      int c = tb.param[inst * nr + r];
      const double* H = hess_e + ((k - 1) * nr + r) * 4;
      if (q0 == q) {
        if (q1 >= 0) Wzz[q * ns + q1] += H[0];
        if (c >= 0) Wzt[q * np + c] += H[1];
      }
      if (q1 == q) {
        if (q0 >= 0) Wzz[q * ns + q0] += H[0];
        if (c >= 0) Wzt[q * np + c] += H[2];
      }
    }
  }
  for (int c = tid(); c < np; c += nthr()) {
    double acc = 0.0;
    for (int r = 0; r < nr; ++r)
      if (tb.param[inst * nr + r] == c) acc += hess_e[((k - 1) * nr + r) * 4 + 3];
    Wtt[c] = acc;
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

// Right-looking elimination of the mI interior columns on register-resident entries.
template <typename T, int TS, int NB>
__device__ inline bool eliminate_regs(T* acc, int mI, int R, int ty, int tx, double* colb,
                                      double* misc) {
  bool ok = true;
#pragma unroll
  for (int J = 0; J < NB; ++J) {
    for (int cc = 0; cc < TS; ++cc) {
      const int c = J * TS + cc;
      if (c >= mI) break;
      if (ty == cc && tx == cc) {
        double piv = (double)acc[J * (J + 1) / 2 + J];
        bool good = piv > 0.0 && isfinite(piv);
        double sq = good ? sqrt(piv) : 1.0;
        acc[J * (J + 1) / 2 + J] = (T)sq;
        misc[0] = good ? 1.0 : 0.0;
        misc[1] = 1.0 / sq;
      }
      __syncthreads();
      if (misc[0] == 0.0) {
        ok = false;
        break;
      }
      const T inv = (T)misc[1];
      if (tx == cc) {
#pragma unroll
        for (int I = J; I < NB; ++I) {
          const int r = I * TS + ty;
          if (r > c && r < R) {
            acc[I * (I + 1) / 2 + J] *= inv;
            colb[r] = (double)acc[I * (I + 1) / 2 + J];
          }
        }
      }
      __syncthreads();
      T cr[NB], cq[NB];
#pragma unroll
      for (int I = J; I < NB; ++I) {
        const int r = I * TS + ty, q = I * TS + tx;
        cr[I] = (r > c && r < R) ? (T)colb[r] : (T)0;
        cq[I] = (q > c && q < R) ? (T)colb[q] : (T)0;
      }
#pragma unroll
      for (int I = J; I < NB; ++I)
#pragma unroll
        for (int J2 = J; J2 <= I; ++J2) acc[I * (I + 1) / 2 + J2] -= cr[I] * cq[J2];
    }
    if (!ok) break;
  }
  return ok;
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

template <typename T, int TS, int NB>
__global__ void __launch_bounds__(TS* TS) k_level0r(Shape S, Tab tb, Ws ws, int fused) {
  extern __shared__ double lds[];
  constexpr int NBLK = NB * (NB + 1) / 2;
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const int ns = S.ns, np = S.np, b = S.b, mI = S.mI, R = S.R, bp = S.b + S.np;
  const int ty = threadIdx.x / TS, tx = threadIdx.x % TS;
  double* d0 = lds;
  double* nd = d0 + ns;
  double* F = nd + ns;
  double* Fth = F + ns * ns;
  double* Wzz = Fth + ns * np;
  double* Wzt = Wzz + ns * ns;
  double* Wtt = Wzt + ns * np;
  double* colb = Wtt + np;
  double* misc = colb + NB * TS;
  double av[NBLK];

  if (fused) {
    const int64_t jl = (int64_t)S.K * S.nr;
    const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
    const double* Ds_e = ws.Ds + gi;
    const double* jac_e = ws.jac + e * jl * 3;
    const double* hess_e = ws.hess + e * jl * 4;
    const double h = tb.elem_h[e], dw = ws.dw[inst];
    for (int t = tid(); t < ns; t += nthr()) d0[t] = Ds_e[t];
    __syncthreads();
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const int r = I * TS + ty, q = J * TS + tx;
        av[I * (I + 1) / 2 + J] = (r < R && q <= r) ? base_entry(S, tb, e, i, dw, d0, r, q) : 0.0;
      }
    for (int k = 1; k <= S.K; ++k) {
      __syncthreads();
      node_data(S, tb, inst, k, jac_e, hess_e, Ds_e, nd, F, Fth, Wzz, Wzt, Wtt);
      __syncthreads();
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) {
          const int r = I * TS + ty, q = J * TS + tx;
          if (r < bp && q <= r)
            av[I * (I + 1) / 2 + J] += node_entry(S, k, h, nd, F, Fth, Wzz, Wzt, Wtt, r, q);
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
  } else {
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J) {
        const int r = I * TS + ty, q = J * TS + tx;
        av[I * (I + 1) / 2 + J] = (r < R && q <= r) ? stored_entry<T>(S, ws, e, r, q) : 0.0;
      }
  }

  bool ok;
  if constexpr (sizeof(T) == 8) {
    ok = eliminate_regs<double, TS, NB>(av, mI, R, ty, tx, colb, misc);
    if (ok) store_regs<double, TS, NB>(S, ws, e, i, av, ty, tx);
  } else {
    float af[NBLK];
#pragma unroll
    for (int B = 0; B < NBLK; ++B) af[B] = (float)av[B];
    ok = eliminate_regs<float, TS, NB>(af, mI, R, ty, tx, colb, misc);
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

size_t level0r_lds_bytes(const Shape& S) {
  int TS = S.R <= 32 ? 8 : 16;
  int NB = (int)cl_ceil_div(S.R, TS);
  return sizeof(double) * (2 * S.ns + 2 * S.ns * S.ns + 2 * S.ns * S.np + S.np + NB * TS + 8);
}

bool level0r_supported(const Shape& S) { return S.R <= 160; }

template <typename T, int TS, int NB>
static void launch_one(const Shape& S, const Tab& tb, const Ws& ws, int fused, hipStream_t st) {
  hipLaunchKernelGGL((k_level0r<T, TS, NB>), dim3((unsigned)tb.n_elem), dim3(TS * TS),
                     level0r_lds_bytes(S), st, S, tb, ws, fused);
}

template <typename T>
static int launch_t(const Shape& S, const Tab& tb, const Ws& ws, int fused, hipStream_t st) {
  if (S.R <= 32) {
    switch ((int)cl_ceil_div(S.R, 8)) {
      case 1: launch_one<T, 8, 1>(S, tb, ws, fused, st); return 0;
      case 2: launch_one<T, 8, 2>(S, tb, ws, fused, st); return 0;
      case 3: launch_one<T, 8, 3>(S, tb, ws, fused, st); return 0;
      case 4: launch_one<T, 8, 4>(S, tb, ws, fused, st); return 0;
    }
  }
  switch ((int)cl_ceil_div(S.R, 16)) {
    case 3: launch_one<T, 16, 3>(S, tb, ws, fused, st); return 0;
    case 4: launch_one<T, 16, 4>(S, tb, ws, fused, st); return 0;
    case 5: launch_one<T, 16, 5>(S, tb, ws, fused, st); return 0;
    case 6: launch_one<T, 16, 6>(S, tb, ws, fused, st); return 0;
    case 7: launch_one<T, 16, 7>(S, tb, ws, fused, st); return 0;
    case 8: launch_one<T, 16, 8>(S, tb, ws, fused, st); return 0;
    case 9: launch_one<T, 16, 9>(S, tb, ws, fused, st); return 0;
    case 10: launch_one<T, 16, 10>(S, tb, ws, fused, st); return 0;
  }
  return -1;
}

int launch_level0(const Shape& S, const Tab& tb, const Ws& ws, int prec, bool fused, hipStream_t st) {
  return prec ? launch_t<float>(S, tb, ws, fused ? 1 : 0, st) : launch_t<double>(S, tb, ws, fused ? 1 : 0, st);
}

}  // namespace cl
