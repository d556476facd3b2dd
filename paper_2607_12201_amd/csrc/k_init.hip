// Collocation-consistent starting states on the device: a forward implicit Runge-Kutta (Radau
// IIA) sweep over each instance's mesh at fixed parameters, the states that satisfy every
// collocation and continuity equation of the NLP (eq. 2b-2d) at those parameters.  The paper takes
// its initial state guesses from a forward solve at the nominal parameters (numerical-results
// section, benchmark setup); solving the collocation equations themselves gives the
// interior-point method a start on the constraint manifold.
//
// One workgroup per instance walks its elements in order.  Element i: the first node is z0
// (i = 0, eq. 2d) or the previous element's last node (eq. 2c, right-Radau nodes); the K stage
// values Z solve  sum_j a_jk z_j - h_i f(z_k, theta) = 0  by Newton's method from Z = first node,
// with the dense K ns x K ns Jacobian  a_k'k I - h_i delta_kk' F(z_k)  factored in LDS by Gaussian
// elimination with partial pivoting (one thread per matrix entry of the trailing update), each
// step halved until the largest residual falls (factor 1 - 1e-4 lambda, at most 30 halvings), a
// full step taken once it changes no stage value by more than 1e-13 (1 + the largest).  An
// element whose iteration fails keeps its first node as every stage value and is reported.
#include <math.h>

#include "../../include/colloc.h"
#include "common.h"
#include "elem.h"
#include "kernels.h"

namespace cl {

constexpr int kInitMaxN = 96;   // K ns of the LDS-resident Newton systems
constexpr int kInitMaxIt = 60;

size_t fwd_init_lds(const Shape& S) {
  const int n = S.K * S.ns;
  return sizeof(double) * ((size_t)n * (n + 1) + 4 * (size_t)n + S.ns + S.nr + 3 * (size_t)S.K * S.nr + 256) +
         sizeof(int) * 8;
}

__global__ void __launch_bounds__(256) k_fwd_init(Shape S, Tab tb, const double* __restrict__ theta,
                                                  double* __restrict__ x, int* __restrict__ status) {
  extern __shared__ double lds[];
  const int inst = blockIdx.x;
  const int ns = S.ns, nr = S.nr, np = S.np, K = S.K, n = K * ns, n1 = n + 1;
  const int N = tb.inst_N[inst];
  const int64_t e0 = tb.inst_e0[inst], xo = tb.inst_x[inst];
  double* J = lds;                    // n x (n + 1), row-major: [Jacobian | -G]
  double* Z = J + (size_t)n * n1;     // K x ns stage values
  double* dZ = Z + n;                 // Newton step
  double* Zt = dZ + n;                // trial stage values
  double* G = Zt + n;                 // residual at the trial values
  double* zf = G + n;                 // first node
  double* kap = zf + ns;              // rate constants
  double* rt = kap + nr;              // [K][nr][3] rates and slot partials at the trial values
  double* red = rt + 3 * K * nr;      // 256 doubles: block reductions
  int* ired = (int*)(red + 256);      // pivot row
  const int t = threadIdx.x, nt = blockDim.x;
  // rates at the stage values V and the residual G(V); returns max |G|
  auto residual = [&](const double* V, double h) {
    __syncthreads();
    for (int q = t; q < K * nr; q += nt) {
      const int k = q / nr, r = q - k * nr;
      const int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
      const double f0 = q0 >= 0 ? V[k * ns + q0] : 1.0, f1 = q1 >= 0 ? V[k * ns + q1] : 1.0;
      rt[q * 3] = kap[r] * f0 * f1;
      rt[q * 3 + 1] = q0 >= 0 ? kap[r] * f1 : 0.0;
      rt[q * 3 + 2] = q1 >= 0 ? kap[r] * f0 : 0.0;
    }
    __syncthreads();
    double gm = 0.0;
    for (int row = t; row < n; row += nt) {
      const int k = row / ns + 1, s = row - (k - 1) * ns;
      double g = S.a[0][k] * zf[s];
      for (int kk = 1; kk <= K; ++kk) g += S.a[kk][k] * V[(kk - 1) * ns + s];
      double f = 0.0;
      const int p0 = tb.sp_ptr[inst * (ns + 1) + s], p1 = tb.sp_ptr[inst * (ns + 1) + s + 1];
      for (int o = p0; o < p1; ++o) f += tb.sp_nu[o] * rt[((k - 1) * nr + tb.sp_r[o]) * 3];
      g -= h * f;
      G[row] = g;
      gm = fmax(gm, fabs(g));
    }
    return block_max(gm, red);
  };
  for (int r = t; r < nr; r += nt) {
    const int pc = tb.param[inst * nr + r];
    kap[r] = exp(pc >= 0 ? theta[(int64_t)inst * np + pc] : tb.logk[inst * nr + r]);
  }
  for (int s = t; s < ns; s += nt) zf[s] = tb.z0[inst * ns + s];
  for (int c = t; c < np; c += nt) x[xo + (int64_t)N * S.b + c] = theta[(int64_t)inst * np + c];
  int bad = 0;
  for (int i = 0; i < N; ++i) {
    const double h = tb.elem_h[e0 + i];
    __syncthreads();
    for (int q = t; q < n; q += nt) Z[q] = zf[q % ns];
    double gn = residual(Z, h);
    bool conv = false;
    for (int it = 0; it < kInitMaxIt && !conv; ++it) {
      // Jacobian at Z (its rates are the last ones formed) with -G as the last column
      for (int row = t; row < n; row += nt) {
        const int k = row / ns + 1, s = row - (k - 1) * ns;
        double* Jr = J + (size_t)row * n1;
        for (int c = 0; c < n; ++c) Jr[c] = 0.0;
        for (int kk = 1; kk <= K; ++kk) Jr[(kk - 1) * ns + s] += S.a[kk][k];
        const int p0 = tb.sp_ptr[inst * (ns + 1) + s], p1 = tb.sp_ptr[inst * (ns + 1) + s + 1];
        for (int o = p0; o < p1; ++o) {
          const int r = tb.sp_r[o];
          const double nu = tb.sp_nu[o];
          const double* R = rt + ((k - 1) * nr + r) * 3;
          const int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
          if (q0 >= 0) Jr[(k - 1) * ns + q0] -= h * nu * R[1];
          if (q1 >= 0) Jr[(k - 1) * ns + q1] -= h * nu * R[2];
        }
        Jr[n] = -G[row];
      }
      // Gaussian elimination with partial pivoting on [J | -G]
      for (int c = 0; c < n; ++c) {
        __syncthreads();
        if (t < 64) {
          double best = -1.0;
          int bi = c;
          for (int r = c + t; r < n; r += 64) {
            const double v = fabs(J[(size_t)r * n1 + c]);
            if (v > best) {
              best = v;
              bi = r;
            }
          }
          for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_down(best, off);
            const int oi = __shfl_down(bi, off);
            if (t + off < 64 && (ob > best || (ob == best && oi < bi))) {
              best = ob;
              bi = oi;
            }
          }
          if (t == 0) ired[0] = bi;
        }
        __syncthreads();
        const int p = ired[0];
        if (p != c)
          for (int j = t; j < n1; j += nt) {
            const double a = J[(size_t)c * n1 + j];
            J[(size_t)c * n1 + j] = J[(size_t)p * n1 + j];
            J[(size_t)p * n1 + j] = a;
          }
        __syncthreads();
        const double piv = J[(size_t)c * n1 + c];
        const int w = n - c - 1;   // rows and columns below / right of the pivot (+ the rhs)
        for (int q = t; q < w * (w + 1); q += nt) {
          const int r = c + 1 + q / (w + 1), j = c + 1 + q % (w + 1);
          J[(size_t)r * n1 + j] -= J[(size_t)r * n1 + c] / piv * J[(size_t)c * n1 + j];
        }
      }
      __syncthreads();
      for (int c = n - 1; c >= 0; --c) {   // back substitution, one column at a time
        if (t == 0) dZ[c] = J[(size_t)c * n1 + n] / J[(size_t)c * n1 + c];
        __syncthreads();
        for (int r = t; r < c; r += nt) J[(size_t)r * n1 + n] -= J[(size_t)r * n1 + c] * dZ[c];
        __syncthreads();
      }
      double dm = 0.0, zm = 0.0;
      for (int q = t; q < n; q += nt) {
        dm = fmax(dm, fabs(dZ[q]));
        zm = fmax(zm, fabs(Z[q] + dZ[q]));
      }
      dm = block_max(dm, red);
      zm = block_max(zm, red);
      if (dm <= 1e-13 * (1.0 + zm)) {   // converged: the full step is taken
        for (int q = t; q < n; q += nt) Z[q] += dZ[q];
        conv = true;
        break;
      }
      // damping: halve the step until the largest residual falls
      double lam = 1.0, gt = 0.0;
      for (int bt = 0; bt < 30; ++bt) {
        __syncthreads();
        for (int q = t; q < n; q += nt) Zt[q] = Z[q] + lam * dZ[q];
        gt = residual(Zt, h);
        if (gt <= (1.0 - 1e-4 * lam) * gn) break;
        lam *= 0.5;
      }
      __syncthreads();
      for (int q = t; q < n; q += nt) Z[q] = Zt[q];
      gn = gt;
    }
    __syncthreads();
    if (!conv) {   // the element keeps its first node as every stage value
      if (!bad) bad = i + 1;
      for (int q = t; q < n; q += nt) Z[q] = zf[q % ns];
    }
    __syncthreads();
    double* xe = x + xo + (int64_t)i * S.b;
    for (int s = t; s < ns; s += nt) xe[s] = zf[s];
    for (int q = t; q < n; q += nt) xe[ns + q] = Z[q];
    __syncthreads();
    for (int s = t; s < ns; s += nt) zf[s] = Z[(K - 1) * ns + s];   // right-Radau: last node
  }
  if (t == 0) status[inst] = bad;
}

int launch_fwd_init(const Shape& S, const Tab& tb, const double* theta, double* x, int* status,
                    hipStream_t st) {
  if (S.K * S.ns > kInitMaxN) return -2;
  const size_t lds = fwd_init_lds(S);
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_fwd_init, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
          hipSuccess)
    return -3;
  hipLaunchKernelGGL(k_fwd_init, dim3(tb.n_inst), dim3(256), lds, st, S, tb, theta, x, status);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace cl
