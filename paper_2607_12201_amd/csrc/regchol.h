// Register-resident partial Cholesky shared by the element, separator-chain and border kernels.
//
// A symmetric matrix of size R lives in registers: a TS x TS thread grid owns its lower-triangle
// entries block-cyclically (thread (ty, tx) owns rows ty + TS*I and columns tx + TS*J, entry
// (I, J) at acc[I*(I+1)/2 + J]).  eliminate_regs factors the first mI columns; on return the
// eliminated columns hold L (diagonal block) and the rows below it L^-1-transformed, and the
// trailing block holds its Schur complement.
#pragma once
#include "elem.h"

namespace cl {

// Right-looking elimination of the first mI columns on register-resident entries, in
// panels of up to 4 columns: the owners copy the panel (rows >= c0) into LDS, one wave factors
// it in registers, the owners take the factored columns back and every thread applies the rank-w
// update to its entries right of the panel.  pbuf: two R x 4 buffers (alternating panels).
template <typename T, int TS, int NB>
__device__ inline bool eliminate_regs(T* acc, int mI, int R, int ty, int tx, double* pbuf,
                                      double* misc) {
  int buf = 0;
#pragma unroll
  for (int J = 0; J < NB; ++J) {
    for (int cb = 0; cb < TS; cb += 4) {
      const int c0 = J * TS + cb;
      if (c0 >= mI) break;
      const int w = min(4, mI - c0);
      double* P = pbuf + buf * R * 4;
      buf ^= 1;
      const int cl_own = tx - cb;
      if (cl_own >= 0 && cl_own < w) {
        const int q = J * TS + tx;
#pragma unroll
        for (int I = J; I < NB; ++I) {
          const int r = I * TS + ty;
          if (r >= q && r < R) P[r * 4 + cl_own] = (double)acc[I * (I + 1) / 2 + J];
        }
      }
      __syncthreads();
      if (tid() < 64) {
        // wave 0 factors the panel in registers: lane t holds panel rows c0 + t + 64 m
        // (R - c0 <= 192); the pivot row values come from their owner lanes by shuffles
        const int lane = tid();
        double p[3][4];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const int r = c0 + lane + 64 * m;
#pragma unroll
          for (int cl = 0; cl < 4; ++cl) p[m][cl] = (r < R && cl < w) ? P[r * 4 + cl] : 0.0;
        }
        bool good = true;
#pragma unroll
        for (int cl = 0; cl < 4; ++cl) {
          if (cl < w && good) {
            const double piv = __shfl(p[0][cl], cl);
            good = piv > 0.0 && isfinite(piv);
            const double sq = good ? sqrt(piv) : 1.0;
            const double inv = 1.0 / sq;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
              const int rl = lane + 64 * m;
              if (rl == cl) p[m][cl] = sq;
              else if (rl > cl) p[m][cl] *= inv;
            }
#pragma unroll
            for (int cl2 = cl + 1; cl2 < 4; ++cl2) {
              if (cl2 < w) {
                const double lc = __shfl(p[0][cl], cl2);
#pragma unroll
                for (int m = 0; m < 3; ++m)
                  if (lane + 64 * m >= cl2) p[m][cl2] -= p[m][cl] * lc;
              }
            }
          }
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const int r = c0 + lane + 64 * m;
#pragma unroll
          for (int cl = 0; cl < 4; ++cl)
            if (r < R && cl < w) P[r * 4 + cl] = p[m][cl];
        }
        if (lane == 0) misc[0] = good ? 1.0 : 0.0;
      }
      __syncthreads();
      if (misc[0] == 0.0) return false;
      if (cl_own >= 0 && cl_own < w) {
        const int q = J * TS + tx;
#pragma unroll
        for (int I = J; I < NB; ++I) {
          const int r = I * TS + ty;
          if (r >= q && r < R) acc[I * (I + 1) / 2 + J] = (T)P[r * 4 + cl_own];
        }
      }
      const int cend = c0 + w;
      for (int cl = 0; cl < w; ++cl) {
        T cr[NB], cq[NB];
#pragma unroll
        for (int I = J; I < NB; ++I) {
          const int r = I * TS + ty, q = I * TS + tx;
          cr[I] = (r >= cend && r < R) ? (T)P[r * 4 + cl] : (T)0;
          cq[I] = (q >= cend && q < R) ? (T)P[q * 4 + cl] : (T)0;
        }
#pragma unroll
        for (int I = J; I < NB; ++I)
#pragma unroll
          for (int J2 = J; J2 <= I; ++J2) acc[I * (I + 1) / 2 + J2] -= cr[I] * cq[J2];
      }
    }
  }
  return true;
}

}  // namespace cl
