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

// Value of x held by lane `lane` of the wave (lane uniform): two scalar lane reads, far cheaper
// than an LDS permute.
__device__ inline double lane_value(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// LDS of eliminate_regs for R rows: two R x 4 panel buffers and the zero-padded copy
// (TS * NB <= R + 23 rows by 4).
__host__ __device__ constexpr int elim_lds_doubles(int R) { return 8 * R + 4 * (R + 24); }

// Right-looking elimination of the first mI columns on register-resident entries, in
// panels of up to 4 columns: the owners copy the panel (rows >= c0) into LDS, one wave factors
// it in registers, the owners take the factored columns back and every thread applies the rank-w
// update to its entries right of the panel.  pbuf: two R x 4 buffers (alternating panels,
// column-major), then Z: the factored panel again over rows J*TS .. NB*TS with zeros in the
// rows above the trailing block and below R, so the update reads its multipliers without masks
// (one buffer suffices: it is written after the barrier that every thread reaches only once its
// previous update is done).
template <typename T, int TS, int NB>
__device__ inline bool eliminate_regs(T* acc, int mI, int R, int ty, int tx, double* pbuf,
                                      double* misc) {
  constexpr int RZ = TS * NB;
  double* Z = pbuf + 8 * R;
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
          if (r >= q && r < R) P[cl_own * R + r] = (double)acc[I * (I + 1) / 2 + J];
        }
      }
      __syncthreads();
      if (tid() < 64) {
        // wave 0 factors the panel in registers: lane t holds panel rows c0 + t + 64 m
        // (R - c0 <= 192); the pivot row values come from their owner lanes by lane reads.
        // Per-row choices are selects, not branches; row groups past R are skipped whole.
        const int lane = tid();
        double p[3][4];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const int r = c0 + lane + 64 * m;
          const int rr = r < R ? r : 0;
#pragma unroll
          for (int cl = 0; cl < 4; ++cl) p[m][cl] = pick(r < R && cl < w, P[cl * R + rr], 0.0);
        }
        bool good = true;
#pragma unroll
        for (int cl = 0; cl < 4; ++cl) {
          if (cl < w && good) {
            // pivot and 1/sqrt(pivot) once per column on the wave-uniform value
            const double piv = lane_value(p[0][cl], cl);
            good = piv > 0.0 && isfinite(piv);
            const double inv = good ? rsqrt(piv) : 1.0;
            const double sq = good ? piv * inv : 1.0;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
              const int rl = lane + 64 * m;
              p[m][cl] = pick(rl == cl, sq, pick(rl > cl, p[m][cl] * inv, p[m][cl]));
            }
#pragma unroll
            for (int cl2 = cl + 1; cl2 < 4; ++cl2) {
              if (cl2 < w) {
                const double lc = lane_value(p[0][cl], cl2);
#pragma unroll
                for (int m = 0; m < 3; ++m)
                  p[m][cl2] = pick(lane + 64 * m >= cl2, p[m][cl2] - p[m][cl] * lc, p[m][cl2]);
              }
            }
          }
        }
        double* dum = misc + 7;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          if (c0 + 64 * m >= RZ) break;
          const int r = c0 + lane + 64 * m;
#pragma unroll
          for (int cl = 0; cl < 4; ++cl) {
            *(r < R && cl < w ? P + cl * R + r : dum) = p[m][cl];
            *(r < RZ ? Z + cl * RZ + r : dum) = pick(r >= c0 + w && r < R && cl < w, p[m][cl], 0.0);
          }
        }
        // rows of earlier panels of this block column
        const int rz = J * TS + lane;
#pragma unroll
        for (int cl = 0; cl < 4; ++cl) *(rz < c0 ? Z + cl * RZ + rz : dum) = 0.0;
        if (lane == 0) misc[0] = good ? 1.0 : 0.0;
      }
      __syncthreads();
      if (misc[0] == 0.0) return false;
      if (cl_own >= 0 && cl_own < w) {
        const int q = J * TS + tx;
#pragma unroll
        for (int I = J; I < NB; ++I) {
          const int r = I * TS + ty;
          if (r >= q && r < R) acc[I * (I + 1) / 2 + J] = (T)P[cl_own * R + r];
        }
      }
      for (int cl = 0; cl < w; ++cl) {
        T cr[NB], cq[NB];
#pragma unroll
        for (int I = J; I < NB; ++I) {
          cr[I] = (T)Z[cl * RZ + I * TS + ty];
          cq[I] = (T)Z[cl * RZ + I * TS + tx];
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
