// Tiled factorization for element blocks too large to live in registers (the 100-species,
// 200-parameter class: 700-row element matrices).  Shared declarations of the tiled kernels.
//
// Storage (workspace, all column-major):
//   ebuf  [n_elem][Rp x Rp]  element matrix over [z (b) | theta (np) | P (ns)], lower triangle;
//                            after the factorization its first mI columns hold L (the interior
//                            block's Cholesky factor and the transformed rows below it) and the
//                            trailing block the Schur complement on (S, theta, P) except the
//                            theta-theta part
//   sbuf  [n_elem][Lp x Lp]  separator s's local matrix over [s | left | right | theta]; its
//                            first ns columns hold [T_s; E_L; E_R; G_s] before and the factor
//                            after elimination, the trailing block the contributions -X X^T
//   bbuf  [n_inst][Bp x Bp]  FP64 border matrix over [separator 0 | theta]
//   ath   [n_elem][np x np]  FP64 assembled theta-theta block of every element
// The theta-theta Schur complement is formed separately in FP64 on matrix cores from the
// transformed theta rows of every element and separator (k_big_theta).
#pragma once
#include "common.h"

namespace cl {

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 matrix-core product accumulate.  Operands per lane l: a = A[l % 16][l / 16]
// (A is 16 x 4), b = B[l / 16][l % 16] (B is 4 x 16).  Result element v of lane l is D[row][col]
// with col = l % 16 and row given by row(l, v): the FP64 instruction interleaves rows
// (l / 16 + 4 v), the FP32 one keeps them in blocks (4 (l / 16) + v).
template <typename T>
struct Mma;
template <>
struct Mma<double> {
  typedef dvec4 acc;
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mma<float> {
  typedef fvec4 acc;
  __device__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// Geometry of the tiled path for a shape class.
struct BigGeom {
  int R, Rp;      // element rows and padded leading dimension
  int Lr, Lp;     // separator local rows (3 ns + np) and padded leading dimension
  int Br, Bp;     // border rows (ns + np) and padded leading dimension
};

__host__ __device__ inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

__host__ __device__ inline BigGeom big_geom(const Shape& S) {
  BigGeom g;
  g.R = S.R;
  g.Rp = round_up(S.R, 32);
  g.Lr = 3 * S.ns + S.np;
  g.Lp = round_up(g.Lr, 32);
  g.Br = S.ns + S.np;
  g.Bp = round_up(g.Br, 32);
  return g;
}

}  // namespace cl
