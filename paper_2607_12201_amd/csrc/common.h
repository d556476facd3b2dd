// Internal structures shared by the host API and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CL_KMAX 5
#define CL_MAX_LS 48
#define CL_FILTER_CAP 128

// Shape class of a batch.  Local variable order inside an element: z[j][s] (b = (K+1) ns);
// the element's interior block I = nodes 0..K-1 (mI = K ns), its separator S = node K.
// Panel rows of the level-0 elimination: I (mI), S (ns), P = previous separator (ns),
// theta (np); R = mI + 2 ns + np rows, mI columns.
struct Shape {
  int ns, nr, np, K, b, mI, R, Rt;
  int lsp, lrq, lpc, mmax;      // longest per-instance lists (species->reactions, reactant
                                // slots, parameter->reactions) and most measurements per element
  int lnf, lct;                 // most nonzeros of F and longest column lists of Fth per
                                // instance (tiled path)
  int lzs, lzt;                 // most sparse-term groups and terms of the z columns per
                                // instance (tiled path)
  int big;                      // 1: tiled matrix-core factorization (large element blocks)
  double a[CL_KMAX + 1][CL_KMAX + 1];  // a[j][k] = l_j'(tau_k)
};

// Device tables (all pointers into the caller's table buffer).
struct Tab {
  double wclk_hz;             // rate of the device wall clock (wall_clock64), ticks per second
  int n_inst;
  int L;                      // cyclic-reduction levels (max over the batch)
  int64_t n_elem;
  const int* inst_N;
  const int64_t* inst_x;      // x offset per instance
  const int64_t* inst_g;      // g offset per instance
  const int64_t* inst_e0;     // first global element per instance
  const int* elem_inst;
  const int* elem_loc;
  const double* elem_h;
  const int* elem_mptr;       // [n_elem + 1] measurement CSR
  const int* meas_sp;
  const double* meas_w;       // [n_meas][K+1]  l_j(tau_m) / sigma_m
  const double* meas_ys;      // y_m / sigma_m
  const int* react;           // [n_inst][nr][2]
  const int* param;           // [n_inst][nr]
  const double* logk;         // [n_inst][nr] fixed natural-log rates (param == -1)
  const int* sp_ptr;          // [n_inst][ns + 1] absolute offsets into sp_r/sp_nu
  const int* sp_r;            // reactions with nu_sr != 0, per species
  const double* sp_nu;
  const int* rq_ptr;          // [n_inst][ns + 1] absolute offsets: reactant slots of species q
  const int* rq_r;            //   reaction of the slot
  const int* rq_t;            //   slot index (0/1)
  const int* pc_ptr;          // [n_inst][np + 1] absolute offsets: reactions using parameter c
  const int* pc_r;
  const int* rx_sp;           // [n_inst][nr][4] species with nu_sr != 0, -1 padded
  const double* rx_nu;        // [n_inst][nr][4]
  const double* z0;           // [n_inst][ns]
  const double* th_lo;        // [n_inst][np]
  const double* th_hi;
  const int* cr_ptr;          // [L + 1]  separators eliminated at level l (q 2^(l-1), q odd)
  const int* cr_inst;         // per work item of a cyclic-reduction level
  const int* cr_j;
  const int* st_ptr;          // [L]  step l (1..L-1): separators that are multiples of 2^l
  const int* st_inst;
  const int* st_s;
  // Nonzero pattern of the point Jacobians F_k (tiled assembly).  A pair q is one nonzero
  // (row s, column u) of F_k: F_k[s][u] = sum over the terms o in [fq_o[q], fq_o[q + 1]) of
  // cf_nu[o] d rho_(cf_r[o]) / d slot cf_t[o].  Pairs are stored by column (fq_ptr, rows fq_s,
  // each column's rows distinct) and indexed by row (fr_ptr; fr_q the pair relative to the
  // instance's first pair, fr_u its column).  Fth_k[s][c] is given by the column lists ct_*
  // with d rho_(ct_r[o]) / d theta.  Absolute offsets per instance.
  const int* fq_ptr;          // [n_inst][ns + 1]
  const int* fq_s;
  const int* fq_o;            // [n_pairs + 1]
  const int* fr_ptr;          // [n_inst][ns + 1]
  const int* fr_q;
  const int* fr_u;
  const int* cf_r;
  const int* cf_t;
  const double* cf_nu;
  const int* ct_ptr;          // [n_inst][np + 1]
  const int* ct_s;
  const int* ct_r;
  const double* ct_nu;
  // Sparse terms of the z columns (tiled assembly).  Species s's columns have the groups
  // [zs_ptr[s], zs_ptr[s + 1]); group g reaches row key zs_key[g] (< ns: that species at the
  // column's node; ns + th: parameter th) and sums the terms [zs_t[g], zs_t[g + 1]) of zt_code:
  // code >= 0 the ct entry code relative to the instance (-h sum_k a_jk Ds_(k,s) Fth_k[s][th]);
  // code < 0, x = -1 - code = 4 rr + 2 sl + kind: reaction rr with s in slot sl, its second
  // derivative in both slots (kind 0) or in slot sl and its parameter (kind 1).
  const int* zs_ptr;          // [n_inst][ns + 1]  absolute
  const int* zs_key;
  const int* zs_t;            // [n_groups + 1]  absolute
  const int* zt_code;
  int cr_items_max;           // largest level
};

// Workspace pointers (device).  Block data of type T (double or float) lives in void*.
struct Ws {
  int prec;                   // 0 fp64, 1 fp32
  void* panel;                // [n_elem][R*mI]  column-major, ld = R
  void* dss;                  // [n_elem][ns*ns] S-S block, then T-self Schur output
  void* bs;                   // [n_elem][ns*np] S-theta block, then G-self
  void* tprev;                // [n_elem][ns*ns]  contribution to the previous separator
  void* e1;                   // [n_elem][ns*ns]  coupling (S_i, S_{i-1})
  void* gprev;                // [n_elem][ns*np]
  void* lsep;                 // [n_elem][ns*ns]  separator factors (separator j = element j)
  void* ul;                   // [n_elem][ns*ns]
  void* ur;                   // [n_elem][ns*ns]
  void* ub;                   // [n_elem][ns*np]
  void* cTl;                  // [n_elem][ns*ns] Schur contributions of an eliminated separator:
  void* cTr;                  //   to its left / right neighbour's block,
  void* cE;                   //   the new coupling (right row, left column),
  void* cGl;                  //   [n_elem][ns*np] to the neighbours' borders
  void* cGr;
  double* dcont;              // [n_elem][ns]   continuity weight on the previous separator
  double* ath;                // [n_elem][np*np] element theta-theta block, then its Schur part
  double* thcr;               // [n_elem][np*np] theta-theta part from each separator
  double* S;                  // [n_inst][np*np] parameter Schur complement / its factor
  double* thred;              // [n_inst][nchunk][np*np] reduction partials
  int nchunk;                 // chunks per instance (max over the batch)
  double* thv;                // [n_inst][nchunk][np] theta right-hand-side chunk partials
  double* yI;                 // [n_elem][mI]
  double* cS;                 // [n_elem][ns]
  double* cP;                 // [n_elem][ns]
  double* cB;                 // [n_elem][np]
  double* ysep;               // [n_elem][ns]
  double* xsep;               // [n_elem][ns]
  double* rcur;               // [n_elem][ns] current right-hand side of surviving separators
  double* cBsep;              // [n_elem][np]
  double* rthp;               // [n_elem][np] right-hand-side theta partials
  double* xth;                // [n_inst][np]
  double* jac;                // derivative values used by assembly and the matvec
  double* hess;
  double* Ds;                 // [m_total] slack-block diagonal Ss + dw
  double* sxdw;               // [n_inst][np] Sx + dw on theta
  double* dw;                 // [n_inst]
  double* vtmp;               // [n_total] refinement residual / correction
  double* vtmp2;              // [n_total]
  double* epart;              // [n_elem][EP_N] element partial sums
  double* ipart;              // [n_inst][EP_N]
  int* flag;                  // [n_inst] factor failure flags
  int* irflag;                // [n_inst] refinement: 1 = instance done (converged / failed)
  int* ircount;               // [n_inst] refinement sweeps (negative: not converged)
  int* runskip;               // [n_inst] 1 = instance not iterating this step
  int* fbflag;                // [n_inst] FP64 fallback mask (0 = re-factor in FP64)
  int* fbneed;                // [n_inst] 1 = the instance re-factors in FP64 this step
  double* irpart;             // [n_elem][6] refinement partial maxima (|d|, |dx| after, |r|, |rhs|,
                              // |dx| before, row-sum bound of |K|)
  double* irnorm;             // [n_inst][2] refinement: row-sum bound of |K|, previous |d|
  // tiled path (Shape::big)
  void* ebuf;                 // [n_elem][Rp x Rp] element matrices / factors
  void* sbuf;                 // [n_elem][Lp x Lp] separator local matrices / factors
  double* bbuf;               // [n_inst][Bp x Bp] border matrices / factors (FP64)
  double* evec;               // [n_elem][Rp] element forward vectors
  double* svec;               // [n_elem][Lp] separator forward vectors
  double* linv;               // [n_elem][32 x 32] inverse diagonal factors of the current panel
};

// Element partial-sum slots (colloc_eval and the interior-point reductions).
enum {
  EP_OBJ = 0,     // sum of r_m^2 / 2
  EP_L1PR,        // sum |g - s|
  EP_INFPR,       // max |g - s|
  EP_INFDU,       // max |grad_z L| and |grad_s L|
  EP_L1Y,         // sum |y|
  EP_L1V,         // sum |vL| + |vU|
  EP_CMAX, EP_CMIN,  // complementarity max/min over slack bounds
  EP_LOGS,        // sum log(s + tau) + log(tau - s)
  EP_NONFIN,      // nonzero when a non-finite value was seen
  EP_FTB_P,       // min primal step ratio
  EP_FTB_D,       // min dual step ratio
  EP_DPHI,        // directional derivative partial
  EP_N
};

__host__ __device__ inline int64_t cl_ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Elements per partial of the parameter Schur reduction.  Fixed, so an instance's summation
// order depends on its own N only (same result alone and inside any batch).
#define CL_THCHUNK 16
