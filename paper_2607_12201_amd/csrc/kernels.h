// Host-side launch wrappers of the gfx950 kernels (defined in the k_*.hip files).
#pragma once
#include "common.h"

namespace cl {

// Host copy of the static work-list sizes (grid sizes of the cyclic-reduction levels).
struct HostPlan {
  int L;
  int lvl[64];   // lvl[l] = separators eliminated at level l (1..L)
  int st[64];    // st[l] = work items of cyclic-reduction step l (1..L-1)
  int ts[3];     // thread grid of the element / chain / border kernels (0 = built-in rule)
};

// Workgroup size of the per-element kernels: one wave for tiny elements, four otherwise.
inline int elem_threads(const Shape& S) {
  int w = S.b + S.np;
  return w <= 32 ? 64 : (w <= 96 ? 128 : 256);
}
size_t sep_solve_lds(const Shape& S);      // separator-chain solve kernels
size_t border_solve_lds(const Shape& S);   // border solve kernel
// Theta partials of each instance over 16-element chunks (a + [i > 0] b - d, b and d optional).
void launch_thpart(const Shape& S, const Tab& tb, const Ws& ws, const double* a, const double* b,
                   const double* d, double* out, hipStream_t st);

int launch_eval(const Shape& S, const Tab& tb, const Ws& ws, const double* x, double* obj,
                double* g, hipStream_t st);
int launch_derivs(const Shape& S, const Tab& tb, const double* x, const double* y, double* grad,
                  double* jac, double* hess, hipStream_t st);

// KKT assembly / factor / solve.  Phases that the timing hooks bracket are reported through
// the callback (phase id, begin=1/end=0).
typedef void (*phase_cb)(void* ctx, int phase, int begin, hipStream_t st);

size_t level0_lds_bytes(const Shape& S, int prec);        // kkt_assemble's LDS blocks
size_t level0r_lds_bytes(const Shape& S);
size_t chain_lds_bytes(const Shape& S, int which);   // which: 1 chain levels, 2 border
bool level0r_supported(const Shape& S);
int launch_level0(const Shape& S, const Tab& tb, const Ws& ws, int prec, bool fused, int ts,
                  hipStream_t st);
int level0_prepare_attrs(const Shape& S);
int launch_chain(const Shape& S, const Tab& tb, const Ws& ws, int prec, int mode, int level,
                 unsigned grid, int ts, hipStream_t st);
// Thread-grid options of the element (which = 0), chain (1) and border (2) kernels for a shape.
int tile_options(const Shape& S, int which, int* ts, int cap);
bool tile_valid(const Shape& S, int which, int ts);
int launch_assemble(const Shape& S, const Tab& tb, const Ws& ws, const double* jac,
                    const double* hess, const double* sigma_x, const double* sigma_s,
                    const double* delta_w, const double* r_x, const double* r_s,
                    const double* r_y, double* rhs, hipStream_t st);
// launch_factor clears the per-instance flags first; launch_factor_nc keeps them (instances
// whose flag is set are skipped).
int launch_factor(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, int prec,
                  bool fused, phase_cb cb, void* ctx, hipStream_t st);
int launch_factor_nc(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, int prec,
                     bool fused, phase_cb cb, void* ctx, hipStream_t st);
// rthp: optional per-element theta partials added to the theta right-hand side.
int launch_solve_p(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws,
                   const double* rhs, const double* rthp, double* dx, phase_cb cb, void* ctx,
                   hipStream_t st);
// FP64 iterative refinement of dx against rhs with the current factor (ws.prec), masked per
// instance by the factor flags; ws.ircount receives the sweep counts.
int launch_refine(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, const double* rhs,
                  double* dx, int ir_max, double ir_tol, phase_cb cb, void* ctx, hipStream_t st);
int launch_refine_report(const Tab& tb, const Ws& ws, int* ir_sweeps, hipStream_t st);
int launch_matvec(const Shape& S, const Tab& tb, const Ws& ws, const double* v, double* out,
                  hipStream_t st);
int launch_copy_flags(const Tab& tb, const Ws& ws, int* info, hipStream_t st);

// Tiled matrix-core path (Shape::big), k_big.hip.
int launch_factor_big(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, int prec,
                      phase_cb cb, void* ctx, hipStream_t st);
int launch_solve_big(const Shape& S, const Tab& tb, const HostPlan& hp, const Ws& ws, const double* rhs,
                     const double* rthp, double* dx, phase_cb cb, void* ctx, hipStream_t st);
size_t big_asm_lds(const Shape& S);
size_t big_solve_lds(const Shape& S);
int big_prepare_attrs(const Shape& S);


// collocation-consistent states at fixed parameters (k_init.hip); -2: K ns above the LDS limit
int launch_fwd_init(const Shape& S, const Tab& tb, const double* theta, double* x, int* status,
                    hipStream_t st);

}  // namespace cl
