// Interior-point state (device pointers into the caller's state buffer) and launches.
#pragma once
#include "../../include/colloc.h"
#include "kernels.h"

namespace cl {

enum { PH_EVAL = 0, PH_RETRY = 1 };

struct IpmState {
  double *x, *s, *y, *vL, *vU, *zL, *zU;
  double *dx, *ds, *dy, *dvL, *dvU, *dzL, *dzU;
  double *g, *grad, *rhs;
  double *fth, *fph;         // [n_inst][CL_FILTER_CAP] filter entries
  double *tpart;             // [n_elem][CL_MAX_LS][3] line-search candidate partials
  colloc_ipm_info* info;     // [n_inst]
};

int launch_ipm_init(const Shape& S, const Tab& tb, const IpmState& st, const Ws& ws,
                    const double* x0, const colloc_ipm_opts& o, hipStream_t s);
// ws64: the FP64 layout of the same workspace (the FP32_IR fallback), unused in FP64 mode.
int launch_ipm_step(const Shape& S, const Tab& tb, const HostPlan& hp, const IpmState& st,
                    const Ws& ws, const Ws& ws64, const colloc_ipm_opts& o, phase_cb cb, void* ctx,
                    hipStream_t s);

}  // namespace cl
