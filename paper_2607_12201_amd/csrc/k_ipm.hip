// a6: interior-point iteration on the device (filter line-search method on the relaxed
// equality form g(x) - s = 0, -tau_r <= s <= tau_r, theta bounds).  Per element kernels write
// partial sums with fixed-order block reductions; one workgroup per instance takes the
// scalar decisions (convergence, barrier update, inertia correction, line-search acceptance).
// The backtracking candidates alpha_max 2^-t are evaluated in parallel and the first
// acceptable one in order is taken, which is the sequential backtracking result.
#include "ipm.h"
#include "elem.h"

namespace cl {

__device__ inline bool running(const IpmState& st, int inst) {
  return st.info[inst].status == COLLOC_RUNNING;
}

// ---------------------------------------------------------------- init
__global__ void k_init_theta(Shape S, Tab tb, IpmState st, const double* __restrict__ x0,
                             colloc_ipm_opts o) {
  const int inst = blockIdx.x;
  const int N = tb.inst_N[inst];
  const int64_t xo = tb.inst_x[inst];
  const int64_t nzi = (int64_t)N * S.b;
  for (int64_t t = tid(); t < nzi; t += nthr()) st.x[xo + t] = x0[xo + t];
  for (int c = tid(); c < S.np; c += nthr()) {
    double lo = tb.th_lo[inst * S.np + c], hi = tb.th_hi[inst * S.np + c];
    double pl = fmin(o.bound_push * fmax(1.0, fabs(lo)), o.bound_frac * (hi - lo));
    double pu = fmin(o.bound_push * fmax(1.0, fabs(hi)), o.bound_frac * (hi - lo));
    double v = x0[xo + nzi + c];
    st.x[xo + nzi + c] = fmin(fmax(v, lo + pl), hi - pu);
    st.zL[inst * S.np + c] = 1.0;
    st.zU[inst * S.np + c] = 1.0;
  }
}

__global__ void k_init_elem(Shape S, Tab tb, IpmState st, Ws ws, colloc_ipm_opts o) {
  __shared__ double red[256];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * S.b;
  const double tr = o.tau_r;
  const double pl = fmin(o.bound_push * fmax(1.0, tr), o.bound_frac * 2.0 * tr);
  double l1 = 0.0;
  for (int t = tid(); t < S.b; t += nthr()) {
    double g = st.g[gi + t];
    double s = fmin(fmax(g, -tr + pl), tr - pl);
    st.s[gi + t] = s;
    st.y[gi + t] = 0.0;
    st.vL[gi + t] = 1.0;
    st.vU[gi + t] = 1.0;
    l1 += fabs(g - s);
  }
  l1 = block_sum(l1, red);
  if (tid() == 0) ws.epart[e * EP_N + EP_L1PR] = l1;
}

__global__ void k_init_inst(Shape S, Tab tb, IpmState st, Ws ws, colloc_ipm_opts o) {
  __shared__ double red[256];
  const int inst = blockIdx.x;
  const int N = tb.inst_N[inst];
  const int64_t e0 = tb.inst_e0[inst];
  double acc = 0.0;
  for (int t = tid(); t < N; t += nthr()) acc += ws.epart[(e0 + t) * EP_N + EP_L1PR];
  acc = block_sum(acc, red);
  if (tid() == 0) {
    colloc_ipm_info I;
    memset(&I, 0, sizeof(I));
    I.status = COLLOC_RUNNING;
    I.phase = PH_EVAL;
    I.mu = o.mu_init;
    I.tau = fmax(o.tau_min, 1.0 - o.mu_init);
    I.theta_max = 1e4 * fmax(1.0, acc);
    I.theta_min = 1e-4 * fmax(1.0, acc);
    I.filter_len = 1;
    I.t_start = (double)wall_clock64() / tb.wclk_hz;
    st.info[inst] = I;
    st.fth[inst * CL_FILTER_CAP] = I.theta_max;
    st.fph[inst * CL_FILTER_CAP] = -INFINITY;
  }
}

// ---------------------------------------------------------------- evaluation
// LDS: z b, th np, kap nr, rho/d0/d1 3 K nr, yl b, yn ns, phi K nr, gz b, jz b, jt np, zp ns, red nt
__global__ void __launch_bounds__(256) k_ipm_eval(Shape S, Tab tb, IpmState st, Ws ws,
                                                  colloc_ipm_opts o) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (!running(st, inst) || st.info[inst].phase != PH_EVAL) return;
  const int N = tb.inst_N[inst];
  const int ns = S.ns, nr = S.nr, b = S.b, np = S.np, K = S.K;
  const double h = tb.elem_h[e];
  const int64_t xo = tb.inst_x[inst];
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  double* z = lds;
  double* th = z + b;
  double* kap = th + np;
  double* rho = kap + nr;
  double* d0 = rho + K * nr;
  double* d1 = d0 + K * nr;
  double* yl = d1 + K * nr;
  double* yn = yl + b;
  double* phi = yn + ns;
  double* gz = phi + K * nr;
  double* jz = gz + b;
  double* jt = jz + b;
  double* zp = jt + np;
  double* gl = zp + ns;
  double* red = gl + b;
  for (int t = tid(); t < b; t += nthr()) {
    z[t] = st.x[xo + (int64_t)i * b + t];
    yl[t] = st.y[gi + t];
  }
  for (int t = tid(); t < np; t += nthr()) th[t] = st.x[xo + (int64_t)N * b + t];
  if (i > 0)
    for (int t = tid(); t < ns; t += nthr()) zp[t] = st.x[xo + (int64_t)(i - 1) * b + K * ns + t];
  if (i + 1 < N)
    for (int t = tid(); t < ns; t += nthr()) yn[t] = st.y[gi + b + t];
  __syncthreads();
  load_kappa(S, tb, inst, th, kap);
  __syncthreads();
  rates(S, tb, inst, z, kap, rho, d0, d1);
  reaction_weights(S, tb, inst, yl, phi);
  double phi_obj = obj_element(S, tb, e, z, gz);
  __syncthreads();
  residual_rows(S, tb, inst, i, h, z, zp, rho, gl);
  // derivative values
  const int64_t jl = (int64_t)K * nr;
  double* je = ws.jac + e * jl * 3;
  double* he = ws.hess + e * jl * 4;
  for (int t = tid(); t < K * nr; t += nthr()) {
    int r = t % nr;
    int c = tb.param[inst * nr + r];
    int q0 = tb.react[(inst * nr + r) * 2], q1 = tb.react[(inst * nr + r) * 2 + 1];
    double w = -h * phi[t];
    double par = c >= 0 ? 1.0 : 0.0;
    je[t * 3 + 0] = d0[t];
    je[t * 3 + 1] = d1[t];
    je[t * 3 + 2] = rho[t] * par;
    he[t * 4 + 0] = (q0 >= 0 && q1 >= 0) ? w * kap[r] : 0.0;
    he[t * 4 + 1] = w * d0[t] * par;
    he[t * 4 + 2] = w * d1[t] * par;
    he[t * 4 + 3] = w * rho[t] * par;
  }
  __syncthreads();
  jtu_rows(S, tb, inst, h, je, yl, (i + 1 < N) ? yn : nullptr, phi, jz, jt);
  __syncthreads();
  // partial sums
  const double tr = o.tau_r;
  double l1pr = 0, infpr = 0, infdu = 0, l1y = 0, l1v = 0, cmax = -INFINITY, cmin = INFINITY, lg = 0;
  double nonfin = 0.0;
  for (int t = tid(); t < b; t += nthr()) {
    double g = gl[t], s = st.s[gi + t], y = yl[t], vl = st.vL[gi + t], vu = st.vU[gi + t];
    st.g[gi + t] = g;
    st.grad[xo + (int64_t)i * b + t] = gz[t];
    double rp = g - s;
    l1pr += fabs(rp);
    infpr = fmax(infpr, fabs(rp));
    double rx = gz[t] + jz[t];
    double rs = -y - vl + vu;
    infdu = fmax(infdu, fmax(fabs(rx), fabs(rs)));
    l1y += fabs(y);
    l1v += fabs(vl) + fabs(vu);
    double sl = s + tr, su = tr - s;
    double c1 = sl * vl, c2 = su * vu;
    cmax = fmax(cmax, fmax(c1, c2));
    cmin = fmin(cmin, fmin(c1, c2));
    lg += log(sl) + log(su);
    if (!isfinite(g) || !isfinite(rx)) nonfin = 1.0;
  }
  for (int c = tid(); c < np; c += nthr()) ws.rthp[e * np + c] = jt[c];
  if (i == 0)
    for (int c = tid(); c < np; c += nthr()) st.grad[xo + (int64_t)N * b + c] = 0.0;
  double v;
  v = block_sum(l1pr, red); if (tid() == 0) ws.epart[e * EP_N + EP_L1PR] = v;
  v = block_max(infpr, red); if (tid() == 0) ws.epart[e * EP_N + EP_INFPR] = v;
  v = block_max(infdu, red); if (tid() == 0) ws.epart[e * EP_N + EP_INFDU] = v;
  v = block_sum(l1y, red); if (tid() == 0) ws.epart[e * EP_N + EP_L1Y] = v;
  v = block_sum(l1v, red); if (tid() == 0) ws.epart[e * EP_N + EP_L1V] = v;
  v = block_max(cmax, red); if (tid() == 0) ws.epart[e * EP_N + EP_CMAX] = v;
  v = block_min(cmin, red); if (tid() == 0) ws.epart[e * EP_N + EP_CMIN] = v;
  v = block_sum(lg, red); if (tid() == 0) ws.epart[e * EP_N + EP_LOGS] = v;
  v = block_max(nonfin, red); if (tid() == 0) ws.epart[e * EP_N + EP_NONFIN] = v;
  if (tid() == 0) ws.epart[e * EP_N + EP_OBJ] = phi_obj;
}

// Per-instance decisions after evaluation: optimality error, termination, barrier update,
// inertia-correction schedule.  One workgroup per instance.
__global__ void __launch_bounds__(1024) k_ipm_decide(Shape S, Tab tb, IpmState st, Ws ws,
                                                     colloc_ipm_opts o) {
  __shared__ double red[1024];
  __shared__ double sh[16];
  extern __shared__ double jty[];   // np
  const int inst = blockIdx.x;
  colloc_ipm_info I = st.info[inst];
  if (I.status != COLLOC_RUNNING) {
    if (tid() == 0) ws.flag[inst] = 1;
    return;
  }
  const int N = tb.inst_N[inst], np = S.np, b = S.b;
  const int64_t e0 = tb.inst_e0[inst];
  const int64_t xo = tb.inst_x[inst] + (int64_t)N * b;
  const double* th = st.x + xo;
  const double* lo = tb.th_lo + inst * np;
  const double* hi = tb.th_hi + inst * np;
  const double* zL = st.zL + inst * np;
  const double* zU = st.zU + inst * np;
  if (I.phase == PH_EVAL) {
    double s_obj = 0, s_l1pr = 0, s_l1y = 0, s_l1v = 0, s_logs = 0;
    double m_infpr = 0, m_infdu = 0, m_cmax = -INFINITY, m_cmin = INFINITY, m_nf = 0;
    for (int t = tid(); t < N; t += nthr()) {
      const double* p = ws.epart + (e0 + t) * EP_N;
      s_obj += p[EP_OBJ];
      s_l1pr += p[EP_L1PR];
      s_l1y += p[EP_L1Y];
      s_l1v += p[EP_L1V];
      s_logs += p[EP_LOGS];
      m_infpr = fmax(m_infpr, p[EP_INFPR]);
      m_infdu = fmax(m_infdu, p[EP_INFDU]);
      m_cmax = fmax(m_cmax, p[EP_CMAX]);
      m_cmin = fmin(m_cmin, p[EP_CMIN]);
      m_nf = fmax(m_nf, p[EP_NONFIN]);
    }
    // theta part: dual residual, complementarity, bound-multiplier norms, barrier logs
    theta_sum(ws.rthp, e0, N, np, jty, red);
    double du_t = 0.0, l1z = 0.0, cmx = -INFINITY, cmn = INFINITY, lgt = 0.0;
    for (int c = tid(); c < np; c += nthr()) {
      double rx = jty[c] - zL[c] + zU[c];
      du_t = fmax(du_t, fabs(rx));
      l1z += fabs(zL[c]) + fabs(zU[c]);
      double tl = th[c] - lo[c], tu = hi[c] - th[c];
      cmx = fmax(cmx, fmax(tl * zL[c], tu * zU[c]));
      cmn = fmin(cmn, fmin(tl * zL[c], tu * zU[c]));
      lgt += log(tl) + log(tu);
      if (!isfinite(rx)) m_nf = 1.0;
    }
    double v[12] = {s_obj, s_l1pr, s_l1y, s_l1v, s_logs, l1z, lgt,
                    m_infpr, fmax(m_infdu, du_t), fmax(m_cmax, cmx), m_nf, fmin(m_cmin, cmn)};
    block_reduce_multi<7, 4, 1>(v, red);
    s_obj = v[0];
    s_l1pr = v[1];
    s_l1y = v[2];
    s_l1v = v[3];
    s_logs = v[4];
    l1z = v[5];
    lgt = v[6];
    m_infpr = v[7];
    m_infdu = v[8];
    m_cmax = v[9];
    m_nf = v[10];
    m_cmin = v[11];
    if (tid() == 0) {
      const int m = N * b;
      double l1all = s_l1y + s_l1v + l1z;
      double sd = fmax(o.s_max, l1all / (double)(m + 2 * np + 2 * m)) / o.s_max;
      double sc = fmax(o.s_max, (s_l1v + l1z) / (double)(2 * np + 2 * m)) / o.s_max;
      auto E = [&](double mu) {
        return fmax(fmax(m_infdu / sd, m_infpr), fmax(m_cmax - mu, mu - m_cmin) / sc);
      };
      double E0 = E(0.0);
      I.E0 = E0;
      I.obj = s_obj;
      I.inf_pr = m_infpr;
      I.inf_du = m_infdu;
      I.s_d = sd;
      I.s_c = sc;
      I.theta_cv = s_l1pr;
      int stt = COLLOC_RUNNING;
      if (!isfinite(E0) || m_nf != 0.0) stt = COLLOC_ENONFINITE;
      else if (E0 <= o.tol) stt = COLLOC_SOLVED;
      else {
        I.acc_count = (E0 <= o.acceptable_tol) ? I.acc_count + 1 : 0;
        if (I.acc_count >= o.acceptable_iter) stt = COLLOC_ACCEPTABLE;
        else if (I.iter >= o.max_iter) stt = COLLOC_MAXITER;
        else if (o.max_wall_s > 0.0 && (double)wall_clock64() / tb.wclk_hz - I.t_start > o.max_wall_s)
          stt = COLLOC_TIMEOUT;
      }
      I.status = stt;
      if (stt == COLLOC_RUNNING) {
        while (E(I.mu) <= o.kappa_eps * I.mu) {
          double nm = fmax(o.tol / 10.0, fmin(o.kappa_mu * I.mu, pow(I.mu, o.theta_mu)));
          if (nm >= I.mu) break;
          I.mu = nm;
          I.filter_len = 1;
          st.fth[inst * CL_FILTER_CAP] = I.theta_max;
          st.fph[inst * CL_FILTER_CAP] = -INFINITY;
        }
        I.Emu = E(I.mu);
        I.tau = fmax(o.tau_min, 1.0 - I.mu);
        I.phi = s_obj - I.mu * (s_logs + lgt);
        I.delta_w = 0.0;
        I.factor_tries = 1;
      }
      sh[0] = (stt == COLLOC_RUNNING) ? 1.0 : 0.0;
      sh[1] = I.mu;
      sh[2] = I.delta_w;
    }
  } else {  // PH_RETRY: the last factorization was not positive definite
    if (tid() == 0) {
      double dw = I.delta_w;
      if (dw == 0.0)
        dw = (I.delta_last == 0.0) ? o.delta_w0 : fmax(o.delta_min, o.kappa_w_minus * I.delta_last);
      else
        dw *= (I.delta_last == 0.0) ? o.kappa_w_plus_bar : o.kappa_w_plus;
      I.delta_w = dw;
      I.factor_tries += 1;
      if (dw > o.delta_max) I.status = COLLOC_ENOTPD;
      sh[0] = (I.status == COLLOC_RUNNING) ? 1.0 : 0.0;
      sh[1] = I.mu;
      sh[2] = I.delta_w;
    }
  }
  __syncthreads();
  const bool go = sh[0] != 0.0;
  if (tid() == 0) {
    st.info[inst] = I;
    ws.flag[inst] = go ? 0 : 1;
    ws.dw[inst] = I.delta_w;
  }
  if (!go) return;
  // Sx + dw on theta, theta rhs base (barrier terms of -r_x(theta))
  const double mu = sh[1], dw = sh[2];
  for (int c = tid(); c < np; c += nthr()) {
    double tl = th[c] - lo[c], tu = hi[c] - th[c];
    ws.sxdw[inst * np + c] = zL[c] / tl + zU[c] / tu + dw;
    st.rhs[xo + c] = mu / tl - mu / tu;
  }
}

// Ds = Ss + dw and the condensed right-hand side (z part; theta partials to rthp):
//   rhs = -grad Phi - J^T u,  u = Ds (g - s) - mu/(s + tau_r) + mu/(tau_r - s)
__global__ void __launch_bounds__(256) k_ipm_prep(Shape S, Tab tb, IpmState st, Ws ws,
                                                  colloc_ipm_opts o) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const int N = tb.inst_N[inst];
  const int ns = S.ns, b = S.b, np = S.np;
  const int64_t xo = tb.inst_x[inst];
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  const double mu = st.info[inst].mu, dw = ws.dw[inst], tr = o.tau_r;
  double* u = lds;
  double* un = u + b;
  double* phi = un + ns;
  double* oz = phi + S.K * S.nr;
  double* ot = oz + b;
  for (int t = tid(); t < b + ((i + 1 < N) ? ns : 0); t += nthr()) {
    double s = st.s[gi + t], vl = st.vL[gi + t], vu = st.vU[gi + t];
    double sl = s + tr, su = tr - s;
    double Ds = vl / sl + vu / su + dw;
    double uu = Ds * (st.g[gi + t] - s) - mu / sl + mu / su;
    if (t < b) {
      u[t] = uu;
      ws.Ds[gi + t] = Ds;
    } else {
      un[t - b] = uu;
    }
  }
  __syncthreads();
  reaction_weights(S, tb, inst, u, phi);
  __syncthreads();
  const int64_t jl = (int64_t)S.K * S.nr;
  jtu_rows(S, tb, inst, tb.elem_h[e], ws.jac + e * jl * 3, u, (i + 1 < N) ? un : nullptr, phi, oz, ot);
  __syncthreads();
  for (int t = tid(); t < b; t += nthr())
    st.rhs[xo + (int64_t)i * b + t] = -st.grad[xo + (int64_t)i * b + t] - oz[t];
  for (int c = tid(); c < np; c += nthr()) ws.rthp[e * np + c] = -ot[c];
}

// Step recovery on the rows: ds = J dx + g - s, dy = Ds ds + rs, dvL, dvU; fraction-to-boundary
// and directional-derivative partials.  LDS: v b, vp ns, vt np, jv b, red nt
__global__ void __launch_bounds__(256) k_ipm_dir(Shape S, Tab tb, IpmState st, Ws ws,
                                                 colloc_ipm_opts o) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const int N = tb.inst_N[inst];
  const int ns = S.ns, b = S.b, np = S.np;
  const int64_t xo = tb.inst_x[inst];
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  double* v = lds;
  double* vp = v + b;
  double* vt = vp + ns;
  double* jv = vt + np;
  double* red = jv + b;
  for (int t = tid(); t < b; t += nthr()) v[t] = st.dx[xo + (int64_t)i * b + t];
  if (i > 0)
    for (int t = tid(); t < ns; t += nthr()) vp[t] = st.dx[xo + (int64_t)(i - 1) * b + S.K * ns + t];
  for (int t = tid(); t < np; t += nthr()) vt[t] = st.dx[xo + (int64_t)N * b + t];
  __syncthreads();
  const int64_t jl = (int64_t)S.K * S.nr;
  jv_rows(S, tb, inst, i, tb.elem_h[e], ws.jac + e * jl * 3, v, vp, vt, jv);
  __syncthreads();
  const double mu = st.info[inst].mu, tau = st.info[inst].tau, tr = o.tau_r;
  double ftbp = 1.0, ftbd = 1.0, dphi = 0.0;
  for (int t = tid(); t < b; t += nthr()) {
    double s = st.s[gi + t], vl = st.vL[gi + t], vu = st.vU[gi + t], y = st.y[gi + t];
    double sl = s + tr, su = tr - s;
    double ds = jv[t] + st.g[gi + t] - s;
    double rs = -y - mu / sl + mu / su;
    double dy = ws.Ds[gi + t] * ds + rs;
    double dvl = mu / sl - vl - (vl / sl) * ds;
    double dvu = mu / su - vu + (vu / su) * ds;
    st.ds[gi + t] = ds;
    st.dy[gi + t] = dy;
    st.dvL[gi + t] = dvl;
    st.dvU[gi + t] = dvu;
    if (ds < 0) ftbp = fmin(ftbp, -tau * sl / ds);
    if (ds > 0) ftbp = fmin(ftbp, tau * su / ds);
    if (dvl < 0) ftbd = fmin(ftbd, -tau * vl / dvl);
    if (dvu < 0) ftbd = fmin(ftbd, -tau * vu / dvu);
    dphi += st.grad[xo + (int64_t)i * b + t] * v[t] - mu * ds / sl + mu * ds / su;
  }
  double r;
  r = block_min(ftbp, red); if (tid() == 0) ws.epart[e * EP_N + EP_FTB_P] = r;
  r = block_min(ftbd, red); if (tid() == 0) ws.epart[e * EP_N + EP_FTB_D] = r;
  r = block_sum(dphi, red); if (tid() == 0) ws.epart[e * EP_N + EP_DPHI] = r;
}

// Per instance: theta bound-multiplier steps, step sizes, alpha_min.
__global__ void k_ipm_steplen(Shape S, Tab tb, IpmState st, Ws ws, colloc_ipm_opts o) {
  __shared__ double red[256];
  const int inst = blockIdx.x;
  if (block_flag(&ws.flag[inst])) return;
  colloc_ipm_info I = st.info[inst];
  const int N = tb.inst_N[inst], np = S.np, b = S.b;
  const int64_t e0 = tb.inst_e0[inst];
  const int64_t xo = tb.inst_x[inst] + (int64_t)N * b;
  const double mu = I.mu, tau = I.tau;
  double ap = 1.0, ad = 1.0, dphi = 0.0;
  for (int t = tid(); t < N; t += nthr()) {
    const double* p = ws.epart + (e0 + t) * EP_N;
    ap = fmin(ap, p[EP_FTB_P]);
    ad = fmin(ad, p[EP_FTB_D]);
    dphi += p[EP_DPHI];
  }
  double dphit = 0.0;
  for (int c = tid(); c < np; c += nthr()) {
    double th = st.x[xo + c], dth = st.dx[xo + c];
    double lo = tb.th_lo[inst * np + c], hi = tb.th_hi[inst * np + c];
    double tl = th - lo, tu = hi - th;
    double zl = st.zL[inst * np + c], zu = st.zU[inst * np + c];
    double dzl = mu / tl - zl - (zl / tl) * dth;
    double dzu = mu / tu - zu + (zu / tu) * dth;
    st.dzL[inst * np + c] = dzl;
    st.dzU[inst * np + c] = dzu;
    if (dth < 0) ap = fmin(ap, -tau * tl / dth);
    if (dth > 0) ap = fmin(ap, tau * tu / dth);
    if (dzl < 0) ad = fmin(ad, -tau * zl / dzl);
    if (dzu < 0) ad = fmin(ad, -tau * zu / dzu);
    dphit += -mu * dth / tl + mu * dth / tu;
  }
  ap = block_min(ap, red);
  ad = block_min(ad, red);
  dphi = block_sum(dphi, red);
  dphit = block_sum(dphit, red);
  if (tid() == 0) {
    double dp = dphi + dphit;
    double thc = I.theta_cv;
    double amin;
    if (dp < 0) {
      amin = fmin(o.gamma_theta, o.gamma_phi * thc / (-dp));
      if (thc <= I.theta_min) amin = fmin(amin, o.delta_sw * pow(thc, o.s_theta) / pow(-dp, o.s_phi));
    } else {
      amin = o.gamma_theta;
    }
    I.alpha_min = amin * o.gamma_alpha;
    I.alpha_pr = ap;
    I.alpha_du = ad;
    I.dphi = dp;
    st.info[inst] = I;
  }
}

// Trial evaluations: thread t of the workgroup evaluates candidate alpha_max 2^-t on the
// element's rows (constraint violation, objective, slack barrier logs).  LDS: z,dz (b each),
// zp,dzp (ns), th,dth (np), kap? (recomputed per thread from theta trial: np exps per thread)
__global__ void __launch_bounds__(1024) k_ipm_trial(Shape S, Tab tb, IpmState st, Ws ws,
                                                   colloc_ipm_opts o) {
  extern __shared__ double lds[];
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const int N = tb.inst_N[inst];
  const int ns = S.ns, b = S.b, np = S.np, nr = S.nr, K = S.K;
  const int nls = o.max_ls;
  const int64_t xo = tb.inst_x[inst];
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  double* z = lds;
  double* dz = z + b;
  double* zp = dz + b;
  double* dzp = zp + ns;
  double* th = dzp + ns;
  double* dth = th + np;
  double* sv = dth + np;
  double* dsv = sv + b;
  double* kap = dsv + b;              // [nls][nr] rate constants at the trial parameters
  double* part = kap + nls * nr;      // [3][nthr] per-thread partial sums
  double* spnu = part + 3 * nthr();   // the instance's species -> reaction lists (S.lsp)
  int* spp = (int*)(spnu + S.lsp);    // [ns + 1] relative offsets
  int* spr = spp + ns + 1;            // [S.lsp]
  int* rea = spr + S.lsp;             // [nr][2] reactant slots
  {
    const int q0 = tb.sp_ptr[inst * (ns + 1)], nq = tb.sp_ptr[inst * (ns + 1) + ns] - q0;
    for (int t = tid(); t <= ns; t += nthr()) spp[t] = tb.sp_ptr[inst * (ns + 1) + t] - q0;
    for (int t = tid(); t < nq; t += nthr()) {
      spr[t] = tb.sp_r[q0 + t];
      spnu[t] = tb.sp_nu[q0 + t];
    }
    for (int t = tid(); t < 2 * nr; t += nthr()) rea[t] = tb.react[inst * nr * 2 + t];
  }
  for (int t = tid(); t < b; t += nthr()) {
    z[t] = st.x[xo + (int64_t)i * b + t];
    dz[t] = st.dx[xo + (int64_t)i * b + t];
    sv[t] = st.s[gi + t];
    dsv[t] = st.ds[gi + t];
  }
  if (i > 0)
    for (int t = tid(); t < ns; t += nthr()) {
      zp[t] = st.x[xo + (int64_t)(i - 1) * b + K * ns + t];
      dzp[t] = st.dx[xo + (int64_t)(i - 1) * b + K * ns + t];
    }
  for (int t = tid(); t < np; t += nthr()) {
    th[t] = st.x[xo + (int64_t)N * b + t];
    dth[t] = st.dx[xo + (int64_t)N * b + t];
  }
  const double alpha0 = st.info[inst].alpha_pr;
  __syncthreads();
  // candidate c: alpha_max 2^-c
  for (int t = tid(); t < nls * nr; t += nthr()) {
    const int c = t / nr, r = t - c * nr;
    const double alpha = ldexp(alpha0, -c);
    const int pc = tb.param[inst * nr + r];
    kap[t] = exp(pc >= 0 ? th[pc] + alpha * dth[pc] : tb.logk[inst * nr + r]);
  }
  __syncthreads();
  // thread (candidate c, group g) covers rows g, g + G, ...; groups are summed in order below
  const int G = nthr() / nls;
  const int c = tid() % nls, g = tid() / nls;
  const double h = tb.elem_h[e], tr = o.tau_r;
  double l1 = 0.0, lg = 0.0, ob = 0.0;
  if (g < G) {
    const double alpha = ldexp(alpha0, -c);
    const double* kc = kap + c * nr;
    for (int row = g; row < b; row += G) {
      const int j = row / ns, s = row - j * ns;
      double gv;
      if (j == 0) {
        const double zt = z[s] + alpha * dz[s];
        gv = zt - (i == 0 ? tb.z0[inst * ns + s] : zp[s] + alpha * dzp[s]);
      } else {
        double acc = 0.0;
        for (int jj = 0; jj <= K; ++jj) acc += S.a[jj][j] * (z[jj * ns + s] + alpha * dz[jj * ns + s]);
        double f = 0.0;
        for (int q = spp[s]; q < spp[s + 1]; ++q) {
          const int r = spr[q];
          const int q0 = rea[2 * r], q1 = rea[2 * r + 1];
          const double u0 = q0 >= 0 ? z[j * ns + q0] + alpha * dz[j * ns + q0] : 1.0;
          const double u1 = q1 >= 0 ? z[j * ns + q1] + alpha * dz[j * ns + q1] : 1.0;
          f += spnu[q] * kc[r] * u0 * u1;
        }
        gv = acc - h * f;
      }
      const double st_ = sv[row] + alpha * dsv[row];
      l1 += fabs(gv - st_);
      lg += log(st_ + tr) + log(tr - st_);
    }
    if (g == 0) {   // objective of the element's measurements
      const int m0 = tb.elem_mptr[e], m1 = tb.elem_mptr[e + 1];
      for (int m = m0; m < m1; ++m) {
        const double* w = tb.meas_w + (int64_t)m * (K + 1);
        const int s = tb.meas_sp[m];
        double pr = -tb.meas_ys[m];
        for (int jj = 0; jj <= K; ++jj) pr += w[jj] * (z[jj * ns + s] + alpha * dz[jj * ns + s]);
        ob += 0.5 * pr * pr;
      }
    }
  }
  part[tid()] = l1;
  part[nthr() + tid()] = ob;
  part[2 * nthr() + tid()] = lg;
  __syncthreads();
  if (tid() < nls) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int gg = 0; gg < G; ++gg) {
      a0 += part[gg * nls + tid()];
      a1 += part[nthr() + gg * nls + tid()];
      a2 += part[2 * nthr() + gg * nls + tid()];
    }
    double* out = st.tpart + (e * CL_MAX_LS + tid()) * 3;
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
  }
}

// Acceptance: the candidates' partial sums are reduced over the instance's elements with a
// (candidate, element group) thread mapping and a fixed-order group sum; thread 0 then scans
// the candidates in order with the filter rules and updates the filter.
__global__ void k_ipm_select(Shape S, Tab tb, IpmState st, Ws ws, colloc_ipm_opts o) {
  __shared__ double cth[CL_MAX_LS], cph[CL_MAX_LS];
  __shared__ int cfl[CL_MAX_LS];
  __shared__ double r0[256], r1[256], r2[256];
  const int inst = blockIdx.x;
  colloc_ipm_info I = st.info[inst];
  if (I.status != COLLOC_RUNNING) return;
  if (block_flag(&ws.flag[inst])) {  // factorization failed: retry with a larger delta_w
    if (tid() == 0) {
      st.info[inst].phase = PH_RETRY;
      st.info[inst].alpha_pr = 0.0;
    }
    return;
  }
  const int N = tb.inst_N[inst], np = S.np, b = S.b;
  const int64_t e0 = tb.inst_e0[inst];
  const int64_t xo = tb.inst_x[inst] + (int64_t)N * b;
  const int nls = o.max_ls;
  const int G = nthr() / nls;
  {
    const int c = tid() % nls, g = tid() / nls;
    double l1 = 0.0, ob = 0.0, lg = 0.0;
    if (g < G)
      for (int i = g; i < N; i += G) {
        const double* p = st.tpart + ((e0 + i) * CL_MAX_LS + c) * 3;
        l1 += p[0];
        ob += p[1];
        lg += p[2];
      }
    r0[tid()] = l1;
    r1[tid()] = ob;
    r2[tid()] = lg;
  }
  __syncthreads();
  const int t = tid();
  if (t < nls) {
    double alpha = I.alpha_pr;
    for (int q = 0; q < t; ++q) alpha *= 0.5;
    double l1 = 0.0, ob = 0.0, lg = 0.0;
    for (int g = 0; g < G; ++g) {
      l1 += r0[g * nls + t];
      ob += r1[g * nls + t];
      lg += r2[g * nls + t];
    }
    for (int c = 0; c < np; ++c) {
      double th = st.x[xo + c] + alpha * st.dx[xo + c];
      lg += log(th - tb.th_lo[inst * np + c]) + log(tb.th_hi[inst * np + c] - th);
    }
    cth[t] = l1;
    cph[t] = ob - I.mu * lg;
  }
  __syncthreads();
  // filter acceptability of every candidate, in parallel (thread t: candidate t)
  const double* fth = st.fth + inst * CL_FILTER_CAP;
  const double* fph = st.fph + inst * CL_FILTER_CAP;
  if (t < nls) {
    const double tht = cth[t], pht = cph[t];
    bool okf = isfinite(tht) && isfinite(pht);
    for (int f = 0; okf && f < I.filter_len; ++f)
      if (!(tht < fth[f] || pht < fph[f])) okf = false;
    cfl[t] = okf ? 1 : 0;
  }
  __syncthreads();
  if (t != 0) return;
  const double thc = I.theta_cv, phc = I.phi, dp = I.dphi;
  double alpha = I.alpha_pr;
  int acc = -1;
  bool ftype = false;
  int ntrial = 0;
  for (int q = 0; q < nls; ++q) {
    if (alpha < I.alpha_min) break;
    ++ntrial;
    const double tht = cth[q], pht = cph[q];
    const bool okf = cfl[q] != 0;
    if (okf) {
      bool sw = dp < 0 && alpha * pow(-dp, o.s_phi) > o.delta_sw * pow(thc, o.s_theta);
      bool arm = pht <= phc + o.eta_phi * alpha * dp;
      if (thc <= I.theta_min && sw) {
        if (arm) { acc = q; ftype = true; }
      } else if (tht <= (1.0 - o.gamma_theta) * thc || pht <= phc - o.gamma_phi * thc) {
        acc = q;
        ftype = sw && arm;
      }
    }
    if (acc >= 0) break;
    alpha *= 0.5;
  }
  I.ls_trials = ntrial;
  if (acc < 0) {
    I.status = COLLOC_RESTORATION_REQUIRED;
    st.info[inst] = I;
    ws.flag[inst] = 1;
    return;
  }
  if (!ftype) {
    double nth = (1.0 - o.gamma_theta) * thc, nph = phc - o.gamma_phi * thc;
    double* wf = st.fth + inst * CL_FILTER_CAP;
    double* wp = st.fph + inst * CL_FILTER_CAP;
    int k = 0;
    for (int f = 0; f < I.filter_len; ++f)
      if (!(wf[f] >= nth && wp[f] >= nph)) {
        wf[k] = wf[f];
        wp[k] = wp[f];
        ++k;
      }
    if (k < CL_FILTER_CAP) {
      wf[k] = nth;
      wp[k] = nph;
      ++k;
    } else {
      I.status = COLLOC_EFILTER;  // filter capacity exhausted
    }
    I.filter_len = k;
  }
  I.alpha_pr = alpha;
  I.phase = PH_EVAL;
  if (I.delta_w > 0.0) I.delta_last = I.delta_w;
  I.iter += 1;
  st.info[inst] = I;
}

// Update of the iterates with the accepted step; bound multipliers with alpha_du and the
// kappa_sigma safeguard.  Element workgroups handle rows; workgroup of element 0 also theta.
__global__ void k_ipm_update(Shape S, Tab tb, IpmState st, Ws ws, colloc_ipm_opts o) {
  const int64_t e = blockIdx.x;
  const int inst = tb.elem_inst[e], i = tb.elem_loc[e];
  if (block_flag(&ws.flag[inst])) return;
  const colloc_ipm_info& I = st.info[inst];
  if (I.phase != PH_EVAL) return;
  const double a = I.alpha_pr, ad = I.alpha_du, mu = I.mu, ks = o.kappa_sigma, tr = o.tau_r;
  const int N = tb.inst_N[inst], b = S.b, np = S.np;
  const int64_t xo = tb.inst_x[inst];
  const int64_t gi = tb.inst_g[inst] + (int64_t)i * b;
  for (int t = tid(); t < b; t += nthr()) {
    st.x[xo + (int64_t)i * b + t] += a * st.dx[xo + (int64_t)i * b + t];
    double s = st.s[gi + t] + a * st.ds[gi + t];
    st.s[gi + t] = s;
    st.y[gi + t] += a * st.dy[gi + t];
    double sl = s + tr, su = tr - s;
    double vl = st.vL[gi + t] + ad * st.dvL[gi + t];
    double vu = st.vU[gi + t] + ad * st.dvU[gi + t];
    st.vL[gi + t] = fmax(fmin(vl, ks * mu / sl), mu / (ks * sl));
    st.vU[gi + t] = fmax(fmin(vu, ks * mu / su), mu / (ks * su));
  }
  if (i == 0) {
    const int64_t xt = xo + (int64_t)N * b;
    for (int c = tid(); c < np; c += nthr()) {
      double th = st.x[xt + c] + a * st.dx[xt + c];
      st.x[xt + c] = th;
      double tl = th - tb.th_lo[inst * np + c], tu = tb.th_hi[inst * np + c] - th;
      double zl = st.zL[inst * np + c] + ad * st.dzL[inst * np + c];
      double zu = st.zU[inst * np + c] + ad * st.dzU[inst * np + c];
      st.zL[inst * np + c] = fmax(fmin(zl, ks * mu / tl), mu / (ks * tl));
      st.zU[inst * np + c] = fmax(fmin(zu, ks * mu / tu), mu / (ks * tu));
    }
  }
}

// ---------------------------------------------------------------- launches
static inline int ok_or() { return hipGetLastError() == hipSuccess ? 0 : -3; }

int launch_ipm_init(const Shape& S, const Tab& tb, const IpmState& st, const Ws& ws,
                    const double* x0, const colloc_ipm_opts& o, hipStream_t s) {
  hipLaunchKernelGGL(k_init_theta, dim3(tb.n_inst), dim3(256), 0, s, S, tb, st, x0, o);
  int rc = launch_eval(S, tb, ws, st.x, ws.vtmp /*obj scratch*/, st.g, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_init_elem, dim3((unsigned)tb.n_elem), dim3(64), 0, s, S, tb, st, ws, o);
  hipLaunchKernelGGL(k_init_inst, dim3(tb.n_inst), dim3(256), 0, s, S, tb, st, ws, o);
  return ok_or();
}

size_t ipm_eval_lds(const Shape& S, int nt) {
  return sizeof(double) * (5 * S.b + 2 * S.ns + S.np * 2 + S.nr + 4 * S.K * S.nr + nt);
}

// Threads of the line-search trial kernel: large elements (whose candidate table fills most of
// a compute unit's LDS) take 1024, so that one workgroup still keeps 16 waves in flight.
int ipm_trial_threads(const Shape& S) { return S.b >= 128 ? 1024 : 256; }

size_t ipm_trial_lds(const Shape& S, int max_ls) {
  return sizeof(double) * (4 * (size_t)S.b + 2 * S.ns + 2 * S.np + (size_t)max_ls * S.nr +
                           3 * (size_t)ipm_trial_threads(S) + S.lsp) +
         sizeof(int) * ((size_t)S.ns + 1 + S.lsp + 2 * (size_t)S.nr);
}

// Dynamic LDS above 64 KiB (large networks) is declared for the evaluation and trial kernels.
int ipm_prepare_attrs(const Shape& S) {
  int rc = 0;
  const size_t ev = ipm_eval_lds(S, elem_threads(S)), tr = ipm_trial_lds(S, CL_MAX_LS);
  if (ev > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_ipm_eval, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ev) != hipSuccess)
    rc = -1;
  if (tr > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_ipm_trial, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tr) != hipSuccess)
    rc = -1;
  return rc;
}

// FP32_IR helpers.  Materialise the theta part of the condensed right-hand side (barrier terms
// already in st.rhs plus the element partials, fixed order) so the refinement residual sees it.
// An instance that once needed the FP64 fallback stays on FP64 factors: its later iterations
// are at least as ill-conditioned (the barrier terms grow as mu falls), so the FP32 attempt
// would only add work.  It is masked out of the FP32 factor and refinement here.
__global__ void k_fp32_prep(Shape S, Tab tb, IpmState st, Ws ws) {
  const int inst = blockIdx.x;
  const int skip = ws.flag[inst];
  __syncthreads();
  if (tid() == 0) {
    ws.runskip[inst] = skip;
    if (!skip && st.info[inst].ir_fallbacks > 0) ws.flag[inst] = 1;
  }
  if (skip) return;
  const int N = tb.inst_N[inst], np = S.np;
  const int64_t e0 = tb.inst_e0[inst], xt = tb.inst_x[inst] + (int64_t)N * S.b;
  (void)e0;
  for (int c = tid(); c < np; c += nthr()) st.rhs[xt + c] += thpart_sum(ws, ws.thv, inst, N, np, c);
}

// Instances whose FP32 factor failed or whose refinement did not converge re-factor in FP64.
__global__ void k_fp32_fallback(Tab tb, IpmState st, Ws ws) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < tb.n_inst; q += gridDim.x * blockDim.x) {
    const bool run = ws.runskip[q] == 0;
    const bool need = run && (ws.flag[q] != 0 || ws.ircount[q] <= 0);
    ws.fbneed[q] = need ? 1 : 0;
    ws.fbflag[q] = need ? 0 : 1;
    if (run) {
      const int c = ws.ircount[q];
      st.info[q].ir_sweeps = c < 0 ? -c : c;
      if (need) st.info[q].ir_fallbacks += 1;
    }
  }
}

__global__ void k_fp32_done(Tab tb, Ws ws) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < tb.n_inst; q += gridDim.x * blockDim.x)
    if (ws.fbneed[q]) ws.flag[q] = ws.fbflag[q];
}

int launch_ipm_step(const Shape& S, const Tab& tb, const HostPlan& hp, const IpmState& st,
                    const Ws& ws, const Ws& ws64, const colloc_ipm_opts& o, phase_cb cb, void* ctx,
                    hipStream_t s) {
  const int nt = elem_threads(S);
  const unsigned ne = (unsigned)tb.n_elem;
  if (cb) cb(ctx, COLLOC_PH_EVAL, 1, s);
  hipLaunchKernelGGL(k_ipm_eval, dim3(ne), dim3(nt), ipm_eval_lds(S, nt), s, S, tb, st, ws, o);
  hipLaunchKernelGGL(k_ipm_decide, dim3(tb.n_inst), dim3(1024), sizeof(double) * S.np, s, S, tb, st, ws, o);
  hipLaunchKernelGGL(k_ipm_prep, dim3(ne), dim3(nt),
                     sizeof(double) * (2 * S.b + S.ns + S.K * S.nr + S.np), s, S, tb, st, ws, o);
  if (cb) cb(ctx, COLLOC_PH_EVAL, 0, s);
  int rc;
  if (ws.prec == 0) {
    rc = launch_factor_nc(S, tb, hp, ws, 0, true, cb, ctx, s);
    if (rc) return rc;
    rc = launch_solve_p(S, tb, hp, ws, st.rhs, ws.rthp, st.dx, cb, ctx, s);
    if (rc) return rc;
  } else {
    // FP32 block factors, FP64 refinement; per-instance FP64 re-factorization where the FP32
    // factor fails or the refinement does not reach its target
    launch_thpart(S, tb, ws, ws.rthp, nullptr, nullptr, ws.thv, s);
    hipLaunchKernelGGL(k_fp32_prep, dim3(tb.n_inst), dim3(64), 0, s, S, tb, st, ws);
    rc = launch_factor_nc(S, tb, hp, ws, 1, true, cb, ctx, s);
    if (rc) return rc;
    rc = launch_solve_p(S, tb, hp, ws, st.rhs, nullptr, st.dx, cb, ctx, s);
    if (rc) return rc;
    rc = launch_refine(S, tb, hp, ws, st.rhs, st.dx, o.ir_max, o.ir_tol, cb, ctx, s);
    if (rc) return rc;
    const unsigned gi = (unsigned)cl_ceil_div(tb.n_inst, 256);
    hipLaunchKernelGGL(k_fp32_fallback, dim3(gi), dim3(256), 0, s, tb, st, ws);
    Ws wf = ws64;
    wf.flag = ws.fbflag;
    rc = launch_factor_nc(S, tb, hp, wf, 0, true, cb, ctx, s);
    if (rc) return rc;
    rc = launch_solve_p(S, tb, hp, wf, st.rhs, nullptr, st.dx, cb, ctx, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_fp32_done, dim3(gi), dim3(256), 0, s, tb, ws);
  }
  if (cb) cb(ctx, COLLOC_PH_STEP, 1, s);
  hipLaunchKernelGGL(k_ipm_dir, dim3(ne), dim3(nt), sizeof(double) * (2 * S.b + S.ns + S.np + nt), s,
                     S, tb, st, ws, o);
  hipLaunchKernelGGL(k_ipm_steplen, dim3(tb.n_inst), dim3(256), 0, s, S, tb, st, ws, o);
  if (cb) cb(ctx, COLLOC_PH_STEP, 0, s);
  if (cb) cb(ctx, COLLOC_PH_LINESEARCH, 1, s);
  hipLaunchKernelGGL(k_ipm_trial, dim3(ne), dim3(ipm_trial_threads(S)), ipm_trial_lds(S, o.max_ls), s, S, tb, st, ws, o);
  hipLaunchKernelGGL(k_ipm_select, dim3(tb.n_inst), dim3(256), 0, s, S, tb, st, ws, o);
  hipLaunchKernelGGL(k_ipm_update, dim3(ne), dim3(nt), 0, s, S, tb, st, ws, o);
  if (cb) cb(ctx, COLLOC_PH_LINESEARCH, 0, s);
  return ok_or();
}

}  // namespace cl
