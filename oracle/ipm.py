"""Filter line-search interior-point iteration (oracle; test infrastructure only).

The paper solves the collocation NLP with a filter line-search interior-point method on a
pivoting-free (condensed) KKT form, with a 1e-6 relative KKT tolerance and a 1e-4 acceptable
level over 15 iterations (Benchmark setup, optimization framework configurations).  The paper
does not restate the method; this module follows the published algorithm it refers to
(Waechter & Biegler, Math. Prog. 106 (2006), Algorithm A with inertia correction IC, no
second-order correction and no restoration phase), applied to the relaxed-equality NLP of
``oracle.kkt``.  Constants are that paper's defaults unless stated in ``Options``.

One call of ``iterate`` performs one iteration, in this order: evaluate functions and
derivatives; test convergence; update the barrier parameter; solve the Newton system with
inertia correction; fraction-to-boundary; backtracking filter line search; update iterates.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import blocksolve, kkt

RUNNING, SOLVED, ACCEPTABLE, MAXITER, TIMEOUT, ENOTPD, ENONFINITE, RESTORATION, IR_FALLBACK = range(9)


@dataclass
class Options:
    tol: float = 1e-6
    acceptable_tol: float = 1e-4
    acceptable_iter: int = 15
    max_iter: int = 3000
    mu_init: float = 0.1
    tau_r: float = 1e-8            # equality relaxation half-width
    kappa_eps: float = 10.0
    kappa_mu: float = 0.2
    theta_mu: float = 1.5
    tau_min: float = 0.99
    kappa_sigma: float = 1e10
    s_max: float = 100.0
    bound_push: float = 1e-2       # kappa_1
    bound_frac: float = 1e-2       # kappa_2
    delta_w0: float = 1e-4
    delta_min: float = 1e-20
    delta_max: float = 1e40
    kappa_w_minus: float = 1.0 / 3.0
    kappa_w_plus: float = 8.0
    kappa_w_plus_bar: float = 100.0
    gamma_theta: float = 1e-5
    gamma_phi: float = 1e-8
    s_theta: float = 1.1
    s_phi: float = 2.3
    eta_phi: float = 1e-8
    delta_sw: float = 1.0
    gamma_alpha: float = 0.05
    max_ls: int = 40               # backtracking trials per iteration


@dataclass
class State:
    x: np.ndarray
    s: np.ndarray
    y: np.ndarray
    zL: np.ndarray
    zU: np.ndarray
    vL: np.ndarray
    vU: np.ndarray
    mu: float
    theta_max: float
    theta_min: float
    filt: list = field(default_factory=list)
    delta_last: float = 0.0
    it: int = 0
    acc_count: int = 0
    status: int = RUNNING
    log: list = field(default_factory=list)
    last_step: tuple = ()


def _push(v, lo, hi, k1, k2):
    pl = np.minimum(k1 * np.maximum(1.0, np.abs(lo)), k2 * (hi - lo))
    pu = np.minimum(k1 * np.maximum(1.0, np.abs(hi)), k2 * (hi - lo))
    return np.minimum(np.maximum(v, lo + pl), hi - pu)


def init_state(model, x0, opt: Options) -> State:
    x = np.array(x0, dtype=float)
    x[model.nz:] = _push(x[model.nz:], model.theta_lo, model.theta_hi, opt.bound_push, opt.bound_frac)
    g = model.constraints(x)
    m, p = model.m, model.np_
    s = _push(g, -opt.tau_r, opt.tau_r, opt.bound_push, opt.bound_frac)
    th0 = float(np.sum(np.abs(g - s)))
    st = State(x=x, s=s, y=np.zeros(m), zL=np.ones(p), zU=np.ones(p), vL=np.ones(m),
               vU=np.ones(m), mu=opt.mu_init, theta_max=1e4 * max(1.0, th0),
               theta_min=1e-4 * max(1.0, th0))
    st.filt = [(st.theta_max, -math.inf)]
    return st


def barrier_phi(model, x, s, mu, tau_r):
    tl, tu, sl, su = kkt.slacks(model, x, s, tau_r)
    return model.objective(x) - mu * (np.sum(np.log(tl)) + np.sum(np.log(tu))
                                      + np.sum(np.log(sl)) + np.sum(np.log(su)))


def constraint_violation(model, x, s):
    return float(np.sum(np.abs(model.constraints(x) - s)))


def optimality_errors(model, st, opt, grad, J, g):
    """Returns a function mu -> E_mu (scaled optimality error of the barrier problem)."""
    tl, tu, sl, su = kkt.slacks(model, st.x, st.s, opt.tau_r)
    rx = grad + J.T @ st.y
    rx[model.nz:] += -st.zL + st.zU
    rs = -st.y - st.vL + st.vU
    rp = g - st.s
    m, p = model.m, model.np_
    l1_all = (np.sum(np.abs(st.y)) + np.sum(np.abs(st.zL)) + np.sum(np.abs(st.zU))
              + np.sum(np.abs(st.vL)) + np.sum(np.abs(st.vU)))
    l1_b = l1_all - np.sum(np.abs(st.y))
    sd = max(opt.s_max, l1_all / (m + 2 * p + 2 * m)) / opt.s_max
    sc = max(opt.s_max, l1_b / (2 * p + 2 * m)) / opt.s_max
    comp = np.concatenate([tl * st.zL, tu * st.zU, sl * st.vL, su * st.vU])
    dual = max(np.max(np.abs(rx)), np.max(np.abs(rs)))
    primal = np.max(np.abs(rp))
    cmax, cmin = np.max(comp), np.min(comp)

    def E(mu):
        return max(dual / sd, primal, max(cmax - mu, mu - cmin) / sc)

    return E, dual, primal


def newton_step(model, st, opt, grad, J, g, W, dw, solver):
    """Solve the primal-dual system with perturbation dw.  Returns None when the matrix does
    not have the inertia the method needs (for the condensed form: not positive definite)."""
    sx, ss = kkt.sigmas(model, st.x, st.s, st.zL, st.zU, st.vL, st.vU, opt.tau_r)
    rx, rs, ry = kkt.newton_residuals(model, grad, J, g, st.x, st.s, st.y, st.mu, opt.tau_r)
    sxf = kkt.full_sigma_x(model, sx)
    if solver == "ldl":
        dx, ds, dy, inertia = kkt.solve_unreduced(W, J, sxf, ss, dw, rx, rs, ry)
        if inertia != (model.n + model.m, model.m, 0):
            return None
    else:
        Kc = kkt.condensed_matrix(W, J, sxf, ss, dw)
        rhs = kkt.condensed_rhs(J, ss, dw, rx, rs, ry)
        try:
            if solver == "block":
                F = blocksolve.factor(Kc, model.N, model.b, model.np_)
                dx = blocksolve.solve(F, rhs)
            else:
                L = sla.cholesky(Kc.toarray(), lower=True)
                dx = sla.cho_solve((L, True), rhs)
        except (blocksolve.NotPositiveDefinite, sla.LinAlgError):
            return None
        ds, dy = kkt.recover(J, ss, dw, dx, rs, ry)
    dzL, dzU, dvL, dvU = kkt.bound_steps(model, st.x, st.s, st.zL, st.zU, st.vL, st.vU, dx, ds,
                                         st.mu, opt.tau_r)
    return dx, ds, dy, dzL, dzU, dvL, dvU


def _max_step(v, dv, tau):
    """Largest alpha in (0, 1] with v + alpha dv >= (1 - tau) v, for v > 0."""
    neg = dv < 0
    if not np.any(neg):
        return 1.0
    return float(min(1.0, np.min(-tau * v[neg] / dv[neg])))


def filter_acceptable(filt, th, ph):
    return all(th < tf or ph < pf for tf, pf in filt)


def filter_add(filt, th, ph):
    kept = [(tf, pf) for tf, pf in filt if not (tf >= th and pf >= ph)]
    kept.append((th, ph))
    return kept


def iterate(model, st: State, opt: Options, solver="ldl"):
    if st.status != RUNNING:
        return st.status
    nz = model.nz
    g = model.constraints(st.x)
    grad = model.gradient(st.x)
    J = model.jacobian(st.x)
    E, dual, primal = optimality_errors(model, st, opt, grad, J, g)
    E0 = E(0.0)
    if not np.isfinite(E0):
        st.status = ENONFINITE
        return st.status
    if E0 <= opt.tol:
        st.status = SOLVED
        return st.status
    st.acc_count = st.acc_count + 1 if E0 <= opt.acceptable_tol else 0
    if st.acc_count >= opt.acceptable_iter:
        st.status = ACCEPTABLE
        return st.status
    if st.it >= opt.max_iter:
        st.status = MAXITER
        return st.status
    # barrier parameter update (monotone, repeated while the barrier problem is solved)
    while E(st.mu) <= opt.kappa_eps * st.mu:
        new_mu = max(opt.tol / 10.0, min(opt.kappa_mu * st.mu, st.mu ** opt.theta_mu))
        if new_mu >= st.mu:
            break
        st.mu = new_mu
        st.filt = [(st.theta_max, -math.inf)]
    tau = max(opt.tau_min, 1.0 - st.mu)

    # Newton step with inertia correction
    W = model.hessian(st.x, st.y)
    dw = 0.0
    tries = 0
    while True:
        step = newton_step(model, st, opt, grad, J, g, W, dw, solver)
        tries += 1
        if step is not None:
            break
        if dw == 0.0:
            dw = opt.delta_w0 if st.delta_last == 0.0 else max(opt.delta_min, opt.kappa_w_minus * st.delta_last)
        else:
            dw *= opt.kappa_w_plus_bar if st.delta_last == 0.0 else opt.kappa_w_plus
        if dw > opt.delta_max:
            st.status = ENOTPD
            return st.status
    if dw > 0.0:
        st.delta_last = dw
    dx, ds, dy, dzL, dzU, dvL, dvU = step
    st.last_step = step   # kept for inspection by tests

    # fraction to the boundary
    tl, tu, sl, su = kkt.slacks(model, st.x, st.s, opt.tau_r)
    dth = dx[nz:]
    a_max = min(_max_step(tl, dth, tau), _max_step(tu, -dth, tau),
                _max_step(sl, ds, tau), _max_step(su, -ds, tau))
    a_z = min(_max_step(st.zL, dzL, tau), _max_step(st.zU, dzU, tau),
              _max_step(st.vL, dvL, tau), _max_step(st.vU, dvU, tau))

    # filter line search
    th_c = float(np.sum(np.abs(g - st.s)))
    ph_c = barrier_phi(model, st.x, st.s, st.mu, opt.tau_r)
    dphi = float(grad @ dx - st.mu * np.sum(dth / tl) + st.mu * np.sum(dth / tu)
                 - st.mu * np.sum(ds / sl) + st.mu * np.sum(ds / su))
    if dphi < 0:
        a_min = min(opt.gamma_theta, opt.gamma_phi * th_c / (-dphi))
        if th_c <= st.theta_min:
            a_min = min(a_min, opt.delta_sw * th_c ** opt.s_theta / (-dphi) ** opt.s_phi)
    else:
        a_min = opt.gamma_theta
    a_min *= opt.gamma_alpha

    alpha = a_max
    accepted = False
    ftype = False
    ntrial = 0
    for t in range(opt.max_ls):
        if alpha < a_min:
            break
        ntrial += 1
        xt = st.x + alpha * dx
        stt = st.s + alpha * ds
        th_t = constraint_violation(model, xt, stt)
        ph_t = barrier_phi(model, xt, stt, st.mu, opt.tau_r)
        if np.isfinite(th_t) and np.isfinite(ph_t) and filter_acceptable(st.filt, th_t, ph_t):
            switching = dphi < 0 and alpha * (-dphi) ** opt.s_phi > opt.delta_sw * th_c ** opt.s_theta
            armijo = ph_t <= ph_c + opt.eta_phi * alpha * dphi
            if th_c <= st.theta_min and switching:
                if armijo:
                    accepted, ftype = True, True
            elif th_t <= (1.0 - opt.gamma_theta) * th_c or ph_t <= ph_c - opt.gamma_phi * th_c:
                accepted, ftype = True, switching and armijo
        if accepted:
            break
        alpha *= 0.5
    if not accepted:
        st.status = RESTORATION
        return st.status
    if not ftype:
        st.filt = filter_add(st.filt, (1.0 - opt.gamma_theta) * th_c, ph_c - opt.gamma_phi * th_c)

    # update
    st.x = st.x + alpha * dx
    st.s = st.s + alpha * ds
    st.y = st.y + alpha * dy
    tl, tu, sl, su = kkt.slacks(model, st.x, st.s, opt.tau_r)
    ks, mu = opt.kappa_sigma, st.mu

    def safeguard(v, slack):
        return np.maximum(np.minimum(v, ks * mu / slack), mu / (ks * slack))

    st.zL = safeguard(st.zL + a_z * dzL, tl)
    st.zU = safeguard(st.zU + a_z * dzU, tu)
    st.vL = safeguard(st.vL + a_z * dvL, sl)
    st.vU = safeguard(st.vU + a_z * dvU, su)
    st.it += 1
    st.log.append(dict(it=st.it, obj=model.objective(st.x), inf_pr=primal, inf_du=dual, E0=E0,
                       mu=st.mu, dw=dw, alpha=alpha, alpha_z=a_z, ls=ntrial, tries=tries))
    return st.status


def solve(model, x0, opt: Options | None = None, solver="ldl", max_iter=None):
    opt = opt or Options()
    st = init_state(model, x0, opt)
    limit = opt.max_iter if max_iter is None else max_iter
    while st.status == RUNNING and st.it <= limit:
        iterate(model, st, opt, solver)
        if max_iter is not None and st.it >= max_iter and st.status == RUNNING:
            break
    return st


def reduced_hessian(model, x, y):
    """Hessian of the Lagrangian reduced to the parameter directions at (x, y).

    The collocation constraints determine the states from the parameters (their Jacobian in the
    states, J_z, is square and nonsingular), so the feasible directions are Z = [-J_z^-1 J_th; I].
    The reduced Hessian Z^T W Z, W = Hessian of Phi + y^T g, is the second derivative of the
    objective along the discrete trajectory z(theta) when y makes the state gradient of the
    Lagrangian vanish (problem statement eq. 1, discretized NLP eq. 2).  Returns the p x p
    matrix and its condition number (inf when it is not positive definite)."""
    J = model.jacobian(x).tocsc()
    nz = model.nz
    Jz, Jth = J[:, :nz], J[:, nz:].toarray()
    import scipy.sparse.linalg as spla
    lu = spla.splu(Jz)
    dz = -lu.solve(Jth)
    Z = np.vstack([dz, np.eye(model.np_)])
    W = model.hessian(x, y)
    H = Z.T @ (W @ Z)
    H = 0.5 * (H + H.T)
    ev = np.linalg.eigvalsh(H)
    kappa = float(ev[-1] / ev[0]) if ev[0] > 0 else math.inf
    return H, kappa
