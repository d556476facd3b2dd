"""Solution quality after a solve (host side, not part of the interior-point path): the
sequential objective of an estimate, Phi_seq(theta), i.e. the least-squares objective (eq. 1a)
evaluated on a high-accuracy stiff ODE solution at theta instead of on the collocation
polynomials, and an analog of the paper's relative objective gap between two estimates.  The
paper (numerical results, solution quality) compares the simultaneous method's optimum with the
sequential method's through Phi_seq; the comparison systems are not available here, so the gap
is taken between any two estimates, e.g. the GPU's and a reference solve's."""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp


def _rates(inst):
    react = np.asarray(inst["react"], np.int64)
    prod = np.asarray(inst["prod"], np.int64)
    param = np.asarray(inst["param"], np.int64)
    ns, nr = int(inst["n_s"]), int(inst["n_r"])
    nu = np.zeros((ns, nr))
    for r in range(nr):
        for q in prod[r]:
            if q >= 0:
                nu[q, r] += 1.0
        for q in react[r]:
            if q >= 0:
                nu[q, r] -= 1.0
    return react, param, nu


def measurement_times(inst):
    """Absolute time of every measurement: the start of its element plus tau h."""
    h = np.asarray(inst["h"], float)
    starts = np.concatenate([[0.0], np.cumsum(h)[:-1]])
    e = np.asarray(inst["meas_elem"], np.int64)
    return starts[e] + np.asarray(inst["meas_tau"], float) * h[e]


def sequential_objective(inst, theta, rtol=1e-10, atol=1e-12):
    """Phi_seq(theta) = 1/2 sum_m ((y_m - z_(s_m)(t_m; theta)) / sigma_m)^2 with z from a stiff
    integrator (Radau IIA, adaptive) on the mass-action kinetics at theta."""
    react, param, nu = _rates(inst)
    theta = np.asarray(theta, float)
    logk = np.asarray(inst["logk_fixed"], float).copy()
    on = param >= 0
    logk[on] = theta[param[on]]
    kap = np.exp(logk)
    z0 = np.asarray(inst["z0"], float)

    def factors(z):
        f0 = np.where(react[:, 0] >= 0, z[np.maximum(react[:, 0], 0)], 1.0)
        f1 = np.where(react[:, 1] >= 0, z[np.maximum(react[:, 1], 0)], 1.0)
        return f0, f1

    def rhs(t, z):
        f0, f1 = factors(z)
        return nu @ (kap * f0 * f1)

    def jac(t, z):
        f0, f1 = factors(z)
        J = np.zeros((len(z), len(z)))
        for slot, (fa, fb) in enumerate(((f0, f1), (f1, f0))):
            q = react[:, slot]
            for r in np.nonzero(q >= 0)[0]:
                J[:, q[r]] += nu[:, r] * kap[r] * fb[r]
        return J

    t = measurement_times(inst)
    T = float(np.sum(inst["h"]))
    ts = np.unique(t)
    sol = solve_ivp(rhs, (0.0, T), z0, method="Radau", t_eval=ts, jac=jac, rtol=rtol, atol=atol)
    if not sol.success:
        raise RuntimeError(f"sequential solve failed: {sol.message}")
    idx = np.searchsorted(ts, t)
    pred = sol.y[np.asarray(inst["meas_species"], np.int64), idx]
    r = (np.asarray(inst["meas_y"], float) - pred) / np.asarray(inst["meas_sigma"], float)
    return 0.5 * float(r @ r)


def relative_objective_gap(inst, theta, theta_ref):
    """|Phi_seq(theta) - Phi_seq(theta_ref)| / |Phi_seq(theta_ref)|."""
    a, b = sequential_objective(inst, theta), sequential_objective(inst, theta_ref)
    return abs(a - b) / abs(b)


def lagrange_values(nodes, t):
    """Values at t of the Lagrange basis polynomials on `nodes` (product formula)."""
    nodes = np.asarray(nodes, float)
    out = np.ones(len(nodes))
    for j in range(len(nodes)):
        for m in range(len(nodes)):
            if m != j:
                out[j] *= (t - nodes[m]) / (nodes[j] - nodes[m])
    return out


def refine_uniform(inst, K, x):
    """One step of a mesh-refinement outer loop: every element is halved, the measurements are
    mapped to the new elements, and the warm start on the new mesh interpolates the solution's
    collocation polynomials at the new nodes (theta kept).  Returns (new instance, x0)."""
    from paper_2607_12201_amd import colloc

    tau, _ = colloc.library_tables(K)
    ns, N, np_ = int(inst["n_s"]), int(inst["N"]), int(inst["n_p"])
    z = np.asarray(x[: N * (K + 1) * ns], float).reshape(N, K + 1, ns)
    theta = np.asarray(x[N * (K + 1) * ns:], float)
    new = dict(inst)
    h = np.asarray(inst["h"], float)
    new["h"] = np.repeat(h / 2.0, 2)
    new["N"] = 2 * N
    e = np.asarray(inst["meas_elem"], np.int64)
    t = np.asarray(inst["meas_tau"], float)
    second = t > 0.5
    new["meas_elem"] = (2 * e + second).astype(np.int32)
    new["meas_tau"] = np.where(second, 2.0 * t - 1.0, 2.0 * t)
    zn = np.empty((2 * N, K + 1, ns))
    for i in range(N):
        for half in range(2):
            for j in range(K + 1):
                w = lagrange_values(tau, 0.5 * half + 0.5 * tau[j])
                zn[2 * i + half, j] = w @ z[i]
    return new, np.concatenate([zn.ravel(), theta])
