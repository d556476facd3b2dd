"""Shared helpers of the GPU parity tests: seeded states and oracle references.
Inputs and expected values come from the generator and the oracle only."""
import contextlib
import os
import sys

import numpy as np
import pytest

from oracle import kkt, problem
from paper_2607_12201_amd import workloads


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2607_12201_amd import colloc
    colloc.load()   # raises if the library is not built
    return torch


CASES = {
    "ab20": lambda: workloads.ab_reversible(0),
    "tiny": lambda: workloads.random_network(5, n_s=4, n_r=7, N=3, n_obs=2, n_times=3, n_fixed=2),
    "ragged37": lambda: workloads.random_network(7, n_s=5, n_r=9, N=37, n_obs=2, n_times=37, n_fixed=1),
    "single": lambda: workloads.random_network(3, n_s=3, n_r=5, N=1, n_obs=2, n_times=1),
    "two": lambda: workloads.random_network(4, n_s=3, n_r=5, N=2, n_obs=2, n_times=2),
    "net20_n1000": lambda: workloads.random_network(0),
    # measurements inside their elements (local time 0.37), not at element ends
    "interior_tau": lambda: workloads.random_network(7, n_s=5, n_r=9, N=12, n_obs=2, n_times=12,
                                                     n_fixed=1, meas_tau=0.37),
}


@contextlib.contextmanager
def factor_path(path):
    """Handles created inside use this factorization path ("tiled" or "register")."""
    old = os.environ.get("COLLOC_FACTOR_PATH")
    os.environ["COLLOC_FACTOR_PATH"] = path
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("COLLOC_FACTOR_PATH", None)
        else:
            os.environ["COLLOC_FACTOR_PATH"] = old


def net100(seed, N):
    """The 100-species, 250-reaction, 200-parameter stiff network on a short mesh (one
    measurement time per element)."""
    return workloads.random_network(seed, n_s=100, n_r=250, N=N, n_obs=20, n_times=N, klo=1e-3, khi=1e4,
                                    n_fixed=50, stiff=True)


def random_state(m, rng, tau_r=1.0, yscale=0.1):
    """Interior point with moderate barrier terms (well-conditioned condensed matrix)."""
    x = workloads.initial_point(m.inst, m.K) + 0.05 * rng.standard_normal(m.n)
    x[: m.nz] = np.abs(x[: m.nz]) + 0.05
    x[m.nz:] = np.clip(m.inst["theta0"] + 0.2 * rng.standard_normal(m.np_), m.theta_lo + 0.5, m.theta_hi - 0.5)
    s = rng.uniform(-0.8, 0.8, m.m) * tau_r
    y = yscale * rng.standard_normal(m.m)
    zL, zU = rng.uniform(0.2, 2.0, m.np_), rng.uniform(0.2, 2.0, m.np_)
    vL, vU = rng.uniform(0.2, 2.0, m.m), rng.uniform(0.2, 2.0, m.m)
    return x, s, y, zL, zU, vL, vU


def oracle_kkt(m, x, s, y, zL, zU, vL, vU, mu, tau_r, dw):
    J = m.jacobian(x)
    W = m.hessian(x, y)
    g = m.constraints(x)
    sx, ss = kkt.sigmas(m, x, s, zL, zU, vL, vU, tau_r)
    rx, rs, ry = kkt.newton_residuals(m, m.gradient(x), J, g, x, s, y, mu, tau_r)
    Kc = kkt.condensed_matrix(W, J, kkt.full_sigma_x(m, sx), ss, dw)
    rhs = kkt.condensed_rhs(J, ss, dw, rx, rs, ry)
    return dict(J=J, W=W, g=g, sx=sx, ss=ss, rx=rx, rs=rs, ry=ry, Kc=Kc, rhs=rhs)


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def term_scales(m, x):
    """Per-entry magnitude of the terms each value of g and grad Phi is summed from (eq. 2b-2d
    and the least-squares gradient), so that entries with cancellation are judged against the
    size of what cancelled: |z| terms of the node-0 rows; sum_j |a_jk z| + h sum_r |nu_sr rho_r| of
    the collocation rows; sum_m (sum_j |w_mj z| + |y_m|) |w_mj| / sigma_m^2 of the gradient."""
    z, th = m.split(x)
    G = np.zeros((m.N, m.K + 1, m.ns))
    G[0, 0] = np.abs(z[0, 0]) + np.abs(m.z0)
    if m.N > 1:
        G[1:, 0] = np.abs(z[1:, 0]) + np.einsum("j,ijs->is", np.abs(m.bw), np.abs(z[:-1]))
    rho, _ = m.rate_parts(z[:, 1:, :], th)
    for k in range(1, m.K + 1):
        G[:, k] = (np.einsum("j,ijs->is", np.abs(m.a[:, k]), np.abs(z))
                   + m.h[:, None] * (np.abs(rho[:, k - 1]) @ np.abs(m.nu.T)))
    # the residual r_m = (sum_j w_mj z - y_m) / sigma_m cancels its prediction against y_m
    gs = np.zeros(m.n)
    for q in range(len(m.my)):
        zz = z[m.me[q], :, m.ms[q]]
        rs = (np.abs(m.momega[q]) @ np.abs(zz) + abs(m.my[q])) / m.msig[q]
        for j in range(m.K + 1):
            gs[m.zidx(m.me[q], j, m.ms[q])] += rs * abs(m.momega[q, j]) / m.msig[q]
    return G.ravel(), gs


def assert_elementwise(got, ref, scale, tol, what):
    """|got - ref| <= tol * (|ref| + scale) entry by entry."""
    got, ref = np.asarray(got).ravel(), np.asarray(ref).ravel()
    bound = tol * (np.abs(ref) + np.asarray(scale).ravel())
    bad = np.abs(got - ref) > bound
    assert not np.any(bad), (what, int(np.sum(bad)), float(np.max(np.abs(got - ref) - bound)))
