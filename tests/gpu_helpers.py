"""Shared helpers of the GPU parity tests: seeded states and oracle references.
Inputs and expected values come from the generator and the oracle only."""
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
}


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
