"""Pins for the oracle's Newton-system algebra.

- The dense LDL^T solve agrees with LAPACK's general solve; its inertia agrees with the
  eigenvalue count.
- The condensed step (W + Sx + dw + J^T Ds J) equals the unreduced primal-dual step.
- Cholesky of the condensed matrix succeeds exactly when the unreduced matrix has the inertia
  (n+m, m, 0) (Haynsworth inertia additivity; Ds > 0).
- The natural-order block Cholesky equals a dense Cholesky solve.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import blocksolve, kkt, problem
from paper_2607_12201_amd import workloads


def test_ldl_solve_matches_lapack_and_eigen_inertia():
    rng = np.random.default_rng(0)
    for n in (5, 12, 30):
        A = rng.standard_normal((n, n))
        A = A + A.T
        A[: n // 3, : n // 3] += 10 * np.eye(n // 3)
        b = rng.standard_normal(n)
        v, inertia = kkt.ldl_solve(A, b)
        assert np.max(np.abs(v - np.linalg.solve(A, b))) < 1e-10 * np.max(np.abs(v))
        ev = np.linalg.eigvalsh(A)
        assert inertia == (int(np.sum(ev > 0)), int(np.sum(ev < 0)), 0)


def _state(m, rng, tau_r, yscale=1.0):
    x = np.concatenate([rng.uniform(0.2, 1.5, m.nz), rng.uniform(-1.0, 1.0, m.np_)])
    s = rng.uniform(-0.9, 0.9, m.m) * tau_r
    y = yscale * rng.standard_normal(m.m)
    zL, zU = rng.uniform(0.1, 2, m.np_), rng.uniform(0.1, 2, m.np_)
    vL, vU = rng.uniform(0.1, 2, m.m), rng.uniform(0.1, 2, m.m)
    return x, s, y, zL, zU, vL, vU


@pytest.fixture(scope="module")
def small():
    inst = workloads.random_network(2, n_s=3, n_r=5, N=4, n_obs=2, n_times=2, n_fixed=1)
    return problem.Model(inst, 3)


def test_condensed_equals_unreduced(small):
    m = small
    rng = np.random.default_rng(1)
    tau_r, mu = 1.0, 0.05
    for trial in range(5):
        x, s, y, zL, zU, vL, vU = _state(m, rng, tau_r)
        J = m.jacobian(x)
        W = m.hessian(x, y)
        g = m.constraints(x)
        sx, ss = kkt.sigmas(m, x, s, zL, zU, vL, vU, tau_r)
        rx, rs, ry = kkt.newton_residuals(m, m.gradient(x), J, g, x, s, y, mu, tau_r)
        dw = 200.0  # keep the condensed matrix positive definite
        sxf = kkt.full_sigma_x(m, sx)
        dx, ds, dy, inertia = kkt.solve_unreduced(W, J, sxf, ss, dw, rx, rs, ry)
        assert inertia == (m.n + m.m, m.m, 0)
        Kc = kkt.condensed_matrix(W, J, sxf, ss, dw).toarray()
        dxc = sla.cho_solve(sla.cho_factor(Kc, lower=True), kkt.condensed_rhs(J, ss, dw, rx, rs, ry))
        dsc, dyc = kkt.recover(J, ss, dw, dxc, rs, ry)
        for a, b in ((dx, dxc), (ds, dsc), (dy, dyc)):
            assert np.max(np.abs(a - b)) <= 1e-10 * max(1.0, np.max(np.abs(a)))


def test_cholesky_success_iff_inertia(small):
    m = small
    rng = np.random.default_rng(2)
    tau_r = 1.0
    seen = set()
    for trial in range(40):
        x, s, y, zL, zU, vL, vU = _state(m, rng, tau_r, yscale=float(rng.choice([0.01, 1.0, 30.0])))
        vL *= 1e-3
        vU *= 1e-3
        J = m.jacobian(x)
        W = m.hessian(x, y)
        sx, ss = kkt.sigmas(m, x, s, zL, zU, vL, vU, tau_r)
        sxf = kkt.full_sigma_x(m, sx)
        for dw in (0.0, 1.0, 100.0, 1e4):
            A = kkt.unreduced_matrix(W, J, sxf, ss, dw)
            _, inertia = kkt.ldl_solve(A, np.ones(A.shape[0]))
            good = inertia == (m.n + m.m, m.m, 0)
            try:
                np.linalg.cholesky(kkt.condensed_matrix(W, J, sxf, ss, dw).toarray())
                pd = True
            except np.linalg.LinAlgError:
                pd = False
            assert good == pd
            seen.add(pd)
    assert seen == {True, False}   # both outcomes were exercised


@pytest.mark.parametrize("N", [1, 4, 20])
def test_block_cholesky_equals_dense(N):
    inst = workloads.ab_reversible(0, N=20)
    inst = dict(inst, N=N, h=np.full(N, 10.0 / N), meas_elem=np.array([N - 1], np.int32),
                meas_species=np.array([0], np.int32), meas_tau=np.ones(1), meas_y=np.ones(1),
                meas_sigma=np.ones(1))
    m = problem.Model(inst, 3)
    rng = np.random.default_rng(N)
    x, s, y, zL, zU, vL, vU = _state(m, rng, 1.0)
    J = m.jacobian(x)
    W = m.hessian(x, y)
    sx, ss = kkt.sigmas(m, x, s, zL, zU, vL, vU, 1.0)
    Kc = kkt.condensed_matrix(W, J, kkt.full_sigma_x(m, sx), ss, 5.0)
    r = rng.standard_normal(m.n)
    F = blocksolve.factor(Kc, m.N, m.b, m.np_)
    v = blocksolve.solve(F, r)
    ref = sla.cho_solve(sla.cho_factor(Kc.toarray(), lower=True), r)
    assert np.max(np.abs(v - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_block_cholesky_reports_not_pd():
    inst = workloads.ab_reversible(0, N=10)
    m = problem.Model(inst, 3)
    rng = np.random.default_rng(0)
    x, s, y, zL, zU, vL, vU = _state(m, rng, 1.0)
    Kc = kkt.condensed_matrix(m.hessian(x, y), m.jacobian(x), np.zeros(m.n), np.ones(m.m), 0.0)
    Kc = Kc - 1e3 * __import__("scipy.sparse", fromlist=["eye"]).eye(m.n)
    with pytest.raises(blocksolve.NotPositiveDefinite):
        blocksolve.factor(Kc, m.N, m.b, m.np_)
