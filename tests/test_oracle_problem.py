"""Pins for the oracle's NLP functions and derivatives (eq. 2, eq. 3).

- Linear A <-> B: the discrete collocation solution at element ends is the Radau IIA stability
  function applied to hA (closed form), so the oracle's g vanishes there.
- Radau K=3 collocation converges with order 2K-1 = 5 at element ends against exp(tA).
- First and second derivatives against complex-step differentiation (exact to rounding).
- The compressed per-pattern derivative values rebuild the same J and W.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import problem
from paper_2607_12201_amd import workloads
from tests.oracle_helpers import ab_matrix, discrete_states, radau3_R


def test_ab_discrete_solution_closed_form():
    inst = workloads.ab_reversible(3, N=20)
    m = problem.Model(inst, 3)
    theta = np.log([0.7, 0.4])
    x = discrete_states(m, theta)
    z, _ = m.split(x)
    R = radau3_R(m.h[0] * ab_matrix(*np.exp(theta)))
    v = m.z0.copy()
    for i in range(m.N):
        v = R @ v
        assert np.max(np.abs(z[i, -1] - v)) < 1e-13
        if i + 1 < m.N:
            assert np.max(np.abs(z[i + 1, 0] - v)) < 1e-13
    assert np.max(np.abs(m.constraints(x))) < 1e-13


def test_ab_sign_convention_of_collocation_rows():
    # g^col = sum_j a_jk z_j - h f(z_k): a constant state with f(z) != 0 gives -h f
    inst = workloads.ab_reversible(0, N=10)
    m = problem.Model(inst, 3)
    theta = np.log([1.0, 0.5])
    x = np.concatenate([np.tile([1.0, 0.0], m.N * 4), theta])
    g = m.constraints(x).reshape(m.N, 4, 2)
    f = ab_matrix(1.0, 0.5) @ np.array([1.0, 0.0])
    for k in range(1, 4):
        assert np.allclose(g[:, k, :], -m.h[:, None] * f[None, :], atol=1e-15)


@pytest.mark.parametrize("family,order", [("radau", 5), ("gauss", 6)])
def test_convergence_order(family, order):
    k1, k2 = 1.3, 0.6
    T = 2.0
    exact = sla.expm(T * ab_matrix(k1, k2)) @ np.array([1.0, 0.0])
    errs = []
    for N in (4, 8, 16):
        inst = workloads.ab_reversible(0, N=10)
        inst = dict(inst, N=N, h=np.full(N, T / N), meas_elem=np.array([N - 1], np.int32),
                    meas_species=np.array([0], np.int32), meas_tau=np.ones(1),
                    meas_y=np.zeros(1), meas_sigma=np.ones(1))
        m = problem.Model(inst, 3, family)
        x = discrete_states(m, np.log([k1, k2]))
        z, _ = m.split(x)
        end = m.bw @ z[-1]
        errs.append(np.max(np.abs(end - exact)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.2), rates


def _rand_point(m, rng):
    x = np.concatenate([rng.uniform(0.2, 1.5, m.nz), rng.uniform(-1.0, 1.0, m.np_)])
    y = rng.standard_normal(m.m)
    return x, y


@pytest.fixture(scope="module")
def tiny():
    # 2A reactions, fixed rates and two-product reactions all appear for this seed
    inst = workloads.random_network(5, n_s=4, n_r=7, N=3, n_obs=2, n_times=3, n_fixed=2)
    assert np.any(inst["react"][:, 0] == inst["react"][:, 1])
    return problem.Model(inst, 3)


def test_jacobian_complex_step(tiny):
    m = tiny
    rng = np.random.default_rng(1)
    x, _ = _rand_point(m, rng)
    J = m.jacobian(x).toarray()
    hstep = 1e-30
    for c in range(m.n):
        xc = x.astype(complex)
        xc[c] += 1j * hstep
        col = m.constraints(xc).imag / hstep
        assert np.max(np.abs(col - J[:, c])) <= 1e-13 * max(1.0, np.max(np.abs(col)))


def test_gradient_complex_step(tiny):
    m = tiny
    rng = np.random.default_rng(2)
    x, _ = _rand_point(m, rng)
    gr = m.gradient(x)
    for c in range(m.n):
        xc = x.astype(complex)
        xc[c] += 1e-30j
        assert abs(m.objective(xc).imag / 1e-30 - gr[c]) <= 1e-12 * max(1.0, abs(gr[c]))


def test_hessian_complex_step(tiny):
    m = tiny
    rng = np.random.default_rng(3)
    x, y = _rand_point(m, rng)
    W = m.hessian(x, y).toarray()
    assert np.max(np.abs(W - W.T)) == 0.0

    def grad_L(xc):
        return m.gradient(xc) + m.jacobian(xc).T @ y

    for c in range(m.n):
        xc = x.astype(complex)
        xc[c] += 1e-30j
        col = np.asarray(grad_L(xc)).imag / 1e-30
        assert np.max(np.abs(col - W[:, c])) <= 1e-12 * max(1.0, np.max(np.abs(col)))


def test_hessian_central_differences(tiny):
    m = tiny
    rng = np.random.default_rng(4)
    x, y = _rand_point(m, rng)
    W = m.hessian(x, y).toarray()

    def L(v):
        return m.objective(v) + y @ m.constraints(v)

    hs = 1e-3
    noise = 1e2 * np.finfo(float).eps * abs(L(x)) / hs ** 2    # cancellation in the 4-point formula
    for c in range(0, m.n, 3):
        for d in range(c, m.n, 5):
            ec = np.zeros(m.n); ec[c] = hs
            ed = np.zeros(m.n); ed[d] = hs
            fd = (L(x + ec + ed) - L(x + ec - ed) - L(x - ec + ed) + L(x - ec - ed)) / (4 * hs * hs)
            assert abs(fd - W[c, d]) <= 1e-6 * max(1.0, abs(W[c, d])) + noise


def test_pattern_values_rebuild_jacobian_and_hessian(tiny):
    """J and W rebuilt from the compressed per-(element, node, reaction) values equal the
    sparse J and W, so the compressed format carries all of the derivative information."""
    m = tiny
    rng = np.random.default_rng(6)
    x, y = _rand_point(m, rng)
    jac, hess = m.pattern_values(x, y)
    J = m.jacobian(x).toarray()
    W = m.hessian(x, y).toarray()
    Jr = np.zeros_like(J)
    Wr = np.zeros_like(W)
    for i in range(m.N):
        s = np.arange(m.ns)
        if i == 0:
            Jr[m.zidx(0, 0, s), m.zidx(0, 0, s)] = 1.0
        else:
            Jr[m.zidx(i, 0, s), m.zidx(i, 0, s)] = 1.0
            Jr[m.zidx(i, 0, s), m.zidx(i - 1, m.K, s)] = -1.0
        for k in range(1, m.K + 1):
            for j in range(m.K + 1):
                Jr[m.zidx(i, k, s), m.zidx(i, j, s)] += m.a[j, k]
            for r in range(m.nr):
                c = m.param[r]
                for sp_ in range(m.ns):
                    nu = m.nu[sp_, r]
                    if nu == 0:
                        continue
                    for t in range(2):
                        q = m.react[r, t]
                        if q >= 0:
                            Jr[m.zidx(i, k, sp_), m.zidx(i, k, q)] -= m.h[i] * nu * jac[i, k - 1, r, t]
                    if c >= 0:
                        Jr[m.zidx(i, k, sp_), m.nz + c] -= m.h[i] * nu * jac[i, k - 1, r, 2]
                q0, q1 = m.react[r]
                H = hess[i, k - 1, r]
                if q0 >= 0 and q1 >= 0:
                    Wr[m.zidx(i, k, q0), m.zidx(i, k, q1)] += H[0]
                    Wr[m.zidx(i, k, q1), m.zidx(i, k, q0)] += H[0]
                if c >= 0:
                    for t, q in enumerate((q0, q1)):
                        if q >= 0:
                            Wr[m.zidx(i, k, q), m.nz + c] += H[1 + t]
                            Wr[m.nz + c, m.zidx(i, k, q)] += H[1 + t]
                    Wr[m.nz + c, m.nz + c] += H[3]
    for mm in range(len(m.my)):
        idx = m.zidx(m.me[mm], np.arange(m.K + 1), m.ms[mm])
        w = m.momega[mm] / m.msig[mm]
        Wr[np.ix_(idx, idx)] += np.outer(w, w)
    assert np.max(np.abs(Jr - J)) < 1e-13
    assert np.max(np.abs(Wr - W)) < 1e-12 * max(1.0, np.max(np.abs(W)))
