"""Pins of the oracle's collocation-consistent starting states (oracle/init.py).

- Linear kinetics: on right-Radau nodes with K = 3, collocation is the 3-stage Radau IIA method,
  whose step maps the element's first node to its last by the (2,3) Pade-type stability function
  R(w) = (1 + 2w/5 + w^2/20) / (1 - 3w/5 + 3w^2/20 - w^3/60) of w = hM (z' = M z): the oracle's
  element ends must equal R(hM) applied step after step (a textbook closed form, independent of
  the collocation tables and of the Newton solve).
- Nonlinear kinetics: the element-end error against scipy's high-accuracy ODE solution falls at
  order 2K - 1 = 5 when the mesh is halved (superconvergence of Radau collocation at the mesh
  points).
- The states satisfy the NLP's own constraints at the parameters (consistency with the model).
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import init, problem
from paper_2607_12201_amd import workloads


def _linear_instance(N, T=2.0):
    """A <-> B, B -> C: three species, first-order reactions only (M constant)."""
    inst = workloads.ab_reversible(0, N=N)
    inst = dict(inst)
    inst["n_s"], inst["n_r"], inst["n_p"] = 3, 3, 3
    inst["react"] = np.array([[0, -1], [1, -1], [1, -1]], np.int32)
    inst["prod"] = np.array([[1, -1], [0, -1], [2, -1]], np.int32)
    inst["param"] = np.array([0, 1, 2], np.int32)
    inst["logk_fixed"] = np.zeros(3)
    inst["z0"] = np.array([1.0, 0.2, 0.0])
    inst["h"] = np.full(N, T / N)
    inst["theta_lo"], inst["theta_hi"] = np.full(3, -10.0), np.full(3, 10.0)
    return inst


def test_linear_kinetics_equal_radau_iia_stability_function():
    inst = _linear_instance(10)
    m = problem.Model(inst, 3)
    theta = np.log(np.array([2.0, 0.5, 1.5]))
    x = init.forward_collocation(m, theta)
    z = x[:m.nz].reshape(m.N, 4, 3)
    k = np.exp(theta)
    M = np.array([[-k[0], k[1], 0.0], [k[0], -k[1] - k[2], 0.0], [0.0, k[2], 0.0]])
    I = np.eye(3)
    u = inst["z0"].copy()
    for i in range(m.N):
        W = inst["h"][i] * M
        P = I + 2.0 / 5.0 * W + W @ W / 20.0
        Q = I - 3.0 / 5.0 * W + 3.0 / 20.0 * W @ W - W @ W @ W / 60.0
        u = np.linalg.solve(Q, P @ u)
        assert np.max(np.abs(z[i, 3] - u)) <= 1e-13 * max(1.0, np.max(np.abs(u))), i


def _end_error(N):
    inst = workloads.random_network(2, n_s=5, n_r=8, N=N, n_obs=2, n_times=N)
    m = problem.Model(inst, 3)
    theta = np.asarray(inst["theta0"], float)
    x = init.forward_collocation(m, theta)
    z = x[:m.nz].reshape(m.N, 4, m.ns)
    t_end = np.cumsum(inst["h"])
    kap = m.kappa(theta)

    def rhs(t, u):
        return m.f(u[None, :], theta)[0]

    sol = solve_ivp(rhs, (0.0, t_end[-1]), m.z0, method="Radau", rtol=1e-13, atol=1e-15,
                    t_eval=t_end, dense_output=False)
    assert sol.success and kap.size == m.nr
    return np.max(np.abs(z[:, 3, :] - sol.y.T))


def test_nonlinear_element_ends_converge_at_order_five():
    e1, e2 = _end_error(40), _end_error(80)
    rate = np.log2(e1 / e2)
    print(f"end errors {e1:.3e} {e2:.3e}, observed order {rate:.2f}")
    assert 4.0 <= rate <= 6.5


def test_states_satisfy_the_collocation_constraints():
    inst = workloads.random_network(0, n_s=6, n_r=12, N=40, n_obs=3, n_times=40)
    m = problem.Model(inst, 3)
    x = init.forward_collocation(m, np.asarray(inst["theta0"], float))
    g = m.constraints(x)
    assert np.max(np.abs(g)) <= 1e-10
