"""Pins for the oracle's collocation tables (eq. 2b-2c, eq. 3) against textbook facts.

Each check would fail for a plausible mistake: wrong node family (order, stability
function), transposed a_jk (row sums vs column sums), wrong derivative (exactness), wrong
continuity weights.
"""
import numpy as np
import pytest

from oracle.tables import collocation_tables, gauss_points, lagrange_values, radau_points


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("family", ["radau", "gauss"])
def test_weights_differentiate_constants_to_zero(K, family):
    _, a, _ = collocation_tables(K, family)
    # sum over j of l_j'(tau_k) is the derivative of the constant 1
    assert np.max(np.abs(a.sum(axis=0))) < 1e-12


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("family", ["radau", "gauss"])
def test_weights_exact_on_polynomials(K, family):
    tau, a, b = collocation_tables(K, family)
    for q in range(1, K + 1):
        lhs = (tau ** q) @ a                       # sum_j a_jk tau_j^q
        rhs = q * tau ** (q - 1)
        assert np.max(np.abs(lhs - rhs)) < 1e-11
        assert abs(b @ tau ** q - 1.0) < 1e-12     # continuity weights interpolate to t = 1


def test_radau_closed_form_nodes():
    assert np.allclose(radau_points(1), [1.0], atol=0)
    assert np.allclose(radau_points(2), [1 / 3, 1.0], atol=1e-15)
    s6 = np.sqrt(6.0)
    assert np.allclose(radau_points(3), [(4 - s6) / 10, (4 + s6) / 10, 1.0], atol=1e-15)
    assert np.allclose(gauss_points(2), [(3 - np.sqrt(3)) / 6, (3 + np.sqrt(3)) / 6], atol=1e-15)


def test_radau_continuity_is_last_node():
    for K in (1, 2, 3, 4):
        _, _, b = collocation_tables(K, "radau")
        e = np.zeros(K + 1)
        e[K] = 1.0
        assert np.max(np.abs(b - e)) < 1e-13


def test_k1_is_implicit_euler():
    tau, a, b = collocation_tables(1, "radau")
    assert np.allclose(tau, [0.0, 1.0])
    assert np.allclose(a[:, 1], [-1.0, 1.0])    # z1 - z0 = h f(z1)


def _one_element_amplification(K, family, zlam):
    """Solve sum_j a_jk z_j = zlam z_k (k = 1..K), z_0 = 1 and return the end value."""
    tau, a, b = collocation_tables(K, family)
    A = a[1:, 1:].T - zlam * np.eye(K)
    rhs = -a[0, 1:]
    zk = np.linalg.solve(A, rhs)
    return b[0] + b[1:] @ zk


@pytest.mark.parametrize("zlam", [-0.3, -2.0, -17.0, 0.4, -1.0 + 2.0j])
def test_radau_stability_function(zlam):
    # Radau IIA stability functions (Pade (K-1, K) approximants of exp)
    R1 = 1 / (1 - zlam)
    R2 = (1 + zlam / 3) / (1 - 2 * zlam / 3 + zlam ** 2 / 6)
    R3 = (1 + 2 * zlam / 5 + zlam ** 2 / 20) / (1 - 3 * zlam / 5 + 3 * zlam ** 2 / 20 - zlam ** 3 / 60)
    for K, R in ((1, R1), (2, R2), (3, R3)):
        got = _one_element_amplification(K, "radau", zlam)
        assert abs(got - R) <= 1e-14 * max(1.0, abs(R))


def _pade_radau(K, z):
    """(K-1, K) Pade approximant of exp(z), the stability function of the K-stage Radau IIA
    method, from its closed-form coefficients."""
    from math import factorial as f
    num = sum(f(2 * K - 1 - j) * f(K - 1) / (f(2 * K - 1) * f(j) * f(K - 1 - j)) * z ** j for j in range(K))
    den = sum(f(2 * K - 1 - j) * f(K) / (f(2 * K - 1) * f(j) * f(K - j)) * (-z) ** j for j in range(K + 1))
    return num / den


@pytest.mark.parametrize("zlam", [-0.3, -2.0, -17.0, 0.4, -1.0 + 2.0j])
def test_radau_stability_function_general_order(zlam):
    """K = 1 .. 5 against the closed-form Pade coefficients (the K <= 3 forms above are the same
    approximants written out).  K = 4, 5 carry the rounding of the monomial-basis derivative
    table (measured up to 6e-14 relative at K = 5), hence 1e-12."""
    for K in range(1, 6):
        R = _pade_radau(K, zlam)
        got = _one_element_amplification(K, "radau", zlam)
        assert abs(got - R) <= (1e-14 if K <= 3 else 1e-12) * max(1.0, abs(R)), (K, abs(got - R))


@pytest.mark.parametrize("zlam", [-0.3, -2.0, 0.4])
def test_gauss_stability_function(zlam):
    # Gauss collocation with K = 2: diagonal Pade (2, 2)
    R = (1 + zlam / 2 + zlam ** 2 / 12) / (1 - zlam / 2 + zlam ** 2 / 12)
    assert abs(_one_element_amplification(2, "gauss", zlam) - R) < 1e-14


def test_lagrange_values_partition_of_unity():
    tau, _, _ = collocation_tables(3)
    for t in (0.0, 0.25, 0.7, 1.0):
        v = lagrange_values(tau, t)
        assert abs(v.sum() - 1.0) < 1e-14
    assert np.allclose(lagrange_values(tau, 1.0), [0, 0, 0, 1], atol=1e-14)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("family", ["radau", "gauss"])
def test_lagrange_values_interpolate_polynomials(K, family):
    """Measurement weights l_j(t) at interior t reproduce every polynomial of degree <= K from
    its node values (a basis built on permuted nodes, or a wrong node, fails this)."""
    tau, _, _ = collocation_tables(K, family)
    rng = np.random.default_rng(K)
    for t in rng.uniform(0.0, 1.0, 7):
        w = lagrange_values(tau, t)
        for q in range(K + 1):
            assert abs(w @ tau ** q - t ** q) < 1e-12
        c = rng.standard_normal(K + 1)
        assert abs(w @ np.polyval(c, tau) - np.polyval(c, t)) < 1e-12 * np.sum(np.abs(c)) * 100
    # and at the nodes themselves the weights are the unit vectors
    for j in range(K + 1):
        assert np.max(np.abs(lagrange_values(tau, tau[j]) - np.eye(K + 1)[j])) < 1e-11
