"""Collocation nodes and weights (oracle; test infrastructure only).

Follows the simultaneous-method formulation: the mesh t_ij = t_(i-1) + h_i tau_j with
tau_0 = 0 and K collocation points per element (eq. 2b), collocation weights
a_j(tau_k) = d l_j / d tau (tau_k) of the degree-K Lagrange basis on tau_0..tau_K (eq. 3),
and continuity weights b_j = l_j(1) (eq. 2c).

Node families: right Radau points (roots of P_K(2t-1) - P_(K-1)(2t-1), last node t = 1) and
Gauss-Legendre points (roots of P_K(2t-1), the family the paper names in the collocation
section).  Polynomials are built with numpy's polynomial module: plain and slow.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def radau_points(K: int) -> np.ndarray:
    """K right-Radau points in (0, 1], ascending; the last one is exactly 1."""
    c = np.zeros(K + 1)
    c[K] = 1.0
    c[K - 1] = -1.0
    x = np.sort(npleg.legroots(c).real)
    tau = (x + 1.0) / 2.0
    assert abs(tau[-1] - 1.0) < 1e-12
    tau[-1] = 1.0
    return tau


def gauss_points(K: int) -> np.ndarray:
    """K Gauss-Legendre points in (0, 1), ascending."""
    c = np.zeros(K + 1)
    c[K] = 1.0
    return (np.sort(npleg.legroots(c).real) + 1.0) / 2.0


def nodes(K: int, family: str = "radau") -> np.ndarray:
    """tau_0 = 0 followed by the K collocation points."""
    pts = radau_points(K) if family == "radau" else gauss_points(K)
    return np.concatenate([[0.0], pts])


def lagrange_polys(tau: np.ndarray):
    """Power-basis coefficients of l_j, j = 0..K, on the nodes tau."""
    out = []
    for j in range(len(tau)):
        c = nppoly.polyfromroots(np.delete(tau, j))
        out.append(c / nppoly.polyval(tau[j], c))
    return out


def collocation_tables(K: int, family: str = "radau"):
    """Returns (tau [K+1], a [K+1, K+1] with a[j, k] = l_j'(tau_k), b [K+1] = l_j(1))."""
    tau = nodes(K, family)
    ls = lagrange_polys(tau)
    a = np.array([[nppoly.polyval(tau[k], nppoly.polyder(ls[j])) for k in range(K + 1)]
                  for j in range(K + 1)])
    b = np.array([nppoly.polyval(1.0, ls[j]) for j in range(K + 1)])
    return tau, a, b


def lagrange_values(tau: np.ndarray, t: float) -> np.ndarray:
    """l_j(t) = prod_(m != j) (t - tau_m) / (tau_j - tau_m) for j = 0..K (measurement
    interpolation weights), straight from the definition of the Lagrange basis: exactly 0 or 1
    at the nodes themselves."""
    K1 = len(tau)
    out = np.empty(K1, dtype=np.result_type(t, float))
    for j in range(K1):
        v = 1.0
        for m in range(K1):
            if m != j:
                v = v * (t - tau[m]) / (tau[j] - tau[m])
        out[j] = v
    return out
