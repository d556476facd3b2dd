"""Collocation-consistent starting states (oracle; test infrastructure only).

The paper takes its mesh and initial state guesses from a forward ODE solve at the nominal
parameters (numerical-results section, benchmark setup) and notes that states that do not
satisfy the collocation equations cost the interior-point method extra iterations.  The
collocation-consistent version of that forward solve, on the same mesh and nodes as the NLP, is
implicit Runge-Kutta (Radau IIA for right-Radau nodes) time stepping: element by element, with the
parameters fixed, the node values z[i, 1..K] solve the collocation equations of eq. 2b / eq. 3,

    sum_j a_jk z[i, j] - h_i f(z[i, k], theta) = 0,   k = 1..K,

given the element's first node z[i, 0]: z0 for the first element (eq. 2d), the continuity
combination sum_j b_j z[i-1, j] of the previous element for the others (eq. 2c).  Each element is
one Newton solve with the dense Jacobian  a_k'k I - h_i delta_kk' F(z[i, k])  (F = df/dz from the
mass-action slot partials), from the constant guess z[i, k] = z[i, 0], damped by halving the step
until the largest residual falls (by the factor 1 - 1e-4 lambda), at most 30 halvings; converged
(and taken whole) once a Newton step changes no stage value by more than tol (1 + the largest
stage value).
"""
from __future__ import annotations

import numpy as np


def species_jacobian(model, u, theta):
    """F[s, q] = d f_s / d u_q at one state u (mass action, slot by slot)."""
    _, d = model.rate_parts(u[None, :], theta)
    d = d[0]
    D = np.zeros((model.nr, model.ns))
    for r in range(model.nr):
        for t in range(2):
            q = model.react[r, t]
            if q >= 0:
                D[r, q] += d[r, t]
    return model.nu @ D


def element_residual(model, z_first, Z, h, theta):
    """G[k-1] = sum_j a_jk z_j - h f(z_k, theta), k = 1..K (z_0 = z_first, z_k = Z[k-1])."""
    zfull = np.vstack([z_first[None, :], Z])
    return np.array([model.a[:, k] @ zfull - h * model.f(Z[k - 1][None, :], theta)[0]
                     for k in range(1, model.K + 1)])


def element_step(model, z_first, h, theta, tol=1e-13, max_newton=60):
    """Node values z[1..K] of one element from its first node (damped Newton on the K ns
    collocation equations).  Returns (z [K+1, ns], Newton iterations)."""
    K, ns, a = model.K, model.ns, model.a
    Z = np.tile(z_first, (K, 1))
    G = element_residual(model, z_first, Z, h, theta)
    for it in range(1, max_newton + 1):
        J = np.zeros((K * ns, K * ns))
        for k in range(1, K + 1):
            for kk in range(1, K + 1):
                J[(k - 1) * ns:k * ns, (kk - 1) * ns:kk * ns] += a[kk, k] * np.eye(ns)
            J[(k - 1) * ns:k * ns, (k - 1) * ns:k * ns] -= h * species_jacobian(model, Z[k - 1], theta)
        dZ = np.linalg.solve(J, -G.ravel()).reshape(K, ns)
        if np.max(np.abs(dZ)) <= tol * (1.0 + np.max(np.abs(Z + dZ))):   # converged: full step
            return np.vstack([z_first[None, :], Z + dZ]), it
        gn, lam = np.max(np.abs(G)), 1.0
        for _ in range(30):
            Zt = Z + lam * dZ
            Gt = element_residual(model, z_first, Zt, h, theta)
            if np.max(np.abs(Gt)) <= (1.0 - 1e-4 * lam) * gn:
                break
            lam *= 0.5
        Z, G = Zt, Gt
    raise RuntimeError("collocation Newton did not converge")


def forward_collocation(model, theta, status=False):
    """x = [z | theta] whose states satisfy every collocation and continuity equation (eq. 2b-2d)
    at the given parameters.  With status=True returns (x, first), first = 0 or 1 + the first
    element whose Newton iteration failed (from there on the element keeps its first node as
    every stage value) instead of raising."""
    z = np.empty((model.N, model.K + 1, model.ns))
    first = np.asarray(model.z0, float)
    failed = 0
    for i in range(model.N):
        try:
            z[i], _ = element_step(model, first, model.h[i], theta)
        except RuntimeError:
            if not status:
                raise
            failed = failed or i + 1
            z[i] = np.tile(first, (model.K + 1, 1))
        first = model.bw @ z[i]
    x = np.concatenate([z.ravel(), np.asarray(theta, float)])
    return (x, failed) if status else x
