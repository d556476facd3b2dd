"""Helpers for oracle pin tests (test code; calls only the oracle)."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import problem


def discrete_states(model, theta, z_guess=None, iters=30):
    """Solve g(z, theta) = 0 for the states with theta fixed (Newton on the square system)."""
    x = np.zeros(model.n)
    if z_guess is not None:
        x[: model.nz] = z_guess
    else:
        x[: model.nz] = np.tile(model.z0, model.N * (model.K + 1))
    x[model.nz:] = theta
    for _ in range(iters):
        g = model.constraints(x)
        if np.max(np.abs(g)) < 1e-14:
            break
        Jz = model.jacobian(x)[:, : model.nz].tocsc()
        x[: model.nz] -= spla.spsolve(Jz, g)
    return x


def ab_matrix(k1, k2):
    return np.array([[-k1, k2], [k1, -k2]])


def radau3_R(M):
    """Radau IIA K=3 stability function applied to a matrix argument."""
    I = np.eye(M.shape[0])
    P = I + 2 * M / 5 + M @ M / 20
    Q = I - 3 * M / 5 + 3 * M @ M / 20 - M @ M @ M / 60
    return np.linalg.solve(Q, P)
