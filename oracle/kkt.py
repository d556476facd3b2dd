"""Relaxed-equality primal-dual Newton system (oracle; test infrastructure only).

The NLP of eq. 2 is solved in the relaxed form used by condensed-space interior-point
methods (the paper's solver reformulates the KKT system into a pivoting-free form):

    min Phi(x)  s.t.  g(x) - s = 0,   -tau_r <= s <= tau_r,   theta_lo <= theta <= theta_hi

with multipliers y (for g - s = 0), zL/zU (theta bounds) and vL/vU (slack bounds).  After the
bound multipliers are eliminated the primal-dual Newton system is the unreduced system

    [ W + Sx + dw I     0        J^T ] [dx]     [ rx ]
    [ 0             Ss + dw I    -I  ] [ds] = - [ rs ]
    [ J                -I         0  ] [dy]     [ ry ]

with Sx = diag(zL/(theta-lo) + zU/(hi-theta)) on theta entries, Ss = diag(vL/(s+tau_r) +
vU/(tau_r-s)), rx = grad Phi + J^T y - mu/(theta-lo) + mu/(hi-theta) (barrier terms on theta
only), rs = -y - mu/(s+tau_r) + mu/(tau_r-s), ry = g - s.  Eliminating ds and dy gives the
condensed matrix  W + Sx + dw I + J^T Ds J,  Ds = Ss + dw I, with right-hand side
-rx - J^T (Ds ry + rs); then ds = J dx + ry and dy = Ds ds + rs.

The parity path solves the unreduced system with a dense Bunch-Kaufman LDL^T
(scipy.linalg.ldl), which also yields its inertia; the condensed form is built separately.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def slacks(model, x, s, tau_r):
    th = x[model.nz:]
    return th - model.theta_lo, model.theta_hi - th, s + tau_r, tau_r - s


def sigmas(model, x, s, zL, zU, vL, vU, tau_r):
    tl, tu, sl, su = slacks(model, x, s, tau_r)
    return zL / tl + zU / tu, vL / sl + vU / su


def newton_residuals(model, grad, J, g, x, s, y, mu, tau_r):
    """(rx, rs, ry) of the barrier problem at (x, s, y)."""
    tl, tu, sl, su = slacks(model, x, s, tau_r)
    rx = grad + J.T @ y
    rx[model.nz:] += -mu / tl + mu / tu
    rs = -y - mu / sl + mu / su
    ry = g - s
    return rx, rs, ry


def full_sigma_x(model, sx_theta):
    out = np.zeros(model.n)
    out[model.nz:] = sx_theta
    return out


def unreduced_matrix(W, J, sx_full, ss, dw):
    n, m = W.shape[0], J.shape[0]
    Wd = W.toarray() if sp.issparse(W) else np.asarray(W)
    Jd = J.toarray() if sp.issparse(J) else np.asarray(J)
    A = np.zeros((n + 2 * m, n + 2 * m))
    A[:n, :n] = Wd + np.diag(sx_full + dw)
    A[n:n + m, n:n + m] = np.diag(ss + dw)
    A[:n, n + m:] = Jd.T
    A[n + m:, :n] = Jd
    A[n:n + m, n + m:] = -np.eye(m)
    A[n + m:, n:n + m] = -np.eye(m)
    return A


def ldl_solve(A, rhs):
    """Solve A v = rhs with scipy's Bunch-Kaufman LDL^T; also return the inertia
    (n_pos, n_neg, n_zero) of A read off the block-diagonal factor."""
    lu, d, perm = sla.ldl(A, lower=True)
    T = lu[perm]
    v1 = sla.solve_triangular(T, rhs[perm], lower=True, unit_diagonal=True)
    v2 = _block_diag_solve(d, v1)
    u = sla.solve_triangular(T.T, v2, lower=False, unit_diagonal=True)
    out = np.empty_like(u)
    out[perm] = u
    ev = np.linalg.eigvalsh(d)
    scale = max(1.0, np.max(np.abs(ev)))
    tol = 1e-300 * scale
    inertia = (int(np.sum(ev > tol)), int(np.sum(ev < -tol)), int(np.sum(np.abs(ev) <= tol)))
    return out, inertia


def _block_diag_solve(d, v):
    """d is block diagonal with 1x1 and 2x2 blocks; solve block by block."""
    n = d.shape[0]
    out = np.empty_like(v)
    i = 0
    while i < n:
        if i + 1 < n and d[i + 1, i] != 0.0:
            out[i:i + 2] = np.linalg.solve(d[i:i + 2, i:i + 2], v[i:i + 2])
            i += 2
        else:
            out[i] = v[i] / d[i, i]
            i += 1
    return out


def solve_unreduced(W, J, sx_full, ss, dw, rx, rs, ry):
    """Dense LDL^T step: returns (dx, ds, dy, inertia)."""
    n, m = W.shape[0], J.shape[0]
    A = unreduced_matrix(W, J, sx_full, ss, dw)
    v, inertia = ldl_solve(A, -np.concatenate([rx, rs, ry]))
    return v[:n], v[n:n + m], v[n + m:], inertia


def condensed_matrix(W, J, sx_full, ss, dw):
    """W + Sx + dw I + J^T (Ss + dw I) J as a sparse matrix."""
    Ds = ss + dw
    n = W.shape[0]
    Jc = sp.csr_matrix(J)
    return (sp.csr_matrix(W) + sp.diags(sx_full + dw) + Jc.T @ sp.diags(Ds) @ Jc).tocsr()


def condensed_rhs(J, ss, dw, rx, rs, ry):
    Ds = ss + dw
    return -rx - J.T @ (Ds * ry + rs)


def recover(J, ss, dw, dx, rs, ry):
    """(ds, dy) from the condensed primal step."""
    ds = J @ dx + ry
    dy = (ss + dw) * ds + rs
    return ds, dy


def bound_steps(model, x, s, zL, zU, vL, vU, dx, ds, mu, tau_r):
    """Steps of the bound multipliers from the primal step (primal-dual bound equations)."""
    tl, tu, sl, su = slacks(model, x, s, tau_r)
    dth = dx[model.nz:]
    dzL = mu / tl - zL - (zL / tl) * dth
    dzU = mu / tu - zU + (zU / tu) * dth
    dvL = mu / sl - vL - (vL / sl) * ds
    dvU = mu / su - vU + (vU / su) * ds
    return dzL, dzU, dvL, dvU
