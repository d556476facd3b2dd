"""Natural-order block Cholesky of the condensed KKT matrix (oracle; test infrastructure only).

The condensed matrix of the collocation NLP is block tridiagonal in the time elements
(element i couples only to element i-1 through the continuity constraint, eq. 2c) with a
dense border in the parameters theta.  This module factors it in the natural time order,
one element after the other, with LAPACK Cholesky/triangular solves on each b x b block
(b = (K+1) n_s), then the p x p parameter Schur complement.  It is the CPU timing path and
a second, independent solve of the condensed system; it does not use the GPU's ordering.

A non-positive pivot raises NotPositiveDefinite.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class NotPositiveDefinite(Exception):
    pass


def _chol(A):
    try:
        return sla.cholesky(A, lower=True, check_finite=True)
    except (sla.LinAlgError, ValueError) as e:
        raise NotPositiveDefinite(str(e))


def factor(Kc, N, b, p):
    """Kc: sparse (CSR) condensed matrix of size N*b + p.  Returns the factor blocks."""
    nz = N * b
    Kc = Kc.tocsr()
    Lii, Lsub, Lth = [], [], []
    prev_L = None
    prev_Lth = None
    S = Kc[nz:, nz:].toarray()
    for i in range(N):
        sl = slice(i * b, (i + 1) * b)
        D = Kc[sl, sl].toarray()
        B = Kc[sl, nz:].toarray()            # b x p
        if i > 0:
            C = Kc[sl, (i - 1) * b:i * b].toarray()   # coupling to element i-1
            Ls = sla.solve_triangular(prev_L, C.T, lower=True).T   # C L_{i-1}^{-T}
            D = D - Ls @ Ls.T
            B = B - Ls @ prev_Lth.T
        else:
            Ls = None
        L = _chol(D)
        Lt = sla.solve_triangular(L, B, lower=True).T                # p x b: B^T L^{-T}
        S -= Lt @ Lt.T
        Lii.append(L)
        Lsub.append(Ls)
        Lth.append(Lt)
        prev_L, prev_Lth = L, Lt
    LS = _chol(S)
    return dict(N=N, b=b, p=p, Lii=Lii, Lsub=Lsub, Lth=Lth, LS=LS)


def solve(F, r):
    N, b, p = F["N"], F["b"], F["p"]
    nz = N * b
    y = np.empty(N * b)
    yth = r[nz:].copy()
    for i in range(N):
        ri = r[i * b:(i + 1) * b].copy()
        if i > 0:
            ri -= F["Lsub"][i] @ y[(i - 1) * b:i * b]
        yi = sla.solve_triangular(F["Lii"][i], ri, lower=True)
        y[i * b:(i + 1) * b] = yi
        yth -= F["Lth"][i] @ yi
    xth = sla.solve_triangular(F["LS"], yth, lower=True)
    xth = sla.solve_triangular(F["LS"].T, xth, lower=False)
    x = np.empty(N * b + p)
    x[nz:] = xth
    nxt = None
    for i in range(N - 1, -1, -1):
        ri = y[i * b:(i + 1) * b] - F["Lth"][i].T @ xth
        if i + 1 < N:
            ri -= F["Lsub"][i + 1].T @ nxt
        xi = sla.solve_triangular(F["Lii"][i].T, ri, lower=False)
        x[i * b:(i + 1) * b] = xi
        nxt = xi
    return x
