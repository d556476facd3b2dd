"""Collocation NLP functions and derivatives (oracle; test infrastructure only).

The simultaneous-method NLP (eq. 2a-2d, collocation in the form of eq. 3) for one ODE
parameter-estimation instance (eq. 1) with mass-action kinetics, in FP64:

  variables   x = [z | theta], z[i, j, s] for element i = 0..N-1, node j = 0..K, species s
  constraints g[i, 0, s] = z[i,0,s] - z0[s]                       (i = 0, eq. 2d)
              g[i, 0, s] = z[i,0,s] - sum_j b_j z[i-1,j,s]         (i >= 1, eq. 2c)
              g[i, k, s] = sum_j a_jk z[i,j,s] - h_i f_s(z[i,k,:], theta)   (k >= 1, eq. 2b / 3)
  objective   Phi = 1/2 sum_m ((sum_j w_mj z[e_m, j, s_m] - y_m) / sigma_m)^2, w_mj = l_j(tau_m)

Mass action: f_s = sum_r nu_sr rho_r, rho_r = kappa_r * prod over the filled reactant slots of
u_(slot species), kappa_r = exp(theta_(param r)) (or exp(logk_fixed_r) for a fixed rate).
Derivatives are taken slot by slot (d rho / d slot_t = kappa * the other slot's species),
so the bimolecular 2A case gets its factor 2 from adding the two slots.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .tables import collocation_tables, lagrange_values


class Model:
    def __init__(self, inst: dict, K: int = 3, family: str = "radau"):
        self.inst = inst
        self.K = K
        self.ns, self.nr, self.np_, self.N = (int(inst[k]) for k in ("n_s", "n_r", "n_p", "N"))
        self.react = np.asarray(inst["react"], np.int64)
        self.prod = np.asarray(inst["prod"], np.int64)
        self.param = np.asarray(inst["param"], np.int64)
        self.logk_fixed = np.asarray(inst["logk_fixed"], float)
        self.h = np.asarray(inst["h"], float)
        self.z0 = np.asarray(inst["z0"], float)
        self.tau, self.a, self.bw = collocation_tables(K, family)
        self.nu = np.zeros((self.ns, self.nr))
        for r in range(self.nr):
            for q in self.prod[r]:
                if q >= 0:
                    self.nu[q, r] += 1.0
            for q in self.react[r]:
                if q >= 0:
                    self.nu[q, r] -= 1.0
        self.b = (K + 1) * self.ns
        self.nz = self.N * self.b
        self.n = self.nz + self.np_
        self.m = self.N * self.b
        self.me = np.asarray(inst["meas_elem"], np.int64)
        self.ms = np.asarray(inst["meas_species"], np.int64)
        self.my = np.asarray(inst["meas_y"], float)
        self.msig = np.asarray(inst["meas_sigma"], float)
        self.momega = np.array([lagrange_values(self.tau, t) for t in inst["meas_tau"]]).reshape(
            len(self.my), K + 1)
        self.theta_lo = np.asarray(inst["theta_lo"], float)
        self.theta_hi = np.asarray(inst["theta_hi"], float)

    # -- layout helpers ------------------------------------------------------------------
    def zidx(self, i, j, s):
        return (np.asarray(i) * (self.K + 1) + np.asarray(j)) * self.ns + np.asarray(s)

    def split(self, x):
        return x[: self.nz].reshape(self.N, self.K + 1, self.ns), x[self.nz:]

    # -- kinetics ------------------------------------------------------------------------
    def kappa(self, theta):
        lk = self.logk_fixed.astype(np.result_type(theta.dtype, float))
        on = self.param >= 0
        lk[on] = theta[self.param[on]]
        return np.exp(lk)

    def rate_parts(self, U, theta):
        """U[..., ns] -> rho[..., nr], slot partials d[..., nr, 2]."""
        kap = self.kappa(theta)
        shape = U.shape[:-1] + (self.nr,)
        fac = []
        for t in range(2):
            q = self.react[:, t]
            v = np.ones(shape, dtype=U.dtype)
            on = q >= 0
            v[..., on] = U[..., q[on]]
            fac.append(v)
        rho = kap * fac[0] * fac[1]
        d = np.zeros(shape + (2,), dtype=rho.dtype)
        for t in range(2):
            on = self.react[:, t] >= 0
            d[..., on, t] = (kap * fac[1 - t])[..., on]
        return rho, d

    def f(self, U, theta):
        rho, _ = self.rate_parts(U, theta)
        return rho @ self.nu.T

    # -- NLP functions -------------------------------------------------------------------
    def constraints(self, x):
        z, th = self.split(x)
        G = np.zeros((self.N, self.K + 1, self.ns), dtype=x.dtype)
        G[0, 0] = z[0, 0] - self.z0
        if self.N > 1:
            G[1:, 0] = z[1:, 0] - np.einsum("j,ijs->is", self.bw, z[:-1])
        for k in range(1, self.K + 1):
            G[:, k] = np.einsum("j,ijs->is", self.a[:, k], z) - self.h[:, None] * self.f(z[:, k], th)
        return G.ravel()

    def residuals(self, x):
        z, _ = self.split(x)
        pred = np.einsum("mj,mj->m", self.momega, z[self.me, :, self.ms])
        return (pred - self.my) / self.msig

    def objective(self, x):
        r = self.residuals(x)
        return 0.5 * np.sum(r * r)

    def gradient(self, x):
        r = self.residuals(x)
        gz = np.zeros(self.n, dtype=x.dtype)
        for m in range(len(r)):
            for j in range(self.K + 1):
                gz[self.zidx(self.me[m], j, self.ms[m])] += r[m] * self.momega[m, j] / self.msig[m]
        return gz

    # -- first derivatives ---------------------------------------------------------------
    def jacobian(self, x):
        """Sparse constraint Jacobian (m x n), CSR."""
        z, th = self.split(x)
        N, K, ns = self.N, self.K, self.ns
        rows, cols, vals = [], [], []
        s = np.arange(ns)
        # node-0 rows
        rows.append(self.zidx(0, 0, s)); cols.append(self.zidx(0, 0, s)); vals.append(np.ones(ns))
        for i in range(1, N):
            rows.append(self.zidx(i, 0, s)); cols.append(self.zidx(i, 0, s)); vals.append(np.ones(ns))
            for j in range(K + 1):
                if self.bw[j] != 0.0:
                    rows.append(self.zidx(i, 0, s)); cols.append(self.zidx(i - 1, j, s))
                    vals.append(np.full(ns, -self.bw[j]))
        # collocation rows: constant a_jk part
        I, S = np.meshgrid(np.arange(N), s, indexing="ij")
        for k in range(1, K + 1):
            for j in range(K + 1):
                rows.append(self.zidx(I, k, S).ravel()); cols.append(self.zidx(I, j, S).ravel())
                vals.append(np.full(I.size, self.a[j, k]))
        # collocation rows: -h_i d f / d (u, theta)
        U = z[:, 1:, :]
        rho, d = self.rate_parts(U, th)
        for k in range(1, K + 1):
            for r in range(self.nr):
                for sp_ in np.nonzero(self.nu[:, r])[0]:
                    coef = -self.h * self.nu[sp_, r]
                    for t in range(2):
                        q = self.react[r, t]
                        if q >= 0:
                            rows.append(self.zidx(np.arange(N), k, sp_))
                            cols.append(self.zidx(np.arange(N), k, q))
                            vals.append(coef * d[:, k - 1, r, t])
                    c = self.param[r]
                    if c >= 0:
                        rows.append(self.zidx(np.arange(N), k, sp_))
                        cols.append(np.full(N, self.nz + c))
                        vals.append(coef * rho[:, k - 1, r])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.m, self.n))

    # -- second derivatives --------------------------------------------------------------
    def hessian(self, x, y):
        """Sparse Hessian of the Lagrangian Phi + y^T g (n x n, both triangles), CSR."""
        z, th = self.split(x)
        N, K = self.N, self.K
        rows, cols, vals = [], [], []
        for m in range(len(self.my)):
            idx = self.zidx(self.me[m], np.arange(K + 1), self.ms[m])
            w = self.momega[m] / self.msig[m]
            rows.append(np.repeat(idx, K + 1)); cols.append(np.tile(idx, K + 1))
            vals.append(np.outer(w, w).ravel())
        Y = y.reshape(N, K + 1, self.ns)
        U = z[:, 1:, :]
        rho, d = self.rate_parts(U, th)
        kap = self.kappa(th)
        for k in range(1, K + 1):
            wr = -self.h[:, None] * (Y[:, k, :] @ self.nu)      # [N, nr]
            ii = np.arange(N)
            for r in range(self.nr):
                q0, q1 = self.react[r]
                c = self.param[r]
                w = wr[:, r]
                if q0 >= 0 and q1 >= 0:
                    for qa, qb in ((q0, q1), (q1, q0)):
                        rows.append(self.zidx(ii, k, qa)); cols.append(self.zidx(ii, k, qb))
                        vals.append(w * kap[r])
                if c >= 0:
                    for t, q in enumerate((q0, q1)):
                        if q >= 0:
                            v = w * d[:, k - 1, r, t]
                            rows.append(self.zidx(ii, k, q)); cols.append(np.full(N, self.nz + c))
                            vals.append(v)
                            rows.append(np.full(N, self.nz + c)); cols.append(self.zidx(ii, k, q))
                            vals.append(v)
                    rows.append(np.full(N, self.nz + c)); cols.append(np.full(N, self.nz + c))
                    vals.append(w * rho[:, k - 1, r])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n, self.n))

    # -- per-pattern derivative values (the library's compressed derivative format) -------
    def pattern_values(self, x, y):
        """Per (element i, collocation node k = 1..K, reaction r):

        jac[i, k-1, r] = (d rho/d slot0, d rho/d slot1, d rho/d theta)  evaluated at z[i,k]
        hess[i, k-1, r] = w_ikr * (d2 rho/d slot0 d slot1, d2 rho/d slot0 d theta,
                                   d2 rho/d slot1 d theta, d2 rho/d theta2)
        with w_ikr = -h_i sum_s y[i,k,s] nu_sr (the weight of rho_r in y^T g)."""
        z, th = self.split(x)
        rho, d = self.rate_parts(z[:, 1:, :], th)
        kap = self.kappa(th)
        par = (self.param >= 0).astype(float)
        two = ((self.react[:, 0] >= 0) & (self.react[:, 1] >= 0)).astype(float)
        jac = np.stack([d[..., 0], d[..., 1], rho * par], axis=-1)
        Y = y.reshape(self.N, self.K + 1, self.ns)[:, 1:, :]
        w = -self.h[:, None, None] * (Y @ self.nu)               # [N, K, nr]
        hess = np.stack([w * kap * two, w * d[..., 0] * par, w * d[..., 1] * par,
                         w * rho * par], axis=-1)
        return jac, hess
