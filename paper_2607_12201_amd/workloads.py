"""Seeded synthetic workloads for ODE parameter estimation with mass-action kinetics.

This module produces problem *data* only: reaction networks, finite-element meshes,
noisy measurements, parameter bounds and starting guesses.  It holds none of the
collocation or interior-point arithmetic; it is shared, as plain numpy arrays, by the
CPU oracle's tests and by the GPU path.

The paper's benchmark models (systems-biology ODE models, problem statement eq. 1) are
not available, so these seeded mass-action networks stand in for them.  Ground-truth
trajectories come from a generic stiff integrator (scipy ``solve_ivp``) on the continuous
ODE, not from the collocation discretization; noise is then added.  Starting state guesses
follow the paper's recipe of an ODE solve at the nominal parameters (Benchmark setup,
optimization framework configurations): the solve at theta0 is sampled at every element's
start time and held constant over the element.

Every instance is a dict with these entries (shapes in brackets):

  n_s, n_r, n_p, N      species, reactions, estimated parameters, finite elements
  react  int32 [n_r,2]  reactant species per reaction slot, -1 = empty slot (2A -> both A)
  prod   int32 [n_r,2]  product species per slot, -1 = empty
  param  int32 [n_r]    index of the natural-log rate parameter, -1 = fixed rate
  logk_fixed [n_r]      natural-log rate used where param == -1
  h [N]                 element widths (t_0 = 0)
  z0 [n_s]              known initial state (eq. 1c / 2d)
  meas_elem, meas_species int32 [M], meas_tau [M] (local time in (0,1]), meas_y, meas_sigma [M]
  theta_lo, theta_hi [n_p]   parameter bounds (eq. 1a)
  theta_true, theta0 [n_p]   generating and starting parameters
  z_start [N+1, n_s]    ODE solution at theta0 at the element boundary times
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp

__all__ = [
    "ab_reversible", "random_network", "stiff_network", "multistart_batch",
    "serving_trace", "initial_point", "tiny_network", "config_by_name",
]


# ----------------------------------------------------------------------------- networks

def _random_stoichiometry(rng, n_s, n_r):
    """Uni (A->B) or bi (A+B->C, A+B->C+D, 2A allowed) reactions, p=1/2 each.

    Molecule count never increases, so trajectories stay bounded."""
    react = -np.ones((n_r, 2), np.int32)
    prod = -np.ones((n_r, 2), np.int32)
    for r in range(n_r):
        if rng.random() < 0.5:
            a = int(rng.integers(n_s))
            b = int(rng.integers(n_s - 1))
            b += b >= a
            react[r, 0], prod[r, 0] = a, b
        else:
            react[r] = rng.integers(n_s, size=2)
            if rng.random() < 0.5:
                prod[r, 0] = rng.integers(n_s)
            else:
                prod[r] = rng.integers(n_s, size=2)
    return react, prod


class _MassAction:
    """Continuous-time mass-action right-hand side, used only to simulate data."""

    def __init__(self, n_s, react, prod, logk):
        self.n_s = n_s
        self.react, self.prod = react, prod
        self.k = np.exp(logk)
        n_r = len(logk)
        self.nu = np.zeros((n_s, n_r))
        for r in range(n_r):
            for q in prod[r]:
                if q >= 0:
                    self.nu[q, r] += 1.0
            for q in react[r]:
                if q >= 0:
                    self.nu[q, r] -= 1.0

    def rates(self, z):
        rho = self.k.copy()
        for t in range(2):
            idx = self.react[:, t]
            on = idx >= 0
            rho[on] *= z[idx[on]]
        return rho

    def __call__(self, t, z):
        return self.nu @ self.rates(z)

    def jac(self, t, z):
        n_r = len(self.k)
        dr = np.zeros((n_r, self.n_s))
        for r in range(n_r):
            a, b = self.react[r]
            if a >= 0 and b >= 0:
                dr[r, a] += self.k[r] * z[b]
                dr[r, b] += self.k[r] * z[a]
            elif a >= 0:
                dr[r, a] += self.k[r]
        return self.nu @ dr


def _simulate(n_s, react, prod, logk, z0, times, stiff):
    rhs = _MassAction(n_s, react, prod, logk)
    sol = solve_ivp(rhs, (0.0, float(times[-1])), z0, method="BDF" if stiff else "LSODA",
                    t_eval=times, rtol=1e-10, atol=1e-12, jac=rhs.jac)
    if not sol.success:
        raise RuntimeError(f"workload simulation failed: {sol.message}")
    return sol.y.T  # [len(times), n_s]


def _logk_full(param, logk_fixed, theta):
    out = logk_fixed.copy()
    on = param >= 0
    out[on] = theta[param[on]]
    return out


def _assemble(n_s, react, prod, param, logk_fixed, theta_true, theta0, N, T, z0,
              obs_species, n_times, sigma_abs, sigma_rel, lo, hi, rng, stiff, meas_tau=1.0):
    n_r = len(param)
    n_p = len(theta_true)
    h = np.full(N, T / N)
    t_bound = np.arange(N + 1) * (T / N)
    if N % n_times:
        raise ValueError("measurement times must align with element ends")
    step = N // n_times
    meas_elem_t = np.arange(1, n_times + 1) * step - 1          # element whose end is t_m
    # measurement time t_m = t_(e-1) + meas_tau h_e inside element e (meas_tau = 1: its end)
    t_meas = t_bound[meas_elem_t] + meas_tau * h[meas_elem_t]
    true_traj = _simulate(n_s, react, prod, _logk_full(param, logk_fixed, theta_true), z0,
                          np.concatenate([[0.0], t_meas]), stiff)
    M = len(obs_species) * n_times
    meas_elem = np.empty(M, np.int32)
    meas_species = np.empty(M, np.int32)
    ztrue = np.empty(M)
    m = 0
    for q, e in enumerate(meas_elem_t):
        for s in obs_species:
            meas_elem[m], meas_species[m] = e, s
            ztrue[m] = true_traj[q + 1, s]
            m += 1
    sigma = np.maximum(sigma_abs, sigma_rel * np.abs(ztrue)) if sigma_rel > 0 else np.full(M, sigma_abs)
    y = ztrue + sigma * rng.standard_normal(M)
    z_start = _simulate(n_s, react, prod, _logk_full(param, logk_fixed, theta0), z0, t_bound, stiff)
    return dict(
        n_s=n_s, n_r=n_r, n_p=n_p, N=N,
        react=react.astype(np.int32), prod=prod.astype(np.int32), param=param.astype(np.int32),
        logk_fixed=logk_fixed.astype(np.float64), h=h, z0=z0.astype(np.float64),
        meas_elem=meas_elem, meas_species=meas_species, meas_tau=np.full(M, float(meas_tau)),
        meas_y=y, meas_sigma=sigma,
        theta_lo=np.full(n_p, lo), theta_hi=np.full(n_p, hi),
        theta_true=theta_true.astype(np.float64), theta0=theta0.astype(np.float64),
        z_start=z_start, T=T,
    )


# ----------------------------------------------------------------------------- recipes

def ab_reversible(seed=0, N=20):
    """Reversible A <-> B, two log-rate parameters with k uniform in [0.1, 2], t in [0, 10],
    [A] observed at t = 1..10 with absolute noise sigma = 0.02."""
    rng = np.random.default_rng(seed)
    theta_true = np.log(rng.uniform(0.1, 2.0, 2))
    theta0 = np.log(np.random.default_rng(seed + 1).uniform(0.1, 2.0, 2))
    react = np.array([[0, -1], [1, -1]], np.int32)
    prod = np.array([[1, -1], [0, -1]], np.int32)
    param = np.array([0, 1], np.int32)
    return _assemble(2, react, prod, param, np.zeros(2), theta_true, theta0, N, 10.0,
                     np.array([1.0, 0.0]), np.array([0]), 10, 0.02, 0.0,
                     np.log(1e-3), np.log(2e2), rng, stiff=False)


def random_network(seed=0, n_s=20, n_r=40, N=1000, n_obs=5, n_times=50, klo=1e-2, khi=1e1,
                   n_fixed=0, stiff=False, lo=None, hi=None, meas_tau=1.0):
    """Random mass-action network: log-uniform rates in [klo, khi], initial state U[0,1],
    n_obs observed species at n_times equally spaced times, 5% relative noise.  meas_tau < 1
    places each measurement inside its element at that local time instead of at its end.

    Reactions n_r-n_fixed .. n_r-1 have fixed, known rates drawn from the same law."""
    rng = np.random.default_rng(seed)
    react, prod = _random_stoichiometry(rng, n_s, n_r)
    logk = rng.uniform(np.log(klo), np.log(khi), n_r)
    n_p = n_r - n_fixed
    param = np.where(np.arange(n_r) < n_p, np.arange(n_r), -1).astype(np.int32)
    logk_fixed = np.where(param < 0, logk, 0.0)
    theta_true = logk[:n_p].copy()
    z0 = rng.uniform(0.0, 1.0, n_s)
    obs = np.sort(rng.choice(n_s, size=n_obs, replace=False))
    theta0 = np.random.default_rng(seed + 1).uniform(np.log(klo), np.log(khi), n_p)
    lo = np.log(klo) - np.log(100.0) if lo is None else lo
    hi = np.log(khi) + np.log(100.0) if hi is None else hi
    return _assemble(n_s, react, prod, param, logk_fixed, theta_true, theta0, N, 10.0, z0,
                     obs, n_times, 0.01 * 0.05, 0.05, lo, hi, rng, stiff, meas_tau)


def stiff_network(seed=0, N=10000):
    """Stiff random network: 100 species, 250 reactions (200 estimated, 50 fixed), rates
    log-uniform in [1e-3, 1e4], 20 observables at 200 times."""
    return random_network(seed, n_s=100, n_r=250, N=N, n_obs=20, n_times=200, klo=1e-3,
                          khi=1e4, n_fixed=50, stiff=True)


def tiny_network(seed=0, n_s=3, n_r=4, N=4, n_obs=2, n_times=2, n_fixed=1):
    """A few species and reactions on a short mesh: brute-force sized test cases."""
    return random_network(seed, n_s=n_s, n_r=n_r, N=N, n_obs=n_obs, n_times=n_times,
                          n_fixed=n_fixed)


def multistart_batch(n_inst=256, n_lo=200, n_hi=2000, seed0=0):
    """Uneven batch of A <-> B instances: seeds seed0.., N uniform in [n_lo, n_hi] rounded
    to a multiple of 10 so the measurement times stay on element ends."""
    rng = np.random.default_rng(10_000 + seed0)
    out = []
    for b in range(n_inst):
        N = int(np.round(rng.integers(n_lo, n_hi + 1) / 10.0) * 10)
        out.append(ab_reversible(seed0 + b, N=N))
    return out


def serving_trace(n_req, rate, seed=0, ns_lo=5, ns_hi=100, N_lo=100, N_hi=10000):
    """Poisson arrivals of estimation requests with uneven network size and mesh.

    Returns (arrival_times, instances).  n_s ~ U{ns_lo..ns_hi}, n_r = 2 n_s, all rates
    estimated, ceil(n_s/5) observed species at 50 times, N log-uniform rounded to 50."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_req)
    arrivals = np.cumsum(gaps)
    insts = []
    for q in range(n_req):
        n_s = int(rng.integers(ns_lo, ns_hi + 1))
        N = int(max(50, np.round(np.exp(rng.uniform(np.log(N_lo), np.log(N_hi))) / 50.0) * 50))
        insts.append(random_network(seed * 100_003 + q, n_s=n_s, n_r=2 * n_s, N=N,
                                    n_obs=-(-n_s // 5), n_times=50))
    return arrivals, insts


def config_by_name(name, seed=0):
    if name == "ab_n20":
        return ab_reversible(seed)
    if name == "net20_n1000":
        return random_network(seed)
    if name == "net100_n10000":
        return stiff_network(seed)
    raise KeyError(name)


# ----------------------------------------------------------------------------- start point

def initial_point(inst, K):
    """Starting primal point x0 = [z | theta0] with z[i, j, s] = z_start[i, s] for every
    node j = 0..K of element i (element-major, node, then species)."""
    N, n_s = inst["N"], inst["n_s"]
    z = np.repeat(inst["z_start"][:N, None, :], K + 1, axis=1)
    return np.concatenate([z.ravel(), inst["theta0"]])
