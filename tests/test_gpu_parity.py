"""GPU parity of every ABI call against the FP64 oracle on identical seeded inputs.

Tolerances: pattern values and derivatives are the same arithmetic in a different order
(relative 1e-12); the condensed Newton step is compared normwise at relative 1e-10 on
well-conditioned states (the step's own tolerance), where the oracle's solve is a dense or
natural-order block Cholesky of its own sparse condensed matrix.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import blocksolve, problem
from paper_2607_12201_amd import colloc, workloads
from tests.gpu_helpers import (CASES, announce, assert_elementwise, need_gpu, oracle_kkt, random_state,
                               rel_err, term_scales)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _setup(name, torch):
    inst = CASES[name]()
    m = problem.Model(inst, 3)
    P = colloc.Problem(inst, 3)
    return inst, m, P


@pytest.mark.parametrize("name", ["ab20", "tiny", "ragged37", "single", "two", "net20_n1000", "interior_tau"])
def test_eval_and_derivs(torch, name):
    announce(f"eval/derivs {name}")
    inst, m, P = _setup(name, torch)
    rng = np.random.default_rng(1)
    x, s, y, *_ = random_state(m, rng)
    ws = P.workspace()
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    yd = torch.tensor(y, dtype=torch.float64, device="cuda")
    obj, g = P.eval(xd, ws)
    grad, jac, hess = P.derivs(xd, yd)
    torch.cuda.synchronize()
    g_o = m.constraints(x)
    gscale, grscale = term_scales(m, x)
    # entry by entry: each value within 1e-13 of the size of the terms it is summed from
    assert_elementwise(g.cpu().numpy(), g_o, gscale, 1e-13, "g")
    assert abs(obj.item() - m.objective(x)) <= 1e-12 * max(1.0, m.objective(x))
    assert_elementwise(grad.cpu().numpy(), m.gradient(x), grscale, 1e-13, "grad")
    jo, ho = m.pattern_values(x, y)
    # products of at most three factors: relative to the value itself
    assert_elementwise(jac.cpu().numpy(), jo.ravel(), 0.0, 1e-14, "jac")
    # the Hessian weights sum y over the species of a reaction: judged against the same sum
    # taken over |y| and |nu|
    import copy
    ma = copy.copy(m)
    ma.nu = np.abs(m.nu)
    _, ho_abs = ma.pattern_values(x, np.abs(y))
    assert_elementwise(hess.cpu().numpy(), ho.ravel(), np.abs(ho_abs).ravel(), 1e-14, "hess")


def _dense_ok(m):
    return m.n <= 3000


def _oracle_solve(m, Kc, r):
    if _dense_ok(m):
        return sla.cho_solve(sla.cho_factor(Kc.toarray(), lower=True), r)
    return blocksolve.solve(blocksolve.factor(Kc, m.N, m.b, m.np_), r)


def _check_step(m, Kc, rhs, dx_gpu, dx_o):
    """Step parity: forward error against the oracle within max(1e-10, 10 kappa eps) where the
    oracle's condition number is known, normwise backward error of the GPU step <= 1e-14."""
    res = Kc @ dx_gpu - rhs
    knorm = abs(Kc).sum(axis=1).max()
    berr = np.max(np.abs(res)) / (knorm * np.max(np.abs(dx_gpu)) + np.max(np.abs(rhs)))
    assert berr <= 1e-14, berr
    tol = 1e-10
    if _dense_ok(m):
        ev = np.linalg.eigvalsh(Kc.toarray())
        tol = max(tol, 10 * (ev[-1] / ev[0]) * np.finfo(float).eps)
    assert rel_err(dx_gpu, dx_o) <= tol, (rel_err(dx_gpu, dx_o), tol)


@pytest.mark.parametrize("name", ["ab20", "tiny", "ragged37", "single", "two", "net20_n1000", "interior_tau"])
def test_assemble_factor_solve(torch, name):
    announce(f"assemble/factor/solve {name}")
    inst, m, P = _setup(name, torch)
    rng = np.random.default_rng(2)
    tau_r, mu, dw = 1.0, 0.1, 0.5
    x, s, y, zL, zU, vL, vU = random_state(m, rng, tau_r)
    ref = oracle_kkt(m, x, s, y, zL, zU, vL, vU, mu, tau_r, dw)
    if _dense_ok(m):   # shift until the oracle's condensed matrix is positive definite
        lam = np.linalg.eigvalsh(ref["Kc"].toarray())[0]
        if lam < 0.5:
            dw += 0.5 - lam
            ref = oracle_kkt(m, x, s, y, zL, zU, vL, vU, mu, tau_r, dw)
    T = lambda a: torch.tensor(np.asarray(a, float), dtype=torch.float64, device="cuda")
    ws = P.workspace()
    grad, jac, hess = P.derivs(T(x), T(y))
    rhs = P.assemble(ws, jac, hess, T(ref["sx"]), T(ref["ss"]), T([dw]), T(ref["rx"]), T(ref["rs"]),
                     T(ref["ry"]))
    info = P.factor(ws)
    dx = P.solve(ws, rhs)
    v = rng.standard_normal(m.n)
    Kv = P.matvec(ws, T(v))
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0]
    assert rel_err(rhs.cpu().numpy(), ref["rhs"]) < 1e-12
    assert rel_err(Kv.cpu().numpy(), ref["Kc"] @ v) < 1e-12
    _check_step(m, ref["Kc"], ref["rhs"], dx.cpu().numpy(), _oracle_solve(m, ref["Kc"], ref["rhs"]))
    # the same factor solves a second right-hand side
    r2 = rng.standard_normal(m.n)
    dx2 = P.solve(ws, T(r2))
    torch.cuda.synchronize()
    _check_step(m, ref["Kc"], r2, dx2.cpu().numpy(), _oracle_solve(m, ref["Kc"], r2))


@pytest.mark.parametrize("name", ["ab20", "tiny", "ragged37"])
def test_factor_flags_indefinite(torch, name):
    announce(f"factor flag {name}")
    inst, m, P = _setup(name, torch)
    rng = np.random.default_rng(3)
    x, s, y, zL, zU, vL, vU = random_state(m, rng, 1.0)
    T = lambda a: torch.tensor(np.asarray(a, float), dtype=torch.float64, device="cuda")
    lam = np.linalg.eigvalsh(oracle_kkt(m, x, s, y, zL, zU, vL, vU, 0.1, 1.0, 0.0)["Kc"].toarray())[0]
    # clearly definite, clearly indefinite (shift dw moves every eigenvalue of W + Sx + dw I
    # and, through Ds, the J^T Ds J term)
    for dw, expect_pd in ((max(1.0, 1.0 - lam), True), (-1e3, False)):
        ref = oracle_kkt(m, x, s, y, zL, zU, vL, vU, 0.1, 1.0, dw)
        try:
            np.linalg.cholesky(ref["Kc"].toarray())
            pd = True
        except np.linalg.LinAlgError:
            pd = False
        assert pd == expect_pd
        ws = P.workspace()
        _, jac, hess = P.derivs(T(x), T(y))
        P.assemble(ws, jac, hess, T(ref["sx"]), T(ref["ss"]), T([dw]), T(ref["rx"]), T(ref["rs"]),
                   T(ref["ry"]))
        info = P.factor(ws)
        torch.cuda.synchronize()
        assert info.cpu().numpy().tolist() == [0 if pd else 1]


def test_batched_uneven_matches_single(torch):
    """Batched uneven instances: each instance's step equals its single-instance step bitwise."""
    announce("batched factor/solve")
    insts = workloads.multistart_batch(5, 20, 90)
    rng = np.random.default_rng(4)
    T = lambda a: torch.tensor(np.asarray(a, float), dtype=torch.float64, device="cuda")
    states, refs, models = [], [], []
    for inst in insts:
        m = problem.Model(inst, 3)
        st = random_state(m, rng, 1.0)
        models.append(m)
        states.append(st)
        refs.append(oracle_kkt(m, *st, 0.1, 1.0, 0.5))
    P = colloc.Problem(insts, 3)
    cat = lambda key: np.concatenate([r[key] for r in refs])
    xs = np.concatenate([s[0] for s in states])
    ys = np.concatenate([s[2] for s in states])
    ws = P.workspace()
    _, jac, hess = P.derivs(T(xs), T(ys))
    rhs = P.assemble(ws, jac, hess, T(cat("sx")), T(cat("ss")), T([0.5] * len(insts)), T(cat("rx")),
                     T(cat("rs")), T(cat("ry")))
    info = P.factor(ws)
    dx = P.solve(ws, rhs).cpu().numpy()
    assert info.cpu().numpy().tolist() == [0] * len(insts)
    for q, (m, r) in enumerate(zip(models, refs)):
        ref = sla.cho_solve(sla.cho_factor(r["Kc"].toarray(), lower=True), r["rhs"])
        part = dx[P.x_off[q]:P.x_off[q] + m.n]
        assert rel_err(part, ref) < 1e-10
        # alone
        P1 = colloc.Problem(insts[q], 3)
        ws1 = P1.workspace()
        _, j1, h1 = P1.derivs(T(states[q][0]), T(states[q][2]))
        rhs1 = P1.assemble(ws1, j1, h1, T(r["sx"]), T(r["ss"]), T([0.5]), T(r["rx"]), T(r["rs"]), T(r["ry"]))
        P1.factor(ws1)
        d1 = P1.solve(ws1, rhs1).cpu().numpy()
        assert np.array_equal(d1, part)
