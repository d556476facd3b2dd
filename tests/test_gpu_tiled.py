"""The tiled matrix-core factorization path against the oracle.

Element blocks above 160 rows (the 100-species, 200-parameter class: 700-row element matrices)
are factored by the tiled path; COLLOC_FACTOR_PATH=tiled forces it on smaller shapes so that it
can be compared with the oracle and with the register-resident path on the same inputs.

- kkt_assemble + kkt_factor + kkt_solve: right-hand side at 1e-12, K v (matrix-free) at 1e-12,
  the step with backward error <= 1e-14 on the oracle's condensed matrix and forward error within
  max(1e-10, 10 kappa eps) of the oracle's dense Cholesky solve (kappa from the dense spectrum);
- the inertia decision: positive definite iff the oracle's Cholesky succeeds;
- a batch of uneven 100-species instances: each instance's step equals its step alone, bitwise;
- whole interior-point solves through ipm_step on the tiled path: the oracle's status and
  final parameters within 1e-6 (reduced-Hessian kappa <= 1e6).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import ipm, problem
from paper_2607_12201_amd import colloc, workloads
from tests.gpu_helpers import CASES, announce, factor_path, need_gpu, net100, oracle_kkt, random_state, rel_err

pytestmark = pytest.mark.gpu

TILED_CASES = dict(CASES)
TILED_CASES["net100_n3"] = lambda: net100(1, 3)
TILED_CASES["net100_n7"] = lambda: net100(1, 7)


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _T(torch, a):
    return torch.tensor(np.asarray(a, float), dtype=torch.float64, device="cuda")


def _pd_state(m, rng):
    """A random interior state and a delta_w that makes the oracle's condensed matrix SPD with
    smallest eigenvalue >= 0.5 (dense spectrum) on cases small enough for it."""
    st = random_state(m, rng, 1.0)
    dw = 0.5
    ref = oracle_kkt(m, *st, 0.1, 1.0, dw)
    kappa = None
    if m.n <= 6000:
        ev = np.linalg.eigvalsh(ref["Kc"].toarray())
        if ev[0] < 0.5:
            dw += 0.5 - ev[0]
            ref = oracle_kkt(m, *st, 0.1, 1.0, dw)
            ev = np.linalg.eigvalsh(ref["Kc"].toarray())
        kappa = ev[-1] / ev[0]
    return st, dw, ref, kappa


def _oracle_solve(m, ref, r):
    if m.n <= 6000:
        return sla.cho_solve(sla.cho_factor(ref["Kc"].toarray(), lower=True), r)
    from oracle import blocksolve
    return blocksolve.solve(blocksolve.factor(ref["Kc"], m.N, m.b, m.np_), r)


def _check(m, ref, kappa, dx, r, dx_o):
    Kc = ref["Kc"]
    res = Kc @ dx - r
    berr = np.max(np.abs(res)) / (abs(Kc).sum(axis=1).max() * np.max(np.abs(dx)) + np.max(np.abs(r)))
    tol = 1e-10 if kappa is None else max(1e-10, 10 * kappa * np.finfo(float).eps)
    fe = rel_err(dx, dx_o)
    print(f"  backward {berr:.2e} forward {fe:.2e} (bound {tol:.2e})", flush=True)
    assert berr <= 1e-14, berr
    assert fe <= tol, (fe, tol)


def _factor_solve(torch, P, st, ref, dw, precision=colloc.FP64, ir_max=0):
    T = lambda a: _T(torch, a)
    ws = P.workspace(precision)
    _, jac, hess = P.derivs(T(st[0]), T(st[2]))
    rhs = P.assemble(ws, jac, hess, T(ref["sx"]), T(ref["ss"]), T([dw] * P.n_inst), T(ref["rx"]), T(ref["rs"]),
                     T(ref["ry"]), precision=precision)
    info = P.factor(ws, precision)
    dx, sw = P.solve(ws, rhs, precision, ir_max=ir_max, ir_tol=1e-15 if ir_max else 0.0, sweeps=True)
    torch.cuda.synchronize()
    return ws, rhs, info.cpu().numpy(), dx, sw.cpu().numpy()


@pytest.mark.parametrize("name", ["ab20", "tiny", "ragged37", "single", "two", "interior_tau", "net20_n1000",
                                  "net100_n3", "net100_n7"])
def test_tiled_assemble_factor_solve(torch, name):
    announce(f"tiled assemble/factor/solve {name}")
    inst = TILED_CASES[name]()
    m = problem.Model(inst, 3)
    st, dw, ref, kappa = _pd_state(m, np.random.default_rng(2))
    with factor_path("tiled"):
        P = colloc.Problem(inst, 3)
    ws, rhs, info, dx, _ = _factor_solve(torch, P, st, ref, dw)
    assert info.tolist() == [0]
    assert rel_err(rhs.cpu().numpy(), ref["rhs"]) < 1e-12
    v = np.random.default_rng(5).standard_normal(m.n)
    Kv = P.matvec(ws, _T(torch, v)).cpu().numpy()
    assert rel_err(Kv, ref["Kc"] @ v) < 1e-12
    _check(m, ref, kappa, dx.cpu().numpy(), ref["rhs"], _oracle_solve(m, ref, ref["rhs"]))
    r2 = np.random.default_rng(6).standard_normal(m.n)
    dx2 = P.solve(ws, _T(torch, r2)).cpu().numpy()
    _check(m, ref, kappa, dx2, r2, _oracle_solve(m, ref, r2))


@pytest.mark.parametrize("name", ["ab20", "tiny", "net100_n3"])
def test_tiled_factor_flags_indefinite(torch, name):
    announce(f"tiled factor flag {name}")
    inst = TILED_CASES[name]()
    m = problem.Model(inst, 3)
    rng = np.random.default_rng(3)
    st = random_state(m, rng, 1.0)
    lam = np.linalg.eigvalsh(oracle_kkt(m, *st, 0.1, 1.0, 0.0)["Kc"].toarray())[0]
    with factor_path("tiled"):
        P = colloc.Problem(inst, 3)
    for dw, expect_pd in ((max(1.0, 1.0 - lam), True), (-1e3, False)):
        ref = oracle_kkt(m, *st, 0.1, 1.0, dw)
        try:
            np.linalg.cholesky(ref["Kc"].toarray())
            pd = True
        except np.linalg.LinAlgError:
            pd = False
        assert pd == expect_pd
        _, _, info, _, _ = _factor_solve(torch, P, st, ref, dw)
        assert info.tolist() == [0 if pd else 1]


def test_tiled_batched_alone_equals_mix(torch):
    """Uneven 100-species instances in one batch: every instance's step equals its step alone
    bitwise (per-instance work lists, fixed reduction order) and meets the oracle's bar."""
    announce("tiled batched 100-species N=3,5,2")
    insts = [net100(11, 3), net100(12, 5), net100(13, 2)]
    models = [problem.Model(i, 3) for i in insts]
    rng = np.random.default_rng(4)
    parts = [_pd_state(m, rng) for m in models]
    dw = max(p[1] for p in parts)
    refs = [oracle_kkt(m, *p[0], 0.1, 1.0, dw) for m, p in zip(models, parts)]
    cat = lambda key: np.concatenate([r[key] for r in refs])
    with factor_path("tiled"):
        P = colloc.Problem(insts, 3)
    st_all = [np.concatenate([p[0][k] for p in parts]) for k in range(7)]
    ref_all = dict(sx=cat("sx"), ss=cat("ss"), rx=cat("rx"), rs=cat("rs"), ry=cat("ry"))
    _, _, info, dx, _ = _factor_solve(torch, P, st_all, ref_all, dw)
    assert info.tolist() == [0, 0, 0]
    dx = dx.cpu().numpy()
    for q, (inst, m, p, r) in enumerate(zip(insts, models, parts, refs)):
        part = dx[P.x_off[q]:P.x_off[q] + m.n]
        ev = np.linalg.eigvalsh(r["Kc"].toarray())
        _check(m, r, ev[-1] / ev[0], part, r["rhs"], _oracle_solve(m, r, r["rhs"]))
        with factor_path("tiled"):
            P1 = colloc.Problem(inst, 3)
        _, _, i1, d1, _ = _factor_solve(torch, P1, p[0], r, dw)
        assert i1.tolist() == [0]
        assert np.array_equal(d1.cpu().numpy(), part), q


@pytest.mark.parametrize("name,tau_r", [("ab20", 1e-8), ("tiny", 1e-6)])
def test_tiled_ipm_solve_matches_oracle(torch, name, tau_r):
    announce(f"tiled ipm solve {name}")
    inst = CASES[name]()
    m = problem.Model(inst, 3)
    x0 = workloads.initial_point(inst, 3)
    st_o = ipm.solve(m, x0, ipm.Options(tau_r=tau_r), solver="ldl")
    _, kappa = ipm.reduced_hessian(m, st_o.x, st_o.y)
    assert kappa <= 1e6
    with factor_path("tiled"):
        P = colloc.Problem(inst, 3)
    opts = colloc.default_opts(tau_r=tau_r)
    ws, state = P.workspace(), P.state()
    P.ipm_init(_T(torch, x0), state, ws, opts)
    for calls in range(1, 401):
        P.ipm_step(state, ws, opts)
        if calls % 5 == 0 and P.info(state)[0]["status"] != colloc.RUNNING:
            break
    info = P.info(state)[0]
    th = P.state_vec(state, "x").cpu().numpy()[m.nz:]
    print(f"oracle status {st_o.status} it {st_o.it}; tiled gpu status {info['status']} it {info['iter']}", flush=True)
    # final parameters (the reduced Hessian is well conditioned); the iteration count may differ
    # by a step where rounding of the two elimination orders moves a line-search decision
    assert info["status"] == st_o.status == ipm.SOLVED
    assert np.max(np.abs(th - st_o.x[m.nz:]) / np.maximum(1.0, np.abs(st_o.x[m.nz:]))) < 1e-6
