"""FP32 block factors with FP64 iterative refinement against the FP64 oracle.

- Step: FP32 factor + refinement reaches the FP64 step bar (normwise backward error <= 1e-14,
  forward error within max(1e-10, 10 kappa eps) of the oracle's dense solve); the plain FP32
  step without refinement is stated too (its error is at the FP32 level, kappa * 6e-8).
- Interior point: FP32_IR solves end with the oracle's status and final parameters (1e-6), and
  the iteration path equals the oracle's where the FP64 path does.
- Batched FP32_IR: each instance's result alone equals its result in the mix, bitwise.
"""
import numpy as np
import pytest

from oracle import ipm, problem
from paper_2607_12201_amd import colloc, workloads
from tests.gpu_helpers import CASES, announce, need_gpu, oracle_kkt, random_state, rel_err
from tests.test_gpu_parity import _check_step, _dense_ok, _oracle_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


@pytest.mark.parametrize("name", ["ab20", "tiny", "ragged37", "net20_n1000"])
def test_fp32_factor_refined_step(torch, name):
    announce(f"fp32 factor + refinement {name}")
    inst = CASES[name]()
    m = problem.Model(inst, 3)
    P = colloc.Problem(inst, 3)
    rng = np.random.default_rng(12)
    tau_r, mu, dw = 1.0, 0.1, 0.5
    x, s, y, zL, zU, vL, vU = random_state(m, rng, tau_r)
    ref = oracle_kkt(m, x, s, y, zL, zU, vL, vU, mu, tau_r, dw)
    if _dense_ok(m):
        lam = np.linalg.eigvalsh(ref["Kc"].toarray())[0]
        if lam < 0.5:
            dw += 0.5 - lam
            ref = oracle_kkt(m, x, s, y, zL, zU, vL, vU, mu, tau_r, dw)
    T = lambda a: torch.tensor(np.asarray(a, float), dtype=torch.float64, device="cuda")
    ws = P.workspace(colloc.FP32_IR)
    _, jac, hess = P.derivs(T(x), T(y))
    rhs = P.assemble(ws, jac, hess, T(ref["sx"]), T(ref["ss"]), T([dw]), T(ref["rx"]), T(ref["rs"]),
                     T(ref["ry"]), precision=colloc.FP32_IR)
    info = P.factor(ws, colloc.FP32_IR)
    dx0 = P.solve(ws, rhs, colloc.FP32_IR)
    dx, sw = P.solve(ws, rhs, colloc.FP32_IR, ir_max=10, ir_tol=1e-14, sweeps=True)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0]
    ref_dx = _oracle_solve(m, ref["Kc"], ref["rhs"])
    e0 = rel_err(dx0.cpu().numpy(), ref_dx)
    nsw = int(sw.cpu().numpy()[0])
    print(f"{name}: FP32 step error {e0:.2e}; refined with {nsw} sweeps: "
          f"{rel_err(dx.cpu().numpy(), ref_dx):.2e}", flush=True)
    assert 1 <= nsw <= 10
    assert e0 < 1e-3
    _check_step(m, ref["Kc"], ref["rhs"], dx.cpu().numpy(), ref_dx)


def _solve(P, x0, opts, torch, max_steps=400):
    ws, state = P.workspace(opts.precision), P.state()
    P.ipm_init(torch.tensor(x0, dtype=torch.float64, device="cuda"), state, ws, opts)
    for calls in range(1, max_steps + 1):
        P.ipm_step(state, ws, opts)
        if calls % 5 == 0 and np.all(P.info(state)["status"] != colloc.RUNNING):
            break
    torch.cuda.synchronize()
    return state, P.info(state)


@pytest.mark.parametrize("name,tau_r", [("ab20", 1e-8), ("tiny", 1e-6)])
def test_ipm_fp32_ir_matches_oracle(torch, name, tau_r):
    announce(f"ipm fp32_ir {name}")
    inst = CASES[name]()
    m = problem.Model(inst, 3)
    x0 = workloads.initial_point(inst, 3)
    st_o = ipm.solve(m, x0, ipm.Options(tau_r=tau_r), solver="ldl")
    P = colloc.Problem(inst, 3)
    opts = colloc.default_opts(tau_r=tau_r, precision=colloc.FP32_IR)
    state, info = _solve(P, x0, opts, torch)
    info = info[0]
    th = P.state_vec(state, "x").cpu().numpy()[m.nz:]
    print(f"oracle status {st_o.status} it {st_o.it}; fp32_ir status {info['status']} it {info['iter']} "
          f"fallbacks {info['ir_fallbacks']} last sweeps {info['ir_sweeps']}", flush=True)
    assert info["status"] == st_o.status
    assert info["iter"] == st_o.it
    assert np.max(np.abs(th - st_o.x[m.nz:]) / np.maximum(1.0, np.abs(st_o.x[m.nz:]))) < 1e-6


def test_fp32_ir_batched_alone_equals_mix(torch):
    announce("ipm fp32_ir batched alone vs mix")
    insts = workloads.multistart_batch(3, 20, 60)
    opts = colloc.default_opts(precision=colloc.FP32_IR)
    P = colloc.Problem(insts, 3)
    x0 = np.concatenate([workloads.initial_point(i, 3) for i in insts])
    state, info = _solve(P, x0, opts, torch)
    xall = P.state_vec(state, "x").cpu().numpy()
    for q, inst in enumerate(insts):
        m = problem.Model(inst, 3)
        P1 = colloc.Problem(inst, 3)
        s1, i1 = _solve(P1, workloads.initial_point(inst, 3), opts, torch)
        assert np.array_equal(P1.state_vec(s1, "x").cpu().numpy(), xall[P.x_off[q]:P.x_off[q] + m.n])
        assert i1[0]["iter"] == info[q]["iter"]
        assert i1[0]["status"] == info[q]["status"]


@pytest.mark.parametrize("name", ["ab20"])
def test_ipm_fp32_ir_factors_used_when_conditioned(torch, name):
    """With a wide equality relaxation (tau_r = 1e-2, slack weights ~1e2) the condensed matrix is
    conditioned well enough for FP32 factors: iterations must be accepted on the FP32 factor after
    refinement (fewer FP64 fallbacks than iterations), and the solve still ends with the oracle's
    status and parameters.  (An accepted step is accurate to its backward-error target, not to the
    FP64 factor's rounding: on the 'tiny' instance at this tau_r the FP32_IR path leaves the
    oracle's after ~20 iterations, which is why that case is not asserted here.)"""
    announce(f"ipm fp32_ir factors used {name}")
    tau_r = 1e-2
    inst = CASES[name]()
    m = problem.Model(inst, 3)
    x0 = workloads.initial_point(inst, 3)
    st_o = ipm.solve(m, x0, ipm.Options(tau_r=tau_r), solver="ldl")
    P = colloc.Problem(inst, 3)
    state, info = _solve(P, x0, colloc.default_opts(tau_r=tau_r, precision=colloc.FP32_IR), torch)
    info = info[0]
    th = P.state_vec(state, "x").cpu().numpy()[m.nz:]
    print(f"oracle status {st_o.status} it {st_o.it}; fp32_ir status {info['status']} it {info['iter']} "
          f"fallbacks {info['ir_fallbacks']} last sweeps {info['ir_sweeps']}", flush=True)
    assert info["status"] == st_o.status
    assert info["ir_fallbacks"] < info["iter"]
    assert np.max(np.abs(th - st_o.x[m.nz:]) / np.maximum(1.0, np.abs(st_o.x[m.nz:]))) < 1e-6


def test_ipm_fp32_ir_without_sweeps_falls_back(torch):
    """ir_max = 0: no refinement can succeed, so the first FP32_IR iteration re-factors in FP64
    and counts a fallback (the instance then stays on FP64 factors); the solve ends like the FP64
    solve (status, iteration count, parameters within 1e-10)."""
    announce("ipm fp32_ir ir_max=0")
    inst = CASES["ab20"]()
    m = problem.Model(inst, 3)
    x0 = workloads.initial_point(inst, 3)
    P = colloc.Problem(inst, 3)
    s64, i64 = _solve(P, x0, colloc.default_opts(), torch)
    o32 = colloc.default_opts(precision=colloc.FP32_IR)
    o32.ir_max = 0
    s32, i32 = _solve(P, x0, o32, torch)
    i64, i32 = i64[0], i32[0]
    print(f"fp64 it {i64['iter']} status {i64['status']}; fp32_ir(ir_max=0) it {i32['iter']} "
          f"status {i32['status']} fallbacks {i32['ir_fallbacks']} tries {i32['factor_tries']}", flush=True)
    assert i32["status"] == i64["status"]
    assert i32["iter"] == i64["iter"]
    assert i32["ir_fallbacks"] >= 1
    th32 = P.state_vec(s32, "x").cpu().numpy()[m.nz:]
    th64 = P.state_vec(s64, "x").cpu().numpy()[m.nz:]
    assert np.max(np.abs(th32 - th64) / np.maximum(1.0, np.abs(th64))) < 1e-10
