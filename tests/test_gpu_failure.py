"""Failure paths, forced from the host so that every kernel still ends normally.

- A wall-clock limit (opts.max_wall_s) that has already passed ends the solve with
  COLLOC_TIMEOUT at its next decision, read from the device clock.
- A non-finite value written into one instance's iterate between iterations ends that instance
  with COLLOC_ENONFINITE; the other instance of the batch goes on exactly as it would alone
  (bitwise the same iterate and status).
"""
import numpy as np
import pytest

from paper_2607_12201_amd import colloc, workloads
from tests.gpu_helpers import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _steps(P, state, ws, opts, n):
    for _ in range(n):
        P.ipm_step(state, ws, opts)


def test_wall_clock_limit_gives_timeout(torch):
    announce("failure: wall-clock limit")
    inst = workloads.ab_reversible(0)
    P = colloc.Problem(inst, 3)
    x0 = torch.tensor(workloads.initial_point(inst, 3), dtype=torch.float64, device="cuda")
    opts = colloc.default_opts(max_wall_s=1e-9)
    ws, state = P.workspace(), P.state()
    P.ipm_init(x0, state, ws, opts)
    _steps(P, state, ws, opts, 3)
    info = P.info(state)[0]
    print(f"status {info['status']} iter {info['iter']}", flush=True)
    assert info["status"] == colloc.TIMEOUT
    assert info["iter"] == 0
    # without the limit the same start runs on
    opts0 = colloc.default_opts()
    ws, state = P.workspace(), P.state()
    P.ipm_init(x0, state, ws, opts0)
    _steps(P, state, ws, opts0, 3)
    assert P.info(state)[0]["status"] in (colloc.RUNNING, colloc.SOLVED)


def test_nonfinite_iterate_is_isolated(torch):
    announce("failure: NaN injected into one instance")
    insts = [workloads.ab_reversible(0), workloads.ab_reversible(1)]
    opts = colloc.default_opts()
    P = colloc.Problem(insts, 3)
    x0 = torch.tensor(np.concatenate([workloads.initial_point(i, 3) for i in insts]), dtype=torch.float64,
                      device="cuda")
    ws, state = P.workspace(), P.state()
    P.ipm_init(x0, state, ws, opts)
    for _ in range(40):   # advance to an iteration boundary of both instances
        P.ipm_step(state, ws, opts)
        info = P.info(state)
        if np.all(info["phase"] == 0) and info["iter"][0] >= 2:
            break
    assert np.all(info["status"] == colloc.RUNNING)
    x = P.state_vec(state, "x")
    x[int(P.x_off[0]) + 3] = float("nan")
    for k in range(400):
        P.ipm_step(state, ws, opts)
        if k % 5 == 4 and np.all(P.info(state)["status"] != colloc.RUNNING):
            break
    info = P.info(state)
    print(f"statuses {info['status'].tolist()} iterations {info['iter'].tolist()}", flush=True)
    assert info["status"][0] == colloc.ENONFINITE
    # instance 1 alone, same options
    P1 = colloc.Problem(insts[1], 3)
    ws1, st1 = P1.workspace(), P1.state()
    P1.ipm_init(torch.tensor(workloads.initial_point(insts[1], 3), dtype=torch.float64, device="cuda"), st1,
                ws1, opts)
    for k in range(400):
        P1.ipm_step(st1, ws1, opts)
        if k % 5 == 4 and P1.info(st1)[0]["status"] != colloc.RUNNING:
            break
    i1 = P1.info(st1)[0]
    assert info["status"][1] == i1["status"] and info["iter"][1] == i1["iter"]
    n1 = int(P.Ns[1]) * P.b + P.np_
    assert np.array_equal(P.state_vec(state, "x").cpu().numpy()[P.x_off[1]:P.x_off[1] + n1],
                          P1.state_vec(st1, "x").cpu().numpy())
