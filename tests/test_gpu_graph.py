"""Graph-captured interior-point steps: every replay equals the eager steps bitwise.

A batch of uneven instances runs 12 eager ipm_step calls; a second state, initialised the same
way, replays a captured 4-step graph three times with eager library and torch work between the
replays.  After each replay its iterate must equal the eager iterate after the same number of
steps, bit for bit.
"""
import numpy as np
import pytest

from paper_2607_12201_amd import colloc, workloads
from tests.gpu_helpers import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


@pytest.mark.parametrize("precision", [colloc.FP64, colloc.FP32_IR])
def test_graph_replays_equal_eager(torch, precision):
    announce(f"graph replay precision={precision}")
    insts = workloads.multistart_batch(3, 20, 60)
    P = colloc.Problem(insts, 3)
    opts = colloc.default_opts(precision=precision)
    x0 = torch.tensor(np.concatenate([workloads.initial_point(i, 3) for i in insts]),
                      dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ws_e, st_e = P.workspace(precision), P.state()
        P.ipm_init(x0, st_e, ws_e, opts)
        eager = []
        for k in range(12):
            P.ipm_step(st_e, ws_e, opts)
            if k % 4 == 3:
                eager.append((P.state_vec(st_e, "x").clone(), P.info(st_e).copy()))
        ws_g, st_g = P.workspace(precision), P.state()
        P.ipm_init(x0, st_g, ws_g, opts)
        g = P.graph_create(st_g, ws_g, opts, steps=4)
        try:
            for rep in range(3):
                P.graph_launch(g)
                side.synchronize()
                x = P.state_vec(st_g, "x")
                assert torch.equal(x, eager[rep][0]), f"replay {rep}"
                info = P.info(st_g)
                assert np.array_equal(info["iter"], eager[rep][1]["iter"])
                assert np.array_equal(info["status"], eager[rep][1]["status"])
                # unrelated eager work between replays
                P.eval(x0, ws_e)
                torch.cuda.synchronize()
        finally:
            P.graph_destroy(g)
