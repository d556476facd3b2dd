"""Continuous-batching serving loop.

Requests of uneven network size and mesh arrive while others are on the device; they are
admitted under an HBM budget, join and leave batches at step boundaries, and every request's
result (status, iteration count, final iterate) must equal its result alone, bit for bit.
The budget is set so that not everything fits at once, so admission really waits.
"""
import numpy as np
import pytest

from paper_2607_12201_amd import colloc, serving, workloads
from tests.gpu_helpers import announce, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


def _trace():
    arrivals, insts = workloads.serving_trace(10, rate=200.0, seed=3, ns_lo=3, ns_hi=4, N_lo=50,
                                              N_hi=150)
    return [serving.Request(q, float(a), inst) for q, (a, inst) in enumerate(zip(arrivals, insts))]


@pytest.mark.parametrize("precision", [colloc.FP64, colloc.FP32_IR])
def test_serving_results_equal_alone(torch, precision):
    announce(f"serving alone vs mix precision={precision}")
    reqs = _trace()
    opts = colloc.default_opts(precision=precision)
    need = [serving.request_bytes(r.inst, 3, precision) for r in reqs]
    budget = int(sum(need) * 0.6)          # forces admission to wait for memory
    assert max(need) <= budget
    res = serving.serve(reqs, opts, budget, steps_per_round=3)
    assert res.peak_bytes <= 1.5 * budget
    assert len({r.shape for r in reqs}) >= 2
    waited = [r for r in reqs if r.t_admit > r.arrival + 1e-3]
    print(res.summary(), f"waited {len(waited)}", flush=True)
    for r in reqs:
        st, it, x, obj, _ = serving.solve_alone(r.inst, opts)
        assert r.status == st, r.rid
        assert r.iters == it, r.rid
        assert np.array_equal(r.x, x), r.rid
        assert r.status != colloc.RUNNING
        assert r.t_done >= r.t_admit >= r.arrival
