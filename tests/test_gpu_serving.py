"""Continuous-batching serving loop.

Requests of uneven network size and mesh arrive while others are on the device; they are
admitted under an HBM budget, join and leave batches at step boundaries, and every request's
result (status, iteration count, final iterate) must equal its result alone, bit for bit, and
the oracle's (status; parameters within 1e-6 when solved).  The budget is set so that not
everything fits at once, so admission really waits; the device memory held (every batch and
every rebuild, by the library's sizes and by the allocator's own peak) stays within it.
"""
import numpy as np
import pytest

from oracle import ipm, problem
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
    need = [serving.admit_bytes([r.inst], 3, precision) for r in reqs]
    budget = int(sum(need) * 0.6)          # forces admission to wait for memory
    assert max(need) <= budget
    res = serving.serve(reqs, opts, budget, steps_per_round=3)
    assert res.peak_bytes <= budget
    assert res.peak_allocator_bytes <= budget
    assert len({r.shape for r in reqs}) >= 2
    waited = [r for r in reqs if r.t_admit > r.arrival + 1e-3]
    print(res.summary(), f"waited {len(waited)}", flush=True)
    assert waited
    for r in reqs:
        st, it, x, obj, _ = serving.solve_alone(r.inst, opts)
        assert r.status == st, r.rid
        assert r.iters == it, r.rid
        assert np.array_equal(r.x, x), r.rid
        assert r.status != colloc.RUNNING
        assert r.t_done >= r.t_admit >= r.arrival


def test_served_results_against_oracle(torch):
    """Served results against the oracle, on instances whose single solves are parity-tested
    (tiny, ragged37 at tau_r = 1e-6): two copies of each arrive while the others run, under a
    budget that makes them wait.  Each served result must end SOLVED like the oracle's solve,
    with the parameter rule of the solve parity tests: parameters within 1e-6 where the oracle's
    reduced Hessian at its optimum has condition number <= 1e6, else the objective within 1e-10."""
    announce("serving vs oracle")
    from tests.gpu_helpers import CASES
    tau_r = 1e-6
    insts = [CASES["tiny"](), CASES["ragged37"](), CASES["tiny"](), CASES["ragged37"]()]
    reqs = [serving.Request(q, 0.002 * q, inst) for q, inst in enumerate(insts)]
    opts = colloc.default_opts(tau_r=tau_r)
    need = [serving.admit_bytes([r.inst], 3, colloc.FP64) for r in reqs]
    budget = max(need) + min(need)
    res = serving.serve(reqs, opts, budget, steps_per_round=3)
    assert res.peak_bytes <= budget and res.peak_allocator_bytes <= budget
    ref = {}
    for r in reqs:
        name = "tiny" if r.inst is insts[0] or r.inst is insts[2] else "ragged37"
        m = problem.Model(r.inst, 3)
        if name not in ref:
            st_o = ipm.solve(m, workloads.initial_point(r.inst, 3), ipm.Options(tau_r=tau_r), solver="ldl")
            _, kappa = ipm.reduced_hessian(m, st_o.x, st_o.y)
            ref[name] = (st_o, kappa)
        st_o, kappa = ref[name]
        th, tho = r.x[m.nz:], st_o.x[m.nz:]
        dth = float(np.max(np.abs(th - tho) / np.maximum(1.0, np.abs(tho))))
        phi_o = m.objective(st_o.x)
        print(f"request {r.rid} ({name}): status {r.status} (oracle {st_o.status}), iterations {r.iters} "
              f"(oracle {st_o.it}), kappa {kappa:.2e}, parameter difference {dth:.2e}, objective "
              f"{r.obj:.12e} (oracle {phi_o:.12e})", flush=True)
        assert r.status == st_o.status == ipm.SOLVED, r.rid
        if kappa <= 1e6:
            assert dth < 1e-6, r.rid
        else:
            assert abs(r.obj - phi_o) <= 1e-10 * max(1.0, abs(phi_o)), r.rid
