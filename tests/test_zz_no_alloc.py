"""colloc_eval_noalloc (static device scratch, no workspace, no allocation) against colloc_eval:
bitwise the same objective and constraint values on two calls in a row, the second on a smaller
problem, and a handle beyond the scratch limit rejected before anything runs."""
import numpy as np
import pytest

from paper_2607_12201_amd import colloc, workloads
from tests.gpu_helpers import announce, need_gpu

pytestmark = pytest.mark.gpu


def test_noalloc_eval_equals_eval():
    torch = need_gpu()
    rng = np.random.default_rng(11)
    for name, inst in (("net20_n1000", workloads.random_network(0)),
                       ("tiny", workloads.random_network(5, n_s=4, n_r=7, N=3, n_obs=2, n_times=3, n_fixed=2))):
        announce(f"colloc_eval_noalloc {name}")
        P = colloc.Problem(inst, 3)
        x = workloads.initial_point(inst, 3) + 0.01 * rng.standard_normal(P.n_total)
        xd = torch.tensor(x, dtype=torch.float64, device="cuda")
        ws = P.workspace()
        obj_ref, g_ref = P.eval(xd, ws)
        obj = torch.full((P.n_inst,), np.nan, dtype=torch.float64, device="cuda")
        g = torch.full((P.m_total,), np.nan, dtype=torch.float64, device="cuda")
        assert P.eval_noalloc(xd, obj, g) == colloc.OK
        torch.cuda.synchronize()
        assert torch.equal(obj, obj_ref) and torch.equal(g, g_ref), name


def test_noalloc_rejects_beyond_scratch():
    torch = need_gpu()
    announce("colloc_eval_noalloc size limit")
    inst = workloads.ab_reversible(0, N=20)
    n_big = (colloc.NOALLOC_MAX_ELEMS // 10 + 1) * 10
    big = workloads.ab_reversible(0, N=n_big)
    P = colloc.Problem(big, 3)
    assert P.n_elem > colloc.NOALLOC_MAX_ELEMS
    xd = torch.zeros(P.n_total, dtype=torch.float64, device="cuda")
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.zeros(P.m_total, dtype=torch.float64, device="cuda")
    assert P.eval_noalloc(xd, obj, g) == colloc.EINVAL
    del inst
