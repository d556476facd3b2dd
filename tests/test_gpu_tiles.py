"""Thread-grid choices of the elimination kernels and the autotuner.

- Every usable thread grid gives the same Newton step, bit for bit (the grid moves entries
  between threads; each entry's arithmetic is unchanged).
- The autotuner picks a usable grid per kernel and caches it by shape class.
"""
import json

import numpy as np
import pytest

from oracle import problem
from paper_2607_12201_amd import autotune, colloc
from tests.gpu_helpers import CASES, announce, need_gpu, oracle_kkt, random_state
from tests.test_gpu_parity import _check_step, _oracle_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


@pytest.mark.parametrize("name", ["ab20", "ragged37", "net20_n1000"])
def test_every_tile_gives_the_same_step(torch, name):
    """All TS x TS grids of a kernel give the same step bit for bit; the blocked LDS variant of
    the chain kernel (TS = 1, different rounding order) meets the step bar against the oracle."""
    announce(f"tiles {name}")
    inst = CASES[name]()
    m = problem.Model(inst, 3)
    P = colloc.Problem(inst, 3)
    rng = np.random.default_rng(21)
    x, s, y, zL, zU, vL, vU = random_state(m, rng, 1.0)
    ref = oracle_kkt(m, x, s, y, zL, zU, vL, vU, 0.1, 1.0, 2.0)
    T = lambda a: torch.tensor(np.asarray(a, float), dtype=torch.float64, device="cuda")
    ws = P.workspace()
    _, jac, hess = P.derivs(T(x), T(y))
    rhs = P.assemble(ws, jac, hess, T(ref["sx"]), T(ref["ss"]), T([2.0]), T(ref["rx"]), T(ref["rs"]),
                     T(ref["ry"]))
    opts = {k: P.tile_options(k) for k in colloc.Problem.TILE_KERNELS}
    assert all(len(v) >= 1 for v in opts.values()), opts

    def step():
        P.assemble(ws, jac, hess, T(ref["sx"]), T(ref["ss"]), T([2.0]), T(ref["rx"]), T(ref["rs"]),
                   T(ref["ry"]))
        info = P.factor(ws)
        dx = P.solve(ws, rhs)
        torch.cuda.synchronize()
        assert info.cpu().numpy().tolist() == [0]
        return dx

    # a grid for the chain so that the comparisons below isolate one kernel at a time
    grid_chain = [t for t in opts["chain"] if t != 1][0]
    P.tile_set("chain", grid_chain)
    base = step().clone()
    for which in colloc.Problem.TILE_KERNELS:
        for ts in opts[which]:
            P.tile_set(which, ts)
            assert P.tile_get(which) == ts
            dx = step()
            if ts == 1:
                _check_step(m, ref["Kc"], ref["rhs"], dx.cpu().numpy(), _oracle_solve(m, ref["Kc"], ref["rhs"]))
            else:
                assert torch.equal(dx, base), (which, ts)
        P.tile_set(which, grid_chain if which == "chain" else 0)
    with pytest.raises(RuntimeError):
        P.tile_set("level0", 40)


def test_autotune_picks_and_caches(torch, tmp_path):
    announce("autotune ragged37")
    inst = CASES["ragged37"]()
    P = colloc.Problem(inst, 3)
    path = str(tmp_path / "tiles.json")
    res = autotune.tune(P, cache_path=path, reps=2)
    for which in colloc.Problem.TILE_KERNELS:
        assert res[which] in P.tile_options(which)
        assert P.tile_get(which) == res[which]
    data = json.load(open(path))
    assert len(data) == 1
    P2 = colloc.Problem(inst, 3)
    res2 = autotune.tune(P2, cache_path=path)
    assert all(P2.tile_get(w) == res[w] for w in colloc.Problem.TILE_KERNELS)
    assert res2 == res
