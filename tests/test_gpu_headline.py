"""The benchmark's headline instance at its full size, on the path the benchmark times: the
100-species stiff network (250 reactions, 200 estimated parameters), N = 10,000 elements, K = 3,
4,000,200 variables, the tiled matrix-core factorization, from the benchmark's starting point.

- eval and derivatives: every entry against the oracle, whose NLP functions are vectorized over
  the elements and run at this size (the same bars as the small parity cases);
- assemble / factor / solve on a positive-definite state (multipliers zero, Sx = Ss = 1,
  dw = 1): the factor succeeds, and the step's normwise backward error against the library's
  matrix-free product K v (a code path separate from the assembly and the factorization: it
  works from the derivative values) is <= 1e-10, with ||K||_inf bounded below by |K 1|_inf and
  |K dx|_inf / |dx|_inf, and the residual is <= 1e-10 of the right-hand side (K >= 2 I at this
  state).  The oracle's condensed matrix has ~5e9 nonzeros at this size, so the step is judged by
  these properties instead of against an oracle solve.
"""
import copy

import numpy as np
import pytest

from oracle import problem
from paper_2607_12201_amd import colloc, workloads
from tests.gpu_helpers import announce, assert_elementwise, need_gpu, term_scales

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


@pytest.fixture(scope="module")
def headline(torch):
    inst = workloads.stiff_network(0)
    x0 = workloads.initial_point(inst, 3)
    P = colloc.Problem(inst, 3)
    return inst, problem.Model(inst, 3), P, x0


def _T(torch, a):
    return torch.tensor(np.asarray(a, float), dtype=torch.float64, device="cuda")


def test_headline_eval_and_derivs(torch, headline):
    inst, m, P, x0 = headline
    announce("headline eval/derivs (100 species, N=10000)")
    y = np.random.default_rng(7).standard_normal(m.m)
    ws = P.workspace()
    obj, g = P.eval(_T(torch, x0), ws)
    grad, jac, hess = P.derivs(_T(torch, x0), _T(torch, y))
    torch.cuda.synchronize()
    gscale, grscale = term_scales(m, x0)
    assert_elementwise(g.cpu().numpy(), m.constraints(x0), gscale, 1e-13, "g")
    assert abs(obj.item() - m.objective(x0)) <= 1e-12 * max(1.0, m.objective(x0))
    assert_elementwise(grad.cpu().numpy(), m.gradient(x0), grscale, 1e-13, "grad")
    jo, ho = m.pattern_values(x0, y)
    assert_elementwise(jac.cpu().numpy(), jo.ravel(), 0.0, 1e-14, "jac")
    ma = copy.copy(m)
    ma.nu = np.abs(m.nu)
    _, ho_abs = ma.pattern_values(x0, np.abs(y))
    assert_elementwise(hess.cpu().numpy(), ho.ravel(), np.abs(ho_abs).ravel(), 1e-14, "hess")
    del ws
    torch.cuda.empty_cache()


def test_headline_step_backward_error(torch, headline):
    inst, m, P, x0 = headline
    announce("headline assemble/factor/solve (100 species, N=10000)")
    rng = np.random.default_rng(8)
    T = lambda a: _T(torch, a)
    ws = P.workspace()
    _, jac, hess = P.derivs(T(x0), T(np.zeros(m.m)))
    rhs = P.assemble(ws, jac, hess, T(np.ones(m.n)), T(np.ones(m.m)), T([1.0]), T(rng.standard_normal(m.n)),
                     T(rng.standard_normal(m.m)), T(rng.standard_normal(m.m)))
    info = P.factor(ws)
    dx = P.solve(ws, rhs)
    Kdx = P.matvec(ws, dx)
    K1 = P.matvec(ws, T(np.ones(m.n)))
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0]
    dx, Kdx, rhs, K1 = (v.cpu().numpy() for v in (dx, Kdx, rhs, K1))
    assert np.all(np.isfinite(dx))
    knorm = max(np.max(np.abs(K1)), np.max(np.abs(Kdx)) / np.max(np.abs(dx)))
    berr = np.max(np.abs(Kdx - rhs)) / (knorm * np.max(np.abs(dx)) + np.max(np.abs(rhs)))
    print(f"backward error {berr:.3e}: |r| {np.max(np.abs(Kdx - rhs)):.3e} |K| >= {knorm:.3e} "
          f"|dx| {np.max(np.abs(dx)):.3e} |rhs| {np.max(np.abs(rhs)):.3e}", flush=True)
    assert berr <= 1e-10
    # at this state K >= 2 I (Sx + dw on the diagonal, the rest positive semidefinite), so the
    # residual of a correct factor stays at rounding level against the right-hand side too
    assert np.max(np.abs(Kdx - rhs)) <= 1e-10 * np.max(np.abs(rhs))
    del ws
    torch.cuda.empty_cache()
