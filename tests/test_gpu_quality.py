"""Solution quality of GPU solves, by the analog of the paper's relative objective gap (ROG):
the sequential objective Phi_seq (the least-squares objective on a high-accuracy stiff ODE
solution) at the GPU's estimate against Phi_seq at the oracle's estimate.  The paper flags a
solve as suboptimal when ROG > 0.02.  The sequential objective at the GPU's estimate must also
agree with the collocation objective there within 0.02 on these meshes (collocation accuracy)."""
import numpy as np
import pytest

from oracle import ipm, problem
from paper_2607_12201_amd import colloc, quality, workloads
from tests.gpu_helpers import CASES, announce, need_gpu
from tests.test_gpu_ipm import run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return need_gpu()


@pytest.mark.parametrize("name,tau_r", [("ab20", 1e-8), ("ragged37", 1e-6)])
def test_relative_objective_gap_against_oracle(torch, name, tau_r):
    announce(f"relative objective gap {name}")
    inst = CASES[name]()
    m = problem.Model(inst, 3)
    x0 = workloads.initial_point(inst, 3)
    st_o = ipm.solve(m, x0, ipm.Options(tau_r=tau_r), solver="ldl")
    P = colloc.Problem(inst, 3)
    state, info, _ = run_gpu(P, x0, colloc.default_opts(tau_r=tau_r), torch)
    assert info[0]["status"] == st_o.status == ipm.SOLVED
    x = P.state_vec(state, "x").cpu().numpy()
    th, th_o = x[m.nz:], st_o.x[m.nz:]
    rog = quality.relative_objective_gap(inst, th, th_o)
    phi_seq, phi_col = quality.sequential_objective(inst, th), m.objective(x)
    print(f"ROG {rog:.2e}; Phi_seq {phi_seq:.6e}, Phi_colloc {phi_col:.6e}", flush=True)
    assert rog <= 0.02
    assert abs(phi_seq - phi_col) <= 0.02 * abs(phi_col)
