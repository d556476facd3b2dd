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


def test_refinement_step_warm_start(torch):
    """One step of a mesh-refinement outer loop on the GPU: ragged37 (N = 37) is solved, its mesh
    halved with the warm start interpolated from the solution (quality.refine_uniform), and the
    refined problem (N = 74) solved from there.  The refined solve ends SOLVED in fewer
    iterations than the cold one, and the two estimates are within the paper's 0.02 by the
    relative objective gap."""
    announce("refinement step ragged37")
    tau_r = 1e-6
    inst = CASES["ragged37"]()
    m = problem.Model(inst, 3)
    opts = colloc.default_opts(tau_r=tau_r)
    P = colloc.Problem(inst, 3)
    state, info, _ = run_gpu(P, workloads.initial_point(inst, 3), opts, torch)
    assert info[0]["status"] == ipm.SOLVED
    x = P.state_vec(state, "x").cpu().numpy()
    new, x0 = quality.refine_uniform(inst, 3, x)
    assert new["N"] == 2 * inst["N"] and len(x0) == 2 * inst["N"] * 4 * inst["n_s"] + inst["n_p"]
    P2 = colloc.Problem(new, 3)
    state2, info2, _ = run_gpu(P2, x0, opts, torch)
    x2 = P2.state_vec(state2, "x").cpu().numpy()
    rog = quality.relative_objective_gap(inst, x2[-inst["n_p"]:], x[m.nz:])
    print(f"coarse: {info[0]['iter']} iterations; refined: status {info2[0]['status']}, "
          f"{info2[0]['iter']} iterations; ROG {rog:.2e}", flush=True)
    assert info2[0]["status"] == ipm.SOLVED
    assert info2[0]["iter"] < info[0]["iter"]
    assert rog <= 0.02
