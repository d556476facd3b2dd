"""Writes net20_n1000_solve.npz: the oracle's whole interior-point solve of the 20-species,
40-reaction, N = 1000 instance (seed 0) with the default options (block Cholesky solver), the
final parameters, objective, status, iteration count and the condition number of the reduced
Hessian at its optimum.  Calls only the oracle and the seeded generator."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ipm, problem  # noqa: E402
from paper_2607_12201_amd import workloads  # noqa: E402


def main():
    inst = workloads.random_network(0)
    m = problem.Model(inst, 3)
    t0 = time.time()
    st = ipm.solve(m, workloads.initial_point(inst, 3), ipm.Options(), solver="block")
    H, kappa = ipm.reduced_hessian(m, st.x, st.y)
    np.savez(os.path.join(HERE, "net20_n1000_solve.npz"), theta=st.x[m.nz:], obj=m.objective(st.x),
             status=st.status, iters=st.it, kappa_reduced=kappa,
             tries=np.array([lg["tries"] for lg in st.log]))
    print(f"status {st.status} iterations {st.it} objective {m.objective(st.x):.12e} "
          f"reduced-Hessian kappa {kappa:.3e} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
