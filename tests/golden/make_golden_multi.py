"""Write oracle reference values for the three-direction workload (the molecule workload N=36,
J=4000, K=16 with three control operators, a Fourier block per direction, P=96): two thetas
(the first rows of the benchmark's batch) with cost, gradient and Hessian.

Calls only the CPU oracle (oracle/) and the seeded input generators; run from the repo root:
    python tests/golden/make_golden_multi.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import qoc_oracle as O  # noqa: E402
from paper_2505_00529_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    out = os.path.join(HERE, "multi_oracle.json")
    w, ms = inputs.multi_direction_workload()
    s = w.system
    ndir = len(ms)
    b0 = O.fourier_basis(w.nt, w.dt, w.k)
    p0 = b0.shape[1]
    bases = np.zeros((ndir, w.nt, ndir * p0))
    for c in range(ndir):
        bases[c, :, c * p0:(c + 1) * p0] = b0
    thetas = inputs.draw_thetas(ndir * p0, 2, w.seed)
    cases = []
    for i, th in enumerate(thetas):
        t0 = time.time()
        c, g, h = O.cost_grad_hess_multi(s.h0, ms, s.psi0, s.psi_target, bases, w.dt, th, w.gamma, w.rho)
        cases.append({"theta_index": i, "cost": c, "grad": g.tolist(), "hess": h.tolist()})
        print(f"theta {i}: {time.time() - t0:.1f} s", flush=True)
    doc = {
        "workload": "multi", "n": s.n, "nt": w.nt, "dt": w.dt, "k": w.k, "directions": ndir,
        "gamma": w.gamma, "rho": w.rho, "seed": w.seed,
        "source": "oracle/qoc_oracle.py cost_grad_hess_multi; operators = inputs.multi_direction_workload(), "
                  "a Fourier block per direction; thetas = inputs.draw_thetas(P, 2, seed)",
        "cases": cases,
    }
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
