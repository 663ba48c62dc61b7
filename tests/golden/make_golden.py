"""Write oracle reference values for a full-size workload: the molecule workload (N=36,
J=4000, K=16) by default, or the 64-level warm-start system (N=64, J=4000, K=32) with
argument "warm".  Two thetas (the first rows of the benchmark's batch) with cost, gradient
and Hessian, and one HVP for the first.

Calls only the CPU oracle (oracle/) and the seeded input generators; run from the repo
root:  python tests/golden/make_golden.py [molecule|warm]
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


def main(name="molecule"):
    out = os.path.join(HERE, f"{name}_oracle.json")
    w = inputs.make_workload(name)
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    args = (s.h0, s.m, s.psi0, s.psi_target, basis, w.dt)
    thetas = inputs.draw_thetas(w.p, 2, w.seed)
    vs = inputs.draw_directions(w.p, 1, w.seed)
    cases = []
    for i, th in enumerate(thetas):
        t0 = time.time()
        c, g, h = O.cost_grad_hess(*args, th, w.gamma, w.rho)
        case = {"theta_index": i, "cost": c, "grad": g.tolist(), "hess": h.tolist()}
        if i == 0:
            hv = O.hvp(*args, th, vs[0], w.gamma, w.rho)
            case["v_index"] = 0
            case["hvp"] = hv.tolist()
        cases.append(case)
        print(f"theta {i}: {time.time() - t0:.1f} s", flush=True)
    doc = {
        "workload": name, "n": w.system.n, "nt": w.nt, "dt": w.dt, "k": w.k,
        "gamma": w.gamma, "rho": w.rho, "seed": w.seed,
        "source": "oracle/qoc_oracle.py cost_grad_hess and hvp; thetas = inputs.draw_thetas(P, 2, seed), "
                  "v = inputs.draw_directions(P, 1, seed)",
        "cases": cases,
    }
    with open(out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "molecule")
