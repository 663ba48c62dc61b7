"""Write oracle reference values for confluent and nearly confluent spectra at the molecule
workload's shape (N=36, J=4000, dt=0.02, Fourier K=16, P=32): cost, gradient and Hessian of
the first two thetas of a batch of 256, for each system of inputs.degenerate_system.

Calls only the CPU oracle (oracle/) and the seeded input generators; run from the repo root:

    python tests/golden/make_golden_degenerate.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import qoc_oracle as O  # noqa: E402
from paper_2505_00529_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "degenerate_oracle.json")

N, NT, DT, K = 36, 4000, 0.02, 16
BATCH = 256
# (system kind, theta scale, theta seed): a weak field keeps the near-crossing pair within
# about 1e-9 of each other on every step
CASES = [("doubled", 0.1, 21), ("near_crossing", 1e-8, 22), ("h0zero", 0.1, 23)]


def main():
    basis = O.fourier_basis(NT, DT, K)
    gamma, rho = 2.0 * DT, 2.0
    out = []
    for kind, sigma, seed in CASES:
        s = inputs.degenerate_system(kind, N)
        thetas = inputs.draw_thetas(2 * K, 2, seed, sigma=sigma)
        for i, th in enumerate(thetas):
            t0 = time.time()
            c, g, h = O.cost_grad_hess(s.h0, s.m, s.psi0, s.psi_target, basis, DT, th, gamma, rho)
            out.append({"kind": kind, "sigma": sigma, "seed": seed, "theta_index": i,
                        "cost": c, "grad": g.tolist(), "hess": h.tolist()})
            print(f"{kind} theta {i}: {time.time() - t0:.1f} s", flush=True)
    doc = {
        "n": N, "nt": NT, "dt": DT, "k": K, "gamma": gamma, "rho": rho, "batch": BATCH,
        "source": "oracle/qoc_oracle.py cost_grad_hess on inputs.degenerate_system(kind, 36); "
                  "thetas = rows of inputs.draw_thetas(P, batch, seed, sigma)",
        "cases": out,
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
