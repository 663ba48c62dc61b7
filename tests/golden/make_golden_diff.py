"""Write oracle reference values for the full-size differentiation workload
(N=128, J=10^4, dt=0.01, Fourier K=64, P=128): the cost, the gradient and three
Hessian-vector products at the workload's theta and directions.

Calls only the CPU oracle (oracle/) and the seeded input generators.  The four
forward-mode passes are independent and run in separate processes (about 5 minutes
each on two BLAS threads); run from the repo root:

    python tests/golden/make_golden_diff.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "diff_oracle.json")
THREADS_PER_TASK = 2


def _task(which):
    os.environ["OPENBLAS_NUM_THREADS"] = str(THREADS_PER_TASK)
    os.environ["OMP_NUM_THREADS"] = str(THREADS_PER_TASK)
    from oracle import qoc_oracle as O
    from paper_2505_00529_amd import inputs

    w = inputs.make_workload("diff")
    s = w.system
    basis = O.fourier_basis(w.nt, w.dt, w.k)
    th = inputs.draw_thetas(w.p, 1, w.seed)[0]
    vs = inputs.draw_directions(w.p, 3, w.seed)
    args = (s.h0, s.m, s.psi0, s.psi_target, basis, w.dt, th)
    t0 = time.time()
    if which == "grad":
        c, g = O.cost_grad(*args, w.gamma, w.rho)
        out = {"cost": c, "grad": g.tolist()}
    else:
        i = int(which[3:])
        out = {"v_index": i, "hvp": O.hvp(*args, vs[i], w.gamma, w.rho).tolist()}
    print(f"{which}: {time.time() - t0:.0f} s", flush=True)
    return which, out


def main():
    import multiprocessing as mp

    from paper_2505_00529_amd import inputs

    w = inputs.make_workload("diff")
    ctx = mp.get_context("spawn")
    with ctx.Pool(4) as pool:
        res = dict(pool.map(_task, ["grad", "hvp0", "hvp1", "hvp2"]))
    doc = {
        "workload": "diff", "n": w.system.n, "nt": w.nt, "dt": w.dt, "k": w.k,
        "gamma": w.gamma, "rho": w.rho, "seed": w.seed,
        "source": "oracle/qoc_oracle.py cost_grad and hvp; theta = inputs.draw_thetas(P, 1, seed)[0], "
                  "v_i = inputs.draw_directions(P, 3, seed)[i]",
        "cost": res["grad"]["cost"],
        "grad": res["grad"]["grad"],
        "hvps": [res[f"hvp{i}"] for i in range(3)],
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
