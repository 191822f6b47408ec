"""Writes c3_oracle_solves.json: the CPU oracle's BF solves of the 3D
128x128x64 workload (1,048,576 cells, sigma 3, five-spot, CFL 10) to a 1e-8
relative residual, at the initial condition of the time step and at the
oracle's own Newton iterate 1 (one oracle Newton step from it, saturation
chop 0.2).  Stored: iteration counts, true relative residuals, norms, and
the solution at 4,096 seeded sample indices.  Calls only the oracle and the
input generator.

Usage (from the repository root, about 5 minutes on one core):
    python tests/golden/make_c3_oracle_solves.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import newton, tpfa  # noqa: E402
from paper_1611_00127_amd import inputs  # noqa: E402

DS_MAX = 0.2
N_SAMPLES = 4096


def record(c, x, info):
    rp, ci, v = tpfa.jacobian(c, c.u, c.u_old)
    b = -tpfa.residual(c, c.u, c.u_old).reshape(-1)
    J = tpfa.bcsr_matrix(rp, ci, v)
    rel = float(np.linalg.norm(b - J @ x) / np.linalg.norm(b))
    idx = np.sort(np.random.Generator(np.random.PCG64(2024)).choice(len(x), N_SAMPLES,
                                                                    replace=False))
    return {"iterations": int(info["iterations"]), "relres_true": rel,
            "norm_b": float(np.linalg.norm(b)), "norm_x": float(np.linalg.norm(x)),
            "max_abs_x": float(np.max(np.abs(x))),
            "sample_index": idx.tolist(), "sample_x": x[idx].tolist()}


def main():
    c = inputs.config_c3()
    out = {"workload": "3d-128x128x64 config_c3(), BF, FGMRES(30), rtol 1e-8, oracle FP64",
           "note": "right-hand side b = -F(u); x solves J x = b", "states": {}}
    t0 = time.time()
    x0, info0, _ = newton.solve(c, "bf", rtol=1e-8)
    out["states"]["initial"] = record(c, x0, info0)
    print(f"initial: {info0['iterations']} its, {time.time() - t0:.0f} s", flush=True)
    c1 = c.replace(u=newton.update(c.u, x0, DS_MAX))
    t0 = time.time()
    x1, info1, _ = newton.solve(c1, "bf", rtol=1e-8)
    out["states"]["newton1"] = record(c1, x1, info1)
    print(f"newton1: {info1['iterations']} its, {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle_solves.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
