"""Write cavity256_50k_oracle.json: the FP64 oracle's state of the 256 x 256 differentially heated
cavity (Ra = 1e5, Pr = 0.71, Ma = 0.1, seeded initial noise) after 50 000 steps, as sampled fields.

Run from the repository root: python tests/golden/make_cavity256_reference.py  (about 4 minutes on
8 cores).  Only the oracle and the seeded input generator are called; the file holds

  - the hot-wall (west) columns x = 0, 1, 2 of T, from which the wall Nusselt number follows;
  - rho, u_x, u_y, T at 512 nodes drawn with numpy's PCG64 from seed 256;
  - the scales max |u_x|, max |u_y| and max |T - T0| of the whole field."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1710_10569_amd import workloads as W  # noqa: E402
from tests.helpers import oracle_from_workload  # noqa: E402

STEPS = 50_000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cavity256_50k_oracle.json")


def main():
    w = W.cavity(256)
    o = oracle_from_workload(w)
    for k in range(10):
        o.step(STEPS // 10)
        print(f"{(k + 1) * STEPS // 10} steps", flush=True)
    rho, ux, uy, T = o.moments()
    rng = np.random.default_rng(256)
    ys = rng.integers(0, w["ny"], 512)
    xs = rng.integers(0, w["nx"], 512)
    out = {"workload": w["name"], "steps": STEPS, "T0": w["T0"],
           "scale": {"ux": float(np.abs(ux).max()), "uy": float(np.abs(uy).max()),
                     "T": float(np.abs(T - w["T0"]).max())},
           "hot_wall_T": T[:, :3].tolist(),
           "samples": {"y": ys.tolist(), "x": xs.tolist(), "rho": rho[ys, xs].tolist(),
                       "ux": ux[ys, xs].tolist(), "uy": uy[ys, xs].tolist(), "T": T[ys, xs].tolist()}}
    with open(OUT, "w") as fh:
        json.dump(out, fh)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
