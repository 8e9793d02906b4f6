"""Write rb8192_rolls_100_oracle.json: the FP64 oracle's state of the 8192 x 4096 Rayleigh-Benard
lattice (Ra = 1e6, Pr = 0.71, Ma = 0.3; the footprint that does not fit the Infinity Cache) started
from convection rolls at half the convective velocity, after 100 steps, as sampled fields.

Run from the repository root: python tests/golden/make_rb8192_reference.py  (about 10 minutes on 8
cores, 8 GB of memory).  Only the oracle and the seeded input generator are called; the file holds

  - rho, u_x, u_y, T at 1024 nodes (the first 1024 of 4096 (y, x) pairs drawn with numpy's PCG64
    from seed 8192), and along the full columns x = 0 and x = 4095 (both walls, a roll's down- and
    upflow);
  - the scales max |u_x|, max |u_y|, max |T - T0| and max |rho - 1| of the whole field."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1710_10569_amd import workloads as W  # noqa: E402
from tests.helpers import oracle_from_workload  # noqa: E402

NX, NY, STEPS = 8192, 4096, 100
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rb8192_rolls_100_oracle.json")


def main():
    w = W.rayleigh_benard(nx=NX, ny=NY, rolls=0.5)
    o = oracle_from_workload(w)
    for k in range(10):
        o.step(STEPS // 10)
        print(f"{(k + 1) * STEPS // 10} steps", flush=True)
    rho, ux, uy, T = o.moments()
    o.close()
    rng = np.random.default_rng(8192)
    ys = rng.integers(0, NY, 4096)[:1024]
    xs = rng.integers(0, NX, 4096)[:1024]
    cols = [0, 4095]
    out = {"workload": w["name"], "steps": STEPS, "T0": w["T0"],
           "scale": {"ux": float(np.abs(ux).max()), "uy": float(np.abs(uy).max()),
                     "T": float(np.abs(T - w["T0"]).max()), "rho": float(np.abs(rho - 1).max())},
           "samples": {"y": ys.tolist(), "x": xs.tolist(), "rho": rho[ys, xs].tolist(),
                       "ux": ux[ys, xs].tolist(), "uy": uy[ys, xs].tolist(), "T": T[ys, xs].tolist()},
           "columns": {"x": cols, "rho": rho[:, cols].T.tolist(), "ux": ux[:, cols].T.tolist(),
                       "uy": uy[:, cols].T.tolist(), "T": T[:, cols].T.tolist()}}
    with open(OUT, "w") as fh:
        json.dump(out, fh)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
