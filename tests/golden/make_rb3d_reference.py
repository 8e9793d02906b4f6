"""Write rb3d_rolls_50_oracle.json: the FP64 oracle's state of the 256 x 256 x 129 Rayleigh-Benard
layer (D3Q27 flow, D3Q7 temperature; Ra = 1e5, Pr = 0.71, Ma = 0.1) started from crossed
convection rolls at half the convective velocity, after 50 steps, as sampled fields.

Run from the repository root: python tests/golden/make_rb3d_reference.py  (about 8 minutes on 8
cores, 6 GB of memory).  Only the oracle and the seeded input generator are called; the file holds

  - rho, u_x, u_y, u_z, T at 1024 nodes (the first 1024 of 4096 (z, y, x) triples drawn with numpy's
    PCG64 from seed 129), and along the full wall-to-wall columns at (x, y) = (0, 0) and (100, 37);
  - the scales max |u| over the three components, max |T - T0| and max |rho - 1| of the whole field."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import o3d  # noqa: E402
from paper_1710_10569_amd import workloads as W  # noqa: E402

SHAPE, STEPS = (256, 256, 129), 50
COLUMNS = [(0, 0), (100, 37)]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rb3d_rolls_50_oracle.json")


def main():
    w = W.rayleigh_benard_3d(*SHAPE, Ra=1e5, Ma=0.1, seed=3, rolls=0.5)
    p = w["physics"]
    w = dict(w, taus=dict(zip(("tau_nu", "tau_alpha", "g_beta"),
                              O.params_from_physics(p["Ra"], p["Pr"], p["Ma"], p["H"], p["dT"]))))
    L = o3d.lattice_from_workload(w)
    for k in range(10):
        L.step(STEPS // 10)
        print(f"{(k + 1) * STEPS // 10} steps", flush=True)
    rho, u, T = L.moments()
    L.close()
    nx, ny, nz = SHAPE
    rng = np.random.default_rng(129)
    zs = rng.integers(0, nz, 4096)[:1024]
    ys = rng.integers(0, ny, 4096)[:1024]
    xs = rng.integers(0, nx, 4096)[:1024]
    pick = lambda a: a[zs, ys, xs].tolist()
    col = lambda a: [a[:, y, x].tolist() for x, y in COLUMNS]
    out = {"workload": w["name"], "steps": STEPS, "T0": w["T0"],
           "scale": {"u": float(max(np.abs(c).max() for c in u)), "T": float(np.abs(T - w["T0"]).max()),
                     "rho": float(np.abs(rho - 1).max())},
           "samples": {"z": zs.tolist(), "y": ys.tolist(), "x": xs.tolist(), "rho": pick(rho),
                       "ux": pick(u[0]), "uy": pick(u[1]), "uz": pick(u[2]), "T": pick(T)},
           "columns": {"xy": COLUMNS, "rho": col(rho), "ux": col(u[0]), "uy": col(u[1]), "uz": col(u[2]),
                       "T": col(T)}}
    with open(OUT, "w") as fh:
        json.dump(out, fh)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
