"""Write table1_oracle.json: the FP64 oracle's steady Nusselt numbers of the eight Table 1 cells
(Sec. 3.3: 60 x 30, Pr = 0.71, Ma = 0.3, wall temperatures centred on T0 = 0 at +-0.05), in the
volume form of Eq. 29 and the hot-wall gradient form, for the GPU's comparison.

Run from the repository root: python tests/golden/make_table1_oracle.py  (about a minute on 8
cores).  Only the oracle and the seeded input generator are called.  A cell is steady when Nu of
Eq. 29 changes by less than 1e-10 of itself over 1000 steps."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1710_10569_amd import workloads as W  # noqa: E402
from tests.helpers import oracle_from_workload  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table1_oracle.json")


def steady_nusselt(Ra):
    w = W.rb_cell(Ra, T_hot=0.05, T_cold=-0.05)
    o = oracle_from_workload(w)
    p = w["physics"]
    alpha = O.alpha_of_tau(O.params_from_physics(p["Ra"], p["Pr"], p["Ma"], p["H"], p["dT"])[1])
    prev, steps = None, 0
    while True:
        o.step(1000)
        steps += 1000
        _, _, uy, T = o.moments()
        nu = O.nusselt_volume(uy.T, T.T, alpha, p["dT"], p["H"], along_periodic=True)
        if prev is not None and abs(nu - prev) < 1e-10 * nu:
            break
        prev = nu
    g = (3 * T[0, :] - 4 * T[1, :] + T[2, :]) / 2.0
    return {"Ra": Ra, "Nu_volume": nu, "Nu_wall": float(g.mean() * p["H"] / p["dT"]), "steps": steps}


def main():
    rows = [steady_nusselt(Ra) for Ra in (2000, 2500, 3000, 5000, 10000, 20000, 30000, 50000)]
    for r in rows:
        print(r, flush=True)
    with open(OUT, "w") as fh:
        json.dump({"setup": "rb_cell 60 x 30, Pr 0.71, Ma 0.3, T_hot/T_cold = +-0.05 about T0 = 0", "rows": rows}, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
