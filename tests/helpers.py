"""Shared test helpers: build the oracle and the GPU lattice from one workload description, and
the error measures the parity tests use."""
import numpy as np

import oracle as O
from oracle import Edge


def oracle_from_workload(w):
    e = w["edges"]
    lat = O.OracleLattice(w["nx"], w["ny"], *[Edge(*e[k]) for k in ("west", "east", "south", "north")],
                          T0=w["T0"])
    if "taus" in w:
        t = w["taus"]
        lat.set_params(t["tau_nu"], t["tau_alpha"], t["g_beta"])
    else:
        p = w["physics"]
        lat.set_params(*O.params_from_physics(p["Ra"], p["Pr"], p["Ma"], p["H"], p["dT"]))
    if "body_force" in w:
        lat.set_body_force(*w["body_force"])
    fl = w["fields"]
    lat.init(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    return lat


def rel_err(x, ref, base=0.0):
    """max |x - ref| / max |ref - base| (NaN anywhere -> inf)."""
    x, ref = np.asarray(x), np.asarray(ref)
    if np.isnan(x).any() or np.isnan(ref).any():
        return float("inf")
    scale = np.abs(ref - base).max()
    return float(np.abs(x - ref).max() / scale) if scale > 0 else float(np.abs(x - ref).max())


def field_errors(gpu_m, orc_m, T0):
    """Relative errors of (rho, ux, uy, T): rho against |rho|, u against max |u| (both components
    together), T against max |T - T0|."""
    r, ux, uy, T = gpu_m
    rr, rux, ruy, rT = orc_m
    umax = max(np.abs(rux).max(), np.abs(ruy).max())
    eu = max(np.abs(ux - rux).max(), np.abs(uy - ruy).max()) / umax if umax > 0 else np.abs(ux - rux).max()
    return {"rho": rel_err(r, rr), "u": float(eu), "T": rel_err(T, rT, T0)}
