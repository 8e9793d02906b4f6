"""Shared test helpers: build the oracle and the GPU lattice from one workload description, and
the error measures the parity tests use."""
import numpy as np

import oracle as O
from oracle import Edge


def oracle_from_workload(w):
    e = w["edges"]
    lat = O.OracleLattice(w["nx"], w["ny"], *[Edge(*e[k]) for k in ("west", "east", "south", "north")],
                          T0=w["T0"])
    if "prescribed_u" in w:
        lat.set_prescribed_velocity(*w["prescribed_u"])
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


def field_errors(gpu_m, orc_m, T0, u_scale=0.0):
    """Relative max-norm errors of (rho, u, T): rho against max |rho|; u (both components) against
    U = max(max |u_ref|, u_scale), u_scale being the workload's characteristic velocity (a flow
    started from rest has |u| far below its scale for many steps); T against max |T_ref - T0|."""
    r, ux, uy, T = gpu_m
    rr, rux, ruy, rT = orc_m
    if any(np.isnan(a).any() for a in (r, ux, uy, T)):
        return {"rho": float("inf"), "u": float("inf"), "T": float("inf")}
    U = max(np.abs(rux).max(), np.abs(ruy).max(), u_scale)
    eu = max(np.abs(ux - rux).max(), np.abs(uy - ruy).max()) / U
    return {"rho": rel_err(r, rr), "u": float(eu), "T": rel_err(T, rT, T0)}
