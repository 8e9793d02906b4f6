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
    """Relative max-norm errors of (rho, u, T).  u (both components) and T against the largest
    departure of the reference from its rest value, max |u_ref| and max |T_ref - T0| (the measure
    the parity bars apply to); rho against max |rho_ref|.  Reported beside them: "rho_p12", rho
    against max |rho_ref - 1| (the pressure departure, O(Ma^2): two FP64 builds of the oracle that
    differ only in multiply-add contraction already differ by ~5e-12 of it, so it is reported, not
    gated), and "u_scaled", the u error against max(max |u_ref|, u_scale), u_scale being the
    workload's characteristic velocity."""
    r, ux, uy, T = gpu_m
    rr, rux, ruy, rT = orc_m
    if any(np.isnan(a).any() for a in (r, ux, uy, T)):
        inf = float("inf")
        return {"rho": inf, "u": inf, "T": inf, "rho_p12": inf, "u_scaled": inf}
    du = max(np.abs(ux - rux).max(), np.abs(uy - ruy).max())
    umax = max(np.abs(rux).max(), np.abs(ruy).max())
    us = max(umax, u_scale)
    return {"rho": rel_err(r, rr), "u": float(du / umax) if umax > 0 else float(du), "T": rel_err(T, rT, T0),
            "rho_p12": rel_err(r, rr, 1.0), "u_scaled": float(du / us) if us > 0 else float(du)}


def worst(e):
    """The largest of the gated errors (rho, u, T) of a field_errors record."""
    return max(e["rho"], e["u"], e["T"])
