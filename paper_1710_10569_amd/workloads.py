"""Seeded synthetic workloads: geometry, physical parameters and initial fields.

This module is shared by the GPU path's tests and benchmark and by the oracle's tests, so it holds
none of the method's arithmetic: only problem descriptions (sizes, walls, Ra/Pr/Ma or relaxation
times) and initial macroscopic fields drawn from seeded generators
(``numpy.random.default_rng(seed)``, PCG64) or written in closed form.  Each side maps the
description onto its own interface.

A workload is a dict (``u_scale`` is the problem's characteristic velocity, the scale against
which velocity errors are reported)::

    {"name": str, "nx": int, "ny": int, "T0": float,
     "edges": {"west"|"east"|"south"|"north": (kind, ux_w, uy_w, T_w)},   # kind: periodic|dirichlet|adiabatic
     "physics": {"Ra", "Pr", "Ma", "H", "dT"}  or  "taus": {"tau_nu", "tau_alpha", "g_beta"},
     "fields": {"rho", "ux", "uy", "T"}  (float64 arrays of shape (ny, nx), or None for a default),
     "u_scale": float}

Walls sit on nodes, so a wall-bounded extent of N nodes has length H = N - 1.
"""
from __future__ import annotations

import math

import numpy as np

PERIODIC = ("periodic", 0.0, 0.0, 0.0)


def _edges(west=PERIODIC, east=PERIODIC, south=PERIODIC, north=PERIODIC):
    return {"west": west, "east": east, "south": south, "north": north}


def taylor_green(n=64, U0=0.01, T0=1.0, Tamp=0.01, tau_nu=0.8, tau_alpha=0.7):
    """Fully periodic n x n Taylor-Green vortex with a sinusoidal temperature mode and no buoyancy.

    u = U0 sin(kx) cos(ky), v = -U0 cos(kx) sin(ky), k = 2 pi / n at node coordinates; the
    density carries the vortex's pressure, rho = 1 + 3 p with p = (U0^2/4)(cos 2kx + cos 2ky), so
    that no sound wave is launched; T = T0 + Tamp sin(kx) sin(ky), a function of the stream function
    so that advection leaves it unchanged."""
    k = 2.0 * math.pi / n
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(n, dtype=np.float64)[:, None]
    ux = U0 * np.sin(k * x) * np.cos(k * y)
    uy = -U0 * np.cos(k * x) * np.sin(k * y)
    p = (U0 * U0 / 4.0) * (np.cos(2 * k * x) + np.cos(2 * k * y))
    rho = 1.0 + 3.0 * p
    T = T0 + Tamp * np.sin(k * x) * np.sin(k * y)
    return {"name": f"taylor_green_{n}x{n}", "nx": n, "ny": n, "T0": T0, "edges": _edges(),
            "taus": {"tau_nu": tau_nu, "tau_alpha": tau_alpha, "g_beta": 0.0},
            "fields": {"rho": rho, "ux": ux, "uy": uy, "T": T},
            "k": k, "U0": U0, "Tamp": Tamp, "u_scale": U0}


def cavity(L=256, Ra=1e5, Pr=0.71, Ma=0.1, seed=2, noise=1e-4, T_hot=0.5, T_cold=-0.5):
    """Differentially heated square cavity of L x L nodes: hot west wall, cold east wall (Dirichlet),
    adiabatic south and north walls, all no-slip, gravity along -y, T0 = 0.  The initial state is
    rest with T drawn from U(-noise, noise) on every node, then the hot and cold wall columns set to
    their wall temperatures."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(-noise, noise, size=(L, L))
    T[:, 0] = T_hot
    T[:, -1] = T_cold
    return {"name": f"cavity_{L}x{L}_Ra{Ra:.3g}", "nx": L, "ny": L, "T0": 0.0,
            "edges": _edges(west=("dirichlet", 0.0, 0.0, T_hot), east=("dirichlet", 0.0, 0.0, T_cold),
                            south=("adiabatic", 0.0, 0.0, 0.0), north=("adiabatic", 0.0, 0.0, 0.0)),
            "physics": {"Ra": Ra, "Pr": Pr, "Ma": Ma, "H": L - 1, "dT": T_hot - T_cold},
            "u_scale": Ma / math.sqrt(3.0),
            "fields": {"rho": None, "ux": None, "uy": None, "T": T}}


def rayleigh_benard(nx=2048, ny=1024, Ra=1e6, Pr=0.71, Ma=0.3, seed=3, amp=1e-3,
                    T_hot=0.5, T_cold=-0.5, T0=0.0, rolls=0.0):
    """Rayleigh-Benard cell, periodic in x, hot south wall and cold north wall (Dirichlet, no-slip),
    gravity along -y.  Initial state: rest, the conduction profile T = T_hot - (T_hot - T_cold) y/H
    on nodes y = 0..H, plus U(-amp, amp) noise on the interior rows.

    rolls > 0 starts instead from convection rolls of that fraction of the convective velocity
    u_c = Ma c_s, one pair per 2H of width (k = 2 pi m / nx with m = round(nx / 2H)): stream
    function psi = (A / k) sin(kx) sin^2(pi y / H), so u_x = A (pi / (k H)) sin(kx) sin(2 pi y / H) and
    u_y = -A cos(kx) sin^2(pi y / H) are divergence-free and vanish on the walls, with the warm
    anomaly -0.1 dT cos(kx) sin(pi y / H) where the fluid rises."""
    rng = np.random.default_rng(seed)
    H = ny - 1
    y = np.arange(ny, dtype=np.float64)[:, None]
    T = np.broadcast_to(T_hot - (T_hot - T_cold) * y / H, (ny, nx)).copy()
    T[1:-1, :] += rng.uniform(-amp, amp, size=(ny - 2, nx))
    ux = uy = None
    u_c = Ma / math.sqrt(3.0)
    if rolls > 0:
        A = rolls * u_c
        m = max(1, round(nx / (2 * H)))
        k = 2 * math.pi * m / nx
        x = np.arange(nx, dtype=np.float64)[None, :]
        s = np.sin(math.pi * y / H)
        ux = A * (math.pi / (k * H)) * np.sin(k * x) * np.sin(2 * math.pi * y / H)
        uy = -A * np.cos(k * x) * s * s
        T = T - 0.1 * (T_hot - T_cold) * np.cos(k * x) * s
    return {"name": f"rayleigh_benard_{nx}x{ny}_Ra{Ra:.3g}" + (f"_rolls{rolls:g}" if rolls > 0 else ""),
            "nx": nx, "ny": ny, "T0": T0,
            "edges": _edges(south=("dirichlet", 0.0, 0.0, T_hot), north=("dirichlet", 0.0, 0.0, T_cold)),
            "physics": {"Ra": Ra, "Pr": Pr, "Ma": Ma, "H": H, "dT": T_hot - T_cold},
            "u_scale": u_c,
            "fields": {"rho": None, "ux": ux, "uy": uy, "T": T}}


def rb_cell(Ra, L=60, H=30, Pr=0.71, Ma=0.3, T_hot=1.05, T_cold=0.95, amp=1e-3):
    """The Rayleigh-Benard cell of the Nusselt table: L x H = 60 x 30 (nodes L x (H + 1), periodic
    in x), T_hot = 1.05, T_cold = 0.95, T0 = 1.  Instead of a density bump the conduction profile is
    perturbed by amp * cos(2 pi x / L) sin(pi y / H), which seeds the same one-wavelength pair of
    rolls."""
    ny = H + 1
    x = np.arange(L, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    T = T_hot - (T_hot - T_cold) * y / H + amp * np.cos(2 * math.pi * x / L) * np.sin(math.pi * y / H)
    return {"name": f"rb_cell_{L}x{H}_Ra{Ra:g}", "nx": L, "ny": ny, "T0": 0.5 * (T_hot + T_cold),
            "edges": _edges(south=("dirichlet", 0.0, 0.0, T_hot), north=("dirichlet", 0.0, 0.0, T_cold)),
            "physics": {"Ra": Ra, "Pr": Pr, "Ma": Ma, "H": H, "dT": T_hot - T_cold},
            "u_scale": Ma / math.sqrt(3.0),
            "fields": {"rho": None, "ux": None, "uy": None, "T": T}}


def poiseuille(nx=4, ny=33, tau_nu=0.8, Fx=1e-6, T0=0.0):
    """Body-force-driven channel: periodic in x, no-slip walls on nodes y = 0 and y = ny - 1,
    constant force density F_v = (Fx, 0), uniform T = T0 (no buoyancy)."""
    return {"name": f"poiseuille_{nx}x{ny}", "nx": nx, "ny": ny, "T0": T0,
            "edges": _edges(south=("dirichlet", 0.0, 0.0, T0), north=("dirichlet", 0.0, 0.0, T0)),
            "taus": {"tau_nu": tau_nu, "tau_alpha": 0.8, "g_beta": 0.0},
            "body_force": (Fx, 0.0),
            "u_scale": Fx * (ny - 1) ** 2 / (8.0 * (tau_nu - 0.5) / 3.0),
            "fields": {"rho": None, "ux": None, "uy": None, "T": None}}


def random_periodic(nx, ny, seed, amp_u=0.05, amp_T=0.1, T0=0.0, g_beta=1e-3, tau_nu=0.7, tau_alpha=0.9):
    """Periodic lattice with seeded random fields: rho = 1 + U(-0.01, 0.01), u = U(-amp_u, amp_u),
    T = T0 + U(-amp_T, amp_T), and buoyancy on, so every term of the step is exercised."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-0.01, 0.01, size=(ny, nx))
    ux = rng.uniform(-amp_u, amp_u, size=(ny, nx))
    uy = rng.uniform(-amp_u, amp_u, size=(ny, nx))
    T = T0 + rng.uniform(-amp_T, amp_T, size=(ny, nx))
    return {"name": f"random_periodic_{nx}x{ny}_s{seed}", "nx": nx, "ny": ny, "T0": T0,
            "edges": _edges(),
            "taus": {"tau_nu": tau_nu, "tau_alpha": tau_alpha, "g_beta": g_beta},
            "u_scale": amp_u,
            "fields": {"rho": rho, "ux": ux, "uy": uy, "T": T}}


def random_walled(nx, ny, seed, kinds=("dirichlet", "dirichlet", "adiabatic", "adiabatic"),
                  amp_u=0.02, amp_T=0.1, g_beta=1e-3, tau_nu=0.7, tau_alpha=0.9, wall_u=0.0):
    """Walled lattice with seeded random interior fields and, if wall_u != 0, moving and permeable
    walls, so every branch of the wall step is exercised.  kinds = (west, east, south, north); a
    periodic pair is allowed."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-0.01, 0.01, size=(ny, nx))
    ux = rng.uniform(-amp_u, amp_u, size=(ny, nx))
    uy = rng.uniform(-amp_u, amp_u, size=(ny, nx))
    T = rng.uniform(-amp_T, amp_T, size=(ny, nx))
    wu = rng.uniform(-wall_u, wall_u, size=(4, 2)) if wall_u else np.zeros((4, 2))
    tw = (0.5, -0.5, 0.25, -0.25)
    names = ("west", "east", "south", "north")
    edges = {}
    for i, (nm, kd) in enumerate(zip(names, kinds)):
        edges[nm] = (kd, float(wu[i, 0]), float(wu[i, 1]), tw[i]) if kd != "periodic" else PERIODIC
    return {"name": f"random_walled_{nx}x{ny}_s{seed}", "nx": nx, "ny": ny, "T0": 0.0,
            "edges": edges,
            "taus": {"tau_nu": tau_nu, "tau_alpha": tau_alpha, "g_beta": g_beta},
            "u_scale": amp_u,
            "fields": {"rho": rho, "ux": ux, "uy": uy, "T": T}}


def batch_cavity_specs(n=512, seed=7, sizes=tuple(range(64, 513, 32)), Ra_range=(3.0, 6.0), Pr=0.71, Ma=0.1):
    """The batched-cavity workload: side lengths drawn uniformly from {64, 96, ..., 512}, then
    Ra = 10**U(3, 6), in that order, from default_rng(seed); cavity i has noise seed 1000 + i.
    Returns (L, Ra, noise_seed) triples."""
    rng = np.random.default_rng(seed)
    Ls = rng.choice(np.array(sizes), n)
    Ras = 10.0 ** rng.uniform(Ra_range[0], Ra_range[1], n)
    return [(int(L), float(Ra), 1000 + i) for i, (L, Ra) in enumerate(zip(Ls, Ras))]


def serving_requests(n=200, lam=1.0, seed=5, L_range=(32, 1024), Ra_range=(1e3, 1e6)):
    """A Poisson stream of cavity requests: exponential inter-arrival times of mean 1/lam (seconds),
    L = round(exp(U(ln L_min, ln L_max))), Ra log-uniform.  Returns dicts with arrival, L, Ra,
    noise_seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / lam, n)
    arrivals = np.cumsum(gaps)
    Ls = np.rint(np.exp(rng.uniform(math.log(L_range[0]), math.log(L_range[1]), n))).astype(int)
    Ras = np.exp(rng.uniform(math.log(Ra_range[0]), math.log(Ra_range[1]), n))
    return [{"id": i, "arrival": float(a), "L": int(L), "Ra": float(Ra), "noise_seed": 5000 + i}
            for i, (a, L, Ra) in enumerate(zip(arrivals, Ls, Ras))]


def normal_plate(L=30, Re=10.0, Pr=0.71, nu=0.1, nx=5, T_L=0.0, T_H=1.0):
    """Normal-plate channel: periodic in x (nx nodes), walls on nodes y = 0 and y = L.  Fluid is
    injected through the bottom plate with v0 and withdrawn through the top plate, which also slides
    with u0; u0 = v0 = Re nu / L.  Bottom plate at T_L, top plate at T_H, no buoyancy.  The D2Q5
    second-order rate follows the zero-numerical-slip relation lambda2 = 12 (lambda1 - 2)/(lambda1 - 12)
    with lambda1 = 1/tau_alpha.  Starts from rest at T = T_L."""
    v0 = Re * nu / L
    alpha = nu / Pr
    tau_nu, tau_alpha = 3.0 * nu + 0.5, 4.0 * alpha + 0.5
    lam1 = 1.0 / tau_alpha
    return {"name": f"normal_plate_L{L}_Re{Re:g}_Pr{Pr:g}", "nx": nx, "ny": L + 1, "T0": T_L,
            "edges": _edges(south=("dirichlet", 0.0, v0, T_L), north=("dirichlet", v0, v0, T_H)),
            "taus": {"tau_nu": tau_nu, "tau_alpha": tau_alpha, "g_beta": 0.0},
            "lambda2": 12.0 * (lam1 - 2.0) / (lam1 - 12.0),
            "u_scale": v0, "Re": Re, "Pr": Pr, "L": L, "u0": v0, "T_L": T_L, "T_H": T_H,
            "fields": {"rho": None, "ux": None, "uy": np.full((L + 1, nx), v0), "T": None}}


def moving_frame(L=100, B=0.01, alpha=0.05, T0=1.0, Ma=0.3, nx=4):
    """Sec. 3.1 (Eq. 24): a temperature wave T = T0 + B sin(phi y), phi = 2 pi / L, on a frame
    moving with the prescribed velocity u = (0, A), A = Ma c_s; periodic in x and y; only the D2Q5
    equation runs (temperature-only lattice), tau_alpha from the given alpha with c_T^2 = 1/4."""
    y = np.arange(L, dtype=np.float64)[:, None]
    T = np.broadcast_to(T0 + B * np.sin(2 * math.pi * y / L), (L, nx)).copy()
    A = Ma / math.sqrt(3.0)
    return {"name": f"moving_frame_L{L}_Ma{Ma:g}", "nx": nx, "ny": L, "T0": T0, "edges": _edges(),
            "taus": {"tau_nu": 0.8, "tau_alpha": 4.0 * alpha + 0.5, "g_beta": 0.0},
            "prescribed_u": (0.0, A), "u_scale": max(A, 1e-3),
            "fields": {"rho": np.ones((L, nx)), "ux": np.zeros((L, nx)), "uy": np.full((L, nx), A), "T": T}}


def prescribed_walled(nx, ny, seed, u=(0.03, -0.05), kinds=("dirichlet", "adiabatic", "adiabatic", "dirichlet"),
                      amp_T=0.1, T0=0.2, tau_alpha=0.9):
    """Temperature-only lattice with walls (every branch of the temperature wall step: Dirichlet and
    adiabatic edges, corners of both kinds) and a seeded random temperature field, advected by the
    uniform prescribed velocity u."""
    rng = np.random.default_rng(seed)
    T = T0 + rng.uniform(-amp_T, amp_T, size=(ny, nx))
    names = ("west", "east", "south", "north")
    tw = (T0 + 0.5, T0 - 0.5, T0 + 0.25, T0 - 0.25)
    edges = {nm: ((kd, 0.0, 0.0, tw[i]) if kd != "periodic" else PERIODIC) for i, (nm, kd) in enumerate(zip(names, kinds))}
    return {"name": f"prescribed_walled_{nx}x{ny}_s{seed}", "nx": nx, "ny": ny, "T0": T0, "edges": edges,
            "taus": {"tau_nu": 0.8, "tau_alpha": tau_alpha, "g_beta": 0.0},
            "prescribed_u": tuple(u), "u_scale": 1.0,
            "fields": {"rho": np.ones((ny, nx)), "ux": np.full((ny, nx), u[0]), "uy": np.full((ny, nx), u[1]), "T": T}}
