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


# ---------------------------------------------------------------------------------------------
# Three-dimensional workloads (D3Q27/D3Q7 path).  Same conventions, with fields of shape
# (nz, ny, nx), "u" a triple (u_x, u_y, u_z), periodic x and y, and "z_walls" None (periodic z) or
# two dicts {"kind": "dirichlet"|"adiabatic", "u": (ux, uy), "T": float} for z = 0 and z = nz - 1;
# gravity acts along -z.  "taus" carries the relaxation times directly, or "physics" the
# dimensionless groups, which each side maps with its own parameter routine (nu = (tau_nu - 1/2)/3,
# alpha = (tau_alpha - 1/2)/4 in three dimensions too).


def _wall3(kind, u=(0.0, 0.0), T=0.0):
    return {"kind": kind, "u": (float(u[0]), float(u[1])), "T": float(T)}


def rayleigh_benard_3d(nx=256, ny=256, nz=129, Ra=1e5, Pr=0.71, Ma=0.1, seed=3, amp=1e-3, T_hot=0.5, T_cold=-0.5,
                       rolls=0.0):
    """Rayleigh-Benard convection in a layer periodic in x and y: hot bottom wall z = 0 at T_hot,
    cold top wall z = nz - 1 at T_cold (H = nz - 1), resting walls, T0 the mean.  Starts from the
    conduction profile with a seeded perturbation: amp dT U(-1, 1) at every interior node.

    rolls > 0 adds two crossed sets of convection rolls of that fraction of u_c = Ma c_s, one pair
    per 2H along x and along y (k = 2 pi m / n, m = round(n / 2H)): stream functions
    psi_x = (A / k_x) sin(k_x x) s^2 in the x-z plane and psi_y = (A / (2 k_y)) sin(k_y y) s^2 in the
    y-z plane, s = sin(pi z / H), so u = (-d psi_x/dz, -d psi_y/dz, d psi_x/dx + d psi_y/dy) is
    divergence-free and vanishes on the walls; the warm anomaly -0.1 dT cos(k_x x) s rides with
    the rising fluid."""
    rng = np.random.default_rng(seed)
    H = nz - 1
    dT = T_hot - T_cold
    T0 = 0.5 * (T_hot + T_cold)
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    T = T_hot - dT * z / H + np.zeros((nz, ny, nx))
    T[1:-1] += amp * dT * rng.uniform(-1.0, 1.0, (nz - 2, ny, nx))
    u = None
    if rolls > 0:
        A = rolls * Ma / math.sqrt(3.0)
        kx = 2 * math.pi * max(1, round(nx / (2 * H))) / nx
        ky = 2 * math.pi * max(1, round(ny / (2 * H))) / ny
        x = np.arange(nx, dtype=np.float64)[None, None, :]
        y = np.arange(ny, dtype=np.float64)[None, :, None]
        s = np.sin(math.pi * z / H)
        ds2 = (math.pi / H) * np.sin(2 * math.pi * z / H)       # d(s^2)/dz
        ux = -(A / kx) * np.sin(kx * x) * ds2 + 0.0 * y
        uy = -(0.5 * A / ky) * np.sin(ky * y) * ds2 + 0.0 * x
        uz = A * np.cos(kx * x) * s * s + 0.5 * A * np.cos(ky * y) * s * s
        u = (ux, uy, uz)
        T = T - 0.1 * dT * np.cos(kx * x) * s
    return {"name": f"rayleigh_benard_3d_{nx}x{ny}x{nz}_Ra{Ra:g}" + (f"_rolls{rolls:g}" if rolls > 0 else ""),
            "nx": nx, "ny": ny, "nz": nz, "T0": T0,
            "z_walls": (_wall3("dirichlet", T=T_hot), _wall3("dirichlet", T=T_cold)),
            "physics": {"Ra": Ra, "Pr": Pr, "Ma": Ma, "H": H, "dT": dT},
            "fields": {"rho": None, "u": u, "T": T}, "u_scale": Ma / math.sqrt(3.0)}


def abc_flow_3d(n=64, A=0.01, tau_nu=0.8, tau_alpha=0.8, T0=0.0):
    """Arnold-Beltrami-Childress flow (A = B = C) on a periodic n^3 box, k = 2 pi / n: a Beltrami
    field whose Navier-Stokes solution decays as exp(-nu k^2 t); T = T0, no buoyancy."""
    k = 2.0 * math.pi / n
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    u = (A * (np.sin(k * z) + np.cos(k * y)), A * (np.sin(k * x) + np.cos(k * z)), A * (np.sin(k * y) + np.cos(k * x)))
    return {"name": f"abc_flow_{n}^3", "nx": n, "ny": n, "nz": n, "T0": T0, "z_walls": None,
            "taus": {"tau_nu": tau_nu, "tau_alpha": tau_alpha, "g_beta": 0.0},
            "fields": {"rho": None, "u": u, "T": None}, "k": k, "A": A, "u_scale": 2.0 * A}


def random_3d(nx, ny, nz, seed, walls=None, amp_u=0.03, amp_T=0.1, T0=0.0, g_beta=1e-3, tau_nu=0.7,
              tau_alpha=0.9, body_force=(1e-5, -2e-5, 1.5e-5), relaxation=None):
    """Random (unsmoothed) fields for parity tests: rho = 1 + 0.01 N(0,1), u = amp_u N(0,1) per
    component, T = T0 + amp_T N(0,1), from default_rng(seed).  walls: None (periodic z) or a pair of
    (kind, (ux, uy), T) for the bottom and top walls; wall nodes then start at the wall data."""
    rng = np.random.default_rng(seed)
    shp = (nz, ny, nx)
    rho = 1.0 + 0.01 * rng.standard_normal(shp)
    u = [amp_u * rng.standard_normal(shp) for _ in range(3)]
    T = T0 + amp_T * rng.standard_normal(shp)
    zw = None
    if walls is not None:
        zw = tuple(_wall3(k, uw, Tw) for k, uw, Tw in walls)
        for zi, w in ((0, zw[0]), (nz - 1, zw[1])):
            u[0][zi], u[1][zi], u[2][zi] = w["u"][0], w["u"][1], 0.0
            if w["kind"] == "dirichlet":
                T[zi] = w["T"]
    out = {"name": f"random_3d_{nx}x{ny}x{nz}_s{seed}" + ("_walls" if walls else ""), "nx": nx, "ny": ny, "nz": nz,
           "T0": T0, "z_walls": zw, "taus": {"tau_nu": tau_nu, "tau_alpha": tau_alpha, "g_beta": g_beta},
           "body_force": tuple(body_force), "fields": {"rho": rho, "u": tuple(u), "T": T}, "u_scale": amp_u}
    if relaxation is not None:
        out["relaxation"] = dict(relaxation)
    return out
