"""FP64 CPU oracle for the CLB thermal lattice Boltzmann method (arXiv 1710.10569).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import this package.  It shares no code with the GPU library and never
imports it.

The arithmetic lives in ``clb_oracle.c`` (plain C, FP64): the D2Q9 CLB collision of Sec. 2.1
(Eqs. 4-13), the D2Q5 CLB collision of Sec. 2.2 (Eqs. 14-23), the Boussinesq force of Eq. 3 and
the wall conditions named in Sec. 3.  This module marshals arguments and adds the diagnostics of
Sec. 3 (the Nusselt number of Eq. 29 and wall-gradient forms, relative L2 errors).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libclb_oracle.so")
_lib = None

KINDS = {"periodic": 0, "dirichlet": 1, "adiabatic": 2}
EDGE_ORDER = ("west", "east", "south", "north")

_dp = ctypes.POINTER(ctypes.c_double)


def _load(path=None):
    """The oracle library (built on first use).  `path` loads another build of the same source
    -- the mutation tests use it for deliberately broken copies -- and makes it current."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    if path is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _build
            _build.build()
        path = _LIBPATH
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp, _dp,
                               ctypes.c_double]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_set_params.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.orc_set_relaxation.argtypes = [vp] + [ctypes.c_double] * 4
    lib.orc_set_body_force.argtypes = [vp, ctypes.c_double, ctypes.c_double]
    lib.orc_set_prescribed_velocity.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    lib.orc_init.argtypes = [vp, _dp, _dp, _dp, _dp]
    lib.orc_step.argtypes = [vp, ctypes.c_longlong]
    lib.orc_step.restype = ctypes.c_int
    lib.orc_moments.argtypes = [vp, _dp, _dp, _dp, _dp]
    lib.orc_moments.restype = ctypes.c_int
    lib.orc_get_state.argtypes = [vp, _dp, _dp]
    lib.orc_set_state.argtypes = [vp, _dp, _dp]
    lib.orc_get_outgoing.argtypes = [vp, _dp]
    lib.orc_set_outgoing.argtypes = [vp, _dp]
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_matrix_M.argtypes = [_dp]
    lib.orc_matrix_N.argtypes = [ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_matrix_Ninv.argtypes = [ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_matrix_Minv.argtypes = [vp, _dp]
    lib.orc_matrix_S.argtypes = [vp, _dp]
    lib.orc_matrix_MT.argtypes = [_dp]
    lib.orc_matrix_NT.argtypes = [ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_matrix_NTinv.argtypes = [ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_matrix_MTinv.argtypes = [vp, _dp]
    lib.orc_feq.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_geq.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_collide9.argtypes = [vp, _dp, ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_collide5.argtypes = [vp, _dp, ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_zou_he.argtypes = [_dp, ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 4
    _lib = lib
    return lib


def use_library(path):
    """Make the oracle library at `path` current (None: the default build); returns the previous one."""
    global _lib
    prev = _lib
    _lib = None
    _load(path)
    return prev


def restore_library(prev):
    global _lib
    _lib = prev


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64)
    return a


def threads() -> int:
    """OpenMP threads the oracle uses (OMP_NUM_THREADS, else all cores)."""
    return _load().orc_threads()


def set_threads(n: int) -> None:
    """Run the following oracle steps on n threads."""
    _load().orc_set_threads(int(n))


class Edge:
    """One side of the domain: kind ('periodic', 'dirichlet', 'adiabatic'), wall velocity, wall T."""

    def __init__(self, kind="periodic", ux=0.0, uy=0.0, T=0.0):
        if kind not in KINDS:
            raise ValueError(f"unknown edge kind {kind!r}")
        self.kind, self.ux, self.uy, self.T = kind, float(ux), float(uy), float(T)


class OracleLattice:
    """A 2D lattice advanced by the FP64 oracle.  Fields are numpy arrays of shape (ny, nx)."""

    def __init__(self, nx, ny, west=None, east=None, south=None, north=None, T0=0.0):
        lib = _load()
        edges = [e if e is not None else Edge() for e in (west, east, south, north)]
        self.nx, self.ny, self.T0 = int(nx), int(ny), float(T0)
        self.edges = dict(zip(EDGE_ORDER, edges))
        kinds = (ctypes.c_int * 4)(*[KINDS[e.kind] for e in edges])
        uw = np.array([[e.ux, e.uy] for e in edges], dtype=np.float64).ravel()
        tw = np.array([e.T for e in edges], dtype=np.float64)
        h = lib.orc_create(self.nx, self.ny, kinds, _ptr(uw), _ptr(tw), self.T0)
        if not h:
            raise ValueError("oracle rejected the lattice description")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # -- parameters --------------------------------------------------------------------------
    def set_params(self, tau_nu, tau_alpha, g_beta=0.0):
        self._lib.orc_set_params(self._h, tau_nu, tau_alpha, g_beta)

    def set_relaxation(self, s_b=1.0, s3=1.0, s4=1.0, lambda2=1.0):
        self._lib.orc_set_relaxation(self._h, s_b, s3, s4, lambda2)

    def set_body_force(self, Fvx, Fvy):
        self._lib.orc_set_body_force(self._h, Fvx, Fvy)

    def set_prescribed_velocity(self, ux, uy, on=True):
        self._lib.orc_set_prescribed_velocity(self._h, int(on), ux, uy)

    # -- state -------------------------------------------------------------------------------
    def init(self, rho=None, ux=None, uy=None, T=None):
        shp = (self.ny, self.nx)
        arrs = [_f64(a, shp) for a in (rho, ux, uy, T)]
        self._lib.orc_init(self._h, *[_ptr(a) for a in arrs])

    def step(self, n=1):
        rc = self._lib.orc_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError("oracle: an unknown population survived the wall step")

    def moments(self):
        shp = (self.ny, self.nx)
        rho, ux, uy, T = (np.empty(shp) for _ in range(4))
        rc = self._lib.orc_moments(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T))
        if rc != 0:
            raise RuntimeError("oracle: an unknown population survived the wall step")
        return rho, ux, uy, T

    def get_state(self):
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((5, self.ny, self.nx))
        self._lib.orc_get_state(self._h, _ptr(f), _ptr(g))
        return f, g

    def set_state(self, f, g):
        f = _f64(f).reshape(9, self.ny, self.nx)
        g = _f64(g).reshape(5, self.ny, self.nx)
        self._lib.orc_set_state(self._h, _ptr(f), _ptr(g))

    def get_outgoing(self):
        """out[9][ny][nx]: the flow populations f*_k that wall nodes sent out of the domain in the
        last step (entry k of a node is defined where x + e_k lies beyond a wall)."""
        out = np.empty((9, self.ny, self.nx))
        self._lib.orc_get_outgoing(self._h, _ptr(out))
        return out

    def set_outgoing(self, out):
        out = _f64(out).reshape(9, self.ny, self.nx)
        self._lib.orc_set_outgoing(self._h, _ptr(out))

    # -- single-node algebra (for the algebra tests) ------------------------------------------
    def matrix_Minv(self):
        out = np.empty(81)
        self._lib.orc_matrix_Minv(self._h, _ptr(out))
        return out.reshape(9, 9)

    def matrix_MTinv(self):
        out = np.empty(25)
        self._lib.orc_matrix_MTinv(self._h, _ptr(out))
        return out.reshape(5, 5)

    def matrix_S(self):
        out = np.empty(81)
        self._lib.orc_matrix_S(self._h, _ptr(out))
        return out.reshape(9, 9)

    def feq(self, rho, ux, uy):
        out = np.empty(9)
        self._lib.orc_feq(self._h, rho, ux, uy, _ptr(out))
        return out

    def geq(self, T, ux, uy):
        out = np.empty(5)
        self._lib.orc_geq(self._h, T, ux, uy, _ptr(out))
        return out

    def collide9(self, f, Fx=0.0, Fy=0.0):
        f = _f64(f)
        out = np.empty(9)
        self._lib.orc_collide9(self._h, _ptr(f), Fx, Fy, _ptr(out))
        return out

    def collide5(self, g, ux, uy):
        g = _f64(g)
        out = np.empty(5)
        self._lib.orc_collide5(self._h, _ptr(g), ux, uy, _ptr(out))
        return out


def matrix_M():
    out = np.empty(81)
    _load().orc_matrix_M(_ptr(out))
    return out.reshape(9, 9)


def matrix_N(ux, uy):
    out = np.empty(81)
    _load().orc_matrix_N(ux, uy, _ptr(out))
    return out.reshape(9, 9)


def matrix_Ninv(ux, uy):
    out = np.empty(81)
    _load().orc_matrix_Ninv(ux, uy, _ptr(out))
    return out.reshape(9, 9)


def matrix_MT():
    out = np.empty(25)
    _load().orc_matrix_MT(_ptr(out))
    return out.reshape(5, 5)


def matrix_NT(ux, uy):
    out = np.empty(25)
    _load().orc_matrix_NT(ux, uy, _ptr(out))
    return out.reshape(5, 5)


def matrix_NTinv(ux, uy):
    out = np.empty(25)
    _load().orc_matrix_NTinv(ux, uy, _ptr(out))
    return out.reshape(5, 5)


def zou_he(f, normal, uw=(0.0, 0.0), F=(0.0, 0.0)):
    """The force-corrected Zou-He closure applied to a copy of the nine populations of one node."""
    f = _f64(f).copy()
    _load().orc_zou_he(_ptr(f), int(normal[0]), int(normal[1]), uw[0], uw[1], F[0], F[1])
    return f


# ---------------------------------------------------------------------------------------------
# Parameter mapping (Sec. 2.1, Sec. 2.2, Sec. 3.3) and diagnostics (Sec. 3).

CS = 1.0 / math.sqrt(3.0)   # D2Q9 sound speed (after Eq. 9)
CT2 = 0.25                  # D2Q5 c_{T,s}^2 (Sec. 3 default c_sT = 1/2)


def params_from_physics(Ra, Pr, Ma, H, dT):
    """(tau_nu, tau_alpha, g*beta) from Ra = g beta dT H^3/(nu alpha), Pr = nu/alpha,
    u_c = sqrt(g beta dT H) = Ma c_s, nu = Ma c_s H sqrt(Pr/Ra) (Sec. 3.3); nu = (tau_nu - 1/2)/3
    (Sec. 2.1) and alpha = (tau_alpha - 1/2) c_{T,s}^2 (Sec. 2.2)."""
    nu = Ma * CS * H * math.sqrt(Pr / Ra)
    alpha = nu / Pr
    g_beta = Ra * nu * alpha / (dT * H ** 3)
    return 3.0 * nu + 0.5, alpha / CT2 + 0.5, g_beta


def nu_of_tau(tau_nu):
    return (tau_nu - 0.5) / 3.0


def alpha_of_tau(tau_alpha):
    return (tau_alpha - 0.5) * CT2


def trapezoid_weights(n):
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    return w


def nusselt_volume(u_normal, T, alpha, dT, H, along_periodic):
    """Eq. 29, Nu = 1 + <u_n T> H / (alpha dT): u_n is the velocity component along the mean heat
    flux.  Arrays are oriented (along, across): 'across' runs from the hot wall (node 0) to the cold
    wall (node H); walls sit on nodes, so that direction is averaged with trapezoid weights, and so
    is 'along' when it is bounded by walls (plain mean when it is periodic)."""
    wa = trapezoid_weights(u_normal.shape[1])
    wl = np.ones(u_normal.shape[0]) if along_periodic else trapezoid_weights(u_normal.shape[0])
    q = (u_normal * T * wl[:, None] * wa[None, :]).sum() / (wl.sum() * wa.sum())
    return float(1.0 + q * H / (alpha * dT))


def nusselt_hot_wall(T, dT):
    """Mean Nusselt number on the hot wall x = 0 of a cavity whose walls sit on nodes: the local
    Nu = -(H/dT) dT/dx averaged over the wall, with the second-order one-sided gradient
    -dT/dx = (3 T_0 - 4 T_1 + T_2)/2 and trapezoid weights along the wall (Delta x = 1, so the
    wall length H = ny - 1 cancels).  T has shape (ny, nx)."""
    g = (3.0 * T[:, 0] - 4.0 * T[:, 1] + T[:, 2]) / 2.0
    w = trapezoid_weights(T.shape[0])
    return float((g * w).sum() / dT)


def rel_l2(x, ref):
    """Relative L2 error sqrt(sum (x - ref)^2 / sum ref^2) (Sec. 3.2)."""
    return float(np.sqrt(((x - ref) ** 2).sum() / (ref ** 2).sum()))
