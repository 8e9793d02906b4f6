"""FP64 CPU oracle for the three-dimensional CLB method (D3Q27 flow, D3Q7 temperature).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import this module.  It shares no code with the GPU library and never imports
it.  The arithmetic lives in ``clb3d_oracle.c``; this module marshals arguments.  Fields are numpy
arrays of shape (nz, ny, nx); velocities are three such arrays (u_x, u_y, u_z).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libclb3d_oracle.so")
_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)

ZKINDS = {"periodic": 0, "dirichlet": 1, "adiabatic": 2}


def _load(path=None):
    """The 3D oracle library (built on first use); `path` loads another build of the same source
    (the mutation tests use it for deliberately broken copies) and makes it current."""
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
    d = ctypes.c_double
    lib.orc3_create.restype = vp
    lib.orc3_create.argtypes = [ctypes.c_int] * 3 + [_ip, _dp, _dp, d]
    lib.orc3_destroy.argtypes = [vp]
    lib.orc3_set_threads.argtypes = [ctypes.c_int]
    lib.orc3_set_params.argtypes = [vp, d, d, d]
    lib.orc3_set_relaxation.argtypes = [vp] + [d] * 6
    lib.orc3_set_body_force.argtypes = [vp, d, d, d]
    lib.orc3_init.argtypes = [vp, _dp, _dp, _dp]
    lib.orc3_step.argtypes = [vp, ctypes.c_longlong]
    lib.orc3_step.restype = ctypes.c_int
    lib.orc3_moments.argtypes = [vp, _dp, _dp, _dp]
    lib.orc3_moments.restype = ctypes.c_int
    lib.orc3_get_state.argtypes = [vp, _dp, _dp]
    lib.orc3_set_state.argtypes = [vp, _dp, _dp]
    lib.orc3_get_outgoing.argtypes = [vp, _dp]
    lib.orc3_velocities.argtypes = [_ip, _ip, _ip]
    lib.orc3_moment_order.argtypes = [_ip]
    lib.orc3_matrix_M.argtypes = [vp, _dp]
    lib.orc3_matrix_N.argtypes = [d, d, d, _dp]
    lib.orc3_matrix_S.argtypes = [vp, _dp]
    lib.orc3_feq.argtypes = [vp, d, d, d, d, _dp]
    lib.orc3_geq.argtypes = [vp, d, d, d, d, _dp]
    lib.orc3_collide27.argtypes = [vp, _dp, d, d, d, _dp]
    lib.orc3_collide7.argtypes = [vp, _dp, d, d, d, _dp]
    _lib = lib
    return lib


def use_library(path):
    """Make the 3D oracle library at `path` current (None: the default build); returns the previous one."""
    global _lib
    prev = _lib
    _lib = None
    _load(path)
    return prev


def restore_library(prev):
    global _lib
    _lib = prev


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    if a is None:
        return None
    if shape is not None:
        return np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape), dtype=np.float64)
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    _load().orc3_set_threads(int(n))


def velocities():
    """(ex, ey, ez) of the D3Q27 set in the oracle's order (the first seven are D3Q7)."""
    e = [(ctypes.c_int * 27)() for _ in range(3)]
    _load().orc3_velocities(*e)
    return tuple(np.array(list(a), dtype=float) for a in e)


def moment_order():
    o = (ctypes.c_int * 81)()
    _load().orc3_moment_order(o)
    return np.array(list(o)).reshape(27, 3)


def matrix_N(ux, uy, uz):
    out = np.empty(27 * 27)
    _load().orc3_matrix_N(ux, uy, uz, _ptr(out))
    return out.reshape(27, 27)


class Wall:
    """A z wall: kind ('dirichlet' or 'adiabatic'), tangential velocity (ux, uy), temperature T."""

    def __init__(self, kind="dirichlet", ux=0.0, uy=0.0, T=0.0):
        if kind not in ("dirichlet", "adiabatic"):
            raise ValueError(f"unknown wall kind {kind!r}")
        self.kind, self.ux, self.uy, self.T = kind, float(ux), float(uy), float(T)


class OracleLattice3D:
    """A 3D lattice (periodic in x and y; z periodic or bounded by two walls) advanced by the FP64
    oracle."""

    def __init__(self, nx, ny, nz, bottom=None, top=None, T0=0.0):
        if (bottom is None) != (top is None):
            raise ValueError("give both z walls or neither")
        lib = _load()
        self.nx, self.ny, self.nz, self.T0 = int(nx), int(ny), int(nz), float(T0)
        walls = (bottom, top)
        kinds = (ctypes.c_int * 2)(*[0 if w is None else ZKINDS[w.kind] for w in walls])
        uw = np.array([[0.0, 0.0] if w is None else [w.ux, w.uy] for w in walls]).ravel()
        tw = np.array([0.0 if w is None else w.T for w in walls])
        h = lib.orc3_create(self.nx, self.ny, self.nz, kinds, _ptr(uw), _ptr(tw), self.T0)
        if not h:
            raise ValueError("oracle rejected the lattice description")
        self._h, self._lib = h, lib

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc3_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_params(self, tau_nu, tau_alpha, g_beta=0.0):
        self._lib.orc3_set_params(self._h, tau_nu, tau_alpha, g_beta)

    def set_relaxation(self, s_b=1.0, s3=1.0, s4=1.0, s5=1.0, s6=1.0, lambda2=1.0):
        self._lib.orc3_set_relaxation(self._h, s_b, s3, s4, s5, s6, lambda2)

    def set_body_force(self, Fx, Fy, Fz):
        self._lib.orc3_set_body_force(self._h, Fx, Fy, Fz)

    def init(self, rho=None, u=None, T=None):
        """u: None or a sequence of three fields (u_x, u_y, u_z), each broadcastable to the shape."""
        shp = self.shape
        uu = None if u is None else np.concatenate([_f64(c, shp).ravel() for c in u])
        self._lib.orc3_init(self._h, _ptr(_f64(rho, shp)), _ptr(uu), _ptr(_f64(T, shp)))

    def step(self, n=1):
        if self._lib.orc3_step(self._h, int(n)) != 0:
            raise RuntimeError("oracle: an unknown population survived the wall step")

    def moments(self):
        """(rho, (u_x, u_y, u_z), T)."""
        shp = self.shape
        n = self.nx * self.ny * self.nz
        rho, u, T = np.empty(n), np.empty(3 * n), np.empty(n)
        if self._lib.orc3_moments(self._h, _ptr(rho), _ptr(u), _ptr(T)) != 0:
            raise RuntimeError("oracle: an unknown population survived the wall step")
        return rho.reshape(shp), tuple(u[i * n:(i + 1) * n].reshape(shp) for i in range(3)), T.reshape(shp)

    def get_state(self):
        f = np.empty((27,) + self.shape)
        g = np.empty((7,) + self.shape)
        self._lib.orc3_get_state(self._h, _ptr(f), _ptr(g))
        return f, g

    def set_state(self, f, g):
        self._lib.orc3_set_state(self._h, _ptr(_f64(f)), _ptr(_f64(g)))

    def get_outgoing(self):
        out = np.empty((27,) + self.shape)
        self._lib.orc3_get_outgoing(self._h, _ptr(out))
        return out

    # -- single-node algebra ------------------------------------------------------------------
    def matrix_M(self):
        out = np.empty(27 * 27)
        self._lib.orc3_matrix_M(self._h, _ptr(out))
        return out.reshape(27, 27)

    def matrix_S(self):
        out = np.empty(27 * 27)
        self._lib.orc3_matrix_S(self._h, _ptr(out))
        return out.reshape(27, 27)

    def feq(self, rho, ux, uy, uz):
        out = np.empty(27)
        self._lib.orc3_feq(self._h, rho, ux, uy, uz, _ptr(out))
        return out

    def geq(self, T, ux, uy, uz):
        out = np.empty(7)
        self._lib.orc3_geq(self._h, T, ux, uy, uz, _ptr(out))
        return out

    def collide27(self, f, F=(0.0, 0.0, 0.0)):
        out = np.empty(27)
        self._lib.orc3_collide27(self._h, _ptr(_f64(f)), F[0], F[1], F[2], _ptr(out))
        return out

    def collide7(self, g, u):
        out = np.empty(7)
        self._lib.orc3_collide7(self._h, _ptr(_f64(g)), u[0], u[1], u[2], _ptr(out))
        return out


def lattice_from_workload(w):
    """An oracle lattice set up from a 3D workload description (see the package's workloads)."""
    walls = w.get("z_walls")
    bottom = top = None
    if walls is not None:
        bottom = Wall(walls[0]["kind"], *walls[0]["u"], T=walls[0]["T"])
        top = Wall(walls[1]["kind"], *walls[1]["u"], T=walls[1]["T"])
    L = OracleLattice3D(w["nx"], w["ny"], w["nz"], bottom, top, T0=w["T0"])
    t = w["taus"]
    L.set_params(t["tau_nu"], t["tau_alpha"], t["g_beta"])
    if "relaxation" in w:
        L.set_relaxation(**w["relaxation"])
    if "body_force" in w:
        L.set_body_force(*w["body_force"])
    fl = w["fields"]
    L.init(fl.get("rho"), fl.get("u"), fl.get("T"))
    return L
