"""Thin ctypes binding to the three-dimensional path of libclb (include/clb3d.h): argument
marshalling only.  Every step runs in the HIP kernels of ``libclb.so``; importing without the
built library raises ImportError (through ``clb``), there is no fallback.

Fields are numpy arrays of shape (nz, ny, nx); velocities are three such arrays (u_x, u_y, u_z).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import clb as _clb
from .clb import CLBError, PRECISIONS, _check, _dp, _ptr, _vp

_lib = _clb._lib
_H = ctypes.c_void_p

CLB3D_PERIODIC, CLB3D_DIRICHLET, CLB3D_ADIABATIC = 0, 1, 2
WALL_KINDS = {"periodic": CLB3D_PERIODIC, "dirichlet": CLB3D_DIRICHLET, "adiabatic": CLB3D_ADIABATIC}


class clb3d_wall(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("ux", ctypes.c_double), ("uy", ctypes.c_double), ("T", ctypes.c_double)]


class clb3d_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("precision", ctypes.c_int),
                ("bottom", clb3d_wall), ("top", clb3d_wall), ("T0", ctypes.c_double)]


class clb3d_diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3), ("heat", ctypes.c_double),
                ("uzT", ctypes.c_double), ("plane_T", ctypes.c_double * 6), ("max_speed", ctypes.c_double),
                ("step", ctypes.c_longlong)]

    def as_dict(self):
        return {"mass": self.mass, "momentum": list(self.momentum), "heat": self.heat, "uzT": self.uzT,
                "plane_T": list(self.plane_T), "max_speed": self.max_speed, "step": self.step}


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


_d = ctypes.c_double
_sig("clb3d_create", ctypes.c_int, [ctypes.POINTER(clb3d_desc), _vp, ctypes.POINTER(_H)])
_sig("clb3d_set_params", ctypes.c_int, [_H, _d, _d, _d])
_sig("clb3d_set_relaxation", ctypes.c_int, [_H] + [_d] * 6)
_sig("clb3d_set_body_force", ctypes.c_int, [_H, _d, _d, _d])
_sig("clb3d_init", ctypes.c_int, [_H, _dp, _dp, _dp])
_sig("clb3d_step", ctypes.c_int, [_H, ctypes.c_longlong])
_sig("clb3d_moments", ctypes.c_int, [_H, _dp, _dp, _dp])
_sig("clb3d_diagnostics", ctypes.c_int, [_H, ctypes.POINTER(clb3d_diag)])
_sig("clb3d_time_steps", ctypes.c_int, [_H, ctypes.c_longlong, _dp])
_sig("clb3d_synchronize", ctypes.c_int, [_H])
_sig("clb3d_footprint", ctypes.c_size_t, [ctypes.POINTER(clb3d_desc)])
_sig("clb3d_destroy", None, [_H])
_sig("clb3d_checkpoint_size", ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_size_t)])
_sig("clb3d_checkpoint_save", ctypes.c_int, [_H, _vp, ctypes.c_size_t])
_sig("clb3d_checkpoint_load", ctypes.c_int, [_H, _vp, ctypes.c_size_t])


def make_desc(nx, ny, nz, precision="fp32_sr", bottom=None, top=None, T0=0.0):
    """bottom/top: None (periodic z) or (kind, (ux, uy), T) with kind 'dirichlet' or 'adiabatic'."""
    if (bottom is None) != (top is None):
        raise ValueError("give both z walls or neither")
    d = clb3d_desc()
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for name, w in (("bottom", bottom), ("top", top)):
        s = getattr(d, name)
        if w is None:
            s.kind, s.ux, s.uy, s.T = CLB3D_PERIODIC, 0.0, 0.0, 0.0
        else:
            kind, (ux, uy), T = w
            s.kind, s.ux, s.uy, s.T = WALL_KINDS[kind], float(ux), float(uy), float(T)
    d.T0 = float(T0)
    return d


def footprint(nx, ny, nz, precision="fp32_sr", walls=False):
    w = ("dirichlet", (0.0, 0.0), 0.0) if walls else None
    return int(_lib.clb3d_footprint(ctypes.byref(make_desc(nx, ny, nz, precision, w, w))))


class Lattice3D:
    """One 3D lattice on the current HIP device (clb3d_create ... clb3d_destroy)."""

    def __init__(self, nx, ny, nz, precision="fp32_sr", bottom=None, top=None, T0=0.0, stream=None):
        self.desc = make_desc(nx, ny, nz, precision, bottom, top, T0)
        self.shape = (int(nz), int(ny), int(nx))
        h = _H()
        _check(_lib.clb3d_create(ctypes.byref(self.desc), None if stream is None else _vp(int(stream)), ctypes.byref(h)))
        self._h = h

    @property
    def n(self):
        return self.shape[0] * self.shape[1] * self.shape[2]

    def close(self):
        if getattr(self, "_h", None):
            _lib.clb3d_destroy(self._h)
            self._h = None

    def __del__(self):
        # at interpreter exit the module's globals may already be cleared; the process
        # releases the device memory then anyway
        if _lib is not None:
            self.close()

    def set_params(self, tau_nu, tau_alpha, g_beta=0.0):
        _check(_lib.clb3d_set_params(self._h, tau_nu, tau_alpha, g_beta))

    def set_relaxation(self, s_b=1.0, s3=1.0, s4=1.0, s5=1.0, s6=1.0, lambda2=1.0):
        _check(_lib.clb3d_set_relaxation(self._h, s_b, s3, s4, s5, s6, lambda2))

    def set_body_force(self, Fx, Fy, Fz):
        _check(_lib.clb3d_set_body_force(self._h, Fx, Fy, Fz))

    def init(self, rho=None, u=None, T=None):
        shp = self.shape

        def plane(a):
            return None if a is None else np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shp))

        uu = None if u is None else np.ascontiguousarray(np.concatenate([plane(c).ravel() for c in u]))
        r, t = plane(rho), plane(T)
        _check(_lib.clb3d_init(self._h, _ptr(r), _ptr(uu), _ptr(t)))

    def step(self, n=1):
        _check(_lib.clb3d_step(self._h, int(n)))

    def moments(self):
        """(rho, (u_x, u_y, u_z), T) as FP64 arrays of shape (nz, ny, nx)."""
        n = self.n
        rho, u, T = np.empty(n), np.empty(3 * n), np.empty(n)
        _check(_lib.clb3d_moments(self._h, _ptr(rho), _ptr(u), _ptr(T)))
        s = self.shape
        return rho.reshape(s), tuple(u[i * n:(i + 1) * n].reshape(s) for i in range(3)), T.reshape(s)

    def diagnostics(self):
        d = clb3d_diag()
        _check(_lib.clb3d_diagnostics(self._h, ctypes.byref(d)))
        return d.as_dict()

    def time_steps(self, n):
        ms = ctypes.c_double()
        _check(_lib.clb3d_time_steps(self._h, int(n), ctypes.byref(ms)))
        return ms.value

    def synchronize(self):
        _check(_lib.clb3d_synchronize(self._h))

    def checkpoint(self):
        """clb3d_checkpoint_save: the lattice's state, parameters and step count as bytes."""
        return _clb.checkpoint_blob(_lib.clb3d_checkpoint_size, _lib.clb3d_checkpoint_save, self._h)

    def restore(self, blob):
        """clb3d_checkpoint_load: continue from a checkpoint of a lattice of the same description."""
        _clb.restore_blob(_lib.clb3d_checkpoint_load, self._h, blob)


def lattice_from_workload(w, precision="fp32_sr", stream=None):
    """A device lattice set up from a 3D workload description (see workloads.py)."""
    walls = w.get("z_walls")
    b = t = None
    if walls is not None:
        b = (walls[0]["kind"], tuple(walls[0]["u"]), walls[0]["T"])
        t = (walls[1]["kind"], tuple(walls[1]["u"]), walls[1]["T"])
    L = Lattice3D(w["nx"], w["ny"], w["nz"], precision, b, t, w["T0"], stream=stream)
    tt = w["taus"]
    L.set_params(tt["tau_nu"], tt["tau_alpha"], tt["g_beta"])
    if "relaxation" in w:
        L.set_relaxation(**w["relaxation"])
    if "body_force" in w:
        L.set_body_force(*w["body_force"])
    fl = w["fields"]
    L.init(fl.get("rho"), fl.get("u"), fl.get("T"))
    return L


__all__ = ["Lattice3D", "lattice_from_workload", "footprint", "make_desc", "CLBError"]
