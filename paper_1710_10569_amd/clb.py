"""Thin ctypes binding to libclb (include/clb.h): argument marshalling only.

Every step of the method runs in the HIP kernels of ``libclb.so``; nothing here computes.  The
library must have been built (``python -m paper_1710_10569_amd.build``); importing this module
without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CLB_LIBRARY selects another build of the same library (the tests load the debug variant this way)
LIBPATH = os.environ.get("CLB_LIBRARY") or os.path.join(_HERE, "libclb.so")

if not os.path.exists(LIBPATH):
    raise ImportError(f"{os.path.basename(LIBPATH)} is not built ({LIBPATH}); run `python -m paper_1710_10569_amd.build`")

# PyTorch ships its own HIP runtime under the same soname; load it first so that libclb binds to
# the same runtime instance and torch streams and device memory can be handed to the library.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is optional for the library itself
    torch = None

_lib = ctypes.CDLL(LIBPATH)

# enums of clb.h
CLB_OK, CLB_EINVAL, CLB_ENOMEM, CLB_EDEVICE, CLB_ESTATE, CLB_EDIVERGED = 0, -1, -2, -3, -4, -5
CLB_FP64, CLB_FP32_DEV, CLB_FP64_DEV, CLB_FP32_SR = 0, 1, 2, 3
CLB_PERIODIC, CLB_WALL_DIRICHLET, CLB_WALL_ADIABATIC = 0, 1, 2
PRECISIONS = {"fp64": CLB_FP64, "fp32": CLB_FP32_DEV, "fp32_dev": CLB_FP32_DEV, "fp64_dev": CLB_FP64_DEV,
              "fp32_sr": CLB_FP32_SR}
KINDS = {"periodic": CLB_PERIODIC, "dirichlet": CLB_WALL_DIRICHLET, "adiabatic": CLB_WALL_ADIABATIC}


class clb_edge(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("ux", ctypes.c_double), ("uy", ctypes.c_double), ("T", ctypes.c_double)]


class clb_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("precision", ctypes.c_int),
                ("west", clb_edge), ("east", clb_edge), ("south", clb_edge), ("north", clb_edge),
                ("T0", ctypes.c_double), ("prescribed_u", ctypes.c_int), ("in_place", ctypes.c_int)]


class clb_diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_longlong), ("mass", ctypes.c_double), ("heat", ctypes.c_double),
                ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double), ("sum_w", ctypes.c_double),
                ("sum_w_ux_T", ctypes.c_double), ("sum_w_uy_T", ctypes.c_double),
                ("wall_flux", ctypes.c_double * 4), ("u_max", ctypes.c_double),
                ("du_max", ctypes.c_double), ("dT_max", ctypes.c_double), ("nonfinite", ctypes.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "wall_flux"}
        d["wall_flux"] = list(self.wall_flux)
        return d


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_H = ctypes.c_void_p


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


_sig("clb_create", ctypes.c_int, [ctypes.POINTER(clb_desc), _vp, ctypes.POINTER(_H)])
_sig("clb_set_params", ctypes.c_int, [_H, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double])
_sig("clb_step", ctypes.c_int, [_H, ctypes.c_longlong])
_sig("clb_moments", ctypes.c_int, [_H, _dp, _dp, _dp])
_sig("clb_destroy", None, [_H])
_sig("clb_init", ctypes.c_int, [_H, _dp, _dp, _dp])
_sig("clb_set_relaxation", ctypes.c_int, [_H] + [ctypes.c_double] * 4)
_sig("clb_set_body_force", ctypes.c_int, [_H, ctypes.c_double, ctypes.c_double])
_sig("clb_set_prescribed_velocity", ctypes.c_int, [_H, ctypes.c_double, ctypes.c_double])
_sig("clb_diagnostics", ctypes.c_int, [_H, ctypes.c_int, ctypes.POINTER(clb_diag)])
_sig("clb_diagnostics_noalloc", ctypes.c_int, [_H, ctypes.POINTER(clb_diag)])
_sig("clb_get_populations", ctypes.c_int, [_H, _dp, _dp])
_sig("clb_checkpoint_size", ctypes.c_int, [_H, ctypes.POINTER(ctypes.c_size_t)])
_sig("clb_checkpoint_save", ctypes.c_int, [_H, _vp, ctypes.c_size_t])
_sig("clb_checkpoint_load", ctypes.c_int, [_H, _vp, ctypes.c_size_t])
_sig("clb_params_from_physics", ctypes.c_int, [ctypes.c_double] * 5 + [_dp, _dp, _dp])
_sig("clb_time_steps", ctypes.c_int, [_H, ctypes.c_longlong, _dp])
_sig("clb_synchronize", ctypes.c_int, [_H])
_sig("clb_last_error", ctypes.c_char_p, [])
_ip = ctypes.POINTER(ctypes.c_int)
_sig("clb_tile_shape_count", ctypes.c_int, [])
_sig("clb_tile_shape_info", ctypes.c_int, [ctypes.c_int, _ip, _ip, _ip, _ip])
_sig("clb_set_tile_shape", ctypes.c_int, [_H, ctypes.c_int])
_sig("clb_get_tile_shape", ctypes.c_int, [_H, _ip])
_sig("clb_autotune", ctypes.c_int, [_H, ctypes.c_int, _ip, _dp])
_sig("clb_time_shape", ctypes.c_int, [_H, ctypes.c_int, ctypes.c_int, _dp])


class CLBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"clb error {code}: {msg}")
        self.code = code


def last_error() -> str:
    return (_lib.clb_last_error() or b"").decode()


def _check(rc):
    if rc != CLB_OK:
        raise CLBError(rc, last_error())
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a, n):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def params_from_physics(Ra, Pr, Ma, H, dT):
    """(tau_nu, tau_alpha, g_beta) from (Ra, Pr, Ma, H, dT) through clb_params_from_physics."""
    t = [ctypes.c_double() for _ in range(3)]
    _check(_lib.clb_params_from_physics(Ra, Pr, Ma, H, dT, *[ctypes.byref(v) for v in t]))
    return tuple(v.value for v in t)


def tile_shapes():
    """[(tx, ty, spt, nontemporal)] of the compiled step-kernel tile shapes."""
    out = []
    for i in range(_lib.clb_tile_shape_count()):
        v = [ctypes.c_int() for _ in range(4)]
        _check(_lib.clb_tile_shape_info(i, *[ctypes.byref(x) for x in v]))
        out.append(tuple(x.value for x in v))
    return out


def make_desc(nx, ny, precision="fp64", edges=None, T0=0.0, prescribed=False, in_place=False):
    """clb_desc from sizes, a precision name or code, and {edge: (kind, ux, uy, T)}; prescribed:
    temperature-only lattice with a prescribed velocity; in_place: one population buffer."""
    d = clb_desc()
    d.nx, d.ny = int(nx), int(ny)
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    edges = edges or {}
    for name in ("west", "east", "south", "north"):
        kind, ux, uy, T = edges.get(name, ("periodic", 0.0, 0.0, 0.0))
        setattr(d, name, clb_edge(KINDS[kind] if isinstance(kind, str) else int(kind), ux, uy, T))
    d.T0 = float(T0)
    d.prescribed_u = 1 if prescribed else 0
    d.in_place = 1 if in_place else 0
    return d


class Lattice:
    """One lattice on the current HIP device (clb_create ... clb_destroy)."""

    def __init__(self, nx, ny, precision="fp64", edges=None, T0=0.0, stream=None, prescribed=False, in_place=False):
        self.desc = make_desc(nx, ny, precision, edges, T0, prescribed, in_place)
        self.nx, self.ny = int(nx), int(ny)
        h = _H()
        _check(_lib.clb_create(ctypes.byref(self.desc), None if stream is None else _vp(int(stream)),
                               ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.clb_destroy(self._h)
            self._h = None

    def __del__(self):
        # at interpreter exit the module's globals may already be cleared; the process
        # releases the device memory then anyway
        if _lib is not None:
            self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_params(self, tau_nu, tau_alpha, g_beta=0.0, Ma=0.0):
        _check(_lib.clb_set_params(self._h, tau_nu, tau_alpha, g_beta, Ma))

    def set_prescribed_velocity(self, ux, uy):
        """Velocity of a temperature-only lattice (created with prescribed=True)."""
        _check(_lib.clb_set_prescribed_velocity(self._h, ux, uy))

    def set_relaxation(self, s_b=1.0, s3=1.0, s4=1.0, lambda2=1.0):
        _check(_lib.clb_set_relaxation(self._h, s_b, s3, s4, lambda2))

    def set_body_force(self, Fvx, Fvy):
        _check(_lib.clb_set_body_force(self._h, Fvx, Fvy))

    def init(self, rho=None, ux=None, uy=None, T=None):
        n = self.nx * self.ny
        u = None
        if ux is not None or uy is not None:
            u = np.zeros(2 * n)
            if ux is not None:
                u[:n] = np.ravel(np.broadcast_to(ux, (self.ny, self.nx)))
            if uy is not None:
                u[n:] = np.ravel(np.broadcast_to(uy, (self.ny, self.nx)))
        r = None if rho is None else _f64(np.broadcast_to(rho, (self.ny, self.nx)), n)
        t = None if T is None else _f64(np.broadcast_to(T, (self.ny, self.nx)), n)
        _check(_lib.clb_init(self._h, _ptr(r), _ptr(u), _ptr(t)))

    def step(self, n=1):
        _check(_lib.clb_step(self._h, int(n)))

    def time_steps(self, n):
        ms = ctypes.c_double()
        _check(_lib.clb_time_steps(self._h, int(n), ctypes.byref(ms)))
        return ms.value

    def synchronize(self):
        _check(_lib.clb_synchronize(self._h))

    @property
    def tile_shape(self):
        v = ctypes.c_int()
        _check(_lib.clb_get_tile_shape(self._h, ctypes.byref(v)))
        return v.value

    @tile_shape.setter
    def tile_shape(self, shape):
        _check(_lib.clb_set_tile_shape(self._h, int(shape)))

    def autotune(self, launches_per_shape=20):
        """Time every tile shape (state unchanged), keep the fastest; returns (shape, us/launch)."""
        b, us = ctypes.c_int(), ctypes.c_double()
        _check(_lib.clb_autotune(self._h, int(launches_per_shape), ctypes.byref(b), ctypes.byref(us)))
        return b.value, us.value

    def time_shape(self, shape, launches=20):
        us = ctypes.c_double()
        _check(_lib.clb_time_shape(self._h, int(shape), int(launches), ctypes.byref(us)))
        return us.value

    def moments(self):
        """(rho, ux, uy, T), each (ny, nx) float64."""
        n = self.nx * self.ny
        rho, u, T = np.empty(n), np.empty(2 * n), np.empty(n)
        _check(_lib.clb_moments(self._h, _ptr(rho), _ptr(u), _ptr(T)))
        s = (self.ny, self.nx)
        return rho.reshape(s), u[:n].reshape(s), u[n:].reshape(s), T.reshape(s)

    def populations(self):
        """Post-streaming populations (f: (9, ny, nx), g: (5, ny, nx)); NaN where unknown."""
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((5, self.ny, self.nx))
        _check(_lib.clb_get_populations(self._h, _ptr(f), _ptr(g)))
        return f, g

    def diagnostics(self, snapshot=False, raise_on_diverged=True):
        d = clb_diag()
        rc = _lib.clb_diagnostics(self._h, int(bool(snapshot)), ctypes.byref(d))
        if rc != CLB_OK and (rc != CLB_EDIVERGED or raise_on_diverged):
            raise CLBError(rc, last_error())
        return d.as_dict()

    def diagnostics_noalloc(self, raise_on_diverged=True):
        """clb_diagnostics_noalloc: the record of diagnostics(snapshot=False) computed without
        allocating device memory (the library's fixed scratch; lattices of at most 8,388,608 nodes)."""
        d = clb_diag()
        rc = _lib.clb_diagnostics_noalloc(self._h, ctypes.byref(d))
        if rc != CLB_OK and (rc != CLB_EDIVERGED or raise_on_diverged):
            raise CLBError(rc, last_error())
        return d.as_dict()

    def checkpoint(self):
        """clb_checkpoint_save: the lattice's state, parameters and step count as bytes."""
        return checkpoint_blob(_lib.clb_checkpoint_size, _lib.clb_checkpoint_save, self._h)

    def restore(self, blob):
        """clb_checkpoint_load: continue from a checkpoint of a lattice of the same description."""
        restore_blob(_lib.clb_checkpoint_load, self._h, blob)


def checkpoint_blob(size_fn, save_fn, h):
    n = ctypes.c_size_t()
    _check(size_fn(h, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(save_fn(h, ctypes.cast(buf, _vp), n.value))
    return buf.raw


def restore_blob(load_fn, h, blob):
    b = bytes(blob)
    buf = ctypes.create_string_buffer(b, len(b))
    _check(load_fn(h, ctypes.cast(buf, _vp), len(b)))


def lattice_from_workload(w, precision="fp64", stream=None, in_place=False):
    """A Lattice set up and initialised from a workload description (see workloads.py)."""
    lat = Lattice(w["nx"], w["ny"], precision, w["edges"], w["T0"], stream=stream,
                  prescribed="prescribed_u" in w, in_place=in_place)
    if "prescribed_u" in w:
        lat.set_prescribed_velocity(*w["prescribed_u"])
    if "taus" in w:
        t = w["taus"]
        lat.set_params(t["tau_nu"], t["tau_alpha"], t["g_beta"], 0.0)
    else:
        p = w["physics"]
        tn, ta, gb = params_from_physics(p["Ra"], p["Pr"], p["Ma"], p["H"], p["dT"])
        lat.set_params(tn, ta, gb, p["Ma"])
    if "body_force" in w:
        lat.set_body_force(*w["body_force"])
    fl = w["fields"]
    lat.init(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    return lat


# ------------------------------------------------------------------------------------------------
# Batches (clb_batch_*).

_B = ctypes.c_void_p
_sig("clb_batch_footprint", ctypes.c_int, [ctypes.POINTER(clb_desc), ctypes.POINTER(ctypes.c_size_t)])
_sig("clb_batch_create", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp,
                                        ctypes.POINTER(_B)])
_sig("clb_batch_add", ctypes.c_int, [_B, ctypes.POINTER(clb_desc)] + [ctypes.c_double] * 4 + [ctypes.POINTER(ctypes.c_int)])
_sig("clb_batch_set_relaxation", ctypes.c_int, [_B, ctypes.c_int] + [ctypes.c_double] * 4)
_sig("clb_batch_set_body_force", ctypes.c_int, [_B, ctypes.c_int, ctypes.c_double, ctypes.c_double])
_sig("clb_batch_init", ctypes.c_int, [_B, ctypes.c_int, _dp, _dp, _dp])
_sig("clb_batch_moments", ctypes.c_int, [_B, ctypes.c_int, _dp, _dp, _dp])
_sig("clb_batch_diagnostics", ctypes.c_int, [_B, ctypes.c_int, ctypes.c_int, ctypes.POINTER(clb_diag)])
_sig("clb_batch_remove", ctypes.c_int, [_B, ctypes.c_int])
_sig("clb_batch_step", ctypes.c_int, [_B, ctypes.c_longlong])
_sig("clb_batch_step_each", ctypes.c_int, [_B, ctypes.c_longlong])
_sig("clb_batch_step_persistent", ctypes.c_int, [_B, ctypes.c_longlong])
_sig("clb_batch_check", ctypes.c_int, [_B])
_sig("clb_batch_time_steps", ctypes.c_int, [_B, ctypes.c_int, ctypes.c_longlong, _dp])
_sig("clb_batch_set_tile_width", ctypes.c_int, [_B, ctypes.c_int, ctypes.c_int])
_sig("clb_batch_autotune", ctypes.c_int, [_B, ctypes.c_int])
_sig("clb_batch_set_nontemporal", ctypes.c_int, [_B, ctypes.c_int])
_sig("clb_batch_get_tile_width", ctypes.c_int, [_B, ctypes.c_int, ctypes.POINTER(ctypes.c_int)])
_sig("clb_batch_get_nontemporal", ctypes.c_int, [_B, ctypes.POINTER(ctypes.c_int)])
_sig("clb_batch_info", ctypes.c_int, [_B, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_longlong)])
_sig("clb_batch_synchronize", ctypes.c_int, [_B])
_sig("clb_batch_residuals", ctypes.c_int, [_B, _dp, _dp, ctypes.POINTER(ctypes.c_int)])
_sig("clb_batch_destroy", None, [_B])

MODES = {"grouped": 0, "each": 1, "persistent": 2}


def footprint(nx, ny, precision="fp32", edges=None, T0=0.0, in_place=False):
    """Pool bytes one lattice occupies in a batch (clb_batch_footprint)."""
    d = make_desc(nx, ny, precision, edges, T0, in_place=in_place)
    v = ctypes.c_size_t()
    _check(_lib.clb_batch_footprint(ctypes.byref(d), ctypes.byref(v)))
    return v.value


class Batch:
    """Many lattices resident in one device pool (clb_batch_create ... clb_batch_destroy).

    pool: None (the library allocates `budget_bytes`) or a CUDA tensor whose memory becomes the
    pool (kept alive by this object)."""

    def __init__(self, capacity, precision="fp32", budget_bytes=1 << 30, pool=None, stream=None):
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self._pool = pool
        h = _B()
        if pool is not None:
            ptr, nbytes = pool.data_ptr(), pool.numel() * pool.element_size()
            rc = _lib.clb_batch_create(int(capacity), self.precision, 0, _vp(ptr), nbytes,
                                       None if stream is None else _vp(int(stream)), ctypes.byref(h))
        else:
            rc = _lib.clb_batch_create(int(capacity), self.precision, int(budget_bytes), None, 0,
                                       None if stream is None else _vp(int(stream)), ctypes.byref(h))
        _check(rc)
        self._h = h
        self._capacity = int(capacity)
        self.shapes = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.clb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        # at interpreter exit the module's globals may already be cleared; the process
        # releases the device memory then anyway
        if _lib is not None:
            self.close()

    def add(self, nx, ny, edges=None, T0=0.0, tau_nu=1.0, tau_alpha=1.0, g_beta=0.0, Ma=0.0, in_place=False):
        d = make_desc(nx, ny, self.precision, edges, T0, in_place=in_place)
        s = ctypes.c_int()
        _check(_lib.clb_batch_add(self._h, ctypes.byref(d), tau_nu, tau_alpha, g_beta, Ma, ctypes.byref(s)))
        self.shapes[s.value] = (int(nx), int(ny))
        return s.value

    def try_add(self, *a, **k):
        """add(), or None if the batch is full or the pool lacks space (CLB_ENOMEM)."""
        try:
            return self.add(*a, **k)
        except CLBError as e:
            if e.code == CLB_ENOMEM:
                return None
            raise

    def add_workload(self, w, in_place=False):
        """Admit and initialise a workload description (see workloads.py); returns the slot or None
        when it does not fit.  in_place: one population buffer (half the pool bytes)."""
        if "taus" in w:
            t = w["taus"]
            tn, ta, gb, Ma = t["tau_nu"], t["tau_alpha"], t["g_beta"], 0.0
        else:
            p = w["physics"]
            tn, ta, gb = params_from_physics(p["Ra"], p["Pr"], p["Ma"], p["H"], p["dT"])
            Ma = p["Ma"]
        slot = self.try_add(w["nx"], w["ny"], w["edges"], w["T0"], tn, ta, gb, Ma, in_place=in_place)
        if slot is None:
            return None
        if "body_force" in w:
            _check(_lib.clb_batch_set_body_force(self._h, slot, *w["body_force"]))
        fl = w["fields"]
        self.init(slot, fl["rho"], fl["ux"], fl["uy"], fl["T"])
        return slot

    def init(self, slot, rho=None, ux=None, uy=None, T=None):
        nx, ny = self.shapes[slot]
        n = nx * ny
        u = None
        if ux is not None or uy is not None:
            u = np.zeros(2 * n)
            if ux is not None:
                u[:n] = np.ravel(np.broadcast_to(ux, (ny, nx)))
            if uy is not None:
                u[n:] = np.ravel(np.broadcast_to(uy, (ny, nx)))
        r = None if rho is None else _f64(np.broadcast_to(rho, (ny, nx)), n)
        t = None if T is None else _f64(np.broadcast_to(T, (ny, nx)), n)
        _check(_lib.clb_batch_init(self._h, int(slot), _ptr(r), _ptr(u), _ptr(t)))

    def set_relaxation(self, slot, s_b=1.0, s3=1.0, s4=1.0, lambda2=1.0):
        _check(_lib.clb_batch_set_relaxation(self._h, int(slot), s_b, s3, s4, lambda2))

    def set_tile_width(self, slot, width):
        _check(_lib.clb_batch_set_tile_width(self._h, int(slot), int(width)))

    def tile_width(self, slot):
        """Current tile width of a slot: 64, 128, 256, or 0 for wrapped rows."""
        v = ctypes.c_int()
        _check(_lib.clb_batch_get_tile_width(self._h, int(slot), ctypes.byref(v)))
        return v.value

    def remove(self, slot):
        _check(_lib.clb_batch_remove(self._h, int(slot)))
        self.shapes.pop(slot, None)

    def step(self, n=1, mode="grouped"):
        fn = {"grouped": _lib.clb_batch_step, "each": _lib.clb_batch_step_each,
              "persistent": _lib.clb_batch_step_persistent}[mode]
        _check(fn(self._h, int(n)))

    def check(self):
        _check(_lib.clb_batch_check(self._h))

    def time_steps(self, n, mode="grouped"):
        ms = ctypes.c_double()
        _check(_lib.clb_batch_time_steps(self._h, MODES[mode], int(n), ctypes.byref(ms)))
        return ms.value

    def autotune(self, launches=5):
        _check(_lib.clb_batch_autotune(self._h, int(launches)))

    def set_nontemporal(self, on):
        _check(_lib.clb_batch_set_nontemporal(self._h, int(bool(on))))

    @property
    def nontemporal(self):
        """Store form of the next grouped step (True: non-temporal stores)."""
        v = ctypes.c_int()
        _check(_lib.clb_batch_get_nontemporal(self._h, ctypes.byref(v)))
        return bool(v.value)

    def synchronize(self):
        _check(_lib.clb_batch_synchronize(self._h))

    def info(self):
        c, u, b, s = ctypes.c_int(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_longlong()
        _check(_lib.clb_batch_info(self._h, ctypes.byref(c), ctypes.byref(u), ctypes.byref(b), ctypes.byref(s)))
        return {"count": c.value, "used_bytes": u.value, "budget_bytes": b.value, "sites": s.value}

    def moments(self, slot):
        nx, ny = self.shapes[slot]
        n = nx * ny
        rho, u, T = np.empty(n), np.empty(2 * n), np.empty(n)
        _check(_lib.clb_batch_moments(self._h, int(slot), _ptr(rho), _ptr(u), _ptr(T)))
        s = (ny, nx)
        return rho.reshape(s), u[:n].reshape(s), u[n:].reshape(s), T.reshape(s)

    def residuals(self):
        """{slot: (du, dT, nonfinite)} for every resident lattice: the max-norm change of u and of T
        since the previous call (or since initialisation); snapshots are then updated."""
        cap = self._capacity
        du, dT = np.empty(cap), np.empty(cap)
        nf = (ctypes.c_int * cap)()
        _check(_lib.clb_batch_residuals(self._h, _ptr(du), _ptr(dT), nf))
        return {s: (float(du[s]), float(dT[s]), bool(nf[s])) for s in self.shapes}

    def diagnostics(self, slot, snapshot=False, raise_on_diverged=True):
        d = clb_diag()
        rc = _lib.clb_batch_diagnostics(self._h, int(slot), int(bool(snapshot)), ctypes.byref(d))
        if rc != CLB_OK and (rc != CLB_EDIVERGED or raise_on_diverged):
            raise CLBError(rc, last_error())
        return d.as_dict()
