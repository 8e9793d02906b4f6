"""CPU-side checks of the C ABI: the library loads, exports every function include/clb.h and
include/clb3d.h declare, and rejects invalid descriptions on the host before touching a device.  No
compute call is made."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(header="clb.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(clb3?d?_[a-z_]+)\s*\(", src)))


def test_header_declares_the_core_calls():
    names = header_functions()
    for core in ("clb_create", "clb_set_params", "clb_step", "clb_moments", "clb_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_1710_10569_amd import clb
    lib = ctypes.CDLL(clb.LIBPATH)
    names = header_functions("clb.h") + header_functions("clb3d.h")
    assert "clb3d_create" in names and "clb3d_step" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("bad", [
    dict(nx=0, ny=4, nz=4),
    dict(nx=4, ny=4, nz=2, walls=True),                                   # walls need nz >= 3
    dict(nx=4, ny=4, nz=4, precision=9),
    dict(nx=4, ny=4, nz=4, bottom_only=True),                             # one wall, one periodic side
    dict(nx=4, ny=4, nz=4, walls=True, T=float("nan")),
    dict(nx=2000, ny=2000, nz=1000),                                      # more than 2e9 nodes
])
def test_3d_create_rejects_bad_descriptions_on_host(bad):
    from paper_1710_10569_amd import clb, clb3d
    w = ("dirichlet", (0.0, 0.0), bad.get("T", 0.0)) if bad.get("walls") else None
    d = clb3d.make_desc(bad["nx"], bad["ny"], bad["nz"], bad.get("precision", "fp64"), w, w)
    if bad.get("bottom_only"):
        d.bottom.kind = clb3d.CLB3D_DIRICHLET
    h = ctypes.c_void_p()
    rc = clb._lib.clb3d_create(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == clb.CLB_EINVAL and not h.value and clb.last_error()
    assert clb._lib.clb3d_footprint(ctypes.byref(d)) == 0


def test_checkpoint_calls_reject_null_arguments():
    from paper_1710_10569_amd import clb
    n = ctypes.c_size_t()
    for fn in (clb._lib.clb_checkpoint_size, clb._lib.clb3d_checkpoint_size):
        assert fn(None, ctypes.byref(n)) == clb.CLB_EINVAL
    for fn in (clb._lib.clb_checkpoint_save, clb._lib.clb_checkpoint_load, clb._lib.clb3d_checkpoint_save,
               clb._lib.clb3d_checkpoint_load):
        assert fn(None, None, 0) == clb.CLB_EINVAL


def test_3d_null_arguments_and_footprint():
    from paper_1710_10569_amd import clb, clb3d
    assert clb._lib.clb3d_create(None, None, None) == clb.CLB_EINVAL
    clb._lib.clb3d_destroy(None)
    assert clb._lib.clb3d_step(None, 1) == clb.CLB_EINVAL
    assert clb._lib.clb3d_moments(None, None, None, None) == clb.CLB_EINVAL
    # two FP32 buffers of 34 populations per node in 64-node chunks, plus FP64 fields and partials
    fp = clb3d.footprint(256, 256, 129, "fp32_sr", walls=True)
    n = 256 * 256 * 129
    assert fp == 2 * 4 * 34 * n + 5 * 8 * n + (n + 255) // 256 * 7 * 8 + 16 * 8


def test_params_from_physics_matches_sec33_relations():
    """nu = Ma c_s H sqrt(Pr/Ra), alpha = nu/Pr, g beta = Ra nu alpha/(dT H^3) (Sec. 3.3), tau_nu =
    3 nu + 1/2 (Sec. 2.1), tau_alpha = 4 alpha + 1/2 (Sec. 2.2 with c_T^2 = 1/4)."""
    from paper_1710_10569_amd import clb
    tn, ta, gb = clb.params_from_physics(1e5, 0.71, 0.1, 255.0, 1.0)
    nu = 0.1 / math.sqrt(3) * 255 * math.sqrt(0.71 / 1e5)
    alpha = nu / 0.71
    assert tn == pytest.approx(3 * nu + 0.5, rel=1e-15)
    assert ta == pytest.approx(4 * alpha + 0.5, rel=1e-15)
    assert gb == pytest.approx(1e5 * nu * alpha / 255 ** 3, rel=1e-14)
    # the resulting characteristic velocity sqrt(g beta dT H) is Ma c_s
    assert math.sqrt(gb * 255) == pytest.approx(0.1 / math.sqrt(3), rel=1e-14)
    with pytest.raises(clb.CLBError):
        clb.params_from_physics(-1.0, 0.71, 0.1, 255.0, 1.0)


@pytest.mark.parametrize("bad", [
    dict(nx=2, ny=10),
    dict(nx=10, ny=10, edges={"west": ("dirichlet", 0, 0, 1)}),            # west wall, east periodic
    dict(nx=10, ny=3, edges={"south": ("adiabatic", 0, 0, 0), "north": ("adiabatic", 0, 0, 0)}),
    dict(nx=10, ny=10, precision=7),
    dict(nx=10, ny=10, edges={"south": ("dirichlet", 0.6, 0, 0), "north": ("dirichlet", 0, 0, 0)}),
    dict(nx=10, ny=10, T0=float("nan")),
    dict(nx=10, ny=10, prescribed=True, in_place=True),                  # in-place is flow lattices only
    dict(nx=3, ny=10, in_place=True, edges={"west": ("dirichlet", 0, 0, 1), "east": ("dirichlet", 0, 0, 0)}),
    dict(nx=10, ny=10, in_place=2),
    dict(nx=3, ny=(1 << 18) + 1),                                         # taller than the launch grids allow
    dict(nx=(1 << 20) + 1, ny=3),
    dict(nx=1 << 15, ny=(1 << 15) + 1),                                   # more than 2^30 nodes
])
def test_create_rejects_bad_descriptions_on_host(bad):
    from paper_1710_10569_amd import clb
    d = clb.make_desc(bad["nx"], bad["ny"], bad.get("precision", "fp64"), bad.get("edges"), bad.get("T0", 0.0),
                      bad.get("prescribed", False), bad.get("in_place", False))
    if bad.get("in_place") == 2:
        d.in_place = 2
    h = ctypes.c_void_p()
    rc = clb._lib.clb_create(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == clb.CLB_EINVAL
    assert not h.value
    assert clb.last_error()


def test_null_arguments():
    from paper_1710_10569_amd import clb
    assert clb._lib.clb_create(None, None, None) == clb.CLB_EINVAL
    clb._lib.clb_destroy(None)   # NULL-safe
    assert clb._lib.clb_step(None, 1) == clb.CLB_EINVAL
    assert clb._lib.clb_moments(None, None, None, None) == clb.CLB_EINVAL


def test_batch_footprint_and_host_side_rejections():
    """Pool bytes per lattice: two population buffers (rows of 64-node chunks of 14 populations:
    ceil(nx / 64) * 14 * 64 values per row) plus an FP64 (u_x, u_y, T) snapshot; bad batch arguments
    are rejected before any device call."""
    from paper_1710_10569_amd import clb
    fp = clb.footprint(100, 60, "fp32")
    row = 2 * 14 * 64                            # 100 nodes: two 64-node chunks per row
    buf = -(-row * 60 * 4 // 256) * 256
    snap = -(-3 * 100 * 60 * 8 // 256) * 256
    assert fp == 2 * buf + snap
    assert clb.footprint(100, 60, "fp64") > fp
    h = ctypes.c_void_p()
    assert clb._lib.clb_batch_create(0, clb.CLB_FP32_DEV, 1 << 20, None, 0, None, ctypes.byref(h)) == clb.CLB_EINVAL
    assert clb._lib.clb_batch_create(4, 9, 1 << 20, None, 0, None, ctypes.byref(h)) == clb.CLB_EINVAL
    assert clb._lib.clb_batch_create(4, clb.CLB_FP32_DEV, 1 << 20, None, 0, None, None) == clb.CLB_EINVAL
    clb._lib.clb_batch_destroy(None)
    assert clb._lib.clb_batch_step(None, 1) == clb.CLB_EINVAL
