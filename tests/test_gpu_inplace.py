"""In-place streaming (one population buffer, AA pattern) through the C ABI: the same per-node
update as two-buffer pull streaming, so every moment and every post-streaming population must be
bitwise equal to the two-buffer path after odd and even step counts, for every wall kind, corner,
ragged size and precision; plus direct oracle parity, the halved footprint, and the error paths."""
import numpy as np
import pytest

from paper_1710_10569_amd import workloads as W
from tests.helpers import field_errors, oracle_from_workload, worst

pytestmark = pytest.mark.gpu


def _clb():
    from paper_1710_10569_amd import clb
    return clb


def cases():
    return [
        W.taylor_green(64),
        W.random_periodic(37, 29, seed=3, T0=0.2),
        W.random_walled(37, 29, seed=1, kinds=("dirichlet", "adiabatic", "adiabatic", "dirichlet"), wall_u=0.02,
                        g_beta=2e-3),
        W.random_walled(64, 21, seed=2, kinds=("adiabatic", "adiabatic", "dirichlet", "dirichlet"), wall_u=0.01),
        W.random_walled(19, 70, seed=4, kinds=("periodic", "periodic", "adiabatic", "dirichlet"), wall_u=0.02),
        W.random_walled(300, 5, seed=5, kinds=("dirichlet", "dirichlet", "periodic", "periodic")),
        W.random_walled(4, 9, seed=6, kinds=("dirichlet", "adiabatic", "dirichlet", "adiabatic"), wall_u=0.01),
        W.cavity(64, Ra=1e5),
        W.rayleigh_benard(300, 41, Ra=1e4, seed=5),
        # four and five rows between adiabatic y walls: the snapshot's depth-1 rows (2 and ny - 3)
        # coincide with a depth-0 row at ny = 4 and with each other at ny = 5
        W.random_walled(37, 4, seed=7, kinds=("dirichlet", "adiabatic", "adiabatic", "adiabatic"), wall_u=0.02,
                        g_beta=2e-3),
        W.random_walled(29, 5, seed=8, kinds=("adiabatic", "dirichlet", "adiabatic", "adiabatic"), wall_u=0.01,
                        g_beta=2e-3),
    ]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_sr"])
@pytest.mark.parametrize("case", range(11))
def test_in_place_equals_two_buffer(gpu, precision, case):
    clb = _clb()
    w = cases()[case]
    print(f"[inplace] {w['name']} {precision}", flush=True)
    a = clb.lattice_from_workload(w, precision, in_place=True)
    b = clb.lattice_from_workload(w, precision)
    done = 0
    for n in (0, 1, 1, 5, 43):
        a.step(n)
        b.step(n)
        done += n
        for x, y in zip(a.moments(), b.moments()):
            assert np.array_equal(x, y), (w["name"], precision, done)
        fa, ga = a.populations()
        fb, gb = b.populations()
        assert np.array_equal(fa, fb, equal_nan=True) and np.array_equal(ga, gb, equal_nan=True), (w["name"], done)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp32_sr"])
def test_in_place_workgroup_widths_agree(gpu, precision):
    """The in-place kernel in 64- and 256-node workgroups, with ordinary and non-temporal stores
    (tile shapes 2, 6, 11, 12), gives bitwise the same lattice after an odd number of steps."""
    clb = _clb()
    w = W.random_walled(300, 37, seed=12, kinds=("dirichlet", "adiabatic", "adiabatic", "dirichlet"), wall_u=0.02,
                        g_beta=2e-3)
    ref = None
    for shape in (2, 6, 11, 12):
        g = clb.lattice_from_workload(w, precision, in_place=True)
        g.tile_shape = shape
        g.step(37)
        f, gg = g.populations()
        g.close()
        if ref is None:
            ref = (f, gg)
        else:
            assert np.array_equal(f, ref[0], equal_nan=True) and np.array_equal(gg, ref[1], equal_nan=True), shape


def test_in_place_matches_oracle(gpu):
    """Walled lattice with moving walls, buoyancy and both wall kinds, 301 steps in FP64."""
    clb = _clb()
    w = W.random_walled(45, 38, seed=8, kinds=("dirichlet", "adiabatic", "adiabatic", "dirichlet"), wall_u=0.02,
                        g_beta=2e-3)
    g = clb.lattice_from_workload(w, "fp64", in_place=True)
    o = oracle_from_workload(w)
    g.step(301)
    o.step(301)
    e = field_errors(g.moments(), o.moments(), w["T0"], w["u_scale"])
    assert worst(e) < 1e-12, e
    g.close()


def test_in_place_halves_the_footprint(gpu):
    import torch
    clb = _clb()
    w = W.rayleigh_benard(4096, 2048, Ra=1e6, seed=3)
    used = {}
    for ip in (False, True):
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        lat = clb.lattice_from_workload(w, "fp32", in_place=ip)
        lat.synchronize()
        used[ip] = free0 - torch.cuda.mem_get_info()[0]
        lat.close()
    buf = 14 * 4 * 4096 * 2048
    print(f"[inplace] device bytes: two-buffer {used[False]}, in-place {used[True]}, buffer {buf}", flush=True)
    assert used[False] - used[True] > 0.9 * buf


def test_in_place_errors(gpu):
    import ctypes
    clb = _clb()
    with pytest.raises(clb.CLBError):
        clb.Lattice(8, 8, "fp64", prescribed=True, in_place=True)
    edges = {k: ("dirichlet", 0.0, 0.0, 0.0) for k in ("west", "east", "south", "north")}
    with pytest.raises(clb.CLBError):
        clb.Lattice(3, 8, "fp64", edges, in_place=True)
    lat = clb.Lattice(8, 8, "fp32", in_place=True)
    with pytest.raises(clb.CLBError):
        lat.autotune(2)
    lat.close()
    b = clb.Batch(2, "fp64", budget_bytes=16 << 20)
    d = clb.make_desc(3, 8, "fp64", edges, in_place=True)      # too narrow for in-place walls
    slot = ctypes.c_int(-1)
    rc = clb._lib.clb_batch_add(b._h, ctypes.byref(d), 0.8, 0.8, 0.0, 0.0, ctypes.byref(slot))
    assert rc == clb.CLB_EINVAL
    b.close()
