"""Temperature-only lattices on the GPU (prescribed velocity, Sec. 3.1): only the D2Q5 CLB equation
runs, with a given uniform velocity.  Parity with the oracle's temperature-only mode, on the moving
frame of Eq. 24 and on walled lattices (every branch of the temperature wall step), and the paper's
Fig. 1b claim measured on the GPU: the measured diffusivity does not depend on Ma."""
import ctypes
import json
import math
import os

import numpy as np
import pytest

from paper_1710_10569_amd import workloads as W
from tests.helpers import field_errors, oracle_from_workload

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = {"fp64": 1e-12, "fp64_dev": 1e-12, "fp32": 1e-5, "fp32_sr": 1e-5}


def _clb():
    from paper_1710_10569_amd import clb
    return clb


def _pair(w, precision, steps, chunks):
    clb = _clb()
    print(f"[prescribed] {w['name']} {precision} steps={steps}", flush=True)
    g = clb.lattice_from_workload(w, precision)
    o = oracle_from_workload(w)
    errs = []
    for _ in range(chunks):
        g.step(steps // chunks)
        o.step(steps // chunks)
        gm, om = g.moments(), o.moments()
        # the velocity comes back in the arithmetic type of the mode (FP32 for "fp32")
        pu = [float(np.float32(v)) if precision == "fp32" else v for v in w["prescribed_u"]]
        assert np.all(gm[0] == 1.0)
        assert np.all(gm[1] == pu[0]) and np.all(gm[2] == pu[1])
        errs.append(field_errors(gm, om, w["T0"], w["u_scale"]))
    g.close()
    return errs


# FP32 collision on the moving frame: the wave is 1 % of the mean temperature (B = 0.01, T0 = 1),
# and the collision forms T = T0 + dT and u T in FP32, resolved to 2^-24 T0 = 6e-8, i.e. 6e-6 of B
# per rounding; measured 1.2e-5 after 2000 steps.  The FP64-collision form (fp32_sr) stays at 1e-5.
MOVING_TOL = dict(TOL, fp32=3e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp64_dev", "fp32", "fp32_sr"])
def test_moving_frame_matches_oracle(gpu, precision):
    """Eq. 24 at Ma = 0.3 (L = 100, B = 0.01, alpha = 0.05), 2000 steps, every node compared."""
    w = W.moving_frame(Ma=0.3)
    for e in _pair(w, precision, 2000, 4):
        assert e["T"] < MOVING_TOL[precision], e


@pytest.mark.parametrize("precision", ["fp64", "fp32_sr"])
@pytest.mark.parametrize("shape,kinds", [
    ((37, 29), ("dirichlet", "adiabatic", "adiabatic", "dirichlet")),
    ((64, 21), ("adiabatic", "adiabatic", "dirichlet", "dirichlet")),
    ((19, 70), ("periodic", "periodic", "adiabatic", "dirichlet")),
])
def test_prescribed_walls_match_oracle(gpu, precision, shape, kinds):
    """Random temperature fields advected by an oblique prescribed velocity between Dirichlet and
    adiabatic walls (edges and corners of every kind), ragged sizes, 300 steps."""
    w = W.prescribed_walled(*shape, seed=shape[0] + 3 * shape[1], kinds=kinds)
    for e in _pair(w, precision, 300, 3):
        assert e["T"] < TOL[precision], e


@pytest.mark.parametrize("precision", ["fp64", "fp32_sr"])
def test_moving_frame_diffusivity_independent_of_Ma(gpu, precision):
    """Fig. 1b on the GPU: the decay rate of the wave's Fourier amplitude up to t* = 2 gives the
    measured diffusivity, equal to the given alpha = 0.05 within 1e-3 and the same (within
    1e-4 alpha) for Ma = 0, 0.1, 0.2, 0.3."""
    clb = _clb()
    g = json.load(open(os.path.join(GOLD, "moving_frame.json")))
    Lw, alpha = g["L"], g["alpha"]
    phi = 2 * math.pi / Lw
    nst = int(2.0 / (phi * phi * alpha))
    measured = []
    for Ma in g["Ma"]:
        w = W.moving_frame(L=Lw, B=g["B"], alpha=alpha, T0=g["T0"], Ma=Ma)
        lat = clb.lattice_from_workload(w, precision)
        ts, am = [], []
        for s in range(0, nst + 1, nst // 10):
            if s:
                lat.step(nst // 10)
            T = lat.moments()[3]
            ts.append(s)
            am.append(abs(np.fft.fft(T[:, 0] - g["T0"])[1]))
        lat.close()
        rate = -np.polyfit(ts[1:], np.log(am[1:]), 1)[0]
        measured.append(rate / (phi * phi))
        print(f"[prescribed] {precision} Ma={Ma}: alpha_eff/alpha - 1 = {measured[-1] / alpha - 1:.3e}", flush=True)
        assert measured[-1] / alpha - 1 == pytest.approx(0, abs=1e-3)
    assert max(measured) - min(measured) < 1e-4 * alpha


def test_prescribed_errors(gpu):
    clb = _clb()
    g = clb.Lattice(8, 8, "fp64")
    with pytest.raises(clb.CLBError):
        g.set_prescribed_velocity(0.0, 0.1)        # not a temperature-only lattice
    g.close()
    p = clb.Lattice(8, 8, "fp64", prescribed=True)
    with pytest.raises(clb.CLBError):
        p.set_prescribed_velocity(0.6, 0.6)        # |u|^2 >= 1/2
    p.close()
    b = clb.Batch(2, "fp64", budget_bytes=16 << 20)
    d = clb.make_desc(8, 8, "fp64", prescribed=True)
    slot = ctypes.c_int(-1)
    rc = clb._lib.clb_batch_add(b._h, ctypes.byref(d), 0.8, 0.8, 0.0, 0.0, ctypes.byref(slot))
    assert rc == clb.CLB_EINVAL and "single-lattice" in clb.last_error()
    b.close()
