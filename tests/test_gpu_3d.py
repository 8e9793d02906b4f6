"""GPU parity of the three-dimensional path (D3Q27 flow, D3Q7 temperature) against the 3D oracle,
through the C ABI (include/clb3d.h).

Bars: FP64 within 1e-12 of the oracle, FP32 storage with stochastic rounding within 1e-5, plain
FP32 within 3e-5 (each field's max-norm error over the largest departure of the oracle's field
from its rest value: rho against max |rho|, u against max |u|, T against max |T - T0|).  Cases:
ragged sizes (nx not a multiple of the 64-node chunk, ny not a multiple of the 4-row tile),
degenerate ones (one node across in x or y), periodic and walled z, moving walls, Dirichlet and
adiabatic, buoyancy, a body force and every relaxation rate away from 1; a Rayleigh-Benard layer
over 1500 steps; the benchmark's full 256 x 256 x 129 layer over a few steps, every node compared;
and properties at full size (mass in a closed box, the ABC decay rate)."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import o3d
from paper_1710_10569_amd import workloads as W
from tests.helpers import rel_err

TOL = {"fp64": 1e-12, "fp32_sr": 1e-5, "fp32": 3e-5}
REL = {"s_b": 1.3, "s3": 1.2, "s4": 1.1, "s5": 1.4, "s6": 1.6, "lambda2": 1.15}


def _clb3():
    from paper_1710_10569_amd import clb3d
    return clb3d


def errors3(gpu_m, orc_m, T0):
    (r, u, T), (rr, ru, rT) = gpu_m, orc_m
    if np.isnan(r).any() or any(np.isnan(c).any() for c in u) or np.isnan(T).any():
        return {"rho": math.inf, "u": math.inf, "T": math.inf}
    du = max(np.abs(a - b).max() for a, b in zip(u, ru))
    umax = max(np.abs(b).max() for b in ru)
    return {"rho": rel_err(r, rr), "u": float(du / umax) if umax > 0 else float(du), "T": rel_err(T, rT, T0)}


def gpu_lattice(w, precision):
    clb3d = _clb3()
    if "physics" in w:
        from paper_1710_10569_amd import clb
        p = w["physics"]
        w = dict(w, taus=dict(zip(("tau_nu", "tau_alpha", "g_beta"), clb.params_from_physics(p["Ra"], p["Pr"], p["Ma"], p["H"], p["dT"]))))
    return clb3d.lattice_from_workload(w, precision)


def oracle_lattice(w):
    if "physics" in w:
        p = w["physics"]
        w = dict(w, taus=dict(zip(("tau_nu", "tau_alpha", "g_beta"), O.params_from_physics(p["Ra"], p["Pr"], p["Ma"], p["H"], p["dT"]))))
    return o3d.lattice_from_workload(w)


WALLS_A = (("dirichlet", (0.01, -0.02), 0.3), ("adiabatic", (-0.005, 0.004), 0.0))
WALLS_B = (("adiabatic", (0.0, 0.0), 0.0), ("dirichlet", (0.02, 0.0), -0.2))
CASES = {
    "periodic_9x7x8": dict(shape=(9, 7, 8), walls=None),
    "periodic_70x5x6": dict(shape=(70, 5, 6), walls=None),
    "periodic_1x1x16": dict(shape=(1, 1, 16), walls=None),
    "walls_9x7x8": dict(shape=(9, 7, 8), walls=WALLS_A),
    "walls_33x9x10": dict(shape=(33, 9, 10), walls=WALLS_B),
    "walls_130x1x5": dict(shape=(130, 1, 5), walls=WALLS_A),
}
_orc_cache = {}


def _case_workload(name):
    c = CASES[name]
    return W.random_3d(*c["shape"], seed=7, walls=c["walls"], relaxation=REL)


def _oracle_moments(name, steps):
    key = (name, steps)
    if key not in _orc_cache:
        L = oracle_lattice(_case_workload(name))
        L.step(steps)
        _orc_cache[key] = L.moments()
    return _orc_cache[key]


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32_sr", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_parity_3d(gpu, precision, case):
    w = _case_workload(case)
    print(f"[3d] {case} {precision}", flush=True)
    L = gpu_lattice(w, precision)
    done = 0
    for steps in (0, 1, 40):
        L.step(steps - done)
        done = steps
        e = errors3(L.moments(), _oracle_moments(case, steps), w["T0"])
        assert max(e.values()) < TOL[precision], (case, precision, steps, e)
    L.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32_sr"])
def test_rayleigh_benard_3d_long_run(gpu, precision):
    """A 24 x 24 x 13 layer at Ra = 1e4 started from crossed convection rolls (u up to 0.04), 1500
    steps.  (From a perturbed conduction profile u stays below 1e-4 this early, and two FP64 builds
    of the oracle that differ only in multiply-add contraction already differ by 8e-12 of it.)"""
    w = W.rayleigh_benard_3d(24, 24, 13, Ra=1e4, Ma=0.1, seed=11, rolls=0.5)
    key = ("rb3d_long", 1500)
    if key not in _orc_cache:
        L = oracle_lattice(w)
        L.step(1500)
        _orc_cache[key] = L.moments()
    print(f"[3d] rb long {precision}", flush=True)
    G = gpu_lattice(w, precision)
    G.step(1500)
    e = errors3(G.moments(), _orc_cache[key], w["T0"])
    assert max(e.values()) < TOL[precision], e
    G.close()


@pytest.mark.gpu
def test_rayleigh_benard_3d_full_size(gpu):
    """The benchmark's layer, 256 x 256 x 129 (8.45 M nodes) started from convection rolls, in the
    launch configuration the benchmark times: three steps, every node of rho, u, T compared with the
    oracle, in the three precisions the benchmark times (FP64, SR and plain FP32)."""
    w = W.rayleigh_benard_3d(256, 256, 129, Ra=1e5, Ma=0.1, seed=3, rolls=0.5)
    print("[3d] full size: oracle", flush=True)
    L = oracle_lattice(w)
    L.step(3)
    ref = L.moments()
    L.close()
    for precision in ("fp64", "fp32_sr", "fp32"):
        print(f"[3d] full size {precision}", flush=True)
        G = gpu_lattice(w, precision)
        G.step(3)
        e = errors3(G.moments(), ref, w["T0"])
        assert max(e.values()) < TOL[precision], (precision, e)
        G.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32_sr", "fp32"])
def test_rayleigh_benard_3d_stored_state(gpu, precision):
    """The benchmark's layer in its launch configuration, 50 steps from crossed rolls: 1024 sampled
    nodes and two wall-to-wall columns against the oracle's state stored by
    tests/golden/make_rb3d_reference.py; u relative to the whole field's max |u| (over the three
    components), T to max |T - T0|, rho absolute."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rb3d_rolls_50_oracle.json")))
    w = W.rayleigh_benard_3d(256, 256, 129, Ra=1e5, Ma=0.1, seed=3, rolls=0.5)
    assert ref["workload"] == w["name"]
    print(f"[3d] stored state {precision} steps={ref['steps']}", flush=True)
    G = gpu_lattice(w, precision)
    G.step(ref["steps"])
    rho, u, T = G.moments()
    G.close()
    s, c = ref["samples"], ref["columns"]
    zs, ys, xs = (np.array(s[k]) for k in ("z", "y", "x"))
    comps = tuple(zip(u, ("ux", "uy", "uz")))
    du = max(np.abs(a[zs, ys, xs] - s[k]).max() for a, k in comps)
    dT = np.abs(T[zs, ys, xs] - s["T"]).max()
    dr = np.abs(rho[zs, ys, xs] - s["rho"]).max()
    for i, (x, y) in enumerate(c["xy"]):
        du = max(du, max(np.abs(a[:, y, x] - np.array(c[k][i])).max() for a, k in comps))
        dT = max(dT, np.abs(T[:, y, x] - np.array(c["T"][i])).max())
        dr = max(dr, np.abs(rho[:, y, x] - np.array(c["rho"][i])).max())
    e = {"u": float(du / ref["scale"]["u"]), "T": float(dT / ref["scale"]["T"]), "rho": float(dr)}
    print(f"[3d]   {precision}: {e}", flush=True)
    assert max(e.values()) < TOL[precision], (precision, e)


@pytest.mark.gpu
def test_3d_beyond_2_31_elements_equals_its_period(gpu):
    """A periodic 512 x 512 x 256 layer (67 M nodes, 2.28e9 population elements, so element offsets
    pass 2^31) initialised with random 64^3 periodic fields (density, velocity, temperature;
    buoyancy and a body force act) tiled 8 x 8 x 4 times: after 20 steps every 64^3 block equals the
    64^3 lattice bitwise in FP64 and plain FP32, and the 64^3 lattice agrees with the oracle."""
    small = W.random_3d(64, 64, 64, seed=17)
    steps = 20
    rx, ry, rz = 8, 8, 4
    fl = small["fields"]
    tile = lambda a: np.tile(a, (rz, ry, rx))
    big = dict(small, name="random_3d_64^3_tiled", nx=64 * rx, ny=64 * ry, nz=64 * rz,
               fields={"rho": tile(fl["rho"]), "u": tuple(tile(c) for c in fl["u"]), "T": tile(fl["T"])})
    assert 34 * big["nx"] * big["ny"] * big["nz"] > 2 ** 31
    L = oracle_lattice(small)
    L.step(steps)
    ref = L.moments()
    L.close()
    for precision in ("fp64", "fp32"):
        G = gpu_lattice(small, precision)
        G.step(steps)
        ms = G.moments()
        G.close()
        e = errors3(ms, ref, small["T0"])
        print(f"[3d] random 64^3 {precision} vs oracle: {e}", flush=True)
        assert max(e.values()) < TOL[precision], e
        print(f"[3d] {big['nx']}x{big['ny']}x{big['nz']} {precision}: {steps} steps", flush=True)
        B = gpu_lattice(big, precision)
        B.step(steps)
        rho, u, T = B.moments()
        B.close()
        for a, r in zip((rho, *u, T), (ms[0], *ms[1], ms[2])):
            blocks = a.reshape(rz, 64, ry, 64, rx, 64)
            assert np.array_equal(blocks, np.broadcast_to(r[None, :, None, :, None, :], blocks.shape)), precision


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32_sr"])
def test_3d_zero_and_negative_steps(gpu, precision):
    """Zero steps leave a walled 3D lattice's state and step count bitwise unchanged; a negative
    count is refused with CLB_EINVAL and changes nothing either."""
    from paper_1710_10569_amd import clb
    w = W.random_3d(9, 7, 8, seed=5, walls=WALLS_A)
    G = gpu_lattice(w, precision)
    G.step(3)
    before = G.moments()
    G.step(0)
    with pytest.raises(clb.CLBError) as e:
        G.step(-2)
    assert e.value.code == clb.CLB_EINVAL
    after = G.moments()
    assert np.array_equal(after[0], before[0]) and np.array_equal(after[2], before[2])
    assert all(np.array_equal(a, b) for a, b in zip(after[1], before[1]))
    assert G.diagnostics()["step"] == 3
    G.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32_sr"])
def test_closed_layer_conserves_mass_at_full_size(gpu, precision):
    """Walls on z = 0 and z = nz - 1 and buoyancy: the total mass stays constant (FP64: to rounding
    of the sums; FP32 storage: to the stochastic rounding's unbiased jitter)."""
    w = W.rayleigh_benard_3d(256, 256, 129, Ra=1e5, Ma=0.1, seed=3, rolls=0.5)
    G = gpu_lattice(w, precision)
    m0 = G.diagnostics()["mass"]
    G.step(300)
    d = G.diagnostics()
    assert d["step"] == 300 and np.isfinite(d["max_speed"]) and d["max_speed"] > 0
    assert abs(d["mass"] - m0) / m0 < (1e-13 if precision == "fp64" else 1e-8), (d["mass"], m0)
    G.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32_sr", "fp32"])
def test_abc_flow_decay_rate_on_gpu(gpu, precision):
    """The ABC flow on 64^3 decays at nu k^2 (Beltrami: exact Navier-Stokes decay), to the
    discretisation error of the 64-node resolution."""
    w = W.abc_flow_3d(64, A=1e-3, tau_nu=0.8)
    G = gpu_lattice(w, precision)
    u0 = w["fields"]["u"]
    amps = []
    for _ in range(2):
        G.step(200)
        u = G.moments()[1]
        amps.append(sum((a * b).sum() for a, b in zip(u, u0)) / sum((b * b).sum() for b in u0))
    rate = -math.log(amps[1] / amps[0]) / 200
    assert abs(rate / ((0.8 - 0.5) / 3 * w["k"] ** 2) - 1) < 1e-3, rate
    G.close()


@pytest.mark.gpu
def test_diagnostics_3d_match_oracle_fields(gpu):
    w = _case_workload("walls_33x9x10")
    G = gpu_lattice(w, "fp64")
    G.step(40)
    d = G.diagnostics()
    r, u, T = _oracle_moments("walls_33x9x10", 40)
    nz = w["nz"]
    wz = np.ones(nz)
    wz[0] = wz[-1] = 0.5
    assert d["mass"] == pytest.approx(r.sum(), rel=1e-13)
    for c in range(3):
        assert d["momentum"][c] == pytest.approx((r * u[c]).sum(), rel=1e-10, abs=1e-13)
    assert d["heat"] == pytest.approx(T.sum(), rel=1e-12, abs=1e-12)
    assert d["uzT"] == pytest.approx((wz[:, None, None] * u[2] * (T - w["T0"])).sum(), rel=1e-10, abs=1e-14)
    planes = [T[z].sum() for z in (0, 1, 2, nz - 3, nz - 2, nz - 1)]
    assert np.allclose(d["plane_T"], planes, rtol=1e-12, atol=1e-12)
    assert d["max_speed"] == pytest.approx(np.sqrt(sum(c * c for c in u)).max(), rel=1e-11)
    G.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32_sr"])
def test_3d_runs_are_repeatable(gpu, precision):
    """Two runs of the same workload give bitwise the same fields (no atomics in the step; the
    stochastic rounding is keyed by node and step)."""
    w = _case_workload("walls_33x9x10")
    out = []
    for _ in range(2):
        G = gpu_lattice(w, precision)
        G.step(25)
        out.append(G.moments())
        G.close()
    (r0, u0, T0), (r1, u1, T1) = out
    assert np.array_equal(r0, r1) and np.array_equal(T0, T1) and all(np.array_equal(a, b) for a, b in zip(u0, u1))
