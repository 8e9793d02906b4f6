"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle on the same seeded
inputs.  FP64 (plain and deviation storage) must agree to 1e-12 relative; FP32 storage with FP64
collision and stochastic rounding to 1e-5 relative in u and T; plain FP32 (FP32 collision,
round-to-nearest storage, not the accuracy-qualified mode) is held to 3e-5.  Velocity errors are
relative to max |u_ref|, temperature errors to max |T_ref - T0|, density errors to max |rho_ref|
(tests/helpers.py).  Sizes span several 64 x 4 workgroup tiles with ragged tails; the full-size
cases are the 2048 x 1024 Rayleigh-Benard cell and the 8192 x 4096 control lattice in the launch
configuration the benchmark times."""
import numpy as np
import pytest

from paper_1710_10569_amd import workloads as W
from tests.helpers import field_errors, oracle_from_workload, rel_err, worst

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5
FP32_RN_TOL = 3e-5   # plain FP32: its round-to-nearest storage bias builds up near steady states


def _clb():
    from paper_1710_10569_amd import clb
    return clb


def run_pair(w, precision, steps, chunks=1):
    clb = _clb()
    print(f"[parity] {w['name']} {precision} steps={steps}", flush=True)
    g = clb.lattice_from_workload(w, precision)
    o = oracle_from_workload(w)
    errs = []
    for _ in range(chunks):
        g.step(steps // chunks)
        o.step(steps // chunks)
        errs.append(field_errors(g.moments(), o.moments(), w["T0"], w.get("u_scale", 0.0)))
    return g, o, errs


@pytest.mark.parametrize("precision", ["fp64", "fp64_dev"])
def test_taylor_green_fp64(gpu, precision):
    """Periodic 64 x 64 Taylor-Green vortex + temperature mode, 1000 steps."""
    w = W.taylor_green(64)
    g, o, errs = run_pair(w, precision, 1000, chunks=4)
    for e in errs:
        assert worst(e) < FP64_TOL, e
    fg, gg = g.populations()
    fo, go = o.get_state()
    assert np.abs(fg - fo).max() < 1e-14 and np.abs(gg - go).max() < 1e-14


@pytest.mark.parametrize("precision", ["fp64", "fp64_dev"])
@pytest.mark.parametrize("shape", [(37, 29), (130, 9), (5, 70)])
def test_random_periodic_fp64(gpu, precision, shape):
    """Random fields with buoyancy and a body force on ragged periodic lattices."""
    w = W.random_periodic(*shape, seed=shape[0] * 7 + shape[1], T0=0.3)
    w["body_force"] = (1e-5, -3e-5)
    _, _, errs = run_pair(w, precision, 300, chunks=3)
    for e in errs:
        assert worst(e) < FP64_TOL, e


WALLS = {
    "cavity": ("dirichlet", "dirichlet", "adiabatic", "adiabatic"),
    "all_dirichlet": ("dirichlet", "dirichlet", "dirichlet", "dirichlet"),
    "all_adiabatic": ("adiabatic", "adiabatic", "adiabatic", "adiabatic"),
    "channel": ("periodic", "periodic", "dirichlet", "adiabatic"),
    "side_walls": ("adiabatic", "dirichlet", "periodic", "periodic"),
}


@pytest.mark.parametrize("precision", ["fp64", "fp64_dev"])
@pytest.mark.parametrize("walls", sorted(WALLS))
def test_walls_fp64(gpu, precision, walls):
    """Every wall kind, corners of every kind pair, moving and permeable walls, buoyancy."""
    w = W.random_walled(67, 45, seed=len(walls), kinds=WALLS[walls], wall_u=0.03, g_beta=2e-3)
    g, o, errs = run_pair(w, precision, 300, chunks=3)
    for e in errs:
        assert worst(e) < FP64_TOL, e
    fg, gg = g.populations()
    fo, go = o.get_state()
    assert np.array_equal(np.isnan(fg), np.isnan(fo)) and np.array_equal(np.isnan(gg), np.isnan(go))
    m = ~np.isnan(fo)
    assert np.abs(fg[m] - fo[m]).max() < 1e-13
    m = ~np.isnan(go)
    assert np.abs(gg[m] - go[m]).max() < 1e-13


def test_cavity_256_fp64(gpu):
    """The differentially heated cavity at its full 256 x 256 size, 2000 steps from rest (max |u|
    grows to 2.9e-3; two FP64 builds of the oracle that differ only in multiply-add contraction
    differ by 7.7e-13 of max |u| after 400 steps and by 1.9e-13 after 2000)."""
    w = W.cavity(256)
    _, _, errs = run_pair(w, "fp64", 2000, chunks=2)
    for e in errs:
        assert worst(e) < FP64_TOL, e


def _against_stored_samples(ref, moments):
    """Errors of GPU fields at a stored oracle state's sampled nodes and full columns, relative to
    the whole oracle field's max |u|, max |T - T0| and max |rho - 1| ("rho" is absolute)."""
    rho, ux, uy, T = moments
    ys, xs = np.array(ref["samples"]["y"]), np.array(ref["samples"]["x"])
    cols = ref["columns"]["x"]
    U = max(ref["scale"]["ux"], ref["scale"]["uy"])
    du = max(np.abs(ux[ys, xs] - ref["samples"]["ux"]).max(), np.abs(uy[ys, xs] - ref["samples"]["uy"]).max(),
             np.abs(ux[:, cols].T - np.array(ref["columns"]["ux"])).max(),
             np.abs(uy[:, cols].T - np.array(ref["columns"]["uy"])).max())
    dT = max(np.abs(T[ys, xs] - ref["samples"]["T"]).max(), np.abs(T[:, cols].T - np.array(ref["columns"]["T"])).max())
    dr = max(np.abs(rho[ys, xs] - ref["samples"]["rho"]).max(), np.abs(rho[:, cols].T - np.array(ref["columns"]["rho"])).max())
    return {"u": du / U, "T": dT / ref["scale"]["T"], "rho": dr, "rho_p12": dr / ref["scale"]["rho"]}


def _stored(name):
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", name)))


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_RN_TOL), ("fp32_sr", FP32_TOL)])
def test_rayleigh_benard_full_size(gpu, precision, tol):
    """2048 x 1024 Rayleigh-Benard at Ra = 1e6, Ma = 0.3 in the benchmark's launch configuration,
    started from convection rolls at half the convective velocity, 1000 steps: 1024 sampled nodes
    and two full columns against the oracle's state stored by
    tests/golden/make_rb2048_reference.py, errors relative to the whole field's max |u|,
    max |T - T0| and max |rho|."""
    clb = _clb()
    ref = _stored("rb2048_rolls_1000_oracle.json")
    w = W.rayleigh_benard(rolls=0.5)
    assert ref["workload"] == w["name"]
    print(f"[parity] {w['name']} {precision} steps={ref['steps']}", flush=True)
    g = clb.lattice_from_workload(w, precision)
    g.step(ref["steps"])
    e = _against_stored_samples(ref, g.moments())
    g.close()
    print(f"[parity]   {precision}: {e}", flush=True)
    assert e["u"] < tol and e["T"] < tol and e["rho"] < tol, e


@pytest.mark.parametrize("precision,tol,in_place", [("fp64", FP64_TOL, False), ("fp32", FP32_RN_TOL, False),
                                                    ("fp32_sr", FP32_TOL, False), ("fp32", FP32_RN_TOL, True)])
def test_rayleigh_benard_control_size(gpu, precision, tol, in_place):
    """8192 x 4096 Rayleigh-Benard (3.8 GB in FP32, far beyond the Infinity Cache: the lattice the
    benchmark takes its single-lattice roofline on) in the benchmark's launch configuration, two
    buffers in three precisions and in place in FP32, started from convection rolls, 100 steps:
    1024 sampled nodes and two full columns against the oracle's state stored by
    tests/golden/make_rb8192_reference.py."""
    clb = _clb()
    ref = _stored("rb8192_rolls_100_oracle.json")
    w = W.rayleigh_benard(nx=8192, ny=4096, rolls=0.5)
    assert ref["workload"] == w["name"]
    print(f"[parity] {w['name']} {precision} in_place={in_place} steps={ref['steps']}", flush=True)
    g = clb.lattice_from_workload(w, precision, in_place=in_place)
    g.step(ref["steps"])
    e = _against_stored_samples(ref, g.moments())
    g.close()
    print(f"[parity]   {precision} in_place={in_place}: {e}", flush=True)
    assert e["u"] < tol and e["T"] < tol and e["rho"] < tol, e


def test_lattice_beyond_2_31_elements_equals_its_period(gpu):
    """Maximum size: a periodic 16384 x 10240 lattice (168 M nodes, 2.35e9 population elements, so
    element offsets pass 2^31 and byte offsets 2^32; 37.6 GB of populations in FP64) initialised
    with the 64 x 64 Taylor-Green fields tiled 256 x 160 times.  The field has period 64, so every
    64 x 64 tile must evolve exactly as the 64 x 64 lattice does: after 50 steps each tile equals it
    bitwise in FP64 and in plain FP32 (round-to-nearest, so the rounding does not depend on the
    node; FP32 also in place), and the 64 x 64 lattice agrees with the oracle."""
    clb = _clb()
    small = W.taylor_green(64)
    rx, ry, steps = 256, 160, 50
    big = dict(small, name="taylor_green_64x64_tiled", nx=64 * rx, ny=64 * ry,
               fields={k: np.tile(v, (ry, rx)) for k, v in small["fields"].items()})
    assert 14 * big["nx"] * big["ny"] > 2 ** 31
    o = oracle_from_workload(small)
    o.step(steps)
    ref = o.moments()
    o.close()
    for precision in ("fp64", "fp32"):
        g = clb.lattice_from_workload(small, precision)
        g.step(steps)
        ms = g.moments()
        g.close()
        e = field_errors(ms, ref, small["T0"])
        print(f"[parity] taylor_green 64x64 {precision} vs oracle: {e}", flush=True)
        assert e["u"] < (FP64_TOL if precision == "fp64" else FP32_RN_TOL), e
        for in_place in ((False, True) if precision == "fp32" else (False,)):
            print(f"[parity] {big['nx']}x{big['ny']} {precision} in_place={in_place}: {steps} steps", flush=True)
            G = clb.lattice_from_workload(big, precision, in_place=in_place)
            G.step(steps)
            mb = G.moments()
            G.close()
            for a, b in zip(mb, ms):
                tiles = a.reshape(ry, 64, rx, 64)
                assert np.array_equal(tiles, np.broadcast_to(b[None, :, None, :], tiles.shape)), (precision, in_place)
            del mb


@pytest.mark.parametrize("nx,ny", [(64, 1 << 18), (1 << 20, 64), (1 << 14, 1 << 16)])
def test_lattice_at_the_size_limits_equals_its_period(gpu, nx, ny):
    """The largest lattices clb_create admits: the tallest (ny = 2^18, the initialisation and moment
    kernels' grid then holds 65536 workgroups along y), the widest (nx = 2^20) and the most nodes
    (2^30 in a 16384 x 65536 lattice: 120 GB of FP32 populations), each periodic and initialised
    with the 64 x 64 Taylor-Green fields tiled; after 20 steps in plain FP32 every 64 x 64 tile
    equals the 64 x 64 lattice bitwise."""
    clb = _clb()
    small = W.taylor_green(64)
    steps = 20
    g = clb.lattice_from_workload(small, "fp32")
    g.step(steps)
    ms = g.moments()
    g.close()
    rx, ry = nx // 64, ny // 64
    big = dict(small, name=f"taylor_green_64x64_tiled_{nx}x{ny}", nx=nx, ny=ny,
               fields={k: np.tile(v, (ry, rx)) for k, v in small["fields"].items()})
    print(f"[parity] {nx}x{ny} fp32: {steps} steps", flush=True)
    G = clb.lattice_from_workload(big, "fp32")
    del big
    G.step(steps)
    mb = G.moments()
    G.close()
    for a, b in zip(mb, ms):
        tiles = a.reshape(ry, 64, rx, 64)
        assert np.array_equal(tiles, np.broadcast_to(b[None, :, None, :], tiles.shape))


def _rest_cavity(L=48, T0=0.3):
    """A closed cavity at rest at its reference temperature, buoyancy on (Dirichlet walls at T0)."""
    w = W.cavity(L, Ra=1e5, seed=2, noise=0.0, T_hot=T0, T_cold=T0)
    return dict(w, name="rest_cavity", T0=T0, taus={"tau_nu": 0.7, "tau_alpha": 0.8, "g_beta": 1e-3},
                fields={"rho": None, "ux": None, "uy": None, "T": np.full((L, L), T0)})


def _conduction(nx=40, ny=33):
    """Pure conduction between a hot south and a cold north wall, linear T, no buoyancy."""
    w = W.rayleigh_benard(nx=nx, ny=ny, amp=0.0)
    return dict(w, name="conduction", taus={"tau_nu": 0.8, "tau_alpha": 0.7, "g_beta": 0.0})


def _check_steady(name, ms, w, precision):
    rho, ux, uy, T = ms
    T_init = w["fields"]["T"]
    dev = precision != "fp64"          # populations stored as deviations from the rest equilibrium
    assert np.all(rho == 1.0), (name, precision)
    if name == "conduction" or dev:
        # no force acts on the flow populations: they stay exactly at the rest equilibrium
        assert np.all(ux == 0.0) and np.all(uy == 0.0), (name, precision)
    else:
        assert max(np.abs(ux).max(), np.abs(uy).max()) < 1e-18, (name, precision)
    dT = np.abs(T - T_init).max()
    if name == "rest" and precision == "fp32":
        # the FP32 collision carries T0 rounded to FP32; every node holds exactly that value
        assert np.all(T == float(np.float32(w["T0"]))), (name, precision)
    elif name == "rest" and dev:
        assert dT == 0.0, (name, precision)
    elif precision in ("fp64", "fp64_dev"):
        assert dT < 1e-15, (name, precision, dT)
    else:
        # FP32 storage: within two spacings of FP32 at the largest |T - T0| (0.5), 1.2e-7
        assert dT < 2.0 ** -23, (name, precision, dT)


@pytest.mark.parametrize("precision", ["fp64", "fp64_dev", "fp32", "fp32_sr"])
def test_steady_states_stay_steady(gpu, precision):
    """Degenerate cases of the method: a closed cavity at rest at its reference temperature with
    buoyancy on, and pure conduction (linear T between Dirichlet walls, no buoyancy) stay steady
    over 1000 steps, single lattice two-buffer and in place and in one grouped batch: rho = 1 and,
    where no force acts on the flow, u = 0 exactly; T to roundoff (exactly where the storage is
    the deviation from T0 at rest)."""
    clb = _clb()
    cases = {"rest": _rest_cavity(), "conduction": _conduction()}
    for name, w in cases.items():
        for in_place in (False, True):
            g = clb.lattice_from_workload(w, precision, in_place=in_place)
            g.step(1000)
            _check_steady(name, g.moments(), w, precision)
            g.close()
    b = clb.Batch(4, precision, budget_bytes=64 << 20)
    slots = {name: b.add_workload(w) for name, w in cases.items()}
    b.step(1000, "grouped")
    for name, w in cases.items():
        _check_steady(name, b.moments(slots[name]), w, precision)
    b.close()


@pytest.mark.parametrize("precision,tol", [("fp32", FP32_RN_TOL), ("fp32_sr", FP32_TOL)])
def test_fp32_taylor_green(gpu, precision, tol):
    """Taylor-Green 64 x 64, 1000 steps: u against the decayed amplitude (max |u_ref| = 0.145 U0)."""
    w = W.taylor_green(64)
    _, _, errs = run_pair(w, precision, 1000, chunks=2)
    for e in errs:
        assert e["u"] < tol and e["T"] < tol, e


@pytest.mark.parametrize("precision,tol", [("fp32", FP32_RN_TOL), ("fp32_sr", FP32_TOL)])
def test_fp32_cavity(gpu, precision, tol):
    """FP32 deviation storage on the 256 x 256 cavity, 3000 steps, against the FP64 oracle."""
    w = W.cavity(256)
    _, _, errs = run_pair(w, precision, 3000, chunks=3)
    for e in errs:
        assert e["u"] < tol and e["T"] < tol, e


def test_diagnostics_match_oracle_fields(gpu):
    """FP64 sums, weighted Nusselt sums and wall fluxes against the same reductions of the oracle's
    moment fields (numpy, FP64)."""
    w = W.random_walled(70, 50, seed=3, kinds=WALLS["cavity"], g_beta=2e-3)
    g, o, _ = run_pair(w, "fp64", 50)
    d = g.diagnostics()
    r, ux, uy, T = o.moments()
    wx = np.ones(70); wx[[0, -1]] = 0.5
    wy = np.ones(50); wy[[0, -1]] = 0.5
    wgt = wy[:, None] * wx[None, :]
    ref = {"mass": r.sum(), "heat": T.sum(), "mom_x": (r * ux).sum(), "mom_y": (r * uy).sum(),
           "sum_w": wgt.sum(), "sum_w_ux_T": (wgt * ux * T).sum(), "sum_w_uy_T": (wgt * uy * T).sum()}
    for k, v in ref.items():
        assert d[k] == pytest.approx(v, rel=1e-12, abs=1e-14), k
    west = (wy * 0.5 * (3 * T[:, 0] - 4 * T[:, 1] + T[:, 2])).sum()
    east = (wy * 0.5 * (3 * T[:, -1] - 4 * T[:, -2] + T[:, -3])).sum()
    south = (wx * 0.5 * (3 * T[0] - 4 * T[1] + T[2])).sum()
    north = (wx * 0.5 * (3 * T[-1] - 4 * T[-2] + T[-3])).sum()
    assert np.allclose(d["wall_flux"], [west, east, south, north], rtol=1e-11, atol=1e-13)
    assert d["u_max"] == pytest.approx(np.sqrt(ux ** 2 + uy ** 2).max(), rel=1e-12)
    assert d["du_max"] == -1.0 and d["nonfinite"] == 0


def test_residual_snapshot(gpu):
    clb = _clb()
    w = W.cavity(64, Ra=1e5)
    g = clb.lattice_from_workload(w, "fp64")
    g.step(100)
    _, ux0, uy0, T0 = g.moments()
    g.diagnostics(snapshot=True)
    g.step(100)
    _, ux1, uy1, T1 = g.moments()
    d = g.diagnostics()
    assert d["du_max"] == pytest.approx(max(np.abs(ux1 - ux0).max(), np.abs(uy1 - uy0).max()), rel=1e-14)
    assert d["dT_max"] == pytest.approx(np.abs(T1 - T0).max(), rel=1e-14)
    assert d["step"] == 200


def test_deterministic(gpu):
    clb = _clb()
    outs = []
    for _ in range(2):
        g = clb.lattice_from_workload(W.random_walled(90, 70, seed=9, wall_u=0.02), "fp32")
        g.step(200)
        outs.append((g.moments(), g.diagnostics()))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(a, b)
    assert outs[0][1] == outs[1][1]


def test_divergence_is_reported(gpu):
    """An unstable run (tau_nu -> 1/2, large velocities) ends in non-finite values: diagnostics
    return CLB_EDIVERGED instead of numbers."""
    clb = _clb()
    w = W.random_periodic(64, 64, seed=1, amp_u=0.45, tau_nu=0.5000001, tau_alpha=0.5000001)
    g = clb.lattice_from_workload(w, "fp64")
    g.step(3000)
    d = g.diagnostics(raise_on_diverged=False)
    assert d["nonfinite"] == 1
    with pytest.raises(clb.CLBError) as ei:
        g.diagnostics()
    assert ei.value.code == clb.CLB_EDIVERGED


def test_host_side_errors(gpu):
    clb = _clb()
    g = clb.Lattice(16, 16, "fp32")
    for args in ((0.5, 0.8, 0.0, 0.1), (0.8, 0.4, 0.0, 0.1), (float("nan"), 0.8, 0.0, 0.0)):
        with pytest.raises(clb.CLBError) as ei:
            g.set_params(*args)
        assert ei.value.code == clb.CLB_EINVAL
    with pytest.raises(clb.CLBError):
        g.set_relaxation(2.0, 1.0, 1.0, 1.0)
    with pytest.raises(clb.CLBError):
        g.step(-1)
    with pytest.raises(clb.CLBError):
        g.init(rho=np.zeros((16, 16)))
    g.close()
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_sr"])
def test_every_tile_shape_gives_identical_results(gpu, precision):
    """Each compiled tile shape (and the XCD-ordered tile mapping) computes the same per-node
    update, so the lattice after 50 steps is bitwise identical whatever the shape; shape 0 also
    matches the oracle.  Ragged 300 x 77 walled lattice: partial tiles in x and y."""
    clb = _clb()
    w = W.random_walled(300, 77, seed=4, kinds=WALLS["cavity"], wall_u=0.02, g_beta=2e-3)
    ref = None
    for s in range(len(clb.tile_shapes())):
        print(f"[parity] shape {s} {precision}", flush=True)
        g = clb.lattice_from_workload(w, precision)
        g.tile_shape = s
        g.step(50)
        f, gg = g.populations()
        m = g.moments()
        g.close()
        if ref is None:
            ref = (f, gg, m)
            o = oracle_from_workload(w)
            o.step(50)
            e = field_errors(m, o.moments(), w["T0"], w["u_scale"])
            assert e["u"] < (FP64_TOL if precision == "fp64" else FP32_TOL), e
        else:
            assert np.array_equal(f, ref[0], equal_nan=True) and np.array_equal(gg, ref[1], equal_nan=True), s


def test_autotune_leaves_state_unchanged(gpu):
    clb = _clb()
    w = W.random_walled(200, 90, seed=8, wall_u=0.01)
    a = clb.lattice_from_workload(w, "fp32")
    b = clb.lattice_from_workload(w, "fp32")
    a.step(20)
    b.step(20)
    best, us = a.autotune(3)
    assert 0 <= best < len(clb.tile_shapes()) and us > 0 and a.tile_shape == best
    a.step(20)
    b.step(20)
    for x, y in zip(a.moments(), b.moments()):
        assert np.array_equal(x, y)
    assert a.diagnostics()["step"] == 40



def _hot_wall_nusselt(T3, dT=1.0):
    """Hot-wall (west) Nusselt number of the cavity from its columns x = 0, 1, 2: the wall's mean of
    -(H / dT) dT/dx with the second-order one-sided gradient (3 T_0 - 4 T_1 + T_2)/2, i.e. its
    trapezoidal sum over the wall nodes divided by dT (unit spacing; the wall length H cancels)."""
    T3 = np.asarray(T3)
    wy = np.ones(T3.shape[0])
    wy[[0, -1]] = 0.5
    return float((wy * 0.5 * (3 * T3[:, 0] - 4 * T3[:, 1] + T3[:, 2])).sum() / dT)


def test_cavity_256_full_run(gpu):
    """The 256 x 256 differentially heated cavity (Ra = 1e5, Pr = 0.71, Ma = 0.1) over its full
    50 000 steps, against the oracle's state stored by tests/golden/make_cavity256_reference.py
    (512 sampled nodes and the hot-wall columns): FP64 within 1e-12; FP32 storage collided in FP64
    with stochastic rounding within 1e-5 in u and T and its hot-wall Nusselt number within 1e-6
    relative.  Plain FP32 (FP32 collision, round-to-nearest storage) is held to 3e-5: near the steady
    state its rounding repeats the same error every step, and T drifts to 1.5e-5 of dT by 50 000
    steps (measured), which is why the stochastic-rounding form serves steady-state solves."""
    import json
    import os
    clb = _clb()
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cavity256_50k_oracle.json")))
    w = W.cavity(256)
    assert ref["workload"] == w["name"]
    ys, xs = np.array(ref["samples"]["y"]), np.array(ref["samples"]["x"])
    U = max(ref["scale"]["ux"], ref["scale"]["uy"], w["u_scale"])
    nu_ref = _hot_wall_nusselt(ref["hot_wall_T"])
    tol = {"fp64": FP64_TOL, "fp32_sr": FP32_TOL, "fp32": 3e-5}
    for precision in ("fp64", "fp32_sr", "fp32"):
        print(f"[parity] {w['name']} {precision} steps={ref['steps']}", flush=True)
        g = clb.lattice_from_workload(w, precision)
        g.step(ref["steps"])
        rho, ux, uy, T = g.moments()
        g.close()
        eu = max(np.abs(ux[ys, xs] - ref["samples"]["ux"]).max(), np.abs(uy[ys, xs] - ref["samples"]["uy"]).max()) / U
        eT = max(np.abs(T[ys, xs] - ref["samples"]["T"]).max(),
                 np.abs(T[:, :3] - np.array(ref["hot_wall_T"])).max()) / ref["scale"]["T"]
        er = np.abs(rho[ys, xs] - ref["samples"]["rho"]).max()
        nu = _hot_wall_nusselt(T[:, :3])
        print(f"[parity]   {precision}: u {eu:.2e} T {eT:.2e} rho {er:.2e} Nu_w {nu:.9f} "
              f"(oracle {nu_ref:.9f}, rel {abs(nu / nu_ref - 1):.2e})", flush=True)
        assert eu < tol[precision] and eT < tol[precision], (precision, eu, eT)
        if precision == "fp32_sr":
            assert abs(nu / nu_ref - 1) < 1e-6


DEGENERATE = [
    ((3, 3), ("dirichlet", "dirichlet", "dirichlet", "dirichlet")),    # one interior node, four corners
    ((4, 4), ("adiabatic", "adiabatic", "adiabatic", "adiabatic")),    # smallest adiabatic box
    ((3, 40), ("periodic", "periodic", "dirichlet", "adiabatic")),     # three periodic columns
    ((65, 4), ("dirichlet", "adiabatic", "adiabatic", "dirichlet")),   # one node in the last chunk
    ((129, 3), ("periodic", "periodic", "dirichlet", "dirichlet")),    # one interior row
    ((4, 200), ("adiabatic", "dirichlet", "periodic", "periodic")),    # tall and narrow
]


@pytest.mark.parametrize("precision", ["fp64", "fp32_sr"])
@pytest.mark.parametrize("shape,kinds", DEGENERATE)
def test_degenerate_sizes(gpu, precision, shape, kinds):
    """The smallest lattices the method allows and chunk-ragged ones, with moving walls and
    buoyancy: every node against the oracle after 200 steps; step(0) changes nothing."""
    clb = _clb()
    w = W.random_walled(*shape, seed=shape[0] * 11 + shape[1], kinds=kinds, wall_u=0.02, g_beta=2e-3)
    g, o, errs = run_pair(w, precision, 200, chunks=2)
    for e in errs:
        assert max(e["u"], e["T"]) < (FP64_TOL if precision == "fp64" else FP32_TOL), e
    before = g.moments()
    g.step(0)
    after = g.moments()
    assert all(np.array_equal(a, b) for a, b in zip(before, after))
    g.close()


def _random_case(seed):
    """A seeded random configuration: size, wall kinds (periodic pairs or Dirichlet/adiabatic walls,
    respecting the minimum sizes), moving walls, buoyancy, precision, streaming form and step count."""
    rng = np.random.default_rng(1000 + seed)
    kinds = []
    for axis in range(2):
        if rng.random() < 0.3:
            kinds += ["periodic", "periodic"]
        else:
            kinds += [str(rng.choice(["dirichlet", "adiabatic"])) for _ in range(2)]
    need = [4 if "adiabatic" in kinds[2 * a:2 * a + 2] else 3 for a in range(2)]
    nx = int(rng.integers(need[0], 200))
    ny = int(rng.integers(need[1], 150))
    precision = str(rng.choice(["fp64", "fp32_sr", "fp64_dev"]))
    walled = [kinds[0] != "periodic", kinds[2] != "periodic"]
    in_place = bool(rng.random() < 0.5) and (not walled[0] or nx >= 4) and (not walled[1] or ny >= 4)
    w = W.random_walled(nx, ny, seed=int(rng.integers(1 << 30)), kinds=tuple(kinds),
                        wall_u=float(rng.choice([0.0, 0.02])), g_beta=float(rng.choice([0.0, 2e-3])))
    return w, precision, in_place, int(rng.integers(1, 61))


@pytest.mark.parametrize("seed", range(24))
def test_random_configurations(gpu, seed):
    """24 seeded random configurations against the oracle, every node compared."""
    clb = _clb()
    w, precision, in_place, steps = _random_case(seed)
    print(f"[parity] random {seed}: {w['name']} {w['edges']['west'][0]}/{w['edges']['east'][0]}/"
          f"{w['edges']['south'][0]}/{w['edges']['north'][0]} {precision} in_place={in_place} steps={steps}", flush=True)
    g = clb.lattice_from_workload(w, precision, in_place=in_place)
    o = oracle_from_workload(w)
    g.step(steps)
    o.step(steps)
    e = field_errors(g.moments(), o.moments(), w["T0"], w["u_scale"])
    g.close()
    tol = FP32_TOL if precision == "fp32_sr" else FP64_TOL
    assert e["u"] < tol and e["T"] < tol and e["rho"] < tol, e
