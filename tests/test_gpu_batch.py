"""GPU tests of the batched path: many lattices of uneven size in one pool, advanced by the grouped
(one launch per step), per-lattice (one launch per lattice per step) and persistent (one
cooperative launch) schedules.  Each lattice's result must be bitwise the one it gets alone
through the single-lattice API, whatever the schedule and whatever else is resident."""
import numpy as np
import pytest

from paper_1710_10569_amd import workloads as W
from tests.helpers import field_errors, oracle_from_workload, worst

pytestmark = pytest.mark.gpu


def _clb():
    from paper_1710_10569_amd import clb
    return clb


def mixed_workloads():
    return [
        W.cavity(64, Ra=1e4),
        W.random_walled(100, 37, seed=1, wall_u=0.02, g_beta=2e-3),
        W.random_walled(45, 130, seed=2, kinds=("periodic", "periodic", "dirichlet", "adiabatic")),
        W.random_periodic(70, 33, seed=3, T0=0.2),
        W.cavity(96, Ra=1e5, seed=9),
        W.rayleigh_benard(300, 41, Ra=1e4, seed=5),
    ]


def alone(w, precision, steps):
    clb = _clb()
    g = clb.lattice_from_workload(w, precision)
    g.step(steps)
    m = g.moments()
    g.close()
    return m


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_sr"])
@pytest.mark.parametrize("mode", ["grouped", "each", "persistent"])
def test_batch_equals_alone(gpu, precision, mode):
    clb = _clb()
    ws = mixed_workloads()
    b = clb.Batch(16, precision, budget_bytes=256 << 20)
    slots = [b.add_workload(w) for w in ws]
    print(f"[batch] {precision} {mode} slots={slots}", flush=True)
    b.step(37, mode)
    b.step(20, mode)
    if mode == "persistent":
        b.check()
    for w, s in zip(ws, slots):
        got = b.moments(s)
        ref = alone(w, precision, 57)
        for a, r in zip(got, ref):
            assert np.array_equal(a, r), (w["name"], mode)
        assert b.diagnostics(s)["step"] == 57
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_sr"])
@pytest.mark.parametrize("width,in_place", [(0, False), (64, False), (256, False), (0, True), (64, True)])
def test_tile_width_keeps_results(gpu, precision, width, in_place):
    """Every batch tile mapping -- row tiles of width 64 or 256 and wrapped rows (0: the rows' 32-node
    runs in row-major order, shifted by one run, two per wavefront) -- covers each node once with the
    same per-node update: the lattices (two-buffer or in place; sides 45-300, most not multiples of
    32) match the single-lattice path bitwise, and so do the residuals' snapshots."""
    clb = _clb()
    ws = mixed_workloads()
    b = clb.Batch(16, precision, budget_bytes=256 << 20)
    slots = [b.add_workload(w, in_place=in_place) for w in ws]
    for s in slots:
        b.set_tile_width(s, width)
    print(f"[batch] {precision} width={width} in_place={in_place}", flush=True)
    b.step(31)
    res = b.residuals()
    b.step(26)
    for w, s in zip(ws, slots):
        for a, r in zip(b.moments(s), alone(w, precision, 57)):
            assert np.array_equal(a, r), (w["name"], width)
        assert res[s][2] == 0 and np.isfinite(res[s][0]) and res[s][0] > 0
    b.close()


def test_batch_fp64_matches_oracle(gpu):
    clb = _clb()
    ws = mixed_workloads()[:3]
    b = clb.Batch(4, "fp64", budget_bytes=64 << 20)
    slots = [b.add_workload(w) for w in ws]
    b.step(120, "persistent")
    b.check()
    for w, s in zip(ws, slots):
        o = oracle_from_workload(w)
        o.step(120)
        e = field_errors(b.moments(s), o.moments(), w["T0"], w["u_scale"])
        assert worst(e) < 1e-12, (w["name"], e)


def test_admission_by_footprint_and_slot_reuse(gpu):
    """The pool holds exactly two 128 x 128 FP32 lattices: a third is refused (CLB_ENOMEM); after a
    removal it fits.  The lattice that stayed resident is unaffected by the others coming and
    going: bitwise equal to its run alone."""
    clb = _clb()
    fp = clb.footprint(128, 128, "fp32")
    b = clb.Batch(8, "fp32", budget_bytes=2 * fp)
    w1, w2, w3 = W.cavity(128, Ra=1e5, seed=1), W.cavity(128, Ra=3e4, seed=2), W.cavity(128, Ra=1e3, seed=3)
    s1, s2 = b.add_workload(w1), b.add_workload(w2)
    assert s1 is not None and s2 is not None
    assert b.add_workload(w3) is None
    assert b.info()["used_bytes"] == 2 * fp
    b.step(50)
    b.remove(s2)
    s3 = b.add_workload(w3)
    assert s3 is not None
    b.step(50)
    got = b.moments(s1)
    ref = alone(w1, "fp32", 100)
    for a, r in zip(got, ref):
        assert np.array_equal(a, r)
    assert b.diagnostics(s3)["step"] == 50
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_sr"])
def test_walls_at_rest_form_equals_general_form(gpu, precision):
    """A batch whose lattices all have unit rates and walls at rest takes the step with u_w = 0 at
    compile time; adding one lattice with a moving wall switches the batch to the general form.  Both
    match every lattice's run alone (the general single-lattice step) bitwise."""
    clb = _clb()
    ws = [W.cavity(64, Ra=1e5, seed=4), W.cavity(97, Ra=3e4, seed=5),
          W.random_walled(70, 45, seed=6, kinds=("adiabatic", "dirichlet", "adiabatic", "dirichlet"), g_beta=2e-3),
          W.random_walled(40, 33, seed=7, kinds=("periodic", "periodic", "dirichlet", "adiabatic"))]
    for extra in (None, W.random_walled(50, 30, seed=8, wall_u=0.02)):
        b = clb.Batch(8, precision, budget_bytes=256 << 20)
        slots = [b.add_workload(w) for w in ws + ([extra] if extra else [])]
        print(f"[batch] rest walls {precision} extra={extra is not None}", flush=True)
        b.step(37)
        for w, s in zip(ws, slots):
            for a, r in zip(b.moments(s), alone(w, precision, 37)):
                assert np.array_equal(a, r), (w["name"], precision, extra is not None)
        b.close()


RATES = dict(s_b=1.2, s3=1.1, s4=0.9, lambda2=1.3)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_sr"])
@pytest.mark.parametrize("in_place", [False, True])
def test_rate_and_wall_forms_equal_general_step(gpu, precision, in_place):
    """The batch step's compile-time forms -- unit rates with walls at rest, unit rates, general rates --
    for two-buffer and in-place lattices (the in-place batch kernel takes them too): a batch of cavities
    at rest, then the same with a moving-wall lattice added, then with a lattice whose rates are away
    from 1 added.  Every lattice matches its run alone (the single-lattice step in its general form,
    with the same rates) bitwise after an odd number of steps."""
    clb = _clb()
    base = [W.cavity(64, Ra=1e5, seed=4), W.cavity(97, Ra=3e4, seed=5),
            W.random_walled(70, 45, seed=6, kinds=("adiabatic", "dirichlet", "adiabatic", "dirichlet"), g_beta=2e-3)]
    moving = W.random_walled(50, 30, seed=8, wall_u=0.02)
    rated = W.random_walled(45, 40, seed=9, kinds=("dirichlet", "adiabatic", "adiabatic", "dirichlet"), g_beta=2e-3)
    for extra in ([], [(moving, None)], [(moving, None), (rated, RATES)]):
        items = [(w, None) for w in base] + extra
        b = clb.Batch(8, precision, budget_bytes=256 << 20)
        slots = []
        for w, rates in items:
            s = b.add_workload(w, in_place=in_place)
            if rates:
                b.set_relaxation(s, **rates)
            slots.append(s)
        print(f"[batch] forms {precision} in_place={in_place} extra={len(extra)}", flush=True)
        b.step(37)
        for (w, rates), s in zip(items, slots):
            g = clb.lattice_from_workload(w, precision)
            if rates:
                g.set_relaxation(**rates)
            g.step(37)
            for a, r in zip(b.moments(s), g.moments()):
                assert np.array_equal(a, r), (w["name"], precision, in_place, len(extra))
            g.close()
        b.close()


def test_admission_refuses_buffers_of_4_gib(gpu):
    """The grouped step addresses a batch lattice's buffers with 32-bit byte offsets: a lattice whose
    population buffer needs 4 GiB or more (16384 x 16384 in FP32: 15 GB) is refused with CLB_EINVAL
    before any pool space is taken; the largest admissible shapes stay admissible by this rule."""
    clb = _clb()
    b = clb.Batch(4, "fp32", budget_bytes=64 << 20)
    with pytest.raises(clb.CLBError) as e:
        b.add(16384, 16384)
    assert e.value.code == clb.CLB_EINVAL and "4 GiB" in str(e.value)
    assert b.info()["used_bytes"] == 0
    s = b.add(64, 64)
    assert s is not None
    b.close()


@pytest.mark.parametrize("in_place", [False, True])
def test_batch_lattice_just_under_4_gib_equals_its_period(gpu, in_place):
    """The largest batch lattices: 8192 x 9344 in FP32, whose population buffer (4,286,578,688 B) is
    8.4 MB short of the 4 GiB the grouped step's 32-bit byte offsets can address, periodic and
    initialised with the 64 x 64 Taylor-Green fields tiled, batched with a small cavity, 20 grouped
    steps: every 64 x 64 tile equals the 64 x 64 lattice run alone bitwise (plain FP32), two-buffer
    and in place."""
    clb = _clb()
    small = W.taylor_green(64)
    steps = 20
    ref = alone(small, "fp32", steps)
    nx, ny = 8192, 9344
    big = dict(small, name="taylor_green_64x64_tiled_8192x9344", nx=nx, ny=ny,
               fields={k: np.tile(v, (ny // 64, nx // 64)) for k, v in small["fields"].items()})
    cav = W.cavity(64, Ra=1e5, seed=2)
    budget = clb.footprint(nx, ny, "fp32", in_place=in_place) + clb.footprint(64, 64, "fp32", in_place=in_place) + (64 << 20)
    b = clb.Batch(4, "fp32", budget_bytes=budget)
    s_big = b.add_workload(big, in_place=in_place)
    s_cav = b.add_workload(cav, in_place=in_place)
    assert s_big is not None and s_cav is not None
    del big
    print(f"[batch] {nx}x{ny} fp32 in_place={in_place}: {steps} grouped steps", flush=True)
    b.step(steps, "grouped")
    b.check()
    mb = b.moments(s_big)
    for a, r in zip(mb, ref):
        tiles = a.reshape(ny // 64, 64, nx // 64, 64)
        assert np.array_equal(tiles, np.broadcast_to(r[None, :, None, :], tiles.shape)), in_place
    for a, r in zip(b.moments(s_cav), alone(cav, "fp32", steps)):
        assert np.array_equal(a, r)
    b.close()


def test_empty_batch_and_zero_steps(gpu):
    """Empty inputs: stepping a batch with no resident lattice (before any admission and after the
    last removal) in every schedule does nothing and succeeds; zero steps leave a resident
    lattice's state and step count bitwise unchanged; a negative count is refused."""
    clb = _clb()
    b = clb.Batch(4, "fp32_sr", budget_bytes=64 << 20)
    for mode in ("grouped", "each", "persistent"):
        b.step(10, mode)
    b.check()
    assert b.residuals() == {}
    s = b.add_workload(W.cavity(48, Ra=1e4, seed=3))
    t = b.add_workload(W.cavity(40, Ra=1e5, seed=4), in_place=True)
    b.step(5)
    before = {k: b.moments(k) for k in (s, t)}
    for mode in ("grouped", "each", "persistent"):
        b.step(0, mode)
    for k in (s, t):
        for a, r in zip(b.moments(k), before[k]):
            assert np.array_equal(a, r)
        assert b.diagnostics(k)["step"] == 5
    with pytest.raises(clb.CLBError) as e:
        b.step(-1)
    assert e.value.code == clb.CLB_EINVAL
    b.remove(s)
    b.remove(t)
    for mode in ("grouped", "each", "persistent"):
        b.step(10, mode)
    b.check()
    assert b.residuals() == {} and b.info()["used_bytes"] == 0
    b.close()


def test_external_torch_pool(gpu):
    import torch
    clb = _clb()
    w = W.random_walled(80, 60, seed=7, wall_u=0.01)
    pool = torch.empty(clb.footprint(80, 60, "fp32") * 3, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    b = clb.Batch(4, "fp32", pool=pool, stream=stream.cuda_stream)
    s = b.add_workload(w)
    b.step(33)
    got = b.moments(s)
    ref = alone(w, "fp32", 33)
    for a, r in zip(got, ref):
        assert np.array_equal(a, r)
    b.close()


def test_batch_autotune_keeps_state(gpu):
    clb = _clb()
    ws = mixed_workloads()
    b1 = clb.Batch(8, "fp32", budget_bytes=128 << 20)
    b2 = clb.Batch(8, "fp32", budget_bytes=128 << 20)
    s1 = [b1.add_workload(w) for w in ws]
    s2 = [b2.add_workload(w) for w in ws]
    b1.step(11)
    b2.step(11)
    b1.autotune(3)
    b1.step(11)
    b2.step(11)
    for a, c in zip(s1, s2):
        for x, y in zip(b1.moments(a), b2.moments(c)):
            assert np.array_equal(x, y)


def test_persistent_long_run_matches_grouped(gpu):
    """A long workgroup-resident run (odd step count) equals the grouped schedule bitwise."""
    clb = _clb()
    ws = [W.cavity(64, Ra=10 ** (3 + i / 3), seed=i) for i in range(6)]
    bp = clb.Batch(8, "fp32", budget_bytes=64 << 20)
    bg = clb.Batch(8, "fp32", budget_bytes=64 << 20)
    sp = [bp.add_workload(w) for w in ws]
    sg = [bg.add_workload(w) for w in ws]
    bp.step(4101, "persistent")
    bp.check()
    bg.step(4101, "grouped")
    for a, c in zip(sp, sg):
        for x, y in zip(bp.moments(a), bg.moments(c)):
            assert np.array_equal(x, y)


def test_batch_residual_snapshot(gpu):
    """Per-slot diagnostics and the one-pass residual of all slots measure the same change of u and
    T between snapshots; the first snapshot is the initial state."""
    clb = _clb()
    b = clb.Batch(4, "fp32", budget_bytes=32 << 20)
    w = W.cavity(64, Ra=1e5)
    s = b.add_workload(w)
    s2 = b.add_workload(W.cavity(80, Ra=1e4, seed=4))
    _, uxi, uyi, Ti = b.moments(s)          # step 0 (wall nodes carry their wall-step values)
    b.step(100)
    _, ux0, uy0, T0 = b.moments(s)
    res = b.residuals()
    assert res[s][0] == pytest.approx(max(np.abs(ux0 - uxi).max(), np.abs(uy0 - uyi).max()), rel=1e-14)
    assert res[s][1] == pytest.approx(np.abs(T0 - Ti).max(), rel=1e-14)
    assert not res[s][2] and set(res) == {s, s2}
    b.step(100)
    _, ux1, uy1, T1 = b.moments(s)
    r2 = b.residuals()
    assert r2[s][0] == pytest.approx(max(np.abs(ux1 - ux0).max(), np.abs(uy1 - uy0).max()), rel=1e-14)
    assert r2[s][1] == pytest.approx(np.abs(T1 - T0).max(), rel=1e-14)
    b.diagnostics(s, snapshot=True)
    b.step(100)
    _, ux2, uy2, T2 = b.moments(s)
    d = b.diagnostics(s)
    assert d["du_max"] == pytest.approx(max(np.abs(ux2 - ux1).max(), np.abs(uy2 - uy1).max()), rel=1e-14)
    assert d["dT_max"] == pytest.approx(np.abs(T2 - T1).max(), rel=1e-14)


@pytest.mark.parametrize("in_place", [False, True])
def test_served_result_same_alone_and_in_mix(gpu, in_place):
    """Continuous batching: a request served alone and the same request served while others
    arrive, run and leave gives bitwise the same fields, stopping step and Nusselt number (with
    two-buffer and with in-place streaming, which must also agree with each other)."""
    from paper_1710_10569_amd import serving as S
    mk = lambda: [S.Request(0, 0.0, 48, 2e4, 11)]
    alone_srv = S.CavityServer(budget_bytes=64 << 20, capacity=16, chunk=500, tol=1e-6, step_cap=40000,
                               schedule="grouped", keep_fields=True, in_place=in_place)
    (a,) = alone_srv.run(mk())
    alone_srv.close()
    if in_place:
        ref_srv = S.CavityServer(budget_bytes=64 << 20, capacity=16, chunk=500, tol=1e-6, step_cap=40000,
                                 schedule="grouped", keep_fields=True)
        (r,) = ref_srv.run(mk())
        ref_srv.close()
        assert r.steps == a.steps and all(np.array_equal(x, y) for x, y in zip(r.fields, a.fields))
    mix = mk() + [S.Request(1, 0.0, 64, 1e5, 12), S.Request(2, 0.0, 40, 3e3, 13), S.Request(3, 0.05, 56, 5e4, 14),
                  S.Request(4, 0.1, 36, 1e3, 15)]
    mix_srv = S.CavityServer(budget_bytes=64 << 20, capacity=16, chunk=500, tol=1e-6, step_cap=40000,
                             schedule="persistent", keep_fields=True, in_place=in_place)
    out = mix_srv.run(mix)
    mix_srv.close()
    m = next(r for r in out if r.id == 0)
    assert a.status == m.status and a.steps == m.steps and a.nu_wall == m.nu_wall
    for x, y in zip(a.fields, m.fields):
        assert np.array_equal(x, y)
    assert all(r.status in ("converged", "fp32_floor", "capped") for r in out)


@pytest.mark.parametrize("precision", ["fp32", "fp32_sr"])
def test_persistent_with_small_and_large_lattices(gpu, precision):
    """The persistent schedule splits a mix: with at least 256 lattices of at most 64 x 64 nodes
    resident, those run workgroup-resident on a second stream while larger ones take grouped
    launches; sampled lattices of both kinds (and in-place ones) match their runs alone bitwise."""
    clb = _clb()
    rng = np.random.default_rng(17)
    small = []
    for i in range(256):
        nx, ny = int(rng.integers(16, 65)), int(rng.integers(16, 65))
        kind = i % 3
        if kind == 0:
            small.append(W.cavity(min(nx, ny), Ra=1e4, seed=i))
        elif kind == 1:
            small.append(W.random_walled(nx, ny, seed=i, wall_u=0.01, g_beta=1e-3))
        else:
            small.append(W.random_periodic(nx, ny, seed=i))
    big = [W.random_walled(200, 100, seed=2, wall_u=0.01), W.rayleigh_benard(320, 65, Ra=1e4, seed=3),
           W.cavity(130, Ra=1e5, seed=5)]
    b = clb.Batch(300, precision, budget_bytes=512 << 20)
    ss = [b.add_workload(w, in_place=(i % 5 == 4)) for i, w in enumerate(small)]
    bs = [b.add_workload(w) for w in big]
    b.step(101, "persistent")
    b.step(40, "grouped")
    b.step(7, "persistent")
    b.check()
    picked = [(small[i], ss[i]) for i in (0, 1, 2, 4, 9, 100, 201, 255)] + list(zip(big, bs))
    for w, s in picked:
        for a, r in zip(b.moments(s), alone(w, precision, 148)):
            assert np.array_equal(a, r), w["name"]
    b.close()


def _serve_against_oracle(precision, cases, step_cap):
    from paper_1710_10569_amd import serving as S
    reqs = [S.Request(i, 0.0, L, Ra, seed) for i, (L, Ra, seed) in enumerate(cases)]
    srv = S.CavityServer(budget_bytes=64 << 20, capacity=8, precision=precision, chunk=1000, tol=1e-9,
                         step_cap=step_cap, schedule="grouped", keep_fields=True, stall_patience=10 ** 9)
    out = srv.run(reqs)
    srv.close()
    errs = []
    for r in out:
        w = W.cavity(r.L, Ra=r.Ra, seed=r.noise_seed)
        o = oracle_from_workload(w)
        o.step(r.steps)
        e = field_errors(r.fields, o.moments(), w["T0"], w["u_scale"])
        print(f"[batch] served {precision} L={r.L} Ra={r.Ra:g} steps={r.steps} {r.status}: {e}", flush=True)
        errs.append(e)
    return errs


def test_served_fp32_matches_fp64_oracle(gpu):
    """Accuracy bar of the served form: FP32 deviation storage (FP64 collision, stochastic
    rounding on store), served through the batch to a near-steady state (30000 steps), against the
    FP64 oracle run for the same number of steps -- max-norm error of u (relative to the convective
    scale Ma c_s) and of T (relative to max |T - T0|) within 1e-5.  With round-to-nearest FP32
    storage the same solves drift to errors above 1e-5 (the rounding bias repeats every step near
    steady state and the slow modes integrate it); stochastic rounding must beat it tenfold."""
    cases = [(40, 2e4, 22), (48, 1e4, 24)]
    sr = _serve_against_oracle("fp32_sr", cases, 30000)
    rtn = _serve_against_oracle("fp32", cases, 30000)
    for e, e0 in zip(sr, rtn):
        assert e["u"] < 1e-5 and e["T"] < 1e-5, e
        assert max(e["u"], e["T"]) * 10 < max(e0["u"], e0["T"]), (e, e0)


def test_served_largest_sides_against_oracle(gpu):
    """The largest cavities the served mix draws (side 1024 at Ra = 1e6, the top of both ranges, and
    the mix's own largest request, side 864) batched with two small ones whose rows end in partial
    storage chunks, FP32 storage with stochastic rounding, one grouped launch per step, two-buffer
    and in place: after 200 steps every node of the large cavities against the FP64 oracle, u and
    T within 1e-5 (relative to max |u_ref| and max |T_ref - T0|)."""
    clb = _clb()
    reqs = W.serving_requests(n=32, lam=1.0, seed=5)
    big = max(reqs, key=lambda r: r["L"])
    small = sorted(reqs, key=lambda r: r["L"])[:2]
    cases = [(1024, 1e6, 31), (big["L"], big["Ra"], big["noise_seed"])] + [(r["L"], r["Ra"], r["noise_seed"]) for r in small]
    steps = 200
    ref = {}
    for L, Ra, sd in cases[:2]:
        o = oracle_from_workload(W.cavity(L, Ra=Ra, seed=sd))
        o.step(steps)
        ref[L] = o.moments()
        o.close()
    for in_place in (False, True):
        budget = sum(clb.footprint(L, L, "fp32_sr", in_place=in_place) for L, _, _ in cases) + (64 << 20)
        b = clb.Batch(len(cases), "fp32_sr", budget_bytes=budget)
        slots = [b.add_workload(W.cavity(L, Ra=Ra, seed=sd), in_place=in_place) for L, Ra, sd in cases]
        b.step(steps, "grouped")
        b.check()
        assert not any(v[2] for v in b.residuals().values())
        for (L, Ra, sd), slot in zip(cases[:2], slots):
            w = W.cavity(L, Ra=Ra, seed=sd)
            e = field_errors(b.moments(slot), ref[L], w["T0"], w["u_scale"])
            print(f"[batch] served side {L} Ra={Ra:.3g} in_place={in_place}: {e}", flush=True)
            assert e["u"] < 1e-5 and e["T"] < 1e-5, (L, in_place, e)
        b.close()


def test_full_batch_sampled_against_oracle(gpu):
    """The 512-cavity batch in the launch configuration the benchmark times (one grouped launch
    per step over all cavities, autotuned tile mappings and store form), 2000 steps, FP32 storage
    with stochastic rounding and plain FP32, and plain FP32 in place (the benchmark's in-place
    batch): a sample of cavities of sides 64 to 256 compared node by node with the oracle, u and T
    within 1e-5 (stochastic rounding) and 3e-5 (plain FP32, round-to-nearest), errors relative to
    max |u_ref| and max |T_ref - T0|; every cavity finite."""
    clb = _clb()
    specs = W.batch_cavity_specs()
    picked = []
    for L, count in ((64, 2), (96, 2), (128, 2), (192, 1), (256, 1)):
        picked += [i for i, sp in enumerate(specs) if sp[0] == L][:count]
    steps = 2000
    ref = {}
    for i in picked:
        L, Ra, sd = specs[i]
        o = oracle_from_workload(W.cavity(L, Ra=Ra, seed=sd))
        o.step(steps)
        ref[i] = o.moments()
        o.close()
    for precision, tol, in_place in (("fp32_sr", 1e-5, False), ("fp32", 3e-5, False), ("fp32", 3e-5, True)):
        budget = sum(clb.footprint(L, L, precision, in_place=in_place) for L, _, _ in specs) + (64 << 20)
        b = clb.Batch(len(specs), precision, budget_bytes=budget)
        slots = [b.add_workload(W.cavity(L, Ra=Ra, seed=sd), in_place=in_place) for L, Ra, sd in specs]
        assert all(s is not None for s in slots)
        b.autotune(2)          # leaves the state untouched
        b.step(steps, "grouped")
        b.check()
        res = b.residuals()
        assert not any(v[2] for v in res.values())
        for i in picked:
            L, Ra, sd = specs[i]
            w = W.cavity(L, Ra=Ra, seed=sd)
            e = field_errors(b.moments(slots[i]), ref[i], w["T0"], w["u_scale"])
            print(f"[batch] full batch {precision} in_place={in_place} cavity {i} L={L} Ra={Ra:.3g}: {e}", flush=True)
            assert e["u"] < tol and e["T"] < tol, (precision, in_place, i, e)
        b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_sr"])
@pytest.mark.parametrize("width", [0, 64, 256])
def test_in_place_without_column_bands(gpu, precision, width):
    """In-place lattices of more than 64^2 nodes whose width is not 1 or 2 modulo 32 keep no column
    bands in their snapshot: their x-wall edge nodes take the inner neighbours x_f and x_ff from the
    adjacent lanes of the wavefront.  Adiabatic and moving x walls (x_ff is read), an x-walled
    lattice periodic in y, widths 99, 127, 128 and the band-keeping 97 and 130 (1 and 2 modulo 32),
    wrapped rows and row tiles: every lattice matches the same lattice alone with two-buffer
    streaming bitwise after odd and even step counts, and the residuals match the two-buffer
    lattices' in the same batch.  The two-buffer lattices take the same lane exchange (at widths 97
    and 130 some east-wall nodes find a neighbour in the previous wavefront and load it instead)
    and match their runs alone bitwise too."""
    clb = _clb()
    ws = [W.random_walled(nx, 45, seed=20 + nx, kinds=("adiabatic", "adiabatic", "dirichlet", "adiabatic"),
                          wall_u=0.02, g_beta=2e-3) for nx in (99, 127, 130)]
    ws.append(W.random_walled(97, 50, seed=7, kinds=("adiabatic", "dirichlet", "adiabatic", "dirichlet"), wall_u=0.01))
    ws.append(W.random_walled(128, 40, seed=8, kinds=("dirichlet", "adiabatic", "periodic", "periodic"), wall_u=0.02))
    b = clb.Batch(16, precision, budget_bytes=256 << 20)
    ip = [b.add_workload(w, in_place=True) for w in ws]
    tb = [b.add_workload(w) for w in ws]
    for s in ip + tb:
        b.set_tile_width(s, width)
    print(f"[batch] no column bands {precision} width={width}", flush=True)
    b.step(31)
    res = b.residuals()
    for s, t in zip(ip, tb):
        assert res[s] == res[t], (s, res[s], res[t])
    b.step(26)
    for w, s, t in zip(ws, ip, tb):
        ref = alone(w, precision, 57)
        for a, c, r in zip(b.moments(s), b.moments(t), ref):
            assert np.array_equal(a, r), (w["name"], width, "in place")
            assert np.array_equal(c, r), (w["name"], width, "two buffers")
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_sr"])
@pytest.mark.parametrize("mode", ["grouped", "each", "persistent"])
def test_in_place_lattices_in_a_batch(gpu, precision, mode):
    """In-place and two-buffer lattices in one batch, admitted at different times (so their step
    counts, and with them the in-place form, differ): each matches the same lattice alone with
    two-buffer streaming bitwise, in every schedule; the in-place ones take about half the pool."""
    clb = _clb()
    ws = mixed_workloads()
    b = clb.Batch(16, precision, budget_bytes=256 << 20)
    first = [b.add_workload(w, in_place=(i % 2 == 0)) for i, w in enumerate(ws[:3])]
    b.step(13, mode)
    later = [b.add_workload(w, in_place=(i % 2 == 1)) for i, w in enumerate(ws[3:])]
    b.step(20, mode)
    b.step(24, mode)
    if mode == "persistent":
        b.check()
    res = b.residuals()
    for w, s in zip(ws[:3], first):
        for a, r in zip(b.moments(s), alone(w, precision, 57)):
            assert np.array_equal(a, r), (w["name"], mode)
    for w, s in zip(ws[3:], later):
        for a, r in zip(b.moments(s), alone(w, precision, 44)):
            assert np.array_equal(a, r), (w["name"], mode)
    assert not any(v[2] for v in res.values())
    b.close()
    two, one = clb.footprint(300, 200, precision), clb.footprint(300, 200, precision, in_place=True)
    assert one < 0.62 * two


def test_tile_width_and_store_form_read_back(gpu):
    """The per-slot tile width and the batch's store form read back as set, and as the defaults
    (wrapped rows with walls in x, else width by lattice width; ordinary stores for a small FP32
    batch)."""
    clb = _clb()
    b = clb.Batch(8, "fp32", budget_bytes=64 << 20)
    s0 = b.add_workload(W.cavity(64, Ra=1e4))
    s1 = b.add_workload(W.cavity(150, Ra=1e4))
    s2 = b.add_workload(W.rayleigh_benard(300, 17, Ra=1e4))
    # two-buffer: wrapped rows with walls in x, else by width
    assert [b.tile_width(s) for s in (s0, s1, s2)] == [0, 0, 256]
    # in-place lattices: wrapped rows with walls in x, else 64-wide rows
    ip = [b.add_workload(w, in_place=True) for w in (W.cavity(96, Ra=1e4), W.cavity(50, Ra=1e4),
                                                     W.rayleigh_benard(320, 17, Ra=1e4))]
    assert [b.tile_width(s) for s in ip] == [0, 0, 64]
    for s in ip:
        b.remove(s)
    assert b.nontemporal is False
    b.set_tile_width(s1, 128)
    b.set_nontemporal(True)
    assert b.tile_width(s1) == 128 and b.nontemporal is True
    with pytest.raises(clb.CLBError):
        b.tile_width(7)
    b.close()
