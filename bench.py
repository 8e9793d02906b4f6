#!/usr/bin/env python3
"""Benchmark of the fused CLB collide-and-stream step on one MI355X.

Headline workload (one "step" = one pass of the whole hot path over every lattice of the batch): 512
differentially heated cavities in one pool, sides drawn from {64, 96, ..., 512} and Ra log-uniform
in [1e3, 1e6] (seed 7), Pr = 0.71, Ma = 0.1, 54 M nodes (7.7 GB of populations, far beyond the
256 MB Infinity Cache); populations stored in FP32 as deviations from the rest equilibrium,
collided in FP64 and rounded stochastically on store (the mode whose results stay within 1e-5 of
the FP64 oracle over long runs); one grouped launch per step over all cavities, tile mappings and
store form chosen by the batch autotuner beforehand.  Inputs are resident in HBM before the timed
region; the timed region is K back-to-back grouped steps on the batch's stream, bracketed by
device synchronisation and timed with HIP events on that stream.

Printed: one JSON line with the headline MLUPS (site updates per second / 1e6; a D2Q9 + D2Q5
update counts as one) and the roofline of the batch step kernel (112 algorithmic bytes per FP32
site update: 14 populations read + 14 written; 224 in FP64), and beside it: the same batch with
FP32 collision and one launch per cavity, and in place; the 2048 x 1024 Rayleigh-Benard lattice in
FP32, FP32 with stochastic rounding and FP64; their field errors against FP64 after exactly 20000
steps; an 8192 x 4096 control lattice; two serving runs of 32 cavity solves from the served size
mix (sides 32-1024: all queued at once, then Poisson arrivals at about half the capacity), with
converged, FP32-floor, stalled, capped and diverged counts; and the FP64 CPU oracle timed on a
bounded sample of the batch's cavities on all host cores and on one, and on the 64 x 64
Taylor-Green run in full.  Progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS (D2Q9+D2Q5) and % HBM roofline, FP32 vs FP64; served p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
BYTES_PER_SITE = {"fp32": 112, "fp32_sr": 112, "fp64": 224, "fp64_dev": 224}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batch_step_kernel_512cavities_fp32sr.json")
ERROR_STEPS = 20000      # the 2048 x 1024 field errors against FP64 are taken after exactly this many steps


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources that define the batch step kernel and of the build flags."""
    h = hashlib.sha256()
    for rel in ("paper_1710_10569_amd/csrc/clb_device.h", "paper_1710_10569_amd/csrc/clb_inplace.h",
                "paper_1710_10569_amd/csrc/clb_batch.hip", "paper_1710_10569_amd/build.py"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(rel.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(sites):
    """HBM bytes per batch step-kernel launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources and the same batch; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("sites") != sites:
        return None
    return t.get("bytes_per_launch")


def run_precision(clb, W, precision, steps, warmup, stream, workload, autotune=False, shape=None, in_place=False):
    lat = clb.lattice_from_workload(workload, precision, stream=stream, in_place=in_place)
    if warmup:
        lat.step(warmup)
    if in_place:
        pass                     # one in-place step kernel, no tile shapes
    elif shape is not None:
        lat.tile_shape = shape
    elif autotune:
        # times every compiled tile shape on scratch copies of the state, keeps the fastest; part
        # of warm-up, outside the timed region
        lat.autotune(20 if workload["nx"] * workload["ny"] <= 1 << 22 else 5)
    shape = lat.tile_shape
    lat.synchronize()
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = lat.time_steps(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sites = workload["nx"] * workload["ny"]
    mlups = sites * steps / (ms * 1e-3) / 1e6
    gbps = BYTES_PER_SITE[precision] * sites / (ms * 1e-3 / steps) / 1e9
    kern = "in-place kernel" if in_place else f"tile shape {shape} {clb.tile_shapes()[shape]}"
    log(f"[bench] {workload['name']} {precision}{' in-place' if in_place else ''}: {kern}, "
        f"{ms / steps * 1e3:.2f} us/step, {mlups:.0f} MLUPS, {gbps:.0f} GB/s algorithmic "
        f"(wall {wall:.3f} s for {steps} steps)")
    return lat, {"ms_total": ms, "ms_per_step": ms / steps, "wall_s": wall, "mlups": mlups, "gbps": gbps,
                 "tile_shape": list(clb.tile_shapes()[shape])}


def copy_bandwidth(torch, nbytes=2 << 30, reps=20):
    """Plain device-to-device copy (torch's elementwise copy kernel) of nbytes: GB/s counted as
    bytes read + bytes written."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def _oracle_cavity(O, W, L, Ra, seed):
    from oracle import Edge
    w = W.cavity(L, Ra=Ra, seed=seed)
    e = w["edges"]
    o = O.OracleLattice(w["nx"], w["ny"], *[Edge(*e[k]) for k in ("west", "east", "south", "north")], T0=w["T0"])
    p = w["physics"]
    o.set_params(*O.params_from_physics(p["Ra"], p["Pr"], p["Ma"], p["H"], p["dT"]))
    o.init(T=w["fields"]["T"])
    return o


def _oracle_sample(O, W, budget_s, steps=200):
    """The oracle on the batch's cavities in order, `steps` steps each, until budget_s seconds have
    passed; returns (site updates, seconds, cavities run)."""
    done, t_all, k = 0, 0.0, 0
    for L, Ra, seed in W.batch_cavity_specs():
        o = _oracle_cavity(O, W, L, Ra, seed)
        t0 = time.perf_counter()
        o.step(steps)
        t_all += time.perf_counter() - t0
        done += L * L * steps
        k += 1
        o.close()
        if t_all >= budget_s:
            break
    return done, t_all, k


def cpu_baseline(W, budget_s=15.0, budget_1t=8.0):
    """The FP64 oracle (plain C, OpenMP over rows) on the host's cores: a bounded sample of the
    headline workload (the batch's cavities in order, 200 steps each, about budget_s seconds), the
    same on one thread (about budget_1t seconds), and the 64 x 64 Taylor-Green run of 1000 steps in
    full."""
    import oracle as O
    from oracle import Edge
    cores = O.threads()
    n_all, t_all, k_all = _oracle_sample(O, W, budget_s)
    O.set_threads(1)
    n_one, t_one, k_one = _oracle_sample(O, W, budget_1t)
    O.set_threads(cores)
    w = W.taylor_green(64)
    o = O.OracleLattice(64, 64, *[Edge(*w["edges"][k]) for k in ("west", "east", "south", "north")], T0=w["T0"])
    t = w["taus"]
    o.set_params(t["tau_nu"], t["tau_alpha"], t["g_beta"])
    fl = w["fields"]
    o.init(fl["rho"], fl["ux"], fl["uy"], fl["T"])
    t0 = time.perf_counter()
    o.step(1000)
    t_tg = time.perf_counter() - t0
    log(f"[bench] cpu oracle: {n_all / t_all / 1e6:.2f} MLUPS on {cores} threads, "
        f"{n_one / t_one / 1e6:.2f} MLUPS on one; Taylor-Green 64x64 x 1000 steps in {t_tg:.2f} s")
    return {"value": n_all / t_all / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"the first {k_all} cavities of the 512-cavity batch, 200 steps each "
                      f"({n_all:.3g} site updates), FP64, {cores} threads",
            "single_thread": {"value": n_one / t_one / 1e6, "unit": "MLUPS", "cores": 1,
                              "sample": f"the first {k_one} cavities, 200 steps each ({n_one:.3g} site updates)"},
            "taylor_green_64x64_1000_steps_s": t_tg}


def run_batch(clb, W, steps, stream, precision="fp32", modes=("grouped", "each"), in_place=False, warmup=2):
    """The 512 batched cavities (sides from {64, 96, ..., 512}, Ra log-uniform in [1e3, 1e6], seed 7)
    in one pool: autotuned tile widths and store form, then the grouped schedule (one launch per step
    over all cavities) and the one-launch-per-cavity schedule, timed with HIP events on the batch's
    stream."""
    import torch
    specs = W.batch_cavity_specs()
    total = sum(L * L for L, _, _ in specs)
    budget = sum(clb.footprint(L, L, precision, in_place=in_place) for L, _, _ in specs) + (64 << 20)
    b = clb.Batch(len(specs), precision, budget_bytes=budget, stream=stream)
    t0 = time.perf_counter()
    slots = []
    for L, Ra, seed in specs:
        slots.append(b.add_workload(W.cavity(L, Ra=Ra, seed=seed), in_place=in_place))
        if slots[-1] is None:
            raise RuntimeError("batch pool too small")
    log(f"[bench] batch {precision}: {len(specs)} cavities, {total:.4g} nodes, pool {budget / 1e9:.2f} GB, "
        f"set up in {time.perf_counter() - t0:.1f} s")
    b.step(20)
    b.autotune(10)
    torch.cuda.synchronize()
    widths = {}
    for slot, (L, _, _) in zip(slots, specs):
        widths.setdefault(str(b.tile_width(slot)), []).append(L)
    out = {"precision": precision, "in_place": in_place, "cavities": len(specs), "sites": total, "steps": steps,
           "pool_GB": budget / 1e9, "nontemporal_stores": b.nontemporal,
           "tile_width_by_side": {w: sorted(set(Ls)) for w, Ls in sorted(widths.items())}}
    for mode in modes:
        n = steps if mode != "each" else max(10, steps // 10)
        b.step(warmup, mode)
        torch.cuda.synchronize()
        ms = b.time_steps(n, mode)
        mlups = total * n / (ms * 1e-3) / 1e6
        gbps = BYTES_PER_SITE[precision] * total * n / (ms * 1e-3) / 1e9
        out[mode] = {"MLUPS": mlups, "ms_per_step": ms / n, "steps_timed": n, "achieved_GBps": gbps,
                     "frac": gbps / HBM_PEAK_GBPS}
        log(f"[bench] batch {precision} {mode}: {ms / n:.3f} ms/step, {mlups:.0f} MLUPS, {gbps:.0f} GB/s")
    b.close()
    return out


def run_serving(clb, W, stream, n=32, lam=0.35, L_range=(32, 1024), tol=1e-8, step_cap=5_000_000, patience=20):
    """A Poisson stream of cavity requests (lam per second; lam = inf: all queued at time 0) served
    with continuous batching (serving.py), FP32 storage with FP64 collision and stochastic rounding.
    Defaults: the served workload's size mix (L log-uniform in 32-1024, Ra log-uniform in 1e3-1e6,
    step cap 5e6) with 32 requests arriving at 0.35 per second, about half the capacity measured for
    this mix; one progress line per finished request."""
    from paper_1710_10569_amd import serving as S
    specs = W.serving_requests(n=n, lam=lam if math.isfinite(lam) else 1.0, L_range=L_range)
    if not math.isfinite(lam):
        for sp in specs:
            sp["arrival"] = 0.0
    reqs = S.requests_from(specs)
    srv = S.CavityServer(budget_bytes=8 << 30, capacity=256, chunk=1000, tol=tol, step_cap=step_cap,
                         schedule="grouped", stall_patience=patience, stream=stream)
    out = srv.run(reqs, log=log)
    summ = S.summarize(out, srv.wall, srv.site_updates)
    srv.close()
    summ.update({"lambda_per_s": lam if math.isfinite(lam) else "all at t=0", "L_range": list(L_range),
                 "Ra_range": [1e3, 1e6], "tol": tol, "step_cap": step_cap, "chunk": 1000,
                 "precision": srv.precision,
                 "stop_rules": {"converged": f"max-norm change of u and T over a chunk below {tol:g}",
                                "fp32_floor": f"change below {srv.floor_max:g} and not below 0.9 x its best "
                                              f"for {patience} chunks (FP32 storage's rounding level)",
                                "stalled": f"the same above {srv.floor_max:g} and below {srv.stall_max:g}",
                                "capped": f"{step_cap} steps"}})
    summ["frac_of_hbm_peak"] = summ["aggregate_MLUPS"] * 1e6 * BYTES_PER_SITE[srv.precision] / 1e9 / HBM_PEAK_GBPS
    log(f"[bench] serving: {summ}")
    return summ


def field_errors_vs_fp64(clb, W, stream, steps=ERROR_STEPS):
    """FP32 and FP32 with stochastic rounding against FP64 on the 2048 x 1024 lattice after exactly
    `steps` steps (the GPU FP64 path being the oracle-checked reference): max-norm errors relative
    to max |u_64| and max |T_64 - T0| (P12), and relative to the convective velocity Ma c_s."""
    w = W.rayleigh_benard()
    fields = {}
    for prec in ("fp64", "fp32", "fp32_sr"):
        lat = clb.lattice_from_workload(w, prec, stream=stream)
        lat.step(steps)
        fields[prec] = lat.moments()
        lat.close()
    _, ux, uy, T = fields["fp64"]
    umax = max(np.abs(ux).max(), np.abs(uy).max())
    out = {"after_steps": steps, "max_u_fp64": float(umax), "u_scale": w["u_scale"]}
    for prec in ("fp32", "fp32_sr"):
        _, a, b, t = fields[prec]
        du = max(np.abs(a - ux).max(), np.abs(b - uy).max())
        out[prec] = {"u": float(du / umax), "T": float(np.abs(t - T).max() / np.abs(T - w["T0"]).max()),
                     "u_vs_u_scale": float(du / w["u_scale"])}
    log(f"[bench] field errors vs fp64 after {steps} steps: {out}")
    return out


BYTES_PER_SITE_3D = {"fp32": 272, "fp32_sr": 272, "fp64": 544}   # 34 populations read + written
RB3D_SHAPE = (256, 256, 129)
TRAFFIC_FILE_3D = os.path.join(ROOT, "profiles", "traffic_step3_kernel_rb3d_256x256x129.json")


def kernel_source_hash_3d():
    """Hash of the sources that define the 3D step kernels and of the build flags."""
    h = hashlib.sha256()
    for rel in ("paper_1710_10569_amd/csrc/clb3d.hip", "paper_1710_10569_amd/csrc/clb_device.h",
                "paper_1710_10569_amd/build.py"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(rel.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic_3d(precision, sites):
    """HBM bytes per 3D step (wall-plane and interior launches) from the committed counter summary,
    if it was taken on the current kernel sources and the same layer; else None."""
    try:
        with open(TRAFFIC_FILE_3D) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash_3d() or t.get("sites") != sites:
        return None
    return t.get("precisions", {}).get(precision, {}).get("bytes_per_step")


def run_3d(W, steps=200, warmup=50, error_steps=2000, precisions=("fp32", "fp32_sr", "fp64"), stream=None):
    """The 3D path on a 256 x 256 x 129 Rayleigh-Benard layer (Ra = 1e5, started from convection
    rolls): steps per precision timed with HIP events, and the FP32 / SR fields against FP64 after
    error_steps steps."""
    from paper_1710_10569_amd import clb, clb3d
    w = W.rayleigh_benard_3d(*RB3D_SHAPE, Ra=1e5, Ma=0.1, seed=3, rolls=0.5)
    p = w["physics"]
    w = dict(w, taus=dict(zip(("tau_nu", "tau_alpha", "g_beta"), clb.params_from_physics(p["Ra"], p["Pr"], p["Ma"], p["H"], p["dT"]))))
    n = RB3D_SHAPE[0] * RB3D_SHAPE[1] * RB3D_SHAPE[2]
    out = {"workload": w["name"], "sites": n}
    for prec in precisions:
        L = clb3d.lattice_from_workload(w, prec, stream=stream)
        L.step(warmup)
        L.synchronize()
        ms = L.time_steps(steps) / steps
        L.close()
        gbps = BYTES_PER_SITE_3D[prec] * n / (ms * 1e-3) / 1e9
        out[prec] = {"MLUPS": n / (ms * 1e-3) / 1e6, "ms_per_step": ms, "steps_timed": steps, "achieved_GBps": gbps,
                     "frac": gbps / HBM_PEAK_GBPS, "bytes_per_site": BYTES_PER_SITE_3D[prec],
                     "traffic": measured_traffic_3d(prec, n),
                     "footprint_GB": clb3d.footprint(*RB3D_SHAPE, prec, walls=True) / 1e9}
        log(f"[bench] 3D {prec}: {out[prec]['MLUPS']:.0f} MLUPS, {gbps:.0f} GB/s")
    if error_steps:
        fields = {}
        for prec in ("fp64", "fp32_sr", "fp32"):
            L = clb3d.lattice_from_workload(w, prec, stream=stream)
            L.step(error_steps)
            fields[prec] = L.moments()
            L.close()
        ref = fields["fp64"]
        umax = max(float(np.abs(c).max()) for c in ref[1])
        Tdev = float(np.abs(ref[2] - w["T0"]).max())
        out["field_error_vs_fp64"] = {"steps": error_steps}
        for prec in ("fp32_sr", "fp32"):
            r, u, T = fields[prec]
            out["field_error_vs_fp64"][prec] = {
                "u": max(float(np.abs(a - b).max()) for a, b in zip(u, ref[1])) / umax,
                "T": float(np.abs(T - ref[2]).max()) / Tdev}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed steps of the headline batch")
    ap.add_argument("--warmup", type=int, default=20, help="untimed steps of the headline batch")
    ap.add_argument("--rb-steps", type=int, default=5000, help="timed steps of each 2048 x 1024 run")
    ap.add_argument("--no-fp64", action="store_true", help="skip the field errors against FP64")
    ap.add_argument("--no-control", action="store_true", help="skip the 8192x4096 control lattice")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--no-copy", action="store_true", help="skip the plain-copy bandwidth reference")
    ap.add_argument("--no-batch", action="store_true", help="skip the FP32 and in-place 512-cavity batches")
    ap.add_argument("--no-inplace", action="store_true", help="skip the in-place streaming runs")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the single-lattice tile shape instead of the library default")
    ap.add_argument("--tile-shape", type=int, default=None, help="force a single-lattice FP32 tile shape")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D Rayleigh-Benard layer")
    ap.add_argument("--3d-only", dest="only_3d", type=int, default=0, metavar="STEPS",
                    help="only time STEPS steps of the 3D layer in each precision (for profiling) and exit")
    ap.add_argument("--copy-only", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the reference kernel for "
                         "scaling hardware byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent lattices would shard by lattice, one lattice by slabs with a halo "
              "exchange; neither is implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_only:
        nbytes = args.copy_only << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}), flush=True)
        return
    from paper_1710_10569_amd import clb, workloads as W
    stream = torch.cuda.Stream()   # default priority
    if args.only_3d:
        print(json.dumps({"rayleigh_benard_3d": run_3d(W, steps=args.only_3d, warmup=2, error_steps=0,
                                                       stream=stream.cuda_stream)}), flush=True)
        return

    # headline: the 512-cavity batch, FP32 storage with stochastic rounding, grouped launches
    hb = run_batch(clb, W, args.steps, stream.cuda_stream, "fp32_sr", modes=("grouped",), warmup=args.warmup)
    torch.cuda.empty_cache()
    g = hb["grouped"]
    result = {
        "metric": METRIC,
        "value": g["MLUPS"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": g["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched_cavities_512", "cavities": 512, "sides": "64..512 by 32 (seed 7)",
                   "Ra": "log-uniform 1e3..1e6", "Pr": 0.71, "Ma": 0.1, "sites": hb["sites"],
                   "storage": "fp32 deviation from rest equilibrium, fp64 collision, stochastic rounding on store",
                   "schedule": "one grouped launch per step over all cavities", "parallelism": "single GPU"},
    }
    traffic = measured_traffic(hb["sites"])
    result["roofline"] = {"bound": "hbm", "achieved": g["achieved_GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                          "frac": g["achieved_GBps"] / HBM_PEAK_GBPS, "traffic": traffic,
                          "kernel": "batch_step_kernel<float, double, DEV=true, NT, unit rates, walls at rest>",
                          "algorithmic_bytes_per_launch": BYTES_PER_SITE["fp32_sr"] * hb["sites"],
                          "avg_launch_us": g["ms_per_step"] * 1e3,
                          "footprint_GB": hb["pool_GB"]}
    result["batched_512_cavities_fp32_sr"] = hb
    if not args.no_batch:
        result["batched_512_cavities"] = run_batch(clb, W, args.batch_steps, stream.cuda_stream, "fp32")
        torch.cuda.empty_cache()
        if not args.no_inplace:
            result["batched_512_cavities_in_place"] = run_batch(clb, W, args.batch_steps, stream.cuda_stream,
                                                                "fp32", modes=("grouped",), in_place=True)
            torch.cuda.empty_cache()

    # the 2048 x 1024 Rayleigh-Benard lattice: three precisions, and the field errors after 20000 steps
    w = W.rayleigh_benard()
    rb = {}
    for prec in ("fp32", "fp32_sr", "fp64"):
        lat, r = run_precision(clb, W, prec, args.rb_steps, 200, stream.cuda_stream, w, args.autotune,
                               args.tile_shape if prec == "fp32" else None)
        lat.close()
        rb[prec] = {"value": r["mlups"], "unit": "MLUPS", "ms_per_step": r["ms_per_step"], "steps": args.rb_steps,
                    "tile_shape": r["tile_shape"], "achieved_GBps": r["gbps"], "frac": r["gbps"] / HBM_PEAK_GBPS,
                    "bytes_per_site": BYTES_PER_SITE[prec],
                    "footprint_GB": 2 * BYTES_PER_SITE[prec] / 2 * w["nx"] * w["ny"] / 1e9}
    rb["note"] = "FP32 footprint 0.235 GB fits the 256 MB Infinity Cache: not an HBM roofline"
    result["rayleigh_benard_2048x1024"] = rb
    if not args.no_fp64:
        result["rayleigh_benard_2048x1024"]["field_error_vs_fp64"] = field_errors_vs_fp64(clb, W, stream.cuda_stream)
    torch.cuda.empty_cache()
    if not args.no_control:
        wc = W.rayleigh_benard(nx=8192, ny=4096)
        result["control_8192x4096"] = {}
        for prec in ("fp32", "fp32_sr", "fp64"):
            latc, rc = run_precision(clb, W, prec, 200, 10, stream.cuda_stream, wc,
                                     args.autotune, args.tile_shape if prec == "fp32" else None)
            latc.close()
            torch.cuda.empty_cache()
            result["control_8192x4096"][prec] = {
                "value": rc["mlups"], "unit": "MLUPS", "achieved_GBps": rc["gbps"], "tile_shape": rc["tile_shape"],
                "frac": rc["gbps"] / HBM_PEAK_GBPS,
                "footprint_GB": 2 * BYTES_PER_SITE[prec] / 2 * 8192 * 4096 / 1e9}
    if not args.no_inplace:
        # in-place streaming: one population buffer (half the footprint), same results bitwise
        result["in_place"] = {}
        for prec, wl, steps in (("fp32", w, args.rb_steps), ("fp32_sr", w, args.rb_steps), ("fp64", w, args.rb_steps),
                                ("fp32", W.rayleigh_benard(nx=8192, ny=4096), 200)):
            lati, ri = run_precision(clb, W, prec, steps, 10, stream.cuda_stream, wl, in_place=True)
            lati.close()
            torch.cuda.empty_cache()
            result["in_place"][f"{prec}_{wl['nx']}x{wl['ny']}"] = {
                "value": ri["mlups"], "unit": "MLUPS", "ms_per_step": ri["ms_per_step"], "achieved_GBps": ri["gbps"],
                "frac": ri["gbps"] / HBM_PEAK_GBPS, "footprint_GB": BYTES_PER_SITE[prec] / 2 * wl["nx"] * wl["ny"] / 1e9}
    if not args.no_3d:
        result["rayleigh_benard_3d_256x256x129"] = run_3d(W, stream=stream.cuda_stream)
        torch.cuda.empty_cache()
    if not args.no_serve:
        result["served_saturated"] = run_serving(clb, W, stream.cuda_stream, lam=math.inf)
        torch.cuda.empty_cache()
        result["served"] = run_serving(clb, W, stream.cuda_stream)
        torch.cuda.empty_cache()
    if not args.no_copy:
        cb = copy_bandwidth(torch)
        log(f"[bench] plain copy: {cb:.0f} GB/s")
        result["torch_copy_GBps"] = cb
        result["roofline"]["frac_of_torch_copy"] = g["achieved_GBps"] / cb
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
