"""Continuous-batching server for steady-state cavity solves on one GPU.

Requests (differentially heated cavities of side L and Rayleigh number Ra) arrive over time.  A
request is admitted as soon as a batch slot and enough pool memory are free (admission by HBM
footprint, first come first served); admitted lattices stay resident and are advanced together by
the batched kernel in chunks of `chunk` steps; after every chunk each resident lattice's FP64
max-norm change of u and T over that chunk is measured on the device, and a lattice whose change
is below `tol` (converged), whose change has stopped falling (at the FP32 storage floor, or above
it without converging), that hits the step cap, or that goes non-finite is read out and its slot
and memory are released for the next request.  A request therefore overlaps on the device with whatever else
is resident, and its result does not depend on the mix: every lattice takes the same per-node
update and the same chunk-aligned stopping test alone or with others.

All arithmetic runs in libclb's kernels; this module only schedules.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import clb
from . import workloads as W


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of the run
    L: int
    Ra: float
    noise_seed: int
    admitted: float = math.nan
    finished: float = math.nan
    steps: int = 0
    status: str = "pending"   # converged | fp32_floor | stalled | capped | diverged | rejected
    du: float = math.nan
    dT: float = math.nan
    best: float = math.inf    # smallest max(du, dT) seen: the level a stopped request settled at
    nu_wall: float = math.nan
    fields: tuple = field(default=None, repr=False)

    @property
    def latency(self):
        return self.finished - self.arrival


class CavityServer:
    """Serve cavity requests through one clb.Batch.

    budget_bytes: HBM pool for resident lattices; capacity: slots; precision: storage/arithmetic
    mode (default FP32 storage, FP64 collision, stochastic rounding on store, whose steady states stay
    within ~1e-7 of the FP64 ones; plain FP32 drifts to ~1e-5); chunk: steps between residual
    checks; in_place: lattices stream in place (one population buffer: about half the pool bytes per
    request, so twice as many resident); tol: max-norm change of u and of T per chunk that counts as
    steady; step_cap: give up after this many steps; schedule: 'grouped' or 'persistent';
    keep_fields: return (rho, ux, uy, T).

    Stopping without converging: the change per chunk is noisy once FP32 storage holds the state
    (each store rounds at random, so the state jitters at the rounding level: about 1e-7 in T for
    cavities with |T| up to 1/2, whose populations are stored to FP32's 3e-8 spacing).  A request
    whose change has not fallen below 0.9 times its best value for stall_patience chunks has
    stopped approaching a fixed point: "fp32_floor" if it runs with FP32 storage and its change is
    below floor_max (converged to FP32's resolution), "stalled" otherwise while the change is below
    stall_max (stopped without converging: an unsteady or under-resolved flow); its best change is
    recorded.  FP64 runs converge to tol.  A slow but steady decay (halving in fewer than about
    6 * stall_patience chunks) keeps running."""

    def __init__(self, budget_bytes=16 << 30, capacity=1024, precision="fp32_sr", chunk=1000, tol=1e-8,
                 step_cap=5_000_000, schedule="persistent", Pr=0.71, Ma=0.1, keep_fields=False,
                 stall_patience=20, floor_max=1e-6, stall_max=1e-5, stream=None, in_place=False):
        self.batch = clb.Batch(capacity, precision, budget_bytes=budget_bytes, stream=stream)
        self.precision, self.chunk, self.tol, self.step_cap = precision, int(chunk), float(tol), int(step_cap)
        self.schedule, self.Pr, self.Ma, self.keep_fields = schedule, Pr, Ma, keep_fields
        self.stall_patience, self.floor_max, self.stall_max = int(stall_patience), float(floor_max), float(stall_max)
        self.fp32_storage = precision in ("fp32", "fp32_sr")
        self.in_place = bool(in_place)
        self.site_updates = 0

    def close(self):
        self.batch.close()

    def _workload(self, r):
        return W.cavity(r.L, Ra=r.Ra, Pr=self.Pr, Ma=self.Ma, seed=r.noise_seed)

    def run(self, requests, clock=time.perf_counter, idle_sleep=1e-3, log=None):
        """Serve `requests` (arrival times in seconds from now); returns them completed."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = deque(reqs)
        waiting = deque()
        active = {}                # slot -> (request, best residual so far, chunks without progress)
        t0 = clock()
        footprint_cache = {}
        budget = self.batch.info()["budget_bytes"]
        while pending or waiting or active:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting:
                r = waiting[0]
                fp = footprint_cache.setdefault(r.L, clb.footprint(r.L, r.L, self.precision, in_place=self.in_place))
                if fp > budget:
                    r.status, r.finished = "rejected", clock() - t0
                    waiting.popleft()
                    continue
                slot = self.batch.add_workload(self._workload(r), in_place=self.in_place)
                if slot is None:
                    break           # wait until memory or a slot frees up
                waiting.popleft()
                r.admitted = clock() - t0
                active[slot] = [r, math.inf, 0]
            if not active:
                if pending:
                    time.sleep(max(0.0, min(idle_sleep, pending[0].arrival - (clock() - t0))))
                continue
            self.batch.step(self.chunk, self.schedule)
            if self.schedule == "persistent":
                self.batch.check()
            self.site_updates += self.chunk * sum(a[0].L * a[0].L for a in active.values())
            done = []
            resid = self.batch.residuals()      # one pass over every resident lattice
            for slot, st in active.items():
                r = st[0]
                r.steps += self.chunk
                r.du, r.dT, nonfinite = resid[slot]
                res = max(r.du, r.dT)
                if not nonfinite:
                    r.best = min(r.best, res)
                if nonfinite:
                    r.status = "diverged"
                elif res < self.tol:
                    r.status = "converged"
                else:
                    if res < 0.9 * st[1]:
                        st[1], st[2] = res, 0
                    else:
                        st[2] += 1
                    if st[2] >= self.stall_patience and res < self.floor_max and self.fp32_storage:
                        r.status = "fp32_floor"    # converged to FP32 storage's resolution
                    elif st[2] >= self.stall_patience and res < self.stall_max:
                        r.status = "stalled"       # stopped approaching a fixed point
                    elif r.steps >= self.step_cap:
                        r.status = "capped"
                if r.status != "pending":
                    if r.status != "diverged":
                        d = self.batch.diagnostics(slot)
                        r.nu_wall = d["wall_flux"][0]       # hot wall, dT = 1: Nu_w
                        if self.keep_fields:
                            r.fields = self.batch.moments(slot)
                    r.finished = clock() - t0
                    done.append(slot)
            for slot in done:
                r = active.pop(slot)[0]
                self.batch.remove(slot)
                if log:
                    log(f"[serve] t={r.finished:.3f}s id={r.id} L={r.L} Ra={r.Ra:.3g} {r.status} "
                        f"steps={r.steps} latency={r.latency:.3f}s resident={len(active)}")
        self.wall = clock() - t0
        return reqs


def _latency(rs, wall):
    if not rs:
        return {"count": 0, "p50_latency_s": None, "p99_latency_s": None, "solves_per_s": 0.0}
    lat = np.array([r.latency for r in rs])
    return {"count": len(rs), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "solves_per_s": len(rs) / wall if wall > 0 else 0.0}


def summarize(reqs, wall, site_updates):
    """Counts by status (converged, fp32_floor, stalled, capped, diverged, rejected); p50/p99
    latency and solves/s over the converged requests ("converged") and over those that reached a
    steady state to the storage's resolution ("settled": converged or fp32_floor); the levels at
    which fp32_floor and stalled requests stopped; aggregate MLUPS over the whole run."""
    counts = {}
    for r in reqs:
        counts[r.status] = counts.get(r.status, 0) + 1
    out = {"requests": len(reqs), "status": counts,
           "converged": _latency([r for r in reqs if r.status == "converged"], wall),
           "settled": _latency([r for r in reqs if r.status in ("converged", "fp32_floor")], wall),
           "aggregate_MLUPS": site_updates / wall / 1e6 if wall > 0 else 0.0, "wall_s": wall}
    for st in ("fp32_floor", "stalled"):
        lv = [r.best for r in reqs if r.status == st]
        if lv:
            out[st + "_level"] = {"p50": float(np.percentile(lv, 50)), "max": float(max(lv))}
    return out


def requests_from(specs):
    return [Request(id=s["id"], arrival=s["arrival"], L=s["L"], Ra=s["Ra"], noise_seed=s["noise_seed"]) for s in specs]


def main(argv=None):
    """Serve a seeded Poisson stream of cavity requests and print one line per finished request and
    a JSON summary: python -m paper_1710_10569_amd.serving --requests 64 --lam inf"""
    import argparse
    import json
    ap = argparse.ArgumentParser(description=main.__doc__.split(":")[0])
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--lam", type=float, default=math.inf, help="arrivals per second (inf: all at t = 0)")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--L-min", type=int, default=32)
    ap.add_argument("--L-max", type=int, default=1024)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--step-cap", type=int, default=5_000_000)
    ap.add_argument("--budget-gib", type=float, default=16.0)
    ap.add_argument("--precision", default="fp32_sr", choices=clb.PRECISIONS)
    ap.add_argument("--schedule", default="grouped", choices=("grouped", "persistent"))
    ap.add_argument("--in-place", action="store_true")
    a = ap.parse_args(argv)
    specs = W.serving_requests(n=a.requests, lam=a.lam if math.isfinite(a.lam) else 1.0, seed=a.seed,
                               L_range=(a.L_min, a.L_max))
    if not math.isfinite(a.lam):
        for sp in specs:
            sp["arrival"] = 0.0
    srv = CavityServer(budget_bytes=int(a.budget_gib * (1 << 30)), capacity=1024, precision=a.precision,
                       tol=a.tol, step_cap=a.step_cap, schedule=a.schedule, in_place=a.in_place)
    out = srv.run(requests_from(specs), log=lambda m: print(m, flush=True))
    summ = summarize(out, srv.wall, srv.site_updates)
    srv.close()
    summ.update({"lambda_per_s": a.lam if math.isfinite(a.lam) else "all at t=0", "seed": a.seed,
                 "L_range": [a.L_min, a.L_max], "tol": a.tol, "step_cap": a.step_cap, "precision": a.precision})
    print(json.dumps(summ), flush=True)


if __name__ == "__main__":
    main()
