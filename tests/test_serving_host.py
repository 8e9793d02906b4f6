"""The serving loop's scheduling on the host, with a scripted stand-in for the batch (no GPU):
admission by free slots and footprint, continuous admission as slots free up, and the stopping
rules -- converged below the tolerance, settled at the FP32 storage floor, stalled without
converging, capped, diverged, and rejected when a request could never fit the pool -- and the
summary's separate counts and latency sets."""
import math

import pytest

from paper_1710_10569_amd import serving as S


class FakeBatch:
    """Per request a scripted residual: r(steps) = a * exp(-steps / tau) + floor (nan: diverged)."""

    def __init__(self, capacity, precision, budget_bytes=0, stream=None):
        self.capacity, self.budget = capacity, budget_bytes
        self.slots = {}
        self.steps = {}
        self.log = []

    def info(self):
        return {"budget_bytes": self.budget}

    def add_workload(self, w, in_place=False):
        if len(self.slots) >= self.capacity:
            return None
        s = min(set(range(self.capacity)) - set(self.slots))
        self.slots[s] = w
        self.steps[s] = 0
        self.log.append(("add", w["req"]))
        return s

    def step(self, n, mode="grouped"):
        for s in self.slots:
            self.steps[s] += n

    def check(self):
        pass

    def residuals(self):
        out = {}
        for s, w in self.slots.items():
            a, tau, floor = w["script"]
            r = a * math.exp(-self.steps[s] / tau) + floor
            out[s] = (r, r, math.isnan(r))
        return out

    def diagnostics(self, s):
        return {"wall_flux": [1.5, 0, 0, 0]}

    def moments(self, s):
        return None

    def remove(self, s):
        self.log.append(("remove", self.slots[s]["req"]))
        del self.slots[s]

    def close(self):
        pass


@pytest.fixture
def server(monkeypatch):
    scripts = {}

    def workload(self, r):
        return {"req": r.id, "script": scripts[r.id]}

    monkeypatch.setattr(S.clb, "Batch", FakeBatch)
    monkeypatch.setattr(S.clb, "footprint", lambda nx, ny, prec, in_place=False: nx * ny * 100)
    monkeypatch.setattr(S.CavityServer, "_workload", workload)
    return scripts


def test_stopping_rules(server):
    server.update({0: (1e-3, 500.0, 0.0),        # decays below tol: converged
                   1: (1e-3, 1e9, 0.0),          # never decays: capped at the step cap
                   2: (1e-4, 300.0, 3e-7),       # levels off at 3e-7: the FP32 storage floor
                   3: (float("nan"), 1.0, 0.0),  # non-finite: diverged
                   4: (1e-3, 1e9, 2e-5),         # stalls above stall_max: runs to the cap
                   5: (1e-4, 300.0, 4e-6)})      # levels off above floor_max: stalled without converging
    reqs = [S.Request(i, 0.0, 32, 1e4, i) for i in range(6)]
    srv = S.CavityServer(budget_bytes=1 << 30, capacity=8, chunk=1000, tol=1e-8, step_cap=40000, stall_patience=5)
    out = {r.id: r for r in srv.run(reqs)}
    assert out[0].status == "converged" and out[0].steps < 40000
    assert out[1].status == "capped" and out[1].steps == 40000
    assert out[2].status == "fp32_floor" and out[2].best == pytest.approx(3e-7, rel=1e-3)
    assert out[3].status == "diverged" and out[3].steps == 1000
    assert out[4].status == "capped" and out[4].steps == 40000
    assert out[5].status == "stalled" and out[5].best == pytest.approx(4e-6, rel=1e-3)
    assert out[0].nu_wall == 1.5
    s = S.summarize(list(out.values()), srv.wall, srv.site_updates)
    assert s["status"] == {"converged": 1, "capped": 2, "fp32_floor": 1, "diverged": 1, "stalled": 1}
    assert s["converged"]["count"] == 1 and s["settled"]["count"] == 2
    assert s["converged"]["p50_latency_s"] == pytest.approx(out[0].latency)
    assert s["fp32_floor_level"]["p50"] == pytest.approx(3e-7, rel=1e-3)
    assert s["stalled_level"]["max"] == pytest.approx(4e-6, rel=1e-3)


def test_fp64_storage_has_no_fp32_floor(server):
    """With FP64 storage a request that levels off below floor_max has stalled, not converged."""
    server.update({0: (1e-4, 300.0, 3e-7)})
    srv = S.CavityServer(budget_bytes=1 << 30, capacity=2, chunk=1000, tol=1e-8, step_cap=40000, stall_patience=5,
                         precision="fp64")
    out = srv.run([S.Request(0, 0.0, 32, 1e4, 0)])
    assert out[0].status == "stalled"
    s = S.summarize(out, srv.wall, srv.site_updates)
    assert s["converged"]["count"] == 0 and s["converged"]["p50_latency_s"] is None


def test_slow_decay_is_not_a_stall(server):
    """A residual that halves only every 60 chunks (e-folding 87 chunks) keeps falling by 10 % within
    the 20-chunk patience, so it runs on to convergence instead of stopping as stalled."""
    server.update({0: (1e-6, 87_000.0, 0.0)})
    srv = S.CavityServer(budget_bytes=1 << 30, capacity=2, chunk=1000, tol=1e-8, step_cap=10 ** 6)
    out = srv.run([S.Request(0, 0.0, 32, 1e4, 0)])
    assert out[0].status == "converged" and 350_000 < out[0].steps < 450_000


def test_continuous_admission_by_slots(server):
    """Three slots, six requests: the later ones are admitted as earlier ones finish, in arrival order."""
    for i in range(6):
        server[i] = (1e-3, 300.0 * (1 + i % 3), 0.0)
    reqs = [S.Request(i, 0.0, 32, 1e4, i) for i in range(6)]
    srv = S.CavityServer(budget_bytes=1 << 30, capacity=3, chunk=1000, tol=1e-8, step_cap=10 ** 6)
    out = srv.run(reqs)
    log = srv.batch.log
    adds = [i for k, i in log if k == "add"]
    assert adds == list(range(6))
    # never more than three resident
    live = 0
    for k, _ in log:
        live += 1 if k == "add" else -1
        assert live <= 3
    assert all(r.status == "converged" for r in out)
    assert all(r.admitted >= r.arrival for r in out)


def test_request_larger_than_the_pool_is_rejected(server):
    server.update({0: (1e-3, 300.0, 0.0), 1: (1e-3, 300.0, 0.0)})
    reqs = [S.Request(0, 0.0, 32, 1e4, 0), S.Request(1, 0.0, 4096, 1e4, 1)]
    srv = S.CavityServer(budget_bytes=32 * 32 * 100 * 4, capacity=4, chunk=1000, tol=1e-8, step_cap=10 ** 5)
    out = {r.id: r for r in srv.run(reqs)}
    assert out[1].status == "rejected" and out[0].status == "converged"


def test_command_line_summary(server, capsys):
    """python -m paper_1710_10569_amd.serving: one line per finished request, then a JSON summary."""
    import json
    for i in range(5):
        server[i] = (1e-3, 300.0, 0.0)
    S.main(["--requests", "5", "--L-max", "64", "--budget-gib", "1"])
    lines = capsys.readouterr().out.strip().splitlines()
    assert sum(line.startswith("[serve]") for line in lines) == 5
    summary = json.loads(lines[-1])
    assert summary["requests"] == 5 and summary["status"] == {"converged": 5}
    assert summary["L_range"] == [32, 64] and summary["lambda_per_s"] == "all at t=0"
