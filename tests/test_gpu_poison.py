"""The debug build libclb_poison.so loads every population whose streaming source lies beyond a
wall as NaN (two-buffer pull, in-place loads, temperature-only loads).  The wall step must
reconstruct all of them without reading one, so every configuration below must still match the
oracle -- a closure that read an unknown population would turn its node's results into NaN.  The
variant is a separate library, loaded beside the product one through the same binding."""
import importlib.util
import os

import numpy as np
import pytest

from paper_1710_10569_amd import workloads as W
from tests.helpers import field_errors, oracle_from_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pclb(gpu):
    from paper_1710_10569_amd import build as B
    assert os.path.exists(B.LIB_POISON), "libclb_poison.so is not built (python -m paper_1710_10569_amd.build --poison)"
    old = os.environ.get("CLB_LIBRARY")
    os.environ["CLB_LIBRARY"] = B.LIB_POISON
    try:
        spec = importlib.util.spec_from_file_location("clb_poison", os.path.join(os.path.dirname(B.__file__), "clb.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
    finally:
        if old is None:
            del os.environ["CLB_LIBRARY"]
        else:
            os.environ["CLB_LIBRARY"] = old
    assert mod.LIBPATH == B.LIB_POISON
    return mod


CASES = [
    ((37, 29), ("dirichlet", "adiabatic", "adiabatic", "dirichlet")),
    ((64, 21), ("adiabatic", "adiabatic", "dirichlet", "dirichlet")),
    ((19, 70), ("periodic", "periodic", "adiabatic", "dirichlet")),
    ((70, 19), ("dirichlet", "dirichlet", "periodic", "periodic")),
    ((3, 3), ("dirichlet", "dirichlet", "dirichlet", "dirichlet")),
    ((4, 4), ("adiabatic", "adiabatic", "adiabatic", "adiabatic")),
    ((65, 4), ("dirichlet", "adiabatic", "adiabatic", "dirichlet")),
]


# in-place streaming needs at least 4 nodes across a walled direction
PARAMS = [(shape, kinds, precision, in_place) for shape, kinds in CASES for precision in ("fp64", "fp32_sr")
          for in_place in (False, True) if not (in_place and min(shape) < 4)]


@pytest.mark.parametrize("shape,kinds,precision,in_place", PARAMS)
def test_unknown_populations_are_never_read(pclb, shape, kinds, precision, in_place):
    w = W.random_walled(*shape, seed=shape[0] * 13 + shape[1], kinds=kinds, wall_u=0.02, g_beta=2e-3)
    print(f"[poison] {w['name']} {kinds} {precision} in_place={in_place}", flush=True)
    from paper_1710_10569_amd import clb
    g = pclb.lattice_from_workload(w, precision, in_place=in_place)
    p = clb.lattice_from_workload(w, precision, in_place=in_place)
    o = oracle_from_workload(w)
    for n in (1, 30):
        g.step(n)
        p.step(n)
        o.step(n)
        m = g.moments()
        assert all(np.isfinite(a).all() for a in m)
        # the product library computes bitwise the same: no unknown value reaches a result
        assert all(np.array_equal(a, b) for a, b in zip(m, p.moments()))
        e = field_errors(m, o.moments(), w["T0"], w["u_scale"])
        assert max(e["u"], e["T"]) < (1e-12 if precision == "fp64" else 1e-5), e
    g.close()
    p.close()


@pytest.mark.parametrize("shape,kinds", [((37, 29), ("dirichlet", "adiabatic", "adiabatic", "dirichlet")),
                                         ((19, 70), ("periodic", "periodic", "adiabatic", "dirichlet"))])
def test_temperature_only_lattices(pclb, shape, kinds):
    w = W.prescribed_walled(*shape, seed=shape[0] + 3 * shape[1], kinds=kinds)
    g = pclb.lattice_from_workload(w, "fp64")
    o = oracle_from_workload(w)
    g.step(50)
    o.step(50)
    m = g.moments()
    assert all(np.isfinite(a).all() for a in m)
    assert field_errors(m, o.moments(), w["T0"], w["u_scale"])["T"] < 1e-12
    g.close()


def test_batch_with_poisoned_loads(pclb):
    """Grouped and persistent batch schedules (two-buffer and in-place lattices) under the poisoned
    loads: every lattice stays finite and equal to the product library's result."""
    from paper_1710_10569_amd import clb
    ws = [W.cavity(48, Ra=1e4, seed=1), W.random_walled(70, 19, seed=3, wall_u=0.01, g_beta=2e-3),
          W.rayleigh_benard(130, 17, Ra=1e4, seed=4)]
    out = []
    for mod in (pclb, clb):
        b = mod.Batch(8, "fp32_sr", budget_bytes=64 << 20)
        slots = [b.add_workload(w, in_place=(i == 1)) for i, w in enumerate(ws)]
        b.step(21, "grouped")
        b.step(10, "persistent")
        out.append([b.moments(s) for s in slots])
        b.close()
    for a, r in zip(out[0], out[1]):
        for x, y in zip(a, r):
            assert np.isfinite(x).all() and np.array_equal(x, y)
