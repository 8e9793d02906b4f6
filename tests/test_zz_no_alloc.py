"""clb_diagnostics_noalloc, the allocation-free variant of clb_diagnostics, called through the C ABI:
its record equals clb_diagnostics' bitwise on two calls in a row, the second on a smaller lattice
(the shared scratch keeps the first call's larger contents), with and without a residual
snapshot; a lattice beyond its scratch is rejected."""
import math

import pytest

from paper_1710_10569_amd import workloads as W

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        x, y = a[k], b[k]
        if isinstance(x, (list, tuple)):
            assert list(x) == list(y), k
        else:
            assert x == y or (isinstance(x, float) and math.isnan(x) and math.isnan(y)), k


def test_noalloc_diagnostics_match(gpu):
    from paper_1710_10569_amd import clb
    big = clb.lattice_from_workload(W.cavity(300, Ra=1e5, seed=3), "fp32_sr")
    small = clb.lattice_from_workload(W.random_walled(45, 37, seed=9, wall_u=0.02, g_beta=2e-3), "fp64")
    print("[no_alloc] cavity 300x300 fp32_sr, then random walled 45x37 fp64", flush=True)
    big.step(200)
    big.diagnostics(snapshot=True)
    big.step(100)
    a = big.diagnostics_noalloc()
    b = big.diagnostics(snapshot=False)
    _same(a, b)
    assert a["du_max"] > 0.0
    small.step(30)
    a = small.diagnostics_noalloc()
    b = small.diagnostics(snapshot=False)
    _same(a, b)
    # again on the big one after the small one used the scratch
    big.step(10)
    _same(big.diagnostics_noalloc(), big.diagnostics(snapshot=False))
    big.close()
    small.close()


def test_noalloc_diagnostics_reject_too_large(gpu):
    from paper_1710_10569_amd import clb
    lat = clb.Lattice(4100, 2048, "fp32", {"west": ("dirichlet", 0, 0, 0.5), "east": ("dirichlet", 0, 0, -0.5),
                                          "south": ("adiabatic", 0, 0, 0), "north": ("adiabatic", 0, 0, 0)}, 0.0)
    with pytest.raises(clb.CLBError) as e:
        lat.diagnostics_noalloc()
    assert e.value.code == clb.CLB_EINVAL and "8388608" in str(e.value)
    lat.close()
