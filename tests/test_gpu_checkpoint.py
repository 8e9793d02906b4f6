"""Checkpoint / resume through the C ABI: a run stopped, saved to a host blob, restored into a fresh
lattice of the same description (as another process would) and stepped on is bitwise the run that
was not interrupted -- two-buffer and in-place 2D lattices in every precision, the residual
snapshot included, and 3D lattices; blobs of another description or truncated ones are refused."""
import numpy as np
import pytest

from paper_1710_10569_amd import workloads as W


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_sr"])
@pytest.mark.parametrize("in_place", [False, True])
def test_resume_2d_is_bitwise(gpu, precision, in_place):
    from paper_1710_10569_amd import clb
    w = W.random_walled(45, 37, seed=4, wall_u=0.02, g_beta=2e-3)
    print(f"[ckpt] 2d {precision} in_place={in_place}", flush=True)
    a = clb.lattice_from_workload(w, precision, in_place=in_place)
    a.set_relaxation(1.2, 1.1, 1.3, 1.05)
    a.step(37)
    a.diagnostics(snapshot=True)
    blob = a.checkpoint()
    a.step(25)
    ref, ref_d = a.moments(), a.diagnostics()
    b = clb.Lattice(w["nx"], w["ny"], precision, w["edges"], w["T0"], in_place=in_place)
    b.restore(blob)
    b.step(25)
    assert _same(b.moments(), ref)
    d = b.diagnostics()
    assert d["step"] == ref_d["step"] == 62
    assert d["du_max"] == ref_d["du_max"] and d["dT_max"] == ref_d["dT_max"]   # the residual snapshot came along
    a.close()
    b.close()


@pytest.mark.gpu
def test_restore_refuses_other_descriptions(gpu):
    from paper_1710_10569_amd import clb
    w = W.cavity(40, Ra=1e4)
    a = clb.lattice_from_workload(w, "fp32_sr")
    blob = a.checkpoint()
    for other in (clb.Lattice(41, 40, "fp32_sr", w["edges"], w["T0"]), clb.Lattice(40, 40, "fp64", w["edges"], w["T0"]),
                  clb.Lattice(40, 40, "fp32_sr", w["edges"], w["T0"], in_place=True)):
        with pytest.raises(clb.CLBError):
            other.restore(blob)
        other.close()
    with pytest.raises(clb.CLBError):
        a.restore(blob[:-1])
    with pytest.raises(clb.CLBError):
        a.restore(b"X" + blob[1:])
    a.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32_sr"])
def test_resume_3d_is_bitwise(gpu, precision):
    from paper_1710_10569_amd import clb3d
    w = W.random_3d(20, 9, 10, seed=5, walls=(("dirichlet", (0.01, 0.0), 0.2), ("adiabatic", (0.0, -0.01), 0.0)),
                    relaxation={"s_b": 1.2, "s3": 1.1, "s4": 1.3, "s5": 1.4, "s6": 1.5, "lambda2": 1.1})
    print(f"[ckpt] 3d {precision}", flush=True)
    a = clb3d.lattice_from_workload(w, precision)
    a.step(21)
    blob = a.checkpoint()
    a.step(14)
    ref = a.moments()
    b = clb3d.Lattice3D(w["nx"], w["ny"], w["nz"], precision, *[(z["kind"], z["u"], z["T"]) for z in w["z_walls"]], T0=w["T0"])
    b.restore(blob)
    b.step(14)
    r, u, T = b.moments()
    assert np.array_equal(r, ref[0]) and np.array_equal(T, ref[2]) and _same(u, ref[1])
    assert b.diagnostics()["step"] == 35
    with pytest.raises(clb3d.CLBError):
        clb3d.Lattice3D(w["nx"], w["ny"], w["nz"] + 1, precision, *[(z["kind"], z["u"], z["T"]) for z in w["z_walls"]],
                        T0=w["T0"]).restore(blob)
    a.close()
    b.close()
