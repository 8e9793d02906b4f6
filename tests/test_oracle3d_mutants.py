"""The 3D pins bind: each plausible mistake planted in a temporary copy of the 3D oracle source (a
sign, a dropped term, a wrong constant or factor, a swapped index) makes the named pin fail.  The
copies are built on the CPU in a temporary directory; the oracle itself is untouched."""
import os
import subprocess

import pytest

from oracle import o3d
from tests import test_oracle3d as P

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "clb3d_oracle.c")

# (name, original text, mutated text, pin that must fail)
MUTANTS = [
    ("binomial_sign", "v *= binom(a, p) * ipow(-u[d], a - p);", "v *= binom(a, p) * ipow(u[d], a - p);",
     P.test_central_moments_by_definition),
    ("binomial_coefficient", "return (a == 2 && p == 1) ? 2.0 : 1.0;", "return 1.0;",
     P.test_central_moments_by_definition),
    ("third_order_forcing_dropped", "if (e != d) p *= m_eq(MA[m][e]);", "if (e != d) p *= (MA[m][e] == 0 ? 1.0 : 0.0);",
     P.test_slab_reproduces_two_dimensional_oracle),
    ("trace_block_two_dimensional", "(L->s_b - L->s_nu) / 3.0;", "(L->s_b - L->s_nu) / 2.0;",
     lambda: P.test_sound_attenuation_sets_bulk_viscosity(1.6)),
    ("fourth_order_at_s3", "else if (o == 4) s = L->s4;", "else if (o == 4) s = L->s3;",
     P.test_slab_reproduces_two_dimensional_oracle),
    ("wrong_cT2", "#define CT2 (1.0 / 4.0)", "#define CT2 (1.0 / 3.0)", P.test_temperature_wave_decay_and_moving_frame),
    ("buoyancy_dropped", "F[2] = L->Fv[2] + L->g_beta * (t - L->T0);", "F[2] = L->Fv[2] + 0.0 * L->g_beta * (t - L->T0);",
     P.test_slab_reproduces_two_dimensional_oracle),
    ("u_without_half_force", "for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / r;",
     "for (int d = 0; d < 3; ++d) u[d] = j[d] / r;", P.test_slab_reproduces_two_dimensional_oracle),
    ("mass_balance_unpaired", "rho_b += unknown ? L->out[L->opp[i] * n + k] : f[i];",
     "rho_b += unknown ? L->out[i * n + k] : f[i];", P.test_closed_box_conserves_mass),
    ("wall_density_extrapolated", "double rho_b = 0.0;\n", "double rho_b = 0.0 * rf;\n    rho_b = rf;\n    if (0)\n",
     P.test_closed_box_conserves_mass),
    ("wall_force_uncorrected", "const double vb[3] = {uw[0] - 0.5 * Fb[0] / rho_b,",
     "const double vb[3] = {uw[0] - 0.0 * Fb[0] / rho_b,", P.test_walls_impose_velocity_and_temperature),
    ("adiabatic_first_order", "Tb = (4.0 * Tf - Tff) / 3.0;", "Tb = Tf;", P.test_walls_impose_velocity_and_temperature),
    ("streaming_reversed", "const int tx = (x + EX[i] + nx) % nx, ty = (y + EY[i] + ny) % ny;",
     "const int tx = (x - EX[i] + nx) % nx, ty = (y - EY[i] + ny) % ny;", P.test_axis_permutation_symmetry),
]


def build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"lib3_{name}.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(path), "-lm"],
                   check=True)
    return str(lib)


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new, pin):
    lib = build_mutant(tmp_path, name, old, new)
    prev = o3d.use_library(lib)
    try:
        with pytest.raises(AssertionError):
            pin()
    finally:
        o3d.restore_library(prev)


def test_unmutated_oracle_passes_the_same_pins():
    for pin in {m[3] for m in MUTANTS}:
        pin()
