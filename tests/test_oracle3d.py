"""Pins of the three-dimensional oracle (D3Q27 flow, D3Q7 temperature) against what mathematics and
the two-dimensional method fix: closed forms of the equilibria, the definition of central moments,
conservation, the two-dimensional oracle on a slab one node thick, symmetry under a permutation of
the axes, exact decays of Navier-Stokes and diffusion solutions, sound attenuation at the bulk
viscosity the relaxation sets, the analytic Poiseuille and conduction states, and exact mass
conservation in a closed box.  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import o3d

EX, EY, EZ = o3d.velocities()


def psi(e, v):
    """One-dimensional factor of the D2Q9 equilibrium: psi(0, v) = 2/3 - v^2,
    psi(+-1, v) = (1/3 +- v + v^2)/2."""
    return np.where(e == 0, 2.0 / 3.0 - v * v, (1.0 / 3.0 + e * v + v * v) / 2.0)


def test_velocity_set_and_moment_order():
    """27 distinct vectors of {0, +-1}^3, the first seven the rest vector and the six axis vectors;
    27 distinct moment exponents in {0, 1, 2}^3 ordered by total order."""
    e = {(int(a), int(b), int(c)) for a, b, c in zip(EX, EY, EZ)}
    assert len(e) == 27 and e == {(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)}
    assert [abs(EX[i]) + abs(EY[i]) + abs(EZ[i]) for i in range(7)] == [0, 1, 1, 1, 1, 1, 1]
    ord_ = o3d.moment_order()
    assert len({tuple(r) for r in ord_}) == 27 and list(ord_.sum(1)) == sorted(ord_.sum(1))


def test_equilibria_closed_forms():
    """f^eq = rho psi(e_x, u_x) psi(e_y, u_y) psi(e_z, u_z) (the product of the D2Q9 factors) and
    g^eq = T (1/4 - |u|^2) at rest, T (1/4 +- u_d + u_d^2)/2 along +-e_d."""
    L = o3d.OracleLattice3D(3, 3, 3)
    rng = np.random.default_rng(11)
    for _ in range(5):
        rho, T = 1.0 + 0.1 * rng.standard_normal(), rng.standard_normal()
        u = 0.1 * rng.standard_normal(3)
        fe = L.feq(rho, *u)
        assert np.abs(fe - rho * psi(EX, u[0]) * psi(EY, u[1]) * psi(EZ, u[2])).max() < 1e-15
        ge = L.geq(T, *u)
        ref = [T * (0.25 - u @ u)] + [T * (0.25 + s * u[d] + u[d] ** 2) / 2 for d in range(3) for s in (1, -1)]
        # the D3Q7 vectors in the oracle's order: +x, -x, +y, -y, +z, -z
        assert [(EX[i], EY[i], EZ[i]) for i in range(1, 7)] == [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                                                                  (0, 0, 1), (0, 0, -1)]
        assert np.abs(ge - ref).max() < 1e-15


def test_central_moments_by_definition():
    """N(u) M f equals sum_i f_i (e_ix - u_x)^a (e_iy - u_y)^b (e_iz - u_z)^c, summed directly."""
    L = o3d.OracleLattice3D(3, 3, 3)
    rng = np.random.default_rng(12)
    f = 0.02 + 0.05 * rng.random(27)
    u = (0.07, -0.11, 0.05)
    K = np.array([[(EX[i] - u[0]) ** a * (EY[i] - u[1]) ** b * (EZ[i] - u[2]) ** c for i in range(27)]
                  for a, b, c in o3d.moment_order()])
    assert np.abs(o3d.matrix_N(*u) @ L.matrix_M() @ f - K @ f).max() < 1e-15


def test_collision_conserves_mass_momentum_and_temperature():
    """Collision keeps sum f, adds F to sum f e (the force acts over one step), keeps sum g."""
    L = o3d.OracleLattice3D(3, 3, 3)
    L.set_params(0.77, 0.9)
    L.set_relaxation(1.3, 1.1, 1.2, 1.4, 1.5, 1.1)
    rng = np.random.default_rng(13)
    f = L.feq(1.02, 0.03, -0.02, 0.01) + 1e-3 * rng.standard_normal(27)
    F = (1e-4, -2e-4, 3e-4)
    fp = L.collide27(f, F)
    assert abs(fp.sum() - f.sum()) < 1e-15
    for e, Fd in zip((EX, EY, EZ), F):
        assert abs((fp * e).sum() - (f * e).sum() - Fd) < 1e-15
    g = L.geq(0.4, 0.03, -0.02, 0.01) + 1e-3 * rng.standard_normal(7)
    assert abs(L.collide7(g, (0.03, -0.02, 0.01)).sum() - g.sum()) < 1e-15


def test_slab_reproduces_two_dimensional_oracle():
    """A 3D lattice one node thick in y, periodic, with fields independent of y and u_y = 0, carries
    the two-dimensional method exactly: summing the 3D populations over e_y gives D2Q9/D2Q5
    populations with the D2Q9 equilibrium, forcing and relaxation (the 3D bulk block couples
    k~020 into the trace, so s_b = s_nu here).  Buoyancy along -z in 3D is buoyancy along -y in 2D.
    The independently pinned 2D oracle (Table 1, the exact step, ...) thus checks the 3D transforms,
    forcing, coupling and streaming."""
    nx, nz = 12, 10
    rng = np.random.default_rng(3)
    r0 = 1 + 0.01 * rng.standard_normal((nz, nx))
    ux0, uz0 = 0.02 * rng.standard_normal((nz, nx)), 0.02 * rng.standard_normal((nz, nx))
    T0 = 0.1 * rng.standard_normal((nz, nx))
    tau_nu, tau_a, gb = 0.7, 0.85, 1e-3
    L2 = O.OracleLattice(nx, nz)
    L2.set_params(tau_nu, tau_a, gb)
    L2.set_relaxation(1 / tau_nu, 1.2, 1.3, 1.15)
    L2.set_body_force(1e-5, -2e-5)
    L2.init(r0, ux0, uz0, T0)
    L3 = o3d.OracleLattice3D(nx, 1, nz)
    L3.set_params(tau_nu, tau_a, gb)
    L3.set_relaxation(1 / tau_nu, 1.2, 1.3, 1.7, 1.9, 1.15)
    L3.set_body_force(1e-5, 0.0, -2e-5)
    L3.init(r0[:, None, :], (ux0[:, None, :], 0.0, uz0[:, None, :]), T0[:, None, :])
    L2.step(60)
    L3.step(60)
    a, b = L2.moments(), L3.moments()
    assert np.abs(a[0] - b[0][:, 0, :]).max() < 1e-13
    assert np.abs(a[1] - b[1][0][:, 0, :]).max() < 1e-14
    assert np.abs(a[2] - b[1][2][:, 0, :]).max() < 1e-14
    assert np.abs(b[1][1]).max() < 1e-15
    assert np.abs(a[3] - b[2][:, 0, :]).max() < 1e-14


def test_axis_permutation_symmetry():
    """Without buoyancy the method treats the three axes alike: a state and its cyclic relabelling
    (x, y, z) -> (y, z, x) stay relabellings of each other, with every rate set apart from 1."""
    rng = np.random.default_rng(14)
    shape = (4, 5, 6)   # (nz, ny, nx)
    r0 = 1 + 0.01 * rng.standard_normal(shape)
    u0 = [0.02 * rng.standard_normal(shape) for _ in range(3)]
    T0 = 0.1 * rng.standard_normal(shape)
    F = (1e-5, -2e-5, 3e-5)

    def run(nx, ny, nz, rho, u, T, F):
        L = o3d.OracleLattice3D(nx, ny, nz)
        L.set_params(0.66, 0.8)
        L.set_relaxation(1.4, 1.2, 1.3, 1.6, 1.7, 1.1)
        L.set_body_force(*F)
        L.init(rho, u, T)
        L.step(25)
        return L.moments()

    a = run(6, 5, 4, r0, u0, T0, F)
    # relabel: new x = old y, new y = old z, new z = old x; arrays are indexed [z][y][x]
    perm = lambda v: np.transpose(v, (2, 0, 1))   # [x_old][z_old][y_old] = [z_new][y_new][x_new]
    b = run(5, 4, 6, perm(r0), (perm(u0[1]), perm(u0[2]), perm(u0[0])), perm(T0), (F[1], F[2], F[0]))
    assert np.abs(perm(a[0]) - b[0]).max() < 1e-15
    for new, old in ((0, 1), (1, 2), (2, 0)):
        assert np.abs(perm(a[1][old]) - b[1][new]).max() < 1e-15
    assert np.abs(perm(a[2]) - b[2]).max() < 1e-15


def _abc(N, tau, steps):
    """Arnold-Beltrami-Childress flow (A = B = C) on N^3: a Beltrami field, so the nonlinear term is
    a gradient and the Navier-Stokes solution decays as exp(-nu k^2 t) exactly."""
    k = 2 * math.pi / N
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    A = 1e-3
    u0 = (A * (np.sin(k * z) + np.cos(k * y)), A * (np.sin(k * x) + np.cos(k * z)), A * (np.sin(k * y) + np.cos(k * x)))
    L = o3d.OracleLattice3D(N, N, N)
    L.set_params(tau, 1.0)
    L.init(None, u0, None)
    amps = []
    for _ in range(2):
        L.step(steps)
        u = L.moments()[1]
        amps.append(sum((a * b).sum() for a, b in zip(u, u0)) / sum((b * b).sum() for b in u0))
    rate = -math.log(amps[1] / amps[0]) / steps
    return rate / ((tau - 0.5) / 3.0 * k * k) - 1.0


def test_abc_flow_decays_at_nu_k2_second_order():
    """nu = (tau - 1/2)/3 in three dimensions: the ABC flow's decay rate approaches nu k^2 with an
    error that falls fourfold when the resolution doubles."""
    e12, e24 = _abc(12, 0.8, 40), _abc(24, 0.8, 40)
    assert abs(e12) < 5e-3 and abs(e24) < 1.5e-3
    assert 3.5 < e12 / e24 < 4.5


def test_shear_wave_decay_in_a_moving_frame():
    """A shear wave u_y = A sin(k x) decays at nu k^2 whether or not the fluid moves along x with
    U = 0.1 (Galilean invariance of the central-moment collision)."""
    N, tau = 32, 0.7
    k = 2 * math.pi / N
    rates = []
    for U in (0.0, 0.1):
        L = o3d.OracleLattice3D(N, 1, 1)
        L.set_params(tau, 1.0)
        x = np.arange(N)[None, None, :]
        L.init(None, (U, 1e-4 * np.sin(k * x), 0.0), None)
        amp = []
        for _ in range(2):
            L.step(150)
            amp.append(abs(np.fft.rfft(L.moments()[1][1][0, 0])[1]))
        rates.append(-math.log(amp[1] / amp[0]) / 150 / ((tau - 0.5) / 3 * k * k))
    assert abs(rates[0] - 1) < 2e-3
    assert abs(rates[1] - rates[0]) < 1e-4


@pytest.mark.parametrize("s_b", [1.25, 1.6, 1.0])
def test_sound_attenuation_sets_bulk_viscosity(s_b):
    """A standing sound wave's acoustic energy decays at 2 Gamma k^2 with
    Gamma = (4 nu/3 + zeta)/2 and zeta = (2/3) c_s^2 (1/s_b - 1/2): the trace of the second-order
    moments relaxes with s_b over three dimensions (the 2D block's 1/2 becomes 1/3)."""
    N, tau = 64, 0.8
    k = 2 * math.pi / N
    x = np.arange(N)
    L = o3d.OracleLattice3D(N, 1, 1)
    L.set_params(tau, 1.0)
    L.set_relaxation(s_b=s_b)
    L.init((1 + 1e-5 * np.cos(k * x))[None, None, :])

    def energy():
        r, u, _ = L.moments()
        return abs(np.fft.rfft(r[0, 0])[1]) ** 2 / 3 + abs(np.fft.rfft(u[0][0, 0])[1]) ** 2

    e0 = energy()
    L.step(333)
    e1 = energy()
    G = 0.5 * (4.0 / 3.0 * (tau - 0.5) / 3 + (2.0 / 9.0) * (1 / s_b - 0.5))
    assert abs(-math.log(e1 / e0) / (2 * 333) / (G * k * k) - 1) < 3e-3


def test_temperature_wave_decay_and_moving_frame():
    """alpha = (tau_alpha - 1/2)/4 on D3Q7: a temperature wave decays at alpha k^2, and at the same
    rate when advected by a uniform flow."""
    N, tau_a = 32, 0.7
    k = 2 * math.pi / N
    alpha = (tau_a - 0.5) / 4
    rates = []
    for U in (0.0, 0.05):
        L = o3d.OracleLattice3D(N, 2, 2)
        L.set_params(0.8, tau_a)
        L.init(None, (U, 0.0, 0.0), 0.01 * np.sin(k * np.arange(N))[None, None, :] * np.ones((2, 2, 1)))
        amp = []
        for _ in range(2):
            L.step(100)
            amp.append(abs(np.fft.rfft(L.moments()[2][0, 0])[1]))
        rates.append(-math.log(amp[1] / amp[0]) / 100 / (alpha * k * k))
    assert abs(rates[0] - 1) < 3e-3
    assert abs(rates[1] - rates[0]) < 1e-4


def test_body_force_adds_momentum_exactly():
    """Periodic box: total mass is constant and total momentum grows by F per node per step."""
    L = o3d.OracleLattice3D(4, 3, 5)
    L.set_params(0.7, 0.8)
    F = (1e-5, -3e-5, 2e-5)
    L.set_body_force(*F)
    rng = np.random.default_rng(15)
    L.init(1 + 0.01 * rng.standard_normal((5, 3, 4)))
    f, _ = L.get_state()
    m0, p0 = f.sum(), [(f * e[:, None, None, None]).sum() for e in (EX, EY, EZ)]
    L.step(30)
    f, _ = L.get_state()
    assert abs(f.sum() - m0) < 1e-12
    for d, e in enumerate((EX, EY, EZ)):
        assert abs((f * e[:, None, None, None]).sum() - p0[d] - 30 * 60 * F[d]) < 1e-13


def test_closed_box_conserves_mass():
    """Walls on z = 0 and z = nz - 1 (moving, Dirichlet and adiabatic), buoyancy: the mass balance
    of the wall density keeps the total mass to rounding."""
    L = o3d.OracleLattice3D(8, 6, 10, o3d.Wall("dirichlet", 0.01, 0.0, 0.5), o3d.Wall("adiabatic", -0.005, 0.002))
    L.set_params(0.6, 0.7, 2e-3)
    rng = np.random.default_rng(2)
    L.init(1 + 0.01 * rng.standard_normal((10, 6, 8)), None, 0.2 * rng.standard_normal((10, 6, 8)))
    m0 = L.moments()[0].sum()
    L.step(200)
    r = L.moments()[0]
    assert r.std() > 1e-4                      # the density field is not trivially uniform
    assert abs(r.sum() - m0) / m0 < 1e-13


def test_walls_impose_velocity_and_temperature():
    """Eq. 13 returns the wall velocity at wall nodes (the force correction included) and Eq. 23 the
    wall temperature (Dirichlet) or its second-order extrapolation (adiabatic), at t = 0 and later."""
    L = o3d.OracleLattice3D(6, 5, 8, o3d.Wall("dirichlet", 0.01, -0.02, 0.5), o3d.Wall("adiabatic", -0.005, 0.002))
    L.set_params(0.6, 0.7, 3e-3)
    L.set_body_force(2e-5, -1e-5, 0.0)
    rng = np.random.default_rng(4)
    L.init(None, None, 0.2 * rng.standard_normal((8, 5, 6)))
    for steps in (0, 1, 50):
        L.step(steps)
        _, u, T = L.moments()
        assert np.abs(u[0][0] - 0.01).max() < 1e-15 and np.abs(u[1][0] + 0.02).max() < 1e-15
        assert np.abs(u[0][-1] + 0.005).max() < 1e-15 and np.abs(u[1][-1] - 0.002).max() < 1e-15
        assert np.abs(u[2][0]).max() < 1e-15 and np.abs(u[2][-1]).max() < 1e-15
        assert np.abs(T[0] - 0.5).max() < 1e-15
        assert np.abs(T[-1] - (4 * T[-2] - T[-3]) / 3).max() < 1e-15


def test_poiseuille_between_walls_second_order():
    """Body force along x between resting walls: u_x(z) -> F z (H - z)/(2 nu) with an error that
    falls fourfold when H doubles."""
    errs = []
    for nz, steps in ((9, 6000), (17, 20000)):
        H, tau, F = nz - 1, 0.8, 1e-6
        L = o3d.OracleLattice3D(2, 2, nz, o3d.Wall(), o3d.Wall())
        L.set_params(tau, 1.0)
        L.set_body_force(F, 0.0, 0.0)
        L.init()
        L.step(steps)
        _, u, _ = L.moments()
        z = np.arange(nz)
        ua = F / (2 * (tau - 0.5) / 3) * z * (H - z)
        errs.append(np.abs(u[0][:, 0, 0] - ua).max() / ua.max())
        assert np.abs(u[2]).max() < 1e-15 and np.abs(u[1]).max() < 1e-15
    assert errs[0] < 0.03 and 3.9 < errs[0] / errs[1] < 4.1


def test_conduction_state_is_steady():
    """Hot bottom, cold top, below the onset of convection: rest with the linear temperature profile
    is a steady state of the scheme (buoyancy balanced by the density gradient it sets up)."""
    nz = 11
    L = o3d.OracleLattice3D(4, 4, nz, o3d.Wall("dirichlet", T=0.5), o3d.Wall("dirichlet", T=-0.5))
    L.set_params(0.8, 0.8, 1e-5)
    T0 = (0.5 - np.arange(nz) / (nz - 1))[:, None, None] * np.ones((1, 4, 4))
    L.init(None, None, T0)
    L.step(2000)
    _, u, T = L.moments()
    assert max(np.abs(c).max() for c in u) < 1e-13
    assert np.abs(T - T0).max() < 1e-13


def test_adiabatic_top_relaxes_to_uniform_temperature():
    """Dirichlet bottom at T = 0.3, adiabatic top, no buoyancy: heat flows until T = 0.3 everywhere
    (zero flux through the adiabatic wall)."""
    nz = 7
    L = o3d.OracleLattice3D(2, 2, nz, o3d.Wall("dirichlet", T=0.3), o3d.Wall("adiabatic"))
    L.set_params(0.8, 1.5)
    L.init(None, None, 0.0)
    L.step(3000)
    T = L.moments()[2]
    assert np.abs(T - 0.3).max() < 1e-8
