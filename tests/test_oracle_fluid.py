"""Pins of the oracle's lattice-Boltzmann part against what mathematics and textbooks fix.

Each test checks the FP64 oracle against something other than itself: lattice isotropy,
closed-form flows (shear-wave decay, Couette, Poiseuille), conservation laws and the Stokes
rotation rate of a free sphere.  CPU only.
"""
import numpy as np
import pytest


def test_lattice_isotropy(orc):
    # App. A: D3Q19 with C^q = 1/3, 1/18, 1/36 and c_s^2 = 1/3.  The weights must make the
    # lattice tensors isotropic up to fourth order; a wrong weight or velocity fails here.
    c, w, opp = orc.lattice()
    c = c.astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.allclose((w[:, None] * c).sum(0), 0, atol=1e-16)
    assert np.allclose(np.einsum("q,qa,qb->ab", w, c, c), np.eye(3) / 3, atol=1e-16)
    assert np.allclose(np.einsum("q,qa,qb,qc->abc", w, c, c, c), 0, atol=1e-16)
    d = np.eye(3)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("q,qa,qb,qc,qd->abcd", w, c, c, c, c), iso4, atol=1e-16)
    for q in range(19):
        assert np.array_equal(c[opp[q]], -c[q])


def test_equilibrium_moments(orc):
    # eq. (4): the equilibrium carries rho, rho u and Pi = rho c_s^2 I + rho u u
    # (the last up to the O(u^3) term the second-order form drops on the diagonal).
    c, w, _ = orc.lattice()
    c = c.astype(float)
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho = 1 + 0.1 * rng.random()
        u = 0.05 * (rng.random(3) - 0.5)
        f = orc.feq(rho, u)
        assert abs(f.sum() - rho) < 1e-14
        assert np.allclose(f @ c, rho * u, atol=1e-15)
        Pi = np.einsum("q,qa,qb->ab", f, c, c)
        ref = rho / 3 * np.eye(3) + rho * np.outer(u, u)
        off = ~np.eye(3, dtype=bool)
        assert np.allclose(Pi[off], ref[off], atol=1e-15)
        assert np.allclose(np.diag(Pi), np.diag(ref), atol=5 * np.abs(u).max() ** 3)


def _shear_wave_nu(orc, L, tau, T, **kw):
    p = orc.make_params(lx=2, ly=L, lz=2, tau=tau, **kw)
    o = orc.Oracle(p)
    f = o.f
    U0 = 1e-5
    for y in range(L):
        f[:, :, y, :] = orc.feq(1.0, [U0 * np.sin(2 * np.pi * y / L), 0, 0])[:, None, None]
    o.step(T // 10)
    _, u = o.moments()
    sy = np.sin(2 * np.pi * np.arange(L) / L)
    a0 = (u[0, 0, :, 0] * sy).sum() * 2 / L
    o.step(T - T // 10)
    _, u = o.moments()
    a1 = (u[0, 0, :, 0] * sy).sum() * 2 / L
    k = 2 * np.pi / L
    return -np.log(a1 / a0) / (k * k * (T - T // 10))


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_shear_wave_viscosity(orc, tau):
    # BGK viscosity nu = (tau - 1/2)/3: a shear wave decays as exp(-nu k^2 t) up to the
    # O(k^2) lattice dispersion, which must fall ~4x when the wavelength doubles.
    nu = (tau - 0.5) / 3
    e32 = abs(_shear_wave_nu(orc, 32, tau, 600) / nu - 1)
    e64 = abs(_shear_wave_nu(orc, 64, tau, 2400) / nu - 1)
    assert e32 < 5e-3
    assert e64 < 0.35 * e32 + 1e-5


def test_mass_momentum_conservation_periodic(orc):
    # Collision conserves mass and momentum; periodic streaming moves them.
    p = orc.make_params(lx=8, ly=8, lz=8, tau=0.7)
    o = orc.Oracle(p)
    rng = np.random.default_rng(5)
    f = o.f
    f *= 1 + 0.01 * (rng.random(f.shape) - 0.5)
    c, _, _ = orc.lattice()
    m0 = f.sum()
    j0 = np.tensordot(c.T.astype(float), f, axes=([1], [0])).reshape(3, -1).sum(1)
    o.step(200)
    f = o.f
    j1 = np.tensordot(c.T.astype(float), f, axes=([1], [0])).reshape(3, -1).sum(1)
    assert abs(f.sum() / m0 - 1) < 1e-13
    assert np.abs(j1 - j0).max() < 1e-13 * m0


def test_lees_edwards_couette(orc):
    # Linear Couette flow is a steady solution across the Lees-Edwards plane: the
    # interpolation is exact for x-uniform fields, so the profile stays linear and the
    # fluid shear stress equals eta0 * gdot from the first step.
    gd = 1e-3
    p = orc.make_params(lx=8, ly=32, lz=2, tau=1.0, shear_kind=1, gamma_dot=gd)
    o = orc.Oracle(p)
    m0 = o.f.sum()
    o.step(400)
    _, u = o.moments()
    lin = gd * (np.arange(32) - 15.5)
    assert np.abs(u[0] - lin[None, :, None]).max() < 1e-12
    sig, _ = o.stress()
    eta0 = (1.0 - 0.5) / 3
    assert abs(sig[0][3] / (eta0 * gd) - 1) < 1e-10
    assert abs(o.f.sum() / m0 - 1) < 1e-12


def test_lees_edwards_mass_nonuniform(orc):
    # The Galilean correction and linear interpolation conserve mass exactly for any field.
    p = orc.make_params(lx=12, ly=16, lz=4, tau=0.9, shear_kind=1, gamma_dot=3.7e-3)
    o = orc.Oracle(p)
    rng = np.random.default_rng(9)
    f = o.f
    f *= 1 + 0.02 * (rng.random(f.shape) - 0.5)
    m0 = f.sum()
    o.step(150)
    assert abs(o.f.sum() / m0 - 1) < 1e-12


def test_moving_wall_couette(orc):
    # eq. (7) with static rows as walls: halfway bounce-back with a moving wall has the
    # exact steady solution u(y) = U_bot + (U_top - U_bot)(y - 1/2)/H, H = ly - 2.
    ly = 12
    ub, ut = -2e-3, 5e-3
    p = orc.make_params(lx=2, ly=ly, lz=2, tau=1.0, wall_y=1, wall_u_bot=ub, wall_u_top=ut)
    o = orc.Oracle(p)
    o.step(6000)
    _, u = o.moments()
    H = ly - 2
    y = np.arange(1, ly - 1)
    ref = ub + (ut - ub) * (y - 0.5) / H
    assert np.abs(u[0, 0, 1:-1, 0] - ref).max() < 1e-10


def _poiseuille_err(orc, H, tau=1.0):
    ly = H + 2
    g = 1e-6 * (16.0 / H) ** 2
    p = orc.make_params(lx=2, ly=ly, lz=2, tau=tau, wall_y=1, gx=g)
    o = orc.Oracle(p)
    nu = (tau - 0.5) / 3
    o.step(int(8 * H * H / nu))
    rho, u = o.moments()
    y = np.arange(1, ly - 1) - 0.5
    ref = g / (2 * nu) * y * (H - y)
    num = u[0, 0, 1:-1, 0]
    return np.sqrt(((num - ref) ** 2).sum() / (ref ** 2).sum())


def test_poiseuille_second_order(orc):
    # Body-force-driven flow between static halfway walls: parabola g y'(H-y')/(2 nu),
    # with an error that converges at second order in H.
    e8 = _poiseuille_err(orc, 8)
    e16 = _poiseuille_err(orc, 16)
    assert e16 < 1e-2
    assert e16 < 0.3 * e8


def test_free_sphere_rotation(orc):
    # Config 1: a torque-free sphere at the centre of simple shear rotates at -gdot/2
    # (Stokes; the sign follows u_x = gdot y).
    gd = 1e-4
    p = orc.make_params(lx=32, ly=32, lz=32, tau=1.0, shear_kind=1, gamma_dot=gd)
    o = orc.Oracle(p, pos=[[15.5, 15.5, 15.5]], radius=[4.5])
    assert o.step(600) == 0
    W = o.part("W")[0]
    assert abs(W[2] / (-gd / 2) - 1) < 3e-3
    assert np.abs(o.part("U")[0]).max() < 1e-12
