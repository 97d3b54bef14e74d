"""Pins of the oracle parts that no other test fixes from outside the oracle itself:

  - the G', G'' quadrature (eqs. 17-18) against the meaning the paper gives the two moduli
    (G' the in-phase, storage modulus of a solid; G'' = eta omega the loss modulus of a
    viscous response), fed with stresses built from the oracle's own shear protocol;
  - the orientation update of the DEM substeps against the closed-form rotation about a
    fixed axis;
  - the particle-surface stress sigma^h (eqs. 9-10, 15) against Einstein's viscosity of a
    dilute suspension, 1 + 2.5 phi (cited in Sec. 1), with the hydrodynamic radius of the
    bounce-back sphere calibrated by the Stokes torque on a held sphere (App. A coupling).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


# ---------------------------------------------------------------------------------------
# G', G'' (eqs. 16-18)

def _strain_history(p, t0, n):
    """gamma(t) and gamma_dot(t) of steps t0 .. t0+n-1 from the oracle's shear protocol:
    offset s = L_y gamma (unwrapped: |s| stays far below lx / 2) and sliding velocity
    L_y gamma_dot."""
    g = np.zeros(n)
    gd = np.zeros(n)
    for k in range(n):
        s, u = O.protocol(p, t0 + k)
        if s > 0.5 * p.lx:
            s -= p.lx
        g[k] = s / p.ly
        gd[k] = u / p.ly
    return g, gd


@pytest.mark.parametrize("theta,period,ncyc_I,ncyc_F", [(0.0, 40, 0, 1), (0.7, 64, 2, 3), (math.pi, 25, 1, 2)])
def test_moduli_of_elastic_and_viscous_responses(theta, period, ncyc_I, ncyc_F):
    # An elastic solid (sigma = G gamma) has storage modulus G and no loss; a Newtonian
    # fluid (sigma = eta gamma_dot) has loss modulus eta omega and no storage (the text
    # after eq. 18: G' is the rigidity, eta = G'' / omega).  The quadrature over whole
    # periods of integer steps makes both exact up to rounding.
    p = O.make_params(lx=1024, ly=16, lz=8, shear_kind=2, g0_I=0.3, g0_F=0.02, period=period,
                      theta=theta, ncyc_I=ncyc_I, ncyc_F=ncyc_F)
    n = (ncyc_I + ncyc_F) * period + 7  # a few steps past the observation window
    g, gd = _strain_history(p, 0, n)
    om = 2 * math.pi / period
    G, eta = 3.5, 0.8
    gg_el = O.gg_series(p, 0, G * g)
    gg_vi = O.gg_series(p, 0, eta * gd)
    gg_mix = O.gg_series(p, 0, G * g + eta * gd)
    assert abs(gg_el[0] - G) < 1e-12 * G and abs(gg_el[1]) < 1e-12 * G
    assert abs(gg_vi[1] - eta * om) < 1e-12 * eta * om and abs(gg_vi[0]) < 1e-12 * eta * om
    assert abs(gg_mix[0] - G) < 1e-12 * G and abs(gg_mix[1] - eta * om) < 1e-11 * eta * om
    # a constant pre-stress adds nothing over whole periods
    gg_c = O.gg_series(p, 0, G * g + 1.25)
    assert abs(gg_c[0] - G) < 1e-12 * G and abs(gg_c[1]) < 1e-12 * G


def test_step_feeds_the_quadrature_its_total_shear_stress():
    # the simulation's G', G'' are the quadrature of its own per-step total sigma_xy
    # (all five parts of eq. 15), taken over the observation steps only
    from paper_1904_02929_amd import synth
    w = synth.monolayer(48, 10, 0.6, seed=3, g0_I=0.05, period=30, ncyc_I=1, ncyc_F=2)
    kw = {k: v for k, v in dict(w.params).items() if k in O.DEFAULTS}
    p = O.make_params(lx=w.box[0], ly=w.box[1], lz=w.box[2], **dict(kw, g0_F=0.02))
    o = O.Oracle(p, w.pos, w.vel, w.omega, w.radius)
    hist = []
    for _ in range(95):
        assert o.step(1) == 0
        hist.append(o.sig_last()[:, 3].sum())
    _, gg = o.stress()
    ref = O.gg_series(p, 0, np.array(hist))
    assert np.allclose(gg, ref, rtol=1e-13, atol=0)
    assert gg[1] > 0  # dissipative


# ---------------------------------------------------------------------------------------
# Orientation (eq. 1 for the orientation; a quaternion per sphere)

def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _rotmat(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _axis_rot(u, ang):
    """Right-handed rotation by ang about the unit axis u (Rodrigues)."""
    K = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def test_quaternion_update_is_a_rotation_about_the_space_axis():
    # Each substep multiplies q from the left by 1 + (dt/2)(0, W) and renormalises: a
    # rotation by 2 atan(dt |W| / 2) about W in the space frame.  After n substeps the
    # orientation is the rotation by 2 n atan(dt |W| / 2) about W applied after q0, which
    # tends to the exact rotation by |W| n dt.
    W = np.array([0.003, -0.004, 0.012])
    wn = np.linalg.norm(W)
    u = W / wn
    q0 = np.array([math.cos(0.4), math.sin(0.4), 0.0, 0.0])  # 0.8 rad about x: not about W
    dt, n = 0.125, 800
    q = q0.copy()
    for _ in range(n):
        q = O.quat_step(q, W, dt)
    ang = 2 * n * math.atan(0.5 * dt * wn)
    exact = _qmul(np.array([math.cos(ang / 2), *(math.sin(ang / 2) * u)]), q0)
    assert np.abs(q - exact).max() < 1e-12
    assert np.abs(_rotmat(q) - _axis_rot(u, ang) @ _rotmat(q0)).max() < 1e-12
    # against the exact rotation by |W| t: the angle differs by n (dt |W|)^3 / 12 + ...
    t = n * dt
    err = np.abs(_rotmat(q) - _axis_rot(u, wn * t) @ _rotmat(q0)).max()
    assert err < 2 * n * (dt * wn) ** 3 / 12 + 1e-12
    # a body frame update (q (x) (0, W)) would turn about the rotated axis instead
    wrong = _qmul(q0, np.array([math.cos(ang / 2), *(math.sin(ang / 2) * u)]))
    assert np.abs(q - wrong).max() > 1e-2


def test_quaternion_of_a_spinning_sphere_in_the_step():
    # a sphere so heavy that the fluid cannot change its spin: after N lattice steps of
    # n_sub substeps its orientation is the closed-form rotation about its angular velocity
    W = np.array([[0.004, 0.002, -0.009]])
    p = O.make_params(lx=24, ly=24, lz=24, rho_p=1e15, n_sub=4)
    o = O.Oracle(p, np.array([[11.5, 11.5, 11.5]]), np.zeros((1, 3)), W, np.array([4.5]))
    N = 30
    assert o.step(N) == 0
    assert np.abs(o.part("W")[0] - W[0]).max() < 1e-15
    wn = np.linalg.norm(W[0])
    ang = 2 * N * p.n_sub * math.atan(0.5 * wn / p.n_sub)
    exact = np.array([math.cos(ang / 2), *(math.sin(ang / 2) * W[0] / wn)])
    assert np.abs(o.part("Q")[0] - exact).max() < 1e-12


# ---------------------------------------------------------------------------------------
# sigma^h: Einstein viscosity of a dilute suspension

def test_einstein_viscosity_from_particle_stress():
    # One sphere (contact radius 4.5, mapped radius 4.275) centred in 32^3 under
    # Lees-Edwards shear 1e-4 (the single-sphere configuration).  Stokes flow gives
    #   held sphere:  T_z = -4 pi eta0 a_h^3 gamma_dot   (defines the hydrodynamic radius)
    #   free sphere:  sigma_xy / (eta0 gamma_dot) - 1 = 2.5 phi_h,  phi_h = 4/3 pi a_h^3 / V
    # (Einstein; the periodic images add a correction of order phi^(2/3); the 15 % bar
    # leaves room for it, and the oracle gives 2.52 in place of 2.5).  The stresslet of a sphere in a linear flow does not depend on its spin, so
    # the held and the free sphere add the same sigma_xy: this fixes the symmetrisation,
    # since the held sphere's torque puts T_z / 2 into the antisymmetric part.  The excess
    # is steady after ~1000 steps (viscous time L^2 / nu ~ 6000 steps for the box, but the
    # images settle much faster); 2000 steps, the last 1000 averaged.
    L, a, gd = 32, 4.5, 1e-4
    c = (L - 1) / 2.0
    eta0 = (1.0 - 0.5) / 3.0

    def run(held):
        kw = dict(lx=L, ly=L, lz=L, shear_kind=1, gamma_dot=gd)
        if held:
            kw["rho_p"] = 1e15  # the fluid cannot turn or move it
        p = O.make_params(**kw)
        om = np.zeros((1, 3)) if held else np.array([[0.0, 0.0, -gd / 2]])
        o = O.Oracle(p, np.array([[c, c, c]]), np.zeros((1, 3)), om, np.array([a]))
        assert o.step(1000) == 0
        o.stress()
        assert o.step(1000) == 0
        sig, _ = o.stress()
        return o, sig

    oh, sh = run(True)
    Tz = oh.part("Th")[0][2]
    assert Tz < 0  # the held sphere is dragged the way the vorticity turns
    ah = (-Tz / (4 * math.pi * eta0 * gd)) ** (1.0 / 3.0)
    assert abs(ah / (0.95 * a) - 1) < 0.1  # about the mapped radius
    of, sf = run(False)
    assert abs(of.part("W")[0][2] / (-gd / 2) - 1) < 0.03  # torque-free: spins at -gdot/2
    phi_h = 4.0 / 3.0 * math.pi * ah ** 3 / L ** 3
    excess = sf[:, 3].sum() / (eta0 * gd) - 1.0
    assert sf[1][3] > 0  # the particle stress adds to the shear stress
    assert abs(excess / (2.5 * phi_h) - 1) < 0.15, (excess, 2.5 * phi_h)
    # the same stresslet for the held sphere (a missing symmetrisation would add
    # T_z / (2 V) ~ 14 eta0 gamma_dot here)
    excess_h = sh[:, 3].sum() / (eta0 * gd) - 1.0
    assert abs(excess_h / excess - 1) < 0.02
    # sigma^h alone carries the excess (the volume average of the fluid part is eta0 gd)
    assert abs(sf[1][3] / (eta0 * gd) / excess - 1) < 0.05
