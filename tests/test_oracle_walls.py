"""Pins of the oracle's wall geometry (Sec. 3: shear applied by moving walls of spheres).

Flat walls halfway outside the first and last rows move at -/+ U_w with U_w = L_y gamma_dot / 2
and carry layers of wall spheres.  Checks: plane Couette flow between the walls is the exact
steady solution of the halfway bounce-back (linear profile, fluid stress eta0 gamma_dot, wall
forces -/+ eta0 gamma_dot A); wall spheres follow the prescribed motion; and the momentum of
the fluid and the free spheres changes by exactly minus the force the suspension puts on the
two walls (flat walls, wall spheres' hydrodynamic and pair forces, and the momentum of nodes
the wall spheres cover and release).  CPU only.
"""
import numpy as np
import pytest


def test_couette_between_walls(orc):
    gd, tau = 1e-3, 0.8
    p = orc.make_params(lx=8, ly=32, lz=4, tau=tau, boundary=1, shear_kind=1, gamma_dot=gd)
    o = orc.Oracle(p)
    assert orc.wall_speed(p, 5) == pytest.approx(0.5 * 32 * gd, rel=1e-15)
    o.step(300)
    o.stress()
    o.wall_force()
    o.step(100)
    _, u = o.moments()
    lin = gd * (np.arange(32) - 15.5)
    assert np.abs(u[0] - lin[None, :, None]).max() < 1e-12
    assert np.abs(u[1]).max() < 1e-14 and np.abs(u[2]).max() < 1e-14
    sig, _ = o.stress()
    eta0 = (tau - 0.5) / 3
    assert sig[0][3] == pytest.approx(eta0 * gd, rel=1e-9)
    F = o.wall_force()
    A = 8 * 4
    assert F[1][0] == pytest.approx(-eta0 * gd * A, rel=1e-9)
    assert F[0][0] == pytest.approx(eta0 * gd * A, rel=1e-9)
    assert abs(F[0][2]) < 1e-15 and abs(F[1][2]) < 1e-15


def _wall_config():
    a = 4.5
    lx, ly, lz = 48, 40, 24
    pos, member = [], []
    for y, m in ((a + 1.0, 1), (ly - a - 1.0, 2)):
        for x in (6.0, 18.0, 30.0, 42.0):
            for z in (6.0, 18.0):
                pos.append([x + (0.3 if m == 2 else 0.0), y, z])
                member.append(m)
    # free spheres: one touching a bottom wall sphere, one near a top wall sphere, one alone
    pos += [[18.4, a + 1.0 + 2 * a - 0.02, 6.2], [30.5, ly - a - 1.0 - 2 * a - 0.3, 17.6],
            [12.0, 20.0, 12.0]]
    member += [0, 0, 0]
    return (lx, ly, lz), np.array(pos), np.full(len(pos), a), np.array(member, np.int32)


def test_wall_spheres_and_momentum_balance(orc):
    box, pos, rad, member = _wall_config()
    gd = 2e-3
    p = orc.make_params(lx=box[0], ly=box[1], lz=box[2], boundary=1, shear_kind=1, gamma_dot=gd,
                        tau=0.9)
    rng = np.random.default_rng(2)
    vel = np.zeros_like(pos)
    vel[member == 0] = rng.uniform(-1e-3, 1e-3, (3, 3))
    o = orc.Oracle(p, pos, vel, None, rad, wall=member)
    c, _, _ = orc.lattice()
    c = c.astype(float)
    m = 4 / 3 * np.pi * rad ** 3
    free = member == 0

    def momentum():
        fl = o.own == -1
        j = np.einsum("qa,qzyx->a", c, o.f * fl[None])
        return j + (m[free, None] * o.part("U")[free]).sum(0)

    R0 = o.part("R").copy()
    uw = orc.wall_speed(p, 0)
    P0 = momentum()
    o.wall_force()
    nst = 6
    for _ in range(nst):
        assert o.step(1) == 0
    P1 = momentum()
    F = o.wall_force() * nst  # total over the steps
    scale = np.abs(F).max()
    assert scale > 1e-4
    assert o.s.nhist > 0  # a free sphere touches a wall sphere
    for k in (0, 2):  # x and z: the rest-state parts of the flat walls cancel
        assert abs((P1[k] - P0[k]) + (F[0][k] + F[1][k])) <= 1e-11 * scale
    # prescribed motion of the wall spheres
    R, U, W = o.part("R"), o.part("U"), o.part("W")
    sgn = np.where(member == 2, 1.0, -1.0)
    for i in np.nonzero(~free)[0]:
        x = (R0[i, 0] + sgn[i] * uw * nst) % box[0]
        assert abs(R[i, 0] - x) < 1e-12
        assert R[i, 1] == R0[i, 1] and R[i, 2] == R0[i, 2]
        assert U[i, 0] == sgn[i] * uw and U[i, 1] == 0 and U[i, 2] == 0 and not W[i].any()


def test_wall_placement_is_checked(orc):
    box, pos, rad, member = _wall_config()
    pos[0, 1] = rad[0] + 0.4  # closer than pair_cutoff / 2 to its face
    p = orc.make_params(lx=box[0], ly=box[1], lz=box[2], boundary=1, shear_kind=1, gamma_dot=1e-3)
    with pytest.raises(ValueError):
        orc.Oracle(p, pos, None, None, rad, wall=member)
