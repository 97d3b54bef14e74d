"""Pins of the oracle's implicit squeeze lubrication (the implicit pairwise update of the
lubrication force that the paper cites for its lubrication corrections).

Per substep the normal squeeze part -zeta n n.(U_i - U_j) of each pair's lubrication force
(zeta = eta0 X^A of App. A) is taken at the new velocities; the rest stays explicit.  Checks:
the Jacobi solver reaches numpy's direct solution of the same linear system; for one pair
the converged update scales the normal relative velocity by 1 / (1 + dt zeta (1/m_i + 1/m_j))
and conserves momentum; and for a pair closing at a gap where the explicit update flips and
amplifies the relative velocity each step, the implicit one makes it decay.  CPU only.
"""
import math

import numpy as np
import pytest


def _system(rng, n=7, npairs=10):
    m = rng.uniform(50, 400, n)
    pi, pj = [], []
    while len(pi) < npairs:
        i, j = sorted(rng.choice(n, 2, replace=False))
        if (i, j) not in zip(pi, pj):
            pi.append(i); pj.append(j)
    zeta = rng.uniform(10, 300, npairs)
    nv = rng.normal(size=(npairs, 3)); nv /= np.linalg.norm(nv, axis=1)[:, None]
    sh = np.zeros((npairs, 3)); sh[:, 0] = rng.choice([-1, 0, 1], npairs) * 0.01
    b = rng.normal(size=(n, 3)) * 0.1
    fixed = np.zeros(n, np.int32); fixed[0] = 1
    return m, fixed, b, np.array(pi), np.array(pj), zeta, nv, sh


def test_solver_reaches_direct_solution(orc):
    rng = np.random.default_rng(4)
    m, fixed, b, pi, pj, zeta, nv, sh = _system(rng)
    dt, n = 0.5, len(m)
    U0 = rng.normal(size=(n, 3)) * 0.01
    U = orc.implicit_solve(m, fixed, b, pi, pj, zeta, nv, sh, dt, 600, U0)
    # the same equations as one dense system over the free spheres' velocities
    free = np.nonzero(fixed == 0)[0]
    idx = {i: k for k, i in enumerate(free)}
    M = np.zeros((3 * len(free), 3 * len(free))); r = np.zeros(3 * len(free))
    for i in free:
        M[3 * idx[i]:3 * idx[i] + 3, 3 * idx[i]:3 * idx[i] + 3] += m[i] * np.eye(3)
        r[3 * idx[i]:3 * idx[i] + 3] += b[i]
    for k in range(len(pi)):
        i, j, P = pi[k], pj[k], dt * zeta[k] * np.outer(nv[k], nv[k])
        # force on i: -zeta n n.(U_i - U_j - s); on j the opposite
        for a, bb, sgn in ((i, j, 1.0), (j, i, -1.0)):
            if fixed[a]:
                continue
            ia = 3 * idx[a]
            M[ia:ia + 3, ia:ia + 3] += P
            if fixed[bb]:
                r[ia:ia + 3] += P @ U0[bb]
            else:
                M[ia:ia + 3, 3 * idx[bb]:3 * idx[bb] + 3] -= P
            r[ia:ia + 3] += sgn * (P @ sh[k])
    x = np.linalg.solve(M, r).reshape(-1, 3)
    np.testing.assert_allclose(U[free], x, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(U[fixed == 1], U0[fixed == 1])


def test_one_pair_closed_form(orc):
    m = np.array([300.0, 120.0])
    U = np.array([[0.01, 0.002, 0.0], [-0.02, 0.0, 0.001]])
    n = np.array([[0.6, 0.8, 0.0]])
    zeta, dt = np.array([900.0]), 1.0
    b = m[:, None] * U
    Un = orc.implicit_solve(m, np.zeros(2, np.int32), b, [0], [1], zeta, n, np.zeros((1, 3)), dt, 200, U)
    du, dn = U[0] - U[1], Un[0] - Un[1]
    f = 1.0 / (1.0 + dt * zeta[0] * (1 / m[0] + 1 / m[1]))
    assert n[0] @ dn == pytest.approx(f * (n[0] @ du), rel=1e-12)
    t = du - (n[0] @ du) * n[0]
    np.testing.assert_allclose(dn - (n[0] @ dn) * n[0], t, atol=1e-15)
    np.testing.assert_allclose((m[:, None] * Un).sum(0), (m[:, None] * U).sum(0), atol=1e-13)


def test_damped_where_explicit_flips(orc):
    # two spheres closing along x at a gap of 0.005 with roughness 1e-4 and one substep per
    # step: dt zeta (2/m) is about 15, so the explicit update flips and amplifies the normal
    # relative velocity every step; the implicit one damps it without changing sign
    a, h = 4.5, 0.005
    pos = np.array([[20.0, 20.0, 20.0], [20.0 + 2 * a + h, 20.0, 20.0]])
    vel = np.array([[2e-4, 0, 0], [-2e-4, 0, 0]])
    res = {}
    for imp in (0, 30):
        p = orc.make_params(lx=48, ly=40, lz=40, n_sub=1, lub_delta=1e-4, F0=0.0, lub_implicit=imp)
        o = orc.Oracle(p, pos, vel, None, np.full(2, a))
        d = orc.resolve(p, [a, a])
        z = orc.lub_squeeze(p, d, a, a, pos[0] - pos[1])
        m = 4 / 3 * math.pi * a ** 3
        assert 2 * z / m > 10
        rel = []
        for _ in range(3):
            o.step(1)
            U = o.part("U")
            rel.append(U[1, 0] - U[0, 0])  # < 0 while the pair closes (starts at -4e-4)
        res[imp] = rel
    ex, im = res[0], res[30]
    # explicit: the sign flips every step and the magnitude grows (the third step fails)
    assert ex[0] > 5 * 4e-4 and ex[1] < -5 * ex[0] and ex[2] > -5 * ex[1]
    # implicit: the relative velocity decays (the explicit fluid force of the first step
    # still overshoots it once)
    assert abs(im[2]) < abs(im[1]) < abs(im[0]) < 4e-4
