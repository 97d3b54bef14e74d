"""Pins of the oracle's particle side: coupling, lists, pair forces and stresses.

Every check compares the FP64 oracle with something independent of it: conservation laws,
brute-force geometry written here with explicit image enumeration, closed forms of the
damped oscillator and of Reynolds lubrication, reciprocity and rigid-body identities of the
resistance matrix, and finite differences of pair energies.  CPU only.
"""
import math

import numpy as np
import pytest


def _params(orc, **kw):
    base = dict(lx=24, ly=24, lz=24, tau=1.0)
    base.update(kw)
    return orc.make_params(**base)


# ----------------------------------------------------------------------------- coupling
def test_rest_state_link_constant_cancels(orc):
    # eqs. (6), (9), (10): in the uniform rest state every link carries 2 w rho0 c.  For a
    # sphere away from the sliding plane the entry and exit links of each lattice line
    # cancel, so the literal sum is zero and measuring link momentum from the rest state
    # changes nothing.  A sphere straddling the Lees-Edwards plane is seen through the
    # integer lattice on one side and the offset ghost points on the other: there the
    # rest-state part does not cancel, which is why it is kept out of the force.
    # eq. (16) with period 2: at t = 1 the phase is pi, so the offset 2 g0 ly is generic and
    # the sliding velocity vanishes; fluid and spheres at rest
    p = _params(orc, shear_kind=2, period=2, g0_I=0.1119, ncyc_I=10)
    o = orc.Oracle(p, pos=[[11.37, 12.81, 10.09], [5.2, 23.6, 15.3]], radius=[4.5, 4.5])
    o.step(1)
    s, ule = orc.protocol(p, 1)
    assert abs(s - 2 * 0.1119 * 24) < 1e-12 and abs(ule) < 1e-13
    o.f[...] = orc.feq(1.0, [0, 0, 0])[:, None, None, None]
    U = o.part("U"); U[...] = 0.0
    W = o.part("W"); W[...] = 0.0
    o.step(1)
    Fh, Th, Fr, Tr = o.part("Fh"), o.part("Th"), o.part("Frest"), o.part("Trest")
    assert o.nlinks[0] > 500 and o.nlinks[1] > 500
    assert np.abs(Fh).max() < 1e-12 and np.abs(Th).max() < 1e-11
    assert np.abs(o.part("Sh")).max() < 1e-11
    assert np.abs(Fr[0]).max() < 1e-13 and np.abs(Tr[0]).max() < 1e-12
    assert np.abs(Fr[1]).max() > 1e-2


def _totals(o, orc):
    c, _, _ = orc.lattice()
    own = o.own
    fluid = own == -1
    f = o.f
    mass = f[:, fluid].sum()
    mom = np.tensordot(c.T.astype(float), f[:, fluid], axes=([1], [0])).sum(1)
    m = o.part("m")
    mom = mom + (m[:, None] * o.part("U")).sum(0)
    return mass, mom


def test_moving_sphere_momentum_and_mass(orc):
    # Bounce-back exchanges exactly -f_link with the fluid; covering/uncovering moves a
    # node's momentum between fluid and particle.  Periodic box, no shear: the total
    # momentum is conserved; fluid mass plus the ledger of absorbed mass is conserved.
    p = _params(orc)
    o = orc.Oracle(p, pos=[[11.3, 12.2, 10.7]], vel=[[0.02, -0.013, 0.007]],
                   omega=[[1e-3, -2e-3, 3e-3]], radius=[4.5])
    m0, P0 = _totals(o, orc)
    own0 = o.own.copy()
    assert o.step(200) == 0
    m1, P1 = _totals(o, orc)
    assert (own0 != o.own).sum() > 20  # nodes were covered and uncovered
    assert abs((m1 + o.s.ledger) / m0 - 1) < 1e-13
    assert np.abs(P1 - P0).max() < 1e-12 * (abs(P0).max() + 1)


# ----------------------------------------------------------------------------- geometry
def _img_d2(R, X, s, L):
    """Squared distance from the points X (..., 3) to the nearest Lees-Edwards/periodic
    image of R (brute force over explicit images)."""
    X = np.asarray(X, float)
    best = np.full(X.shape[:-1], np.inf)
    for k in (-1, 0, 1):
        for mx in (-2, -1, 0, 1, 2):
            for mz in (-1, 0, 1):
                img = np.array([R[0] + k * s + mx * L[0], R[1] + k * L[1], R[2] + mz * L[2]])
                d = X - img
                best = np.minimum(best, (d * d).sum(-1))
    return best


def _random_state(orc, seed, n=6, L=(20, 22, 18), steps=7):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) * np.array(L)
    pos[0, 1] = 0.4      # straddle the Lees-Edwards plane
    pos[1, 1] = L[1] - 0.8
    rad = rng.choice([2.6, 3.4], n)
    p = orc.make_params(lx=L[0], ly=L[1], lz=L[2], shear_kind=1, gamma_dot=0.3, n_sub=1,
                        rho_p=1e9)
    o = orc.Oracle(p, pos=pos, radius=rad)
    o.step(steps)  # moves the Lees-Edwards offset to a generic value
    o.s.flags = 0
    o.remap()
    return o, np.array(L)


@pytest.mark.parametrize("seed", [1, 2])
def test_node_map_bruteforce(orc, seed):
    # The owner map (App. A mapped spheres, a_map = 0.95 a) equals a brute-force scan of
    # every node against every Lees-Edwards/periodic image of every sphere.
    o, L = _random_state(orc, seed)
    s = o.s.s_next
    R, amap = o.part("R"), o.part("amap")
    own = o.own
    z, y, x = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
    X = np.stack([x, y, z], -1).astype(float)
    exp = np.full(own.shape, -1)
    for p in range(len(R) - 1, -1, -1):  # lowest id wins a (never expected) tie
        exp[_img_d2(R[p], X, s, L) < amap[p] ** 2] = p
    assert (exp >= 0).sum() > 100
    assert np.array_equal(own, exp)


def test_ghost_owner_bruteforce(orc):
    # Ghost points (x,-1,z) and (x,ly,z) belong to a sphere if inside one of its images.
    o, L = _random_state(orc, 3)
    o.step(1)
    s = o.s.s
    # the ghost planes were built with the pre-step positions; rebuild that state
    o2, _ = _random_state(orc, 3)
    R, amap = o2.part("R").copy(), o2.part("amap")
    o2.step(1)
    assert abs(o2.s.s - s) == 0
    g = o2.gown
    z, x = np.meshgrid(np.arange(L[2]), np.arange(L[0]), indexing="ij")
    for gi, gy in enumerate((-1.0, float(L[1]))):
        X = np.stack([x, np.full_like(x, gy, dtype=float), z], -1).astype(float)
        exp = np.full(x.shape, -1)
        for p in range(len(R) - 1, -1, -1):
            exp[_img_d2(R[p], X, s, L) < amap[p] ** 2] = p
        assert np.array_equal(g[gi], exp)
    assert (g >= 0).sum() > 10


def test_pair_list_bruteforce(orc):
    # Neighbour list: all i<j whose nearest-image gap is below the list cutoff.
    rng = np.random.default_rng(11)
    L = np.array([30, 28, 26])
    n = 40
    pos = rng.random((n, 3)) * L
    rad = rng.choice([2.5, 3.5], n)
    p = orc.make_params(lx=30, ly=28, lz=26, shear_kind=1, gamma_dot=0.21, n_sub=1, rho_p=1e12)
    o = orc.Oracle(p, pos=pos, radius=rad)
    o.step(5)
    s = o.s.s_next
    o.s.flags = 0
    R = o.part("R").copy()
    o.step(1)  # builds the list from R at s
    pi, pj = o.pairs()
    got = set(zip(pi.tolist(), pj.tolist()))
    exp = set()
    for i in range(n):
        for j in range(i + 1, n):
            if _img_d2(R[j], R[i], s, L) < (rad[i] + rad[j] + 1.0) ** 2:
                exp.add((i, j))
    assert got == exp
    assert list(zip(pi.tolist(), pj.tolist())) == sorted(got)


# ----------------------------------------------------------------------------- contacts
def _derived(orc, radius=(4.5, 6.3), **kw):
    p = orc.make_params(lx=64, ly=64, lz=64, **kw)
    return p, orc.resolve(p, np.array(radius))


def test_derived_constants(orc):
    # Sec. 2: dt = 0.6 sqrt(m0/kn) with dt = 1; eta_n = sqrt(m0 kn); lambda = 0.02 a_min;
    # delta = 0.01 a_min; F0 = 2e-4 kn (oscillatory-shear value).
    p, d = _derived(orc)
    m0 = 0.5 * (4 / 3 * math.pi * (4.5**3 + 6.3**3))
    assert abs(d.m0 / m0 - 1) < 1e-15
    assert abs(0.6 * math.sqrt(d.m0 / d.kn) - 1) < 1e-14
    assert abs(d.eta_n / math.sqrt(m0 * d.kn) - 1) < 1e-14
    assert abs(d.debye_lambda - 0.09) < 1e-15 and abs(d.lub_delta - 0.045) < 1e-15
    assert abs(d.F0 / d.kn - 2e-4) < 1e-18
    assert abs(d.eta0 - 1 / 6) < 1e-16


def test_restitution_damped_oscillator(orc):
    # A dry head-on collision of the linear spring-dashpot is a damped oscillator with
    # restitution e = exp(-pi z / sqrt(1 - z^2)), z = eta_n / (2 sqrt(m_eff kn)).
    p, d = _derived(orc, radius=(4.5, 4.5), kn=40.0, eta_n=15.0)
    a = 4.5
    m = 4 / 3 * math.pi * a**3
    meff = m / 2
    z = d.eta_n / (2 * math.sqrt(meff * d.kn))
    e_exact = math.exp(-math.pi * z / math.sqrt(1 - z * z))
    v0 = 0.05
    xi = np.zeros(3)
    Ri, Rj = np.array([0.0, 0, 0]), np.array([-9.0 - 1e-9, 0, 0])
    Ui, Uj = np.array([-v0 / 2, 0, 0]), np.array([v0 / 2, 0, 0])
    Z = np.zeros(3)
    dt = 1.0 / 64
    for _ in range(200000):
        on, xi, Fi, _, _, _ = orc.contact(p, d, a, a, Ri - Rj, Ui, Uj, Z, Z, dt, xi)
        Ui = Ui + dt * Fi / m
        Uj = Uj - dt * Fi / m
        Ri = Ri + dt * Ui
        Rj = Rj + dt * Uj
        if not on and (Ui[0] - Uj[0]) > 0:
            break
    e = (Ui[0] - Uj[0]) / v0
    assert abs(e / e_exact - 1) < 0.01


def test_tangential_ramp_and_coulomb_cap(orc):
    # Stick: F_t = -kt v t grows linearly; slip: |F_t| = mu |F_n| and the spring is reset
    # to -F_t/kt (Sec. 2 Coulomb rule).
    p, d = _derived(orc, radius=(4.5, 4.5), mu=0.5)
    a = 4.5
    dv = np.array([0.0, 9.0 - 0.01, 0.0])  # i above j, overlap 0.01
    v = 2e-3
    Ui, Uj = np.array([v, 0, 0]), np.zeros(3)
    Z = np.zeros(3)
    xi = np.zeros(3)
    dt = 0.125
    Fn = d.kn * 0.01
    for k in range(1, 4000):
        on, xi, Fi, Ti, Tj, Fnv = orc.contact(p, d, a, a, dv, Ui, Uj, Z, Z, dt, xi)
        assert on == 1
        Ft = Fi - Fnv
        stick = d.kt * v * k * dt
        if stick < 0.5 * Fn * (1 - 1e-12):
            assert abs(Ft[0] + stick) < 1e-12 * max(1, stick)
        elif stick > 0.5 * Fn * (1 + 1e-12):
            assert abs(np.linalg.norm(Ft) - 0.5 * Fn) < 1e-12 * Fn
            assert np.allclose(xi, -Ft / d.kt, rtol=0, atol=1e-15)
        # eq. (11t): T_i = a_i n_ij x F_t with n_ij toward j; friction on i's bottom
        assert np.allclose(Ti, np.cross(-a * dv / np.linalg.norm(dv), Ft), atol=1e-14)


def test_coulomb_bound_random(orc):
    p, d = _derived(orc, radius=(4.5, 6.3))
    rng = np.random.default_rng(2)
    for _ in range(300):
        ai, aj = rng.choice([4.5, 6.3], 2)
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        dv = n * (ai + aj - 0.05 * rng.random())
        xi = 0.01 * rng.normal(size=3)
        for _ in range(5):
            U = 0.02 * rng.normal(size=(2, 3)); W = 0.01 * rng.normal(size=(2, 3))
            on, xi, Fi, _, _, Fn = orc.contact(p, d, ai, aj, dv, U[0], U[1], W[0], W[1], 0.125, xi)
            Ft = Fi - Fn
            assert np.linalg.norm(Ft) <= p.mu * np.linalg.norm(Fn) * (1 + 4e-16) + 1e-300
            assert abs(Ft @ n) < 1e-12 * (np.linalg.norm(Ft) + 1e-30)


# ----------------------------------------------------------------------------- DLVO
def test_dlvo_shape(orc):
    # eq. (13): F0 exp(-h/lambda) along n, clamped at contact, zero beyond the cutoff.
    p, d = _derived(orc)
    n = np.array([0.6, 0.0, 0.8])
    f = lambda h: orc.dlvo(p, d, 4.5, 6.3, n * (10.8 + h))
    F1, F2 = f(0.2), f(0.2 + d.debye_lambda)
    assert abs(np.linalg.norm(F1) / np.linalg.norm(F2) / math.e - 1) < 1e-12
    assert np.allclose(np.cross(F1, n), 0, atol=1e-18) and F1 @ n > 0
    assert abs(np.linalg.norm(f(-0.01)) / d.F0 - 1) < 1e-14
    assert np.all(f(1.0) == 0)


# ----------------------------------------------------------------------------- lubrication
def _lub_params(orc, sub=0):
    return _derived(orc, radius=(4.5, 6.3), lub_subtract_hc=sub)


def test_lub_reynolds_squeeze(orc):
    # Reynolds: two spheres approaching along their line of centres feel
    # F = 6 pi eta (a_i a_j / (a_i + a_j))^2 V / gap (leading order, gap = h + delta).
    p, d = _lub_params(orc)
    rng = np.random.default_rng(4)
    for _ in range(20):
        ai, aj = rng.uniform(3, 7, 2)
        h = rng.uniform(0.0, 0.45)
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        V = 1e-3
        Fi, Ti, Tj, Si, Sj = orc.lubrication(p, d, ai, aj, n * (ai + aj + h), -V * n, 0 * n, 0 * n, 0 * n)
        ref = 6 * math.pi * d.eta0 * (ai * aj / (ai + aj)) ** 2 * V / (h + d.lub_delta)
        assert abs(Fi @ n / ref - 1) < 1e-12
        assert np.linalg.norm(np.cross(Fi, n)) < 1e-14 * ref


def test_lub_equal_sphere_shear_coefficient(orc):
    # Equal spheres in relative tangential motion: Y^A = (1/6) ln(1/xi) (Jeffrey & Onishi).
    p, d = _lub_params(orc)
    a, h = 4.5, 0.2
    n = np.array([0, 1.0, 0])
    Ut = np.array([1e-3, 0, 0])
    Fi, *_ = orc.lubrication(p, d, a, a, n * (2 * a + h), Ut, 0 * Ut, 0 * Ut, 0 * Ut)
    xi = 2 * (h + d.lub_delta) / (2 * a)
    ref = -6 * math.pi * d.eta0 * a * (1 / 6) * math.log(1 / xi) * 1e-3
    assert abs(Fi[0] / ref - 1) < 1e-12


@pytest.mark.parametrize("sub", [0, 1])
def test_lub_rigid_rotation_is_free(orc, sub):
    # A rigidly rotating touching pair has no relative surface motion in the gap, so the
    # singular terms give no force, torque or stresslet.  This fixes beta = a_j/a_i, the
    # direction of n and the relative signs of the B, C, G and H blocks.
    p, d = _lub_params(orc, sub)
    rng = np.random.default_rng(6)
    for _ in range(200):
        ai, aj = rng.uniform(2, 8, 2)
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        W = rng.normal(size=3) * 1e-3
        dv = n * (ai + aj)
        Ui = rng.normal(size=3) * 1e-3
        Uj = Ui - np.cross(W, dv)
        Fi, Ti, Tj, Si, Sj = orc.lubrication(p, d, ai, aj, dv, Ui, Uj, W, W)
        scale = d.eta0 * 100 * 1e-3 * 50
        assert np.abs(Fi).max() < 1e-12 * scale
        assert np.abs(Ti).max() < 1e-11 * scale and np.abs(Tj).max() < 1e-11 * scale
        assert np.abs(Si).max() < 1e-11 * scale and np.abs(Sj).max() < 1e-11 * scale


def _lub_matrix_apply(orc, p, d, ai, aj, dv, x):
    U, Wi, Wj = x[:3], x[3:6], x[6:]
    Fi, Ti, Tj, _, _ = orc.lubrication(p, d, ai, aj, dv, U, np.zeros(3), Wi, Wj)
    return np.concatenate([Fi, Ti, Tj])


def test_lub_reciprocity_and_dissipation(orc):
    # Lorentz reciprocity: the force/torque block is symmetric; dissipation
    # -(F.U + T_i.W_i + T_j.W_j) is non-negative.
    p, d = _lub_params(orc, 1)
    rng = np.random.default_rng(8)
    for _ in range(100):
        ai, aj = rng.uniform(2, 8, 2)
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        dv = n * (ai + aj + rng.uniform(0, 0.49))
        M = np.stack([_lub_matrix_apply(orc, p, d, ai, aj, dv, e) for e in np.eye(9)], 1)
        assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
        x = rng.normal(size=9)
        assert x @ M @ x <= 1e-12 * np.abs(M).max() * (x @ x)


def test_lub_stresslet_matches_force_dipole(orc):
    # For a closing pair the X^G stresslets add up to the deviatoric part of the force
    # dipole -(a_i + a_j) n (x) F_i: compressive on approach.
    p, d = _lub_params(orc, 1)
    rng = np.random.default_rng(10)
    for _ in range(20):
        ai, aj = rng.uniform(3, 7, 2)
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        dv = n * (ai + aj + rng.uniform(0, 0.4))
        Fi, _, _, Si, Sj = orc.lubrication(p, d, ai, aj, dv, -1e-3 * n, 0 * n, 0 * n, 0 * n)
        D = -(ai + aj) * np.outer(n, Fi)
        D = 0.5 * (D + D.T)
        D -= np.trace(D) / 3 * np.eye(3)
        S = Si + Sj
        Sm = np.array([[S[0], S[3], S[4]], [S[3], S[1], S[5]], [S[4], S[5], S[2]]])
        assert np.abs(Sm - D).max() < 1e-12 * np.abs(D).max()
        assert n @ Sm @ n < 0


# ----------------------------------------------------------------------------- stresses
def _static_system(orc, kind):
    L = 40
    if kind == "contact":
        pos = [[10.0, 10.0, 10.0], [10.0 + 9.0 - 0.02, 10.3, 10.0], [10.1, 10.0 + 10.8 - 0.01, 10.2]]
        rad = [4.5, 4.5, 6.3]
    else:
        pos = [[10.0, 10.0, 10.0], [10.0 + 9.3, 10.2, 10.1], [10.3, 10.0 + 10.8 + 0.4, 10.0]]
        rad = [4.5, 4.5, 6.3]
    p = orc.make_params(lx=L, ly=L, lz=L, n_sub=1, rho_p=1e15, kn=30.0, F0=0.01,
                        debye_lambda=0.15, lub_hc=0.0)
    return p, np.array(pos), np.array(rad)


@pytest.mark.parametrize("kind", ["contact", "dlvo"])
def test_pair_stress_is_energy_derivative(orc, kind):
    # eqs. (12), (14) read as -(1/V) sum over pairs of sym(r_ij (x) F_ij): for a conservative
    # pair force this is (1/V) dE/d(eps) under an affine strain eps (finite differences of
    # the pair energy written here).  Fixes the sign and the factor of the double sum.
    p, pos, rad = _static_system(orc, kind)
    o = orc.Oracle(p, pos=pos, radius=rad)
    o.step(1)
    sig = o.sig_last()[3 if kind == "contact" else 4]
    d = orc.resolve(p, rad)
    V = float(p.lx) ** 3

    def energy(eps):
        E = 0.0
        X = pos @ (np.eye(3) + eps).T
        for i in range(3):
            for j in range(i + 1, 3):
                r = np.linalg.norm(X[i] - X[j])
                h = r - rad[i] - rad[j]
                if kind == "contact" and h < 0:
                    E += 0.5 * d.kn * h * h
                if kind == "dlvo" and 0 <= h < 1.0:
                    E += d.F0 * d.debye_lambda * math.exp(-h / d.debye_lambda)
        return E

    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    eh = 1e-7
    for c, (a, b) in enumerate(idx):
        e = np.zeros((3, 3))
        e[a, b] += 0.5 * eh
        e[b, a] += 0.5 * eh
        # with eps_ab = eps_ba = eh/2 the central difference is V sigma_ab for every ab
        num = (energy(e) - energy(-e)) / (2 * eh) / V
        assert abs(sig[c] - num) < 1e-6 * np.abs(sig).max() + 1e-15


def test_pure_fluid_loss_modulus(orc):
    # eqs. (16)-(18): a Newtonian fluid under oscillatory Lees-Edwards strain has the
    # volume-averaged shear stress eta0 gdot(t), i.e. G'' = eta0 omega and G' = 0.
    P = 4000
    p = orc.make_params(lx=2, ly=16, lz=2, tau=1.0, shear_kind=2, g0_I=0.02, g0_F=0.01,
                        period=P, theta=0.3, ncyc_I=1, ncyc_F=1)
    o = orc.Oracle(p)
    o.step(2 * P)
    _, gg = o.stress()
    eta0, om = 1 / 6, 2 * math.pi / P
    assert abs(gg[1] / (eta0 * om) - 1) < 2e-3
    assert abs(gg[0]) < 5e-3 * eta0 * om
