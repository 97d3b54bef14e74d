"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle.

One-step parity starts both sides from the same oracle-made state, rounded on the host to
the storage precision exactly as the library stores it, and compares:
  - lists bit-exactly: owner map, ghost owners, cell list, neighbour pairs, contacts at the
    start of the step, per-sphere boundary-link counts, the link list;
  - fields to the per-step tolerance: 1e-12 (FP64), 1e-6 (FP32), 1e-3 (FP16 storage) on
    all 19 population deviations d_q = n_q - w_q rho0 of every fluid node (relative to the
    largest |d_q|: the stored post-collision state, so the collision output, ghost-mode
    relaxation and FP16 rounding are all inside the comparison), density and velocity,
    particle force/torque/stresslet, positions, velocities, spins and orientations, spring
    history, the five stress parts and, inside the observation cycles, G' and G''.
  - in FP64, also the non-equilibrium part n_q - n_q^eq(rho, u) of every fluid node
    relative to its largest magnitude (1e-9), which BGK at tau = 1 sets to zero.
"""
import sys

import numpy as np
import pytest

import parity_util as PU
from oracle import oracle as O

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-6, 2: 1e-3}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02929_amd import susp
    susp.lib()
    yield


def _announce(msg):
    print("\n[parity] " + msg, flush=True)
    sys.stdout.flush()


def _one_step_parity(box, pos, vel, om, rad, kw, precision, presteps):
    from paper_1904_02929_amd import susp
    o = PU.oracle_for(box, kw, pos, vel, om, rad)
    assert o.step(presteps) == 0
    g = PU.gpu_for(box, kw, pos, vel, om, rad, precision)
    PU.load_oracle_state(o, g, precision)
    R0 = o.part("R").copy()
    s0 = o.s.s_next
    assert np.array_equal(g.get_accumulators(), PU.oracle_accumulators(o))
    o.stress(); g.stress()
    _announce("one step from oracle step %d, precision %d, box %s, n=%d" % (o.s.step, precision, box, len(rad)))
    # link list of the start state vs an enumeration of the oracle's map and ghost points
    links_g = g.lists(susp.LIST_LINKS)
    rc_o = o.step(1)
    rc_g = g.step(1, check=False)
    assert rc_o == 0 and rc_g == 0, susp.lib().susp_last_error()
    tol = TOL[precision]
    # ---- lists, bit-exact ----
    assert np.array_equal(g.lists(susp.LIST_OWNER), o.own)
    assert np.array_equal(g.lists(susp.LIST_GHOST), o.gown)
    pi, pj = o.pairs()
    gp = g.lists(susp.LIST_PAIRS)
    assert np.array_equal(gp, np.stack([pi, pj], 1).reshape(-1, 2))
    exp_c = PU.contacts_at_start(o.params, R0, rad, s0, zip(pi, pj))
    assert [tuple(x) for x in g.lists(susp.LIST_CONTACTS).tolist()] == exp_c
    if len(rad):
        cs = g.lists(susp.LIST_CELLS)
        st, ids = PU.cell_list(box, R0, rad)
        assert np.array_equal(cs[: len(st)], st) and np.array_equal(cs[len(st):], ids)
    F, T, S, nl = g.hydro()
    assert np.array_equal(nl, o.nlinks)
    assert int(nl.sum()) == len(links_g)
    # ---- fields ----
    own = o.own
    fluid = own == -1
    fg = g.get_populations()[:, fluid]
    fo = o.f[:, fluid]
    wr = PU.weights()[:, None] * o.params.rho0
    e_d = PU.rel(fg - wr, fo - wr)  # all 19 deviations of every fluid node
    rg, ug = PU.moments(fg)
    ro, uo = PU.moments(fo)
    e_rho = float(np.abs(rg - ro).max())
    e_u = PU.rel(ug, uo)
    msg = "e_d %.3e e_rho %.3e e_u %.3e" % (e_d, e_rho, e_u)
    if precision == 0 and fo.shape[1]:
        neq_o = fo - PU.equilibrium(ro, uo)
        if np.abs(neq_o).max() > 1e-14:
            e_neq = PU.rel(fg - PU.equilibrium(rg, ug), neq_o)
            msg += " e_neq %.3e" % e_neq
            assert e_neq <= 1e-9, msg
    _announce(msg)
    assert e_d <= tol and e_rho <= tol and e_u <= tol, msg
    if len(rad):
        Fo, To = o.part("Fh"), o.part("Th")
        So = o.part("Sh").reshape(-1, 3, 3)
        So = 0.5 * (So + So.transpose(0, 2, 1))
        So6 = np.stack([So[:, 0, 0], So[:, 1, 1], So[:, 2, 2], So[:, 0, 1], So[:, 0, 2], So[:, 1, 2]], 1)
        # floors: hydrodynamic forces/torques below 1e-4 (a centred sphere in shear has
        # none) are compared in absolute terms
        e_F, e_T, e_S = PU.rel(F, Fo, 1e-4), PU.rel(T, To, 1e-4), PU.rel(S, So6, 1e-4)
        Rg, Ug, Wg, Qg = g.get_particles()
        e_R = float(np.abs(Rg - o.part("R")).max())
        e_U = PU.rel(Ug, o.part("U"), 1e-6)
        e_W = PU.rel(Wg, o.part("W"), 1e-7)
        e_Q = float(np.abs(Qg - o.part("Q")).max())  # unit quaternions
        _announce("e_F %.3e e_T %.3e e_S %.3e e_R %.3e e_U %.3e e_W %.3e e_Q %.3e" % (e_F, e_T, e_S, e_R, e_U, e_W, e_Q))
        assert max(e_F, e_T, e_S, e_U, e_W) <= max(tol, 1e-10) and e_R <= 1e-10 and e_Q <= 1e-10
        hi, hj, hx = g.get_history()
        oi, oj, ox = o.history()
        assert np.array_equal(hi, oi) and np.array_equal(hj, oj)
        if len(ox):
            assert PU.rel(hx, ox) <= max(tol, 1e-10)
    sg, gg = g.stress()
    so, go = o.stress()
    for k in range(5):
        assert PU.rel(sg[k], so[k]) <= max(tol, 1e-9), (k, sg[k], so[k])
    # G', G'' of this step: 2 / g0_F times sigma_xy times cos, sin of its phase (zero
    # outside the observation cycles), so the bar is the stress bar on that scale
    if o.params.shear_kind == 2 and o.params.g0_F != 0.0:
        scale = 2.0 / abs(o.params.g0_F) * max(float(np.abs(so[:, 3]).max()), 1e-30)
        e_gg = float(np.abs(gg - go).max()) / scale
        _announce("G' %.6e / %.6e  G'' %.6e / %.6e  e_gg %.3e" % (gg[0], go[0], gg[1], go[1], e_gg))
        assert e_gg <= max(tol, 1e-9)
    return o, g


def test_single_sphere_fp64():
    w = __import__("paper_1904_02929_amd.synth", fromlist=["x"]).single_sphere(32, 4.5, 1e-4)
    _one_step_parity(w.box, w.pos, w.vel, w.omega, w.radius, dict(w.params), 0, presteps=20)


def test_single_sphere_config_1000_steps_fp64():
    # the single-sphere configuration as stated: FP64, 32^3, sphere of radius 4.5 at the
    # centre starting at rest in the sheared fluid, 1000 steps; a torque-free sphere in
    # simple shear spins at -gamma_dot / 2 (Stokes), and both sides give the same run
    from paper_1904_02929_amd import synth
    w = synth.single_sphere(32, 4.5, 1e-4)
    kw = dict(w.params)
    _announce("single sphere 32^3, 1000 steps, FP64")
    o = PU.oracle_for(w.box, kw, w.pos, w.vel, w.omega, w.radius)
    g = PU.gpu_for(w.box, kw, w.pos, w.vel, w.omega, w.radius, 0)
    assert o.step(1000) == 0
    g.step(1000)
    Rg, Ug, Wg, Qg = g.get_particles()
    gd = kw["gamma_dot"]
    _announce("Omega_z gpu %.6e oracle %.6e, -gdot/2 %.6e" % (Wg[0, 2], o.part("W")[0, 2], -gd / 2))
    assert abs(Wg[0, 2] / (-gd / 2) - 1) < 0.03
    # the centred sphere does not translate: velocities relative to the shear scale gd L
    assert PU.rel(Wg, o.part("W")) < 1e-9 and PU.rel(Ug, o.part("U"), gd * w.box[1]) < 1e-9
    assert np.abs(Qg - o.part("Q")).max() < 1e-12 and np.abs(Rg - o.part("R")).max() < 1e-12
    fluid = o.own == -1
    wr = PU.weights()[:, None]
    assert PU.rel(g.get_populations()[:, fluid] - wr, o.f[:, fluid] - wr) < 1e-9
    sg, _ = g.stress()
    so, _ = o.stress()
    assert PU.rel(sg, so) < 1e-9
    g.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_dense_one_step(precision):
    box, pos, vel, om, rad, kw = PU.dense_workload()
    o, g = _one_step_parity(box, pos, vel, om, rad, kw, precision, presteps=40)
    assert o.s.nhist > 0  # contacts are active in the compared step


@pytest.mark.parametrize("brick", [(8, 4), (16, 8)])
def test_dense_partial_bricks_fp32(brick):
    # bricks that divide none of 41 x 48 x 37 (x: one brick of 64 over 41 columns; the last
    # z brick is short), so that brick enumeration wraps through a short brick
    box, pos, vel, om, rad, kw = PU.dense_workload(seed=5)
    kw = dict(kw, brick_y=brick[0], brick_z=brick[1])
    o, g = _one_step_parity(box, pos, vel, om, rad, kw, 1, presteps=12)
    F, T, S, nl = g.hydro()
    assert np.array_equal(nl, o.nlinks)


def test_dense_straddling_le_plane_fp32():
    # spheres placed across the sliding plane and across the x and z faces
    box, pos, vel, om, rad, kw = PU.dense_workload(seed=3)
    pos = pos.copy()
    pos[0] = [0.3, 0.2, 36.8]     # across x, y (sliding plane) and z faces
    pos[1] = [20.5, 47.7, 18.0]   # across the sliding plane only
    L = np.array(box, float)
    keep = [0, 1]
    for i in range(2, len(pos)):
        ok = True
        for k in keep:
            d = pos[i] - pos[k]
            d -= L * np.round(d / L)
            ok &= np.linalg.norm(d) > rad[i] + rad[k] + 0.2
        if ok:
            keep.append(i)
    pos, vel, om, rad = pos[keep], vel[keep], om[keep], rad[keep]
    _one_step_parity(box, pos, vel, om, rad, kw, 1, presteps=15)


def test_monolayer_oscillatory_fp32():
    from paper_1904_02929_amd import synth
    w = synth.monolayer(64, 10, 0.7, seed=2, g0_I=0.2, period=400, ncyc_I=1, ncyc_F=1)
    _one_step_parity(w.box, w.pos, w.vel, w.omega, w.radius, dict(w.params), 1, presteps=30)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_monolayer_observation_window(precision):
    # the compared step lies inside the observation cycles, so it adds to G' and G''
    from paper_1904_02929_amd import synth
    w = synth.monolayer(64, 10, 0.7, seed=6, g0_I=0.05, period=40, ncyc_I=1, ncyc_F=2)
    kw = dict(w.params, g0_F=0.02)
    o, g = _one_step_parity(w.box, w.pos, w.vel, w.omega, w.radius, kw, precision, presteps=57)
    assert o.s.gp_count == 18  # steps 40 .. 57 (the last one compared)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_dense_bgk_tau07_one_step(precision):
    # BGK with tau = 0.7: the post-collision state keeps (1 - 1/tau) of the
    # non-equilibrium part, so the collision output is not fixed by rho and u alone
    box, pos, vel, om, rad, kw = PU.dense_workload(seed=17)
    _one_step_parity(box, pos, vel, om, rad, dict(kw, tau=0.7), precision, presteps=30)


def test_pure_fluid_le_fp32():
    kw = dict(shear_kind=1, gamma_dot=2e-3)
    _one_step_parity((24, 40, 17), np.zeros((0, 3)), None, None, np.zeros(0), kw, 1, presteps=25)


def test_le_offset_wraps_fp64():
    # u = gamma_dot * ly = 0.08: the Lees-Edwards offset passes lx = 16 between steps 199
    # and 200, so the compared step moves the solid map across the wrap of the offset
    from paper_1904_02929_amd import synth
    box = (16, 40, 17)
    pos = np.array([[8.0, 10.0, 8.0], [8.0, 29.0, 8.5], [3.0, 39.6, 9.0]])
    rad = np.array([4.5, 4.5, 4.5])
    vel, om = synth.affine_start(pos, rad, 2e-3, box[1])
    _one_step_parity(box, pos, vel, om, rad, dict(shear_kind=1, gamma_dot=2e-3), 0, presteps=199)


def test_full_size_one_step_fp32():
    # the benchmark workload at its full size (256^3, 12,914 spheres) in the launch
    # configuration bench.py times (heuristic bricks, FP32): one step from the oracle's start
    from paper_1904_02929_amd import synth
    w = synth.bulk3d(256, 0.55, 1e-4, seed=1)
    _one_step_parity(w.box, w.pos, w.vel, w.omega, w.radius, dict(w.params), 1, presteps=0)


# eq. (5) as the linearised operator with three distinct eigenvalues (shear, bulk, ghost)
MULTI = dict(collision=1, tau=0.8, tau_bulk=0.65, tau_ghost=1.25)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_multi_eigenvalue_dense_one_step(precision):
    box, pos, vel, om, rad, kw = PU.dense_workload(seed=13)
    _one_step_parity(box, pos, vel, om, rad, dict(kw, **MULTI), precision, presteps=30)


def test_multi_eigenvalue_monolayer_fp32():
    from paper_1904_02929_amd import synth
    w = synth.monolayer(96, 10, 0.75, seed=4, g0_I=0.05, period=400)
    _one_step_parity(w.box, w.pos, w.vel, w.omega, w.radius, dict(w.params, **MULTI), 1, presteps=25)


def test_multi_eigenvalue_full_size_fp32():
    from paper_1904_02929_amd import synth
    w = synth.bulk3d(256, 0.55, 1e-4, seed=1)
    _one_step_parity(w.box, w.pos, w.vel, w.omega, w.radius, dict(w.params, **MULTI), 1, presteps=0)


@pytest.mark.parametrize("precision", [0, 1])
def test_implicit_squeeze_dense_one_step(precision):
    # the squeeze terms taken at the new velocities by 6 Jacobi sweeps per substep
    box, pos, vel, om, rad, kw = PU.dense_workload(seed=9)
    _one_step_parity(box, pos, vel, om, rad, dict(kw, lub_implicit=6), precision, presteps=20)


def test_implicit_squeeze_closing_pair_fp64():
    # a pair closing at a gap of 0.005 with one substep per step (the oracle pin's case):
    # three steps from creation on both sides, the explicit update would blow up here
    a, h = 4.5, 0.005
    pos = np.array([[20.0, 20.0, 20.0], [20.0 + 2 * a + h, 20.0, 20.0]])
    vel = np.array([[2e-4, 0, 0], [-2e-4, 0, 0]])
    kw = dict(n_sub=1, lub_delta=1e-4, F0=0.0, lub_implicit=30)
    _announce("implicit squeeze, closing pair")
    o = PU.oracle_for((48, 40, 40), kw, pos, vel, np.zeros((2, 3)), np.full(2, a))
    g = PU.gpu_for((48, 40, 40), kw, pos, vel, np.zeros((2, 3)), np.full(2, a), 0)
    assert o.step(3) == 0
    g.step(3)
    Rg, Ug, Wg, _ = g.get_particles()
    assert np.abs(Rg - o.part("R")).max() < 1e-12
    assert PU.rel(Ug, o.part("U")) < 1e-10
    g.close()


def test_multistep_fp64_from_create():
    # both sides start from their own initial state and run 25 steps
    box, pos, vel, om, rad, kw = PU.dense_workload(seed=11)
    o = PU.oracle_for(box, kw, pos, vel, om, rad)
    g = PU.gpu_for(box, kw, pos, vel, om, rad, 0)
    assert o.step(25) == 0
    g.step(25)
    Rg, Ug, Wg, _ = g.get_particles()
    assert np.abs(Rg - o.part("R")).max() < 1e-9
    assert PU.rel(Ug, o.part("U")) < 1e-8
    fluid = o.own == -1
    assert np.array_equal(g.lists(__import__("paper_1904_02929_amd.susp", fromlist=["x"]).LIST_OWNER), o.own)
    _, ug = PU.moments(g.get_populations()[:, fluid])
    _, uo = PU.moments(o.f[:, fluid])
    assert PU.rel(ug, uo) < 1e-9


def test_overlap_is_reported():
    from paper_1904_02929_amd import susp
    box = (32, 48, 32)
    pos = np.array([[10.0, 20.0, 10.0], [18.0, 20.0, 10.0]])  # gap -1: mapped spheres overlap
    rad = np.array([4.5, 4.5])
    with pytest.raises(susp.SuspError) as ei:
        PU.gpu_for(box, {}, pos, None, None, rad, 1)
    assert ei.value.code == susp.EUNSTABLE
    o = PU.oracle_for(box, {}, pos, None, None, rad)
    assert o.step(1) == -4


def test_invalid_parameters():
    from paper_1904_02929_amd import susp
    with pytest.raises(susp.SuspError) as ei:
        PU.gpu_for((32, 20, 32), {}, np.array([[5.0, 5.0, 5.0]]), None, None, np.array([4.5]), 1)
    assert ei.value.code == susp.EINVAL
    with pytest.raises(susp.SuspError):
        PU.gpu_for((32, 48, 32), {}, np.array([[5.0, 50.0, 5.0]]), None, None, np.array([4.5]), 1)
