"""GPU parity of the wall geometry (Sec. 3: shear by moving walls of spheres) through the C ABI.

Both sides start from their own creation with the same inputs and step together: plane
Couette flow between bare walls, and walls carrying layers of spheres with free spheres that
touch them.  Compared: owner map and spring-history pairs exactly, populations, particle
states and the force on each wall within 1e-10 in FP64 and 1e-6 (relative) in FP32; graph
replay bitwise equal to plain launches.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02929_amd import susp as S
    from oracle import oracle as O
    S.lib()
    return S, O


def _config():
    # the oracle pin's configuration (tests/test_oracle_walls.py)
    import test_oracle_walls as W
    return W._wall_config()


def _pair(S, O, box, pos, vel, rad, member, prec, gd, tau=0.9):
    kw = dict(boundary=1, shear_kind=1, gamma_dot=gd, tau=tau)
    o = O.Oracle(O.make_params(lx=box[0], ly=box[1], lz=box[2], **kw), pos, vel, None, rad,
                 wall=member)
    p = S.make_params(box, radius=rad, pos=pos, vel=vel, precision=prec, wall=member, **kw)
    return o, S.Simulation(p)


def _rel(a, b, floor=0.0):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor, 1e-300))


def test_couette_between_walls_fp64(env):
    S, O = env
    print("\n[walls] Couette (8, 32, 8), FP64", flush=True)
    o, g = _pair(S, O, (8, 32, 8), None, None, None, None, S.FP64, 1e-3, tau=0.8)
    assert o.step(60) == 0
    g.step(60)
    assert _rel(g.get_populations(), o.f) < 1e-13
    Fo, Fg = o.wall_force(), g.wall_force()
    assert _rel(Fg, Fo) < 1e-11
    g.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5)])
def test_wall_spheres(env, prec, tol):
    S, O = env
    box, pos, rad, member = _config()
    vel = np.zeros_like(pos)
    vel[member == 0] = np.random.default_rng(2).uniform(-1e-3, 1e-3, (3, 3))
    print("\n[walls] %d wall + %d free spheres, box %s, precision %d"
          % ((member > 0).sum(), (member == 0).sum(), box, prec), flush=True)
    o, g = _pair(S, O, box, pos, vel, rad, member, prec, 2e-3)
    seen = False
    for steps in (3, 3):
        assert o.step(steps) == 0
        assert g.step(steps, check=False) == 0
        assert np.array_equal(g.lists(S.LIST_OWNER), o.own)
        hi, hj, _ = g.get_history()
        oi, oj, _ = o.history()
        assert np.array_equal(hi, oi) and np.array_equal(hj, oj)
        seen = seen or len(hi) > 0
        R, U, W, _ = g.get_particles()
        assert np.abs(R - o.part("R")).max() < max(tol, 1e-12) * 10
        assert _rel(U, o.part("U"), 1e-6) < tol and _rel(W, o.part("W"), 1e-7) < tol
        fl = o.own == -1
        assert _rel(g.get_populations()[:, fl], o.f[:, fl]) < tol
        Fo, Fg = o.wall_force(), g.wall_force()
        assert _rel(Fg, Fo) < max(tol, 1e-9) * 10, (Fg, Fo)
    assert seen  # a free sphere touched a wall sphere
    g.close()


def test_graph_replay_bitwise(env):
    import torch
    S, O = env
    box, pos, rad, member = _config()
    print("\n[walls] graphs vs plain launches, 20 steps", flush=True)
    out = []
    for graphs in (False, True):
        p = S.make_params(box, radius=rad, pos=pos, precision=S.FP32, wall=member, boundary=1,
                          shear_kind=2, g0_I=0.05, period=200, ncyc_I=1, ncyc_F=1)
        if graphs:
            g = S.Simulation(p, stream=torch.cuda.Stream())
            g.use_graphs(5)
        else:
            g = S.Simulation(p)
        g.step(20)
        out.append((g.wall_force(), g.get_particles()[0], g.get_populations()))
        g.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_walled_suspension_128_fp32(env):
    # a 128^3 suspension between walls of spheres (the measured workload's kind), FP32,
    # two steps from creation on both sides
    S, O = env
    from paper_1904_02929_amd import synth
    w = synth.walled3d(128, 0.50, 1e-3, seed=2)
    print("\n[walls] %s: %d spheres (%d in walls)" % (w.box, w.n, (w.wall > 0).sum()), flush=True)
    kw = dict(w.params)
    o = O.Oracle(O.make_params(lx=w.box[0], ly=w.box[1], lz=w.box[2], **kw), w.pos, w.vel, w.omega,
                 w.radius, wall=w.wall)
    p = S.make_params(w.box, radius=w.radius, pos=w.pos, vel=w.vel, omega=w.omega, precision=S.FP32,
                      wall=w.wall, **kw)
    g = S.Simulation(p)
    assert o.step(2) == 0
    g.step(2)
    assert np.array_equal(g.lists(S.LIST_OWNER), o.own)
    R, U, W, _ = g.get_particles()
    assert np.abs(R - o.part("R")).max() < 1e-8
    assert _rel(U, o.part("U"), 1e-6) < 1e-5 and _rel(W, o.part("W"), 1e-7) < 1e-5
    Fo, Fg = o.wall_force(), g.wall_force()
    assert _rel(Fg, Fo) < 1e-5, (Fg, Fo)
    so, _ = o.stress()
    sg, _ = g.stress()
    for k in range(5):
        assert _rel(sg[k], so[k], 1e-12) < 1e-5, k
    g.close()


@pytest.mark.parametrize("prec,tol", [(1, 1e-5), (2, 2e-3)])
def test_walls_with_multi_eigenvalue_and_contact_statistics(env, prec, tol):
    # the three added options together: walls of spheres, the multi-eigenvalue collision
    # and the contact statistics, FP32 and FP16 storage, four steps from creation
    S, O = env
    box, pos, rad, member = _config()
    vel = np.zeros_like(pos)
    vel[member == 0] = np.random.default_rng(5).uniform(-1e-3, 1e-3, (3, 3))
    kw = dict(boundary=1, shear_kind=2, g0_I=0.05, period=400, ncyc_I=1, ncyc_F=1, tau=0.8,
              collision=1, tau_bulk=0.7, tau_ghost=1.1, contact_bins=18)
    print("\n[walls] walls + multi-eigenvalue + contact statistics, precision %d" % prec, flush=True)
    o = O.Oracle(O.make_params(lx=box[0], ly=box[1], lz=box[2], **kw), pos, vel, None, rad, wall=member)
    p = S.make_params(box, radius=rad, pos=pos, vel=vel, precision=prec, wall=member, **kw)
    g = S.Simulation(p)
    assert o.step(4) == 0
    assert g.step(4, check=False) == 0
    assert np.array_equal(g.lists(S.LIST_OWNER), o.own)
    R, U, W, _ = g.get_particles()
    assert _rel(U, o.part("U"), 1e-6) < tol and _rel(W, o.part("W"), 1e-7) < tol
    assert _rel(g.wall_force(), o.wall_force()) < tol * 10
    ho, so = o.contact_stats(18)
    hg, sg = g.contact_stats(18)
    assert so[0] == sg[0] == 4 and so[1] == sg[1]
    assert np.array_equal(np.rint(ho[0] * so[1] * 4 * np.pi / 18), np.rint(hg[0] * sg[1] * 4 * np.pi / 18))
    sgo, _ = o.stress()
    sgg, _ = g.stress()
    for k in range(5):
        assert _rel(sgg[k], sgo[k], 1e-12) < tol * 10, k
    g.close()
