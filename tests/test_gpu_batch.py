"""Batches through the C ABI: jobs stepped together give the results of the same jobs
stepped alone, bit for bit; admission by footprint; slot reuse; autotuned brick shapes."""
import sys

import numpy as np
import pytest

import parity_util as PU

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def susp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02929_amd import susp as S
    S.lib()
    return S


def _jobs(S):
    out = []
    for box, phi, seed, gd in (((64, 48, 40), 0.30, 5, 1e-3), ((41, 48, 37), 0.40, 6, 5e-4),
                               ((70, 44, 33), 0.25, 8, 8e-4)):
        b, pos, vel, om, rad, kw = PU.dense_workload(box, phi, seed, gd)
        out.append((b, pos, vel, om, rad, kw))
    # an oscillatory one
    b, pos, vel, om, rad, _ = PU.dense_workload((48, 41, 36), 0.30, 9, 0.0)
    out.append((b, pos, vel, om, rad, dict(shear_kind=2, g0_I=0.004, g0_F=0.002, period=20,
                                          ncyc_I=1, ncyc_F=1, theta=0.5)))
    return out


def _params(S, job, brick=None):
    b, pos, vel, om, rad, kw = job
    kw = dict(kw)
    if brick is not None:
        kw["brick_y"], kw["brick_z"] = brick
    return S.make_params(b, radius=rad, pos=pos, vel=vel, omega=om, precision=S.FP32, **kw)


def _state(sim):
    R, U, W, Q = sim.get_particles()
    F, T, S, nl = sim.hydro()
    return [sim.get_populations(), R, U, W, Q, F, T, S, nl]


def test_batched_equals_alone(susp):
    S = susp
    jobs = _jobs(S)
    print("\n[batch] %d jobs: %s" % (len(jobs), [j[0] for j in jobs]), flush=True)
    sys.stdout.flush()
    batch = S.Batch(8, 1 << 34, autotune=True)
    slots, bricks = [], []
    for j in jobs:
        p = _params(S, j)
        bricks.append(batch.tune(p))
        slots.append(batch.add(p))
    assert None not in slots and len(set(slots)) == len(slots)
    for by, bz in bricks:
        assert (by, bz) == (0, 0) or (by % 4 == 0 and by >= 4 and bz >= 1)
    for n in (9, 4, 1):
        batch.step(n)
    got = [(_state(batch.job(s)), batch.stress(s)) for s in slots]
    for j, br, (st, (sig, gg)) in zip(jobs, bricks, got):
        alone = S.Simulation(_params(S, j, br))
        alone.step(14)
        ref = _state(alone)
        for k, (x, y) in enumerate(zip(st, ref)):
            assert np.array_equal(x, y), "box %s field %d differs" % (j[0], k)
        sig_a, gg_a = alone.stress()
        assert np.array_equal(sig, sig_a) and np.array_equal(gg, gg_a)
        alone.close()
    batch.close()


def test_batched_job_matches_oracle(susp):
    # a job stepped inside a batch (beside another job) against the oracle: one step from
    # the oracle's state at the FP32 per-step tolerance
    S = susp
    box, pos, vel, om, rad, kw = PU.dense_workload(seed=21)
    o = PU.oracle_for(box, kw, pos, vel, om, rad)
    assert o.step(20) == 0
    print("\n[batch] job vs oracle, box %s, n=%d" % (box, len(rad)), flush=True)
    batch = S.Batch(4, 1 << 33, autotune=True)
    batch.add(_params(S, _jobs(S)[1]))
    slot = batch.add(S.make_params(box, radius=rad, pos=pos, vel=vel, omega=om, precision=S.FP32, **kw))
    g = batch.job(slot)
    PU.load_oracle_state(o, g, 1)
    o.stress(); batch.stress(slot)
    batch.step(1)
    assert o.step(1) == 0
    tol = 1e-6
    assert np.array_equal(g.lists(S.LIST_OWNER), o.own)
    fluid = o.own == -1
    wr = PU.weights()[:, None]
    e_d = PU.rel(g.get_populations()[:, fluid] - wr, o.f[:, fluid] - wr)
    F, T, Sg, nl = g.hydro()
    Rg, Ug, Wg, Qg = g.get_particles()
    errs = dict(d=e_d, F=PU.rel(F, o.part("Fh"), 1e-4), T=PU.rel(T, o.part("Th"), 1e-4),
                U=PU.rel(Ug, o.part("U"), 1e-6), W=PU.rel(Wg, o.part("W"), 1e-7))
    e_R = float(np.abs(Rg - o.part("R")).max())
    print("[batch] " + " ".join("e_%s %.3e" % kv for kv in errs.items()) + " e_R %.3e" % e_R, flush=True)
    assert np.array_equal(nl, o.nlinks)
    assert max(errs.values()) <= tol and e_R <= 1e-10
    sg, _ = batch.stress(slot)
    so, _ = o.stress()
    for k in range(5):
        assert PU.rel(sg[k], so[k]) <= 1e-6
    batch.close()


def test_admission_and_slot_reuse(susp):
    S = susp
    jobs = _jobs(S)[:3]
    # the largest job first: once it leaves, its block can hold the third
    jobs.sort(key=lambda j: -S.footprint_bytes(_params(S, j)))
    fp = [S.footprint_bytes(_params(S, j)) for j in jobs]
    budget = fp[0] + fp[1]  # room for job 2 only once job 0 has left
    batch = S.Batch(3, budget, autotune=False)
    a = batch.add(_params(S, jobs[0]))
    b = batch.add(_params(S, jobs[1]))
    assert a is not None and b is not None
    assert batch.bytes_in_use() == fp[0] + fp[1]
    assert batch.add(_params(S, jobs[2])) is None  # over budget: refused, nothing changed
    assert batch.bytes_in_use() == fp[0] + fp[1]
    batch.step(3)
    batch.remove(a)
    assert batch.bytes_in_use() == fp[1]
    c = batch.add(_params(S, jobs[2]))
    assert c == a  # the freed slot is reused
    batch.step(2)
    batch.remove(b)
    batch.remove(c)
    assert batch.bytes_in_use() == 0
    batch.step(1)  # no jobs: nothing to do
    batch.close()


def test_batch_full(susp):
    S = susp
    jobs = _jobs(S)
    batch = S.Batch(1, 1 << 34, autotune=False)
    assert batch.add(_params(S, jobs[0])) == 0
    with pytest.raises(S.SuspError) as e:
        batch.add(_params(S, jobs[1]))
    assert e.value.code == S.ESTATE
    batch.close()


def test_launch_and_poll_equal_alone(susp):
    import time
    S = susp
    jobs = _jobs(S)[:3]
    batch = S.Batch(4, 1 << 34, autotune=False)
    steps = (23, 8, 15)
    slots = [batch.add(_params(S, j)) for j in jobs]
    for s, n in zip(slots, steps):
        batch.launch(s, n)
    t0 = time.time()
    left = set(slots)
    while left:
        for s in list(left):
            done, rc = batch.poll(s)
            if done:
                assert rc == S.OK
                left.discard(s)
        assert time.time() - t0 < 60.0, "jobs did not finish"
        time.sleep(0.001)
    for j, s, n in zip(jobs, slots, steps):
        alone = S.Simulation(_params(S, j))
        alone.step(n)
        for k, (x, y) in enumerate(zip(_state(batch.job(s)), _state(alone))):
            assert np.array_equal(x, y), "box %s field %d differs" % (j[0], k)
        alone.close()
    batch.close()


def test_failed_job_is_reported_alone(susp):
    # a non-finite population in one job: that job reports SUSP_EUNSTABLE, the other runs on
    # and gives the result it gives alone
    S = susp
    jobs = _jobs(S)[:2]
    print("\n[batch] one failing job of 2", flush=True)
    batch = S.Batch(4, 1 << 33, autotune=False)
    slots = [batch.add(_params(S, j)) for j in jobs]
    bad = batch.job(slots[0])
    f = bad.get_populations()
    own = bad.lists(S.LIST_OWNER).reshape(-1)
    flat = f.reshape(19, -1)
    flat[3, int(np.flatnonzero(own == -1)[100])] = np.nan
    bad.set_populations(flat.reshape(f.shape))
    for s in slots:
        batch.launch(s, 12)
    status = {}
    import time
    t0 = time.time()
    while len(status) < 2 and time.time() - t0 < 60:
        for s in slots:
            if s not in status:
                done, rc = batch.poll(s)
                if done:
                    status[s] = rc
    assert status[slots[0]] == S.EUNSTABLE and status[slots[1]] == S.OK
    got = _state(batch.job(slots[1]))
    batch.close()
    alone = S.Simulation(_params(S, jobs[1]))
    alone.step(12)
    ref = _state(alone)
    alone.close()
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def _wait(batch, slots):
    import time
    for s in slots:
        while True:
            done, rc = batch.poll(s)
            if done:
                assert rc == 0, "job in slot %d reported %d" % (s, rc)
                break
            time.sleep(0.001)


def test_lockstep_equals_alone(susp):
    # lockstep runs (one launch per kernel over all jobs): jobs of different boxes and
    # protocols, FP16-storage, FP64 and multi-eigenvalue-collision jobs (other kernel
    # sequences), a job with another brick (steps on its own stream), a job joining and one
    # leaving between runs, and an odd run
    S = susp
    jobs = _jobs(S)
    multi = dict(collision=1, tau_bulk=0.65, tau_ghost=1.25, tau=0.8)
    specs = [(jobs[0], S.FP32, None), (jobs[1], S.FP32, None), (jobs[3], S.FP32, None),
             (jobs[2], S.FP16STORE, None), (jobs[1], S.FP32, (8, 8)), (jobs[0], S.FP64, None),
             (jobs[3], S.FP64, None), ((jobs[1][:5] + ({**jobs[1][5], **multi},)), S.FP32, None)]
    late = (jobs[2], S.FP32, None)

    def params(spec):
        j, prec, brick = spec
        p = _params(S, j, brick)
        p.precision = prec
        return p

    print("\n[batch] lockstep: %d jobs + 1 late" % len(specs), flush=True)
    batch = S.Batch(12, 1 << 34, autotune=False)
    slots = [batch.add(params(sp)) for sp in specs]
    assert None not in slots
    steps = {s: 0 for s in slots}
    batch.launch_all(6)
    _wait(batch, slots)
    for s in slots:
        steps[s] += 6
    ls = batch.add(params(late))
    slots.append(ls)
    specs.append(late)
    steps[ls] = 0
    batch.launch_all(4)
    _wait(batch, slots)
    for s in slots:
        steps[s] += 4
    gone = slots[1]
    batch.remove(gone)
    keep = [(s, sp) for s, sp in zip(slots, specs) if s != gone]
    batch.launch_all(3)
    _wait(batch, [s for s, _ in keep])
    for s, _ in keep:
        steps[s] += 3
    for s, sp in keep:
        st = _state(batch.job(s))
        sig, gg = batch.stress(s)
        alone = S.Simulation(params(sp))
        alone.step(steps[s])
        ref = _state(alone)
        print("[batch] slot %d box %s precision %d brick %s: %d steps" % (s, sp[0][0], sp[1], sp[2], steps[s]),
              flush=True)
        for k, (x, y) in enumerate(zip(st, ref)):
            assert np.array_equal(x, y), "slot %d field %d differs" % (s, k)
        sig_a, gg_a = alone.stress()
        assert np.array_equal(sig, sig_a) and np.array_equal(gg, gg_a)
        alone.close()
    batch.close()


def test_lockstep_long_run_equals_alone(susp):
    # a lockstep run longer than one clock table (two uploads, the second after the first
    # part has run), issued directly after the jobs changed and then replayed from the
    # recorded pair; then a run of the same jobs again (replay only)
    S = susp
    jobs = [PU.dense_workload(box, phi, seed, gd)
            for box, phi, seed, gd in (((44, 42, 40), 0.15, 31, 5e-4), ((36, 44, 41), 0.12, 32, 4e-4))]
    print("\n[batch] lockstep long run: 2 jobs, 4100 + 4 steps", flush=True)
    batch = S.Batch(4, 1 << 33, autotune=False)
    slots = [batch.add(_params(S, j)) for j in jobs]
    assert None not in slots
    batch.launch_all(4100)
    _wait(batch, slots)
    batch.launch_all(4)
    _wait(batch, slots)
    for s, j in zip(slots, jobs):
        alone = S.Simulation(_params(S, j))
        alone.step(4104)
        st, ref = _state(batch.job(s)), _state(alone)
        for k, (x, y) in enumerate(zip(st, ref)):
            assert np.array_equal(x, y), "slot %d field %d differs" % (s, k)
        alone.close()
    batch.close()


def test_lockstep_job_matches_oracle(susp):
    # a job stepped in lockstep beside another job, against the oracle: two steps from the
    # oracle's state at the FP32 per-step tolerance
    S = susp
    box, pos, vel, om, rad, kw = PU.dense_workload(seed=21)
    o = PU.oracle_for(box, kw, pos, vel, om, rad)
    assert o.step(20) == 0
    print("\n[batch] lockstep job vs oracle, box %s, n=%d" % (box, len(rad)), flush=True)
    batch = S.Batch(4, 1 << 33, autotune=False)
    other = batch.add(_params(S, _jobs(S)[1]))
    slot = batch.add(S.make_params(box, radius=rad, pos=pos, vel=vel, omega=om, precision=S.FP32, **kw))
    g = batch.job(slot)
    PU.load_oracle_state(o, g, 1)
    o.stress(); batch.stress(slot)
    batch.launch_all(2)
    _wait(batch, [other, slot])
    assert o.step(2) == 0
    tol = 1e-6
    assert np.array_equal(g.lists(S.LIST_OWNER), o.own)
    fluid = o.own == -1
    wr = PU.weights()[:, None]
    e_d = PU.rel(g.get_populations()[:, fluid] - wr, o.f[:, fluid] - wr)
    F, T, Sg, nl = g.hydro()
    Rg, Ug, Wg, Qg = g.get_particles()
    errs = dict(d=e_d, F=PU.rel(F, o.part("Fh"), 1e-4), T=PU.rel(T, o.part("Th"), 1e-4),
                U=PU.rel(Ug, o.part("U"), 1e-6), W=PU.rel(Wg, o.part("W"), 1e-7))
    e_R = float(np.abs(Rg - o.part("R")).max())
    print("[batch] " + " ".join("e_%s %.3e" % kv for kv in errs.items()) + " e_R %.3e" % e_R, flush=True)
    assert np.array_equal(nl, o.nlinks)
    # positions: the one-step bound (1e-10 lattice units) for each of the two steps, plus the
    # first step's velocity error carried through the second step's displacement
    assert max(errs.values()) <= tol and e_R <= 3e-10
    sg, _ = batch.stress(slot)
    so, _ = o.stress()
    for k in range(5):
        assert PU.rel(sg[k], so[k]) <= 1e-6
    batch.close()
