"""Failure detection and checkpoints through the C ABI.

* A non-finite population put in from the host (susp_set_populations) makes the next step
  return SUSP_EUNSTABLE with the fluid flag (32); a healthy run reports no fast node-steps
  and a mass drift at rounding level (susp_health).
* A checkpoint -- clock, particles, spring history, populations and the running sums
  (stress sums, G', G'' quadrature, mass ledger) -- loaded into a fresh simulation continues
  the run bit for bit in FP32.  In FP64 the populations cross the ABI as n = d + w_q rho0
  (the stored deviation d plus the rest weight), a sum that rounds d by up to 2^-53 w_q rho0;
  the continued run then agrees to 1e-12 relative.
"""
import re

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


def test_nonfinite_population_is_reported(susp):
    S = susp
    box, pos, vel, om, rad, kw = PU.dense_workload(seed=11)
    print("\n[state] NaN population, box %s, %d spheres" % (box, len(rad)), flush=True)
    g = PU.gpu_for(box, kw, pos, vel, om, rad, S.FP32)
    g.step(3)
    fast, umax, drift = g.health()
    assert fast == 0 and umax == 0.0 and abs(drift) < 1e-6
    f = g.get_populations()
    own = g.lists(S.LIST_OWNER)
    fluid = np.flatnonzero(own.reshape(-1) == -1)
    node = int(fluid[len(fluid) // 2])
    flat = f.reshape(19, -1)
    flat[7, node] = np.nan
    g.set_populations(flat.reshape(f.shape))
    with pytest.raises(S.SuspError) as ei:
        g.step(1)
    assert ei.value.code == S.EUNSTABLE
    m = re.search(r"flags 0x([0-9a-f]+)", str(ei.value))
    assert m and int(m.group(1), 16) & 32
    g.close()


def _snapshot(g):
    return dict(clock=g.clock()[0], particles=g.get_particles(), history=g.get_history(),
                populations=g.get_populations(), acc=g.get_accumulators())


def _load(g, st):
    g.set_clock(st["clock"])
    g.set_particles(*st["particles"])
    g.set_populations(st["populations"])
    g.set_history(*st["history"])
    g.set_accumulators(st["acc"])


@pytest.mark.parametrize("prec", [0, 1])
def test_checkpoint_continues_the_run_bitwise(susp, prec):
    S = susp
    # oscillatory shear, so that the G', G'' quadrature runs through the checkpoint
    box, pos, vel, om, rad, _ = PU.dense_workload((48, 41, 36), 0.35, 9, 0.0)
    kw = dict(shear_kind=2, g0_I=0.004, g0_F=0.002, period=20, ncyc_I=1, ncyc_F=2, theta=0.5)
    print("\n[state] checkpoint, precision %d, box %s, %d spheres" % (prec, box, len(rad)), flush=True)
    a = PU.gpu_for(box, kw, pos, vel, om, rad, prec)
    a.step(23)
    st = _snapshot(a)
    a.step(17)
    b = PU.gpu_for(box, kw, pos, vel, om, rad, prec)
    _load(b, st)
    b.step(17)
    ra, rb = _snapshot(a), _snapshot(b)
    assert ra["clock"] == rb["clock"] == 40
    sa, ga = a.stress()
    sb, gb = b.stress()
    if prec == 1:
        same = np.array_equal
    else:
        def same(x, y):
            x, y = np.asarray(x, float), np.asarray(y, float)
            return np.abs(x - y).max(initial=0.0) <= 1e-12 * max(np.abs(x).max(initial=0.0), 1e-300)
    for x, y in zip(ra["particles"], rb["particles"]):
        assert same(x, y)
    assert same(ra["populations"], rb["populations"])
    assert np.array_equal(ra["history"][0], rb["history"][0])
    assert np.array_equal(ra["history"][1], rb["history"][1])
    assert same(ra["history"][2], rb["history"][2])
    assert same(ra["acc"], rb["acc"])
    assert same(sa, sb) and same(ga, gb)
    a.close()
    b.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_whole_state_checkpoint_is_bitwise(susp, prec):
    # susp_get_state / susp_set_state: the populations travel as stored, so the continued run
    # is bit for bit the same in every precision, FP64 included
    S = susp
    box, pos, vel, om, rad, _ = PU.dense_workload((48, 41, 36), 0.35, 9, 0.0)
    kw = dict(shear_kind=2, g0_I=0.004, g0_F=0.002, period=20, ncyc_I=1, ncyc_F=2, theta=0.5)
    print("\n[state] whole-state checkpoint, precision %d, box %s, %d spheres" % (prec, box, len(rad)), flush=True)
    a = PU.gpu_for(box, kw, pos, vel, om, rad, prec)
    a.step(23)
    st = a.get_state()
    a.step(17)
    b = PU.gpu_for(box, kw, pos, vel, om, rad, prec)
    b.set_state(st)
    b.step(17)
    ra, rb = _snapshot(a), _snapshot(b)
    assert ra["clock"] == rb["clock"] == 40
    for x, y in zip(ra["particles"], rb["particles"]):
        assert np.array_equal(x, y)
    assert np.array_equal(ra["populations"], rb["populations"])
    for x, y in zip(ra["history"], rb["history"]):
        assert np.array_equal(x, y)
    assert np.array_equal(ra["acc"], rb["acc"])
    sa, ga = a.stress()
    sb, gb = b.stress()
    assert np.array_equal(sa, sb) and np.array_equal(ga, gb)
    assert a.get_state() == b.get_state()
    # a state of another box is refused and changes nothing
    c = PU.gpu_for((48, 41, 40), kw, pos, vel, om, rad, prec)  # the same spheres, a taller box
    before = c.get_state()
    with pytest.raises(S.SuspError) as ei:
        c.set_state(st)
    assert ei.value.code == S.ESTATE
    assert c.get_state() == before
    for g in (a, b, c):
        g.close()
