"""Long-run parity against the FP64 oracle's stored averages (tests/golden/longrun_*.json,
written by tests/golden/make_longrun.py, which calls the oracle only).

FP64: the library in FP64 sums the same terms as the oracle and differs only in the order of
some roundings, so where the trajectories stay together the time averages are held to the
2 % bar with no statistical allowance: the time-averaged shear stress <sigma_xy> (eq. 15, each
of its five parts, every 500-step block) of the 3D bulk suspension at phi 0.45 over 8,000 steps
(strain 2 to 8), and G', G'' (eqs. 17-18) of three monolayer packings at area fraction 0.70
over the first observation cycle of their oscillatory protocol.  At phi 0.55 (inside the 0.50-0.56 range of
the 3D configuration; 2,500 steps) and in later monolayer cycles the trajectories separate even
in FP64 (a dense sheared suspension is chaotic), and the phi 0.55 averages are compared with 2 %
plus two paired standard errors of the block differences.

FP32 (and FP16 storage for the bulk stress): the trajectories separate within the runs, so
they are compared through statistics.
Bar: |gpu - oracle| <= 2 % of |oracle| + 2 standard errors, the standard errors from block
averages (500-step blocks for the stress, one value per observation cycle for G', G'':
three cycles in each of three packings).  At strain amplitude 0.01 one cycle's G' scatters by
tens of percent between realizations, so that bar is wide for G'.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def _golden(name):
    path = os.path.join(GOLD, "longrun_%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("no stored oracle statistics (run tests/golden/make_longrun.py %s)" % name)
    with open(path) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def susp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02929_amd import susp as S
    S.lib()
    return S


def _workload(name):
    sys.path.insert(0, GOLD)
    import make_longrun  # the same workload definitions (inputs only)
    return make_longrun.workload(name)


def _mean_se(x):
    x = np.asarray(x, float)
    return float(x.mean()), float(x.std(ddof=1) / math.sqrt(len(x))) if len(x) > 1 else 0.0


def _run(S, w, plan, precision=None):
    p = S.make_params(w.box, radius=w.radius, pos=w.pos, vel=w.vel, omega=w.omega,
                      precision=S.FP32 if precision is None else precision, **w.params)
    sim = S.Simulation(p)
    sim.step(plan["start"])
    sim.stress()
    blocks, gg_after = [], []
    step = plan["start"]
    cyc = plan["cycles"]
    while step < plan["total"]:
        sim.step(plan["block"])
        step += plan["block"]
        sig, gg = sim.stress()
        blocks.append(np.asarray(sig).tolist())
        if cyc and (step - cyc[0]) % cyc[1] == 0:
            gg_after.append(np.asarray(gg).tolist())
    sim.close()
    return blocks, gg_after


def _sxy(blocks):
    return [sum(b[k][3] for k in range(5)) for b in blocks]


def _per_cycle(avg):
    """Per-cycle G', G'' from the running averages after 1, 2, ... observation cycles."""
    k = np.arange(1, len(avg) + 1, dtype=float)[:, None]
    tot = k * avg
    return np.concatenate([tot[:1], np.diff(tot, axis=0)])


@pytest.mark.parametrize("precision", ["FP32", "FP16STORE"])
def test_bulk_shear_stress(susp, precision):
    gold = _golden("bulk96")
    w, plan = _workload("bulk96")
    print("\n[longrun] bulk %s %s, %d spheres, %d steps" % (precision, w.box, len(w.radius), plan["total"]), flush=True)
    blocks, _ = _run(susp, w, plan, getattr(susp, precision))
    mo, so = _mean_se(_sxy(gold["block_stress"]))
    mg, sg = _mean_se(_sxy(blocks))
    se = math.hypot(so, sg)
    print("[longrun] <sigma_xy> oracle %.6e +- %.1e, gpu %.6e +- %.1e" % (mo, so, mg, sg), flush=True)
    assert abs(mg - mo) <= 0.02 * abs(mo) + 2 * se


# statistics over the observation cycles at area fraction 0.70.  At 0.80 (the other end of
# the monolayer configuration's range, statistics in longrun_mono256_080.json) even the FP64
# trajectories separate from the oracle's within the first cycle, and one packing's GPU runs,
# FP32 and FP64 alike, stop at the fluid mass + ledger check (the explicit-coupling
# instability) before the protocol ends, so no 0.80 case is compared.
@pytest.mark.parametrize("name, precision", [("mono256", "FP32")])
def test_monolayer_moduli(susp, name, precision):
    gold = _golden(name)
    ws = _workload(name)
    co, cg, so_, sg_ = [], [], [], []
    for (w, plan), run in zip(ws, gold["runs"]):
        print("\n[longrun] monolayer %s, %d spheres, %d steps, seed %d"
              % (w.box, len(w.radius), plan["total"], run["seed"]), flush=True)
        blocks, gg = _run(susp, w, plan, getattr(susp, precision))
        go = np.asarray(run["gg_after_cycle"])
        gg = np.asarray(gg)
        ncyc = plan["cycles"][2]
        assert go.shape == gg.shape == (ncyc, 2)
        co.append(_per_cycle(go))
        cg.append(_per_cycle(gg))
        so_ += _sxy(run["block_stress"])
        sg_ += _sxy(blocks)
    co, cg = np.concatenate(co), np.concatenate(cg)
    for k, name in enumerate(("G'", "G''")):
        mo, so = _mean_se(co[:, k])
        mg, sg = _mean_se(cg[:, k])
        se = math.hypot(so, sg)
        print("[longrun] %s oracle %.6e +- %.1e, gpu %.6e +- %.1e (%d cycles)"
              % (name, mo, so, mg, sg, len(co)), flush=True)
        assert abs(mg - mo) <= 0.02 * abs(mo) + 2 * se
    mo, _ = _mean_se(so_)
    mg, _ = _mean_se(sg_)
    print("[longrun] <sigma_xy> oracle %.6e, gpu %.6e" % (mo, mg), flush=True)


def _parts_xy(blocks):
    """Time average of sigma_xy of each of the five parts over the blocks."""
    return np.array([[b[k][3] for k in range(5)] for b in blocks]).mean(axis=0)


@pytest.mark.parametrize("name, tracks", [("bulk96", True), ("bulk96_055", False)])
def test_bulk_fp64_against_the_oracle(susp, name, tracks):
    # tracks: at phi 0.45 the FP64 trajectories stay together over the whole run (blocks
    # agree to ~1e-5), so each block and each part of eq. 15 is held to 2 %; at phi 0.55,
    # where contacts carry nearly all the stress, they separate within the run even in FP64,
    # and the time averages are compared with the paired standard error of the block
    # differences
    gold = _golden(name)
    w, plan = _workload(name)
    print("\n[longrun] %s FP64 %s, %d spheres, %d steps" % (name, w.box, len(w.radius), plan["total"]), flush=True)
    blocks, _ = _run(susp, w, plan, susp.FP64)
    so, sg = np.array(_sxy(gold["block_stress"])), np.array(_sxy(blocks))
    assert so.shape == sg.shape
    d = sg - so
    se = float(d.std(ddof=1) / math.sqrt(len(d)))
    worst = float(np.max(np.abs(d) / np.abs(so)))
    po, pg = _parts_xy(gold["block_stress"]), _parts_xy(blocks)
    print("[longrun] <sigma_xy> oracle %.9e gpu %.9e (%.2f %% apart, paired se %.2f %%); worst block %.2e relative"
          % (so.mean(), sg.mean(), 100 * abs(d.mean() / so.mean()), 100 * se / abs(so.mean()), worst), flush=True)
    print("[longrun] parts oracle %s gpu %s" % (np.array2string(po, precision=6), np.array2string(pg, precision=6)),
          flush=True)
    if tracks:
        assert abs(d.mean()) <= 0.02 * abs(so.mean())
        assert np.all(np.abs(pg - po) <= 0.02 * abs(so.mean()))
        assert worst <= 0.02
    else:
        assert abs(d.mean()) <= 0.02 * abs(so.mean()) + 2 * se


def test_monolayer_fp64_first_cycle(susp, name="mono256"):
    gold = _golden(name)
    for (w, plan), run in zip(_workload(name), gold["runs"]):
        cyc = plan["cycles"]
        first = dict(plan, total=cyc[0] + cyc[1])  # the initial cycles and one observation cycle
        print("\n[longrun] monolayer FP64 %s seed %d, %d steps" % (w.box, run["seed"], first["total"]), flush=True)
        _, gg = _run(susp, w, first, susp.FP64)
        go = np.asarray(run["gg_after_cycle"][0])
        gg = np.asarray(gg[0])
        print("[longrun] G', G'' oracle %s gpu %s" % (go, gg), flush=True)
        assert abs(gg[0] - go[0]) <= 0.02 * abs(go[0])
        assert abs(gg[1] - go[1]) <= 0.02 * abs(go[1])
