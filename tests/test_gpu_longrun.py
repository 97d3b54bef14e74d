"""Long-run statistical parity: the library in FP32 against the FP64 oracle's stored averages.

The trajectories of a sheared suspension separate after enough steps, so long runs are
compared through statistics: the time-averaged shear stress <sigma_xy> (eq. 15, all five
parts) of a 3D bulk suspension under simple shear, and G', G'' (eqs. 17-18) of a monolayer
under oscillatory shear.  Bar: |gpu - oracle| <= 2 % of |oracle| + 2 standard errors, the
standard errors from block averages (500-step blocks for the stress, one value per
observation cycle for G', G'': three cycles in each of three packings).  The oracle's values are written by
tests/golden/make_longrun.py (oracle only) into tests/golden/longrun_*.json.
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


def _run(S, w, plan):
    p = S.make_params(w.box, radius=w.radius, pos=w.pos, vel=w.vel, omega=w.omega,
                      precision=S.FP32, **w.params)
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


def test_bulk_shear_stress(susp):
    gold = _golden("bulk96")
    w, plan = _workload("bulk96")
    print("\n[longrun] bulk %s, %d spheres, %d steps" % (w.box, len(w.radius), plan["total"]), flush=True)
    blocks, _ = _run(susp, w, plan)
    mo, so = _mean_se(_sxy(gold["block_stress"]))
    mg, sg = _mean_se(_sxy(blocks))
    se = math.hypot(so, sg)
    print("[longrun] <sigma_xy> oracle %.6e +- %.1e, gpu %.6e +- %.1e" % (mo, so, mg, sg), flush=True)
    assert abs(mg - mo) <= 0.02 * abs(mo) + 2 * se


def test_monolayer_moduli(susp):
    gold = _golden("mono256")
    ws = _workload("mono256")
    co, cg, so_, sg_ = [], [], [], []
    for (w, plan), run in zip(ws, gold["runs"]):
        print("\n[longrun] monolayer %s, %d spheres, %d steps, seed %d"
              % (w.box, len(w.radius), plan["total"], run["seed"]), flush=True)
        blocks, gg = _run(susp, w, plan)
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
