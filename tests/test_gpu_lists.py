"""GPU neighbour lists (Sec. 2: contacts found through a cell list) against the oracle, bit-exact,
where one sphere has far more candidates than a wave has lanes.

One sphere of radius 8 carries a shell of radius-1.5 spheres at gaps 0.3 and -0.02 (in
contact) in turn, all within the pair cutoff of 1, and 170 more small spheres are scattered
through a 64^3 box.  The cells are at least 2 a_max + cutoff wide, so the box holds three cells
per axis and every sphere sees every other one as a candidate (more than 200: four rounds of
64 lanes).  With 40 shell spheres the
lists, their ascending order and the carried spring history match the oracle's after each of
two steps; with 52 (more than the 48 slots of a list) the step reports neighbour overflow.
"""
import re
import sys

import numpy as np
import pytest

import parity_util as PU

pytestmark = pytest.mark.gpu

BOX = (64, 64, 64)


def _susp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02929_amd import susp
    susp.lib()
    return susp


def _cluster(n_shell, seed=3, n_free=170):
    c = np.array([32.0, 32.0, 32.0])
    big, a = 8.0, 1.5
    k = np.arange(n_shell) + 0.5
    th = np.arccos(1 - 2 * k / n_shell)
    ph = np.pi * (1 + 5 ** 0.5) * k
    d = big + a + np.where(k.astype(int) % 2 == 0, 0.3, -0.02)  # every other one in contact
    shell = c + d[:, None] * np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    P = np.vstack([c, shell])
    R = np.concatenate([[big], np.full(n_shell, a)])
    rng = np.random.default_rng(seed)
    while len(P) < 1 + n_shell + n_free:
        x = rng.uniform(0.0, 64.0, 3)
        dd = P - x
        dd -= 64.0 * np.rint(dd / 64.0)
        if (np.sqrt((dd ** 2).sum(1)) > R + a + 0.6).all():
            P = np.vstack([P, x])
            R = np.append(R, a)
    return P, R


def _partners(P, R, i, cutoff=1.0):
    dd = P - P[i]
    dd -= 64.0 * np.rint(dd / 64.0)
    r = np.sqrt((dd ** 2).sum(1))
    m = r < R + R[i] + cutoff
    m[i] = False
    return np.nonzero(m)[0]


def test_lists_with_many_candidates():
    susp = _susp()
    P, R = _cluster(40)
    nb = _partners(P, R, 0)
    assert 40 <= len(nb) <= 48 and len(R) > 3 * 64
    print("\n[lists] %d spheres, sphere 0 has %d partners" % (len(R), len(nb)), flush=True)
    sys.stdout.flush()
    o = PU.oracle_for(BOX, {}, P, None, None, R)
    g = PU.gpu_for(BOX, {}, P, None, None, R, 0)
    for step in range(2):
        assert o.step(1) == 0
        g.step(1)
        pi, pj = o.pairs()
        gp = g.lists(susp.LIST_PAIRS)
        assert np.array_equal(gp, np.stack([pi, pj], 1).reshape(-1, 2)), step
        assert int(((gp[:, 0] == 0) | (gp[:, 1] == 0)).sum()) == len(nb)
        hi, hj, hx = g.get_history()
        oi, oj, ox = o.history()
        assert np.array_equal(hi, oi) and np.array_equal(hj, oj)
        if len(ox):
            assert PU.rel(hx, ox) <= 1e-10
    g.close()


def test_list_overflow_is_reported():
    susp = _susp()
    P, R = _cluster(52)
    assert len(_partners(P, R, 0)) > 48
    print("\n[lists] overflow: %d spheres" % len(R), flush=True)
    g = PU.gpu_for(BOX, {}, P, None, None, R, 1)
    with pytest.raises(susp.SuspError) as ei:
        g.step(1)
    m = re.search(r"flags 0x([0-9a-f]+)", str(ei.value))
    assert ei.value.code == susp.EUNSTABLE and m and int(m.group(1), 16) & 4
    g.close()
