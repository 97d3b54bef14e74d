"""The allocation-free contact read-out (susp_contact_stats_noalloc) against the ordinary one
(susp_contact_stats), through the C ABI.

Two simulations start from the same state and take the same steps; one is read out through
each entry point.  The kernels are the same and deterministic, so the read-outs agree bit for
bit.  Two rounds in a row, the second with fewer bins (a smaller staging) than the first, so
that the second call runs over what the first left in the static staging.  A bin count above
the staging's limit is refused before anything runs.
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
    S.lib()
    return S


def _sims(S, nbins, seed):
    from paper_1904_02929_amd import synth
    w = synth.bulk3d(48, 0.52, 1e-3, seed=seed)
    kw = dict(w.params, contact_bins=nbins)
    # radii 1.2 % above the packing's, so that contacts exist from the start
    mk = lambda: S.Simulation(S.make_params(w.box, radius=w.radius * 1.012, pos=w.pos, vel=w.vel,
                                            omega=w.omega, precision=S.FP32, **kw))
    return mk(), mk()


@pytest.mark.parametrize("nbins,steps,seed", [(180, 3, 3), (36, 2, 5)])
def test_noalloc_matches_the_ordinary_read_out(env, nbins, steps, seed):
    S = env
    print("\n[no-alloc] %d bins, %d steps, seed %d" % (nbins, steps, seed), flush=True)
    a, b = _sims(S, nbins, seed)
    a.step(steps)
    b.step(steps)
    ha, sa = a.contact_stats(nbins)
    hb, sb = b.contact_stats_noalloc(nbins)
    a.close()
    b.close()
    assert sa[0] == sb[0] == steps and sa[1] > 20
    assert np.array_equal(ha, hb)
    assert np.array_equal(sa, sb)


def test_noalloc_refuses_more_bins_than_the_staging_holds(env):
    S = env
    a, b = _sims(S, 360, 3)
    b.close()
    a.step(1)
    with pytest.raises(Exception, match="static staging"):
        a.contact_stats_noalloc(360)
    a.close()
