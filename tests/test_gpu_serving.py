"""The serving loop on the GPU: small requests of both kinds arrive as a Poisson process, are
served in lockstep runs (one launch per kernel over all admitted jobs) with admission by
footprint against a budget that holds only some of them at once, and every served result
(stress, G', G'', positions) equals the same request run alone, bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def susp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02929_amd import susp as S
    S.lib()
    return S


def test_lockstep_server_results_equal_alone(susp):
    from paper_1904_02929_amd import serve
    specs = []
    for k in range(8):
        if k % 2 == 0:  # monolayer, oscillatory shear over a short period
            specs.append(serve.JobSpec(k, "2d", 64 + 16 * (k % 3), 0.70 + 0.02 * k, 100 + k, 120,
                                       g0=0.01, theta=0.4 * k, period=40))
        else:           # 3D bulk, simple shear
            specs.append(serve.JobSpec(k, "3d", 48 + 8 * (k % 3), 0.40 + 0.01 * k, 200 + k, 120,
                                       gamma_dot=2e-4 * k))
    ws = serve.build_workloads(specs, workers=1)
    fps = [susp.footprint_bytes(serve.job_params(s, ws[s.jid])) for s in specs]
    budget = int(sum(sorted(fps)[-3:]) * 1.05)  # about three jobs at a time
    arr = serve.poisson_arrivals(len(specs), 40.0, seed=7)
    for s, a in zip(specs, arr):
        s.arrival = float(a)
    print("\n[serving] %d requests, budget %.1f MB, boxes %s" % (len(specs), budget / 1e6,
          [ws[s.jid].box for s in specs]), flush=True)
    ex = serve.BatchExecutor(ws, budget, max_jobs=len(specs), autotune=False)
    srv = serve.LockstepServer(ex, budget, chunk=30)
    done = srv.run(specs)
    ex.close()
    assert sorted(d.jid for d in done) == list(range(len(specs)))
    assert max(n for _, n in srv.log) > 1  # jobs shared runs
    assert max(n for _, n in srv.log) < len(specs)  # and the budget held some back
    for d in done:
        assert d.status == 0 and d.result is not None
        s = specs[d.jid]
        _, alone = serve.run_alone(s, ws[s.jid])
        for a, b in zip(d.result, alone):
            assert np.array_equal(np.asarray(a), np.asarray(b)), "request %d differs from its run alone" % d.jid
    print("[serving] %d runs, all %d results identical alone" % (len(srv.runs), len(done)), flush=True)
