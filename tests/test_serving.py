"""The continuous-batching server: every request's result equals the result
of the same request run alone, whatever else was on the GPU with it.

Requests of mixed shape classes arrive at staggered times, under an HBM budget
and a slot limit that force queueing and joining mid-run, with iteration
counts that do not line up with the server's chunks.  Alone and in the mix the
kernels do the same per-request arithmetic in the same order, so the
separated spectra and log-likelihood must be identical.
"""

import numpy as np
import pytest

from paper_1903_03237_amd import synth

pytestmark = pytest.mark.gpu

# (M, N, K, T, iters, arrival s)
SPECS = [
    (2, 2, 8, 120, 12, 0.00),
    (4, 3, 16, 90, 7, 0.00),
    (8, 5, 32, 64, 12, 0.00),
    (2, 2, 8, 200, 9, 0.02),
    (8, 4, 32, 150, 12, 0.03),
    (4, 2, 8, 50, 5, 0.05),
    (2, 3, 16, 300, 12, 0.05),
]
F = 40


def _requests():
    from paper_1903_03237_amd import serve

    reqs = []
    for i, (M, N, K, T, iters, t) in enumerate(SPECS):
        X, init, delta = synth.random_problem(F, T, M, N, K, seed=3000 + i, delta_rel=1e-8, random_q=True)
        reqs.append(serve.Request(i, t, X, N, K, init, delta, iters))
    return reqs


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_served_equals_alone(device, precision):
    from paper_1903_03237_amd import fmnmf, serve

    reqs = _requests()
    fps = sorted(serve.footprint(r, precision) for r in reqs)
    srv = serve.Server(precision=precision, hbm_budget=sum(fps[-3:]), max_active=4, chunk=5,
                       device=device, keep_outputs=True)
    got = srv.run(reqs)
    assert [r.rid for r in got] == list(range(len(reqs)))
    for r in got:
        assert r.admitted >= r.arrival - 1e-6 and r.finished >= r.admitted
    alone = serve.run_sequential(reqs, precision=precision, device=device, keep_outputs=True)
    for g, a in zip(got, alone):
        assert g.loglik == a.loglik, (g.rid, g.loglik, a.loglik)
        np.testing.assert_array_equal(g.Y.cpu().numpy(), a.Y.cpu().numpy())
    s = serve.summary(got, reqs)
    assert s["requests"] == len(reqs) and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_request_over_budget_is_rejected(device):
    from paper_1903_03237_amd import serve

    reqs = _requests()[:1]
    with pytest.raises(ValueError):
        serve.Server(hbm_budget=1024, device=device).run(reqs)


def test_faulting_request_retires_while_others_match_alone(device):
    """A request whose mixture holds a NaN latches a numerical fault in its own
    context (a non-finite likelihood, and from the first IP update on a
    singular system, which is reported first); the server retires it with
    that code and the other requests, batched with it, still equal the same
    requests run alone."""
    from paper_1903_03237_amd import fmnmf, serve

    reqs = _requests()[:5]
    bad = reqs[2]
    Xb = bad.X.copy()
    Xb[3, 7, 1] = complex(np.nan, 0.0)
    reqs[2] = serve.Request(bad.rid, bad.arrival, Xb, bad.N, bad.K, bad.init, bad.delta, bad.iters)
    srv = serve.Server(precision="bf16", hbm_budget=1 << 34, max_active=8, chunk=4, device=device,
                       keep_outputs=True)
    got = srv.run(reqs)
    assert got[2].error in (fmnmf.E_NONFINITE, fmnmf.E_SINGULAR) and got[2].Y is None
    good = [r for i, r in enumerate(reqs) if i != 2]
    alone = serve.run_sequential(good, precision="bf16", device=device, keep_outputs=True)
    for g, a in zip([r for r in got if r.rid != 2], alone):
        assert g.error == 0 and g.loglik == a.loglik
        np.testing.assert_array_equal(g.Y.cpu().numpy(), a.Y.cpu().numpy())
