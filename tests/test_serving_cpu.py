"""The serving loop's scheduling on the CPU, with the library replaced by a
stand-in that only counts iterations: admission by slots and HBM budget,
requests that need no iteration, and a request whose context latches a
numerical fault being retired with that code while the others finish."""

import numpy as np
import pytest

from paper_1903_03237_amd import fmnmf, serve


class _Ev:
    def record(self, stream):
        pass

    def synchronize(self):
        pass


class _Model:
    live = 0
    peak = 0

    def __init__(self, X, N, K, init, precision="bf16", delta=0.0, **kw):
        self.X, self.N, self.K, self.done, self.stream = X, N, K, 0, None
        self.bad = bool(np.isnan(np.asarray(X)).any())
        _Model.live += 1
        _Model.peak = max(_Model.peak, _Model.live)

    def separate(self, out=None):
        if self.bad:
            raise fmnmf.FmnmfError(fmnmf.E_NONFINITE, "the log-likelihood is not finite")
        return out

    def loglik(self):
        if self.bad:
            raise fmnmf.FmnmfError(fmnmf.E_NONFINITE, "the log-likelihood is not finite")
        return float(-self.done)

    def close(self):
        _Model.live -= 1


@pytest.fixture
def fake(monkeypatch):
    import torch

    _Model.live = _Model.peak = 0
    monkeypatch.setattr(serve.fmnmf, "FastMNMF", _Model)
    monkeypatch.setattr(serve.fmnmf, "step_batch", lambda models, n: [setattr(m, "done", m.done + n) for m in models])
    monkeypatch.setattr(serve, "footprint", lambda req, precision: 100)
    monkeypatch.setattr(torch.cuda, "Event", _Ev)
    return _Model


def _req(rid, iters, T=8, bad=False, arrival=0.0):
    X = np.zeros((4, T, 2), dtype=np.complex64)
    if bad:
        X[1, 2, 0] = np.nan
    return serve.Request(rid, arrival, X, 2, 3, None, 0.0, iters)


def test_every_request_gets_its_iterations(fake):
    reqs = [_req(i, iters) for i, iters in enumerate([7, 30, 1, 12, 25])]
    srv = serve.Server(precision="fp32", hbm_budget=10_000, max_active=3, chunk=5, device="cpu", max_bins=10**9)
    res = srv.run(reqs)
    assert [r.rid for r in res] == list(range(5))
    assert [r.loglik for r in res] == [-7.0, -30.0, -1.0, -12.0, -25.0]
    assert all(r.error == 0 for r in res)
    assert fake.peak <= 3 and fake.live == 0


def test_zero_iterations_is_retired_at_admission(fake):
    reqs = [_req(0, 0), _req(1, 4), _req(2, 0, arrival=0.01)]
    srv = serve.Server(precision="fp32", hbm_budget=10_000, max_active=4, chunk=2, device="cpu", max_bins=10**9)
    res = srv.run(reqs)  # must terminate
    assert [r.loglik for r in res] == [0.0, -4.0, 0.0]
    assert fake.live == 0


def test_a_faulting_request_is_retired_with_its_code(fake):
    reqs = [_req(0, 6), _req(1, 6, bad=True), _req(2, 9), _req(3, 3, bad=True, arrival=0.005)]
    srv = serve.Server(precision="fp32", hbm_budget=10_000, max_active=8, chunk=4, device="cpu", max_bins=10**9)
    res = srv.run(reqs)
    assert [r.error for r in res] == [0, fmnmf.E_NONFINITE, 0, fmnmf.E_NONFINITE]
    assert res[0].loglik == -6.0 and res[2].loglik == -9.0
    assert "not finite" in res[1].message and np.isnan(res[1].loglik)
    assert fake.live == 0


def test_budget_limits_the_admitted_footprint(fake):
    reqs = [_req(i, 10) for i in range(6)]
    srv = serve.Server(precision="fp32", hbm_budget=250, max_active=16, chunk=3, device="cpu", max_bins=10**9)
    res = srv.run(reqs)
    assert fake.peak == 2  # 100 bytes each, budget 250
    assert all(r.loglik == -10.0 for r in res)


def test_sjf_admits_the_least_work_first(fake):
    """With one slot, requests that have all arrived are admitted least work
    (F*T*iters) first under "sjf" and in arrival order under "fcfs"."""
    reqs = [_req(0, 9), _req(1, 3), _req(2, 6), _req(3, 1)]

    def admitted_order(order):
        srv = serve.Server(precision="fp32", hbm_budget=10_000, max_active=1, chunk=2, device="cpu",
                           max_bins=10**9, order=order)
        res = srv.run(reqs)
        assert all(r.error == 0 for r in res)
        return [r.rid for r in sorted(res, key=lambda r: r.admitted)]

    assert admitted_order("fcfs") == [0, 1, 2, 3]
    assert admitted_order("sjf") == [3, 1, 2, 0]
    with pytest.raises(ValueError):
        serve.Server(order="lifo")
