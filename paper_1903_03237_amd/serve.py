"""Continuous-batching FastMNMF server on one GPU.

Requests (mixtures of different M, N, K and T) arrive over time.  The server

* admits requests first come, first served (or least work first, order
  "sjf"), as soon as a slot is free, its
  HBM footprint (fmnmf_footprint_bytes: mixture, workspace and separated
  output) fits the budget and the admitted work (time-frequency bins) stays
  near what fills the GPU, and keeps its mixture and parameters resident;
* advances all admitted requests together with fmnmf_step_batch: every
  kernel of an iteration runs once per shape class for all requests of that
  class, from a HIP graph captured per composition;
* lets requests that arrive while others run join at the next chunk
  boundary, and separates finished requests (Wiener filter) on their own
  streams while the next chunk of the others runs;
* retires a request whose context latched a numerical fault (a singular IP
  system, a non-finite likelihood) with that error code, while the others
  continue: every context's arithmetic and status word are its own.

`run_sequential` serves the same requests one at a time with fmnmf_step, the
baseline the batched server is compared with.
"""

from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import fmnmf


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float   # seconds after the start of the run
    X: object        # [F, T, M] complex: host array, or a tensor already on the device
    N: int
    K: int
    init: tuple      # (W0, H0, G0, Q0)
    delta: float
    iters: int


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    loglik: float
    Y: object = None  # separated images [N, F, T, M] (device tensor) when kept
    error: int = 0    # 0, or the FMNMF_E_* code the request was retired with
    message: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class _Slot:
    req: Request
    model: object
    out: object
    admitted: float
    done: int = 0


def _device_mixture(X, precision: str, device):
    """A contiguous device copy of a request's mixture in the path's type."""
    import torch

    if isinstance(X, np.ndarray):
        dt = np.complex128 if precision == "fp64" else np.complex64
        return torch.from_numpy(np.ascontiguousarray(X.astype(dt))).to(device)
    tdt = torch.complex128 if precision == "fp64" else torch.complex64
    return X.to(device=device, dtype=tdt).contiguous()


def footprint(req: Request, precision: str) -> int:
    F, T, M = req.X.shape
    return fmnmf.footprint_bytes(fmnmf.make_dims(F, T, M, req.N, req.K, precision, req.delta))


class Server:
    def __init__(self, precision: str = "bf16", hbm_budget: int = 64 << 30, max_active: int = 64,
                 max_bins: int = 1_000_000, chunk: int = 10, device: str = "cuda:0",
                 keep_outputs: bool = False, order: str = "fcfs"):
        """hbm_budget: bytes of device memory the admitted requests may hold;
        max_active: slots; max_bins: time-frequency bins (sum of F*T) admitted
        together per waiting request, about what fills the GPU: with one
        request waiting the admitted work stays near max_bins (a larger
        request runs alone), a backlog of b waiting requests allows b times
        as much.  order: which arrived request is admitted next, "fcfs"
        (first come, first served) or "sjf" (the least work, F*T*iters,
        first; ties by arrival)."""
        if order not in ("fcfs", "sjf"):
            raise ValueError(f"unknown admission order {order!r}")
        self.order = order
        self.precision = precision
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.max_bins = int(max_bins)
        self.chunk = int(chunk)
        self.device = device
        self.keep = keep_outputs

    def _admit(self, req: Request, now: float) -> _Slot:
        import torch

        tdt = torch.complex128 if self.precision == "fp64" else torch.complex64
        X = _device_mixture(req.X, self.precision, self.device)
        F, T, M = req.X.shape
        out = torch.empty((req.N, F, T, M), dtype=tdt, device=self.device)
        model = fmnmf.FastMNMF(X, req.N, req.K, req.init, precision=self.precision, delta=req.delta)
        return _Slot(req, model, out, now)

    def run(self, requests) -> list[Result]:
        """Serve `requests` (their arrival times are relative to the call).

        Up to two chunks are in flight: while the GPU runs them, the host
        waits for the older one, admits new arrivals (they join the next
        chunk) and separates the requests that chunk finished."""
        import collections

        import torch

        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            if footprint(r, self.precision) > self.budget:
                raise ValueError(f"request {r.rid} alone exceeds the HBM budget")
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        pi, used = 0, 0
        active: list[_Slot] = []      # admitted and not finished
        planned: dict[int, int] = {}  # rid -> iterations enqueued so far
        inflight = collections.deque()  # (event, slots, n)
        results: list[Result] = []

        bins = lambda r: r.X.shape[0] * r.X.shape[1]  # noqa: E731

        arrived: list[Request] = []  # arrived and not admitted, in arrival order
        work = lambda r: (bins(r) * r.iters, r.arrival, r.rid)  # noqa: E731

        def admit():
            nonlocal pi, used
            now = clock()
            while pi < len(pending) and pending[pi].arrival <= now:
                arrived.append(pending[pi])
                pi += 1
            while arrived and len(active) < self.max_active:
                j = 0 if self.order == "fcfs" else min(range(len(arrived)), key=lambda i: work(arrived[i]))
                r = arrived[j]
                fp = footprint(r, self.precision)
                load = sum(bins(s.req) for s in active)
                # work cap, raised by the backlog of arrived requests still waiting
                cap = self.max_bins * len(arrived)
                if used + fp > self.budget or (active and load + bins(r) > cap):
                    break
                arrived.pop(j)
                s = self._admit(r, clock())
                active.append(s)
                planned[s.req.rid] = 0
                used += fp
                if s.req.iters == 0:  # nothing to iterate: the filter of its initial state
                    retire(s)

        def retire(s, err=None):
            """Separate a finished request (or record its error) and free its slot."""
            nonlocal used
            active.remove(s)
            code, msg, ll = 0, "", float("nan")
            try:
                if err is not None:
                    raise err
                s.model.separate(out=s.out)  # on its own stream
                ll = s.model.loglik()
            except fmnmf.FmnmfError as e:  # a numerical fault of this request only
                code, msg = e.code, str(e)
            results.append(Result(s.req.rid, s.req.arrival, s.admitted, clock(), ll,
                                  s.out if (self.keep and code == 0) else None, code, msg))
            used -= footprint(s.req, self.precision)
            planned.pop(s.req.rid, None)
            s.model.close()

        def enqueue():
            comp = [s for s in active if planned[s.req.rid] < s.req.iters]
            if not comp:
                return False
            n = min(self.chunk, min(s.req.iters - planned[s.req.rid] for s in comp))
            try:
                fmnmf.step_batch([s.model for s in comp], n)
            except fmnmf.FmnmfError as e:  # a launch failed: retire the batch's requests
                for s in comp:
                    retire(s, e)
                return True
            ev = torch.cuda.Event()
            ev.record(comp[0].model.stream)
            for s in comp:
                planned[s.req.rid] += n
            inflight.append((ev, comp, n))
            return True

        while pi < len(pending) or arrived or active:
            admit()
            while len(inflight) < 2 and enqueue():
                pass
            if not inflight:
                if pi < len(pending):
                    wait = pending[pi].arrival - clock()
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            ev, comp, n = inflight.popleft()
            ev.synchronize()
            for s in comp:
                s.done += n
            # refill before the host-side work below
            admit()
            while len(inflight) < 2 and enqueue():
                pass
            done = [s for s in comp if s.done >= s.req.iters and s in active]
            for s in done:
                retire(s)
        return sorted(results, key=lambda r: r.rid)


def run_sequential(requests, precision: str = "bf16", device: str = "cuda:0",
                   keep_outputs: bool = False) -> list[Result]:
    """The same requests served one at a time, in arrival order (fmnmf_step)."""
    import torch

    tdt = torch.complex128 if precision == "fp64" else torch.complex64
    t0 = time.perf_counter()
    results = []
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        wait = r.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        adm = time.perf_counter() - t0
        X = _device_mixture(r.X, precision, device)
        F, T, M = r.X.shape
        out = torch.empty((r.N, F, T, M), dtype=tdt, device=device)
        m = fmnmf.FastMNMF(X, r.N, r.K, r.init, precision=precision, delta=r.delta)
        code, msg, ll = 0, "", float("nan")
        try:
            m.step(r.iters)
            m.separate(out=out)
            ll = m.loglik()
        except fmnmf.FmnmfError as e:
            code, msg = e.code, str(e)
        results.append(Result(r.rid, r.arrival, adm, time.perf_counter() - t0, ll,
                              out if (keep_outputs and code == 0) else None, code, msg))
        m.close()
    return sorted(results, key=lambda r: r.rid)


def summary(results, requests) -> dict:
    """p50 / p99 latency, makespan and throughput (TF-bins/s and iters/s)."""
    lat = np.array([r.latency for r in results])
    by = {q.rid: q for q in requests}
    work = sum(by[r.rid].X.shape[0] * by[r.rid].X.shape[1] * by[r.rid].iters for r in results)
    iters = sum(by[r.rid].iters for r in results)
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    return {"requests": len(results), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "makespan_s": float(span),
            "tf_bins_per_s": work / span, "iters_per_s": iters / span, "requests_per_s": len(results) / span}
