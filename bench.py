#!/usr/bin/env python3
"""FastMNMF benchmark on one MI355X.

Workload: the headline shape, M=8 microphones, F=513 bins (1024-point STFT),
T=3000 frames, N=5 sources, K=32 bases, synthetic NMF-structured mixture with
-5 dB diffuse noise, model floor delta = 1e-8 mean|x|^2.  A "step" is one full
iteration (W, H, G~ updates, V_fm + IP update of Q, projection and
log-likelihood); the timed region is exactly --steps steps followed by the
final multichannel Wiener filter, with the mixture already resident in HBM.

The headline path is the mixed-precision one (bf16 MFMA operands for the NMF
contractions, FP32 bulk, FP64 IP solve / normalisation / log-det); the FP32
and plain FP64 paths are timed on the same workload for the speedup.  The
FP64 CPU oracle is timed on a bounded sample (a few iterations) as the
cpu_baseline.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FastMNMF iters/s at M=8,F=513,T=3000 (mixed vs FP64); served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
VALU_FP32_TFLOPS = 157.3
VALU_FP64_TFLOPS = 78.6


def kernel_model(F, T, M, N, K, rb):
    """Algorithmic bytes and flops per launch of each iteration kernel.

    Bytes are what the method must move (x~ or X in, x~ out), not partial sums
    or re-reads; flops count the arithmetic the kernel's formulas need;
    mfma_flops the part of it that is the NMF contractions (lambda = W H and,
    in the W and H passes, the numerator / denominator sums of Eqs. 23-24)."""
    FT = F * T
    cb = 2 * rb
    return {
        "wpass": {"bytes": FT * M * rb, "flops": FT * (6 * N * K + 6 * N * M), "mfma_flops": FT * 6 * N * K,
                  "bound": "hbm"},
        "hpass": {"bytes": FT * M * rb, "flops": FT * (6 * N * K + 6 * N * M), "mfma_flops": FT * 6 * N * K,
                  "bound": "hbm"},
        "gpass": {"bytes": FT * M * rb, "flops": FT * (2 * N * K + 6 * N * M), "mfma_flops": FT * 2 * N * K,
                  "bound": "hbm"},
        "vpass": {"bytes": FT * M * cb, "flops": FT * (M * M * (4 + 2 * M) + 2 * N * K), "bound": "hbm"},
        "proj": {"bytes": FT * M * (cb + rb), "flops": FT * (8 * M * M + 2 * N * K + 5 * M), "bound": "hbm"},
    }


def iteration_bytes(F, T, M, rb):
    """Algorithmic HBM bytes of one iteration: x~ read by the W, H and G~
    passes and written by the projection, X read by the V pass and the
    projection: F T M (4 b_r + 2 b_c)."""
    return F * T * M * (4 * rb + 2 * 2 * rb)


def wiener_bytes(F, T, M, N, rb):
    """The filter reads X and writes N images: F T M b_c (1 + N)."""
    return F * T * M * 2 * rb * (1 + N)


MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}


def roofline_table(kms, F, T, M, N, K, precision, wiener_ms=None):
    """Per-kernel achieved rates from mean launch times (ms): algorithmic
    GB/s and the fraction of the 8 TB/s HBM peak; for the NMF contractions
    also the MFMA rate against the dense peak of the path's operand type and
    the ceiling that the x~ stream (HBM at peak) puts on it."""
    rb = 8 if precision == "fp64" else 4
    km = kernel_model(F, T, M, N, K, rb)
    out = {}
    for k, d in km.items():
        if not kms.get(k):
            continue
        sec = kms[k] * 1e-3
        e = {"ms": round(kms[k], 5), "algorithmic_bytes": d["bytes"],
             "hbm_gbs": d["bytes"] / sec / 1e9, "hbm_frac": d["bytes"] / sec / 1e9 / HBM_PEAK_GBS}
        if "mfma_flops" in d:
            peak = MFMA_PEAK_TFLOPS[precision]
            e["mfma_tflops"] = d["mfma_flops"] / sec / 1e12
            e["mfma_frac"] = e["mfma_tflops"] / peak
            # at most this fraction of the MFMA peak while x~ streams at the HBM peak
            e["mfma_ceiling_frac"] = min(1.0, d["mfma_flops"] / (d["bytes"] / (HBM_PEAK_GBS * 1e9)) / 1e12 / peak)
        out[k] = e
    if wiener_ms:
        b = wiener_bytes(F, T, M, N, rb)
        out["wiener"] = {"ms": round(wiener_ms, 5), "algorithmic_bytes": b, "hbm_gbs": b / (wiener_ms * 1e-3) / 1e9,
                         "hbm_frac": b / (wiener_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


# Source files that define each kernel and its launch shape.
KERNEL_SOURCES = {
    "wpass": "nmf_passes.inc", "hpass": "nmf_passes.inc", "gpass": "nmf_passes.inc",
    "vpass": "spatial.inc", "proj": "spatial.inc", "wiener": "spatial.inc", "ip": "small.inc",
    "lampass": "nmf_passes.inc",
}
COMMON_SOURCES = ["kern_common.h", "kargs.h", "launch.inc", "fmnmf.cpp"]


def kernel_sources_digest(kernel):
    """SHA-256 over the HIP sources that define `kernel` and its launch."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1903_03237_amd", "csrc")
    for name in [KERNEL_SOURCES[kernel], *COMMON_SOURCES]:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel, precision):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, scaled by the copy-kernel calibration; None
    when there is none for this kernel and path or the kernel's sources have
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_fp32_m8_513x3000.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get("kernels", {}).get(f"{kernel}/{precision}")
    if not e or e.get("sources_sha256") != kernel_sources_digest(kernel):
        return None
    return (e["fetch_kib"] * t["fetch_scale"] + e["write_kib"] * t["write_scale"]) * 1024.0


def copy_calibration(torch, mib=512):
    """One plain device-to-device copy of `mib` MiB (the reference kernel for
    scaling the HBM byte counters)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def run_gpu(torch, fmnmf, X, init, delta, N, K, precision, steps, warmup, out_cache):
    dt = np.complex128 if precision == "fp64" else np.complex64
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(dt))).to("cuda:0")
    m = fmnmf.FastMNMF(Xd, N, K, init, precision=precision, delta=delta)
    F, T, M = X.shape
    tdt = torch.complex128 if precision == "fp64" else torch.complex64
    key = (precision,)
    if key not in out_cache:
        out_cache.clear()
        out_cache[key] = torch.empty((N, F, T, M), dtype=tdt, device="cuda:0")
    out = out_cache[key]
    m.step(warmup)
    m.loglik()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(steps)
    m.separate(out=out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ll = m.loglik()
    # Wiener filter alone, and per-kernel means with HIP events on the
    # library's stream (instrumented iterations of the same workload).
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    m.separate(out=out)
    torch.cuda.synchronize()
    wiener_ms = (time.perf_counter() - t1) * 1e3
    kms = m.profile(5)
    # one step from the initial state, for the error against the oracle
    m.set_state(*init)
    m.step(1)
    ll1 = m.loglik()
    # the paper's initialisation of Q and G~ from the average observed SCM
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    m.init_scm()
    m.loglik()
    init_scm_ms = (time.perf_counter() - t2) * 1e3
    m.close()
    del Xd
    return {"elapsed": elapsed, "ll_end": ll, "wiener_ms": wiener_ms, "kernels_ms": kms, "ll_step1": ll1,
            "init_scm_ms": init_scm_ms}


def fca_leg(torch, fmnmf, synth, X, delta, N, precision, steps, warmup):
    """FastFCA (unconstrained lambda, Eq. 22) on the same mixture: iterations/s
    and the lambda pass against the HBM roofline."""
    F, T, M = X.shape
    rb = 8 if precision == "fp64" else 4
    dt = np.complex128 if precision == "fp64" else np.complex64
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(dt))).to("cuda:0")
    init = synth.make_fca_init(F, T, M, N, seed=synth.SEED_BASE + 3600)
    m = fmnmf.FastFCA(Xd, N, init, precision=precision, delta=delta)
    m.step(warmup)
    m.loglik()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms = m.profile(5)
    m.close()
    del Xd
    lam_bytes = F * T * (M + 2 * N) * rb  # x~ and lambda in, lambda out
    ach = lam_bytes / (kms["lam"] * 1e-3) / 1e9
    return {"iters_per_s": steps / elapsed, "ms_per_step": elapsed * 1e3 / steps,
            "kernels_ms": {k: round(v, 5) for k, v in kms.items() if v > 0},
            "lam_pass": {"bound": "hbm", "algorithmic_bytes": lam_bytes, "achieved": ach, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                         "traffic": measured_traffic("lampass", precision + "-fca")}}


def config_leg(torch, fmnmf, synth, cfg_id, precision, steps, warmup):
    """Another workload of the catalogue on one path: iterations/s with the
    final Wiener filter in the timed region (as the headline), the filter
    alone, per-kernel times and their roofline fractions."""
    c = synth.CONFIGS[cfg_id]
    X, init, delta = synth.workload(cfg_id)
    dt = np.complex128 if precision == "fp64" else np.complex64
    tdt = torch.complex128 if precision == "fp64" else torch.complex64
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(dt))).to("cuda:0")
    del X
    out = torch.empty((c.N, c.F, c.T, c.M), dtype=tdt, device="cuda:0")
    m = fmnmf.FastMNMF(Xd, c.N, c.K, init, precision=precision, delta=delta)
    m.step(warmup)
    m.loglik()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(steps)
    m.separate(out=out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    t1 = time.perf_counter()
    m.separate(out=out)
    torch.cuda.synchronize()
    wiener_ms = (time.perf_counter() - t1) * 1e3
    kms = m.profile(5)
    m.close()
    del Xd, out
    torch.cuda.empty_cache()
    iters = steps / elapsed
    rb = 8 if precision == "fp64" else 4
    it_ms = (elapsed * 1e3 - wiener_ms) / steps  # the steps' share of the timed run
    return {"workload": f"{c.name}: M={c.M} N={c.N} K={c.K} F={c.F} T={c.T}", "precision": precision,
            "steps": steps, "iters_per_s": iters, "ms_per_step": elapsed * 1e3 / steps,
            "tf_bins_per_s": iters * c.F * c.T, "wiener_ms": wiener_ms,
            "kernels_ms": {k: round(v, 5) for k, v in kms.items() if v},
            "iteration_hbm_frac": iteration_bytes(c.F, c.T, c.M, rb) / (it_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "kernels_roofline": roofline_table(kms, c.F, c.T, c.M, c.N, c.K, precision, wiener_ms)}


def cpu_baseline(X, init, delta, seconds):
    from oracle import fastmnmf as fm

    try:
        from threadpoolctl import threadpool_info

        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas_threads = None
    s = fm.State(*init)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    n = 0
    ll1 = None
    while True:
        s = fm.step(X, s, delta)
        n += 1
        if ll1 is None:
            ll1 = fm.loglik(X, s, delta)
            t_ll = time.perf_counter()
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    # the likelihood evaluation after step 1 is not part of an iteration
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return {"iters": n, "elapsed": el, "cpu_s": cpu, "ll_step1": ll1,
            "avail_cores": len(os.sched_getaffinity(0)), "blas_threads": blas_threads}


def serving_leg(torch, n_requests, precision, iters=100):
    """Config-5 style serving: closed-loop capacity of the batched server, then
    Poisson arrivals at 0.7 x that capacity through the batched server and
    through the one-at-a-time path."""
    from paper_1903_03237_amd import serve, synth

    print(f"[bench] serving: generating base mixtures for {n_requests} requests", file=sys.stderr, flush=True)
    bases = synth.serving_bases()
    # the base mixtures stay resident; a request's mixture is a device crop
    tdt = torch.complex128 if precision == "fp64" else torch.complex64
    dbases = {M: torch.from_numpy(X).to("cuda:0", dtype=tdt) for M, X in bases.items()}
    specs0 = synth.serving_specs(n_requests, None)
    prep = {sp.rid: synth.serving_request(sp, bases) for sp in specs0}

    def build(rate):
        reqs = []
        for sp in synth.serving_specs(n_requests, rate):
            _, init, delta = prep[sp.rid]
            X = dbases[sp.M][:, :sp.T, :]
            reqs.append(serve.Request(sp.rid, sp.arrival, X, sp.N, sp.K, init, delta, iters))
        return reqs

    order = os.environ.get("FMNMF_SERVE_ORDER", "fcfs")
    max_bins = int(os.environ.get("FMNMF_SERVE_MAX_BINS", 1_000_000))
    srv = serve.Server(precision=precision, hbm_budget=96 << 30, max_active=64, chunk=10,
                       max_bins=max_bins, order=order)
    print("[bench] serving: closed loop (all requests at t = 0)", file=sys.stderr, flush=True)
    closed = build(None)
    cap = serve.summary(srv.run(closed), closed)
    print("[bench] serving: closed loop, one at a time", file=sys.stderr, flush=True)
    cap_seq = serve.summary(serve.run_sequential(closed, precision=precision), closed)
    rate = 0.7 * cap["requests_per_s"]
    reqs = build(rate)
    print(f"[bench] serving: Poisson arrivals at {rate:.2f} requests/s, batched", file=sys.stderr, flush=True)
    batched = serve.summary(srv.run(reqs), reqs)
    print("[bench] serving: the same arrivals one at a time", file=sys.stderr, flush=True)
    seq = serve.summary(serve.run_sequential(reqs, precision=precision), reqs)
    torch.cuda.synchronize()
    return {"requests": n_requests, "iters_per_request": iters, "precision": precision,
            "admission": {"order": order, "max_bins": max_bins},
            "workload": "M in {2,4,8}, N in {2..5}, K in {8,16,32}, F=513, T ~ U{200..4000}; "
                        "crops of seeded base mixtures, seeded per-request initial states",
            "closed_loop": cap, "closed_loop_one_at_a_time": cap_seq, "arrival_rate_per_s": rate, "batched": batched, "one_at_a_time": seq,
            "p50_latency_s": batched["p50_latency_s"], "p99_latency_s": batched["p99_latency_s"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--paths", default="bf16,fp32,fp64", help="precision paths to time; first is the headline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests of the serving leg (0 disables it)")
    ap.add_argument("--fca-paths", default="fp32,fp64",
                    help="precision paths of the FastFCA leg on the same mixture (empty disables it)")
    ap.add_argument("--legs", default="2:fp64,4:bf16",
                    help="other workloads of the catalogue to time, as config:path pairs (empty disables)")
    ap.add_argument("--leg-steps", type=int, default=20)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 512 MiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding of this "
              "path is a design note, not a measured configuration.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1903_03237_amd import fmnmf, synth

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        print("[bench] copy calibration: 512 MiB device-to-device", file=sys.stderr, flush=True)
        copy_calibration(torch)
    cfg = synth.CONFIGS[3]
    F, T, M, N, K = cfg.F, cfg.T, cfg.M, cfg.N, cfg.K
    print(f"[bench] generating workload {cfg.name}", file=sys.stderr, flush=True)
    X, init, delta = synth.workload(3)
    paths = [p.strip() for p in args.paths.split(",") if p.strip()]
    res = {}
    cache = {}
    for p in paths:
        print(f"[bench] timing {p}: {args.warmup} warmup + {args.steps} steps", file=sys.stderr, flush=True)
        res[p] = run_gpu(torch, fmnmf, X, init, delta, N, K, p, args.steps, args.warmup, cache)
    cache.clear()
    fca = {}
    for p in [q.strip() for q in args.fca_paths.split(",") if q.strip()]:
        print(f"[bench] FastFCA {p}: {args.warmup} warmup + {args.steps} steps", file=sys.stderr, flush=True)
        fca[p] = fca_leg(torch, fmnmf, synth, X, delta, N, p, args.steps, args.warmup)

    legs = {}
    for item in [q.strip() for q in args.legs.split(",") if q.strip()]:
        cid, prec = item.split(":")
        print(f"[bench] workload {cid} on {prec}: {args.warmup} warmup + {args.leg_steps} steps", file=sys.stderr,
              flush=True)
        legs[item] = config_leg(torch, fmnmf, synth, int(cid), prec, args.leg_steps, args.warmup)

    serving = None
    if args.serving_requests > 0:
        serving = serving_leg(torch, args.serving_requests, paths[0])

    base = None
    if not args.no_cpu_baseline:
        print(f"[bench] timing the FP64 CPU oracle for ~{args.cpu_seconds:.0f} s", file=sys.stderr, flush=True)
        base = cpu_baseline(X, init, delta, args.cpu_seconds)

    head = paths[0]
    h = res[head]
    value = args.steps / h["elapsed"]
    rb = 8 if head == "fp64" else 4
    km = kernel_model(F, T, M, N, K, rb)
    kms = h["kernels_ms"]
    dom = max(km, key=lambda k: kms.get(k, 0.0))
    d = km[dom]
    sec = kms[dom] * 1e-3
    if d["bound"] == "hbm":
        roof = {"kernel": dom, "bound": "hbm", "achieved": d["bytes"] / sec / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        peak = VALU_FP64_TFLOPS if head == "fp64" else VALU_FP32_TFLOPS
        roof = {"kernel": dom, "bound": "alu", "achieved": d["flops"] / sec / 1e12, "peak": peak,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, head)
    roof["algorithmic_per_launch"] = d["bytes"] if d["bound"] == "hbm" else d["flops"]
    roof["avg_launch_ms"] = kms[dom]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["elapsed"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp32": "f32", "fp64": "f64"}[head],
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: M={M} N={N} K={K} F={F} T={T}, -5 dB diffuse noise, "
                               f"delta=1e-8 mean|x|^2; {args.steps} iterations + Wiener filter",
                   "F": F, "T": T, "M": M, "N": N, "K": K, "precision": head},
        "tf_bins_per_s": value * F * T,
        "paths": {},
        "kernels_ms": {k: round(v, 5) for k, v in kms.items()},
        "wiener_ms": h["wiener_ms"],
        "roofline": roof,
        "kernels_roofline": roofline_table(kms, F, T, M, N, K, head, h["wiener_ms"]),
        # one iteration's algorithmic bytes over its time in the timed run (the
        # steps' share: elapsed minus one Wiener filter)
        "iteration_hbm_frac": iteration_bytes(F, T, M, rb) * args.steps
        / (h["elapsed"] - h["wiener_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }
    for p, r in res.items():
        e = {"iters_per_s": args.steps / r["elapsed"], "ms_per_step": r["elapsed"] * 1e3 / args.steps,
             "iter_ms_kernels": sum(r["kernels_ms"].values()), "wiener_ms": r["wiener_ms"],
             "init_scm_ms": r["init_scm_ms"]}
        if base is not None:
            ref = base["ll_step1"]
            e["ll_rel_err_step1"] = abs(r["ll_step1"] - ref) / max(abs(ref), F * T * M)
        out["paths"][p] = e
    if legs:
        out["other_workloads"] = legs
    if fca:
        out["fastfca"] = fca
    if serving is not None:
        out["serving"] = serving
    if "fp64" in res and head != "fp64":
        out["speedup_vs_fp64"] = out["paths"][head]["iters_per_s"] / out["paths"]["fp64"]["iters_per_s"]
    if base is not None:
        out["cpu_baseline"] = {
            "value": base["iters"] / base["elapsed"],
            "unit": "iters/s",
            "cores": round(base["cpu_s"] / base["elapsed"], 2),
            "kind": "oracle",
            "sample": f"{base['iters']} FP64 NumPy oracle iterations of the same workload from the same "
                      f"initial state ({base['elapsed']:.1f} s wall; {base['avail_cores']} cores available, "
                      f"BLAS threads {base['blas_threads']}; cores = CPU-seconds / wall-seconds)",
        }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
