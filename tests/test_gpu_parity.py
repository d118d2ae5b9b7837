"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

FP64 path: one-step parity from identical states, element by element
(|gpu - ref| <= 1e-10 |ref| + 1e-13 max|ref| for every entry of W, H, G~, Q,
x~, y~ and the separated images; |dL| <= 1e-10 |L|), on shapes that span
several 16-wide tiles and ragged tails in F and T, every supported M class
and several (N, K).  FP32 / mixed-bf16 paths: the error bounds stated for
them (log-likelihood 1e-5 relative per step).
"""

import numpy as np
import pytest

from oracle import fastmnmf as fm
from paper_1903_03237_amd import synth
from parity_util import FP64, assert_close, rel_norm as _rel

pytestmark = pytest.mark.gpu


def _model(device, X, N, K, init, precision, delta, derived=False):
    import torch

    from paper_1903_03237_amd import fmnmf

    dt = np.complex128 if precision == "fp64" else np.complex64
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(dt))).to(device)
    return fmnmf.FastMNMF(Xd, N, K, init, precision=precision, delta=delta, derived=derived)


# (F, T, M, N, K, delta_rel, random_q)
FP64_CASES = [
    (21, 37, 3, 2, 5, 0.0, True),
    (129, 100, 2, 2, 4, 0.0, False),
    (40, 70, 1, 1, 1, 0.0, True),
    (33, 90, 4, 3, 16, 1e-6, True),
    (17, 130, 5, 5, 20, 1e-8, True),
    (50, 64, 8, 6, 40, 1e-8, True),
    (16, 16, 2, 8, 64, 0.0, True),
    (70, 33, 6, 4, 33, 1e-8, True),
    (1, 1, 1, 1, 1, 0.0, True),
    (3, 5, 2, 1, 2, 0.0, True),
]


@pytest.mark.parametrize("case", FP64_CASES, ids=lambda c: "F%dT%dM%dN%dK%d" % c[:5])
def test_fp64_one_step_parity(device, case):
    F, T, M, N, K, drel, rq = case
    X, init, delta = synth.random_problem(F, T, M, N, K, seed=F * 7 + T, delta_rel=drel, random_q=rq)
    s0 = fm.State(*init)
    m = _model(device, X, N, K, init, "fp64", delta, derived=True)
    # initial projection, model and likelihood
    assert abs(m.loglik() - fm.loglik(X, s0, delta)) <= 1e-10 * abs(fm.loglik(X, s0, delta))
    assert_close("x~0", m.derived(0), fm.project(X, s0.Q), rtol=1e-12, atol_rel=1e-14)
    assert_close("y~0", m.derived(1), fm.model(fm.psd(s0.W, s0.H), s0.G, delta), rtol=1e-12, atol_rel=1e-14)
    # one step from the initial state
    m.step(1)
    s1 = fm.step(X, s0, delta)
    W, H, G, Q = m.get_state()
    for name, a, b in (("W", W, s1.W), ("H", H, s1.H), ("G", G, s1.G), ("Q", Q, s1.Q)):
        assert_close(name, a, b, **FP64)
    l1 = fm.loglik(X, s1, delta)
    assert abs(m.loglik() - l1) <= 1e-10 * abs(l1)
    assert_close("x~1", m.derived(0), fm.project(X, s1.Q), **FP64)
    assert_close("y~1", m.derived(1), fm.model(fm.psd(s1.W, s1.H), s1.G, delta), **FP64)
    # inject a later oracle state and step once more
    s3 = fm.step(X, fm.step(X, s1, delta), delta)
    m.set_state(s3.W, s3.H, s3.G, s3.Q)
    assert abs(m.loglik() - fm.loglik(X, s3, delta)) <= 1e-10 * abs(fm.loglik(X, s3, delta))
    m.step(1)
    s4 = fm.step(X, s3, delta)
    W, H, G, Q = m.get_state()
    for name, a, b in (("W", W, s4.W), ("H", H, s4.H), ("G", G, s4.G), ("Q", Q, s4.Q)):
        assert_close(name, a, b, **FP64)
    # separation of the final state
    Y = m.separate().cpu().numpy()
    assert_close("separated", Y, fm.separate(X, s4, delta), **FP64)
    m.close()


def test_fewer_frames_than_channels_is_singular(device):
    """T < M: every V_fm = (1/T) sum_t x x^H / y~ has rank T < M, so the IP
    system of Eq. (19) is singular; the library reports it (and the oracle's
    solve degenerates too) instead of producing numbers."""
    from paper_1903_03237_amd import fmnmf

    X, init, delta = synth.random_problem(5, 2, 3, 1, 1, seed=1, random_q=True)
    m = _model(device, X, 1, 1, init, "fp64", delta)
    m.step(1)
    with pytest.raises(fmnmf.FmnmfError) as ei:
        m.loglik()
    assert ei.value.code == fmnmf.E_SINGULAR
    m.close()


def test_fp64_trajectory_small_config(device):
    """The oracle-sized workload (M=2, N=2, K=4, F=129, T=100), 10 free-running
    iterations from the same seeded state; monotone and within 1e-9."""
    X, init, delta = synth.workload(1)
    m = _model(device, X, 2, 4, init, "fp64", delta)
    s = fm.State(*init)
    lls = [m.loglik()]
    for _ in range(10):
        m.step(1)
        lls.append(m.loglik())
    s, ref = fm.run(X, s, 10, delta)
    np.testing.assert_allclose(lls, ref, rtol=1e-9)
    assert np.all(np.diff(lls) >= -1e-10 * abs(lls[-1]))
    W, H, G, Q = m.get_state()
    for name, a, b in (("W", W, s.W), ("H", H, s.H), ("G", G, s.G), ("Q", Q, s.Q)):
        assert_close(name, a, b, rtol=1e-9, atol_rel=1e-12)
    m.close()


def test_fp64_deterministic(device):
    X, init, delta = synth.random_problem(45, 80, 4, 3, 12, seed=3, random_q=True)
    outs = []
    for _ in range(2):
        m = _model(device, X, 3, 12, init, "fp64", delta)
        m.step(3)
        outs.append((m.loglik(),) + tuple(m.get_state()))
        m.close()
    assert outs[0][0] == outs[1][0]
    for a, b in zip(outs[0][1:], outs[1][1:]):
        assert np.array_equal(a, b)


# Log-likelihood error is measured against max(|L|, F T M): L sums F T M terms
# of order one that largely cancel, so |L| alone can be small.  bf16 operands
# round W and H to 8 significant bits, which at these tiny sizes does not
# average out; the full-size errors are reported by the precision study.
@pytest.mark.parametrize("precision,tol_ll,tol_state", [("fp32", 1e-5, 2e-3), ("bf16", 5e-4, 5e-2)])
@pytest.mark.parametrize("case", [(33, 90, 4, 3, 16), (50, 200, 8, 5, 32), (21, 37, 3, 2, 5),
                                  (65, 96, 8, 6, 64), (40, 80, 7, 8, 48), (21, 45, 8, 2, 5),
                                  (33, 60, 8, 3, 16), (40, 80, 8, 7, 48)],
                         ids=lambda c: "F%dT%dM%dN%dK%d" % c)
def test_reduced_precision_one_step(device, precision, tol_ll, tol_state, case):
    F, T, M, N, K = case
    X, init, delta = synth.random_problem(F, T, M, N, K, seed=11 + F, delta_rel=1e-8, random_q=True)
    X = X.astype(np.complex64).astype(np.complex128)  # the oracle sees the same rounded input
    s0 = fm.State(*init)
    m = _model(device, X, N, K, init, precision, delta, derived=True)
    l0 = fm.loglik(X, s0, delta)
    scale = lambda ll: max(abs(ll), F * T * M)
    assert abs(m.loglik() - l0) <= tol_ll * scale(l0)
    assert _rel(m.derived(0), fm.project(X, s0.Q)) < 1e-5
    s3 = fm.step(X, fm.step(X, fm.step(X, s0, delta), delta), delta)
    m.set_state(s3.W, s3.H, s3.G, s3.Q)
    m.step(1)
    s4 = fm.step(X, s3, delta)
    l4 = fm.loglik(X, s4, delta)
    assert abs(m.loglik() - l4) <= tol_ll * scale(l4), (m.loglik(), l4)
    W, H, G, Q = m.get_state()
    for name, a, b in (("W", W, s4.W), ("H", H, s4.H), ("G", G, s4.G), ("Q", Q, s4.Q)):
        assert _rel(a, b) < tol_state, (name, _rel(a, b))
    Y = m.separate().cpu().numpy()
    assert _rel(Y, fm.separate(X, s4, delta)) < tol_state
    m.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_v_pass_long_frame_splits(device, precision, monkeypatch):
    """The V pass with its frames in two splits (FMNMF_SPLITS), so that the
    workgroups walk 29 and 28 steps of 16 frames (an odd and an even count,
    the last step ragged), at M = 8 (on the FP32 and bf16 paths the 4x4x1
    form), one step from an injected oracle state against the oracle's."""
    F, T, M, N, K = 33, 900, 8, 3, 8
    X, init, delta = synth.random_problem(F, T, M, N, K, seed=5, delta_rel=1e-8, random_q=True)
    if precision != "fp64":
        X = X.astype(np.complex64).astype(np.complex128)  # the oracle sees the same rounded input
    s1 = fm.step(X, fm.State(*init), delta)
    monkeypatch.setenv("FMNMF_SPLITS", "0,0,0,2")
    m = _model(device, X, N, K, init, precision, delta)
    m.set_state(s1.W, s1.H, s1.G, s1.Q)
    m.step(1)
    s2 = fm.step(X, s1, delta)
    l2 = fm.loglik(X, s2, delta)
    W, H, G, Q = m.get_state()
    pairs = (("W", W, s2.W), ("H", H, s2.H), ("G", G, s2.G), ("Q", Q, s2.Q))
    if precision == "fp64":
        assert abs(m.loglik() - l2) <= 1e-10 * abs(l2)
        for name, a, b in pairs:
            assert_close(name, a, b, **FP64)
    else:
        tol_ll, tol_state = (1e-5, 2e-3) if precision == "fp32" else (5e-4, 5e-2)
        assert abs(m.loglik() - l2) <= tol_ll * max(abs(l2), F * T * M), (m.loglik(), l2)
        for name, a, b in pairs:
            assert _rel(a, b) < tol_state, (name, _rel(a, b))
    m.close()


@pytest.mark.parametrize("M", [4, 5])
def test_separate_into_8_byte_aligned_output(device, M):
    """The filter writes 16-byte vectors only to 16-byte aligned outputs with
    M == MP; an output that is only 8-byte aligned (allowed by the ABI) gets
    the same values through element stores."""
    import torch

    F, T, N, K = 19, 70, 2, 4
    X, init, delta = synth.random_problem(F, T, M, N, K, seed=77, random_q=True)
    m = _model(device, X, N, K, init, "fp32", delta)
    m.step(2)
    ref = m.separate().cpu().numpy()
    buf = torch.zeros(N * F * T * M + 1, dtype=torch.complex64, device=device)
    view = buf[1:].view(N, F, T, M)  # data pointer 8 bytes past a 256-byte boundary
    assert view.data_ptr() % 16 == 8
    torch.cuda.synchronize()
    m.separate(out=view)
    assert np.array_equal(view.cpu().numpy(), ref)
    assert buf[0].item() == 0
    m.close()


# Options: the frequency-tied G~ (Eq. 21 summed over f) and the scale
# normalisation, each against the oracle's step with the same option.
@pytest.mark.parametrize("tie_g,norm", [(True, False), (False, True), (True, True)])
@pytest.mark.parametrize("case", [(21, 37, 3, 2, 5), (50, 64, 8, 6, 40), (33, 90, 4, 3, 16)],
                         ids=lambda c: "F%dT%dM%dN%dK%d" % c)
def test_fp64_options_parity(device, case, tie_g, norm):
    F, T, M, N, K = case
    X, init, delta = synth.random_problem(F, T, M, N, K, seed=F * 11 + T, delta_rel=1e-8, random_q=True)
    if tie_g:  # the tied variant starts from a frequency-independent g~
        init = (init[0], init[1], np.broadcast_to(init[2][:, :1, :], init[2].shape).copy(), init[3])
    import torch

    from paper_1903_03237_amd import fmnmf

    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(device)
    m = fmnmf.FastMNMF(Xd, N, K, init, precision="fp64", delta=delta, tie_g=tie_g, normalize=norm)
    s = fm.State(*init)
    for _ in range(3):
        m.step(1)
        s = fm.step(X, s, delta, tie_g=tie_g, norm=norm)
        L = fm.loglik(X, s, delta)
        assert abs(m.loglik() - L) <= 1e-10 * abs(L)
    W, H, G, Q = m.get_state()
    for name, a, b in (("W", W, s.W), ("H", H, s.H), ("G", G, s.G), ("Q", Q, s.Q)):
        assert_close(name, a, b, **FP64)
    if tie_g:
        assert np.ptp(G, axis=1).max() <= 1e-12 * np.abs(G).max()
    m.close()


def test_options_reduced_precision(device):
    # the options on the FP32 and mixed paths: L within the per-step bound
    F, T, M, N, K = 50, 200, 8, 5, 32
    X, init, delta = synth.random_problem(F, T, M, N, K, seed=77, delta_rel=1e-8, random_q=True)
    init = (init[0], init[1], np.broadcast_to(init[2][:, :1, :], init[2].shape).copy(), init[3])
    import torch

    from paper_1903_03237_amd import fmnmf

    s1 = fm.step(X, fm.State(*init), delta, tie_g=True, norm=True)
    L1 = fm.loglik(X, s1, delta)
    for p, tol in (("fp32", 1e-5), ("bf16", 5e-4)):
        Xd = torch.from_numpy(np.ascontiguousarray(X.astype(np.complex64))).to(device)
        m = fmnmf.FastMNMF(Xd, N, K, init, precision=p, delta=delta, tie_g=True, normalize=True)
        m.step(1)
        assert abs(m.loglik() - L1) <= tol * max(abs(L1), F * T * M), p
        m.close()
