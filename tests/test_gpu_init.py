"""GPU parity of the paper's initialisation (fmnmf_init_scm, Sec. IV-A) with the
oracle's ``init_from_scm``.

Each row of Q_f is unique up to a unit complex factor (distinct eigenvalues
of the seeded SCMs), so Q is compared after aligning each row's phase; g~,
x~ and Eq. (17), which do not depend on those factors, are compared
directly, and so is the first iteration started from the initialisation.
"""

import numpy as np
import pytest

from oracle import fastfca as fca
from oracle import fastmnmf as fm
from paper_1903_03237_amd import synth
from parity_util import FP64, assert_close, rel_norm as _rel

pytestmark = pytest.mark.gpu


def _align_rows(Qg, Qo):
    """Qg with each row multiplied by the unit factor that best matches Qo."""
    d = np.einsum("fmj,fmj->fm", Qg.conj(), Qo)
    return Qg * (d / np.abs(d))[:, :, None]


def _model(device, X, N, K, init, precision, delta=0.0, derived=False):
    import torch

    from paper_1903_03237_amd import fmnmf

    dt = np.complex128 if precision == "fp64" else np.complex64
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(dt))).to(device)
    return fmnmf.FastMNMF(Xd, N, K, init, precision=precision, delta=delta, derived=derived)


@pytest.mark.parametrize("M", [1, 2, 3, 5, 8])
def test_init_scm_fp64_parity(device, M):
    F, T, N, K = 37, 150, 3, 6
    X, (W0, H0, G0, Q0), delta = synth.random_problem(F, T, M, N, K, seed=300 + M, random_q=True)
    m = _model(device, X, N, K, (W0, H0, G0, Q0), "fp64", delta, derived=True)
    m.init_scm()
    Go, Qo = fm.init_from_scm(X, N)
    s0 = fm.State(W0, H0, Go, Qo)
    l0 = fm.loglik(X, s0, delta)
    assert abs(m.loglik() - l0) <= 1e-10 * abs(l0)
    W, H, G, Q = m.get_state()
    assert np.array_equal(W, W0) and np.array_equal(H, H0)
    # eigenvalues to 1e-12, eigenvectors (each row up to its unit factor) to
    # 1e-10 of the entry plus 1e-12 of the largest
    assert_close("G", G, Go, rtol=1e-12, atol_rel=1e-14)
    assert_close("Q", _align_rows(Q, Qo), Qo, rtol=1e-10, atol_rel=1e-12)
    assert_close("x~", m.derived(0), fm.project(X, Qo), rtol=1e-10, atol_rel=1e-12)
    m.step(1)
    s1 = fm.step(X, s0, delta)
    W, H, G, Q = m.get_state()
    for name, a, b in (("W", W, s1.W), ("H", H, s1.H), ("G", G, s1.G)):
        assert_close(name, a, b, **FP64)
    assert_close("Q1", _align_rows(Q, s1.Q), s1.Q, rtol=1e-10, atol_rel=1e-12)
    l1 = fm.loglik(X, s1, delta)
    assert abs(m.loglik() - l1) <= 1e-10 * abs(l1)
    m.close()


def test_init_scm_fp32(device):
    F, T, M, N, K = 65, 300, 8, 5, 16
    X, init, delta = synth.random_problem(F, T, M, N, K, seed=310, delta_rel=1e-8)
    m = _model(device, X, N, K, init, "fp32", delta)
    m.init_scm()
    Go, Qo = fm.init_from_scm(X, N)
    ref = fm.loglik(X, fm.State(init[0], init[1], Go, Qo), delta)
    assert abs(m.loglik() - ref) <= 1e-5 * max(abs(ref), F * T * M)
    _, _, G, Q = m.get_state()
    assert _rel(G, Go) < 1e-5
    assert _rel(_align_rows(Q, Qo), Qo) < 1e-4
    m.close()


def test_init_scm_fastfca(device):
    import torch

    from paper_1903_03237_amd import fmnmf

    F, T, M, N = 33, 120, 4, 3
    X, (lam0, G0, Q0), delta = synth.random_fca_problem(F, T, M, N, seed=311, random_q=True)
    m = fmnmf.FastFCA(torch.from_numpy(X).to(device), N, (lam0, G0, Q0), precision="fp64", delta=delta)
    m.init_scm()
    Go, Qo = fm.init_from_scm(X, N)
    s0 = fca.State(np.ascontiguousarray(np.moveaxis(lam0, 0, 2)), Go, Qo)
    m.step(1)
    s1 = fca.step(X, s0, delta)
    lam, G, Q = m.get_state()
    assert_close("lam", lam, np.moveaxis(s1.lam, 2, 0), **FP64)
    assert_close("G", G, s1.G, **FP64)
    assert abs(m.loglik() - fca.loglik(X, s1, delta)) <= 1e-10 * abs(fca.loglik(X, s1, delta))
    m.close()


def test_init_scm_rank_deficient_is_reported(device):
    """T < M: the average SCM has rank T < M, so some eigenvalue is not positive."""
    from paper_1903_03237_amd import fmnmf

    X, init, delta = synth.random_problem(5, 2, 4, 2, 2, seed=312, random_q=True)
    m = _model(device, X, 2, 2, init, "fp64", delta)
    m.init_scm()
    with pytest.raises(fmnmf.FmnmfError) as ei:
        m.loglik()
    assert ei.value.code == fmnmf.E_SINGULAR
    m.close()
