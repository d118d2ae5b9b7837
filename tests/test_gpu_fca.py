"""GPU parity of FastFCA (flag FMNMF_FCA: lambda by Eq. 22, then G~, IP, x~, L)
through the C ABI against the FP64 CPU oracle ``oracle.fastfca``.

FP64: one step from identical states to 1e-10 relative, on shapes spanning
several 16-wide tiles, ragged tails in F and T, more than one 256-frame block
of the lambda pass, every M class and N class, with and without delta and the
tied G~.  FP32: L within 1e-5 relative per step.
"""

import numpy as np
import pytest

from oracle import fastfca as fca
from paper_1903_03237_amd import synth
from parity_util import FP64, assert_close, rel_norm as _rel

pytestmark = pytest.mark.gpu


def _abi_lam(lam_ftn):  # oracle [F, T, N] -> ABI [N, F, T]
    return np.ascontiguousarray(np.moveaxis(lam_ftn, 2, 0))


def _oracle_lam(lam_nft):
    return np.ascontiguousarray(np.moveaxis(lam_nft, 0, 2))


def _problem(F, T, M, N, seed, drel=0.0, rq=True):
    X, (lam0, G0, Q0), delta = synth.random_fca_problem(F, T, M, N, seed=seed, delta_rel=drel, random_q=rq)
    return X, (lam0, G0, Q0), fca.State(_oracle_lam(lam0), G0, Q0), delta


def _model(device, X, N, init, precision, delta, derived=False, tie_g=False):
    import torch

    from paper_1903_03237_amd import fmnmf

    dt = np.complex128 if precision == "fp64" else np.complex64
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(dt))).to(device)
    return fmnmf.FastFCA(Xd, N, init, precision=precision, delta=delta, derived=derived, tie_g=tie_g)


# (F, T, M, N, delta_rel, random_q, tie_g)
CASES = [
    (21, 37, 3, 2, 0.0, True, False),
    (129, 100, 2, 2, 0.0, False, False),
    (40, 70, 1, 1, 0.0, True, False),
    (33, 90, 4, 3, 1e-6, True, True),
    (50, 300, 8, 5, 1e-8, True, False),
    (17, 130, 5, 8, 1e-8, True, False),
    (70, 600, 6, 6, 1e-8, True, True),
    (1, 1, 1, 1, 0.0, True, False),
    (3, 5, 2, 1, 0.0, True, True),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "F%dT%dM%dN%d" % c[:4] + ("tied" if c[6] else ""))
def test_fca_fp64_one_step_parity(device, case):
    F, T, M, N, drel, rq, tie = case
    X, init, s0, delta = _problem(F, T, M, N, seed=F * 5 + T, drel=drel, rq=rq)
    m = _model(device, X, N, init, "fp64", delta, derived=True, tie_g=tie)
    from oracle import fastmnmf as fm

    l0 = fca.loglik(X, s0, delta)
    assert abs(m.loglik() - l0) <= 1e-10 * abs(l0)
    assert_close("x~0", m.derived(0), fm.project(X, s0.Q), rtol=1e-12, atol_rel=1e-14)
    assert_close("y~0", m.derived(1), fm.model(s0.lam, s0.G, delta), rtol=1e-12, atol_rel=1e-14)
    m.step(1)
    s1 = fca.step(X, s0, delta, tie_g=tie)
    lam, G, Q = m.get_state()
    for name, a, b in (("lam", lam, _abi_lam(s1.lam)), ("G", G, s1.G), ("Q", Q, s1.Q)):
        assert_close(name, a, b, **FP64)
    l1 = fca.loglik(X, s1, delta)
    assert abs(m.loglik() - l1) <= 1e-10 * abs(l1)
    # inject a later oracle state and step once more
    s3 = fca.step(X, fca.step(X, s1, delta, tie_g=tie), delta, tie_g=tie)
    m.set_state(_abi_lam(s3.lam), s3.G, s3.Q)
    l3 = fca.loglik(X, s3, delta)
    assert abs(m.loglik() - l3) <= 1e-10 * abs(l3)
    m.step(1)
    s4 = fca.step(X, s3, delta, tie_g=tie)
    lam, G, Q = m.get_state()
    for name, a, b in (("lam", lam, _abi_lam(s4.lam)), ("G", G, s4.G), ("Q", Q, s4.Q)):
        assert_close(name, a, b, **FP64)
    Y = m.separate().cpu().numpy()
    assert_close("separated", Y, fca.separate(X, s4, delta), **FP64)
    m.close()


def test_fca_fp64_trajectory(device):
    """10 free-running iterations from the same seeded state: monotone, within 1e-9."""
    X, init, s, delta = _problem(129, 100, 2, 2, seed=77)
    m = _model(device, X, 2, init, "fp64", delta)
    lls = [m.loglik()]
    for _ in range(10):
        m.step(1)
        lls.append(m.loglik())
    s, ref = fca.run(X, s, 10, delta)
    np.testing.assert_allclose(lls, ref, rtol=1e-9)
    assert np.all(np.diff(lls) >= -1e-10 * abs(lls[-1]))
    lam, G, Q = m.get_state()
    for name, a, b in (("lam", lam, _abi_lam(s.lam)), ("G", G, s.G), ("Q", Q, s.Q)):
        assert_close(name, a, b, rtol=1e-9, atol_rel=1e-12)
    m.close()


@pytest.mark.parametrize("case", [(33, 90, 4, 3, 1e-6), (65, 400, 8, 5, 1e-8)], ids=lambda c: "F%dT%dM%dN%d" % c[:4])
def test_fca_fp32_per_step(device, case):
    F, T, M, N, drel = case
    X, init, s, delta = _problem(F, T, M, N, seed=F + T, drel=drel)
    m = _model(device, X, N, init, "fp32", delta)
    for _ in range(3):
        m.set_state(_abi_lam(s.lam), s.G, s.Q)
        m.step(1)
        s = fca.step(X, s, delta)
        ref = fca.loglik(X, s, delta)
        assert abs(m.loglik() - ref) <= 1e-5 * max(abs(ref), F * T * M)
        lam, G, Q = m.get_state()
        assert _rel(lam, _abi_lam(s.lam)) < 2e-3 and _rel(G, s.G) < 2e-3
    m.close()


def test_fca_batched_equals_alone(device):
    """FastFCA contexts batched with each other and with a FastMNMF context give
    bitwise the results of stepping each alone."""
    from paper_1903_03237_amd import fmnmf

    probs = [_problem(40, 150, 4, 3, seed=5), _problem(33, 260, 3, 2, seed=6)]
    Xm, initm, deltam = synth.random_problem(30, 120, 4, 3, 8, seed=7, random_q=True)

    def build():
        import torch

        ms = [_model(device, X, s.G.shape[0], init, "fp64", delta) for X, init, s, delta in probs]
        Xd = torch.from_numpy(Xm).to(device)
        ms.append(fmnmf.FastMNMF(Xd, 3, 8, initm, precision="fp64", delta=deltam))
        return ms

    alone = build()
    for m in alone:
        m.step(3)
    batched = build()
    fmnmf.step_batch(batched, 3)
    for a, b in zip(alone, batched):
        assert a.loglik() == b.loglik()
        for x, y in zip(a.get_state(), b.get_state()):
            assert np.array_equal(x, y)
        a.close()
        b.close()


def test_fca_profile_runs_the_lambda_pass(device):
    X, init, _, delta = _problem(65, 300, 4, 3, seed=9)
    m = _model(device, X, 3, init, "fp32", delta)
    ms = m.profile(2)
    assert ms["lam"] > 0 and ms["gpass"] > 0 and ms["ip"] > 0 and ms["proj"] > 0
    assert ms["wpass"] == 0 and ms["hpass"] == 0 and ms["mu_w"] == 0 and ms["mu_h"] == 0
    m.close()
