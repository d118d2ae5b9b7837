"""Pins of the FastFCA oracle (Sec. III-C; lambda by Eq. 22) to facts outside it.

As for FastMNMF, nothing here compares the oracle with itself: the checks are
brute-force evaluations of the full-rank formulas on explicit M x M matrices,
finite differences of Eq. (17), a closed form of the rank-one case, and the
monotonicity that the MM / IP updates guarantee.
"""

import numpy as np
import pytest

from oracle import fastfca as fca
from oracle import fastmnmf as fm
from oracle import fullrank as fr
from paper_1903_03237_amd import synth


def _problem(F=3, T=6, M=3, N=2, seed=31, delta_rel=0.0, random_q=True):
    X, (lam0, G0, Q0), delta = synth.random_fca_problem(F, T, M, N, seed=seed, delta_rel=delta_rel,
                                                        random_q=random_q)
    return X, fca.State(np.ascontiguousarray(np.moveaxis(lam0, 0, 2)), G0, Q0), delta


@pytest.mark.parametrize("delta_rel", [0.0, 1e-2])
def test_lambda_terms_equal_fullrank_traces(delta_rel):
    """Eq. (22)'s sums over m equal tr(G_nf Y^-1 X_ft Y^-1) and tr(G_nf Y^-1)
    of the full-rank model with G_nf = Q_f^-1 Diag(g~_nf) Q_f^-H."""
    X, s, delta = _problem(F=3, T=5, M=3, N=2, seed=40, delta_rel=delta_rel)
    num, den = fca.terms_lam(fm.project(X, s.Q), s.lam, s.G, delta)
    extra = fr.floor_scm(s.Q, delta) if delta > 0 else None
    tn, td = fr.mnmf_traces(X, s.lam, fr.scm_from_diag(s.Q, s.G), extra)  # [N, F, T]
    np.testing.assert_allclose(num, np.moveaxis(tn, 0, 2), rtol=1e-10)
    np.testing.assert_allclose(den, np.moveaxis(td, 0, 2), rtol=1e-10)


def test_lambda_update_is_the_fullrank_rule():
    """lambda <- lambda sqrt(tr(G Y^-1 X Y^-1) / tr(G Y^-1)), evaluated on explicit matrices."""
    X, s, delta = _problem(F=2, T=7, M=2, N=3, seed=41)
    tn, td = fr.mnmf_traces(X, s.lam, fr.scm_from_diag(s.Q, s.G))
    ref = s.lam * np.sqrt(np.moveaxis(tn / td, 0, 2))
    np.testing.assert_allclose(fca.update_lam(fm.project(X, s.Q), s.lam, s.G, delta), ref, rtol=1e-11)


def test_lambda_terms_are_gradient_parts():
    """d/dlambda_ftn of sum(x~/y~) = -num and of sum(log y~) = den (finite differences)."""
    X, s, delta = _problem(F=3, T=4, M=2, N=2, seed=42, delta_rel=1e-3)
    Xt = fm.project(X, s.Q)
    num, den = fca.terms_lam(Xt, s.lam, s.G, delta)
    rng = np.random.default_rng(3)
    for _ in range(8):
        idx = tuple(int(rng.integers(0, d)) for d in s.lam.shape)
        h = 1e-6 * s.lam[idx]

        def fd(fun):
            lp, lm = s.lam.copy(), s.lam.copy()
            lp[idx] += h
            lm[idx] -= h
            return (fun(fm.model(lp, s.G, delta)) - fun(fm.model(lm, s.G, delta))) / (2 * h)

        assert abs(-fd(lambda Y: np.sum(Xt / Y)) - num[idx]) < 1e-6 * abs(num[idx])
        assert abs(fd(lambda Y: np.sum(np.log(Y))) - den[idx]) < 1e-6 * abs(den[idx])


def test_rank_one_lambda_step_is_geometric_mean_with_ml():
    """N = M = 1, delta = 0: y~ = lambda g, the ML lambda of a bin is x~/g, and
    Eq. (22) returns sqrt(lambda * x~/g)."""
    X, s, _ = _problem(F=4, T=9, M=1, N=1, seed=43)
    Xt = fm.project(X, s.Q)
    lam, g = s.lam[:, :, 0], s.G[0, :, 0]
    expect = np.sqrt(lam * Xt[:, :, 0] / g[:, None])
    np.testing.assert_allclose(fca.update_lam(Xt, s.lam, s.G)[:, :, 0], expect, rtol=1e-13)


@pytest.mark.parametrize("delta_rel", [0.0, 1e-2])
def test_fast_loglik_and_filter_equal_fullrank(delta_rel):
    """Eq. (17) with a free lambda equals Eq. (4); the filter equals Eq. (3)."""
    X, s, delta = _problem(F=3, T=5, M=3, N=2, seed=44, delta_rel=delta_rel)
    Gfull = fr.scm_from_diag(s.Q, s.G)
    extra = fr.floor_scm(s.Q, delta) if delta > 0 else None
    brute = fr.loglik_fullrank(X, s.lam, Gfull, extra)
    assert abs(fca.loglik(X, s, delta) - brute) <= 1e-11 * abs(brute)
    if delta == 0.0:
        np.testing.assert_allclose(fca.separate(X, s), fr.mwf_fullrank(X, s.lam, Gfull), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("tie_g", [False, True])
def test_monotone_after_every_substep_and_row(tie_g):
    """The MM bound for lambda and G~ and the IP coordinate ascent: Eq. (17) never
    decreases, after lambda, after G~ and after each row of each Q_f."""
    X, s, delta = _problem(F=4, T=12, M=3, N=2, seed=45, delta_rel=1e-6)
    F, T, M = X.shape
    slack = 1e-12 * F * T * M
    trace = [fca.loglik(X, s, delta)]
    cur = {}

    def on_substep(name, st):
        cur["lam"], cur["G"] = st.lam, st.G
        trace.append(fca.loglik(X, st, delta))

    def on_row(f, m, Qn, V):
        lam, G = cur["lam"], cur["G"]
        trace.append(fm.loglik_terms(fm.project(X, Qn), fm.model(lam, G, delta), Qn))

    for _ in range(5):
        s = fca.step(X, s, delta, tie_g=tie_g, on_substep=on_substep, on_row=on_row)
    d = np.diff(trace)
    assert d.min() >= -slack, d.min()
    assert trace[-1] > trace[0]


def test_after_ip_every_channel_is_normalised():
    """After the IP step, (1/T) sum_t x~_ftm / y~_ftm = 1 for every (f, m) (Eq. 20)."""
    X, s, delta = _problem(F=3, T=20, M=3, N=2, seed=46)
    s = fca.step(X, s, delta)
    ratio = np.mean(fm.project(X, s.Q) / fm.model(s.lam, s.G, delta), axis=1)
    np.testing.assert_allclose(ratio, 1.0, rtol=1e-10)


def test_fca_run_is_monotone_and_fits_better_than_its_start():
    X, s, delta = _problem(F=5, T=30, M=2, N=2, seed=47, delta_rel=1e-8)
    _, lls = fca.run(X, s, 30, delta)
    assert np.all(np.diff(lls) >= -1e-12 * abs(lls[-1]))
    assert lls[-1] > lls[0]


@pytest.mark.parametrize("tie_g", [False, True])
def test_tied_g_factor_is_shared_over_frequencies(tie_g):
    """With the tied variant every g~_nf. gets the same factor (the sums of Eq. 21
    also run over f); per-frequency factors differ otherwise."""
    X, s, delta = _problem(F=4, T=10, M=2, N=2, seed=48)
    Xt = fm.project(X, s.Q)
    ratio = fca.update_G(Xt, s, delta, tie_over_f=tie_g) / s.G  # [N, F, M]
    spread = np.max(np.abs(ratio - ratio[:, :1, :]))
    assert (spread < 1e-13) if tie_g else (spread > 1e-3)
