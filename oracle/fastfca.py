"""FastFCA, written out in FP64 on the CPU (Sec. III-C, "FastFCA").

TEST INFRASTRUCTURE ONLY (see the package docstring).

FastFCA keeps the jointly diagonalisable spatial model of FastMNMF (Eq. 16,
the G~ update of Eq. 21 and the IP update of Q of Eqs. 18-20) and replaces
the NMF source model by the unconstrained one (Sec. III-B): every PSD lambda_ftn is a free
parameter, updated by the multiplicative rule of Eq. (22).  The paper
estimates it with the MM algorithm and the IP step, which is what this
module does.

Notation as in ``fastmnmf``; the state is
  lam [F, T, N]   PSDs lambda_ftn (free, > 0)
  G   [N, F, M]   g~_nfm
  Q   [F, M, M]   Q_f, row m = q_fm^H

Readings where the paper is silent (the same as for FastMNMF):
  * one iteration updates lambda (Eq. 22), then G~ (Eq. 21), then every row
    of every Q_f by IP (Eqs. 18-20), then re-projects X~; y~ is rebuilt from
    the current parameters before every update;
  * Eq. (22) updates all sources of a bin at once, from one y~ (the MM bound
    is built at the current parameters and then maximised over all lambda);
  * the floor delta and the log-likelihood are those of ``fastmnmf``.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import fastmnmf as fm


@dataclasses.dataclass
class State:
    """Parameters of FastFCA: lambda (unconstrained), G~ and Q (Eq. 16)."""

    lam: np.ndarray  # [F, T, N] float64
    G: np.ndarray  # [N, F, M] float64
    Q: np.ndarray  # [F, M, M] complex128

    def copy(self) -> "State":
        return State(self.lam.copy(), self.G.copy(), self.Q.copy())


def terms_lam(Xt: np.ndarray, lam: np.ndarray, G: np.ndarray, delta: float = 0.0):
    """Numerator and denominator of Eq. (22), each [F, T, N]:
    sum_m g~_nfm x~_ftm / y~_ftm^2  and  sum_m g~_nfm / y~_ftm."""
    Yt = fm.model(lam, G, delta)
    num = np.einsum("nfm,ftm->ftn", G, Xt / Yt ** 2, optimize=True)
    den = np.einsum("nfm,ftm->ftn", G, 1.0 / Yt, optimize=True)
    return num, den


def update_lam(Xt: np.ndarray, lam: np.ndarray, G: np.ndarray, delta: float = 0.0) -> np.ndarray:
    """Eq. (22): lambda_ftn <- lambda_ftn sqrt(sum_m g~ x~/y~^2 / sum_m g~/y~)."""
    num, den = terms_lam(Xt, lam, G, delta)
    return lam * np.sqrt(num / den)


def update_G(Xt: np.ndarray, s: State, delta: float = 0.0, tie_over_f: bool = False) -> np.ndarray:
    """Eq. (21) with the unconstrained lambda."""
    num, den = fm.terms_G_psd(Xt, s.lam, s.G, delta, tie_over_f)
    return s.G * np.sqrt(num / den)


def loglik(X: np.ndarray, s: State, delta: float = 0.0) -> float:
    """Eq. (17) (constant -F T M log(pi) omitted)."""
    return fm.loglik_terms(fm.project(X, s.Q), fm.model(s.lam, s.G, delta), s.Q)


def step(X: np.ndarray, s: State, delta: float = 0.0, *, tie_g: bool = False,
         on_substep=None, on_row=None) -> State:
    """One FastFCA iteration: lambda (22) -> G~ (21) -> Q by IP (18-20).

    ``on_substep(name, state)`` is called after lambda, G and Q.
    """
    Xt = fm.project(X, s.Q)
    s = s.copy()
    s.lam = update_lam(Xt, s.lam, s.G, delta)
    if on_substep is not None:
        on_substep("lam", s)
    s.G = update_G(Xt, s, delta, tie_over_f=tie_g)
    if on_substep is not None:
        on_substep("G", s)
    Yt = fm.model(s.lam, s.G, delta)
    s.Q = fm.update_Q(X, s.Q, Yt, on_row=on_row)
    if on_substep is not None:
        on_substep("Q", s)
    return s


def run(X: np.ndarray, s: State, n_iter: int, delta: float = 0.0, **kw):
    """n_iter iterations from ``s``; returns (final state, [L_0, ..., L_n])."""
    lls = [loglik(X, s, delta)]
    for _ in range(n_iter):
        s = step(X, s, delta, **kw)
        lls.append(loglik(X, s, delta))
    return s, lls


def separate(X: np.ndarray, s: State, delta: float = 0.0) -> np.ndarray:
    """The multichannel Wiener filter (Eq. 3 with Eq. 16) with the unconstrained
    lambda.  Returns [N, F, T, M] complex128."""
    return fm.separate_psd(X, s.lam, s.G, s.Q, delta)
