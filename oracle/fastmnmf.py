"""FastMNMF, written out in FP64 on the CPU, in the paper's order and notation.

TEST INFRASTRUCTURE ONLY (see the package docstring).  It is deliberately
plain: NumPy complex128/float64, library primitives (einsum, matmul, solve,
slogdet, inv) as single steps, no blocking or fusion beyond what the
formulas state.

Notation (Sec. II-A, III-A of the paper):
  X   [F, T, M] complex   observed multichannel spectra x_ft
  W   [N, K, F]           NMF bases w_nkf              (Eq. 9)
  H   [N, K, T]           NMF activations h_nkt        (Eq. 9)
  G   [N, F, M]           diagonal SCM gains g~_nfm    (Eq. 16)
  Q   [F, M, M] complex   diagonalisers Q_f, row m of Q_f is q_fm^H (Eq. 16)
  lam [F, T, N]           PSDs lambda_ftn              (Eq. 9)
  Xt  [F, T, M]           x~_ftm = |(Q_f x_ft)_m|^2    (definition under Eq. 17)
  Yt  [F, T, M]           y~_ftm = sum_n lambda_ftn g~_nfm (+ delta)

Readings where the paper is silent:
  * one iteration updates W (Eq. 23), then H (Eq. 24), then G~ (Eq. 21),
    then every row of every Q_f by iterative projection (Eqs. 18-20), then
    re-projects X~; the model Y~ is rebuilt from the current parameters
    before every update (the MM bound is only tight there);
  * the IP sweep is sequential over m = 1..M, each solve using the Q_f whose
    earlier rows were already replaced;
  * the additive floor ``delta`` (default 0) is a fixed model component,
    y~ = sum_n lambda g~ + delta; with delta = 0 this is the paper verbatim;
  * the log-likelihood is Eq. (17) without the constant -F T M log(pi);
    log|Q_f Q_f^H| is evaluated as log|det Q_f|^2.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class State:
    """Parameters of FastMNMF: W, H (Eq. 9), G~ and Q (Eq. 16)."""

    W: np.ndarray  # [N, K, F] float64
    H: np.ndarray  # [N, K, T] float64
    G: np.ndarray  # [N, F, M] float64
    Q: np.ndarray  # [F, M, M] complex128, row m = q_fm^H

    def copy(self) -> "State":
        return State(self.W.copy(), self.H.copy(), self.G.copy(), self.Q.copy())


# ----------------------------------------------------------------------------
# The model (Eq. 9, definitions under Eq. 17)
# ----------------------------------------------------------------------------

def psd(W: np.ndarray, H: np.ndarray) -> np.ndarray:
    """NMF source model, Eq. (9): lambda_ftn = sum_k w_nkf h_nkt.  -> [F, T, N]."""
    return np.einsum("nkf,nkt->ftn", W, H, optimize=True)


def model(lam: np.ndarray, G: np.ndarray, delta: float = 0.0) -> np.ndarray:
    """Diagonal model under Eq. (17): y~_ftm = sum_n lambda_ftn g~_nfm (+ delta)."""
    return np.einsum("ftn,nfm->ftm", lam, G, optimize=True) + delta


def project(X: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Projection under Eq. (17): x~_ft = |Q_f x_ft|^(o2), i.e. x~_ftm = |q_fm^H x_ft|^2."""
    Y = np.einsum("fmj,ftj->ftm", Q, X, optimize=True)
    return Y.real ** 2 + Y.imag ** 2


def log_det_QQH(Q: np.ndarray) -> np.ndarray:
    """log|Q_f Q_f^H| = log|det Q_f|^2 for every f (last term of Eq. 17).  -> [F]."""
    _, logabs = np.linalg.slogdet(Q)
    return 2.0 * logabs


def loglik_terms(Xt: np.ndarray, Yt: np.ndarray, Q: np.ndarray) -> float:
    """Eq. (17) from its pieces: sum_ftm(-x~/y~ - log y~) + T sum_f log|Q_f Q_f^H|."""
    T = Xt.shape[1]
    return float(np.sum(-Xt / Yt - np.log(Yt)) + T * np.sum(log_det_QQH(Q)))


def loglik(X: np.ndarray, s: State, delta: float = 0.0) -> float:
    """Log-likelihood of Eq. (17) (constant -FTM log pi omitted)."""
    Xt = project(X, s.Q)
    Yt = model(psd(s.W, s.H), s.G, delta)
    return loglik_terms(Xt, Yt, s.Q)


# ----------------------------------------------------------------------------
# Multiplicative updates (Eqs. 21, 23, 24)
# ----------------------------------------------------------------------------

def nmf_terms(Xt: np.ndarray, Yt: np.ndarray, G: np.ndarray):
    """The m-sums inside Eqs. (23)-(24), per source and bin:

    A_nft = sum_m g~_nfm x~_ftm / y~_ftm^2   (numerator weight)
    B_nft = sum_m g~_nfm / y~_ftm            (denominator weight)
    """
    A = np.einsum("nfm,ftm->nft", G, Xt / Yt ** 2, optimize=True)
    B = np.einsum("nfm,ftm->nft", G, 1.0 / Yt, optimize=True)
    return A, B


def terms_W(Xt, s: State, delta: float = 0.0):
    """Numerator and denominator of Eq. (23), each [N, K, F]:
    sum_tm h_nkt g~_nfm x~_ftm / y~_ftm^2  and  sum_tm h_nkt g~_nfm / y~_ftm."""
    Yt = model(psd(s.W, s.H), s.G, delta)
    A, B = nmf_terms(Xt, Yt, s.G)
    num = np.einsum("nkt,nft->nkf", s.H, A, optimize=True)
    den = np.einsum("nkt,nft->nkf", s.H, B, optimize=True)
    return num, den


def update_W(Xt, s: State, delta: float = 0.0) -> np.ndarray:
    """Eq. (23): w_nkf <- w_nkf sqrt(sum_tm h g~ x~/y~^2 / sum_tm h g~ / y~)."""
    num, den = terms_W(Xt, s, delta)
    return s.W * np.sqrt(num / den)


def terms_H(Xt, s: State, delta: float = 0.0):
    """Numerator and denominator of Eq. (24), each [N, K, T]:
    sum_fm w_nkf g~_nfm x~_ftm / y~_ftm^2  and  sum_fm w_nkf g~_nfm / y~_ftm."""
    Yt = model(psd(s.W, s.H), s.G, delta)
    A, B = nmf_terms(Xt, Yt, s.G)
    num = np.einsum("nkf,nft->nkt", s.W, A, optimize=True)
    den = np.einsum("nkf,nft->nkt", s.W, B, optimize=True)
    return num, den


def update_H(Xt, s: State, delta: float = 0.0) -> np.ndarray:
    """Eq. (24): h_nkt <- h_nkt sqrt(sum_fm w g~ x~/y~^2 / sum_fm w g~ / y~)."""
    num, den = terms_H(Xt, s, delta)
    return s.H * np.sqrt(num / den)


def terms_G(Xt, s: State, delta: float = 0.0, tie_over_f: bool = False):
    """Numerator and denominator of Eq. (21), each [N, F, M]:
    sum_t lambda_ftn x~_ftm / y~_ftm^2  and  sum_t lambda_ftn / y~_ftm.

    ``tie_over_f`` gives the frequency-independent variant g~_nm: both sums
    are also taken over f (and broadcast back over f).  Not the paper's default.
    """
    return terms_G_psd(Xt, psd(s.W, s.H), s.G, delta, tie_over_f)


def terms_G_psd(Xt, lam, G, delta: float = 0.0, tie_over_f: bool = False):
    """The sums of Eq. (21) for any source model lambda [F, T, N] (NMF or
    unconstrained): sum_t lambda x~/y~^2 and sum_t lambda/y~, each [N, F, M]."""
    Yt = model(lam, G, delta)
    num = np.einsum("ftn,ftm->nfm", lam, Xt / Yt ** 2, optimize=True)
    den = np.einsum("ftn,ftm->nfm", lam, 1.0 / Yt, optimize=True)
    if tie_over_f:
        num = np.broadcast_to(num.sum(axis=1, keepdims=True), num.shape)
        den = np.broadcast_to(den.sum(axis=1, keepdims=True), den.shape)
    return num, den


def update_G(Xt, s: State, delta: float = 0.0, tie_over_f: bool = False) -> np.ndarray:
    """Eq. (21): g~_nfm <- g~_nfm sqrt(sum_t lambda x~/y~^2 / sum_t lambda / y~)."""
    num, den = terms_G(Xt, s, delta, tie_over_f)
    return s.G * np.sqrt(num / den)


# ----------------------------------------------------------------------------
# Iterative projection for Q_f (Eqs. 18-20)
# ----------------------------------------------------------------------------

def spatial_cov(X: np.ndarray, Yt: np.ndarray) -> np.ndarray:
    """Eq. (18): V_fm = (1/T) sum_t x_ft x_ft^H / y~_ftm.  -> [F, M, M, M] (f, m, i, j)."""
    T = X.shape[1]
    R = 1.0 / Yt  # [F, T, M]
    # V[f, m] = X_f^T diag(R[f, :, m]) conj(X_f) / T, one batched product per m.
    XT = np.swapaxes(X, 1, 2)  # [F, M(i), T]
    V = np.empty((X.shape[0], X.shape[2], X.shape[2], X.shape[2]), dtype=np.complex128)
    for m in range(X.shape[2]):
        V[:, m] = np.matmul(XT * R[:, None, :, m], X.conj()) / T
    return V


def ip_row(Qf: np.ndarray, Vfm: np.ndarray, m: int) -> np.ndarray:
    """One IP update of row m of Q_f (Eqs. 19-20); returns the new Q_f.

    q_fm <- (Q_f V_fm)^{-1} e_m ;  q_fm <- q_fm / sqrt(q_fm^H V_fm q_fm) ;
    row m of Q_f := q_fm^H.
    """
    M = Qf.shape[0]
    e = np.zeros(M, dtype=np.complex128)
    e[m] = 1.0
    q = np.linalg.solve(Qf @ Vfm, e)
    quad = np.real(np.vdot(q, Vfm @ q))  # q^H V q, real for Hermitian V
    q = q / np.sqrt(quad)
    out = Qf.copy()
    out[m, :] = q.conj()
    return out


def update_Q(X: np.ndarray, Q: np.ndarray, Yt: np.ndarray, on_row=None) -> np.ndarray:
    """All rows of all Q_f by IP, sequential over m (Eqs. 18-20).

    ``on_row(f, m, Q_f_new, V_fm)``, if given, is called after each row update
    (used by tests to check the per-row identities and monotonicity).
    """
    V = spatial_cov(X, Yt)
    Qn = Q.copy()
    for f in range(Q.shape[0]):
        for m in range(Q.shape[1]):
            Qn[f] = ip_row(Qn[f], V[f, m], m)
            if on_row is not None:
                on_row(f, m, Qn, V[f, m])
    return Qn


# ----------------------------------------------------------------------------
# Optional scale normalisation (not in the paper; leaves Eq. 17 unchanged)
# ----------------------------------------------------------------------------

def normalize(s: State) -> State:
    """Rescale the redundant scales without changing y~ / x~ ratios or Eq. (17).

    phi_f = (1/M) sum_ij |Q_f,ij|^2 ; Q_f /= sqrt(phi_f) ; g~_nf. /= phi_f
    mu_nf = sum_m g~_nfm ; g~ /= mu ; w_n.f *= mu_nf
    nu_nk = sum_f w_nkf ; w /= nu ; h_nk. *= nu_nk
    """
    M = s.Q.shape[1]
    phi = np.sum(np.abs(s.Q) ** 2, axis=(1, 2)) / M  # [F]
    Q = s.Q / np.sqrt(phi)[:, None, None]
    G = s.G / phi[None, :, None]
    mu = G.sum(axis=2)  # [N, F]
    G = G / mu[:, :, None]
    W = s.W * mu[:, None, :]
    nu = W.sum(axis=2)  # [N, K]
    W = W / nu[:, :, None]
    H = s.H * nu[:, :, None]
    return State(W, H, G, Q)


# ----------------------------------------------------------------------------
# The paper's initialisation of the spatial model (Sec. IV-A)
# ----------------------------------------------------------------------------

def init_from_scm(X: np.ndarray, N: int):
    """G_1f = (1/T) sum_t x_ft x_ft^H (average observed SCM), G_nf = I for
    n >= 2; Q_f and g~ from the spectral decomposition G_1f = U Diag(e) U^H:
    Q_f = U^H (rows by ascending eigenvalue), g~_1f = e, g~_nf = 1.
    Returns (G [N, F, M], Q [F, M, M])."""
    F, T, M = X.shape
    R = np.einsum("fti,ftj->fij", X, X.conj(), optimize=True) / T
    e, U = np.linalg.eigh(R)  # ascending eigenvalues, eigenvectors in columns
    Q = np.conj(np.swapaxes(U, 1, 2))
    G = np.ones((N, F, M))
    G[0] = e
    return G, Q


# ----------------------------------------------------------------------------
# One full iteration and a run
# ----------------------------------------------------------------------------

def step(X: np.ndarray, s: State, delta: float = 0.0, *, tie_g: bool = False,
         norm: bool = False, on_substep=None, on_row=None) -> State:
    """One FastMNMF iteration: W (23) -> H (24) -> G~ (21) -> Q by IP (18-20).

    x~ is the projection with the Q the iteration starts from; y~ is rebuilt
    before every update.  ``on_substep(name, state)`` is called after W, H, G
    and Q so tests can evaluate Eq. (17) in between.
    """
    Xt = project(X, s.Q)
    s = s.copy()
    s.W = update_W(Xt, s, delta)
    if on_substep is not None:
        on_substep("W", s)
    s.H = update_H(Xt, s, delta)
    if on_substep is not None:
        on_substep("H", s)
    s.G = update_G(Xt, s, delta, tie_over_f=tie_g)
    if on_substep is not None:
        on_substep("G", s)
    Yt = model(psd(s.W, s.H), s.G, delta)
    s.Q = update_Q(X, s.Q, Yt, on_row=on_row)
    if on_substep is not None:
        on_substep("Q", s)
    if norm:
        s = normalize(s)
    return s


def run(X: np.ndarray, s: State, n_iter: int, delta: float = 0.0, **kw):
    """n_iter iterations from ``s``; returns (final state, [L_0, L_1, ..., L_n])."""
    lls = [loglik(X, s, delta)]
    for _ in range(n_iter):
        s = step(X, s, delta, **kw)
        lls.append(loglik(X, s, delta))
    return s, lls


# ----------------------------------------------------------------------------
# Separation: the multichannel Wiener filter of Eq. (3) with Eq. (16)
# ----------------------------------------------------------------------------

def separate(X: np.ndarray, s: State, delta: float = 0.0) -> np.ndarray:
    """Posterior mean of every source image, Eq. (3), in jointly diagonalised form.

    With Y_ftn = lambda_ftn Q_f^-1 Diag(g~_nf) Q_f^-H and
    Y_ft = Q_f^-1 Diag(y~_ft) Q_f^-H (Eq. 16 substituted into Eq. 3):
        x^_ftn = Q_f^-1 Diag(lambda_ftn g~_nf / y~_ft) Q_f x_ft.
    Returns [N, F, T, M] complex128.
    """
    return separate_psd(X, psd(s.W, s.H), s.G, s.Q, delta)


def separate_psd(X: np.ndarray, lam: np.ndarray, G: np.ndarray, Q: np.ndarray, delta: float = 0.0) -> np.ndarray:
    """The filter of ``separate`` for any source model lambda [F, T, N]."""
    Yt = model(lam, G, delta)  # [F, T, M]
    Qinv = np.linalg.inv(Q)  # [F, M, M]
    Z = np.einsum("fmj,ftj->ftm", Q, X, optimize=True)  # Q_f x_ft
    out = np.empty((G.shape[0],) + X.shape, dtype=np.complex128)
    for n in range(G.shape[0]):
        gain = lam[:, :, n, None] * G[n][:, None, :] / Yt  # [F, T, M]
        out[n] = np.einsum("fij,ftj->fti", Qinv, gain * Z, optimize=True)
    return out
