"""Brute-force full-rank companions of the fast formulas (tiny inputs only).

TEST INFRASTRUCTURE ONLY.  These build the explicit M x M matrices of the
full-rank spatial model (Sec. II-A) and evaluate the paper's full-rank
formulas directly, so that the jointly diagonalised shortcuts of Sec. III can
be checked against them:

  G_nf      = Q_f^-1 Diag(g~_nf) Q_f^-H              (Eq. 16 solved for G_nf)
  Y_ft      = sum_n lambda_ftn G_nf (+ delta Q_f^-1 Q_f^-H for the floor)
  loglik    = -sum_ft [ tr(X_ft Y_ft^-1) + log det Y_ft ]           (Eq. 4)
  mwf       = Y_ftn Y_ft^-1 x_ft                                      (Eq. 3)
  traces    = tr(G_nf Y^-1 X Y^-1), tr(G_nf Y^-1)          (inside Eqs. 10-11)
"""

from __future__ import annotations

import numpy as np


def scm_from_diag(Q: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Full-rank SCMs implied by Eq. (16): G_nf = Q_f^-1 Diag(g~_nf) Q_f^-H.  -> [N, F, M, M]."""
    Qi = np.linalg.inv(Q)  # [F, M, M]
    return np.einsum("fij,nfj,fkj->nfik", Qi, G, Qi.conj())


def floor_scm(Q: np.ndarray, delta: float) -> np.ndarray:
    """The covariance contributed by the additive floor delta in y~: delta Q_f^-1 Q_f^-H.  -> [F, M, M]."""
    Qi = np.linalg.inv(Q)
    return delta * np.einsum("fij,fkj->fik", Qi, Qi.conj())


def mixture_cov(lam: np.ndarray, Gfull: np.ndarray, extra=None) -> np.ndarray:
    """Eq. (2): Y_ft = sum_n lambda_ftn G_nf (+ extra_f).  -> [F, T, M, M]."""
    Y = np.einsum("ftn,nfij->ftij", lam, Gfull)
    if extra is not None:
        Y = Y + extra[:, None, :, :]
    return Y


def loglik_fullrank(X: np.ndarray, lam: np.ndarray, Gfull: np.ndarray, extra=None) -> float:
    """Eq. (4): -sum_ft [ tr(X_ft Y_ft^-1) + log det Y_ft ], with X_ft = x_ft x_ft^H."""
    Y = mixture_cov(lam, Gfull, extra)
    Yi = np.linalg.inv(Y)
    quad = np.einsum("fti,ftij,ftj->ft", X.conj(), Yi, X).real  # tr(x x^H Y^-1) = x^H Y^-1 x
    _, logdet = np.linalg.slogdet(Y)
    return float(-np.sum(quad + logdet))


def mwf_fullrank(X: np.ndarray, lam: np.ndarray, Gfull: np.ndarray, extra=None) -> np.ndarray:
    """Eq. (3): x_ftn = Y_ftn Y_ft^-1 x_ft with Y_ftn = lambda_ftn G_nf.  -> [N, F, T, M]."""
    Y = mixture_cov(lam, Gfull, extra)
    z = np.linalg.solve(Y, X[..., None])[..., 0]  # Y_ft^-1 x_ft
    return np.einsum("ftn,nfij,ftj->nfti", lam, Gfull, z)


def mnmf_traces(X: np.ndarray, lam: np.ndarray, Gfull: np.ndarray, extra=None):
    """Per (n, f, t): tr(G_nf Y^-1 X_ft Y^-1) and tr(G_nf Y^-1) (inside Eqs. 10-11)."""
    Y = mixture_cov(lam, Gfull, extra)
    Yi = np.linalg.inv(Y)
    z = np.einsum("ftij,ftj->fti", Yi, X)  # Y^-1 x
    # tr(G Y^-1 x x^H Y^-1) = (Y^-1 x)^H G (Y^-1 x)
    num = np.einsum("fti,nfij,ftj->nft", z.conj(), Gfull, z).real
    den = np.einsum("nfij,ftji->nft", Gfull, Yi).real
    return num, den
