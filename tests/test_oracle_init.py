"""Pins of the oracle's version of the paper's initialisation (Sec. IV-A):
G_1f = average observed SCM, G_nf = I (n >= 2), Q_f and g~ from the spectral
decomposition of G_1f.

The checks use what the construction must satisfy whatever routine computed
it: Eq. (16) holds for every source (Q_f G_nf Q_f^H = Diag(g~_nf)), Q_f is
unitary, the eigenvalues of a 2 x 2 Hermitian matrix have a closed form, the
reconstruction Q_f^H Diag(g~_1f) Q_f equals the SCM written out as a sum over
frames, and the order is ascending.
"""

import numpy as np
import pytest

from oracle import fastmnmf as fm
from paper_1903_03237_amd import synth


def _scm_loop(X):
    F, T, M = X.shape
    R = np.zeros((F, M, M), dtype=np.complex128)
    for f in range(F):
        for t in range(T):
            R[f] += np.outer(X[f, t], X[f, t].conj())
    return R / T


@pytest.mark.parametrize("M", [1, 2, 3, 5, 8])
def test_init_diagonalises_every_source_scm(M):
    F, T, N = 6, 40, 3
    X = synth.make_mixture(F, T, M, N, 2, dof=2 * M, seed=900 + M, gain=True)
    G, Q = fm.init_from_scm(X, N)
    R = _scm_loop(X)
    eye = np.eye(M)
    for f in range(F):
        np.testing.assert_allclose(Q[f] @ Q[f].conj().T, eye, atol=1e-12)
        scale = np.abs(R[f]).max()
        np.testing.assert_allclose(Q[f] @ R[f] @ Q[f].conj().T, np.diag(G[0, f]), atol=1e-12 * scale)
        np.testing.assert_allclose(Q[f].conj().T @ np.diag(G[0, f]) @ Q[f], R[f], atol=1e-12 * scale)
        for n in range(1, N):  # G_nf = I: Q I Q^H = I = Diag(g~_nf)
            np.testing.assert_allclose(G[n, f], 1.0)
        assert np.all(np.diff(G[0, f]) >= 0)


def test_two_channel_eigenvalues_closed_form():
    X = synth.make_mixture(5, 30, 2, 2, 2, dof=4, seed=950, gain=True)
    G, _ = fm.init_from_scm(X, 2)
    R = _scm_loop(X)
    a, d, b = R[:, 0, 0].real, R[:, 1, 1].real, R[:, 0, 1]
    mid, rad = (a + d) / 2, np.sqrt(((a - d) / 2) ** 2 + np.abs(b) ** 2)
    np.testing.assert_allclose(G[0, :, 0], mid - rad, rtol=1e-12)
    np.testing.assert_allclose(G[0, :, 1], mid + rad, rtol=1e-12)


def test_single_channel_init_is_the_mean_power():
    X = synth.make_mixture(4, 25, 1, 2, 2, dof=2, seed=951, gain=True)
    G, Q = fm.init_from_scm(X, 2)
    np.testing.assert_allclose(G[0, :, 0], np.mean(np.abs(X[:, :, 0]) ** 2, axis=1), rtol=1e-13)
    np.testing.assert_allclose(np.abs(Q[:, 0, 0]), 1.0, rtol=1e-14)


def test_init_then_iterate_is_monotone():
    X = synth.make_mixture(8, 60, 3, 2, 3, dof=6, seed=952, gain=True)
    W0, H0, _, _ = synth.make_init(8, 60, 3, 2, 3, seed=953)
    G0, Q0 = fm.init_from_scm(X, 2)
    _, lls = fm.run(X, fm.State(W0, H0, G0, Q0), 8)
    assert np.all(np.diff(lls) >= -1e-12 * abs(lls[-1]))
