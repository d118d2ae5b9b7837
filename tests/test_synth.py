"""The seeded input generator: determinism and the stated distributions."""

import numpy as np

from paper_1903_03237_amd import synth


def test_seeded_determinism():
    a = synth.make_mixture(5, 7, 3, 2, 2, dof=6, seed=3, gain=True)
    b = synth.make_mixture(5, 7, 3, 2, 2, dof=6, seed=3, gain=True)
    c = synth.make_mixture(5, 7, 3, 2, 2, dof=6, seed=4, gain=True)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_init_state():
    W0, H0, G0, Q0 = synth.make_init(4, 6, 3, 2, 5, seed=1)
    assert W0.shape == (2, 5, 4) and H0.shape == (2, 5, 6)
    assert G0.shape == (2, 4, 3) and Q0.shape == (4, 3, 3)
    assert W0.min() >= 0.1 and W0.max() < 1.0
    np.testing.assert_array_equal(G0, 1.0 / 3)
    np.testing.assert_array_equal(Q0, np.broadcast_to(np.eye(3), (4, 3, 3)))


def test_complex_gaussian_and_wishart_moments():
    rng = np.random.default_rng(0)
    z = synth._cn(rng, 200000)
    assert abs(np.mean(np.abs(z) ** 2) - 1) < 0.01
    assert abs(np.mean(z.real * z.imag)) < 0.01
    Z = synth._cn(rng, (4000, 3, 6))
    R = Z @ np.swapaxes(Z.conj(), 1, 2) / 6
    np.testing.assert_allclose(R.mean(axis=0), np.eye(3), atol=0.03)


def test_noise_level():
    """Diffuse noise at -5 dB: removing it drops the power by 10^(-0.5)."""
    clean = synth.make_mixture(33, 400, 4, 2, 3, dof=8, seed=9, gain=True)
    noisy = synth.make_mixture(33, 400, 4, 2, 3, dof=8, seed=9, gain=True, noise_db=-5.0)
    pc = np.mean(np.abs(clean) ** 2)
    pn = np.mean(np.abs(noisy - clean) ** 2)
    assert abs(10 * np.log10(pn / pc) + 5.0) < 0.1


def test_delta():
    X = np.full((2, 2, 2), 2.0 + 0j)
    assert synth.delta_for(X, 1e-8) == 4e-8
    assert synth.delta_for(X, 0.0) == 0.0
