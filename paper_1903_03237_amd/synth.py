"""Seeded synthetic mixtures and initial states.

This module only draws random inputs; it holds none of the separation
method's arithmetic.  Both the GPU path's tests/bench and the CPU oracle take
their inputs from here.

Mixture recipe (the paper's CHiME-3 speech recordings are not available, so
NMF-structured Gaussian mixtures of the same shape stand in for them):

  * per source n: W ~ Gamma(0.5, 1) [F, K], H ~ Gamma(0.5, 1) [K, T],
    PSD p_ft = (W H)_ft, optionally times a source gain a_n ~ Gamma(1, 1);
  * per source and frequency a full-rank SCM R_nf = (1/dof) Z Z^H with
    Z in C^{M x dof} i.i.d. CN(0, 1) (complex Wishart);
  * source image x_ftn = sqrt(p_ft) chol(R_nf) z, z ~ CN(0, I_M);
  * mixture x_ft = sum_n x_ftn, optionally plus spatially white, spectrally
    flat diffuse noise CN(0, s2 I_M) at ``noise_db`` dB below the mean
    per-channel source power.

Initial state: Q_f = I, g~_nfm = 1/M, W0, H0 ~ Uniform[0.1, 1).
"""

from __future__ import annotations

import dataclasses

import numpy as np

SEED_BASE = 190303237


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    F: int
    T: int
    M: int
    N: int
    K: int
    dof: int
    iters: int
    gain: bool = False
    noise_db: float | None = None
    delta_rel: float = 0.0
    precision: str = "fp64"


# The benchmark workloads.  "small" is the oracle-sized case; "fp64_513x1000"
# the plain FP64 case; "fp32_m8_513x3000" the headline shape (M=8 microphones,
# F=513 bins of a 1024-point STFT, T=3000 frames); "bf16_m8_1025x4000" the
# largest mixed-precision case.
CONFIGS = {
    1: Config("small_m2_129x100", F=129, T=100, M=2, N=2, K=4, dof=4, iters=10),
    2: Config("fp64_m4_513x1000", F=513, T=1000, M=4, N=3, K=16, dof=8, iters=100,
              gain=True),
    3: Config("fp32_m8_513x3000", F=513, T=3000, M=8, N=5, K=32, dof=16, iters=100,
              gain=True, noise_db=-5.0, delta_rel=1e-8, precision="fp32"),
    4: Config("bf16_m8_1025x4000", F=1025, T=4000, M=8, N=6, K=64, dof=16, iters=200,
              gain=True, delta_rel=1e-8, precision="bf16"),
}


def _cn(rng: np.random.Generator, shape) -> np.ndarray:
    """i.i.d. circular complex Gaussian CN(0, 1)."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)


def make_mixture(F: int, T: int, M: int, N: int, K: int, *, dof: int, seed: int,
                 gain: bool = False, noise_db: float | None = None) -> np.ndarray:
    """Seeded mixture X [F, T, M] complex128 following the module recipe."""
    rng = np.random.default_rng(seed)
    X = np.zeros((F, T, M), dtype=np.complex128)
    for _ in range(N):
        Wt = rng.gamma(0.5, 1.0, size=(F, K))
        Ht = rng.gamma(0.5, 1.0, size=(K, T))
        p = Wt @ Ht  # [F, T]
        if gain:
            p = p * rng.gamma(1.0, 1.0)
        Z = _cn(rng, (F, M, dof))
        R = Z @ np.swapaxes(Z.conj(), 1, 2) / dof  # [F, M, M] Wishart
        L = np.linalg.cholesky(R)
        z = _cn(rng, (F, T, M))
        X += np.sqrt(p)[:, :, None] * np.einsum("fij,ftj->fti", L, z)
    if noise_db is not None:
        s2 = float(np.mean(np.abs(X) ** 2)) * 10.0 ** (noise_db / 10.0)
        X += np.sqrt(s2) * _cn(rng, (F, T, M))
    return X


def make_init(F: int, T: int, M: int, N: int, K: int, *, seed: int):
    """Initial (W0 [N,K,F], H0 [N,K,T], G0 [N,F,M], Q0 [F,M,M] complex)."""
    rng = np.random.default_rng(seed)
    W0 = rng.uniform(0.1, 1.0, size=(N, K, F))
    H0 = rng.uniform(0.1, 1.0, size=(N, K, T))
    G0 = np.full((N, F, M), 1.0 / M)
    Q0 = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    return W0, H0, G0, Q0


def delta_for(X: np.ndarray, rel: float) -> float:
    """Additive model floor delta = rel * mean_ftm |x_ftm|^2 (0 when rel == 0)."""
    if rel == 0.0:
        return 0.0
    return float(rel * np.mean(X.real ** 2 + X.imag ** 2))


def workload(cfg: int | Config, request: int = 0, *, T: int | None = None):
    """(X, (W0, H0, G0, Q0), delta) for a configuration, seeded by config and request."""
    c = CONFIGS[cfg] if isinstance(cfg, int) else cfg
    idx = cfg if isinstance(cfg, int) else 0
    T = c.T if T is None else T
    X = make_mixture(c.F, T, c.M, c.N, c.K, dof=c.dof,
                     seed=SEED_BASE + 1000 * idx + request, gain=c.gain,
                     noise_db=c.noise_db)
    init = make_init(c.F, T, c.M, c.N, c.K, seed=SEED_BASE + 1000 * idx + request + 500)
    return X, init, delta_for(X, c.delta_rel)


def random_problem(F: int, T: int, M: int, N: int, K: int, *, seed: int,
                   dof: int | None = None, delta_rel: float = 0.0, random_q: bool = False):
    """A small seeded problem for tests: mixture + init (+ optionally a random
    well-conditioned Q0 and perturbed G0 so that no symmetry hides an index error)."""
    X = make_mixture(F, T, M, N, K, dof=dof or max(2 * M, 2), seed=seed, gain=True)
    W0, H0, G0, Q0 = make_init(F, T, M, N, K, seed=seed + 500)
    if random_q:
        rng = np.random.default_rng(seed + 777)
        Q0 = Q0 + 0.3 * _cn(rng, (F, M, M))
        G0 = G0 * rng.uniform(0.5, 1.5, size=G0.shape)
    return X, (W0, H0, G0, Q0), delta_for(X, delta_rel)


def make_fca_init(F: int, T: int, M: int, N: int, *, seed: int):
    """Initial state of the unconstrained source model (FastFCA):
    (lam0 [N,F,T] ~ U[0.1, 1), G0 [N,F,M] = 1/M, Q0 = I)."""
    rng = np.random.default_rng(seed)
    lam0 = rng.uniform(0.1, 1.0, size=(N, F, T))
    G0 = np.full((N, F, M), 1.0 / M)
    Q0 = np.broadcast_to(np.eye(M, dtype=np.complex128), (F, M, M)).copy()
    return lam0, G0, Q0


def random_fca_problem(F: int, T: int, M: int, N: int, *, seed: int, dof: int | None = None,
                       delta_rel: float = 0.0, random_q: bool = False):
    """random_problem for FastFCA: mixture + (lam0 [N,F,T], G0, Q0) + delta."""
    X = make_mixture(F, T, M, N, 2, dof=dof or max(2 * M, 2), seed=seed, gain=True)
    lam0, G0, Q0 = make_fca_init(F, T, M, N, seed=seed + 500)
    if random_q:
        rng = np.random.default_rng(seed + 777)
        Q0 = Q0 + 0.3 * _cn(rng, (F, M, M))
        G0 = G0 * rng.uniform(0.5, 1.5, size=G0.shape)
    return X, (lam0, G0, Q0), delta_for(X, delta_rel)


# ----------------------------------------------------------------------------
# Serving workload: many requests of different shapes arriving over time.
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class ServingSpec:
    """One request of the serving workload (no data yet)."""
    rid: int
    arrival: float  # seconds after the start of the run
    M: int
    N: int
    K: int
    T: int


def serving_specs(n: int, rate: float | None, *, seed: int = SEED_BASE + 5000,
                  Ms=(2, 4, 8), Ns=(2, 3, 4, 5), Ks=(8, 16, 32), T_range=(200, 4000)):
    """n request shapes drawn uniformly from the given sets, T ~ U{T_range};
    Poisson arrivals at `rate` requests/s (all at t = 0 when rate is None)."""
    rng = np.random.default_rng(seed)  # shapes: the same whatever the rate
    shapes = [(int(rng.choice(Ms)), int(rng.choice(Ns)), int(rng.choice(Ks)),
               int(rng.integers(T_range[0], T_range[1] + 1))) for _ in range(n)]
    arr = np.random.default_rng(seed + 1)
    gaps = arr.exponential(1.0 / rate, size=n) if rate else np.zeros(n)
    t = np.cumsum(gaps) - gaps[0]
    return [ServingSpec(i, float(t[i]), *shapes[i]) for i in range(n)]


def serving_bases(F: int = 513, T: int = 4000, Ms=(2, 4, 8), *, seed: int = SEED_BASE + 6000):
    """One seeded base mixture per microphone count (3 NMF-structured sources,
    Wishart SCMs with dof = 2M); requests use crops of these."""
    return {M: make_mixture(F, T, M, 3, 16, dof=2 * M, seed=seed + M, gain=True) for M in Ms}


def serving_request(spec: ServingSpec, bases, *, seed: int = SEED_BASE + 7000, delta_rel: float = 1e-8):
    """(X [F, T, M], init, delta) of a request: the first T frames of the base
    mixture for its M (a view, no copy), with its own seeded initial state."""
    X = bases[spec.M][:, :spec.T, :]
    F = X.shape[0]
    init = make_init(F, spec.T, spec.M, spec.N, spec.K, seed=seed + spec.rid)
    return X, init, delta_for(X, delta_rel)
