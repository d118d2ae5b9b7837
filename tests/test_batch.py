"""Batched iterations (fmnmf_step_batch) against each context stepped alone.

Contexts of different shapes and classes (M, N, K, T, precision) are stepped
together; each must end in exactly the state it reaches alone with
fmnmf_step, because a batched launch runs the same per-context arithmetic.
"""

import numpy as np
import pytest

from paper_1903_03237_amd import synth

pytestmark = pytest.mark.gpu

# (F, T, M, N, K, precision)
CASES = [
    (33, 90, 2, 2, 8, "fp32"),
    (33, 150, 2, 2, 8, "fp32"),    # same class as the first, other T
    (40, 70, 4, 3, 16, "fp32"),
    (21, 37, 8, 5, 32, "bf16"),
    (50, 64, 8, 5, 32, "bf16"),    # same class, other F / T
    (17, 130, 3, 4, 20, "fp64"),
]


def _make(device, case, seed, stream=None):
    import torch

    from paper_1903_03237_amd import fmnmf

    F, T, M, N, K, p = case
    X, init, delta = synth.random_problem(F, T, M, N, K, seed=seed, delta_rel=1e-8, random_q=True)
    dt = np.complex128 if p == "fp64" else np.complex64
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(dt))).to(device)
    return fmnmf.FastMNMF(Xd, N, K, init, precision=p, delta=delta, stream=stream)


def _state(m):
    W, H, G, Q = m.get_state()
    return W, H, G, Q, m.loglik()


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_alone(device, graph, monkeypatch):
    from paper_1903_03237_amd import fmnmf

    if not graph:
        monkeypatch.setenv("FMNMF_NO_GRAPH", "1")
    alone = []
    for i, c in enumerate(CASES):
        m = _make(device, c, 1000 + i)
        m.step(4)
        alone.append(_state(m))
        m.close()
    mix = [_make(device, c, 1000 + i) for i, c in enumerate(CASES)]
    fmnmf.step_batch(mix, 3)
    fmnmf.step_batch(mix[::-1], 1)  # another composition and order
    for m, ref in zip(mix, alone):
        got = _state(m)
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(np.asarray(g), np.asarray(r))
    for m in mix:
        m.close()


def test_batch_rejects_duplicates(device):
    from paper_1903_03237_amd import fmnmf

    m = _make(device, CASES[0], 7)
    with pytest.raises(fmnmf.FmnmfError):
        fmnmf.step_batch([m, m], 1)
    m.close()
