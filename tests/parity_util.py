"""Comparison helpers for the GPU parity tests.

Element by element: every entry of the GPU result must satisfy
    |gpu - ref| <= atol + rtol |ref|,   atol = atol_rel * max|ref|,
so an error confined to a few entries (one frequency's Q_f rows, the
low-energy bins of a separated image) is not diluted by the size of the
tensor.  The message names the worst entry.
"""

from __future__ import annotations

import numpy as np


def assert_close(name: str, got, ref, rtol: float, atol_rel: float) -> float:
    """Element-wise check; returns the largest |gpu - ref| / (atol + rtol |ref|)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    atol = atol_rel * scale
    err = np.abs(got - ref)
    bound = atol + rtol * np.abs(ref)
    if ref.size == 0:
        return 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0), np.where(err > 0, np.inf, 0.0))
    worst = float(np.max(ratio))
    if not worst <= 1.0 or not np.all(np.isfinite(got)):
        i = np.unravel_index(int(np.nanargmax(np.where(np.isfinite(ratio), ratio, np.inf))), ref.shape)
        bad = int(np.count_nonzero(~(err <= bound)))
        raise AssertionError(
            f"{name}: {bad} of {ref.size} entries outside |d| <= {atol:.3e} + {rtol:.1e}|ref|; "
            f"worst at {tuple(int(j) for j in i)}: gpu {got[i]!r}, ref {ref[i]!r}, |d| {err[i]:.3e}")
    return worst


def rel_norm(a, b) -> float:
    """||a - b|| / ||b|| over the whole tensor (used for reported error figures)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b) -> float:
    """max |a - b| / max |b|: the largest entry error relative to the tensor's scale."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# FP64 path: per entry, relative 1e-10 with a floor of 1e-13 of the tensor's
# largest magnitude.
FP64 = dict(rtol=1e-10, atol_rel=1e-13)
