"""FP64 CPU oracle for FastMNMF (Sekiguchi et al., "Fast Multichannel Source
Separation Based on Jointly Diagonalizable Spatial Covariance Matrices").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, constants or
helpers with the HIP implementation under ``paper_1903_03237_amd/``.

Modules
-------
fastmnmf   the method itself, step by step in the paper's order and notation
           (Sec. III-A/B: Eqs. (9), (17)-(21), (23)-(24)), plus the
           multichannel Wiener filter of Eq. (3) in the jointly
           diagonalised form obtained by substituting Eq. (16).
fastfca    FastFCA (Sec. III-C): the same spatial model and IP step with the
           unconstrained source model, lambda updated by Eq. (22).
fullrank   brute-force companions on explicit M x M matrices (Eqs. (1)-(4),
           (10)-(11)) used to pin the fast formulas on tiny inputs.
"""

from . import fastfca, fastmnmf, fullrank  # noqa: F401
