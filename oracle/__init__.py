"""FP64 CPU oracle for Bluebild standard synthesis -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct definition the GPU library
is checked against.  It is imported only by ``tests/``, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``; the product
path (``paper_2310_09200_amd``) never imports, links or calls it, and it shares
no code with that path.  Inputs come from the seeded generators in ``sims``.

Modules
-------
bluebild_ref
    Gram matrix, generalized eigensolve, selection, levels, phases, synthesis
    (two evaluators), and the closed-form images used as pins.
grad_ref
    Analytic FP64 gradient of a weighted image loss w.r.t. (W, lambda, x),
    and central finite differences of the same loss.
levels_ref
    Exact one-dimensional k-means of the eigenvalues and the level intervals
    it gives.
weighting_ref
    Uniform image weighting: uv cell densities and the weighted visibilities.
nufft_ref
    NUFFT synthesis: per-level Gram-corrected visibilities, the exact type-3
    sum over baselines, and its NUFFT approximation step by step.

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_pins.py``, ``tests/test_oracle_levels_weighting.py`` and
``tests/test_oracle_nufft.py`` (closed forms, invariants, special cases, brute
force); none is "parity unpinned".
"""

from .bluebild_ref import *  # noqa: F401,F403
from . import grad_ref, levels_ref, nufft_ref, weighting_ref  # noqa: F401
