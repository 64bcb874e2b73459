"""FP64 CPU oracle for the exx action and the ACE build (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never imports, links or calls it, and it imports nothing from the
product path: it shares only the seeded input generator.

The heavy part (pair density, multipoles, boundary values, CG, scatter) is
plain C in ``sea_oracle.c`` (built with gcc by ``build()``); the ACE algebra
is written here with NumPy/SciPy library primitives (matmul, triangular
solve) around the oracle's own Cholesky, and so is SCDM (its pivoted QR
written out as the greedy column choice, numpy's eigensolver for the inverse
square root).

Every pinned function is checked in ``tests/test_oracle_*.py`` against closed
forms, brute force or textbook library routines.  Parity unpinned: the C1
wrap-duplicate edge effect (a domain wider than the cell) is defined only by
the oracle's own reading.
"""
from .core import (build, lib_path, fd_weights, build_pairs, real_ylm,
                   moments_points, me_eval, neg_lap_padded, cg, pair_potential,
                   pair_me_start, exx, cholesky, ace_build, ace_apply, ace_energy,
                   eps_boxes, eps_pairs, successive_idempotency, scdm_pivots, scdm, back_rotate,
                   qrcp_residual_norms, PairList, ExxResult, AceResult, ScdmResult)

__all__ = ["build", "lib_path", "fd_weights", "build_pairs", "real_ylm",
           "moments_points", "me_eval", "neg_lap_padded", "cg",
           "pair_potential", "pair_me_start", "exx", "cholesky", "ace_build", "ace_apply",
           "ace_energy", "eps_boxes", "eps_pairs", "successive_idempotency", "scdm_pivots", "scdm",
           "back_rotate", "qrcp_residual_norms", "PairList", "ExxResult", "AceResult", "ScdmResult"]
