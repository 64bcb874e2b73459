"""Write oracle-computed expected values for full-size parity tests.

Calls only the FP64 oracle (``oracle/``) and the seeded input generator.
Run: ``python tests/golden/make_golden.py c1`` (minutes on 8 cores).
Output: ``tests/golden/<name>.json`` with E_xx (Eq. 8), per-pair e_ij,
iteration counts, and W = D_xx sampled at fixed (orbital, grid point) pairs.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2208_06097_amd import synth  # noqa: E402

TOL = 1e-12


def sample_points(n_occ, Ng, k, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_occ, k), rng.integers(0, Ng, k)


def make(name):
    if name == "c1":
        cell = synth.config1(seed=101)
        hw = 6.0
    elif name == "c2":
        cell = synth.config2(seed=2000)
        hw = 6.0
    else:
        raise SystemExit(f"unknown case {name}")
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, hw)
    t = time.time()
    res = oracle.exx(cell.phi, cell.N, cell.L, pl, tol=TOL)
    dt = time.time() - t
    Ng = cell.N ** 3
    # samples: every orbital at points where W is non-negligible, plus random points
    oi, gi = sample_points(cell.n_occ, Ng, 512, 7)
    Wf = res.W.reshape(cell.n_occ, -1)
    big = np.argpartition(-np.abs(Wf), 8, axis=1)[:, :8]
    oi = np.concatenate([oi, np.repeat(np.arange(cell.n_occ), 8)])
    gi = np.concatenate([gi, big.ravel()])
    W_val = Wf[oi, gi].tolist()
    ace = oracle.ace_build(cell.phi, res.W, cell.h ** 3)
    del res.W
    out = dict(case=name, seed=cell.seed, N=cell.N, L=cell.L, half_width=hw, r_pair=6.0, tol=TOL,
               n_pairs=len(pl), E=res.E, e_pairs=res.e_pairs.tolist(), iters=res.iters.tolist(),
               W_orb=oi.tolist(), W_pt=gi.tolist(), W_val=W_val,
               trace_M=float(np.trace(ace.M)), E_ace=oracle.ace_energy(cell.phi, ace.xi, cell.h ** 3),
               oracle_seconds=dt)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"{name}: {len(pl)} pairs, E = {res.E:.12f}, {dt:.1f} s -> {path}")


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c1"]:
        make(n)
