"""The 256-molecule cell (1024 orbitals, 190^3 grid) at full size, in the
launch configuration of the large-cell run (FP32 CG state, 63^3 domains, all
pair solves of a strided sample of its pairs in one call): pair energies of
sampled pairs against the FP64 oracle one by one, the three starts agreeing,
and the learned start saving iterations over the zero start.  Bars: 1e-7 Ha
per pair energy (the whole-cell E_xx bar is 1e-6 Ha over ~9.5k pairs)."""
import os

import numpy as np
import pytest

import oracle
from paper_2208_06097_amd import sea, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2208_06097_amd",
                       "weights", "unet_f32cg.npy")


@pytest.fixture(scope="module")
def large():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cell = synth.config5(with_phi=False)
    phi = synth.fill_orbitals_device(cell, dtype=torch.float32)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 6.0)
    sample = pairs[::97].copy()      # strided sample: ~100 pairs spread over the cell
    return cell, phi, pairs, sample


def _oracle_pair(cell, p):
    """Oracle solve of one pair from only its two orbitals (FP32-rounded, as on the GPU)."""
    i, j = int(p["i"]), int(p["j"])
    sub = [i] if i == j else [i, j]
    c2 = synth.Cell(L=cell.L, N=cell.N, o_centres=cell.o_centres, centres=cell.centres[sub], a=cell.a[sub],
                    seed=cell.seed)
    phi2 = synth.fill_orbitals(c2, dtype=np.float32).phi.astype(np.float64)
    ij = np.array([[0, 0 if i == j else 1]], dtype=np.int32)
    pl = oracle.PairList(ij, p["lo"][None].astype(np.int32), p["n"][None].astype(np.int32), p["origin"][None].copy())
    return oracle.pair_potential(phi2, cell.N, cell.L, pl, 0, tol=1e-12)[2]["e"]


def test_large_cell_sampled_pairs(large):
    cell, phi, pairs, sample = large
    print(f"case 256-molecule cell: {len(pairs)} pairs, sample {len(sample)}", flush=True)
    assert 8000 < len(pairs) < 12000
    res = {}
    for name, start in (("zero", sea.SEA_START_ZERO), ("multipole", sea.SEA_START_MULTIPOLE),
                        ("learned", sea.SEA_START_LEARNED)):
        ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32, start=start)
        if start == sea.SEA_START_LEARNED:
            st = ctx.nn_state(np.load(WEIGHTS))
            ctx.nn_attach(st)
        v, Q, e, stats, status = ctx.pair_solve(phi, cell.N, cell.L, sample, want_Q=False)
        assert status == sea.SEA_OK and np.all(stats["converged"] == 1) and np.all(stats["rel_res"] <= 1e-8)
        res[name] = (e.cpu().numpy(), stats["iters"].astype(float))
        print(f"{name}: mean iterations {stats['iters'].mean():.1f}", flush=True)
        del v
        ctx.close()
    e0 = res["zero"][0]
    for name in ("multipole", "learned"):
        assert np.max(np.abs(res[name][0] - e0)) < 1e-7, name
    assert res["learned"][1].mean() < 0.85 * res["zero"][1].mean()
    # one self pair and one distinct pair against the oracle, one by one
    k_self = int(np.nonzero(sample["i"] == sample["j"])[0][0])
    k_pair = int(np.nonzero(sample["i"] != sample["j"])[0][0])
    for k in (k_self, k_pair):
        e_ref = _oracle_pair(cell, sample[k])
        print(f"pair ({sample['i'][k]}, {sample['j'][k]}): GPU {res['learned'][0][k]:.12f} oracle {e_ref:.12f}",
              flush=True)
        assert abs(res["learned"][0][k] - e_ref) < 1e-7
