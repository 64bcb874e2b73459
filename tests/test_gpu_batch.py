"""Batched exx action and HIP-graph plans (many cells, one launch sequence).

Every pair's work depends only on its own cell, so a batched call must give
W, E_xx and per-pair statistics bit-identical to one call per cell; a plan
replayed from its graph must give the eager batched result on every replay,
with unrelated eager work and synchronizations between replays.  Each cell is
also checked against the FP64 oracle (|dE_xx| < 1e-6 Ha, max|dW| < 1e-5).
"""
import numpy as np
import pytest

import oracle
from paper_2208_06097_amd import sea, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cells():
    """Three small cubic cells of different size, spacing and pair count."""
    out = []
    for seed, n_mol, L, N in ((7, 3, 9.0, 30), (8, 4, 10.0, 32), (9, 2, 8.0, 28)):
        c = synth.mini(seed=seed, n_mol=n_mol, L=L, N=N)
        pairs = sea.build_pairs(c.N, c.L, c.centres, 6.0, 4.0)
        out.append((c, pairs))
    return out


@pytest.fixture(scope="module")
def cells():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return _cells()


@pytest.fixture(scope="module")
def oracle_refs(cells):
    refs = []
    for c, _ in cells:
        pl = oracle.build_pairs(c.N, c.L, c.centres, 6.0, 4.0)
        refs.append(oracle.exx(c.phi, c.N, c.L, pl, tol=1e-12))
    return refs


def _phis(cells, dtype):
    return [torch.from_numpy(c.phi.astype(dtype)).cuda() for c, _ in cells]


@pytest.mark.parametrize("form", ["f64-zero", "f32-multipole", "f32-zero-f32phi"])
def test_batched_equals_per_cell_and_oracle(cells, oracle_refs, form):
    print(f"case batched vs per-cell {form}", flush=True)
    sdt = sea.SEA_F64 if form.startswith("f64") else sea.SEA_F32
    start = sea.SEA_START_MULTIPOLE if "multipole" in form else sea.SEA_START_ZERO
    phis = _phis(cells, np.float32 if form.endswith("f32phi") else np.float64)
    ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sdt, start=start)
    singles = []
    for (c, pairs), phi in zip(cells, phis):
        W, E, stats, st = ctx.exx_action(phi, c.N, c.L, pairs)
        assert st == sea.SEA_OK
        singles.append((W.clone(), E, stats.copy()))
    batch = [(phi, c.N, c.L, pairs) for (c, pairs), phi in zip(cells, phis)]
    Ws, Es, stats, st = ctx.exx_action_batched(batch)
    assert st == sea.SEA_OK
    off = 0
    for k, (W1, E1, s1) in enumerate(singles):
        assert torch.equal(Ws[k], W1), k
        assert Es[k] == E1, k
        n = len(s1)
        assert np.array_equal(stats[off:off + n], s1), k
        off += n
    assert off == len(stats)
    for k, ref in enumerate(oracle_refs):
        assert abs(Es[k] - ref.E) < 1e-6, (k, Es[k], ref.E)
        assert np.max(np.abs(Ws[k].cpu().numpy() - ref.W)) < 1e-5, k
    ctx.close()


def test_batched_cell_without_pairs(cells):
    """A cell with no pairs yields W = 0 and E = 0 and leaves the others intact."""
    print("case batched with an empty cell", flush=True)
    phis = _phis(cells, np.float64)
    ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32)
    (c0, p0), (c1, _) = cells[0], cells[1]
    W0, E0, _, _ = ctx.exx_action(phis[0], c0.N, c0.L, p0)
    W0 = W0.clone()
    empty = np.zeros(0, dtype=sea.PAIR_DTYPE)
    W1 = torch.full(phis[1].shape, 7.0, dtype=torch.float64, device="cuda")
    Ws, Es, stats, st = ctx.exx_action_batched([(phis[1], c1.N, c1.L, empty, W1),
                                                (phis[0], c0.N, c0.L, p0)])
    assert st == sea.SEA_OK
    assert Es[0] == 0.0 and float(torch.max(torch.abs(Ws[0]))) == 0.0
    assert Es[1] == E0 and torch.equal(Ws[1], W0)
    assert len(stats) == len(p0)
    ctx.close()


def test_batched_f32_state_rejects_non_cubic(cells):
    (c, pairs) = cells[0]
    print("case batched non-cubic rejection", flush=True)
    phi = torch.from_numpy(c.phi).cuda()
    ctx = sea.Context(stencil_dtype=sea.SEA_F32)
    L = (c.L, c.L, c.L * 1.01)
    with pytest.raises(sea.SeaError) as ei:
        ctx.exx_action_batched([(phi, c.N, c.L, pairs), (phi, c.N, L, pairs)])
    assert ei.value.status == sea.SEA_E_ARG
    ctx.close()


@pytest.mark.parametrize("start", [sea.SEA_START_ZERO, sea.SEA_START_MULTIPOLE])
def test_plan_replays_match_eager(cells, start):
    """Graph replays (with eager library work, torch work and host syncs in
    between) reproduce the eager batched result bit for bit on every replay."""
    print(f"case plan replay start={start}", flush=True)
    phis = _phis(cells, np.float32)
    ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32, start=start)
    batch = [(phi, c.N, c.L, pairs) for (c, pairs), phi in zip(cells[:2], phis[:2])]
    W_ref, E_ref, s_ref, st = ctx.exx_action_batched(batch)
    W_ref = [w.clone() for w in W_ref]
    assert st == sea.SEA_OK
    plan = ctx.exx_plan(batch)
    c2, p2 = cells[2]
    for rep in range(4):
        for w in plan.W:
            w.fill_(float("nan"))
        plan.launch()
        E, stats, st = plan.results()
        assert st == sea.SEA_OK
        assert np.array_equal(E, E_ref), rep
        assert np.array_equal(stats, s_ref), rep
        for k in range(2):
            assert torch.equal(plan.W[k], W_ref[k]), (rep, k)
        # eager work between replays: another cell through the library, torch reductions
        W2, E2, _, _ = ctx.exx_action(phis[2], c2.N, c2.L, p2)
        _ = float(torch.sum(W2 * W2))
        torch.cuda.synchronize()
    plan.close()
    ctx.close()


def test_plan_device_energy_without_host_sync(cells):
    """exx_dev receives E_xx on the device; launches queue without host waits."""
    print("case plan device energy", flush=True)
    phis = _phis(cells, np.float64)
    ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32)
    e_dev = torch.zeros(3, dtype=torch.float64, device="cuda")
    batch = [(phi, c.N, c.L, pairs, None, e_dev[k:k + 1]) for k, ((c, pairs), phi) in enumerate(zip(cells, phis))]
    plan = ctx.exx_plan(batch)
    for _ in range(3):
        plan.launch()
    E, _, st = plan.results()
    assert st == sea.SEA_OK
    assert np.array_equal(e_dev.cpu().numpy(), E)
    plan.close()
    ctx.close()


def test_autotune_picks_fastest_and_variants_agree(cells, tmp_path):
    """CG kernel variants of one arithmetic (they differ in load scheduling
    only) give bit-identical W and E; the paired-update variants (-xc) form
    a second such group, whose results agree with the first to the CG
    tolerance.  The tuner's choice is the argmin of its timings and is
    cached by key."""
    print("case autotune", flush=True)
    phis = _phis(cells, np.float32)
    batch = [(phi, c.N, c.L, pairs) for (c, pairs), phi in zip(cells, phis)]
    ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32)
    names = ctx.cg_variants()
    assert len(names) >= 2
    refs = {}
    for v in range(len(names)):
        ctx.set_opts(cg_variant=v)
        Ws, Es, stats, st = ctx.exx_action_batched(batch)
        assert st == sea.SEA_OK and np.all(stats["converged"] == 1)
        group = names[v].endswith("-xc")
        if group not in refs:
            refs[group] = ([w.clone() for w in Ws], Es.copy(), stats.copy())
        else:
            ref = refs[group]
            assert np.array_equal(Es, ref[1]), names[v]
            assert np.array_equal(stats, ref[2]), names[v]
            for a, b in zip(Ws, ref[0]):
                assert torch.equal(a, b), names[v]
    ref = refs[False]
    if True in refs:
        alt = refs[True]
        assert np.max(np.abs(alt[1] - ref[1])) < 2e-7
        assert abs(alt[2]["iters"].mean() - ref[2]["iters"].mean()) < 0.05 * ref[2]["iters"].mean()
        for a, b in zip(alt[0], ref[0]):
            assert float((a - b).abs().max()) < 1e-5
    ref = refs[False]
    ctx.set_opts(cg_variant=-1)
    cache = str(tmp_path / "tune.json")
    res = ctx.autotune(batch, sample_pairs=64, iters=10, cache=cache)
    assert not res["cached"]
    ms = res["ms"]
    assert set(ms) == set(names) and all(t > 0 for t in ms.values())
    assert res["variant"] == min(ms, key=ms.get)
    again = ctx.autotune(batch, sample_pairs=64, iters=10, cache=cache)
    assert again["cached"] and again["variant"] == res["variant"]
    Ws, Es, _, st = ctx.exx_action_batched(batch)
    assert np.array_equal(Es, refs[res["variant"].endswith("-xc")][1])
    ctx.close()


def test_plan_create_destroy_returns_device_memory(cells):
    """A plan's graph and stream go back when the plan is destroyed: 20
    create / launch / destroy cycles of a 2-cell spectral-start plan on one
    workspace leave the free device memory (as the driver reports it) within
    256 MiB of where it started (under 1% of it).  (A two-stream form of the plans, since removed,
    lost memory this way: a 200-cell batch ran out after about 50 plans.)"""
    print("case plan memory", flush=True)
    ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32, start=sea.SEA_START_SPECTRAL)
    batch = [(phi, c.N, c.L, pairs) for (c, pairs), phi in zip(cells[:2], _phis(cells[:2], np.float32))]
    ws = ctx.workspace(ctx.exx_batched_workspace_bytes(batch))
    plan = ctx.exx_plan(batch, ws=ws)          # first plan: one-time library and runtime set-up
    plan.launch()
    torch.cuda.synchronize()
    E0, _, _ = plan.results()
    plan.close()
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    for rep in range(20):
        plan = ctx.exx_plan(batch, ws=ws)
        plan.launch()
        torch.cuda.synchronize()
        E, _, st = plan.results()
        assert st == sea.SEA_OK and np.array_equal(E, E0)
        plan.close()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    print(f"free device memory {free0 / 2**30:.3f} -> {free1 / 2**30:.3f} GiB", flush=True)
    assert free1 >= free0 - min(0.01 * free0, 256 * 2**20)
    ctx.close()
