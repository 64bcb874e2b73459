"""GPU network kernels (learned CG warm start) against the FP64 NumPy oracle.

Forward, gradient and Adam through the C ABI (sea_nn_*), at a small grid
(D = 16, batch 2) where the oracle is quick.  Weights: FP32, and BF16 with
the oracle fed the same BF16-rounded weights; FP32 accumulation on the GPU.
"""
import numpy as np
import pytest

import oracle
from oracle import nn
from paper_2208_06097_amd import sea, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _bf16_round(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def net_case():
    rng = np.random.default_rng(11)
    p = nn.init_params(3)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    # parameters exactly representable in FP32 on both sides
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    x = rng.standard_normal((2, 1, 16, 16, 16)).astype(np.float32).astype(np.float64)
    t = rng.standard_normal((2, 1, 16, 16, 16)).astype(np.float32).astype(np.float64)
    return p, x, t


def _ctx(wdt):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return sea.Context(nn_weight_dtype=wdt)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.mark.parametrize("wdt", [sea.SEA_F32, sea.SEA_BF16])
def test_nn_forward_matches_oracle(net_case, wdt):
    p, x, t = net_case
    print(f"case nn forward wdt={wdt}", flush=True)
    ctx = _ctx(wdt)
    st = ctx.nn_state(sea.nn_pack(p))
    y = ctx.nn_forward(st, torch.from_numpy(x[:, 0].astype(np.float32)).cuda()).cpu().numpy()
    # BF16 applies to the weights; biases stay FP32
    pw = p if wdt == sea.SEA_F32 else {k: (_bf16_round(v) if k.endswith(".w") else v) for k, v in p.items()}
    yo, _ = nn.forward(pw, x)
    assert _rel(y, yo[:, 0]) < 2e-5
    if wdt == sea.SEA_BF16:
        yf, _ = nn.forward(p, x)
        assert _rel(y, yf[:, 0]) < 2e-2
    ctx.close()


@pytest.mark.parametrize("wdt", [sea.SEA_F32, sea.SEA_BF16])
def test_nn_gradient_and_adam_match_oracle(net_case, wdt):
    p, x, t = net_case
    print(f"case nn gradient wdt={wdt}", flush=True)
    ctx = _ctx(wdt)
    st = ctx.nn_state(sea.nn_pack(p))
    grad = torch.zeros(ctx.nn_param_count(), dtype=torch.float32, device="cuda")
    xd = torch.from_numpy(x[:, 0].astype(np.float32)).cuda()
    td = torch.from_numpy(t[:, 0].astype(np.float32)).cuda()
    lr = 1e-3
    loss = ctx.nn_train_step(st, xd, td, lr, 1, grad=grad)
    pw = p if wdt == sea.SEA_F32 else {k: (_bf16_round(v) if k.endswith(".w") else v) for k, v in p.items()}
    yo, act = nn.forward(pw, x)
    Lo, gy = nn.mse(yo, t)
    go = nn.backward(pw, act, gy)
    assert abs(loss / Lo - 1) < 1e-5
    gg = sea.nn_unpack(grad.cpu().numpy())
    for name, _, _, _ in nn.LAYERS:
        for sfx in (".w", ".b"):
            assert _rel(gg[name + sfx], go[name + sfx]) < 1e-4, (name, sfx)
    # Adam: GPU parameters after one step vs the oracle's update of the FP32 master
    po = {k: v.copy() for k, v in p.items()}
    nn.adam_step(po, {k: go[k] for k in p}, {}, lr, 1)
    pg = sea.nn_unpack(ctx.nn_get_params(st))
    for k in p:
        d = np.abs(pg[k] - po[k])
        # first Adam step moves by ~lr sign(g); only near-zero gradients may differ
        ok = (d < 1e-6) | (np.abs(go[k]) < 1e-4 * np.max(np.abs(go[k])))
        assert np.all(ok), k
    ctx.close()


def test_nn_infer_matrix_cores_matches_oracle():
    """Matrix-core inference (BF16 weights and activations, FP32 accumulation)
    on the 32^3 grid against the FP64 oracle fed the same BF16 weights.  Bar:
    every activation is rounded to BF16 (relative 2^-9) once per layer, 15
    layers in sequence: relative L2 error < 15 * 2^-9 ~ 3e-2."""
    print("case nn infer (matrix cores) D=32", flush=True)
    rng = np.random.default_rng(12)
    p = nn.init_params(5)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    x = rng.standard_normal((2, 1, 32, 32, 32)).astype(np.float32).astype(np.float64)
    ctx = _ctx(sea.SEA_BF16)
    st = ctx.nn_state(sea.nn_pack(p))
    xd = torch.from_numpy(x[:, 0].astype(np.float32)).cuda()
    y = ctx.nn_infer(st, xd).cpu().numpy()
    y_valu = ctx.nn_forward(st, xd).cpu().numpy()
    pw = {k: (_bf16_round(v) if k.endswith(".w") else v) for k, v in p.items()}
    yo, _ = nn.forward(pw, x)
    err = _rel(y, yo[:, 0])
    print(f"matrix-core inference rel err vs oracle {err:.2e}, vs FP32-activation path "
          f"{_rel(y, y_valu):.2e}", flush=True)
    assert np.all(np.isfinite(y))
    assert err < 3e-2
    # a batch that is not a multiple of anything and a second call reuse
    y1 = ctx.nn_infer(st, xd[1:].contiguous()).cpu().numpy()
    assert np.array_equal(y1[0], y[1])
    ctx.close()


@pytest.fixture(scope="module")
def samples():
    """Training samples from converged solves of two small cells (29^3 domains)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32)
    xs, ts = [], []
    for seed in (7, 8, 9):
        cell = synth.mini(seed=seed)
        pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
        x, t, s, stats = ctx.exx_nn_samples(torch.from_numpy(cell.phi).cuda(), cell.N, cell.L, pairs, D=32)
        assert np.all(stats["converged"] == 1)
        xs.append(x)
        ts.append(t)
    ctx.close()
    return torch.cat(xs), torch.cat(ts)


def test_nn_samples_match_oracle_resampling():
    """x = resample(rho/s) and t = resample((v - v_ME)/s) on 32^3 for one pair,
    against the oracle's own pair density, pair potential (at 1e-12),
    regularized multipole start v_ME and trilinear resampling."""
    cell = synth.mini(seed=7)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
    print("case nn samples", flush=True)
    ctx = sea.Context(rel_tol=1e-12)
    x, t, s, stats = ctx.exx_nn_samples(torch.from_numpy(cell.phi).cuda(), cell.N, cell.L, pairs, D=32)
    ctx.close()
    k = 3
    i, j = pl.ij[k]
    lo, n = pl.lo[k], pl.n[k]
    iz = np.mod(lo[2] + np.arange(n[2]), cell.N)
    iy = np.mod(lo[1] + np.arange(n[1]), cell.N)
    ix = np.mod(lo[0] + np.arange(n[0]), cell.N)
    rho = cell.phi[i][np.ix_(iz, iy, ix)] * cell.phi[j][np.ix_(iz, iy, ix)]
    s_ref = cell.h ** 3 * np.sum(np.abs(rho))
    assert abs(s[k].item() / s_ref - 1) < 1e-12
    want_x = nn.resample(rho / s_ref, 32)
    assert np.max(np.abs(x[k].cpu().numpy() - want_x)) < 1e-5 * np.max(np.abs(want_x))
    v, _, info = oracle.pair_potential(cell.phi, cell.N, cell.L, pl, k, tol=1e-12)
    v_me = oracle.pair_me_start(cell.phi, cell.N, cell.L, pl, k)
    want_t = nn.resample((v - v_me) / s_ref, 32)
    err_t = np.max(np.abs(t[k].cpu().numpy() - want_t))
    print(f"t: max |dt| {err_t:.3e} of max |t| {np.max(np.abs(want_t)):.3e}", flush=True)
    # FP32 samples: 6e-8 relative rounding; the solves agree to 1e-12
    assert err_t < 1e-5 * np.max(np.abs(want_t))
    assert np.max(np.abs(want_t)) > 1e-3 * np.max(np.abs(v))    # the correction is not trivially zero


def test_training_lowers_loss(samples):
    x, t = samples
    print(f"case nn training on {x.shape[0]} samples", flush=True)
    ctx = sea.Context(nn_weight_dtype=sea.SEA_BF16)
    st = ctx.nn_state(sea.nn_pack(nn.init_params(0)))
    n = x.shape[0]
    B = 16
    ws = ctx.nn_workspace(B, 32)
    gen = torch.Generator(device="cpu").manual_seed(0)
    first = None
    losses = []
    step = 0
    for epoch in range(20):
        perm = torch.randperm(n, generator=gen)
        for b0 in range(0, n - B + 1, B):
            idx = perm[b0:b0 + B].cuda()
            step += 1
            L = ctx.nn_train_step(st, x[idx].contiguous(), t[idx].contiguous(), 2e-3, step, ws=ws)
            losses.append(L)
            if first is None:
                first = L
    assert np.isfinite(losses).all()
    assert np.mean(losses[-5:]) < 0.5 * first
    ctx.close()


@pytest.fixture(scope="module")
def trained_state(samples):
    x, t = samples
    ctx = sea.Context(nn_weight_dtype=sea.SEA_BF16)
    st = ctx.nn_state(sea.nn_pack(nn.init_params(1)))
    B = 16
    ws = ctx.nn_workspace(B, 32)
    gen = torch.Generator(device="cpu").manual_seed(1)
    step = 0
    for epoch in range(30):
        perm = torch.randperm(x.shape[0], generator=gen)
        for b0 in range(0, x.shape[0] - B + 1, B):
            idx = perm[b0:b0 + B].cuda()
            step += 1
            ctx.nn_train_step(st, x[idx].contiguous(), t[idx].contiguous(), 2e-3, step, ws=ws, want_loss=False)
    torch.cuda.synchronize()
    params = ctx.nn_get_params(st)
    ctx.close()
    return params


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_learned_start_same_result_and_gain(trained_state, dtype):
    """Held-out cell: the learned start reaches the oracle's E and W at the
    same 1e-8 true residual, in fewer CG iterations than the zero start."""
    cell = synth.mini(seed=10)
    print(f"case learned start {dtype}", flush=True)
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
    ref = oracle.exx(cell.phi, cell.N, cell.L, pl, tol=1e-12)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
    sdt = sea.SEA_F64 if dtype == "f64" else sea.SEA_F32
    phi = torch.from_numpy(cell.phi).cuda()
    c0 = sea.Context(rel_tol=1e-8, stencil_dtype=sdt)
    _, _, s0, _ = c0.exx_action(phi, cell.N, cell.L, pairs)
    c0.close()
    cl = sea.Context(rel_tol=1e-8, stencil_dtype=sdt, start=sea.SEA_START_LEARNED)
    st = cl.nn_state(trained_state)
    cl.nn_attach(st)
    W, E, s1, stat = cl.exx_action(phi, cell.N, cell.L, pairs)
    cl.close()
    assert stat == sea.SEA_OK and np.all(s1["converged"] == 1) and np.all(s1["rel_res"] <= 1e-8)
    assert abs(E - ref.E) < 1e-6
    assert np.max(np.abs(W.cpu().numpy() - ref.W)) < 1e-5
    print(f"mean iterations: zero {s0['iters'].mean():.1f}  learned {s1['iters'].mean():.1f}", flush=True)
    assert s1["iters"].mean() < s0["iters"].mean()


def test_learned_start_requires_network():
    cell = synth.mini(seed=10)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
    cl = sea.Context(start=sea.SEA_START_LEARNED)
    with pytest.raises(sea.SeaError) as ei:
        cl.exx_action(torch.from_numpy(cell.phi).cuda(), cell.N, cell.L, pairs)
    assert ei.value.status == sea.SEA_E_ARG
    cl.close()


def test_learned_beats_multipole_on_held_out_cell():
    """The committed network on the 64-molecule cell (seed 2000, 1.0 g/cm^3;
    the training cells are other seeds and densities): the learned start
    needs fewer CG iterations than the multipole start it corrects, which
    needs fewer than the zero start; all three reach the same E_xx at the
    same true residual (FP32 state)."""
    import os
    weights = os.path.join(os.path.dirname(sea.__file__), "weights", "unet_f32cg.npy")
    cell = synth.config2(with_phi=False)
    phi = synth.fill_orbitals_device(cell, dtype=torch.float32)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 6.0)
    print(f"case learned vs multipole: {len(pairs)} pairs", flush=True)
    res = {}
    for name, start in (("zero", sea.SEA_START_ZERO), ("multipole", sea.SEA_START_MULTIPOLE),
                        ("learned", sea.SEA_START_LEARNED)):
        ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32, start=start)
        if start == sea.SEA_START_LEARNED:
            ctx.nn_attach(ctx.nn_state(np.load(weights)))
        _, E, stats, status = ctx.exx_action(phi, cell.N, cell.L, pairs)
        assert status == sea.SEA_OK and np.all(stats["converged"] == 1) and np.all(stats["rel_res"] <= 1e-8)
        res[name] = (E, stats["iters"].mean())
        print(f"{name}: mean iterations {stats['iters'].mean():.2f}  E {E:.10f}", flush=True)
        ctx.close()
    assert res["learned"][1] < res["multipole"][1] < res["zero"][1]
    for name in ("multipole", "learned"):
        assert abs(res[name][0] - res["zero"][0]) < 1e-6, name


@pytest.mark.parametrize("half_width", [4.0, 10.0])
def test_learned_start_is_multipole_plus_upsampled_network(half_width):
    """The learned start before any CG iteration (FP64 state, max_iter 0) is
    the oracle's regularized multipole start plus s times the oracle's
    tricubic map of the GPU network's 32^3 output, pair by pair: domains of
    27-29 points (the separable LDS-ring kernel) and of 69 points, wider
    than the cell (the per-point kernel)."""
    import os
    weights = os.path.join(os.path.dirname(sea.__file__), "weights", "unet_f32cg.npy")
    cell = synth.mini(seed=7)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, half_width)
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, half_width)
    print(f"case learned x0, half width {half_width}: {len(pairs)} pairs, n {pairs['n'].max()}", flush=True)
    phi = torch.from_numpy(cell.phi).cuda()
    ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F64, start=sea.SEA_START_LEARNED, max_iter=0)
    st = ctx.nn_state(np.load(weights))
    ctx.nn_attach(st)
    v, _, _, stats, _ = ctx.pair_solve(phi, cell.N, cell.L, pairs, want_Q=False)
    x, _, s, _ = ctx.exx_nn_samples(phi, cell.N, cell.L, pairs)
    y = ctx.nn_infer(st, x.contiguous()).cpu().numpy().astype(np.float64)
    s = s.cpu().numpy()
    v = v.cpu().numpy()
    ctx.close()
    assert np.all(stats["iters"] == 0)
    for k in range(0, len(pairs), max(1, len(pairs) // 4)):
        n = pl.n[k]
        got = v[k, :n[0] * n[1] * n[2]].reshape(n[2], n[1], n[0])
        corr = s[k] * nn.upsample_cubic(y[k], (n[2], n[1], n[0]))
        want = oracle.pair_me_start(cell.phi, cell.N, cell.L, pl, k) + corr
        err = np.max(np.abs(got - want))
        print(f"pair {k}: n {tuple(n)} max |x0 - want| {err:.2e} of max |s up(y)| {np.max(np.abs(corr)):.2e}",
              flush=True)
        # FP32 network values interpolated through an FP32 ring (relative
        # 1e-6 of the correction) plus the start's FP64 rounding
        assert err < 1e-6 * np.max(np.abs(corr)) + 1e-10 * np.max(np.abs(want))
