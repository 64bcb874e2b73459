"""GPU parity of the exx action and the ACE build against the FP64 oracle.

All calls go through the C ABI (libsea.so via the ctypes binding).  The
oracle runs at a relative residual of 1e-12 (effectively the exact discrete
solution); the GPU runs at the product tolerance 1e-8 unless a test says
otherwise.  Bars: |dE_xx| < 1e-6 Ha and max|dW| < 1e-5 at 1e-8; tighter
element-wise bars when both sides solve to 1e-12.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2208_06097_amd import sea, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _unpack_v(v_row, n):
    return v_row[: n[0] * n[1] * n[2]].reshape(n[2], n[1], n[0])


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = sea.Context(rel_tol=1e-8)
    yield c
    c.close()


@pytest.fixture(scope="module")
def mini():
    cell = synth.mini()
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
    ref = oracle.exx(cell.phi, cell.N, cell.L, pl, tol=1e-12)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
    return cell, pl, ref, pairs


def test_pair_solve_elementwise_tight(ctx, mini):
    """Both sides at 1e-12: potentials, moments and pair energies agree."""
    cell, pl, ref, pairs = mini
    print("case mini pair_solve tol 1e-12", flush=True)
    ctx.set_opts(rel_tol=1e-12)
    try:
        v, Q, e, stats, st = ctx.pair_solve(_dev(cell.phi), cell.N, cell.L, pairs)
    finally:
        ctx.set_opts(rel_tol=1e-8)
    assert st == sea.SEA_OK
    v, Q, e = v.cpu().numpy(), Q.cpu().numpy(), e.cpu().numpy()
    for k in range(len(pl)):
        vo, Qo, info = oracle.pair_potential(cell.phi, cell.N, cell.L, pl, k, tol=1e-12)
        vg = _unpack_v(v[k], pl.n[k])
        assert np.max(np.abs(vg - vo)) <= 1e-9 * max(1.0, np.max(np.abs(vo))), k
        assert np.max(np.abs(Q[k] - Qo)) <= 1e-12 * max(1.0, np.max(np.abs(Qo))), k
        assert abs(e[k] - info["e"]) <= 1e-10 * max(1e-3, abs(info["e"])), k
        assert stats["converged"][k] == 1 and stats["rel_res"][k] <= 1e-12
        assert abs(stats["s_abs"][k] - info["s_abs"]) <= 1e-12
        assert abs(stats["q"][k] - info["q"]) <= 1e-12


def test_exx_action_mini(ctx, mini):
    cell, pl, ref, pairs = mini
    print("case mini exx_action tol 1e-8", flush=True)
    W, E, stats, st = ctx.exx_action(_dev(cell.phi), cell.N, cell.L, pairs)
    assert st == sea.SEA_OK
    assert abs(E - ref.E) < 1e-6
    assert np.max(np.abs(W.cpu().numpy() - ref.W)) < 1e-5
    assert np.all(stats["converged"] == 1) and np.all(stats["rel_res"] <= 1e-8)


@pytest.fixture(scope="module")
def ctx32():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32)
    yield c
    c.close()


def test_exx_action_fp32_state_mini(ctx32, mini):
    """FP32 CG state with FP64 refinement reaches the same 1e-8 true residual."""
    cell, pl, ref, pairs = mini
    print("case mini exx_action fp32 state", flush=True)
    W, E, stats, st = ctx32.exx_action(_dev(cell.phi), cell.N, cell.L, pairs)
    assert st == sea.SEA_OK
    assert np.all(stats["converged"] == 1) and np.all(stats["rel_res"] <= 1e-8)
    assert abs(E - ref.E) < 1e-6
    assert np.max(np.abs(W.cpu().numpy() - ref.W)) < 1e-5


def test_exx_action_fp32_state_wrap(ctx32):
    cell = synth.mini(n_mol=2)
    print("case mini-wrap fp32 state", flush=True)
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, 5.0)
    ref = oracle.exx(cell.phi, cell.N, cell.L, pl, tol=1e-12)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 5.0)
    W, E, stats, st = ctx32.exx_action(_dev(cell.phi), cell.N, cell.L, pairs)
    assert np.all(stats["converged"] == 1)
    assert abs(E - ref.E) < 1e-6
    assert np.max(np.abs(W.cpu().numpy() - ref.W)) < 1e-5


def test_non_cubic_grid_generic_path(ctx):
    """Unequal spacings take the generic (global-memory stencil) CG kernel."""
    cell = synth.mini(n_mol=2)
    print("case non-cubic", flush=True)
    N = np.array([30, 30, 30])
    L = np.array([cell.L, cell.L, cell.L * 1.04])
    # re-sample the orbitals on the stretched grid through the generator's formula
    cell2 = synth.make_centres(2, cell.L, 30, cell.seed, dmin=3.5)
    phi = np.empty((cell2.n_occ, 30, 30, 30))
    for i in range(cell2.n_occ):
        ax = [np.arange(30) * (L[k] / 30) for k in range(3)]
        d = [ax[k] - cell2.centres[i, k] - L[k] * np.round((ax[k] - cell2.centres[i, k]) / L[k]) for k in range(3)]
        g = np.exp(-(d[2][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[0][None, None, :] ** 2) / (2 * synth.SIGMA ** 2))
        f = (1 + cell2.a[i, 0] * d[0][None, None, :] + cell2.a[i, 1] * d[1][None, :, None]
             + cell2.a[i, 2] * d[2][:, None, None]) * g
        phi[i] = f / np.sqrt(np.prod(L / N) * np.sum(f * f))
    pl = oracle.build_pairs(N, L, cell2.centres, 6.0, 4.0)
    ref = oracle.exx(phi, N, L, pl, tol=1e-12)
    pairs = sea.build_pairs(N, L, cell2.centres, 6.0, 4.0)
    W, E, stats, st = ctx.exx_action(_dev(phi), N, L, pairs)
    assert st == sea.SEA_OK
    assert abs(E - ref.E) < 1e-6
    assert np.max(np.abs(W.cpu().numpy() - ref.W)) < 1e-5


def test_exx_action_deterministic(ctx, mini):
    cell, pl, ref, pairs = mini
    print("case mini determinism", flush=True)
    phi = _dev(cell.phi)
    W1, E1, _, _ = ctx.exx_action(phi, cell.N, cell.L, pairs)
    W2, E2, _, _ = ctx.exx_action(phi, cell.N, cell.L, pairs)
    assert E1 == E2 and torch.equal(W1, W2)


def test_exx_action_domain_wider_than_cell(ctx):
    """35-point domains in a 30-point cell: wrapped duplicates accumulate."""
    cell = synth.mini(n_mol=2)
    print("case mini-wrap", flush=True)
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, 5.0)
    ref = oracle.exx(cell.phi, cell.N, cell.L, pl, tol=1e-12)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 5.0)
    assert pairs["n"][0, 0] > cell.N
    W, E, stats, st = ctx.exx_action(_dev(cell.phi), cell.N, cell.L, pairs)
    assert abs(E - ref.E) < 1e-6
    assert np.max(np.abs(W.cpu().numpy() - ref.W)) < 1e-5


def test_exx_action_fp32_orbitals(ctx, mini):
    """FP32 orbital storage: inputs rounded to FP32 on both sides."""
    cell, pl, ref, pairs = mini
    print("case mini fp32 phi", flush=True)
    phi32 = cell.phi.astype(np.float32)
    ref32 = oracle.exx(phi32.astype(np.float64), cell.N, cell.L, pl, tol=1e-12)
    W, E, stats, st = ctx.exx_action(_dev(phi32), cell.N, cell.L, pairs)
    assert abs(E - ref32.E) < 1e-6
    assert np.max(np.abs(W.cpu().numpy() - ref32.W)) < 1e-5


def test_ace_build_apply_energy_mini(ctx, mini):
    cell, pl, ref, pairs = mini
    print("case mini ace f64", flush=True)
    dV = cell.h ** 3
    phi = _dev(cell.phi)
    W = _dev(ref.W)
    M, Lm, xi, fp = ctx.ace_build(phi, W, dV)
    want = oracle.ace_build(cell.phi, ref.W, dV)
    assert fp == 0
    assert np.max(np.abs(M.cpu().numpy() - want.M)) <= 1e-12 * np.max(np.abs(want.M))
    assert np.max(np.abs(Lm.cpu().numpy() - want.L)) <= 1e-11 * np.max(np.abs(want.L))
    assert np.max(np.abs(xi.cpu().numpy().reshape(want.xi.shape) - want.xi)) <= 1e-10 * np.max(np.abs(want.xi))
    K = ctx.ace_apply(xi, phi, dV).cpu().numpy()
    Kw = oracle.ace_apply(want.xi, cell.phi, dV)
    assert np.max(np.abs(K - Kw)) <= 1e-10 * np.max(np.abs(Kw))
    E = ctx.ace_energy(phi, xi, dV)
    assert abs(E - oracle.ace_energy(cell.phi, want.xi, dV)) < 1e-9
    assert abs(E - ref.E) < 1e-6


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_ace_matrix_core_dtypes_multi_tile(dt):
    """ACE build / apply / energy on the matrix cores at sizes that span
    several output tiles with ragged edges (150 orbitals over 128-row tiles,
    70 trial vectors, 21^3 grid points over 128-column tiles and uneven K
    slices), per ace_dtype against the FP64 oracle.  M, its Cholesky factor
    and the energy reduction are FP64 in every dtype; xi and K psi carry the
    dtype's rounding: bars are FP64 1e-10, FP32 (2^-24 per operand, FP32
    accumulation) 1e-5, BF16 (2^-9 per operand) 1e-2 relative."""
    print(f"case ace matrix cores {dt}", flush=True)
    rng = np.random.default_rng(3)
    n_occ, N, n_vec = 150, 21, 70
    ng, dV = N ** 3, 0.3 ** 3
    phi = rng.standard_normal((n_occ, ng)) / np.sqrt(ng * dV)
    A = rng.standard_normal((n_occ, n_occ))
    G = A @ A.T / n_occ + np.eye(n_occ)
    W = G @ phi
    psi = rng.standard_normal((n_vec, ng)) / np.sqrt(ng * dV)
    want = oracle.ace_build(phi, W, dV)
    adt = {"f64": sea.SEA_F64, "f32": sea.SEA_F32, "bf16": sea.SEA_BF16}[dt]
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt]
    bar = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-2}[dt]
    ctx = sea.Context(ace_dtype=adt)
    M, Lm, xi, fp = ctx.ace_build(_dev(phi), _dev(W), dV)
    assert fp == 0
    assert np.max(np.abs(M.cpu().numpy() - want.M)) <= 1e-12 * np.max(np.abs(want.M))
    assert np.max(np.abs(Lm.cpu().numpy() - want.L)) <= 1e-10 * np.max(np.abs(want.L))
    xi_h = xi.double().cpu().numpy()
    assert np.linalg.norm(xi_h - want.xi) <= bar * np.linalg.norm(want.xi)
    psi_d = _dev(psi).to(tdt)
    K = ctx.ace_apply(xi, psi_d, dV).double().cpu().numpy()
    Kw = oracle.ace_apply(want.xi, psi_d.double().cpu().numpy(), dV)
    rel_k = np.linalg.norm(K - Kw) / np.linalg.norm(Kw)
    E = ctx.ace_energy(_dev(phi), xi, dV)
    Ew = oracle.ace_energy(phi, want.xi, dV)
    print(f"ace {dt}: |dxi|/|xi| {np.linalg.norm(xi_h - want.xi) / np.linalg.norm(want.xi):.2e}  "
          f"|dKpsi|/|Kpsi| {rel_k:.2e}  |dE|/|E| {abs(E - Ew) / abs(Ew):.2e}", flush=True)
    assert rel_k <= bar
    assert abs(E - Ew) <= bar * abs(Ew)
    ctx.close()


@pytest.mark.parametrize("n_occ", [64, 256, 300])
def test_ace_cholesky_blocked_sizes(n_occ):
    """The blocked Cholesky of M at a single block, at whole blocks and with a
    ragged last block, against LAPACK's factor of the same M (FP64), and
    the factor's product against M.  Also xi and K psi against the oracle:
    1 to 3 row blocks of the short-K product over 14 column tiles (fewer
    than two per XCD, so that some persistent workgroups take one tile and
    some none)."""
    print(f"case ace cholesky n_occ={n_occ}", flush=True)
    rng = np.random.default_rng(n_occ)
    N = 12
    ng, dV = N ** 3, 0.25 ** 3
    phi = rng.standard_normal((n_occ, ng)) / np.sqrt(ng * dV)
    A = rng.standard_normal((n_occ, n_occ))
    W = (A @ A.T / n_occ + np.eye(n_occ)) @ phi
    ctx = sea.Context()
    M, Lm, xi, fp = ctx.ace_build(_dev(phi), _dev(W), dV)
    assert fp == 0
    want_ace = oracle.ace_build(phi, W, dV)
    xi_h = xi.cpu().numpy()
    assert np.max(np.abs(xi_h - want_ace.xi)) <= 1e-10 * np.max(np.abs(want_ace.xi))
    psi = rng.standard_normal((70, ng)) / np.sqrt(ng * dV)
    K = ctx.ace_apply(xi, _dev(psi), dV).cpu().numpy()
    Kw = oracle.ace_apply(want_ace.xi, psi, dV)
    assert np.max(np.abs(K - Kw)) <= 1e-10 * np.max(np.abs(Kw))
    Mh = M.cpu().numpy()
    Mh = 0.5 * (Mh + Mh.T)
    Lh = Lm.cpu().numpy()
    want = np.linalg.cholesky(Mh)
    assert np.max(np.abs(np.triu(Lh, 1))) == 0.0
    assert np.max(np.abs(Lh - want)) <= 1e-11 * np.max(np.abs(want))
    assert np.max(np.abs(Lh @ Lh.T - Mh)) <= 1e-12 * np.max(np.abs(Mh))
    ctx.close()


def test_ace_not_positive_definite(ctx, mini):
    cell, pl, ref, pairs = mini
    print("case ace not-PD", flush=True)
    phi = _dev(cell.phi)
    W = _dev(-ref.W)   # negated action: M negative definite
    with pytest.raises(sea.SeaError) as ei:
        ctx.ace_build(phi, W, cell.h ** 3)
    assert ei.value.status == sea.SEA_E_NOT_PD


def test_edge_cases(ctx, mini):
    cell, pl, ref, pairs = mini
    print("case edge cases", flush=True)
    phi = _dev(cell.phi)
    # no pairs: W = 0, E = 0
    W, E, stats, st = ctx.exx_action(phi, cell.N, cell.L, pairs[:0])
    assert E == 0.0 and not torch.any(W)
    # a single pair
    W, E, stats, st = ctx.exx_action(phi, cell.N, cell.L, pairs[:1])
    assert abs(E + ref.e_pairs[0]) < 1e-6
    # bad pair (i > j) is rejected before launch
    bad = pairs.copy()
    bad["i"][3], bad["j"][3] = 5, 2
    with pytest.raises(sea.SeaError) as ei:
        ctx.exx_action(phi, cell.N, cell.L, bad)
    assert ei.value.status == sea.SEA_E_ARG
    # workspace too small
    with pytest.raises(sea.SeaError) as ei:
        ctx.exx_action(phi, cell.N, cell.L, pairs, ws=ctx.workspace(1024))
    assert ei.value.status == sea.SEA_E_NOMEM
    # iteration cap: outputs written, warning status
    ctx.set_opts(max_iter=5)
    try:
        W, E, stats, st = ctx.exx_action(phi, cell.N, cell.L, pairs)
    finally:
        ctx.set_opts(max_iter=10000)
    assert st == sea.SEA_W_NOT_CONVERGED and np.all(stats["iters"] <= 5)
    # non-finite input
    phin = cell.phi.copy()
    phin[0, 3, 4, 5] = np.nan
    with pytest.raises(sea.SeaError) as ei:
        ctx.exx_action(_dev(phin), cell.N, cell.L, pairs)
    assert ei.value.status == sea.SEA_E_NONFINITE


def test_c1_full_against_golden(ctx):
    """Full config-1 cell (8 molecules, 60^3, 63^3 domains) in the launch
    configuration of the benchmark, against stored oracle values."""
    path = os.path.join(GOLDEN, "c1.json")
    g = json.load(open(path))
    cell = synth.config1(seed=g["seed"])
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, g["r_pair"], g["half_width"])
    assert len(pairs) == g["n_pairs"]
    print("case c1 full", flush=True)
    W, E, stats, st = ctx.exx_action(_dev(cell.phi), cell.N, cell.L, pairs)
    assert st == sea.SEA_OK
    assert abs(E - g["E"]) < 1e-6
    Wf = W.reshape(cell.n_occ, -1)
    idx_o = torch.tensor(g["W_orb"], device="cuda")
    idx_g = torch.tensor(g["W_pt"], device="cuda")
    got = Wf[idx_o, idx_g].cpu().numpy()
    assert np.max(np.abs(got - np.array(g["W_val"]))) < 1e-5
    e = stats["e_ij"]
    assert np.max(np.abs(e - np.array(g["e_pairs"]))) < 1e-7


CG_VARIANTS = ["nt1024-pf-d1", "nt1024-pf-d2", "nt1024-d1", "nt1024-d2", "buf-pf-d1", "buf-pf-d2", "buf-d2",
               "buf-pf-d1-xc", "buf-pf-d2-xc", "nt1024-pf-d1-xc"]


@pytest.mark.parametrize("variant,beta_min", [(v, 0.0) for v in CG_VARIANTS]
                         + [("buf-pf-d1-xc", 10.0), ("buf-pf-d1-xc", 1e-300)])
def test_c1_full_fp32_state_against_golden(variant, beta_min):
    """Every FP32 CG kernel variant on the full config-1 cell against the
    stored oracle values; for the paired-update kernel also with every
    pending step written by the separate pass (beta_min 10) and with none
    written that way (beta_min ~ 0: only refreshes flush)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = json.load(open(os.path.join(GOLDEN, "c1.json")))
    cell = synth.config1(seed=g["seed"])
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, g["r_pair"], g["half_width"])
    print(f"case c1 full fp32 state, CG variant {variant}, beta_min {beta_min}", flush=True)
    ctx32 = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32)
    assert CG_VARIANTS == ctx32.cg_variants()
    ctx32.set_opts(cg_variant=CG_VARIANTS.index(variant), cg_xc_beta_min=beta_min)
    W, E, stats, st = ctx32.exx_action(_dev(cell.phi), cell.N, cell.L, pairs)
    ctx32.close()
    assert st == sea.SEA_OK and np.all(stats["rel_res"] <= 1e-8)
    assert abs(E - g["E"]) < 1e-6
    Wf = W.reshape(cell.n_occ, -1)
    got = Wf[torch.tensor(g["W_orb"], device="cuda"), torch.tensor(g["W_pt"], device="cuda")].cpu().numpy()
    assert np.max(np.abs(got - np.array(g["W_val"]))) < 1e-5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_multipole_start_same_result_fewer_iterations(mini, dtype):
    """The multipole start changes only the CG start: the same 1e-8 true
    residual, the same E and W within the bars, fewer iterations."""
    cell, pl, ref, pairs = mini
    print(f"case mini multipole start {dtype}", flush=True)
    sdt = sea.SEA_F64 if dtype == "f64" else sea.SEA_F32
    c0 = sea.Context(rel_tol=1e-8, stencil_dtype=sdt)
    c1 = sea.Context(rel_tol=1e-8, stencil_dtype=sdt, start=sea.SEA_START_MULTIPOLE)
    phi = _dev(cell.phi)
    W0, E0, s0, _ = c0.exx_action(phi, cell.N, cell.L, pairs)
    W1, E1, s1, st = c1.exx_action(phi, cell.N, cell.L, pairs)
    c0.close()
    c1.close()
    assert st == sea.SEA_OK and np.all(s1["converged"] == 1) and np.all(s1["rel_res"] <= 1e-8)
    assert abs(E1 - ref.E) < 1e-6
    assert np.max(np.abs(W1.cpu().numpy() - ref.W)) < 1e-5
    assert s1["iters"].mean() < s0["iters"].mean()


def _eig_case(n=150, N=21, dV=0.3 ** 3, seed=6, mixed=True):
    rng = np.random.default_rng(seed)
    ng = N ** 3
    Qf, _ = np.linalg.qr(rng.standard_normal((ng, n)))
    phi = Qf.T / np.sqrt(dV)
    lam = rng.uniform(0.2, 3.0, n)
    if mixed:
        lam[rng.choice(n, n // 5, replace=False)] *= -1.0
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    G = U @ np.diag(lam) @ U.T
    return phi, G @ phi, dV, rng.standard_normal((40, ng)) / np.sqrt(ng * dV)


@pytest.mark.parametrize("decomp", ["eigen", "auto"])
def test_ace_eigen_scheme_matches_oracle(decomp):
    """App. A on the GPU (parallel Jacobi) for a symmetrized M with negative
    eigenvalues: K psi and E_ACE against the oracle's eigen scheme (invariant
    to eigenvector order and signs); AUTO reports the fallback."""
    print(f"case ace eigen scheme {decomp}", flush=True)
    phi, W, dV, psi = _eig_case()
    want = oracle.ace_build(phi, W, dV, decomp="eigen")
    dc = sea.SEA_DECOMP_EIGEN if decomp == "eigen" else sea.SEA_DECOMP_AUTO
    c = sea.Context(ace_decomp=dc)
    M, Lm, xi, fp = c.ace_build(_dev(phi), _dev(W), dV)
    assert c.last_status == (sea.SEA_OK if decomp == "eigen" else sea.SEA_W_EIGEN_FALLBACK)
    K = c.ace_apply(xi, _dev(psi), dV).cpu().numpy()
    Kw = oracle.ace_apply(want.xi, psi, dV)
    assert np.linalg.norm(K - Kw) <= 1e-10 * np.linalg.norm(Kw)
    E = c.ace_energy(_dev(phi), xi, dV)
    assert abs(E - oracle.ace_energy(phi, want.xi, dV)) <= 1e-10 * abs(E)
    # L_dev holds Q |Lambda|^{-1/2}: (Q|L|^-1/2)(Q|L|^-1/2)^T = Q |Lambda|^-1 Q^T = |Mbar|^-1
    Z = Lm.cpu().numpy()
    lam, Q = np.linalg.eigh(want.Mbar)
    assert np.allclose(Z @ Z.T, Q @ np.diag(1 / np.abs(lam)) @ Q.T, atol=1e-9)
    c.close()


def test_ace_eigen_scheme_equals_cholesky_when_positive_definite():
    print("case ace eigen vs cholesky (PD)", flush=True)
    phi, W, dV, psi = _eig_case(mixed=False)
    out = []
    for dc in (sea.SEA_DECOMP_CHOLESKY, sea.SEA_DECOMP_EIGEN, sea.SEA_DECOMP_AUTO):
        c = sea.Context(ace_decomp=dc)
        _, _, xi, fp = c.ace_build(_dev(phi), _dev(W), dV)
        assert fp == 0 and c.last_status == sea.SEA_OK
        out.append(c.ace_apply(xi, _dev(psi), dV).cpu().numpy())
        c.close()
    assert np.linalg.norm(out[1] - out[0]) <= 1e-10 * np.linalg.norm(out[0])
    assert np.array_equal(out[2], out[0])


def test_successive_idempotency():
    """App. B: dI = 0 for the same occupied space in any orthonormal basis,
    the oracle's value otherwise."""
    print("case successive idempotency", flush=True)
    rng = np.random.default_rng(8)
    n, ng, dV = 150, 21 ** 3, 0.3 ** 3
    Q, _ = np.linalg.qr(rng.standard_normal((ng, n)))
    phi = Q.T / np.sqrt(dV)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    c = sea.Context()
    assert abs(c.successive_idempotency(_dev(phi), _dev(phi), dV)) < 1e-12
    assert abs(c.successive_idempotency(_dev(U @ phi), _dev(phi), dV)) < 1e-12
    Q2, _ = np.linalg.qr(Q + 0.05 * rng.standard_normal((ng, n)))
    phi2 = Q2.T / np.sqrt(dV)
    d = c.successive_idempotency(_dev(phi2), _dev(phi), dV)
    assert abs(d - oracle.successive_idempotency(phi2, phi, dV)) < 1e-12 and d > 1e-4
    c.close()


def test_cg_xc_beta_min_rejects_bad_values():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for bad in (-1.0, float("nan"), float("inf")):
        c = sea.Context()
        with pytest.raises(sea.SeaError) as ei:
            c.set_opts(cg_xc_beta_min=bad)
        assert ei.value.status == sea.SEA_E_ARG
        c.close()


def test_fp64_row_tile_cg_against_the_per_pair_kernel(mini):
    """FP64 state: an eager call runs the row-tile CG (one launch per sweep
    over all pairs), a captured plan the per-pair kernel.  Both solve every
    pair to the same true residual: E and W against the oracle, the reported
    residual is the true one (<= rel_tol), and the iteration counts of the
    two CG schedules agree to a few iterations."""
    cell, pl, ref, pairs = mini
    print("case fp64 row-tile CG vs per-pair kernel", flush=True)
    c = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F64)
    phi = _dev(cell.phi)
    W1, E1, s1, st = c.exx_action(phi, cell.N, cell.L, pairs)
    W1 = W1.clone()
    assert st == sea.SEA_OK and np.all(s1["converged"] == 1) and np.all(s1["rel_res"] <= 1e-8)
    plan = c.exx_plan([(phi, cell.N, cell.L, pairs)])
    plan.launch()
    E2, s2, st = plan.results()
    assert st == sea.SEA_OK and np.all(s2["converged"] == 1) and np.all(s2["rel_res"] <= 1e-8)
    W2 = plan.W[0]
    for E, W in ((E1, W1), (E2[0], W2)):
        assert abs(E - ref.E) < 1e-6
        assert np.max(np.abs(W.cpu().numpy() - ref.W)) < 1e-5
    d = np.abs(s1["iters"].astype(int) - s2["iters"].astype(int))
    print(f"iterations row-tile {s1['iters'].mean():.1f} per-pair {s2['iters'].mean():.1f}, max diff {d.max()}",
          flush=True)
    assert d.max() <= 3
    plan.close()
    c.close()


@pytest.mark.parametrize("form", ["f64-zero", "f32-zero", "f64-spectral", "f32-multipole"])
def test_residual_histories(mini, form):
    """Per-pair residual histories: entry 0 is the start's true residual (1
    for a zero start, the reported residual for a start that already meets
    the target), entries 1 .. iters the CG's recursive residual, NaN after;
    a history stays untouched once recording is off."""
    cell, pl, ref, pairs = mini
    print(f"case residual histories {form}", flush=True)
    sdt = sea.SEA_F64 if form.startswith("f64") else sea.SEA_F32
    start = {"zero": sea.SEA_START_ZERO, "spectral": sea.SEA_START_SPECTRAL,
             "multipole": sea.SEA_START_MULTIPOLE}[form.split("-")[1]]
    c = sea.Context(rel_tol=1e-8, stencil_dtype=sdt, start=start)
    phi = _dev(cell.phi)
    L = 600
    hist = c.residual_history(len(pairs), L)
    _, E, s, st = c.exx_action(phi, cell.N, cell.L, pairs)
    assert st == sea.SEA_OK and np.all(s["converged"] == 1)
    h = hist.cpu().numpy()
    for k in range(len(pairs)):
        t = int(s["iters"][k])
        assert t <= L
        assert np.all(np.isfinite(h[k, :t + 1])) and np.all(np.isnan(h[k, t + 1:])), k
        if start == sea.SEA_START_ZERO:
            assert abs(h[k, 0] - 1.0) < 1e-12
        if t == 0:
            assert abs(h[k, 0] - s["rel_res"][k]) <= 1e-12 * max(1.0, s["rel_res"][k])
        else:
            assert h[k, t] < 1e-7 and h[k, t] < h[k, 0]
    print(f"iterations mean {s['iters'].mean():.1f}; first pair {h[0, :min(4, int(s['iters'][0]) + 1)]}", flush=True)
    hist.fill_(7.0)
    c.residual_history(0, -1)
    c.exx_action(phi, cell.N, cell.L, pairs)
    torch.cuda.synchronize()
    assert torch.all(hist == 7.0)
    c.close()
