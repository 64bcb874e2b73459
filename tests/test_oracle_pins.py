"""Pins of the FP64 oracle against closed forms, brute force and library routines.

Nothing here compares the oracle with itself or with the GPU path: every
expected value comes from mathematics the paper relies on (Eq. 7-11, 18-19,
App. A, App. C), from SciPy/NumPy routines used as black boxes, or from a
brute-force alternative (k-d tree neighbour search, FFT free-space solve).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import erf

import oracle
from paper_2208_06097_amd import synth

SIG = synth.SIGMA


# --------------------------------------------------------------------------
# finite-difference Laplacian (App. C: O(h^12), half order M = 6)

def _poly_field(k, h, n, M):
    """f = x^k + 2 y^k - z^k sampled on a padded box centred on the origin."""
    m = n + 2 * M
    ax = (np.arange(m) - (m - 1) / 2.0) * h
    X, Y, Z = ax[None, None, :], ax[:, None, None] * 0 + ax[None, :, None], ax[:, None, None]
    f = X ** k + 2.0 * Y ** k - Z ** k
    f = np.broadcast_to(f, (m, m, m)).copy()
    if k >= 2:
        lap = k * (k - 1) * (X ** (k - 2) + 2.0 * Y ** (k - 2) - Z ** (k - 2))
    else:
        lap = np.zeros((1, 1, 1))
    lap = np.broadcast_to(lap, (m, m, m))[M:M + n, M:M + n, M:M + n]
    return f, -lap


@pytest.mark.parametrize("k", list(range(0, 14)))
def test_fd_laplacian_exact_on_polynomials(k):
    h, n, M = 0.125, 5, 6
    f, want = _poly_field(k, h, n, M)
    got = oracle.neg_lap_padded(f, h, M)
    assert np.max(np.abs(got - want)) <= 1e-9 * max(1.0, np.max(np.abs(want)))


def test_fd_laplacian_order_is_twelve():
    """Degree 14 is the first polynomial the O(h^12) stencil misses."""
    h, n, M = 0.125, 5, 6
    f, want = _poly_field(14, h, n, M)
    got = oracle.neg_lap_padded(f, h, M)
    err = np.max(np.abs(got - want))
    # leading error term: 2 (M!)^2/(2M+2)! h^{2M} f^{(2M+2)}, f^{(14)} = 14! for x^14
    lead = 2 * math.factorial(6) ** 2 / math.factorial(14) * h ** 12 * math.factorial(14) * 3 / 14 / 13
    assert err > 1e-3 * lead


def test_fd_weights_symbol():
    """Fourier symbol c0 + 2 sum c_k cos(k t) = -t^2 + O(t^14)."""
    c = oracle.fd_weights(6)
    for t in (0.05, 0.1, 0.2):
        sym = c[0] + 2 * sum(c[k] * math.cos(k * t) for k in range(1, 7))
        assert abs(sym + t * t) <= 2e-5 * t ** 14 + 5e-15


def test_fd_planted_mistake_is_caught():
    """A lower-order stencil (a plausible slip) fails the degree-13 pin."""
    h, n = 0.125, 5
    f, want = _poly_field(12, h, n, 5)
    got = oracle.neg_lap_padded(f, h, 5)
    assert np.max(np.abs(got - want)) > 1e-9


# --------------------------------------------------------------------------
# real spherical harmonics and the multipole expansion (Eq. 10-11)

def _scipy_real_ylm(l, m, v):
    from scipy.special import sph_harm_y
    r = np.linalg.norm(v)
    theta = math.acos(v[2] / r)
    phi = math.atan2(v[1], v[0])
    if m == 0:
        return float(np.real(sph_harm_y(l, 0, theta, phi)))
    y = sph_harm_y(l, abs(m), theta, phi)
    s = math.sqrt(2.0) * (-1) ** abs(m)
    return float(s * (np.real(y) if m > 0 else np.imag(y)))


def test_real_ylm_match_scipy():
    rng = np.random.default_rng(1)
    for _ in range(25):
        v = rng.standard_normal(3) * rng.uniform(0.1, 5.0)
        got = oracle.real_ylm(6, v)
        for l in range(7):
            for m in range(-l, l + 1):
                assert abs(got[l * l + l + m] - _scipy_real_ylm(l, m, v)) < 1e-13


def test_real_ylm_orthonormal():
    """Gauss-Legendre x uniform-phi quadrature is exact for degree <= 12."""
    xg, wg = np.polynomial.legendre.leggauss(16)
    nphi = 32
    Ys, ws = [], []
    for x, w in zip(xg, wg):
        st = math.sqrt(1 - x * x)
        for kphi in range(nphi):
            ph = 2 * math.pi * kphi / nphi
            Ys.append(oracle.real_ylm(6, [st * math.cos(ph), st * math.sin(ph), x]))
            ws.append(w * 2 * math.pi / nphi)
    Y = np.array(Ys)
    G = (Y * np.array(ws)[:, None]).T @ Y
    assert np.max(np.abs(G - np.eye(49))) < 1e-13


def test_me_single_charge_exact():
    o = np.array([0.3, -0.2, 0.1])
    Q = oracle.moments_points(6, o[None, :], np.array([1.7]), o)
    assert abs(Q[0] - 1.7 / math.sqrt(4 * math.pi)) < 1e-15 and np.max(np.abs(Q[1:])) < 1e-15
    t = o + np.array([2.0, -3.0, 1.5])
    assert abs(oracle.me_eval(6, Q, o, t) - 1.7 / np.linalg.norm(t - o)) < 1e-14


def test_me_point_cluster_converges():
    """ME of a cluster of radius a vs the direct Coulomb sum: error falls with
    l_max and is bounded by sum|q| (a/r)^{l+1} / (r - a)."""
    rng = np.random.default_rng(2)
    a = 1.0
    pos = rng.standard_normal((12, 3))
    pos *= (a * rng.uniform(0, 1, 12) ** (1 / 3) / np.linalg.norm(pos, axis=1))[:, None]
    q = rng.standard_normal(12)
    o = np.zeros(3)
    for r in (4.0, 8.0):
        t = r * np.array([0.48, -0.6, 0.64])
        exact = float(np.sum(q / np.linalg.norm(t - pos, axis=1)))
        errs = []
        for lmax in range(7):
            Q = oracle.moments_points(lmax, pos, q, o)
            errs.append(abs(oracle.me_eval(lmax, Q, o, t) - exact))
        bound = np.sum(np.abs(q)) * (a / r) ** 7 / (r - a)
        assert errs[6] <= bound
        assert errs[6] < errs[2] < errs[0]


# --------------------------------------------------------------------------
# CG on the interior operator (Eq. 9) vs a sparse direct solve

def _sparse_neg_lap(n, h, c):
    M = len(c) - 1
    offs = [0] + [k for k in range(1, M + 1)] + [-k for k in range(1, M + 1)]
    vals = [c[0]] + [c[k] for k in range(1, M + 1)] * 2
    D = sp.diags([np.full(n - abs(o), v) for o, v in zip(offs, vals)], offs, shape=(n, n))
    I = sp.identity(n)
    lap = (sp.kron(sp.kron(I, I), D) + sp.kron(sp.kron(I, D), I) + sp.kron(sp.kron(D, I), I)) / h ** 2
    return (-lap).tocsc()


def test_cg_matches_sparse_direct_solve():
    n, h = 15, 0.3
    rng = np.random.default_rng(3)
    b = rng.standard_normal((n, n, n))
    A = _sparse_neg_lap(n, h, oracle.fd_weights(6))
    want = spla.spsolve(A, b.ravel()).reshape(b.shape)
    x, it, rel, st = oracle.cg(b, h, tol=1e-13)
    assert st == 0 and rel <= 1e-13
    assert np.max(np.abs(x - want)) <= 1e-10 * np.max(np.abs(want))


def test_cg_zero_rhs_and_max_iter():
    x, it, rel, st = oracle.cg(np.zeros((5, 6, 7)), 0.2)
    assert st == 0 and it == 0 and not np.any(x)
    b = np.random.default_rng(4).standard_normal((9, 9, 9))
    x, it, rel, st = oracle.cg(b, 0.2, tol=1e-14, max_iter=3)
    assert st == 1 and it == 3 and rel > 1e-14


# --------------------------------------------------------------------------
# Gaussian closed forms (Eq. 7-9 with a = 0 orbitals)

def _a0_cell(n_mol, L, N, seed):
    cell = synth.make_centres(n_mol, L, N, seed, dmin=1.0)
    cell.a[:] = 0.0
    return synth.fill_orbitals(cell)


def test_normalization_closed_form():
    """Generator check: N^-2 = pi^{3/2} sigma^3 (1 + |a|^2 sigma^2 / 2)."""
    cell = synth.make_centres(1, 13.7, 70, 21, dmin=1.0)
    cell = synth.fill_orbitals(cell)
    h = cell.h
    for i in range(cell.n_occ):
        a = cell.a[i]
        c = cell.centres[i]
        ax = np.arange(cell.N) * h
        d = [ax - c[k] - cell.L * np.round((ax - c[k]) / cell.L) for k in range(3)]
        g = np.exp(-(d[2][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[0][None, None, :] ** 2) / (2 * SIG ** 2))
        f = (1 + a[0] * d[0][None, None, :] + a[1] * d[1][None, :, None] + a[2] * d[2][:, None, None]) * g
        Nn = np.sum(cell.phi[i] * f) / np.sum(f * f)
        want = 1.0 / math.sqrt(math.pi ** 1.5 * SIG ** 3 * (1 + a @ a * SIG ** 2 / 2))
        assert abs(Nn / want - 1) < 1e-12


def test_self_pair_gaussian_potential():
    """P2: a normalized a = 0 orbital: rho is a unit Gaussian charge of std
    sigma/sqrt2, v = erf(r/sigma)/r and e_ii = sqrt(2/pi)/sigma."""
    L, N = 13.7, 70
    cell = _a0_cell(1, L, N, 11)
    cell.centres = cell.centres[:1]
    cell.phi = cell.phi[:1]
    pl = oracle.build_pairs(N, L, cell.centres, 6.0, 6.0)
    v, Q, info = oracle.pair_potential(cell.phi, N, L, pl, 0, tol=1e-12)
    h = L / N
    lo, n = pl.lo[0], pl.n[0]
    c = cell.centres[0]
    X = (lo[0] + np.arange(n[0]))[None, None, :] * h - c[0]
    Y = (lo[1] + np.arange(n[1]))[None, :, None] * h - c[1]
    Z = (lo[2] + np.arange(n[2]))[:, None, None] * h - c[2]
    r = np.sqrt(X * X + Y * Y + Z * Z)
    want = erf(r / SIG) / r
    assert np.max(np.abs(v - want)) < 1e-6
    assert abs(info["e"] / (math.sqrt(2 / math.pi) / SIG) - 1) < 1e-8
    assert abs(Q[0] * math.sqrt(4 * math.pi) - 1.0) < 1e-12


@pytest.fixture(scope="module")
def a0_molecule():
    """One a = 0 molecule (4 orbitals, all 10 pairs kept) on h = 0.1957."""
    L, N = 13.7, 70
    cell = _a0_cell(1, L, N, 31)
    pl = oracle.build_pairs(N, L, cell.centres, 6.0, 6.0)
    res = oracle.exx(cell.phi, N, L, pl, tol=1e-12)
    return cell, pl, res


def _minimg(d, L):
    return d - L * np.round(d / L)


def test_a0_exchange_energy_closed_form(a0_molecule):
    """P3: rho_ij = S_ij x Gaussian(m_ij, sigma/sqrt2), S_ij = exp(-d^2/(4 sigma^2)),
    so E = -sqrt(2/pi)/sigma sum_ordered exp(-d^2/(2 sigma^2))."""
    cell, pl, res = a0_molecule
    assert len(pl) == 10 and res.n_unconverged == 0
    tot = 0.0
    for (i, j) in pl.ij:
        d = np.linalg.norm(_minimg(cell.centres[j] - cell.centres[i], cell.L))
        tot += (1.0 if i == j else 2.0) * math.exp(-d * d / (2 * SIG ** 2))
    want = -math.sqrt(2 / math.pi) / SIG * tot
    assert abs(res.E / want - 1) < 1e-8


def test_a0_ace_matrix_closed_form(a0_molecule):
    """P4: M_ij = sum_k S_ik S_jk erf(R/(sqrt2 sigma))/R, R = |m_ik - m_jk|;
    Cholesky and the Eq. 19 energy then follow from numpy.linalg."""
    cell, pl, res = a0_molecule
    c = cell.centres
    n = cell.n_occ
    S = np.zeros((n, n))
    mid = np.zeros((n, n, 3))
    for i in range(n):
        for j in range(n):
            d = _minimg(c[j] - c[i], cell.L)
            S[i, j] = math.exp(-(d @ d) / (4 * SIG ** 2))
            mid[i, j] = c[i] + 0.5 * d
    Mw = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            for k in range(n):
                R = np.linalg.norm(mid[i, k] - mid[j, k])
                I = (math.sqrt(2) / (SIG * math.sqrt(math.pi)) if R < 1e-12
                     else math.erf(R / (math.sqrt(2) * SIG)) / R)
                Mw[i, j] += S[i, k] * S[j, k] * I
    dV = cell.h ** 3
    ace = oracle.ace_build(cell.phi, res.W, dV)
    assert ace.failed_pivot == 0
    assert np.max(np.abs(ace.M - Mw)) < 1e-7 * np.max(np.abs(Mw))
    Lw = np.linalg.cholesky(Mw)
    assert np.max(np.abs(ace.L - Lw)) < 1e-6 * np.max(np.abs(Lw))
    E_ace = oracle.ace_energy(cell.phi, ace.xi, dV)
    assert abs(E_ace / -np.trace(Mw) - 1) < 1e-7


def _gather(phi, lo, n, N):
    iz = np.mod(lo[2] + np.arange(n[2]), N)
    iy = np.mod(lo[1] + np.arange(n[1]), N)
    ix = np.mod(lo[0] + np.arange(n[0]), N)
    return phi[np.ix_(iz, iy, ix)]


def _fft_free_space(rho, h):
    """Free-space potential of a boxed density by a truncated-Coulomb kernel
    (Spencer-Alavi): K(G) = 4 pi (1 - cos(G Rc))/G^2, K(0) = 2 pi Rc^2, with
    Rc >= the box diagonal and a zero-padded FFT box of side >= 2 Rc."""
    n = rho.shape
    D = math.sqrt(sum((k - 1) ** 2 for k in n)) * h
    nb = int(math.ceil(2 * D / h)) + 2
    nb += nb % 2
    box = np.zeros((nb, nb, nb))
    box[:n[0], :n[1], :n[2]] = rho
    Rc = D * 1.0001
    g = 2 * np.pi * np.fft.fftfreq(nb, d=h)
    gr = 2 * np.pi * np.fft.rfftfreq(nb, d=h)
    G2 = g[:, None, None] ** 2 + g[None, :, None] ** 2 + gr[None, None, :] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        K = 4 * np.pi * (1 - np.cos(np.sqrt(G2) * Rc)) / G2
    K[0, 0, 0] = 2 * np.pi * Rc * Rc
    v = np.fft.irfftn(np.fft.rfftn(box) * K, s=box.shape, axes=(0, 1, 2))
    return v[:n[0], :n[1], :n[2]]


@pytest.fixture(scope="module")
def general_molecule():
    L, N = 13.7, 70
    cell = synth.fill_orbitals(synth.make_centres(1, L, N, 21, dmin=1.0))
    pl = oracle.build_pairs(N, L, cell.centres, 6.0, 6.0)
    return cell, pl


@pytest.mark.parametrize("k", [0, 1])
def test_general_pair_vs_fft_reference(general_molecule, k):
    """P5: a != 0 pairs against a spectral free-space solve of the same
    gathered density; the gap is the O(h^12) FD error plus the l <= 6 cut."""
    cell, pl = general_molecule
    h = cell.h
    v, Q, info = oracle.pair_potential(cell.phi, cell.N, cell.L, pl, k, tol=1e-12)
    i, j = pl.ij[k]
    rho = _gather(cell.phi[i], pl.lo[k], pl.n[k], cell.N) * _gather(cell.phi[j], pl.lo[k], pl.n[k], cell.N)
    vf = _fft_free_space(rho, h)
    e_f = h ** 3 * np.sum(rho * vf)
    assert np.max(np.abs(v - vf)) < 1e-6
    assert abs(info["e"] / e_f - 1) < 1e-7
    assert abs(info["q"] - h ** 3 * rho.sum()) < 1e-12
    # planted slip: dropping every multipole above l = 0 breaks the pin
    v0, _, _ = oracle.pair_potential(cell.phi, cell.N, cell.L, pl, k, tol=1e-10, lmax=0)
    assert np.max(np.abs(v0 - vf)) > 1e-4


# --------------------------------------------------------------------------
# ACE algebra (Eq. 18-19, App. A)

def test_cholesky_recovers_constructed_factor():
    rng = np.random.default_rng(5)
    n = 40
    L0 = np.tril(rng.standard_normal((n, n))) * (0.5 / math.sqrt(n))
    L0[np.diag_indices(n)] = rng.uniform(0.5, 2.0, n)
    A = L0 @ L0.T
    Lo, fail = oracle.cholesky(A)
    assert fail == 0 and np.max(np.abs(Lo - L0)) < 1e-12 * np.max(np.abs(L0)) * n
    B = A.copy()
    B[7, 7] = -1.0
    _, fail = oracle.cholesky(B)
    assert fail == 8


def test_ace_identity_symmetric_operator():
    """P7: for W_i = u(r) phi_i with u > 0, M is symmetric PD, and the ACE
    operator reproduces the action exactly: K phi_i = -W_i, E_ACE = -tr M."""
    cell = synth.mini(seed=9)
    dV = cell.h ** 3
    rng = np.random.default_rng(6)
    u = 0.5 + rng.uniform(0, 1, cell.phi.shape[1:])
    W = cell.phi * u[None]
    ace = oracle.ace_build(cell.phi, W, dV)
    assert ace.failed_pivot == 0
    K = oracle.ace_apply(ace.xi, cell.phi, dV)
    assert np.max(np.abs(K + W)) < 1e-10 * np.max(np.abs(W))
    assert abs(oracle.ace_energy(cell.phi, ace.xi, dV) / -np.trace(ace.M) - 1) < 1e-12
    assert np.all(np.linalg.eigvalsh(ace.Mbar) > 0)


# --------------------------------------------------------------------------
# pair selection and domains (Sec. II.B; cube reading)

def test_pair_list_vs_kdtree():
    from scipy.spatial import cKDTree
    cell = synth.config1(with_phi=False)
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, 6.0)
    tree = cKDTree(cell.centres, boxsize=cell.L)
    want = set(tree.query_pairs(6.0)) | {(i, i) for i in range(cell.n_occ)}
    got = {tuple(x) for x in pl.ij.tolist()}
    # query_pairs keeps d <= r; the method keeps d < r: equal unless d == r exactly
    assert got == want
    h = cell.h
    w = math.ceil(6.0 / h - 1e-12)
    assert np.all(pl.n == 2 * w + 1)
    for k, (i, j) in enumerate(pl.ij):
        m = cell.centres[i] + 0.5 * _minimg(cell.centres[j] - cell.centres[i], cell.L)
        kc = pl.lo[k] + w
        assert np.all(np.abs(kc * h - m) <= 0.5 * h + 1e-12)
        assert np.allclose(pl.origin[k], kc * h, rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# the action as a whole

@pytest.fixture(scope="module")
def mini_exx():
    cell = synth.mini()
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
    return cell, pl, oracle.exx(cell.phi, cell.N, cell.L, pl, tol=1e-12)


def test_exx_scatter_by_definition(mini_exx):
    """W_i = sum over kept pairs of v_ij phi_j on the pair domain (Eq. 13-14),
    rebuilt here with numpy index arithmetic from per-pair potentials."""
    cell, pl, res = mini_exx
    N = cell.N
    W = np.zeros_like(cell.phi)
    E = 0.0
    for k in range(len(pl)):
        v, _, info = oracle.pair_potential(cell.phi, N, cell.L, pl, k, tol=1e-12)
        i, j = pl.ij[k]
        lo, n = pl.lo[k], pl.n[k]
        iz = np.mod(lo[2] + np.arange(n[2]), N)[:, None, None]
        iy = np.mod(lo[1] + np.arange(n[1]), N)[None, :, None]
        ix = np.mod(lo[0] + np.arange(n[0]), N)[None, None, :]
        np.add.at(W[i], (iz, iy, ix), v * cell.phi[j][iz, iy, ix])
        if i != j:
            np.add.at(W[j], (iz, iy, ix), v * cell.phi[i][iz, iy, ix])
        E -= (1 if i == j else 2) * info["e"]
    assert np.max(np.abs(W - res.W)) < 1e-13
    assert abs(E - res.E) < 1e-12


def test_exx_energy_equals_minus_trace_M(mini_exx):
    """Eq. 8 energy = -tr M: an exact identity of the scatter vs the energy."""
    cell, pl, res = mini_exx
    ace = oracle.ace_build(cell.phi, res.W, cell.h ** 3)
    assert abs(res.E / -np.trace(ace.M) - 1) < 1e-12
    assert ace.failed_pivot == 0
    assert abs(oracle.ace_energy(cell.phi, ace.xi, cell.h ** 3) / res.E - 1) < 1e-8


def test_exx_thread_count_invariant(mini_exx):
    cell, pl, res = mini_exx
    r1 = oracle.exx(cell.phi, cell.N, cell.L, pl, tol=1e-12, n_threads=1)
    assert r1.E == res.E and np.array_equal(r1.W, res.W)


def test_exx_wrapped_domain_wider_than_cell():
    """Domain (35 points) wider than the cell (30): duplicates accumulate and
    the trace identity still holds exactly."""
    cell = synth.mini(n_mol=2)
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, 5.0)
    assert pl.n[0, 0] > cell.N
    res = oracle.exx(cell.phi, cell.N, cell.L, pl, tol=1e-11)
    M = cell.h ** 3 * cell.phi.reshape(cell.n_occ, -1) @ res.W.reshape(cell.n_occ, -1).T
    assert abs(res.E / -np.trace(M) - 1) < 1e-12


def test_ace_eigen_scheme_closed_form():
    """App. A scheme on a constructed case: orthonormal orbitals Phi and
    W = G Phi with G symmetric of mixed-sign spectrum give Mbar = G, and
    K = -xi xi^T acts on u_k = sum_m Q_mk phi_m as -|lambda_k| (eigen
    scheme); the Cholesky scheme reports the non-positive pivot.  For a
    positive definite G both schemes give the same K."""
    rng = np.random.default_rng(5)
    n, ng, dV = 12, 400, 0.5
    A = rng.standard_normal((ng, n))
    Qf, _ = np.linalg.qr(A)
    phi = Qf.T / np.sqrt(dV)                       # dV phi phi^T = I
    lam = np.array([3.0, 2.5, 2.0, 1.5, 1.0, 0.8, 0.5, 0.3, -0.2, -0.7, -1.1, 0.05])
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    G = U @ np.diag(lam) @ U.T
    W = G @ phi
    res = oracle.ace_build(phi, W, dV, decomp="eigen")
    assert np.allclose(res.Mbar, G, atol=1e-12)
    K = lambda v: -res.xi.T @ (dV * (res.xi @ v))   # noqa: E731
    for k in range(n):
        u = U[:, k] @ phi
        assert np.allclose(K(u), -abs(lam[k]) * u, atol=1e-10)
    assert oracle.ace_build(phi, W, dV).failed_pivot > 0
    Gp = U @ np.diag(np.abs(lam)) @ U.T
    Wp = Gp @ phi
    r1 = oracle.ace_build(phi, Wp, dV, decomp="eigen")
    r2 = oracle.ace_build(phi, Wp, dV)
    K1 = r1.xi.T @ r1.xi
    K2 = r2.xi.T @ r2.xi
    assert np.allclose(K1, K2, atol=1e-10)


# --------------------------------------------------------------------------
# regularized multipole start v_ME (the CG's initial guess; the paper leaves
# it open, the reading: q erf(r/r_s)/r plus the l >= 1 terms of Eq. 10
# damped by (1 - exp(-r^2/r_s^2))^(l+1), r_s = sqrt(2<r^2>/3))

def _on_grid_a0_self_pair(L=13.7, N=70):
    """One a = 0 orbital centred on a grid point: its self-pair domain is
    centred there too (origin = centre), and every moment with l >= 1
    vanishes by the cube's symmetry up to the grid sum's spectral error."""
    cell = synth.make_centres(1, L, N, 11, dmin=1.0)
    cell.centres = np.full((1, 3), 35 * (L / N))
    cell.a = np.zeros((1, 3))
    cell = synth.fill_orbitals(cell)
    pl = oracle.build_pairs(N, L, cell.centres, 6.0, 6.0)
    assert np.allclose(pl.origin[0], cell.centres[0], atol=1e-12)
    return cell, pl


def test_me_start_self_pair_closed_form():
    """a = 0 self pair, origin at the centre: rho is a unit Gaussian charge
    exp(-r^2/sigma^2) / (pi sigma^2)^{3/2}, <r^2> = 3 sigma^2 / 2, so
    r_s = sigma and v_ME = erf(r/sigma)/r exactly (the exact potential, P2),
    2/(sigma sqrt(pi)) at the centre."""
    cell, pl = _on_grid_a0_self_pair()
    v = oracle.pair_me_start(cell.phi, cell.N, cell.L, pl, 0)
    h = cell.h
    lo, n = pl.lo[0], pl.n[0]
    c = cell.centres[0]
    X = (lo[0] + np.arange(n[0]))[None, None, :] * h - c[0]
    Y = (lo[1] + np.arange(n[1]))[None, :, None] * h - c[1]
    Z = (lo[2] + np.arange(n[2]))[:, None, None] * h - c[2]
    r = np.sqrt(X * X + Y * Y + Z * Z)
    with np.errstate(invalid="ignore", divide="ignore"):
        want = np.where(r > 0, erf(r / SIG) / np.where(r > 0, r, 1.0), 2.0 / (SIG * math.sqrt(math.pi)))
    assert np.max(np.abs(v - want)) < 1e-9
    assert abs(v[n[2] // 2, n[1] // 2, n[0] // 2] - 2.0 / (SIG * math.sqrt(math.pi))) < 1e-9
    # planted slip: r_s from <r^2> without the factor 2/3 (r_s = sigma sqrt(3/2))
    # changes the start by far more than the bar
    rs_bad = SIG * math.sqrt(1.5)
    with np.errstate(invalid="ignore", divide="ignore"):
        bad = np.where(r > 0, erf(r / rs_bad) / np.where(r > 0, r, 1.0), 2.0 / (rs_bad * math.sqrt(math.pi)))
    assert np.max(np.abs(bad - want)) > 1e-2


def _general_self_pair_cell():
    cell = synth.mini(seed=7)
    pl = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, 4.0)
    k = int(np.flatnonzero(pl.ij[:, 0] == pl.ij[:, 1])[0])
    return cell, pl, k


def test_me_start_far_field_is_the_expansion():
    """Far from the charge (r >> r_s) the damping is 1 to machine precision
    and v_ME is the multipole expansion of Eq. 10 itself (pinned against the
    direct Coulomb sum, P10), with the pair's own moments (Eq. 11)."""
    cell, pl, _ = _general_self_pair_cell()
    k = int(np.flatnonzero(pl.ij[:, 0] != pl.ij[:, 1])[0])   # a ≠ 0, i ≠ j: every l present
    v = oracle.pair_me_start(cell.phi, cell.N, cell.L, pl, k)
    _, Q, _ = oracle.pair_potential(cell.phi, cell.N, cell.L, pl, k, tol=0.0, max_iter=0)
    assert np.max(np.abs(Q[1:])) > 1e-4 * abs(Q[0]) or abs(Q[0]) < 1e-3
    h = cell.h
    lo, n, o = pl.lo[k], pl.n[k], pl.origin[k]
    for (z, y, x) in [(0, 0, 0), (n[2] - 1, 0, n[0] - 1), (0, n[1] - 1, n[0] - 1), (n[2] - 1, n[1] - 1, 0)]:
        t = np.array([(lo[0] + x) * h, (lo[1] + y) * h, (lo[2] + z) * h])
        want = oracle.me_eval(6, Q, o, t)
        assert abs(v[z, y, x] - want) <= 1e-12 * abs(want)


def test_me_start_dipole_term_vanishes_smoothly_at_the_origin():
    """Small-r limit of the damped l = 1 term.  With Y_1m(d/r) = sqrt(3/(4 pi))
    d_m / r the l = 1 term of Eq. 10 is sqrt(4 pi/3) (Q_1 . d) / r^3; damped
    by (1 - e^{-r^2/r_s^2})^2 ~ r^4/r_s^4 it vanishes at the origin like
    sqrt(4 pi/3) (Q_1 . d) r / r_s^4.  Along an axis e through the origin the
    odd part [v(o + h e) - v(o - h e)] / 2 comes from the odd l only, and the
    l = 3 terms are damped by a further r^4: it is the l = 1 term
    sqrt(4 pi/3) Q_e (1 - e^{-h^2/r_s^2})^2 / h^2 to a few percent (Q_e =
    Q_11, Q_1-1, Q_10 for x, y, z).  A damping power of l instead of l + 1
    would make it 1/(1 - e^{-h^2/r_s^2}) times larger (8x here); a swapped
    or sign-flipped real harmonic would put another axis's moment there."""
    cell, pl, k = _general_self_pair_cell()
    v = oracle.pair_me_start(cell.phi, cell.N, cell.L, pl, k)
    _, Q, info = oracle.pair_potential(cell.phi, cell.N, cell.L, pl, k, tol=0.0, max_iter=0)
    h = cell.h
    lo, n, o = pl.lo[k], pl.n[k], pl.origin[k]
    c = [int(round(o[a] / h)) - lo[a] for a in range(3)]
    assert np.allclose((np.array(c) + lo) * h, o)
    # r_s from the gathered density (|rho|-weighted second moment about o)
    iz, iy, ix = (np.mod(lo[a] + np.arange(n[a]), cell.N) for a in (2, 1, 0))
    i, j = pl.ij[k]
    rho = cell.phi[i][np.ix_(iz, iy, ix)] * cell.phi[j][np.ix_(iz, iy, ix)]
    X = (lo[0] + np.arange(n[0]))[None, None, :] * h - o[0]
    Y = (lo[1] + np.arange(n[1]))[None, :, None] * h - o[1]
    Z = (lo[2] + np.arange(n[2]))[:, None, None] * h - o[2]
    rs = math.sqrt(2.0 / 3.0 * np.sum(np.abs(rho) * (X * X + Y * Y + Z * Z)) / np.sum(np.abs(rho)))
    damp = 1.0 - math.exp(-h * h / rs ** 2)
    for ax, qi in ((0, 3), (1, 1), (2, 2)):
        assert abs(Q[qi]) > 1e-2
        e = [0, 0, 0]
        e[ax] = 1
        odd = (v[c[2] + e[2], c[1] + e[1], c[0] + e[0]] - v[c[2] - e[2], c[1] - e[1], c[0] - e[0]]) / 2
        want = math.sqrt(4 * math.pi / 3) * Q[qi] * damp ** 2 / h ** 2
        assert abs(odd - want) <= 0.05 * abs(want)


# --------------------------------------------------------------------------
# successive idempotency (App. B)

def _orthonormal_set(n, ng, dV, seed):
    """n + 1 grid vectors orthonormal in <f, g> = dV sum f g."""
    A = np.random.default_rng(seed).standard_normal((ng, n + 1))
    Qf, _ = np.linalg.qr(A)
    return Qf.T / np.sqrt(dV)


def test_successive_idempotency_closed_form():
    """One orbital of an orthonormal set rotated by theta out of the
    occupied space (towards a vector orthogonal to it): the overlap matrix
    is diag(cos theta, 1, ..., 1), so dI = 1 - (n - sin^2 theta)/n =
    sin^2 theta / n.  Two orbitals rotated by theta_1, theta_2 towards two
    such vectors: (sin^2 theta_1 + sin^2 theta_2) / n.  A rotation within
    the occupied space leaves the projector, so dI = 0."""
    n, ng, dV = 6, 300, 0.37
    B = _orthonormal_set(n + 1, ng, dV, 3)     # n + 2 vectors
    old = B[:n]
    for th in (0.0, 0.1, 0.7, math.pi / 2):
        new = old.copy()
        new[2] = math.cos(th) * old[2] + math.sin(th) * B[n]
        assert abs(oracle.successive_idempotency(new, old, dV) - math.sin(th) ** 2 / n) < 1e-13
    t1, t2 = 0.3, 1.1
    new = old.copy()
    new[0] = math.cos(t1) * old[0] + math.sin(t1) * B[n]
    new[4] = math.cos(t2) * old[4] + math.sin(t2) * B[n + 1]
    want = (math.sin(t1) ** 2 + math.sin(t2) ** 2) / n
    assert abs(oracle.successive_idempotency(new, old, dV) - want) < 1e-13
    U = np.linalg.qr(np.random.default_rng(4).standard_normal((n, n)))[0]
    assert abs(oracle.successive_idempotency(U @ old, old, dV)) < 1e-13


def test_successive_idempotency_planted_slips_are_caught():
    """Plausible slips in dI (the inner product without dV, or squared dV;
    N_occ^2 in the denominator; the overlap not squared) all miss the
    closed form sin^2 theta / n of the single-rotation case."""
    n, ng, dV, th = 6, 300, 0.37, 0.7
    B = _orthonormal_set(n, ng, dV, 5)
    old = B[:n]
    new = old.copy()
    new[1] = math.cos(th) * old[1] + math.sin(th) * B[n]
    want = math.sin(th) ** 2 / n
    S = lambda d: d * (new @ old.T)                              # noqa: E731
    slips = [1.0 - np.sum(S(1.0) ** 2) / n,                      # dV dropped
             1.0 - np.sum(S(dV * dV) ** 2) / n,                  # dV squared
             1.0 - np.sum(S(dV) ** 2) / n ** 2,                  # N_occ^2
             1.0 - np.sum(np.abs(S(dV))) / n]                    # not squared
    for s in slips:
        assert abs(s - want) > 1e-3
    assert abs(oracle.successive_idempotency(new, old, dV) - want) < 1e-13
