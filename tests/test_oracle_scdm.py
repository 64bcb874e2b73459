"""Pins of the oracle's SCDM localization (Eq. 1-6) and back-rotation (Eq. 15).

The pivot order against LAPACK's column-pivoted QR (scipy) and against a
brute-force greedy choice by least squares; invariance of the pivots and the
localized orbitals under any rotation of the input orbitals (both depend
only on the density matrix); exact recovery of disjoint-support orbitals
(closed form); orthogonality of U and of the localized orbitals; the
back-rotation undoing the forward one.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2208_06097_amd import synth


def _orthonormal(A):
    """Orthonormal rows spanning the rows of A (Euclidean), by SVD."""
    u, s, vt = np.linalg.svd(A, full_matrices=False)
    return u @ vt


def _mini_phi(n_mol=3, seed=7):
    c = synth.mini(seed=seed, n_mol=n_mol)
    return c, c.phi.reshape(c.phi.shape[0], -1)


@pytest.mark.parametrize("kind", ["random", "mini"])
def test_pivots_match_lapack_qrcp(kind):
    if kind == "random":
        A = np.random.default_rng(3).standard_normal((8, 300))
    else:
        _, A = _mini_phi()
    piv, rdiag = oracle.scdm_pivots(A)
    _, R, P = sla.qr(A, pivoting=True, mode="economic")
    n = A.shape[0]
    assert np.array_equal(piv, P[:n])
    np.testing.assert_allclose(rdiag, np.abs(np.diag(R)), rtol=1e-10)
    assert np.all(np.diff(rdiag) <= 1e-12 * rdiag[0])     # |R_kk| never grows


def test_pivots_brute_force_least_squares():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((5, 40)) * rng.uniform(0.2, 3.0, size=40)[None, :]
    piv, rdiag = oracle.scdm_pivots(A)
    chosen = []
    for k in range(A.shape[0]):
        best, arg = -1.0, -1
        for c in range(A.shape[1]):
            if c in chosen:
                continue
            if chosen:
                B = A[:, chosen]
                coef = np.linalg.lstsq(B, A[:, c], rcond=None)[0]
                d = np.linalg.norm(A[:, c] - B @ coef)
            else:
                d = np.linalg.norm(A[:, c])
            if d > best:
                best, arg = d, c
        assert piv[k] == arg, k
        assert abs(rdiag[k] - best) < 1e-12 * max(1.0, best)
        chosen.append(arg)


def test_rotation_invariance():
    _, A = _mini_phi(n_mol=3, seed=9)
    G = synth.random_rotation(A.shape[0], 5)
    assert np.allclose(G.T @ G, np.eye(A.shape[0]), atol=1e-12)
    r0 = oracle.scdm(A)
    r1 = oracle.scdm(G.T @ A)           # orbitals phi'_k = sum_j phi_j G_jk
    assert np.array_equal(r0.piv, r1.piv)
    scale = np.abs(r0.phi_loc).max()
    assert np.abs(r1.phi_loc - r0.phi_loc).max() < 1e-11 * scale
    np.testing.assert_allclose(r1.U, G.T @ r0.U, atol=1e-11)


def test_disjoint_support_orbitals_recovered():
    rng = np.random.default_rng(4)
    n, per = 6, 25
    A = np.zeros((n, n * per + 17))
    for i in range(n):
        A[i, i * per:(i + 1) * per] = rng.standard_normal(per)
    A /= np.linalg.norm(A, axis=1)[:, None]
    G = synth.random_rotation(n, 8)
    r = oracle.scdm(G.T @ A)
    # each localized orbital is one of the originals up to sign
    O = r.phi_loc.reshape(n, -1) @ A.T
    assert np.allclose(np.sort(np.abs(O), axis=1)[:, -1], 1.0, atol=1e-12)
    assert np.allclose(np.sort(np.abs(O), axis=1)[:, :-1], 0.0, atol=1e-12)
    assert sorted(np.argmax(np.abs(O), axis=1).tolist()) == list(range(n))


def test_unitary_and_same_space():
    c, A = _mini_phi(n_mol=4, seed=12)
    Ao = _orthonormal(A)
    G = synth.random_rotation(Ao.shape[0], 21)
    r = oracle.scdm(G.T @ Ao)
    n = Ao.shape[0]
    np.testing.assert_allclose(r.U.T @ r.U, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(r.U @ r.U.T, np.eye(n), atol=1e-12)
    F = r.phi_loc.reshape(n, -1)
    np.testing.assert_allclose(F @ F.T, np.eye(n), atol=1e-12)
    # same occupied space: the projector onto the rows is unchanged
    np.testing.assert_allclose(F.T @ (F @ Ao.T), Ao.T, atol=1e-12)


def test_localizes_rotated_orbitals():
    """Delocalized inputs (orthonormalized synthetic orbitals under a dense
    rotation) come back localized: every SCDM orbital keeps most of its
    weight inside a sphere of 3 bohr about its own peak, as the originals do,
    while the rotated inputs do not."""
    c, A = _mini_phi(n_mol=4, seed=12)
    Ao = _orthonormal(A)
    G = synth.random_rotation(Ao.shape[0], 21)
    D = G.T @ Ao
    r = oracle.scdm(D)
    N, L = c.N, c.L
    h = L / N
    idx = np.indices((N, N, N)).reshape(3, -1)[::-1].T * h     # (x, y, z) of each grid point

    def weight_near_peak(f):
        p = idx[np.argmax(f * f)]
        d = idx - p
        d -= L * np.round(d / L)
        return float(np.sum((f * f)[np.sum(d * d, axis=1) < 9.0]) / np.sum(f * f))

    w_loc = [weight_near_peak(f) for f in r.phi_loc.reshape(A.shape[0], -1)]
    w_del = [weight_near_peak(f) for f in D]
    w_org = [weight_near_peak(f) for f in Ao]
    assert min(w_loc) > 0.9 and min(w_org) > 0.9
    assert np.mean(w_del) < 0.6 and min(w_loc) > max(w_del) + 0.2


def test_back_rotation_inverts_forward():
    _, A = _mini_phi(n_mol=3, seed=9)
    G = synth.random_rotation(A.shape[0], 5)
    D = G.T @ A
    r = oracle.scdm(D)
    np.testing.assert_allclose(oracle.back_rotate(r.phi_loc, r.U), D, atol=1e-12 * np.abs(D).max())
    # a transposed U would not undo it (U is not symmetric)
    assert np.abs(oracle.back_rotate(r.phi_loc, r.U.T) - D).max() > 1e-3 * np.abs(D).max()


def test_residual_norms_brute_force():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((6, 50))
    piv, rdiag = oracle.scdm_pivots(A)
    for k in range(A.shape[0]):
        nr = oracle.qrcp_residual_norms(A, piv[:k])
        nr[piv[:k]] = -1
        assert np.argmax(nr) == piv[k]
        assert abs(np.sqrt(nr[piv[k]]) - rdiag[k]) < 1e-12 * rdiag[0]


def test_rank_deficient_raises():
    A = np.zeros((3, 20))
    A[0, :5] = 1.0
    A[1, :5] = 2.0          # same column space as row 0
    A[2, 10:] = 1.0
    with pytest.raises(ValueError):
        oracle.scdm_pivots(A)
