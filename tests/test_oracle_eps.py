"""Pins of the oracle's epsilon-driven domains and pair screening (Eq. 16-17).

Brute force over every cyclic index run on small grids, the coverage bound,
an isotropic Gaussian's closed-form marginal, the eps -> 0 limit, the
intersection against boolean masks, and the overlap integral by direct sums.
"""
import math

import numpy as np
import pytest
from scipy.special import erfinv

import oracle
from paper_2208_06097_amd import synth


def _marginals(f):
    g = f * f
    return [g.sum(axis=(0, 1)), g.sum(axis=(0, 2)), g.sum(axis=(1, 2))]   # x, y, z (array is [z][y][x])


def _runs(m):
    """All cyclic runs (start, length, mass) of a 1-D marginal, brute force."""
    n = len(m)
    out = []
    for ln in range(1, n + 1):
        for s in range(n if ln < n else 1):
            out.append((s, ln, float(sum(m[(s + t) % n] for t in range(ln)))))
    return out


@pytest.mark.parametrize("eps", [1e-2, 10 ** -3.5])
def test_boxes_are_the_shortest_runs_brute_force(eps):
    c = synth.make_centres(1, 4.0, 12, seed=3, dmin=1.0)
    c = synth.fill_orbitals(c)
    lo, ln = oracle.eps_boxes(c.phi, c.N, eps)
    for i in range(c.n_occ):
        for a, m in enumerate(_marginals(c.phi[i])):
            T = float(np.sum(m))
            ok = [(s, L_, w) for s, L_, w in _runs(m) if w >= (1 - eps / 3) * T]
            Lmin = min(L_ for _, L_, _ in ok)
            assert ln[i, a] == Lmin
            if Lmin < c.N:
                best = max(w for s, L_, w in ok if L_ == Lmin)
                s_best = min(s for s, L_, w in ok if L_ == Lmin and w == best)
                assert lo[i, a] == s_best


def test_box_coverage_bound():
    c = synth.mini(seed=8)
    for eps in (1e-2, 1e-3, 1e-4):
        lo, ln = oracle.eps_boxes(c.phi, c.N, eps)
        for i in range(c.n_occ):
            idx = [np.mod(lo[i, a] + np.arange(ln[i, a]), c.N) for a in range(3)]
            inside = np.sum(c.phi[i][np.ix_(idx[2], idx[1], idx[0])] ** 2)
            assert inside >= (1 - eps) * np.sum(c.phi[i] ** 2)


def test_isotropic_gaussian_closed_form():
    """phi^2 = exp(-r^2/sigma^2) has x-marginal ~ exp(-x^2/sigma^2): the run
    holding 1 - eps/3 spans 2 sigma erfinv(1 - eps/3) (within the grid step)."""
    N, L = 60, 12.0
    h = L / N
    c = synth.make_centres(1, L, N, seed=1, dmin=1.0)
    c.centres[0] = [30 * h, 30 * h, 30 * h]
    c.a[0] = 0.0
    c = synth.fill_orbitals(c)
    for eps in (1e-2, 1e-3, 10 ** -3.5):
        lo, ln = oracle.eps_boxes(c.phi, N, eps)
        w = 2 * synth.SIGMA * erfinv(1 - eps / 3)
        for a in range(3):
            assert abs(ln[0, a] * h - w) <= 2 * h, (eps, a, ln[0, a] * h, w)
            # centred on the Gaussian
            assert abs(lo[0, a] + (ln[0, a] - 1) / 2 - 30) <= 0.5


def test_eps_zero_is_the_whole_cell():
    c = synth.mini(seed=9)
    lo, ln = oracle.eps_boxes(c.phi, c.N, 0.0)
    assert np.all(ln == c.N) and np.all(lo == 0)


def test_pair_boxes_and_overlap_by_masks():
    c = synth.mini(seed=7)
    eps = 10 ** -3.5
    lo, ln = oracle.eps_boxes(c.phi, c.N, eps)
    pl, S = oracle.eps_pairs(c.phi, c.N, c.L, lo, ln, 0.0)
    h3 = c.h ** 3
    kept = set()
    for k in range(len(pl)):
        i, j = pl.ij[k]
        kept.add((i, j))
        for a in range(3):
            mi = np.zeros(c.N, bool)
            mi[np.mod(lo[i, a] + np.arange(ln[i, a]), c.N)] = True
            mj = np.zeros(c.N, bool)
            mj[np.mod(lo[j, a] + np.arange(ln[j, a]), c.N)] = True
            mk = np.zeros(c.N, bool)
            mk[np.mod(pl.lo[k, a] + np.arange(pl.n[k, a]), c.N)] = True
            assert np.array_equal(mk, mi & mj)          # single-piece intersections here
            assert pl.lo[k, a] >= lo[i, a] and pl.lo[k, a] + pl.n[k, a] <= lo[i, a] + ln[i, a]
            assert abs(pl.origin[k, a] / c.h - (pl.lo[k, a] + 0.5 * (pl.n[k, a] - 1))) < 1e-12
        idx = [np.mod(pl.lo[k, a] + np.arange(pl.n[k, a]), c.N) for a in range(3)]
        box = np.ix_(idx[2], idx[1], idx[0])
        s_ref = h3 * np.sum(np.abs(c.phi[i][box] * c.phi[j][box]))
        assert abs(S[k] - s_ref) <= 1e-13 * max(1.0, s_ref)
    # every pair with an empty intersection on some axis is absent; self pairs present
    for i in range(c.n_occ):
        assert (i, i) in kept
        for j in range(i + 1, c.n_occ):
            empty = False
            for a in range(3):
                mi = np.zeros(c.N, bool)
                mi[np.mod(lo[i, a] + np.arange(ln[i, a]), c.N)] = True
                mj = np.zeros(c.N, bool)
                mj[np.mod(lo[j, a] + np.arange(ln[j, a]), c.N)] = True
                empty |= not np.any(mi & mj)
            assert ((i, j) in kept) == (not empty)


def test_screening_is_monotone_in_delta():
    c = synth.mini(seed=7)
    lo, ln = oracle.eps_boxes(c.phi, c.N, 1e-3)
    p0, S0 = oracle.eps_pairs(c.phi, c.N, c.L, lo, ln, 0.0)
    p1, S1 = oracle.eps_pairs(c.phi, c.N, c.L, lo, ln, 1e-3)
    p2, S2 = oracle.eps_pairs(c.phi, c.N, c.L, lo, ln, 1e-2)
    a0 = {tuple(x) for x in p0.ij}
    a1 = {tuple(x) for x in p1.ij}
    a2 = {tuple(x) for x in p2.ij}
    assert a2 <= a1 <= a0 and len(a2) < len(a0)
    assert a1 == {tuple(p0.ij[k]) for k in range(len(p0)) if S0[k] >= 1e-3}


def test_padding_grows_boxes_symmetrically_within_the_cell():
    c = synth.mini(seed=7)
    lo, ln = oracle.eps_boxes(c.phi, c.N, 1e-3)
    p0, S0 = oracle.eps_pairs(c.phi, c.N, c.L, lo, ln, 1e-3, pad=0)
    for pad in (3, 9):
        p, S = oracle.eps_pairs(c.phi, c.N, c.L, lo, ln, 1e-3, pad=pad)
        assert np.array_equal(p.ij, p0.ij) and np.array_equal(S, S0)   # screening on the unpadded boxes
        want_n = np.minimum(p0.n + 2 * pad, c.N)
        assert np.array_equal(p.n, want_n)
        assert np.array_equal(p.lo, p0.lo - (want_n - p0.n) // 2)
        assert np.all(p.lo <= p0.lo) and np.all(p.lo + p.n >= p0.lo + p0.n)
        assert np.allclose(p.origin / c.h, p.lo + 0.5 * (p.n - 1), atol=1e-12)


def test_dboxes_are_the_orbital_boxes_in_the_pair_frame():
    c = synth.mini(seed=7)
    lo, ln = oracle.eps_boxes(c.phi, c.N, 1e-3)
    pl, S, db = oracle.eps_pairs(c.phi, c.N, c.L, lo, ln, 1e-3, pad=2, with_dbox=True)
    for k in range(len(pl)):
        i, j = pl.ij[k]
        for a in range(3):
            # each W box = the orbital box (in some frame) joined with the pair domain
            if i == j:
                n0 = min(2 * ln[i, a], c.N)
                l0 = lo[i, a] - (n0 - ln[i, a]) // 2
            else:
                n0, l0 = ln[j, a], lo[j, a]
            for side, (ll, nn) in enumerate(((l0, n0), (lo[i, a], ln[i, a]))):
                b0, bn = db[k, 6 * side + a], db[k, 6 * side + 3 + a]
                shifts = [ll + m * c.N for m in (-1, 0, 1)]
                ok = any(b0 == min(sh, pl.lo[k, a]) and
                         bn == min(max(sh + nn, pl.lo[k, a] + pl.n[k, a]) - min(sh, pl.lo[k, a]), c.N)
                         for sh in shifts)
                assert ok, (k, a, side)
                assert b0 <= pl.lo[k, a] and b0 + bn >= min(pl.lo[k, a] + pl.n[k, a], b0 + c.N)
            # nearest frame: centres within half a cell of the pair box centre
            for side in (0, 1):
                cen = db[k, 6 * side + a] + 0.5 * db[k, 6 * side + 3 + a]
                assert abs(cen - (pl.lo[k, a] + 0.5 * pl.n[k, a])) <= c.N / 2


def test_exx_with_dboxes_equal_to_the_domains_is_the_plain_action():
    c = synth.mini(seed=7)
    lo, ln = oracle.eps_boxes(c.phi, c.N, 1e-3)
    pl, S = oracle.eps_pairs(c.phi, c.N, c.L, lo, ln, 1e-3, pad=2)
    db = np.concatenate([pl.lo, pl.n, pl.lo, pl.n], axis=1).astype(np.int32)
    r0 = oracle.exx(c.phi, c.N, c.L, pl, tol=1e-10)
    r1 = oracle.exx(c.phi, c.N, c.L, pl, tol=1e-10, dbox=db)
    assert r1.E == r0.E and np.array_equal(r1.W, r0.W)


def test_far_field_of_a_spherical_orbital_is_the_monopole():
    """One spherical orbital (a = 0): on the doubled box, outside the pair
    domain, W = (q / r) phi with q = h^3 sum rho over the domain.  The density
    cut to a box keeps the box's l = 4, 6 (and, for a box of even extent
    around the centre, odd) moments, all carried by the mass the cut removed
    (<= eps), so the far field is the monopole to a relative eps."""
    N, L = 48, 9.6
    h = L / N
    c = synth.make_centres(1, L, N, seed=2, dmin=1.0)
    c.centres = c.centres[:1].copy()
    c.a = np.zeros((1, 3))
    c.centres[0] = [24 * h, 24 * h, 24 * h]
    c = synth.fill_orbitals(c)
    lo, ln = oracle.eps_boxes(c.phi, N, 1e-3)
    pl, S, db = oracle.eps_pairs(c.phi, N, L, lo, ln, 1e-3, pad=0, with_dbox=True)
    assert len(pl) == 1
    r = oracle.exx(c.phi, N, L, pl, tol=1e-12, dbox=db)
    box = [np.arange(pl.lo[0, a], pl.lo[0, a] + pl.n[0, a]) for a in range(3)]
    rho = c.phi[0][np.ix_(box[2] % N, box[1] % N, box[0] % N)] ** 2
    q = h ** 3 * rho.sum()
    checked = 0
    for z in range(db[0, 2], db[0, 2] + db[0, 5], 3):
        for y in range(db[0, 1], db[0, 1] + db[0, 4], 3):
            for x in range(db[0, 0], db[0, 0] + db[0, 3], 3):
                inside = all(pl.lo[0, a] <= p < pl.lo[0, a] + pl.n[0, a] for a, p in enumerate((x, y, z)))
                if inside:
                    continue
                d = np.array([x, y, z]) * h - pl.origin[0]
                want = q / np.linalg.norm(d) * c.phi[0][z % N, y % N, x % N]
                assert abs(r.W[0][z % N, y % N, x % N] - want) <= 1e-3 * abs(want) + 1e-14
                checked += 1
    assert checked > 100
