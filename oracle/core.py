"""ctypes front end of the C oracle plus the ACE algebra (TEST INFRASTRUCTURE).

Conventions (shared with the inputs, not with any GPU code):
  * grid point (ix, iy, iz) sits at h*(ix, iy, iz), x fastest;
  * orbital arrays are orbital-major, shape (n_occ, Nz, Ny, Nx);
  * <f, g> = h^3 sum f g (grid quadrature of the integral);
  * pairs are (i <= j) with a cube domain {lo[3], n[3]} and the multipole
    origin (Sec. II.B pair selection and domain truncation).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sea_oracle.c")
_LIB = os.path.join(_HERE, "build", "libsea_oracle.so")
_lib = None

FD_HALF_ORDER = 6   # O(h^12) Laplacian (App. C)
LMAX = 6            # multipole order (App. C)


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                        "-Wall", "-Wno-unused-variable", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.POINTER
        d, i32, i = C.c_double, C.c_int32, C.c_int
        lib.orc_fd_weights.argtypes = [i, P(d)]
        lib.orc_build_pairs.argtypes = [P(i32), P(d), i, P(d), d, d, i, P(i32), P(d), P(i)]
        lib.orc_real_ylm.argtypes = [i, d, d, d, P(d)]
        lib.orc_real_ylm.restype = None
        lib.orc_moments_points.argtypes = [i, i, P(d), P(d), P(d), P(d)]
        lib.orc_moments_points.restype = None
        lib.orc_me_eval.argtypes = [i, P(d), P(d), P(d)]
        lib.orc_me_eval.restype = d
        lib.orc_neg_lap_padded.argtypes = [P(i32), P(d), i, P(d), P(d)]
        lib.orc_cg.argtypes = [P(i32), P(d), i, P(d), P(d), d, i, P(d)]
        lib.orc_pair_potential.argtypes = [P(i32), P(d), i, P(d), P(i32), P(d), i, i, d, i,
                                           P(d), P(d), P(d), P(d)]
        lib.orc_pair_me_start.argtypes = [P(i32), P(d), i, P(d), P(i32), P(d), i, P(d)]
        lib.orc_exx.argtypes = [P(i32), P(d), i, P(d), i, P(i32), P(d), P(i32), i, i, d, i, i,
                                P(d), P(d), P(i32), P(d), P(d)]
        lib.orc_cholesky.argtypes = [i, P(d), P(d)]
        lib.orc_eps_boxes.argtypes = [P(i32), i, P(d), d, P(i32), P(i32)]
        lib.orc_eps_pairs.argtypes = [P(i32), P(d), i, P(d), P(i32), P(i32), d, i, i, P(i32), P(d), P(d),
                                      P(i32), P(i)]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _grid(N, L):
    N3 = np.ascontiguousarray(np.broadcast_to(np.asarray(N, dtype=np.int32), (3,)))
    L3 = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    return N3, L3


# ---------------------------------------------------------------------------

def fd_weights(M: int = FD_HALF_ORDER) -> np.ndarray:
    c = np.zeros(M + 1)
    if _load().orc_fd_weights(M, _dp(c)):
        raise ValueError("bad half order")
    return c


@dataclasses.dataclass
class PairList:
    ij: np.ndarray       # (n, 2) int32
    lo: np.ndarray       # (n, 3) int32
    n: np.ndarray        # (n, 3) int32
    origin: np.ndarray   # (n, 3) float64

    def __len__(self):
        return self.ij.shape[0]

    def packed(self) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate([self.ij, self.lo, self.n], axis=1).astype(np.int32))

    def subset(self, idx) -> "PairList":
        idx = np.asarray(idx)
        return PairList(self.ij[idx].copy(), self.lo[idx].copy(), self.n[idx].copy(),
                        self.origin[idx].copy())


def build_pairs(N, L, centres, r_pair=6.0, half_width=6.0) -> PairList:
    """Pair selection and pair domains (Sec. II.B; cube reading of the domain)."""
    lib = _load()
    N3, L3 = _grid(N, L)
    cen = np.ascontiguousarray(centres, dtype=np.float64)
    n_occ = cen.shape[0]
    cap = n_occ * (n_occ + 1) // 2
    out = np.zeros((max(cap, 1), 8), dtype=np.int32)
    org = np.zeros((max(cap, 1), 3))
    cnt = C.c_int(0)
    st = lib.orc_build_pairs(_ip(N3), _dp(L3), n_occ, _dp(cen), r_pair, half_width, cap,
                             _ip(out), _dp(org), C.byref(cnt))
    if st != 0:
        raise ValueError(f"orc_build_pairs failed ({st})")
    k = cnt.value
    return PairList(out[:k, 0:2].copy(), out[:k, 2:5].copy(), out[:k, 5:8].copy(), org[:k].copy())


def successive_idempotency(phi_new, phi_old, dV) -> float:
    """dI = 1 - Tr[P_new P_old] / Tr[P_new P_new] for the orbital projectors,
    = 1 - sum_ij <phi_new_i, phi_old_j>^2 / n_occ for orthonormal orbitals (App. B)."""
    A = phi_new.reshape(phi_new.shape[0], -1)
    B = phi_old.reshape(phi_old.shape[0], -1)
    S = dV * (A @ B.T)
    return 1.0 - float(np.sum(S * S)) / A.shape[0]


def eps_boxes(phi, N, eps):
    """Orbital boxes at 1 - eps coverage (Eq. 16): (lo, len), each (n_occ, 3)."""
    lib = _load()
    N3, _ = _grid(N, 1.0)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    n_occ = phi.shape[0]
    lo = np.zeros((n_occ, 3), dtype=np.int32)
    ln = np.zeros((n_occ, 3), dtype=np.int32)
    st = lib.orc_eps_boxes(_ip(N3), n_occ, _dp(phi), eps, _ip(lo), _ip(ln))
    if st != 0:
        raise ValueError(f"orc_eps_boxes failed ({st})")
    return lo, ln


def eps_pairs(phi, N, L, lo, ln, delta, pad=0, with_dbox=False):
    """Pair boxes Omega_ii ∩ Omega_jj screened by S_ij >= delta (Eq. 17),
    written out grown by ``pad`` points a side: (PairList, S) or, with
    ``with_dbox``, (PairList, S, dbox) with the boxes where W takes each pair."""
    lib = _load()
    N3, L3 = _grid(N, L)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    n_occ = phi.shape[0]
    cap = n_occ * (n_occ + 1) // 2
    out = np.zeros((max(cap, 1), 8), dtype=np.int32)
    org = np.zeros((max(cap, 1), 3))
    S = np.zeros(max(cap, 1))
    db = np.zeros((max(cap, 1), 12), dtype=np.int32)
    cnt = C.c_int(0)
    st = lib.orc_eps_pairs(_ip(N3), _dp(L3), n_occ, _dp(phi), _ip(np.ascontiguousarray(lo, dtype=np.int32)),
                           _ip(np.ascontiguousarray(ln, dtype=np.int32)), delta, int(pad), cap, _ip(out), _dp(org),
                           _dp(S), _ip(db), C.byref(cnt))
    if st != 0:
        raise ValueError(f"orc_eps_pairs failed ({st})")
    k = cnt.value
    pl = PairList(out[:k, 0:2].copy(), out[:k, 2:5].copy(), out[:k, 5:8].copy(), org[:k].copy())
    return (pl, S[:k].copy(), db[:k].copy()) if with_dbox else (pl, S[:k].copy())


def real_ylm(lmax: int, v) -> np.ndarray:
    out = np.zeros((lmax + 1) ** 2)
    _load().orc_real_ylm(lmax, float(v[0]), float(v[1]), float(v[2]), _dp(out))
    return out


def moments_points(lmax, pos, q, origin) -> np.ndarray:
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    Q = np.zeros((lmax + 1) ** 2)
    _load().orc_moments_points(lmax, pos.shape[0], _dp(pos), _dp(q), _dp(o), _dp(Q))
    return Q


def me_eval(lmax, Q, origin, target) -> float:
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    t = np.ascontiguousarray(target, dtype=np.float64)
    return _load().orc_me_eval(lmax, _dp(Q), _dp(o), _dp(t))


def neg_lap_padded(f_padded: np.ndarray, h, M: int = FD_HALF_ORDER) -> np.ndarray:
    """-Lap_h on the interior of a padded (nz+2M, ny+2M, nx+2M) array."""
    f = np.ascontiguousarray(f_padded, dtype=np.float64)
    n = np.array([f.shape[2] - 2 * M, f.shape[1] - 2 * M, f.shape[0] - 2 * M], dtype=np.int32)
    h3 = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (3,)))
    out = np.zeros((n[2], n[1], n[0]))
    if _load().orc_neg_lap_padded(_ip(n), _dp(h3), M, _dp(f), _dp(out)):
        raise ValueError("bad half order")
    return out


def cg(b: np.ndarray, h, M: int = FD_HALF_ORDER, tol=1e-12, max_iter=10000, x0=None):
    """Plain CG on -Lap_h x = b with zero values outside the interior (Eq. 9)."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = np.array([b.shape[2], b.shape[1], b.shape[0]], dtype=np.int32)
    h3 = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (3,)))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    info = np.zeros(2)
    st = _load().orc_cg(_ip(n), _dp(h3), M, _dp(b), _dp(x), tol, max_iter, _dp(info))
    return x, int(info[0]), float(info[1]), st


def pair_potential(phi, N, L, pairs: PairList, k: int, tol=1e-12, max_iter=10000,
                   M=FD_HALF_ORDER, lmax=LMAX, x0=None):
    """Potential of pair k on its interior, plus (Q_lm, info dict)."""
    lib = _load()
    N3, L3 = _grid(N, L)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    pk = np.ascontiguousarray(pairs.packed()[k])
    org = np.ascontiguousarray(pairs.origin[k])
    n = pairs.n[k]
    v = np.zeros((n[2], n[1], n[0]))
    Q = np.zeros((lmax + 1) ** 2)
    info = np.zeros(8)
    x0p = None
    if x0 is not None:
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        x0p = _dp(x0)
    st = lib.orc_pair_potential(_ip(N3), _dp(L3), phi.shape[0], _dp(phi), _ip(pk), _dp(org), M,
                                lmax, tol, max_iter, x0p, _dp(v), _dp(Q), _dp(info))
    if st < 0:
        raise ValueError("bad pair")
    return v, Q, dict(iters=int(info[0]), rel_res=info[1], e=info[2], s_abs=info[3],
                      q=info[4], bnorm=info[5], status=int(info[6]))


def pair_me_start(phi, N, L, pairs: PairList, k: int, lmax=LMAX) -> np.ndarray:
    """Regularized multipole start v_ME of pair k on its interior (nz, ny, nx):
    q erf(r/r_s)/r plus the l >= 1 terms of Eq. 10 damped by
    (1 - exp(-r^2/r_s^2))^(l+1), r_s = sqrt(2<r^2>/3) from the |rho|-weighted
    second moment about the domain origin.  The paper leaves the CG's initial
    guess open; this is the reading the multipole and learned starts use."""
    lib = _load()
    N3, L3 = _grid(N, L)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    pk = np.ascontiguousarray(pairs.packed()[k])
    org = np.ascontiguousarray(pairs.origin[k])
    n = pairs.n[k]
    out = np.zeros((n[2], n[1], n[0]))
    if lib.orc_pair_me_start(_ip(N3), _dp(L3), phi.shape[0], _dp(phi), _ip(pk), _dp(org), lmax, _dp(out)):
        raise ValueError("bad pair")
    return out


@dataclasses.dataclass
class ExxResult:
    E: float
    W: np.ndarray
    e_pairs: np.ndarray
    iters: np.ndarray
    rel_res: np.ndarray
    n_unconverged: int


def exx(phi, N, L, pairs: PairList, tol=1e-12, max_iter=10000, M=FD_HALF_ORDER, lmax=LMAX,
        n_threads=0, dbox=None) -> ExxResult:
    """The whole V_xx action: W = D_xx (Eq. 13-14), E (Eq. 8).  W is taken on
    the pair domains, or with ``dbox`` ((n_pairs, 12) int32: for W_i the box
    lo[3], n[3], then for W_j) on those boxes with the multipole potential
    outside the pair domain."""
    lib = _load()
    N3, L3 = _grid(N, L)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    n_occ = phi.shape[0]
    npairs = len(pairs)
    packed = pairs.packed() if npairs else np.zeros((1, 8), np.int32)
    org = np.ascontiguousarray(pairs.origin) if npairs else np.zeros((1, 3))
    W = np.zeros_like(phi)
    e = np.zeros(max(npairs, 1))
    it = np.zeros(max(npairs, 1), dtype=np.int32)
    rr = np.zeros(max(npairs, 1))
    E = C.c_double(0.0)
    db = None
    if dbox is not None and npairs:
        db = np.ascontiguousarray(dbox, dtype=np.int32).reshape(npairs, 12)
    st = lib.orc_exx(_ip(N3), _dp(L3), n_occ, _dp(phi), npairs, _ip(packed), _dp(org),
                     _ip(db) if db is not None else None, M, lmax,
                     tol, max_iter, n_threads, _dp(W), _dp(e), _ip(it), _dp(rr), C.byref(E))
    if st < 0:
        raise ValueError("bad pair list")
    return ExxResult(E.value, W, e[:npairs], it[:npairs], rr[:npairs], st)


def cholesky(A: np.ndarray):
    """Lower Cholesky factor (own unblocked loops); returns (L, failed_pivot)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    Lo = np.zeros_like(A)
    st = _load().orc_cholesky(n, _dp(A), _dp(Lo))
    return Lo, int(st)


# --------------------------- ACE (Eq. 18-19) -------------------------------

@dataclasses.dataclass
class AceResult:
    M: np.ndarray      # h^3 Phi^T W (unsymmetrized)
    Mbar: np.ndarray   # (M + M^T)/2
    L: np.ndarray      # lower Cholesky factor of Mbar
    xi: np.ndarray     # orbital-major (n_occ, Ng): xi = W L^{-T}
    failed_pivot: int


def ace_build(phi, W, dV, decomp="cholesky") -> AceResult:
    """M = <phi_i, W_j>, symmetrize (App. A), Cholesky, xi = W L^{-T} (Eq. 18).

    decomp="eigen" (App. A): Mbar = Q Lambda Q^T (numpy's symmetric
    eigensolver), zeta = W Q Lambda^{-1/2} with the imaginary factor of a
    negative eigenvalue cancelling against its conjugate in |zeta><zeta|, i.e.
    xi = W Q |Lambda|^{-1/2} and K = -xi xi^T; null eigenvalues (<= 1e-14 of
    the largest) are dropped.  The L field then holds Q |Lambda|^{-1/2}."""
    import scipy.linalg as sla
    P = phi.reshape(phi.shape[0], -1)
    Wm = W.reshape(W.shape[0], -1)
    M = dV * (P @ Wm.T)
    Mbar = 0.5 * (M + M.T)
    if decomp == "eigen":
        lam, Q = np.linalg.eigh(Mbar)
        a = np.abs(lam)
        keep = a > 1e-14 * a.max()
        Zit = np.where(keep[None, :], Q / np.sqrt(np.where(keep, a, 1.0))[None, :], 0.0)
        # xi (orbital-major): xi_k = sum_i W_i (Q |Lambda|^{-1/2})_ik
        return AceResult(M, Mbar, Zit, Zit.T @ Wm, 0)
    Lo, fail = cholesky(Mbar)
    if fail:
        return AceResult(M, Mbar, Lo, np.zeros_like(Wm), fail)
    # xi (grid-major) = W L^{-T}  <=>  xi^T = L^{-1} W^T (orbital-major)
    xi = sla.solve_triangular(Lo, Wm, lower=True, check_finite=False)
    return AceResult(M, Mbar, Lo, xi, 0)


def ace_apply(xi, psi, dV) -> np.ndarray:
    """K psi = -xi (h^3 xi^T psi), orbital-major in and out (Eq. 18)."""
    X = xi.reshape(xi.shape[0], -1)
    Pm = psi.reshape(psi.shape[0], -1)
    Cm = dV * (X @ Pm.T)            # (n_occ, n_vec)
    return -(Cm.T @ X).reshape(psi.shape)


def ace_energy(phi, xi, dV) -> float:
    """E = -sum_ik <phi_i, xi_k>^2 (Eq. 19)."""
    P = phi.reshape(phi.shape[0], -1)
    X = xi.reshape(xi.shape[0], -1)
    S = dV * (P @ X.T)
    return -float(np.sum(S * S))


@dataclasses.dataclass
class ScdmResult:
    piv: np.ndarray      # (n_occ,) selected grid columns C, in pivot order
    rdiag: np.ndarray    # (n_occ,) |R_kk|: norm of the pivot column after the earlier ones are removed
    U: np.ndarray        # (n_occ, n_occ) Eq. 5
    phi_loc: np.ndarray  # orbital-major, Eq. 6: phi_loc_k = sum_j phi_j U_jk


def scdm_pivots(phi):
    """Column-pivoted QR of Phi^T (Eq. 1), pivots only.

    Phi^T is n_occ x N_grid (row i = orbital i, column g = grid point g).  At
    step k the pivot is the column whose part orthogonal to the k columns
    already chosen is longest (first index on ties); that part, normalized,
    becomes the k-th column of Q, and its length is |R_kk|.  Written with an
    explicit residual matrix: every remaining column loses its component
    along the new Q column, and the norms are summed afresh each step."""
    A = np.asarray(phi, dtype=np.float64).reshape(phi.shape[0], -1)
    n, ng = A.shape
    if ng < n:
        raise ValueError("fewer grid points than orbitals")
    res = A.copy()
    chosen = np.zeros(ng, dtype=bool)
    piv = np.zeros(n, dtype=np.int64)
    rdiag = np.zeros(n)
    for k in range(n):
        norms = np.einsum("ij,ij->j", res, res)
        norms[chosen] = -1.0
        c = int(np.argmax(norms))
        r = float(np.sqrt(norms[c]))
        if not r > 0.0:
            raise ValueError(f"Phi^T has rank {k} < n_occ")
        q = res[:, c] / r
        res -= np.outer(q, q @ res)
        chosen[c] = True
        piv[k], rdiag[k] = c, r
    return piv, rdiag


def scdm(phi) -> ScdmResult:
    """SCDM localization (Eq. 1-6).

    B = (Phi^T)_{:,C} holds the orbitals at the selected points; the proto
    orbitals X = Phi B (Eq. 2) are orthogonalized with P_CC^{-1/2} (Eq. 3),
    where P_CC is the density matrix at the selected points, B^T B (equal to
    X^T X for orbitals orthonormal as grid vectors); then U = B P_CC^{-1/2}
    (Eq. 5) is orthogonal for any Phi of full rank, and phi_loc = Phi U
    (Eq. 6).  The inverse square root uses numpy's symmetric eigensolver."""
    A = np.asarray(phi, dtype=np.float64).reshape(phi.shape[0], -1)
    piv, rdiag = scdm_pivots(A)
    B = A[:, piv]
    lam, V = np.linalg.eigh(B.T @ B)
    P_mhalf = (V / np.sqrt(lam)[None, :]) @ V.T
    U = B @ P_mhalf
    phi_loc = (U.T @ A).reshape(phi.shape)
    return ScdmResult(piv, rdiag, U, phi_loc)


def back_rotate(D_loc, U):
    """D^i = sum_j D_loc^j (U^{-1})_ji (Eq. 15), orbital-major in and out;
    U^{-1} by numpy's general inverse."""
    Dm = np.asarray(D_loc, dtype=np.float64).reshape(D_loc.shape[0], -1)
    return (np.linalg.inv(U).T @ Dm).reshape(D_loc.shape)


def qrcp_residual_norms(phi, prefix):
    """Squared norms of every column of Phi^T after removing its components
    along the columns ``prefix`` (brute force: orthonormal basis of the
    prefix columns by numpy's QR, then a projection)."""
    A = np.asarray(phi, dtype=np.float64).reshape(phi.shape[0], -1)
    if len(prefix) == 0:
        return np.einsum("ij,ij->j", A, A)
    Qp, _ = np.linalg.qr(A[:, np.asarray(prefix)])
    R = A - Qp @ (Qp.T @ A)
    return np.einsum("ij,ij->j", R, R)
