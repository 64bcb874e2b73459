"""Seeded synthetic "water-like" inputs: orbital centres and localized orbitals.

This module builds only the *inputs* of the exact-exchange path; it contains
none of the method's arithmetic (no pair selection, no Poisson solve, no ACE).
Both the FP64 oracle (``oracle/``) and the GPU library consume its output, and
it is the only code the two sides share.

Recipe (paper workload stand-in; the paper's (H2O)64 configurations, PBE0
orbitals and pseudopotentials are not available, so synthetic cells with the
same shapes stand in for them):

* ``n_mol`` "molecules": oxygen centres drawn by random sequential addition
  (uniform proposals in the periodic cube [0, L)^3, accepted when the
  minimum-image distance to every earlier centre is >= d_min, by default
  4.7 bohr scaled with the mean spacing L / n_mol^(1/3) relative to 64
  molecules in 23.5 bohr).
* 4 localized orbitals per molecule (a water molecule has 4 doubly occupied
  valence orbitals), centred at O + 1.0 bohr along a direction drawn uniformly
  on the sphere (a normalized standard-normal 3-vector), wrapped into [0, L).
* phi(r) = N (1 + a.d) exp(-|d|^2 / (2 sigma^2)), d = minimum-image(r - c),
  sigma = 0.8 bohr, a ~ N(0, 0.5^2 I) per orbital, N fixed by the grid sum
  h^3 sum phi^2 = 1.  Orbitals are not orthogonalized.
* Draw order from ``numpy.random.Generator(PCG64(seed))``: O centres (RSA),
  then 4 directions for every molecule, then ``a`` for every orbital.

Grid convention: point (ix, iy, iz) sits at h*(ix, iy, iz), h = L/N, x fastest;
``phi`` is orbital-major, shape (n_occ, N, N, N) indexed [i, iz, iy, ix].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SIGMA = 0.8          # orbital Gaussian width (bohr)
A_STD = 0.5          # std of each component of the linear coefficient a
BOND = 1.0           # orbital centre offset from O (bohr)
REF_L = 23.5         # 64-molecule cell side at 1.0 g/cm^3 (bohr)
REF_DMIN = 4.7       # minimum O-O separation at REF_L (bohr)
H_TARGET = 0.196     # grid spacing held fixed across densities (bohr)


@dataclasses.dataclass
class Cell:
    """One synthetic cell: grid, orbital centres and (optionally) orbitals."""
    L: float                  # cube side (bohr)
    N: int                    # grid points per axis
    o_centres: np.ndarray     # (n_mol, 3)
    centres: np.ndarray       # (n_occ, 3), wrapped into [0, L)
    a: np.ndarray             # (n_occ, 3) linear coefficients
    seed: int
    phi: np.ndarray | None = None   # (n_occ, N, N, N) float64, normalized

    @property
    def h(self) -> float:
        return self.L / self.N

    @property
    def n_occ(self) -> int:
        return self.centres.shape[0]


def _minimg(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def _rsa(rng: np.random.Generator, n: int, L: float, dmin: float,
         max_tries: int = 1_000_000) -> np.ndarray:
    pts = np.empty((n, 3))
    k = 0
    tries = 0
    while k < n:
        if tries >= max_tries:
            raise RuntimeError(
                f"random sequential addition failed: placed {k}/{n} centres in "
                f"L={L} with d_min={dmin} after {max_tries} proposals")
        tries += 1
        p = rng.uniform(0.0, L, size=3)
        if k:
            d = _minimg(pts[:k] - p, L)
            if np.min(np.einsum("ij,ij->i", d, d)) < dmin * dmin:
                continue
        pts[k] = p
        k += 1
    return pts


def make_centres(n_mol: int, L: float, N: int, seed: int,
                 dmin: float | None = None) -> Cell:
    """Draw O centres, orbital centres and a-vectors (no grid work)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if dmin is None:  # same packing fraction as 64 molecules in REF_L with REF_DMIN
        cb = n_mol ** (1.0 / 3.0)
        cb = float(round(cb)) if abs(cb - round(cb)) < 1e-9 else cb
        dmin = REF_DMIN * L / REF_L * (4.0 / cb)
    o = _rsa(rng, n_mol, L, dmin)
    dirs = rng.standard_normal((n_mol, 4, 3))
    dirs /= np.linalg.norm(dirs, axis=2, keepdims=True)
    c = (o[:, None, :] + BOND * dirs).reshape(-1, 3)
    c = np.mod(c, L)
    c[c >= L] -= L                     # guard the fp edge of mod
    a = A_STD * rng.standard_normal((4 * n_mol, 3))
    return Cell(L=float(L), N=int(N), o_centres=o, centres=c, a=a, seed=seed)


def _axis_factors(c: float, a: float, L: float, N: int):
    h = L / N
    x = h * np.arange(N)
    d = _minimg(x - c, L)
    g = np.exp(-d * d / (2.0 * SIGMA * SIGMA))
    return g, a * d * g


def fill_orbitals(cell: Cell, dtype=np.float64) -> Cell:
    """Evaluate and normalize every orbital on the full periodic grid."""
    N, L = cell.N, cell.L
    h3 = cell.h ** 3
    phi = np.empty((cell.n_occ, N, N, N), dtype=dtype)
    for i in range(cell.n_occ):
        gx, ax = _axis_factors(cell.centres[i, 0], cell.a[i, 0], L, N)
        gy, ay = _axis_factors(cell.centres[i, 1], cell.a[i, 1], L, N)
        gz, az = _axis_factors(cell.centres[i, 2], cell.a[i, 2], L, N)
        # (1 + a.d) g = gx gy gz + (ax dx gx) gy gz + gx (ay dy gy) gz + gx gy (az dz gz)
        f = (gz[:, None, None] * (gy[None, :, None] * (gx + ax)[None, None, :]
                                  + ay[None, :, None] * gx[None, None, :])
             + az[:, None, None] * (gy[None, :, None] * gx[None, None, :]))
        f *= 1.0 / math.sqrt(h3 * float(np.einsum("ijk,ijk->", f, f)))
        phi[i] = f
    cell.phi = phi
    return cell


def fill_orbitals_device(cell: Cell, device="cuda", dtype=None, chunk: int = 32):
    """Same orbitals as fill_orbitals, assembled on a torch device.

    The seeded draws and the per-axis factors are the same NumPy values; only
    the outer products and the normalization sums run on the device (FP64), so
    the result equals fill_orbitals up to the order of the normalization sum.
    Used for large cells whose host-side evaluation would dominate a run.
    Returns a contiguous (n_occ, N, N, N) tensor of ``dtype`` (default FP64)."""
    import torch
    dtype = dtype or torch.float64
    N, L = cell.N, cell.L
    h3 = cell.h ** 3
    out = torch.empty((cell.n_occ, N, N, N), dtype=dtype, device=device)
    for i0 in range(0, cell.n_occ, chunk):
        i1 = min(cell.n_occ, i0 + chunk)
        fac = [[_axis_factors(cell.centres[i, ax], cell.a[i, ax], L, N) for ax in range(3)] for i in range(i0, i1)]
        t = lambda ax, k: torch.from_numpy(np.stack([f[ax][k] for f in fac])).to(device)  # noqa: E731
        gx, ax_ = t(0, 0), t(0, 1)
        gy, ay = t(1, 0), t(1, 1)
        gz, az = t(2, 0), t(2, 1)
        f = (gz[:, :, None, None] * (gy[:, None, :, None] * (gx + ax_)[:, None, None, :]
                                     + ay[:, None, :, None] * gx[:, None, None, :])
             + az[:, :, None, None] * (gy[:, None, :, None] * gx[:, None, None, :]))
        norm = torch.sqrt(h3 * torch.sum(f * f, dim=(1, 2, 3)))
        out[i0:i1] = (f / norm[:, None, None, None]).to(dtype)
    return out


# ---- the five workload recipes -------------------------------------------

def config1(seed: int = 101, with_phi: bool = True) -> Cell:
    """8 molecules, L = 11.7 bohr, 60^3 grid (32 orbitals)."""
    cell = make_centres(8, 11.7, 60, seed, dmin=4.7)
    return fill_orbitals(cell) if with_phi else cell


def config2(seed: int = 2000, density: float = 1.0, with_phi: bool = True,
            dtype=np.float64) -> Cell:
    """64 molecules at ``density`` g/cm^3 (L = 23.5 bohr, 120^3 at 1.0)."""
    L = (1.0 / density) ** (1.0 / 3.0) * REF_L
    N = 120 if density == 1.0 else int(round(L / H_TARGET))
    cell = make_centres(64, L, N, seed)
    return fill_orbitals(cell, dtype) if with_phi else cell


def config3_densities(n_cells: int = 200, seed: int = 3999) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.4, 1.7, size=n_cells)


def config3_cell(k: int, with_phi: bool = True, dtype=np.float64) -> Cell:
    """Cell k of the 200-cell batch: density U(0.4, 1.7), h held near 0.196."""
    rho = float(config3_densities()[k])
    L = (1.0 / rho) ** (1.0 / 3.0) * REF_L
    N = int(round(L / H_TARGET))
    cell = make_centres(64, L, N, 3000 + k)
    return fill_orbitals(cell, dtype) if with_phi else cell


def config5(seed: int = 5000, with_phi: bool = True, dtype=np.float64) -> Cell:
    """256 molecules, L = 37.3 bohr, 190^3 grid (1024 orbitals)."""
    cell = make_centres(256, 37.3, 190, seed)
    return fill_orbitals(cell, dtype) if with_phi else cell


def mini(seed: int = 7, n_mol: int = 3, L: float = 9.0, N: int = 30,
         with_phi: bool = True) -> Cell:
    """Small cell for fast parity tests (coarse grid, few molecules)."""
    cell = make_centres(n_mol, L, N, seed, dmin=3.5)
    return fill_orbitals(cell) if with_phi else cell


def random_rotation(n: int, seed: int) -> np.ndarray:
    """Seeded dense orthogonal n x n matrix: the Cayley transform
    (I - S)^{-1} (I + S) of an antisymmetric S with standard-normal entries.
    Rotating localized orbitals by it gives delocalized orbitals that span
    the same space (the stand-in for canonical orbitals)."""
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((n, n))
    S = 0.5 * (R - R.T)
    eye = np.eye(n)
    return np.linalg.solve(eye - S, eye + S)


def rotate(phi: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Orbital-major rotation: out_k = sum_j phi_j G_jk."""
    A = phi.reshape(phi.shape[0], -1)
    return (G.T @ A).reshape(phi.shape).astype(phi.dtype)


def trial_vectors(cell: Cell, seed: int) -> np.ndarray:
    """Fresh orbitals of the same recipe (another seed) used as ACE trial vectors."""
    other = make_centres(cell.o_centres.shape[0], cell.L, cell.N, seed)
    return fill_orbitals(other).phi
