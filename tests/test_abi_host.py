"""Host-side checks of the C ABI (no GPU): exports, pair builder, harmonics."""
import ctypes
import re

import numpy as np
import pytest

import oracle
from paper_2208_06097_amd import sea, synth

HEADER = __import__("os").path.join(__import__("os").path.dirname(__file__), "..", "include", "sea.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sea_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(sea.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(sea.EXPORTS) | {"sea_version"}


def test_noalloc_scratch_size_matches_the_header():
    txt = open(HEADER).read()
    m = re.search(r"#define\s+SEA_NOALLOC_SCRATCH_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)", txt)
    assert m, "SEA_NOALLOC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == sea.NOALLOC_SCRATCH_BYTES


def test_stage_names_cover_the_stage_enum():
    txt = open(HEADER).read()
    count = int(re.search(r"SEA_STAGE_COUNT\s*=\s*(\d+)", txt).group(1))
    assert len(sea.STAGES) == count


def test_kernel_variant_names():
    """The schedule and kernel variants the autotuners choose among have
    distinct names, NULL past the end (host code only)."""
    lib = ctypes.CDLL(sea.LIB_PATH)
    for count, name in (("sea_scatter_variant_count", "sea_scatter_variant_name"),
                        ("sea_spectral_variant_count", "sea_spectral_variant_name"),
                        ("sea_cg_variant_count", "sea_cg_variant_name")):
        getattr(lib, count).restype = ctypes.c_int
        getattr(lib, name).restype = ctypes.c_char_p
        getattr(lib, name).argtypes = [ctypes.c_int]
        n = getattr(lib, count)()
        assert n >= 2, count
        names = [getattr(lib, name)(v) for v in range(n)]
        assert all(names) and len(set(names)) == n, names
        assert getattr(lib, name)(n) is None and getattr(lib, name)(-1) is None


def test_struct_layouts():
    assert sea.PAIR_DTYPE.itemsize == 56
    assert sea.STAT_DTYPE.itemsize == 40
    assert ctypes.sizeof(sea.SeaGrid) == 40
    assert ctypes.sizeof(sea.SeaCell) == 96


@pytest.mark.parametrize("cfg", ["c1", "mini", "c3_dense"])
def test_build_pairs_matches_oracle_bit_exact(cfg):
    if cfg == "c1":
        cell, hw = synth.config1(with_phi=False), 6.0
    elif cfg == "mini":
        cell, hw = synth.mini(with_phi=False), 4.0
    else:
        cell, hw = synth.config3_cell(int(np.argmax(synth.config3_densities())), with_phi=False), 6.0
    got = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, hw)
    want = oracle.build_pairs(cell.N, cell.L, cell.centres, 6.0, hw)
    assert len(got) == len(want)
    assert np.array_equal(np.stack([got["i"], got["j"]], 1), want.ij)
    assert np.array_equal(got["lo"], want.lo)
    assert np.array_equal(got["n"], want.n)
    assert np.array_equal(got["origin"], want.origin)


def test_build_pairs_capacity_error():
    cell = synth.mini(with_phi=False)
    lib = sea.load()
    g = sea._grid(cell.N, cell.L)
    out = np.zeros(3, dtype=sea.PAIR_DTYPE)
    n = ctypes.c_int(0)
    c = np.ascontiguousarray(cell.centres)
    st = lib.sea_build_pairs(ctypes.byref(g), cell.n_occ, c.ctypes.data, 6.0, 4.0, out.ctypes.data, 3, ctypes.byref(n))
    assert st == sea.SEA_E_NOMEM and n.value > 3


def test_solid_harmonics_recurrence_vs_legendre():
    rng = np.random.default_rng(0)
    for _ in range(50):
        v = rng.standard_normal(3) * rng.uniform(0.05, 8.0)
        r = np.linalg.norm(v)
        got = sea.solid_harmonics_host(6, v)
        Y = oracle.real_ylm(6, v)
        want = np.array([r ** l * Y[l * l + l + m] for l in range(7) for m in range(-l, l + 1)])
        assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))
