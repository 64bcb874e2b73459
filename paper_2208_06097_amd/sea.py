"""ctypes binding of ``libsea.so`` (the C ABI in ``include/sea.h``).

Argument marshalling only: every step of the exx action and the ACE build
runs in the library's HIP kernels.  PyTorch provides device memory and the
current stream.  The library must have been built (``build.build()``); a
missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsea.so")

SEA_OK, SEA_W_NOT_CONVERGED, SEA_W_EIGEN_FALLBACK = 0, 1, 2
SEA_E_ARG, SEA_E_HIP, SEA_E_NOMEM, SEA_E_NOT_PD, SEA_E_NONFINITE, SEA_E_RANK = -1, -2, -3, -4, -5, -6
SEA_F64, SEA_F32, SEA_BF16 = 0, 1, 2
SEA_START_ZERO, SEA_START_MULTIPOLE, SEA_START_LEARNED, SEA_START_SPECTRAL = 0, 1, 2, 3
SEA_DECOMP_CHOLESKY, SEA_DECOMP_EIGEN, SEA_DECOMP_AUTO = 0, 1, 2

# exported symbols declared in include/sea.h
EXPORTS = [
    "sea_version", "sea_opts_default", "sea_create", "sea_destroy", "sea_last_error",
    "sea_set_opts", "sea_build_pairs", "sea_exx_workspace_bytes", "sea_exx_action",
    "sea_exx_pair_solve", "sea_ace_workspace_bytes", "sea_ace_build", "sea_ace_apply",
    "sea_ace_energy", "sea_solid_harmonics_host", "sea_stage_times",
    "sea_nn_param_count", "sea_nn_state_bytes", "sea_nn_set_params", "sea_nn_get_params",
    "sea_nn_workspace_bytes", "sea_nn_forward", "sea_nn_train_step", "sea_nn_attach",
    "sea_exx_nn_samples", "sea_exx_batched_workspace_bytes", "sea_exx_action_batched",
    "sea_exx_plan_create", "sea_exx_plan_launch", "sea_exx_plan_results", "sea_exx_plan_destroy",
    "sea_cg_variant_count", "sea_cg_variant_name", "sea_exx_autotune",
    "sea_nn_infer_workspace_bytes", "sea_nn_infer", "sea_eps_workspace_bytes", "sea_build_pairs_eps",
    "sea_successive_idempotency", "sea_scdm_workspace_bytes", "sea_scdm", "sea_rotate",
    "sea_ace_apply_noalloc", "sea_spectral_variant_count", "sea_spectral_variant_name",
    "sea_set_spectral_variants", "sea_spectral_autotune", "sea_exx_plan_workspace_bytes",
    "sea_set_residual_history", "sea_scatter_variant_count", "sea_scatter_variant_name",
    "sea_set_scatter_variant", "sea_scatter_autotune",
]

# size of the library's static scratch array per GPU (SEA_NOALLOC_SCRATCH_BYTES
# in include/sea.h), which sea_ace_apply_noalloc works in
NOALLOC_SCRATCH_BYTES = 32 << 20

# the network's layers (name, c_in, c_out, relu), in parameter order
NN_LAYERS = [
    ("e0a", 1, 16, True), ("e0b", 16, 16, True), ("e1a", 16, 16, True), ("e1b", 16, 16, True),
    ("e2a", 16, 16, True), ("e2b", 16, 16, True), ("e3a", 16, 16, True), ("e3b", 16, 16, True),
    ("d2a", 32, 16, True), ("d2b", 16, 16, True), ("d1a", 32, 16, True), ("d1b", 16, 16, True),
    ("d0a", 32, 16, True), ("d0b", 16, 16, True), ("head", 16, 1, False),
]


def nn_pack(params: dict) -> np.ndarray:
    """Flatten {name.w: (O, C, 3, 3, 3), name.b: (O,)} into the library's order."""
    parts = []
    for name, _, _, _ in NN_LAYERS:
        parts.append(np.asarray(params[name + ".w"], dtype=np.float32).ravel())
        parts.append(np.asarray(params[name + ".b"], dtype=np.float32).ravel())
    return np.ascontiguousarray(np.concatenate(parts))


def nn_unpack(flat: np.ndarray) -> dict:
    out, off = {}, 0
    for name, ci, co, _ in NN_LAYERS:
        nw = co * ci * 27
        out[name + ".w"] = flat[off:off + nw].reshape(co, ci, 3, 3, 3)
        off += nw
        out[name + ".b"] = flat[off:off + co]
        off += co
    return out

PAIR_DTYPE = np.dtype([("i", "<i4"), ("j", "<i4"), ("lo", "<i4", 3), ("n", "<i4", 3),
                       ("origin", "<f8", 3)])
STAT_DTYPE = np.dtype([("iters", "<i4"), ("converged", "<i4"), ("rel_res", "<f8"),
                       ("e_ij", "<f8"), ("s_abs", "<f8"), ("q", "<f8")])


class SeaGrid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3)]


class SeaOpts(C.Structure):
    _fields_ = [("fd_half_order", C.c_int32), ("lmax", C.c_int32), ("rel_tol", C.c_double),
                ("max_iter", C.c_int32), ("stencil_dtype", C.c_int), ("ace_dtype", C.c_int),
                ("start", C.c_int), ("cg_variant", C.c_int32), ("profile", C.c_int32),
                ("nn_weight_dtype", C.c_int), ("hip_stream", C.c_void_p), ("ace_decomp", C.c_int),
                ("cg_xc_beta_min", C.c_double)]


class SeaCell(C.Structure):
    _fields_ = [("grid", SeaGrid), ("n_occ", C.c_int32), ("phi_dtype", C.c_int), ("phi_dev", C.c_void_p),
                ("n_pairs", C.c_int32), ("pairs_host", C.c_void_p), ("W_dev", C.c_void_p),
                ("exx_dev", C.c_void_p), ("dbox_host", C.c_void_p)]


STAGES = ["gather", "boundary", "guess", "cg", "scatter", "energy", "ace_m", "ace_chol", "ace_xi",
          "ace_apply", "finish", "scdm", "rotate", "dst", "dst_plane_fwd", "dst_zline", "dst_plane_inv",
          "residual", "face", "fold"]


class SeaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sea status {status}: {msg}")
        self.status = status


_lib = None


def load() -> C.CDLL:
    """Load libsea.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2208_06097_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P, vp, i, d, sz = C.POINTER, C.c_void_p, C.c_int, C.c_double, C.c_size_t
    lib.sea_version.restype = C.c_char_p
    lib.sea_opts_default.argtypes = [P(SeaOpts)]
    lib.sea_opts_default.restype = None
    lib.sea_create.argtypes = [P(SeaOpts), P(vp)]
    lib.sea_destroy.argtypes = [vp]
    lib.sea_last_error.argtypes = [vp]
    lib.sea_last_error.restype = C.c_char_p
    lib.sea_set_opts.argtypes = [vp, P(SeaOpts)]
    lib.sea_build_pairs.argtypes = [P(SeaGrid), i, vp, d, d, vp, i, P(i)]
    lib.sea_exx_workspace_bytes.argtypes = [vp, P(SeaGrid), i, i, vp, P(sz)]
    lib.sea_exx_action.argtypes = [vp, P(SeaGrid), i, vp, i, i, vp, vp, sz, vp, vp, vp, vp]
    lib.sea_exx_pair_solve.argtypes = [vp, P(SeaGrid), i, vp, i, i, vp, vp, sz, vp, vp, vp, vp]
    lib.sea_ace_workspace_bytes.argtypes = [vp, C.c_int64, i, i, P(sz)]
    lib.sea_ace_build.argtypes = [vp, C.c_int64, i, d, vp, vp, vp, sz, vp, vp, vp, P(i)]
    lib.sea_ace_apply.argtypes = [vp, C.c_int64, i, d, vp, i, vp, vp, sz, vp]
    lib.sea_ace_energy.argtypes = [vp, C.c_int64, i, d, vp, vp, vp, sz, P(d)]
    lib.sea_ace_apply_noalloc.argtypes = [vp, C.c_int64, i, d, vp, i, vp, vp]
    lib.sea_solid_harmonics_host.argtypes = [i, d, d, d, vp]
    lib.sea_stage_times.argtypes = [vp, vp]
    lib.sea_nn_param_count.restype = C.c_size_t
    lib.sea_nn_state_bytes.argtypes = [vp, P(sz)]
    lib.sea_nn_set_params.argtypes = [vp, vp, vp]
    lib.sea_nn_get_params.argtypes = [vp, vp, vp]
    lib.sea_nn_workspace_bytes.argtypes = [vp, i, i, P(sz)]
    lib.sea_nn_forward.argtypes = [vp, vp, i, i, vp, vp, vp, sz]
    lib.sea_nn_train_step.argtypes = [vp, vp, i, i, vp, vp, C.c_float, i, vp, sz, vp, vp]
    lib.sea_nn_attach.argtypes = [vp, vp]
    lib.sea_exx_nn_samples.argtypes = [vp, P(SeaGrid), i, vp, i, i, vp, vp, sz, i, vp, vp, vp, vp]
    lib.sea_exx_batched_workspace_bytes.argtypes = [vp, i, vp, P(sz)]
    lib.sea_exx_plan_workspace_bytes.argtypes = [vp, i, vp, P(sz)]
    lib.sea_exx_action_batched.argtypes = [vp, i, vp, vp, sz, vp, vp]
    lib.sea_exx_plan_create.argtypes = [vp, i, vp, vp, sz, P(vp)]
    lib.sea_exx_plan_launch.argtypes = [vp, vp]
    lib.sea_exx_plan_results.argtypes = [vp, vp, vp]
    lib.sea_exx_plan_destroy.argtypes = [vp]
    lib.sea_cg_variant_count.argtypes = []
    lib.sea_cg_variant_count.restype = i
    lib.sea_cg_variant_name.argtypes = [i]
    lib.sea_cg_variant_name.restype = C.c_char_p
    lib.sea_exx_autotune.argtypes = [vp, i, vp, vp, sz, i, i, vp, P(i)]
    lib.sea_spectral_variant_count.argtypes = []
    lib.sea_spectral_variant_count.restype = i
    lib.sea_spectral_variant_name.argtypes = [i]
    lib.sea_spectral_variant_name.restype = C.c_char_p
    lib.sea_set_spectral_variants.argtypes = [vp, i, i]
    lib.sea_set_residual_history.argtypes = [vp, vp, i]
    lib.sea_spectral_autotune.argtypes = [vp, i, vp, vp, sz, i, vp, P(i), P(i)]
    lib.sea_scatter_variant_count.argtypes = []
    lib.sea_scatter_variant_count.restype = i
    lib.sea_scatter_variant_name.argtypes = [i]
    lib.sea_scatter_variant_name.restype = C.c_char_p
    lib.sea_set_scatter_variant.argtypes = [vp, i]
    lib.sea_scatter_autotune.argtypes = [vp, i, vp, vp, sz, vp, P(i)]
    lib.sea_nn_infer_workspace_bytes.argtypes = [vp, i, P(sz)]
    lib.sea_nn_infer.argtypes = [vp, vp, i, vp, vp, vp, sz]
    lib.sea_eps_workspace_bytes.argtypes = [vp, P(SeaGrid), i, P(sz)]
    lib.sea_successive_idempotency.argtypes = [vp, C.c_int64, i, d, vp, vp, vp, sz, P(d)]
    lib.sea_build_pairs_eps.argtypes = [vp, P(SeaGrid), i, vp, i, d, d, i, vp, sz, vp, vp, vp, i, P(i)]
    lib.sea_scdm_workspace_bytes.argtypes = [vp, C.c_int64, i, P(sz)]
    lib.sea_scdm.argtypes = [vp, C.c_int64, i, vp, i, vp, sz, vp, vp, vp, vp, P(i)]
    lib.sea_rotate.argtypes = [vp, C.c_int64, i, i, vp, i, vp, vp]
    _lib = lib
    return lib


def version() -> str:
    return load().sea_version().decode()


def _grid(N, L) -> SeaGrid:
    g = SeaGrid()
    Ns = np.broadcast_to(np.asarray(N, dtype=np.int64), (3,))
    Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    for k in range(3):
        g.n[k] = int(Ns[k])
        g.L[k] = float(Ls[k])
    return g


def build_pairs(N, L, centres, r_pair=6.0, half_width=6.0) -> np.ndarray:
    """Host pair selection and domains (sea_build_pairs)."""
    lib = load()
    g = _grid(N, L)
    c = np.ascontiguousarray(centres, dtype=np.float64)
    n_occ = c.shape[0]
    cap = max(1, n_occ * (n_occ + 1) // 2)
    out = np.zeros(cap, dtype=PAIR_DTYPE)
    n = C.c_int(0)
    st = lib.sea_build_pairs(C.byref(g), n_occ, c.ctypes.data, r_pair, half_width,
                             out.ctypes.data, cap, C.byref(n))
    if st != SEA_OK:
        raise SeaError(st, "sea_build_pairs failed")
    return out[:n.value].copy()


def solid_harmonics_host(lmax, v) -> np.ndarray:
    out = np.zeros((lmax + 1) ** 2)
    st = load().sea_solid_harmonics_host(lmax, float(v[0]), float(v[1]), float(v[2]), out.ctypes.data)
    if st != SEA_OK:
        raise SeaError(st, "bad lmax")
    return out


def pair_stride(pairs: np.ndarray) -> int:
    n = int(np.max(np.prod(pairs["n"].astype(np.int64), axis=1))) if len(pairs) else 1
    return (n + 31) // 32 * 32


class Context:
    """A library context bound to the current torch CUDA device and stream."""

    def __init__(self, rel_tol=1e-8, max_iter=10000, lmax=6, stencil_dtype=SEA_F64,
                 ace_dtype=SEA_F64, start=SEA_START_ZERO, cg_variant=-1, profile=False,
                 nn_weight_dtype=SEA_BF16, stream=None, ace_decomp=SEA_DECOMP_CHOLESKY):
        import torch
        self._torch = torch
        self.lib = load()
        o = SeaOpts()
        self.lib.sea_opts_default(C.byref(o))
        o.rel_tol, o.max_iter, o.lmax = rel_tol, max_iter, lmax
        o.stencil_dtype, o.ace_dtype, o.start, o.cg_variant = stencil_dtype, ace_dtype, start, cg_variant
        o.profile = 1 if profile else 0
        o.nn_weight_dtype = nn_weight_dtype
        o.ace_decomp = ace_decomp
        if stream is None:
            stream = torch.cuda.current_stream()
        o.hip_stream = C.c_void_p(stream.cuda_stream)
        self.opts = o
        h = C.c_void_p()
        st = self.lib.sea_create(C.byref(o), C.byref(h))
        if st != SEA_OK:
            raise SeaError(st, "sea_create failed (no gfx950 device current, or bad options)")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.sea_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow_warn=True):
        if st == SEA_OK or (allow_warn and st > 0):
            return st
        raise SeaError(st, self.lib.sea_last_error(self.h).decode())

    def set_opts(self, **kw):
        for k, v in kw.items():
            setattr(self.opts, k, v)
        self._check(self.lib.sea_set_opts(self.h, C.byref(self.opts)))

    def stage_times(self) -> dict:
        """Per-stage milliseconds of the latest profiled calls (HIP events)."""
        ms = np.zeros(len(STAGES), dtype=np.float32)
        self._check(self.lib.sea_stage_times(self.h, ms.ctypes.data))
        return {k: float(v) for k, v in zip(STAGES, ms)}

    # ---------------------------------------------------------------- exx
    def exx_workspace_bytes(self, N, L, n_occ, pairs) -> int:
        g = _grid(N, L)
        b = C.c_size_t(0)
        p = np.ascontiguousarray(pairs, dtype=PAIR_DTYPE)
        self._check(self.lib.sea_exx_workspace_bytes(self.h, C.byref(g), n_occ, len(p),
                                                     p.ctypes.data if len(p) else None, C.byref(b)))
        return b.value

    def workspace(self, nbytes):
        return self._torch.empty(max(int(nbytes), 256), dtype=self._torch.uint8, device="cuda")

    @staticmethod
    def _phi_dtype(phi):
        import torch
        if phi.dtype == torch.float64:
            return SEA_F64
        if phi.dtype == torch.float32:
            return SEA_F32
        raise TypeError("phi must be float64 or float32")

    def exx_action(self, phi, N, L, pairs, ws=None, W=None, exx_dev=None, want_host=True, dbox=None):
        """Returns (W, E_host or None, stats or None, status).  ``dbox``
        (n_pairs x 12): the boxes where W takes each pair (see sea_cell)."""
        torch = self._torch
        if dbox is not None:
            Ws, Es, stats, st = self.exx_action_batched([(phi, N, L, pairs, W, exx_dev, dbox)], ws=ws,
                                                        want_host=want_host)
            return Ws[0], (float(Es[0]) if want_host else None), stats, st
        assert phi.is_cuda and phi.is_contiguous()
        n_occ = phi.shape[0]
        p = np.ascontiguousarray(pairs, dtype=PAIR_DTYPE)
        if ws is None:
            ws = self.workspace(self.exx_workspace_bytes(N, L, n_occ, p))
        if W is None:
            W = torch.empty(phi.shape, dtype=torch.float64, device=phi.device)
        g = _grid(N, L)
        E = C.c_double(0.0)
        stats = np.zeros(max(len(p), 1), dtype=STAT_DTYPE)
        st = self.lib.sea_exx_action(self.h, C.byref(g), n_occ, phi.data_ptr(), self._phi_dtype(phi), len(p),
                                     p.ctypes.data if len(p) else None, ws.data_ptr(), ws.numel(), W.data_ptr(),
                                     exx_dev.data_ptr() if exx_dev is not None else None,
                                     C.byref(E) if want_host else None,
                                     stats.ctypes.data if want_host else None)
        st = self._check(st)
        return W, (E.value if want_host else None), (stats[:len(p)] if want_host else None), st

    def _cells(self, cells, need_W=True):
        """Marshal [(phi, N, L, pairs, W or None, exx_dev or None, dbox or None), ...]
        into a sea_cell array; allocates W where it is None.  Keeps the pair
        tables alive in the returned tuple."""
        torch = self._torch
        arr = (SeaCell * len(cells))()
        keep, Ws = [], []
        for k, c in enumerate(cells):
            phi, N, L, pairs = c[0], c[1], c[2], c[3]
            W = c[4] if len(c) > 4 else None
            exx_dev = c[5] if len(c) > 5 else None
            dbox = c[6] if len(c) > 6 else None
            assert phi.is_cuda and phi.is_contiguous()
            p = np.ascontiguousarray(pairs, dtype=PAIR_DTYPE)
            keep.append(p)
            if W is None and need_W:
                W = torch.empty(phi.shape, dtype=torch.float64, device=phi.device)
            Ws.append(W)
            arr[k].grid = _grid(N, L)
            arr[k].n_occ = phi.shape[0]
            arr[k].phi_dtype = self._phi_dtype(phi)
            arr[k].phi_dev = phi.data_ptr()
            arr[k].n_pairs = len(p)
            arr[k].pairs_host = p.ctypes.data if len(p) else None
            arr[k].W_dev = W.data_ptr() if W is not None else None
            arr[k].exx_dev = exx_dev.data_ptr() if exx_dev is not None else None
            if dbox is not None:
                db = np.ascontiguousarray(dbox, dtype=np.int32).reshape(len(p), 12)
                keep.append(db)
                arr[k].dbox_host = db.ctypes.data if len(p) else None
        return arr, Ws, keep

    def exx_batched_workspace_bytes(self, cells) -> int:
        arr, _, keep = self._cells(cells, need_W=False)
        b = C.c_size_t(0)
        self._check(self.lib.sea_exx_batched_workspace_bytes(self.h, len(cells), arr, C.byref(b)))
        return b.value

    def exx_plan_workspace_bytes(self, cells) -> int:
        arr, _, keep = self._cells(cells, need_W=False)
        b = C.c_size_t(0)
        self._check(self.lib.sea_exx_plan_workspace_bytes(self.h, len(cells), arr, C.byref(b)))
        return b.value

    def exx_action_batched(self, cells, ws=None, want_host=True):
        """All pairs of all cells in one launch sequence.
        Returns (list of W, E per cell or None, stats of all pairs or None, status)."""
        arr, Ws, keep = self._cells(cells)
        if ws is None:
            ws = self.workspace(self.exx_batched_workspace_bytes(cells))
        n_all = sum(len(c[3]) for c in cells)
        E = np.zeros(len(cells))
        stats = np.zeros(max(n_all, 1), dtype=STAT_DTYPE)
        st = self.lib.sea_exx_action_batched(self.h, len(cells), arr, ws.data_ptr(), ws.numel(),
                                             E.ctypes.data if want_host else None,
                                             stats.ctypes.data if want_host else None)
        st = self._check(st)
        return Ws, (E if want_host else None), (stats[:n_all] if want_host else None), st

    def cg_variants(self) -> list:
        return [self.lib.sea_cg_variant_name(k).decode() for k in range(self.lib.sea_cg_variant_count())]

    def autotune(self, cells, sample_pairs=2048, iters=20, ws=None, cache=None):
        """Pick the FP32-state CG kernel variant for this workload.

        Times every variant on a strided sample of the cells' pairs (same
        work for each) and keeps the fastest for this context.  With
        ``cache`` (a JSON path), a stored choice for the same device, variant
        set and domain shapes is reused without timing, and new results are
        stored.  Returns {"variant": name, "ms": {name: ms} or None, "cached": bool}."""
        import json
        torch = self._torch
        names = self.cg_variants()
        shapes = sorted({tuple(int(v) for v in n) for c in cells for n in np.asarray(c[3]["n"]).reshape(-1, 3)})
        key = "|".join([torch.cuda.get_device_name(), ",".join(names), f"sample={sample_pairs}", f"iters={iters}",
                        ";".join("x".join(map(str, t)) for t in shapes[:8])])
        store = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                store = json.load(f)
            hit = store.get(key)
            if hit and hit.get("variant") in names:
                self.set_opts(cg_variant=names.index(hit["variant"]))
                return {"variant": hit["variant"], "ms": hit.get("ms"), "cached": True}
        arr, _, keep = self._cells(cells, need_W=False)
        if ws is None:
            ws = self.workspace(self.exx_batched_workspace_bytes(cells))
        ms = np.zeros(len(names), dtype=np.float32)
        best = C.c_int(-1)
        self._check(self.lib.sea_exx_autotune(self.h, len(cells), arr, ws.data_ptr(), ws.numel(), sample_pairs,
                                              iters, ms.ctypes.data, C.byref(best)))
        self.set_opts(cg_variant=-1)
        out = {"variant": names[best.value], "ms": {n: float(t) for n, t in zip(names, ms)}, "cached": False}
        if cache:
            store[key] = {"variant": out["variant"], "ms": out["ms"]}
            with open(cache, "w") as f:
                json.dump(store, f, indent=1)
        return out

    def spectral_variants(self):
        """(plane variant names, z-line variant names) of the sine-transform passes."""
        n = self.lib.sea_spectral_variant_count()
        names = [self.lib.sea_spectral_variant_name(v).decode() for v in range(n)]
        return [x for x in names if x.startswith("plane-")], [x for x in names if x.startswith("zline-")]

    def set_spectral_variants(self, plane=-1, zline=-1):
        """Fix the transform variants (index or name; -1: the tuned choice)."""
        pn, zn = self.spectral_variants()
        plane = pn.index(plane) if isinstance(plane, str) else plane
        zline = zn.index(zline) if isinstance(zline, str) else zline
        self._check(self.lib.sea_set_spectral_variants(self.h, int(plane), int(zline)))

    def scatter_variants(self):
        """Names of the scatter's schedules (workgroup orders)."""
        return [self.lib.sea_scatter_variant_name(v).decode() for v in range(self.lib.sea_scatter_variant_count())]

    def set_scatter_variant(self, variant=-1):
        """Fix the scatter schedule (index or name; -1: the tuned choice)."""
        names = self.scatter_variants()
        variant = names.index(variant) if isinstance(variant, str) else variant
        self._check(self.lib.sea_set_scatter_variant(self.h, int(variant)))

    def scatter_autotune(self, cells, ws=None):
        """Time one scatter of every schedule on these cells and keep the
        fastest.  The cells' W (allocated where None) are overwritten.
        Returns {"variant": name, "ms": {name: ms}}."""
        names = self.scatter_variants()
        arr, Ws, keep = self._cells(cells, need_W=True)
        if ws is None:
            ws = self.workspace(self.exx_batched_workspace_bytes(cells))
        ms = np.zeros(len(names), dtype=np.float32)
        best = C.c_int(-1)
        self._check(self.lib.sea_scatter_autotune(self.h, len(cells), arr, ws.data_ptr(), ws.numel(), ms.ctypes.data,
                                                  C.byref(best)))
        self.set_scatter_variant(-1)
        return {"variant": names[best.value], "ms": {n: float(t) for n, t in zip(names, ms)}}

    def residual_history(self, n_pairs, length):
        """Turns on per-pair residual histories for the next exx calls and
        returns their buffer: (n_pairs, length + 1) FP64 on the device,
        entry [k, t] the relative residual of pair k after t iterations
        (NaN after its last).  length < 0 turns them off (returns None)."""
        torch = self._torch
        if length < 0:
            self._check(self.lib.sea_set_residual_history(self.h, None, -1))
            self._hist = None
            return None
        self._hist = torch.empty((max(n_pairs, 1), length + 1), dtype=torch.float64, device="cuda")
        self._check(self.lib.sea_set_residual_history(self.h, self._hist.data_ptr(), int(length)))
        return self._hist

    def spectral_autotune(self, cells, sample_pairs=512, ws=None, cache=None):
        """Pick the sine-transform kernel variants of the spectral start for
        this workload (fastest plane pass and z-line pass on a strided
        sample of the pairs).  With ``cache`` (a JSON path) a stored choice
        for the same device, variant set and domain shapes is reused.
        Returns {"plane": name, "zline": name, "ms": {name: ms} or None, "cached": bool}."""
        import json
        torch = self._torch
        pn, zn = self.spectral_variants()
        shapes = sorted({tuple(int(v) for v in n) for c in cells for n in np.asarray(c[3]["n"]).reshape(-1, 3)})
        key = "|".join([torch.cuda.get_device_name(), ",".join(pn + zn), f"sample={sample_pairs}",
                        ";".join("x".join(map(str, t)) for t in shapes[:8])])
        store = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                store = json.load(f)
            hit = store.get(key)
            if hit and hit.get("plane") in pn and hit.get("zline") in zn:
                self.set_spectral_variants(hit["plane"], hit["zline"])
                return {"plane": hit["plane"], "zline": hit["zline"], "ms": hit.get("ms"), "cached": True}
        saved = self.opts.start
        arr, _, keep = self._cells(cells, need_W=False)
        if ws is None:
            self.set_opts(start=SEA_START_SPECTRAL)
            try:
                ws = self.workspace(self.exx_batched_workspace_bytes(cells))
            finally:
                self.set_opts(start=saved)
        ms = np.zeros(len(pn) + len(zn), dtype=np.float32)
        bp, bz = C.c_int(-1), C.c_int(-1)
        self._check(self.lib.sea_spectral_autotune(self.h, len(cells), arr, ws.data_ptr(), ws.numel(), sample_pairs,
                                                   ms.ctypes.data, C.byref(bp), C.byref(bz)))
        self.set_spectral_variants(-1, -1)
        out = {"plane": pn[bp.value], "zline": zn[bz.value],
               "ms": {n: float(t) for n, t in zip(pn + zn, ms)}, "cached": False}
        if cache:
            store[key] = {"plane": out["plane"], "zline": out["zline"], "ms": out["ms"]}
            with open(cache, "w") as f:
                json.dump(store, f, indent=1)
        return out

    def exx_plan(self, cells, ws=None):
        """A replayable HIP-graph plan of the batched action (see Plan)."""
        return Plan(self, cells, ws)

    def build_pairs_eps(self, phi, N, L, eps, delta, pad=0, with_dbox=False):
        """Pairs and boxes of the epsilon rule (Eq. 16-17), boxes grown by
        ``pad`` points a side: (pairs, S), or (pairs, S, dbox) with the boxes
        where W takes each pair (the paper's Omega^D)."""
        assert phi.is_cuda and phi.is_contiguous()
        n_occ = phi.shape[0]
        g = _grid(N, L)
        b = C.c_size_t(0)
        self._check(self.lib.sea_eps_workspace_bytes(self.h, C.byref(g), n_occ, C.byref(b)))
        ws = self.workspace(b.value)
        cap = n_occ * (n_occ + 1) // 2
        out = np.zeros(max(cap, 1), dtype=PAIR_DTYPE)
        S = np.zeros(max(cap, 1))
        db = np.zeros((max(cap, 1), 12), dtype=np.int32)
        n = C.c_int(0)
        self._check(self.lib.sea_build_pairs_eps(self.h, C.byref(g), n_occ, phi.data_ptr(), self._phi_dtype(phi),
                                                 eps, delta, int(pad), ws.data_ptr(), ws.numel(), out.ctypes.data,
                                                 S.ctypes.data, db.ctypes.data, cap, C.byref(n)))
        k = n.value
        return (out[:k].copy(), S[:k].copy(), db[:k].copy()) if with_dbox else (out[:k].copy(), S[:k].copy())

    def pair_solve(self, phi, N, L, pairs, ws=None, want_Q=True):
        """Per-pair potentials: returns (v (n_pairs x stride), Q or None, e, stats, status)."""
        torch = self._torch
        n_occ = phi.shape[0]
        p = np.ascontiguousarray(pairs, dtype=PAIR_DTYPE)
        if ws is None:
            ws = self.workspace(self.exx_workspace_bytes(N, L, n_occ, p))
        stride = pair_stride(p)
        v = torch.empty((max(len(p), 1), stride), dtype=torch.float64, device=phi.device)
        Q = torch.empty((max(len(p), 1), 49), dtype=torch.float64, device=phi.device) if want_Q else None
        e = torch.empty(max(len(p), 1), dtype=torch.float64, device=phi.device)
        g = _grid(N, L)
        stats = np.zeros(max(len(p), 1), dtype=STAT_DTYPE)
        st = self.lib.sea_exx_pair_solve(self.h, C.byref(g), n_occ, phi.data_ptr(), self._phi_dtype(phi), len(p),
                                         p.ctypes.data if len(p) else None, ws.data_ptr(), ws.numel(), v.data_ptr(),
                                         Q.data_ptr() if want_Q else None, e.data_ptr(), stats.ctypes.data)
        st = self._check(st)
        return v, Q, e, stats[:len(p)], st

    # ---------------------------------------------------------------- ACE
    def ace_workspace_bytes(self, n_grid, n_occ, n_vec=0) -> int:
        b = C.c_size_t(0)
        self._check(self.lib.sea_ace_workspace_bytes(self.h, int(n_grid), n_occ, n_vec, C.byref(b)))
        return b.value

    def _xi_torch_dtype(self):
        torch = self._torch
        return {SEA_F64: torch.float64, SEA_F32: torch.float32, SEA_BF16: torch.bfloat16}[self.opts.ace_dtype]

    def ace_build(self, phi, W, dV, ws=None):
        """Returns (M, L, xi, failed_pivot); raises SeaError on a non-PD M
        with the Cholesky decomposition.  self.last_status holds the status
        (SEA_W_EIGEN_FALLBACK when the AUTO decomposition fell back)."""
        torch = self._torch
        n_occ = phi.shape[0]
        ng = phi.numel() // n_occ
        if ws is None:
            ws = self.workspace(self.ace_workspace_bytes(ng, n_occ, n_occ))
        M = torch.empty((n_occ, n_occ), dtype=torch.float64, device=phi.device)
        Lm = torch.empty_like(M)
        xi = torch.empty(phi.shape, dtype=self._xi_torch_dtype(), device=phi.device)
        fp = C.c_int(0)
        st = self.lib.sea_ace_build(self.h, ng, n_occ, dV, phi.data_ptr(), W.data_ptr(), ws.data_ptr(), ws.numel(),
                                    M.data_ptr(), Lm.data_ptr(), xi.data_ptr(), C.byref(fp))
        self.last_status = self._check(st)
        return M, Lm, xi, fp.value

    def ace_apply(self, xi, psi, dV, ws=None):
        torch = self._torch
        n_occ = xi.shape[0]
        n_vec = psi.shape[0]
        ng = xi.numel() // n_occ
        if ws is None:
            ws = self.workspace(self.ace_workspace_bytes(ng, n_occ, n_vec))
        out_dtype = torch.float32 if self.opts.ace_dtype == SEA_BF16 else self._xi_torch_dtype()
        assert psi.dtype == self._xi_torch_dtype(), "psi must be in the context's ace_dtype"
        out = torch.empty(psi.shape, dtype=out_dtype, device=psi.device)
        st = self.lib.sea_ace_apply(self.h, ng, n_occ, dV, xi.data_ptr(), n_vec, psi.data_ptr(), ws.data_ptr(),
                                    ws.numel(), out.data_ptr())
        self._check(st)
        return out

    def ace_apply_noalloc(self, xi, psi, dV, out=None):
        """K psi through sea_ace_apply_noalloc: no workspace; the library
        works in its static scratch array (calls that overlap on one GPU race)."""
        torch = self._torch
        n_occ = xi.shape[0]
        n_vec = psi.shape[0]
        ng = xi.numel() // n_occ
        out_dtype = torch.float32 if self.opts.ace_dtype == SEA_BF16 else self._xi_torch_dtype()
        assert psi.dtype == self._xi_torch_dtype(), "psi must be in the context's ace_dtype"
        if out is None:
            out = torch.empty(psi.shape, dtype=out_dtype, device=psi.device)
        st = self.lib.sea_ace_apply_noalloc(self.h, ng, n_occ, dV, xi.data_ptr(), n_vec, psi.data_ptr(),
                                            out.data_ptr())
        self._check(st)
        return out

    @staticmethod
    def noalloc_scratch_bytes() -> int:
        return NOALLOC_SCRATCH_BYTES

    def ace_energy(self, phi, xi, dV, ws=None) -> float:
        n_occ = phi.shape[0]
        ng = phi.numel() // n_occ
        if ws is None:
            ws = self.workspace(self.ace_workspace_bytes(ng, n_occ, n_occ))
        E = C.c_double(0.0)
        st = self.lib.sea_ace_energy(self.h, ng, n_occ, dV, phi.data_ptr(), xi.data_ptr(), ws.data_ptr(),
                                     ws.numel(), C.byref(E))
        self._check(st)
        return E.value

    def successive_idempotency(self, phi_new, phi_old, dV, ws=None) -> float:
        """dI = 1 - sum_ij <phi_new_i, phi_old_j>^2 / n_occ (App. B)."""
        n_occ = phi_new.shape[0]
        ng = phi_new.numel() // n_occ
        if ws is None:
            ws = self.workspace(self.ace_workspace_bytes(ng, n_occ, 0))
        dI = C.c_double(0.0)
        self._check(self.lib.sea_successive_idempotency(self.h, ng, n_occ, dV, phi_new.data_ptr(),
                                                        phi_old.data_ptr(), ws.data_ptr(), ws.numel(),
                                                        C.byref(dI)))
        return dI.value

    # ---------------------------------------------------------------- SCDM
    def scdm_workspace_bytes(self, n_grid, n_occ) -> int:
        b = C.c_size_t(0)
        self._check(self.lib.sea_scdm_workspace_bytes(self.h, int(n_grid), int(n_occ), C.byref(b)))
        return b.value

    def scdm(self, phi, ws=None, want_loc=True):
        """SCDM of orbital-major phi (Eq. 1-6): dict with U (device FP64,
        U[j, k] = U_jk), phi_loc (device, phi's dtype; None without
        want_loc), piv and rdiag (host) and the number of pivot rounds."""
        torch = self._torch
        n_occ = phi.shape[0]
        ng = phi.numel() // n_occ
        if ws is None:
            ws = self.workspace(self.scdm_workspace_bytes(ng, n_occ))
        U = torch.empty((n_occ, n_occ), dtype=torch.float64, device="cuda")
        loc = torch.empty_like(phi) if want_loc else None
        piv = np.zeros(n_occ, dtype=np.int32)
        rdiag = np.zeros(n_occ)
        rounds = C.c_int(0)
        self._check(self.lib.sea_scdm(self.h, ng, n_occ, phi.data_ptr(), self._phi_dtype(phi), ws.data_ptr(),
                                      ws.numel(), U.data_ptr(), loc.data_ptr() if loc is not None else None,
                                      piv.ctypes.data, rdiag.ctypes.data, C.byref(rounds)))
        return {"U": U, "phi_loc": loc, "piv": piv, "rdiag": rdiag, "rounds": rounds.value}

    def rotate(self, X, U, inverse=False, out=None):
        """Y_k = sum_j X_j U_jk (Eq. 6) or, inverse, Y_i = sum_j X_j (U^-1)_ji (Eq. 15)."""
        n_occ = X.shape[0]
        ng = X.numel() // n_occ
        Y = self._torch.empty_like(X) if out is None else out
        self._check(self.lib.sea_rotate(self.h, ng, n_occ, self._phi_dtype(X), U.data_ptr(), int(bool(inverse)),
                                        X.data_ptr(), Y.data_ptr()))
        return Y

    # ---------------------------------------------------------------- network
    def nn_param_count(self) -> int:
        return int(self.lib.sea_nn_param_count())

    def nn_state(self, params_flat=None):
        """Device state (FP32 params, BF16 copy, Adam moments); optionally loaded."""
        b = C.c_size_t(0)
        self._check(self.lib.sea_nn_state_bytes(self.h, C.byref(b)))
        st = self._torch.zeros(b.value, dtype=self._torch.uint8, device="cuda")
        if params_flat is not None:
            self.nn_set_params(st, params_flat)
        return st

    def nn_set_params(self, state, params_flat):
        p = np.ascontiguousarray(params_flat, dtype=np.float32)
        assert p.size == self.nn_param_count()
        self._check(self.lib.sea_nn_set_params(self.h, state.data_ptr(), p.ctypes.data))

    def nn_get_params(self, state) -> np.ndarray:
        p = np.zeros(self.nn_param_count(), dtype=np.float32)
        self._check(self.lib.sea_nn_get_params(self.h, state.data_ptr(), p.ctypes.data))
        return p

    def nn_workspace(self, batch, D):
        b = C.c_size_t(0)
        self._check(self.lib.sea_nn_workspace_bytes(self.h, batch, D, C.byref(b)))
        return self.workspace(b.value)

    def nn_forward(self, state, x, ws=None):
        """x: (B, D, D, D) float32 cuda tensor -> y of the same shape."""
        B, D = x.shape[0], x.shape[-1]
        if ws is None:
            ws = self.nn_workspace(B, D)
        y = self._torch.empty_like(x)
        self._check(self.lib.sea_nn_forward(self.h, state.data_ptr(), B, D, x.data_ptr(), y.data_ptr(),
                                            ws.data_ptr(), ws.numel()))
        return y

    def nn_infer(self, state, x, ws=None):
        """Matrix-core inference (BF16 weights/activations, FP32 accumulation), 32^3 only."""
        torch = self._torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and tuple(x.shape[1:]) == (32, 32, 32)
        B = x.shape[0]
        if ws is None:
            b = C.c_size_t(0)
            self._check(self.lib.sea_nn_infer_workspace_bytes(self.h, B, C.byref(b)))
            ws = self.workspace(b.value)
        y = torch.empty_like(x)
        self._check(self.lib.sea_nn_infer(self.h, state.data_ptr(), B, x.data_ptr(), y.data_ptr(), ws.data_ptr(),
                                          ws.numel()))
        return y

    def nn_train_step(self, state, x, t, lr, step, ws=None, want_loss=True, grad=None):
        B, D = x.shape[0], x.shape[-1]
        if ws is None:
            ws = self.nn_workspace(B, D)
        loss = C.c_double(0.0)
        self._check(self.lib.sea_nn_train_step(self.h, state.data_ptr(), B, D, x.data_ptr(), t.data_ptr(),
                                               float(lr), int(step), ws.data_ptr(), ws.numel(),
                                               C.byref(loss) if want_loss else None,
                                               grad.data_ptr() if grad is not None else None))
        return loss.value if want_loss else None

    def nn_attach(self, state):
        self._nn_state_ref = state
        self._check(self.lib.sea_nn_attach(self.h, state.data_ptr() if state is not None else None))

    def exx_nn_samples(self, phi, N, L, pairs, D=32, ws=None):
        """Solve the pairs and return (x, t, s, stats): x = resample(rho/s), t = resample((v - v_ME)/s)."""
        torch = self._torch
        n_occ = phi.shape[0]
        p = np.ascontiguousarray(pairs, dtype=PAIR_DTYPE)
        if ws is None:
            ws = self.workspace(self.exx_workspace_bytes(N, L, n_occ, p))
        x = torch.empty((len(p), D, D, D), dtype=torch.float32, device=phi.device)
        t = torch.empty_like(x)
        s = torch.empty(len(p), dtype=torch.float64, device=phi.device)
        g = _grid(N, L)
        stats = np.zeros(max(len(p), 1), dtype=STAT_DTYPE)
        self._check(self.lib.sea_exx_nn_samples(self.h, C.byref(g), n_occ, phi.data_ptr(), self._phi_dtype(phi),
                                                len(p), p.ctypes.data, ws.data_ptr(), ws.numel(), D,
                                                x.data_ptr(), t.data_ptr(), s.data_ptr(), stats.ctypes.data))
        return x, t, s, stats[:len(p)]


class Plan:
    """Tables uploaded once, the batched action captured into a HIP graph.

    ``launch(stream)`` replays it (default: torch's current stream);
    ``results()`` waits and returns (E per cell, stats of all pairs, status).
    ``W`` holds the per-cell output tensors."""

    def __init__(self, ctx: Context, cells, ws=None):
        self.ctx = ctx
        arr, self.W, self._keep = ctx._cells(cells)
        self._cells = arr
        self._n_pairs = sum(len(c[3]) for c in cells)
        self.ws = ws if ws is not None else ctx.workspace(ctx.exx_plan_workspace_bytes(cells))
        h = C.c_void_p()
        ctx._check(ctx.lib.sea_exx_plan_create(ctx.h, len(cells), arr, self.ws.data_ptr(), self.ws.numel(),
                                               C.byref(h)))
        self.h = h
        self.n_cells = len(cells)

    def launch(self, stream=None):
        if stream is None:
            stream = self.ctx._torch.cuda.current_stream()
        self.ctx._check(self.ctx.lib.sea_exx_plan_launch(self.h, C.c_void_p(stream.cuda_stream)))

    def results(self):
        E = np.zeros(self.n_cells)
        stats = np.zeros(max(self._n_pairs, 1), dtype=STAT_DTYPE)
        st = self.ctx.lib.sea_exx_plan_results(self.h, E.ctypes.data, stats.ctypes.data)
        st = self.ctx._check(st)
        return E, stats[:self._n_pairs], st

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.sea_exx_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
