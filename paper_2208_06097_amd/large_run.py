"""The 256-molecule cell (1024 orbitals, L = 37.3 bohr, 190^3 grid): V_xx action
from the zero, multipole, learned and spectral starts, same 1e-8 true residual.

Orbitals are assembled on the device (FP32, 28 GB), W is FP64 (56 GB), the
exx workspace is shared by the three forms.  Reports, per form, the V_xx
action time (HIP events per stage), CG iterations and E_xx, and the
iterations and time the learned start saves over the plain (zero) start.

    python -m paper_2208_06097_amd.large_run --out large.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import sea, synth

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "unet_f32cg.npy")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=5000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    cell = synth.config5(seed=args.seed, with_phi=False)
    phi = synth.fill_orbitals_device(cell, dtype=torch.float32)
    pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 6.0)
    torch.cuda.synchronize()
    log(f"inputs: {cell.n_occ} orbitals on {cell.N}^3, {len(pairs)} pairs, {time.perf_counter() - t0:.1f} s")
    W = torch.empty((cell.n_occ,) + (cell.N,) * 3, dtype=torch.float64, device="cuda")
    forms = {"zero-f32": sea.SEA_START_ZERO, "multipole-f32": sea.SEA_START_MULTIPOLE,
             "learned-f32": sea.SEA_START_LEARNED, "spectral-f32": sea.SEA_START_SPECTRAL}
    ws, variant, out = None, None, {}
    for name in ("spectral-f32", "learned-f32", "multipole-f32", "zero-f32"):   # largest workspace first
        ctx = sea.Context(rel_tol=args.tol, stencil_dtype=sea.SEA_F32, start=forms[name], profile=True)
        if name == "learned-f32":
            st = ctx.nn_state(np.load(args.weights))
            ctx.nn_attach(st)
        if ws is None:
            ws = ctx.workspace(ctx.exx_workspace_bytes(cell.N, cell.L, cell.n_occ, pairs))
            log(f"workspace {ws.numel() / 2**30:.1f} GiB")
        if variant is None:
            variant = ctx.autotune([(phi, cell.N, cell.L, pairs)], sample_pairs=2048, iters=20, ws=ws)["variant"]
        else:
            ctx.set_opts(cg_variant=ctx.cg_variants().index(variant))
        _, E, stats, status = ctx.exx_action(phi, cell.N, cell.L, pairs, ws=ws, W=W)
        ms = ctx.stage_times()
        vxx = sum(ms[k] for k in ("gather", "boundary", "guess", "cg", "finish", "scatter", "energy"))
        out[name] = {"E_xx": E, "vxx_ms": vxx, "cg_ms": ms["cg"], "guess_ms": ms["guess"],
                     "iters_mean": float(stats["iters"].mean()), "iters_max": int(stats["iters"].max()),
                     "max_rel_res": float(stats["rel_res"].max()), "all_converged": bool(np.all(stats["converged"] == 1)),
                     "status": int(status)}
        log(f"{name}: {vxx:.1f} ms (CG {ms['cg']:.1f}, guess {ms['guess']:.1f}), iters {out[name]['iters_mean']:.1f}, "
            f"E {E:.9f}")
        if name == "learned-f32":
            del st
        ctx.close()
    z, l = out["zero-f32"], out["learned-f32"]
    res = {"workload": "256-molecule water-like cell, L=37.3 bohr, 190^3 grid, 1024 orbitals, 63^3 pair domains, "
                       "FP32 CG state + FP64 reliable updates to a relative true residual",
           "seed": args.seed, "n_pairs": len(pairs), "rel_tol": args.tol, "cg_variant": variant, "forms": out,
           "learned_vs_zero": {"iters_saved_frac": 1 - l["iters_mean"] / z["iters_mean"],
                               "time_saved_frac": 1 - l["vxx_ms"] / z["vxx_ms"]},
           "spectral_vs_zero": {"time_saved_frac": 1 - out["spectral-f32"]["vxx_ms"] / z["vxx_ms"]},
           "max_dE_between_forms": float(max(v["E_xx"] for v in out.values()) - min(v["E_xx"] for v in out.values()))}
    line = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    main()
