"""Batched V_xx actions over many cells (the 200-cell batching workload).

Cells of the 0.4-1.7 g/cm^3 recipe (64 molecules, 256 orbitals, grid
spacing held near 0.196 bohr, grids of 100^3-163^3) are streamed through the
GPU in groups: each group's pairs of every cell run in one persistent CG
launch, the whole kernel sequence of a group is captured once into a HIP
graph (a plan) and replayed.  Orbitals are assembled on the device (same
seeded recipe as the host generator), FP32 CG state with FP64 reliable
updates, the CG kernel variant picked by the autotuner on the first group.

    python -m paper_2208_06097_amd.batch_run --cells 200 --group 4 --out batch.json

Reports pairs per second over the replayed plans (inputs resident, tables
uploaded, timed with HIP events around each graph launch), E_xx per cell and
CG iteration statistics.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import runlog, sea, synth


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=200)
    ap.add_argument("--first", type=int, default=0, help="index of the first cell of the recipe")
    ap.add_argument("--group", type=int, default=4, help="cells per plan (memory: about 25 GB per cell)")
    ap.add_argument("--start", default="multipole", choices=["zero", "multipole", "learned", "spectral"])
    ap.add_argument("--weights", default=None, help="network checkpoint for the learned start")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--replays", type=int, default=1, help="timed graph replays per group")
    ap.add_argument("--out", default=None)
    ap.add_argument("--metrics-jsonl", default=None, help="append per-group records here")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    start = {"zero": sea.SEA_START_ZERO, "multipole": sea.SEA_START_MULTIPOLE,
             "learned": sea.SEA_START_LEARNED, "spectral": sea.SEA_START_SPECTRAL}[args.start]
    ctx = sea.Context(rel_tol=args.tol, stencil_dtype=sea.SEA_F32, start=start)
    if start == sea.SEA_START_LEARNED:
        import os
        w = args.weights or os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_f32cg.npy")
        net = ctx.nn_state(np.load(w))
        ctx.nn_attach(net)
    ids = list(range(args.first, args.first + args.cells))
    dens = synth.config3_densities()
    per_cell, tuned = [], None
    total_pairs, total_ms, total_iters = 0, 0.0, 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for g0 in range(0, len(ids), args.group):
        grp = ids[g0:g0 + args.group]
        t0 = time.perf_counter()
        cells, tensors = [], []
        for k in grp:
            c = synth.config3_cell(k, with_phi=False)
            phi = synth.fill_orbitals_device(c, dtype=torch.float32)
            pairs = sea.build_pairs(c.N, c.L, c.centres, 6.0, 6.0)
            cells.append((phi, c.N, c.L, pairs))
            tensors.append((k, c, pairs))
        torch.cuda.synchronize()
        t_gen = time.perf_counter() - t0
        if tuned is None:
            tuned = ctx.autotune(cells[:1], sample_pairs=2048, iters=20)
            log(f"autotune: {tuned['variant']} " + " ".join(f"{k} {v:.1f}" for k, v in tuned["ms"].items()))
        plan = ctx.exx_plan(cells)
        ms = []
        for _ in range(args.replays):
            stream = torch.cuda.current_stream()
            ev0.record(stream)
            plan.launch(stream)
            ev1.record(stream)
            ev1.synchronize()
            ms.append(ev0.elapsed_time(ev1))
        E, stats, st = plan.results()
        n_pairs = len(stats)
        t_ms = float(np.median(ms))
        total_pairs += n_pairs
        total_ms += t_ms
        total_iters += int(stats["iters"].sum())
        off = 0
        for (k, c, pairs), e in zip(tensors, E):
            s = stats[off:off + len(pairs)]
            off += len(pairs)
            per_cell.append({"cell": k, "density": float(dens[k]), "N": c.N, "L": c.L, "pairs": len(pairs),
                             "E_xx": float(e), "iters_mean": float(s["iters"].mean()),
                             "converged": bool(np.all(s["converged"] == 1))})
        free_b, total_b = torch.cuda.mem_get_info()
        runlog.append(args.metrics_jsonl, "batch_group", group=g0 // args.group, cells=grp, pairs=n_pairs,
                      gpu_ms=t_ms, replay_ms=ms, iters_mean=float(stats["iters"].mean()), status=int(st),
                      input_s=t_gen, free_gib=free_b / 2**30)
        log(f"group {g0 // args.group}: cells {grp[0]}..{grp[-1]}, {n_pairs} pairs, {t_ms:.1f} ms "
            f"({n_pairs / t_ms * 1e3:.0f} pairs/s), iters {stats['iters'].mean():.1f}, status {st}, "
            f"inputs {t_gen:.1f} s, device memory free {free_b / 2**30:.0f} of {total_b / 2**30:.0f} GiB")
        plan.close()
        del plan, cells, tensors
        torch.cuda.empty_cache()
    out = {"workload": f"{len(ids)} cells of the 64-molecule 0.4-1.7 g/cm^3 batch recipe (cells {ids[0]}.."
                       f"{ids[-1]}), {args.group} cells per HIP-graph plan",
           "form": f"{args.start}-f32", "rel_tol": args.tol, "cg_variant": tuned["variant"] if tuned else None,
           "pairs": total_pairs, "gpu_ms": total_ms, "pair_solves_per_s": total_pairs / total_ms * 1e3,
           "cg_iters_mean": total_iters / max(total_pairs, 1),
           "all_converged": all(c["converged"] for c in per_cell), "cells": per_cell}
    line = json.dumps(out)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
