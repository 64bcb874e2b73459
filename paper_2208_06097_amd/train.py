"""Train the learned CG warm start on pair solves the method itself generates.

Samples: for every pair of the training cells, x = resample(rho/s) and
t = resample((v - v_ME)/s) on 32^3 from converged solves (sea_exx_nn_samples,
FP32 CG state with FP64 reliable updates, relative residual 1e-8).  Training
cells: 64-molecule cells of the 200-cell batch recipe (densities 0.4-1.7
g/cm^3) and the 1.66 / 0.99 / 0.42 g/cm^3 64-molecule variants; the 1.0 g/cm^3
cell of seed 2000 (the benchmark workload) is held out.  Samples are drawn
without replacement (seed 4242) and split 90/10 into training and validation.
Adam with a cosine learning-rate decay; the network, its backward pass and
the optimizer all run in the library's kernels.

    python -m paper_2208_06097_amd.train --out weights.npy [--cells 12] [--epochs 8]
        [--checkpoint ckpt.npz --stop-after K]   (resumable: run again to continue)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import runlog, sea, synth


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def he_init(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, flattened in the library's order."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, _ in sea.NN_LAYERS:
        p[name + ".w"] = rng.standard_normal((co, ci, 3, 3, 3)) * math.sqrt(2.0 / (ci * 27))
        p[name + ".b"] = np.zeros(co)
    return sea.nn_pack(p)


def training_cells(n_batch_cells: int):
    """(label, cell) for the training set; excludes the benchmark cell."""
    out = []
    for seed, dens in ((2166, 1.66), (2099, 0.99), (2042, 0.42)):
        out.append((f"c2 d={dens} seed={seed}", lambda s=seed, d=dens: synth.config2(seed=s, density=d,
                                                                                       dtype=np.float32)))
    for k in range(n_batch_cells):
        out.append((f"c3 cell {k}", lambda k=k: synth.config3_cell(k, dtype=np.float32)))
    return out


def make_samples(ctx, cells, D=32, max_samples=None):
    import torch
    xs, ts = [], []
    total = 0
    for label, mk in cells:
        t0 = time.perf_counter()
        cell = mk()
        pairs = sea.build_pairs(cell.N, cell.L, cell.centres, 6.0, 6.0)
        phi = torch.from_numpy(cell.phi).cuda()
        x, t, s, stats = ctx.exx_nn_samples(phi, cell.N, cell.L, pairs, D=D)
        del phi
        xs.append(x)
        ts.append(t)
        total += len(pairs)
        log(f"samples: {label}: {len(pairs)} pairs, iters mean {stats['iters'].mean():.1f}, "
            f"{time.perf_counter() - t0:.1f} s (total {total})")
        if max_samples and total >= max_samples:
            break
    return torch.cat(xs), torch.cat(ts)


def save_checkpoint(path, state, step, epoch, gen, hist):
    """Whole device state (FP32 parameters, BF16 copy, Adam m and v), the step
    and epoch reached, the shuffling generator's state and the history."""
    tmp = path + ".tmp.npz"
    np.savez(tmp, state=state.cpu().numpy(), step=np.int64(step), epoch=np.int64(epoch),
             gen=gen.get_state().numpy(), hist=np.frombuffer(json.dumps(hist).encode(), dtype=np.uint8))
    os.replace(tmp, path)


def load_checkpoint(path):
    import torch
    z = np.load(path, allow_pickle=False)
    return (torch.from_numpy(z["state"]).cuda(), int(z["step"]), int(z["epoch"]), torch.from_numpy(z["gen"]),
            json.loads(bytes(z["hist"]).decode()))


def train(ctx, x, t, epochs=8, batch=32, lr=2e-3, seed=4242, init_seed=0, max_samples=None, state=None,
          checkpoint=None, stop_after=None, metrics=None):
    """Adam with cosine decay over `epochs`.  With `checkpoint` (a .npz path)
    the state is saved after every epoch and, when the file exists, training
    resumes from it (same samples, same shuffles, same schedule); with
    `stop_after` it stops after that many epochs of this call."""
    import torch
    n = x.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(n, generator=g)
    if max_samples:
        perm = perm[:max_samples]
    n = perm.numel()
    nval = max(1, n // 10)
    val_idx, tr_idx = perm[:nval].cuda(), perm[nval:].cuda()
    xv, tv = x[val_idx].contiguous(), t[val_idx].contiguous()
    if state is None:
        state = ctx.nn_state(he_init(init_seed))
    ws = ctx.nn_workspace(batch, x.shape[-1])
    wsv = ctx.nn_workspace(min(batch, nval), x.shape[-1])
    steps_per_epoch = (tr_idx.numel()) // batch
    total_steps = max(1, steps_per_epoch * epochs)

    def val_loss():
        tot, cnt = 0.0, 0
        for b0 in range(0, nval - min(batch, nval) + 1, min(batch, nval)):
            yb = ctx.nn_forward(state, xv[b0:b0 + min(batch, nval)], ws=wsv)
            tot += float(torch.mean((yb - tv[b0:b0 + min(batch, nval)]) ** 2)) * yb.shape[0]
            cnt += yb.shape[0]
        return tot / max(cnt, 1)

    tv2 = float(torch.mean(tv ** 2))
    step, ep0 = 0, 0
    if checkpoint and os.path.exists(checkpoint):
        state, step, ep0, gstate, hist = load_checkpoint(checkpoint)
        g.set_state(gstate)
        log(f"resumed from {checkpoint}: epoch {ep0}, step {step}")
    else:
        hist = [{"epoch": 0, "val": val_loss(), "val_rel": None}]
        hist[0]["val_rel"] = hist[0]["val"] / tv2
        log(f"epoch 0: val {hist[0]['val']:.4e} (rel {hist[0]['val_rel']:.3f})")
    done = 0
    for ep in range(ep0 + 1, epochs + 1):
        if stop_after is not None and done >= stop_after:
            break
        t0 = time.perf_counter()
        order = tr_idx[torch.randperm(tr_idx.numel(), generator=g).cuda()]
        tl = []
        for b in range(steps_per_epoch):
            idx = order[b * batch:(b + 1) * batch]
            step += 1
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * (step - 1) / total_steps))
            L = ctx.nn_train_step(state, x[idx].contiguous(), t[idx].contiguous(), max(lr_t, 1e-6), step, ws=ws,
                                  want_loss=(b % 50 == 0))
            if L is not None:
                tl.append(L)
        v = val_loss()
        hist.append({"epoch": ep, "train": float(np.mean(tl)) if tl else None, "val": v, "val_rel": v / tv2,
                     "seconds": time.perf_counter() - t0})
        log(f"epoch {ep}: train {hist[-1]['train']:.4e} val {v:.4e} (rel {v / tv2:.3f}) "
            f"{hist[-1]['seconds']:.1f} s")
        runlog.append(metrics, "train_epoch", **hist[-1])
        done += 1
        if checkpoint:
            save_checkpoint(checkpoint, state, step, ep, g, hist)
    return state, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--cells", type=int, default=12, help="cells of the 200-cell batch recipe")
    ap.add_argument("--max-samples", type=int, default=50000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--weights", default="bf16", choices=["bf16", "f32"])
    ap.add_argument("--checkpoint", default=None, help="per-epoch checkpoint (.npz): saved, and resumed from")
    ap.add_argument("--stop-after", type=int, default=None, help="epochs to run in this call (then checkpoint)")
    ap.add_argument("--metrics-jsonl", default=None, help="append per-epoch records here")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    wdt = sea.SEA_BF16 if args.weights == "bf16" else sea.SEA_F32
    ctx = sea.Context(rel_tol=1e-8, stencil_dtype=sea.SEA_F32, nn_weight_dtype=wdt)
    t0 = time.perf_counter()
    x, t = make_samples(ctx, training_cells(args.cells), max_samples=args.max_samples)
    log(f"{x.shape[0]} samples in {time.perf_counter() - t0:.1f} s")
    state, hist = train(ctx, x, t, epochs=args.epochs, batch=args.batch, lr=args.lr,
                        max_samples=args.max_samples, checkpoint=args.checkpoint, stop_after=args.stop_after,
                        metrics=args.metrics_jsonl)
    params = ctx.nn_get_params(state)
    np.save(args.out, params)
    meta = {"samples": int(min(x.shape[0], args.max_samples)), "epochs": args.epochs, "batch": args.batch,
            "lr": args.lr, "weights": args.weights, "history": hist}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(f"saved {args.out}")


if __name__ == "__main__":
    main()
