"""Learned warm start: training data from the library's own solves, GPU
training of the network with the library's kernels, and weights I/O.

Data: for seeded layouts shaped like the small workloads (N=10 patches of
radius 0.1 and N=1000 of radius 0.01, uniform, area fraction 0.025, both
problems), the FP64 solution f_i of every patch is the target, divided by
the layout's mean f_i[0] (the network predicts the shape; the solver fits the
overall scale by one system apply). Inputs are the NCE_FEATURES per-patch
features computed by the library.

    python -m paper_1906_04209_amd.warmstart --out paper_1906_04209_amd/weights/warmstart.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

import layouts  # noqa: E402

from . import FAR_AUTO, FP64, INTERIOR, EXTERIOR, Context, Mlp, FEATURES  # noqa: E402

WEIGHTS = Path(__file__).resolve().parent / "weights" / "warmstart.npz"
SHAPE = (FEATURES, 256, 3, 136)


def layout_samples(centers, eps, problem, tol_id=1e-11):
    """(features, normalised targets, solve info) of one layout."""
    ctx = Context(centers, eps, problem=problem, tol_id=tol_id, tol_gmres=1e-10, far_field=FAR_AUTO)
    r = ctx.solve()
    x = r["x"]
    scale = x[:, 0].mean()
    t = (x / scale).float()
    f = ctx.features()
    ctx.close()
    return f, t, r


def generate(n_small: int, n_large: int, base_seed: int = 0, log=print):
    import torch
    F, T = [], []
    t0 = time.time()
    for s in range(n_small):
        c = layouts.uniform_centers(10, 0.1, 10000 + base_seed + s)
        for prob in (INTERIOR, EXTERIOR):
            f, t, _ = layout_samples(c, 0.1, prob)
            F.append(f)
            T.append(t)
    for s in range(n_large):
        c = layouts.uniform_centers(1000, 0.01, 20000 + base_seed + s)
        prob = INTERIOR if s % 4 else EXTERIOR
        f, t, r = layout_samples(c, 0.01, prob)
        F.append(f)
        T.append(t)
        if s % 10 == 0:
            log(f"  data: layout {s + 1}/{n_large} iters {r['iters_fp64']} ({time.time() - t0:.0f} s)")
    return torch.cat(F), torch.cat(T)


def train(F, T, steps: int = 4000, batch: int = 2048, lr: float = 1e-3, seed: int = 0, log=print) -> Mlp:
    import torch
    net = Mlp(*SHAPE, seed=seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    n = F.shape[0]
    for it in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), device="cuda", generator=g)
        lr_t = lr * (0.5 * (1 + np.cos(np.pi * it / steps)))  # cosine decay
        loss = net.train_step(F[idx].contiguous(), T[idx].contiguous(), lr_t)
        if it % 500 == 0 or it == steps - 1:
            log(f"  train: step {it} loss {loss:.3e}")
    return net


def save(net: Mlp, path: Path, meta: dict) -> None:
    path.parent.mkdir(parents=True, exist_ok=True)
    np.savez(path, params=net.get_params(), shape=np.array(net.shape), meta=json.dumps(meta))


def load(path: Path = WEIGHTS) -> Mlp:
    z = np.load(path, allow_pickle=False)
    shape = tuple(int(v) for v in z["shape"])
    net = Mlp(*shape)
    net.set_params(z["params"])
    return net


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=str(WEIGHTS))
    ap.add_argument("--small", type=int, default=200)
    ap.add_argument("--large", type=int, default=48)
    ap.add_argument("--steps", type=int, default=4000)
    args = ap.parse_args()
    os.environ.setdefault("NCE_CACHE", "/tmp")
    t0 = time.time()
    F, T = generate(args.small, args.large, log=lambda *a: print(*a, flush=True))
    print(f"samples {F.shape[0]} ({time.time() - t0:.0f} s)", flush=True)
    net = train(F, T, steps=args.steps, log=lambda *a: print(*a, flush=True))
    save(net, Path(args.out), {"samples": int(F.shape[0]), "small_layouts": args.small,
                               "large_layouts": args.large, "steps": args.steps})
    print(f"saved {args.out} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
