"""Learned warm start: training data from the library's own solves, GPU
training of the network with the library's kernels, and weights I/O.

The initial guess of a solve is x0_i = a_i m_i: a_i is the patch's amplitude
from the coarse (monopole) solve, which carries the long-range coupling of
the whole layout, and m_i (K coefficients) is the network's prediction of the
patch's own solution shape from its neighbourhood and a_i. Training data: for
seeded layouts shaped like the small workloads (N=10 patches of radius 0.1,
N=1000 of radius 0.01, uniform, area fraction 0.025, both problems; optionally
N=10,000 of radius 0.003 at the same area fraction), inputs
are the NCE_FEATURES per-patch features and targets the FP64 solutions f_i
divided by a_i.

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
    """(features, targets f_i / a_i, solve info) of one layout."""
    ctx = Context(centers, eps, problem=problem, tol_id=tol_id, tol_gmres=1e-10, far_field=FAR_AUTO)
    r = ctx.solve()
    a, _ = ctx.coarse()
    a = a.clamp(min=0.05 * float(a.mean()))
    t = (r["x"] / a[:, None]).float()
    f = ctx.features()
    ctx.close()
    return f, t, r


def generate(n_small: int, n_large: int, base_seed: int = 0, log=print, n_xl: int = 0):
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
    for s in range(n_xl):
        # larger layouts at the same area fraction: the long-range coupling (and
        # so the coarse amplitudes the network sees) of the benchmark sizes
        c = layouts.uniform_centers(10000, 0.003, 30000 + base_seed + s)
        prob = INTERIOR if s % 3 else EXTERIOR
        f, t, r = layout_samples(c, 0.003, prob)
        F.append(f)
        T.append(t)
        log(f"  data: N=10000 layout {s + 1}/{n_xl} iters {r['iters_fp64']} ({time.time() - t0:.0f} s)")
    return torch.cat(F), torch.cat(T)


def _last_layer(shape):
    """Offsets of the last layer's W (n_out x width) and b in the flat parameters."""
    n_in, width, hidden, n_out = shape
    dims = [n_in] + [width] * hidden + [n_out]
    off = 0
    for l in range(len(dims) - 1):
        w0 = off
        off += dims[l] * dims[l + 1]
        b0 = off
        off += dims[l + 1]
    return w0, b0, dims[-2], dims[-1]


def train(F, T, steps: int = 4000, batch: int = 2048, lr: float = 1e-3, seed: int = 0, log=print) -> Mlp:
    """Fit the network to the corrections T - e_0 of the coarse start, scaled to
    unit RMS so that the loss resolves them; the scale and the e_0 offset are
    then folded into the last layer, so the network's output is T itself."""
    import torch
    net = Mlp(*SHAPE, seed=seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    C = T.clone()
    C[:, 0] -= 1.0
    S = float(1.0 / torch.sqrt((C.double() ** 2).mean()))
    C = (C * S).contiguous()
    log(f"  train: correction RMS {1.0 / S:.3e}")
    n = F.shape[0]
    for it in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), device="cuda", generator=g)
        lr_t = lr * (0.5 * (1 + np.cos(np.pi * it / steps)))  # cosine decay
        loss = net.train_step(F[idx].contiguous(), C[idx].contiguous(), lr_t)
        if it % 500 == 0 or it == steps - 1:
            log(f"  train: step {it} loss {loss:.3e} (relative to the correction RMS)")
    th = net.get_params().astype(np.float64)
    w0, b0, n_prev, n_out = _last_layer(net.shape)
    th[w0:w0 + n_prev * n_out] /= S
    th[b0:b0 + n_out] /= S
    th[b0] += 1.0
    net.set_params(th.astype(np.float32))
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
    ap.add_argument("--large", type=int, default=50)
    ap.add_argument("--xl", type=int, default=8, help="layouts of N=10,000 (eps 0.003)")
    ap.add_argument("--steps", type=int, default=6000)
    args = ap.parse_args()
    os.environ.setdefault("NCE_CACHE", "/tmp")
    t0 = time.time()
    F, T = generate(args.small, args.large, log=lambda *a: print(*a, flush=True), n_xl=args.xl)
    print(f"samples {F.shape[0]} ({time.time() - t0:.0f} s)", flush=True)
    net = train(F, T, steps=args.steps, log=lambda *a: print(*a, flush=True))
    save(net, Path(args.out), {"samples": int(F.shape[0]), "small_layouts": args.small,
                               "large_layouts": args.large, "xl_layouts": args.xl, "steps": args.steps})
    print(f"saved {args.out} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
