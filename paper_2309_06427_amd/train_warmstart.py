"""Train the per-knot warm-start networks on the GPU and save their weights.

    python -m paper_2309_06427_amd.train_warmstart [--nx 6 14 26] [--problems 4096]
        [--epochs 30] [--hidden 128] [--out DIR]

For each state size: draw a training pool from the ragged generator restricted
to that nx (seed 4), build it in FP64 and label it with the library's own FP64
PCG to 1e-10, fit the input standardisation, then run Adam on the residual
loss.  Weights go to ``DIR/warmstart_nx{nx}_h{hidden}.npz`` together with the
per-epoch loss and the training time.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_DIR = os.path.join(HERE, "weights")
TRAIN_SEED = 4


def weights_path(nx: int, hidden: int = 128, root: str = DEFAULT_DIR) -> str:
    return os.path.join(root, f"warmstart_nx{nx}_h{hidden}.npz")


def train_one(nx: int, problems: int, epochs: int, hidden: int, out_dir: str, log=print) -> dict:
    import torch

    from . import inputs
    from .warmstart import WarmStartNet, training_pool
    t0 = time.perf_counter()
    db, lam_star = training_pool(nx, problems, seed=TRAIN_SEED)
    torch.cuda.synchronize()
    t_pool = time.perf_counter() - t0
    knots = int(db.batch.N.sum())
    log(f"[train nx={nx}] pool: {problems} problems, {knots} knots, labelled in {t_pool:.1f} s")
    net = WarmStartNet(nx, hidden)
    net.set_params(inputs.mlp_init(nx, hidden, seed=nx).astype(np.float32))
    net.fit_scaling(db, lam_star)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = net.train(db, lam_star, epochs=epochs, problems_per_step=16, lr=1e-3, lr_final=5e-5, seed=nx,
                     log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    os.makedirs(out_dir, exist_ok=True)
    path = weights_path(nx, hidden, out_dir)
    net.save(path, loss=hist.astype(np.float64), epochs=epochs, problems=problems, knots=knots,
             train_seconds=t_train, seed=TRAIN_SEED)
    log(f"[train nx={nx}] {epochs} epochs in {t_train:.1f} s, loss {hist[0]:.4g} -> {hist[-1]:.4g}; saved {path}")
    return dict(nx=nx, loss=hist, seconds=t_train, knots=knots, path=path)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, nargs="+", default=[6, 14, 26])
    ap.add_argument("--problems", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--out", default=DEFAULT_DIR)
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("train_warmstart: no GPU visible", file=sys.stderr)
        return 1
    for nx in args.nx:
        train_one(nx, args.problems, args.epochs, args.hidden, args.out,
                  log=lambda s: print(s, flush=True))
    return 0


if __name__ == "__main__":
    sys.exit(main())
