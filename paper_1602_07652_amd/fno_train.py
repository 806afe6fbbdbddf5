"""Training of the learned preconditioner on solves the method generates.

Data: for each seed, a Gaussian-random-field medium and an incident angle
(ls_inputs.fno_sample_recipe), the right-hand side f = -w^2 G (m u_I) and
the solution u of H u = f (the library's own solver, FP64, tol 1e-8).  The
network input is make_inputs(m, u_I, r = f) and its target the correction
(u - f) / s with s = ||f||_2 / n, as real and imaginary channels, so that
z = f + s y reproduces u.  Everything runs through the library (plans,
solves, network kernels); torch only holds the device arrays.

Training: Adam (the library's kernel) on the mean relative squared error,
cosine learning-rate decay, minibatches drawn by a seeded permutation.

    python -m paper_1602_07652_amd.fno_train --samples 2000 --epochs 30 \
        --out paper_1602_07652_amd/weights/fno_grf256.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

import ls_inputs as li
from . import Fno, Plan

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "fno_grf256.npz")


def log(msg):
    print(f"[fno-train] {msg}", flush=True)


def omega_for(n: int) -> float:
    """10 points per wavelength on the unit square with h = 1/n."""
    return 2 * np.pi * n / 10


def generate(fno: Fno, seeds, n=256, tol=1e-8, device="cuda:0"):
    """(X [S][5][n][n], Y [S][2][n][n]) float32 device tensors and the
    solver statistics of the generating solves."""
    dev = torch.device(device)
    S = len(seeds)
    X = torch.empty((S, 5, n, n), dtype=torch.float32, device=dev)
    Y = torch.empty((S, 2, n, n), dtype=torch.float32, device=dev)
    omega = omega_for(n)
    its, t0 = [], time.perf_counter()
    for k, seed in enumerate(seeds):
        m, theta = li.fno_sample_recipe(seed, n)
        md = torch.from_numpy(m).to(dev)
        plan = Plan(n, 1.0 / n, omega, md, slabs=max(1, n // 64), autotune=0, use_graphs=0)
        uI = torch.from_numpy(li.plane_wave(n, omega, theta)).to(dev)[None]
        f = plan.rhs_from_incident(uI)
        u, info = plan.solve(f, tol=tol)
        its.append(info[0]["outer_its"])
        x, s = fno.make_inputs(md, uI, f)
        X[k] = x[0]
        corr = (u[0] - f[0]) / s[0]
        Y[k, 0] = corr.real.float()
        Y[k, 1] = corr.imag.float()
        plan.close()
        if (k + 1) % 100 == 0 or k + 1 == S:
            log(f"generated {k + 1}/{S} solves in {time.perf_counter() - t0:.1f} s "
                f"(outer its mean {np.mean(its):.2f})")
    return X, Y, {"outer_its_mean": float(np.mean(its)), "gen_s": time.perf_counter() - t0}


def evaluate(fno: Fno, X, Y, batch):
    """Mean relative squared error over a data set (no training)."""
    tot, cnt = 0.0, 0
    dy = None
    for b0 in range(0, X.shape[0], batch):
        xb, yb = X[b0:b0 + batch], Y[b0:b0 + batch]
        y = fno.forward(xb)
        dy = torch.empty_like(y)
        L, _ = fno.loss(y, yb, dy)
        tot += L * xb.shape[0]
        cnt += xb.shape[0]
    return tot / cnt


def train(fno: Fno, X, Y, Xv, Yv, epochs=30, batch=16, lr=1e-3, lr_min=1e-5, seed=0, init_seed=0):
    init = torch.from_numpy(li.fno_initial_parameters(init_seed).astype(np.float32)).to(X.device)
    fno.set_params(init)
    rng = np.random.default_rng(seed)
    S = X.shape[0]
    steps_per_epoch = S // batch
    total = epochs * steps_per_epoch
    grad = torch.empty(fno.nparams, dtype=torch.float32, device=X.device)
    hist, t, t0 = [], 0, time.perf_counter()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(S)).to(X.device)
        acc = 0.0
        for it in range(steps_per_epoch):
            idx = perm[it * batch:(it + 1) * batch]
            xb, yb = X[idx].contiguous(), Y[idx].contiguous()
            y = fno.forward(xb, keep=True)
            L, dy = fno.loss(y, yb)
            fno.backward(dy, grad)
            t += 1
            cur = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * (t - 1) / total))
            fno.adam(grad, cur, t)
            acc += L
        val = evaluate(fno, Xv, Yv, batch)
        hist.append({"epoch": ep + 1, "train": acc / steps_per_epoch, "val": val})
        log(f"epoch {ep + 1}/{epochs}: train {acc / steps_per_epoch:.4f} val {val:.4f} "
            f"({time.perf_counter() - t0:.1f} s)")
    return hist, time.perf_counter() - t0


def save_weights(path, params: torch.Tensor, meta: dict):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez_compressed(path, params=params.detach().cpu().numpy().astype(np.float16),
                        meta=np.array(json.dumps(meta)))


def load_weights(path=DEFAULT_WEIGHTS, device="cuda:0"):
    """Parameters (float32 device tensor) and metadata of a saved network."""
    with np.load(path, allow_pickle=False) as z:
        p = torch.from_numpy(z["params"].astype(np.float32)).to(device)
        meta = json.loads(str(z["meta"]))
    return p, meta


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--samples", type=int, default=2000)
    ap.add_argument("--val", type=int, default=200)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("fno_train needs a GPU")
    fno = Fno(max_batch=args.batch, max_n=args.n)
    seeds = list(range(args.seed0, args.seed0 + args.samples))
    X, Y, gen = generate(fno, seeds, args.n)
    nt = args.samples - args.val
    hist, train_s = train(fno, X[:nt], Y[:nt], X[nt:], Y[nt:], args.epochs, args.batch, args.lr)
    meta = {"n": args.n, "omega": omega_for(args.n), "samples": args.samples, "val": args.val,
            "seeds": [args.seed0, args.seed0 + args.samples - 1], "epochs": args.epochs,
            "batch": args.batch, "lr": args.lr, "history": hist, "train_s": train_s, **gen}
    save_weights(args.out, fno.get_params(), meta)
    log(f"saved {args.out}: final val {hist[-1]['val']:.4f}")
    print(json.dumps({"train_s": train_s, "gen_s": gen["gen_s"], "val": hist[-1]["val"]}))
    fno.close()


if __name__ == "__main__":
    main()
