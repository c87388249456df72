"""Unsupervised training of the unfolded PGD network (Sec. V; Sec. VI-A) on the GPU.

Host control only: the epoch shuffle (seeded numpy permutation, passed to the
library as channel indices), the epoch loop and early stopping.  Every
gradient, Adam update and projection runs in dmimo_ufpgd_train; validation
costs come from dmimo_ufpgd_grad; the test-set metrics from dmimo_pgd and
dmimo_beamform.

The paper's setting: K = 8 users, M = 64 antennas, 1e5 training and 5000
validation channels H ~ CN(0, 1), gamma = 10 dB, sigma = 1, the cost's
lambda = 1/15, I = 20 layers, Adam at lr 1e-3, batch 64, up to 200 epochs
with early stopping.  The network starts as 20 iterations of plain PGD
(lambda = 1/15, eta = 1/L~).

    python -m paper_2304_12745_amd.train --epochs 200 --out trained.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class FitResult:
    lambdas: list
    etas: list
    best_epoch: int
    epochs_run: int
    val_cost: list = field(default_factory=list)
    train_cost: list = field(default_factory=list)
    seconds: float = 0.0
    steps: int = 0


class EarlyStopping:
    """Early stopping on the validation cost (Sec. VI-A): remember the epoch
    with the lowest cost; stop after `patience` epochs in a row without a new
    lowest.  update() returns True when the epoch is the new best."""

    def __init__(self, patience: int):
        self.patience = patience
        self.best_cost = math.inf
        self.best_epoch = -1
        self.bad = 0

    def update(self, epoch: int, cost: float) -> bool:
        if cost < self.best_cost:
            self.best_cost, self.best_epoch, self.bad = cost, epoch, 0
            return True
        self.bad += 1
        return False

    @property
    def stop(self) -> bool:
        return self.bad >= self.patience


def fit(Htrain, Hval, gamma_lin, sigma2=1.0, lam_c=1.0 / 15.0, layers=20, epochs=200, batch=64,
        lr=1e-3, patience=10, seed=0, log=None) -> FitResult:
    """Train lambda_i, eta_i.  Htrain, Hval: device complex64 [n][K][M].

    Early stopping: keep the parameters of the epoch with the lowest mean
    validation cost; stop after `patience` epochs without a new lowest."""
    import torch

    from . import dmimo as D

    n, K, M = Htrain.shape
    dev = Htrain.device
    L = (math.sqrt(K) + math.sqrt(M)) ** 2
    state = D.UfpgdState([1.0 / 15.0] * layers, [1.0 / L] * layers, dev)
    rng = np.random.default_rng(seed)
    full = n // batch * batch
    ws = torch.empty((D.ufpgd_workspace_size(batch, K, M, layers),), dtype=torch.uint8, device=dev)
    res = FitResult([], [], -1, 0)
    es = EarlyStopping(patience)
    best = None
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(n).astype(np.int32)
        idx = torch.from_numpy(perm[:full].reshape(-1, batch)).to(dev)
        bc = D.ufpgd_train(Htrain, state, idx, gamma_lin, sigma2, lam_c, lr=lr, ws=ws)
        tc = bc.sum()
        nb = idx.shape[0]
        if full < n:
            tail = torch.from_numpy(perm[full:].reshape(1, -1)).to(dev)
            tc = tc + D.ufpgd_train(Htrain, state, tail, gamma_lin, sigma2, lam_c, lr=lr).sum()
            nb += 1
        val = D.ufpgd_grad(Hval, state.lambdas, state.etas, gamma_lin, sigma2, lam_c,
                           want_grad=False).cost.mean().item()
        res.train_cost.append(tc.item() / nb)
        res.val_cost.append(val)
        res.epochs_run = ep + 1
        if es.update(ep, val):
            best, res.best_epoch = state.clone(), ep
        if log:
            log(f"epoch {ep + 1}: train cost {res.train_cost[-1]:.6f} val cost {val:.6f} "
                f"({time.perf_counter() - t0:.1f} s)")
        if es.stop:
            break
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    res.steps = state.t
    res.lambdas = best.lambdas.cpu().tolist()
    res.etas = best.etas.cpu().tolist()
    return res


def evaluate(H, lambdas, etas, gamma_lin, sigma2=1.0):
    """Mean sum rate and PCG = ||W_ZF||_{2,1} / ||W||_{2,1} (Sec. VI-B) of the
    network with the given schedule on device channels H [B][K][M]; ZF with
    the paper's scaling H W^T = sigma D_gamma^{1/2}."""
    from . import dmimo as D

    r = D.pgd(H, lambdas, etas, gamma_lin, sigma2)
    zf = D.beamform(H, "zf", gamma_lin, sigma2, 0.0, "f32")
    pcg = (zf.l21 / r.l21).mean().item()
    return {"rsum": r.rsum.mean().item(), "pcg": pcg}


def convergence(H, lambdas, etas, gamma_lin, sigma2=1.0,
                long_iters=(20, 50, 100, 200, 500, 1000, 2000, 3500, 5000)):
    """Mean R_sum and PCG per layer (Sec. VI-C): the trained network cut after
    layer i, and plain PGD (lambda = 1/15, eta = 1/L~) after i iterations, for
    i = 1 .. I; plain PGD also at the longer iteration counts.  Every point is
    one dmimo_pgd launch over all channels H [B][K][M] from W(0) = H^*."""
    I = len(lambdas)
    K, M = H.shape[1], H.shape[2]
    L = (math.sqrt(K) + math.sqrt(M)) ** 2
    uf = [evaluate(H, lambdas[:i], etas[:i], gamma_lin, sigma2) for i in range(1, I + 1)]
    pgd = [evaluate(H, [1.0 / 15.0] * i, [1.0 / L] * i, gamma_lin, sigma2) for i in range(1, I + 1)]
    long = [dict(iterations=n, **evaluate(H, [1.0 / 15.0] * n, [1.0 / L] * n, gamma_lin, sigma2))
            for n in long_iters]
    return {"layers": list(range(1, I + 1)),
            "ufpgd": {"pcg": [x["pcg"] for x in uf], "rsum": [x["rsum"] for x in uf]},
            "pgd": {"pcg": [x["pcg"] for x in pgd], "rsum": [x["rsum"] for x in pgd]},
            "pgd_long": long}


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--epochs", type=int, default=200)
    p.add_argument("--patience", type=int, default=10)
    p.add_argument("--n-train", type=int, default=100000)
    p.add_argument("--n-val", type=int, default=5000)
    p.add_argument("--n-test", type=int, default=5000)
    p.add_argument("--layers", type=int, default=20)
    p.add_argument("--batch", type=int, default=64)
    p.add_argument("--lr", type=float, default=1e-3)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--out", default=None, help="write the trained schedule and metrics as JSON")
    p.add_argument("--curve", action="store_true",
                   help="also evaluate R_sum and PCG per layer / iteration on the test set")
    a = p.parse_args(argv)

    import torch

    from . import dmimo as D
    from . import workloads as WL

    if not torch.cuda.is_available():
        print("training needs a GPU", file=sys.stderr)
        return 1
    D.lib()
    dev = torch.device("cuda:0")
    sets = WL.ufpgd_datasets(a.n_train, a.n_val, a.n_test, seed=a.seed)
    Htr, Hva, Hte = (torch.from_numpy(x).to(dev) for x in (sets.train, sets.val, sets.test))
    g = sets.gamma_lin
    K, M = Htr.shape[1:]
    L = (math.sqrt(K) + math.sqrt(M)) ** 2
    base = evaluate(Hte, [1.0 / 15.0] * a.layers, [1.0 / L] * a.layers, g)
    print(f"PGD, {a.layers} iterations: {base}", flush=True)
    res = fit(Htr, Hva, g, layers=a.layers, epochs=a.epochs, batch=a.batch, lr=a.lr,
              patience=a.patience, seed=a.seed, log=lambda s: print(s, flush=True))
    test = evaluate(Hte, res.lambdas, res.etas, g)
    print(f"UfPGD, {a.layers} layers, best epoch {res.best_epoch + 1}: {test}", flush=True)
    curve = None
    if a.curve:
        curve = convergence(Hte, res.lambdas, res.etas, g)
        for i, n in enumerate(curve["layers"]):
            print(f"layer {n:2d}: UfPGD PCG {curve['ufpgd']['pcg'][i]:.4f} R_sum "
                  f"{curve['ufpgd']['rsum'][i]:.3f} | PGD PCG {curve['pgd']['pcg'][i]:.4f} R_sum "
                  f"{curve['pgd']['rsum'][i]:.3f}", flush=True)
        for x in curve["pgd_long"]:
            print(f"PGD {x['iterations']:5d} iterations: PCG {x['pcg']:.4f} R_sum {x['rsum']:.3f}",
                  flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"lambdas": res.lambdas, "etas": res.etas, "best_epoch": res.best_epoch + 1,
                       "epochs_run": res.epochs_run, "steps": res.steps, "seconds": res.seconds,
                       "val_cost": res.val_cost, "train_cost": res.train_cost,
                       "test": test, "pgd_baseline": base, "curve": curve, "args": vars(a)},
                      f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
