"""Train the GCIN smoother-coefficient predictor on the GPU (Alg. 1 of the paper).

Training problems (all levels of all meshes of a mini-batch in one GCIN launch), by family:
  delaunay  P1 Laplacians on Delaunay meshes of Gaussian-mixture-clustered points, 2k-16k nodes;
  cmesh     finite-volume C-meshes around random NACA 4-digit sections, ~24k-41k cells, wall
            aspect ratios 1e3-1e4 (for the 4M-cell airfoil mesh, 128 times larger);
  tet       finite-volume Poisson on jittered Kuhn tetrahedral meshes, ~8k-55k cells;
  grid      5-point Laplacians on square structured grids, 2k-16k nodes, Dirichlet (the
            structured case, for which the paper proposes the smaller 32-channel GCIN, App. B.3:
            --hidden 32);
  mixed     the three unstructured families in turn (a union of 2D and 3D problems, as in the paper's
            combined training set).
Each step:
batched GCIN forward, per-problem smoother assembly and nvc V(1,1) cycles from u = 0 with a
fresh uniform random zero-mean right-hand side, residual-reduction loss (Sec. 3.3, Eq. 11;
the multi-cycle form when nvc > 1), hand-written adjoint, GCIN backward, clipping at 1.0 and
Adam (App. B.1, Tab. 7). Every `--val-every` steps the validation metric of Eq. 13 (loss
relative to omega-Jacobi on held-out meshes) is evaluated and the best parameters are kept
(the paper's early stopping on the best validation model); the learning rate is halved when
the validation metric has not improved for --plateau-patience evaluations (the paper's
ReduceLROnPlateau scheduler, Tab. 7; its factor and patience are not given). With --seeds K
the whole training is repeated from K initialisations (the paper's seed ensemble, Sec. 4.2):
the ensemble's validation metrics are recorded and the best model is kept.

    python -m paper_2606_19251_amd.train --out weights.npz --steps 300
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def make_matrix(family, rng, seed):
    """One training matrix of the given family, drawn from rng."""
    import workloads as W

    if family == "delaunay":
        return W.delaunay_p1(W.gmm_points(int(rng.integers(2000, 16001)), seed))
    if family == "cmesh":
        code = f"{int(rng.integers(0, 5))}{int(rng.integers(2, 6))}{int(rng.integers(9, 16)):02d}"
        ni = int(rng.choice([224, 256, 288]))
        aspect = float(10 ** rng.uniform(3.0, 4.0))
        return W.cmesh_fv(ni, ni // 2, code, aspect)
    if family == "tet":
        P, T = W.kuhn_tets(int(rng.integers(12, 23)), seed, float(rng.uniform(0.05, 0.15)))
        return W.tet_fv_mesh(P, T)
    if family == "grid":
        return W.grid5(int(rng.integers(45, 127)))
    raise ValueError(family)


FAMILIES = ("delaunay", "cmesh", "tet")


def build_problems(family, seed0, count, device, max_coarse=100):
    from .solver import DeviceSolver, HostHierarchy

    rng = np.random.default_rng(seed0)
    out = []
    for k in range(count):
        fam = FAMILIES[k % len(FAMILIES)] if family == "mixed" else family
        A = make_matrix(fam, rng, seed0 * 1000 + k)
        hh = HostHierarchy.build(A.rowptr, A.col, A.val, max_coarse=max_coarse)
        out.append(DeviceSolver(hh, device.index or 0))
    return out


def train_one(args, seed, train, val, dev):
    """One training run from the initialisation `seed`: returns (best validation metric, its
    parameters, history)."""
    import torch

    import workloads as W
    from . import capi
    from . import gcin as G

    rng = np.random.default_rng(seed)
    nu = (args.nu, args.nu)

    def rhs_for(problems, s):
        r = np.random.default_rng(s)
        return [torch.from_numpy(W.rhs_uniform(ds.n, int(r.integers(1 << 30)), zero_mean=bool(ds.singular))).to(dev)
                for ds in problems]

    pred = G.Predictor(G.init_flat(args.degree, seed, hidden=args.hidden), dev, args.degree, capi.GCIN_BF16X3,
                       args.hidden)
    nb = max(1, len(train) // args.batch)
    trainers = [G.Trainer(train[b * args.batch:(b + 1) * args.batch], rhs_for(train[b * args.batch:(b + 1) * args.batch], b),
                          pred, lr=args.lr, nu=nu, nvc=args.nvc) for b in range(nb)]
    # one optimizer state shared by all mini-batches
    for tr in trainers[1:]:
        tr.m, tr.v = trainers[0].m, trainers[0].v
    val_rhs = rhs_for(val, 12345)
    val_tr = G.Trainer(val, val_rhs, pred, nu=nu, nvc=args.nvc)
    jac = torch.zeros(len(val), dtype=torch.float64, device=dev)
    dc = torch.zeros(16, 2 * args.degree + 1, dtype=torch.float64, device=dev)
    for p, ds in enumerate(val):
        ds.set_jacobi(2.0 / 3.0)
        capi.amgg_vcycle_loss_adjoint(ds.ctx, nu[0], nu[1], 32, args.nvc, val_rhs[p].data_ptr(), 0,
                                      jac[p:p + 1].data_ptr(), dc.data_ptr(), val_tr.batch.stream)

    def validate():
        val_tr.loss_and_grad()
        return float((val_tr.losses - jac).mean())  # Eq. 13: log10(||r|| / ||r_Jacobi||), mean over meshes

    best = validate()
    best_flat = pred.params.cpu().numpy().copy()
    history = [{"step": 0, "val": best, "seed": seed}]
    print(f"[train] seed {seed} step 0 val {best:+.4f}", flush=True)
    lr, stale = args.lr, 0
    step = 0
    t0 = time.time()
    while step < args.steps:
        tr = trainers[step % nb]
        tr.rhs = rhs_for(tr.solvers, int(rng.integers(1 << 30)))
        tr.step_count = step
        losses = tr.step()
        step += 1
        if step % args.val_every == 0 or step == args.steps:
            v = validate()
            if v < best:
                best, stale = v, 0
                best_flat = pred.params.cpu().numpy().copy()
            else:
                stale += 1
                if stale >= args.plateau_patience and lr > args.min_lr:
                    lr, stale = max(args.min_lr, lr * args.plateau_factor), 0
                    for t in trainers:
                        t.lr = lr
            rec = {"step": step, "loss": float(losses.mean()), "val": v, "lr": lr, "gnorm": float(tr.gnorm.item()),
                   "s": round(time.time() - t0, 1)}
            history.append(rec)
            print(f"[train] {json.dumps(rec)}", flush=True)
    return best, best_flat, history


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--degree", type=int, default=2)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--train-meshes", type=int, default=64)
    ap.add_argument("--val-meshes", type=int, default=8)
    ap.add_argument("--nvc", type=int, default=4)
    ap.add_argument("--nu", type=int, default=1, help="pre- and post-smoothing steps of the training cycles")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--val-every", type=int, default=25)
    ap.add_argument("--plateau-patience", type=int, default=4)
    ap.add_argument("--plateau-factor", type=float, default=0.5)
    ap.add_argument("--min-lr", type=float, default=1e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--seeds", type=int, default=1, help="independent initialisations; the best is kept")
    ap.add_argument("--family", choices=[*FAMILIES, "grid", "mixed"], default="delaunay")
    ap.add_argument("--hidden", type=int, choices=[64, 32], default=64, help="GCIN channels")
    args = ap.parse_args(argv)

    import torch

    dev = torch.device("cuda", 0)
    t0 = time.time()
    train = build_problems(args.family, 100 + args.seed, args.train_meshes, dev)
    val = build_problems(args.family, 900 + args.seed, args.val_meshes, dev)
    print(f"[train] {len(train)} training and {len(val)} validation meshes built in {time.time() - t0:.1f} s", flush=True)
    runs = []
    for k in range(args.seeds):
        best, flat, history = train_one(args, args.seed + k, train, val, dev)
        runs.append((best, flat, history))
        print(f"[train] seed {args.seed + k}: best validation {best:+.4f}", flush=True)
    vals = np.array([r[0] for r in runs])
    best, flat, history = runs[int(np.argmin(vals))]
    np.savez(args.out, params=flat, degree=np.int64(args.degree), hidden=np.int64(args.hidden), nvc=np.int64(args.nvc),
             nu=np.int64(args.nu), family=args.family, history=json.dumps(history), ensemble_val=vals)
    print(f"[train] ensemble of {len(vals)}: validation mean {vals.mean():+.4f} std {vals.std():.4f} "
          f"best {best:+.4f}; saved {args.out}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
