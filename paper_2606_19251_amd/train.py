"""Train the GCIN smoother-coefficient predictor on the GPU (Alg. 1 of the paper).

Training problems (all levels of all meshes of a mini-batch in one GCIN launch), by family:
  delaunay  P1 Laplacians on Delaunay meshes of Gaussian-mixture-clustered points, 2k-16k nodes;
  cmesh     finite-volume C-meshes around random NACA 4-digit sections, ~24k-41k cells, wall
            aspect ratios 1e3-1e4 (for the 4M-cell airfoil mesh, 128 times larger);
  tet       finite-volume Poisson on jittered Kuhn tetrahedral meshes, ~8k-55k cells;
  tetdel    the same on Delaunay tetrahedralisations of jittered lattices, ~9k-50k cells;
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
    if family == "tetdel":
        return W.tet_fv(W.jittered_lattice(int(rng.integers(12, 21)), seed))
    if family == "grid":
        return W.grid5(int(rng.integers(45, 127)))
    raise ValueError(family)


FAMILIES = ("delaunay", "cmesh", "tet")


class Plateau:
    """Learning-rate schedule on the validation metric (App. B.1, Tab. 7: ReduceLROnPlateau; its
    factor and patience are not given) with the best model kept (Sec. 3.3: the validation metric
    is the early-stopping criterion): a lower metric is a new best; otherwise the evaluation is
    stale, and `patience` stale evaluations in a row multiply the rate by `factor` (not below
    `min_lr`) and start the count again."""

    def __init__(self, lr, patience, factor, min_lr):
        self.lr, self.patience, self.factor, self.min_lr = lr, patience, factor, min_lr
        self.best = float("inf")
        self.stale = 0

    def update(self, v: float) -> bool:
        """Record one evaluation; True when it is a new best."""
        if v < self.best:
            self.best, self.stale = v, 0
            return True
        self.stale += 1
        if self.stale >= self.patience and self.lr > self.min_lr:
            self.lr, self.stale = max(self.min_lr, self.lr * self.factor), 0
        return False


def best_run(vals) -> int:
    """Index of the ensemble member kept (Sec. 4.2: seed ensembles): the lowest validation metric,
    the first one among equals."""
    return int(np.argmin(np.asarray(vals, np.float64)))


class Validator:
    """Eq. 13 on held-out problems: the mean over meshes of log10(||r_nvc|| / ||r_nvc^omega-J||) after
    nvc cycles from u = 0 (the difference of the two Eq. 11 losses), formed on the device by
    amgg_validation_metric."""

    def __init__(self, val, rhs, pred, nu, nvc, cycle_precision=32):
        import torch

        from . import capi
        from . import gcin as G

        self.torch = torch
        self.tr = G.Trainer(val, rhs, pred, nu=nu, nvc=nvc, cycle_precision=cycle_precision)
        dev = pred.device
        self.jac = torch.zeros(len(val), dtype=torch.float64, device=dev)
        dc = torch.zeros(16, 2 * pred.degree + 1, dtype=torch.float64, device=dev)
        for p, ds in enumerate(val):
            ds.set_jacobi(2.0 / 3.0)
            capi.amgg_vcycle_loss_adjoint(ds.ctx, nu[0], nu[1], cycle_precision, nvc, rhs[p].data_ptr(), 0,
                                          self.jac[p:p + 1].data_ptr(), dc.data_ptr(), self.tr.batch.stream)
        self.out = torch.zeros(1, dtype=torch.float64, device=dev)

    def __call__(self) -> float:
        from . import capi

        self.tr.loss_and_grad()
        capi.amgg_validation_metric(len(self.tr.solvers), self.tr.losses.data_ptr(), self.jac.data_ptr(),
                                    self.out.data_ptr(), self.tr.batch.stream)
        return float(self.out.item())


VAL_RHS_SEED = 12345  # the held-out problems' right-hand sides are fixed for a whole run


def seeded_rhs(problems, seed, device):
    """One U[-1, 1] right-hand side per problem (zero mean for all-Neumann ones), drawn from `seed`."""
    import torch

    import workloads as W

    r = np.random.default_rng(seed)
    return [torch.from_numpy(W.rhs_uniform(ds.n, int(r.integers(1 << 30)), zero_mean=bool(ds.singular))).to(device)
            for ds in problems]


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

    rhs_for = lambda problems, s: seeded_rhs(problems, s, dev)

    pred = G.Predictor(G.init_flat(args.degree, seed, hidden=args.hidden), dev, args.degree, capi.GCIN_BF16X3,
                       args.hidden, getattr(args, "diag_levels", 0))
    nb = max(1, len(train) // args.batch)
    trainers = [G.Trainer(train[b * args.batch:(b + 1) * args.batch], rhs_for(train[b * args.batch:(b + 1) * args.batch], b),
                          pred, lr=args.lr, nu=nu, nvc=args.nvc) for b in range(nb)]
    # one optimizer state shared by all mini-batches
    for tr in trainers[1:]:
        tr.m, tr.v = trainers[0].m, trainers[0].v
    validate = Validator(val, rhs_for(val, VAL_RHS_SEED), pred, nu, args.nvc)
    sched = Plateau(args.lr, args.plateau_patience, args.plateau_factor, args.min_lr)
    v0 = validate()
    sched.update(v0)
    best_flat = pred.params.detach().cpu().numpy().copy()
    history = [{"step": 0, "val": v0, "lr": sched.lr, "seed": seed}]
    print(f"[train] seed {seed} step 0 val {v0:+.4f}", flush=True)
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
            if sched.update(v):
                best_flat = pred.params.detach().cpu().numpy().copy()
            for t in trainers:
                t.lr = sched.lr
            rec = {"step": step, "loss": float(losses.mean()), "val": v, "lr": sched.lr,
                   "gnorm": float(tr.gnorm.item()), "s": round(time.time() - t0, 1)}
            history.append(rec)
            print(f"[train] {json.dumps(rec)}", flush=True)
    return sched.best, best_flat, history


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
    ap.add_argument("--family", choices=[*FAMILIES, "tetdel", "grid", "mixed"], default="delaunay")
    ap.add_argument("--hidden", type=int, choices=[64, 32], default=64, help="GCIN channels")
    ap.add_argument("--diag-levels", type=int, default=0,
                    help="finest levels whose smoother takes the diagonal form of Eq. 5 (f_o = 0)")
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
    best, flat, history = runs[best_run(vals)]
    np.savez(args.out, params=flat, degree=np.int64(args.degree), hidden=np.int64(args.hidden),
             diag_levels=np.int64(args.diag_levels), nvc=np.int64(args.nvc),
             nu=np.int64(args.nu), family=args.family, history=json.dumps(history), ensemble_val=vals)
    print(f"[train] ensemble of {len(vals)}: validation mean {vals.mean():+.4f} std {vals.std():.4f} "
          f"best {best:+.4f}; saved {args.out}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
