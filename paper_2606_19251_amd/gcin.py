"""Plumbing for the GCIN predictor: device memory for batches and parameters (torch tensors),
checkpoint I/O, and the training loop that sequences the C entry points.

Every arithmetic step (graph batching, forward, backward, V-cycle loss and adjoint, Adam)
runs in libamggnn; this module only allocates, passes pointers and orders the calls
(Alg. 1 of the paper: batched inference over all levels of all problems, per-problem
smoother assembly and V-cycle, batch-mean loss, optimizer step).
"""
from __future__ import annotations

import numpy as np

from . import capi

HIDDEN = 64
LAYERS = 4


def param_shapes(degree: int = 2, hidden: int = HIDDEN):
    """(name, shape) of every tensor in the flat parameter vector, in storage order (hidden
    width 64, or 32 for the smaller variant)."""
    shapes = []
    for l in range(LAYERS):
        shapes += [(f"conv{l}.W", (2 if l == 0 else hidden, hidden)), (f"conv{l}.b", (hidden,)),
                   (f"norm{l}.gamma", (hidden,)), (f"norm{l}.beta", (hidden,))]
    for l in range(LAYERS):
        shapes += [(f"readout{l}.W", (2 * hidden, 32)), (f"readout{l}.b", (32,))]
    shapes += [("ln.gamma", (128,)), ("ln.beta", (128,)), ("mlp0.W", (128, 128)), ("mlp0.b", (128,)),
               ("mlp1.W", (128, 64)), ("mlp1.b", (64,)), ("mlp2.W", (64, 2 * degree + 1)),
               ("mlp2.b", (2 * degree + 1,))]
    return shapes


def hidden_of(params: dict) -> int:
    return int(np.shape(params["conv0.W"])[1])


def pack(params: dict, degree: int = 2) -> np.ndarray:
    """Flat float32 vector from a {name: array} dict (the hidden width is read from conv0.W)."""
    hidden = hidden_of(params)
    flat = np.concatenate([np.asarray(params[k], np.float64).reshape(-1) for k, _ in param_shapes(degree, hidden)])
    assert flat.size == capi.gcin_param_count(degree, hidden)
    return flat.astype(np.float32)


def unpack(flat: np.ndarray, degree: int = 2, hidden: int = HIDDEN) -> dict:
    out, k = {}, 0
    for name, shape in param_shapes(degree, hidden):
        sz = int(np.prod(shape))
        out[name] = np.asarray(flat[k:k + sz], np.float64).reshape(shape)
        k += sz
    return out


def init_flat(degree: int = 2, seed: int = 0, omega: float = 2.0 / 3.0, hidden: int = HIDDEN) -> np.ndarray:
    """Initial parameters: uniform(+-1/sqrt(fan_in)) weights, zero biases, unit norm gains; the
    last layer is scaled by 1e-2 and its bias set to (omega, 0, ...), so the untrained
    predictor starts next to omega-Jacobi."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in param_shapes(degree, hidden):
        if name.endswith(".W"):
            b = 1.0 / np.sqrt(shape[0])
            p[name] = rng.uniform(-b, b, size=shape)
        elif name.endswith("gamma"):
            p[name] = np.ones(shape)
        else:
            p[name] = np.zeros(shape)
    p["mlp2.W"] *= 1e-2
    p["mlp2.b"][0] = omega
    return pack(p, degree)


class GraphBatch:
    """A batch of level graphs on the GPU (gcin_batch_create); keeps its workspace alive."""

    def __init__(self, graphs, device, hidden: int = HIDDEN, inference: bool = False):
        """graphs: list of (rowptr, col, val) CUDA tensors (int32, int32, float64) of level matrices.
        inference: forward passes only (no activations kept for a backward, a smaller workspace)."""
        import torch

        self.torch = torch
        self.device = device
        self.hidden = hidden
        self.flags = capi.GCIN_INFERENCE if inference else 0
        self.ngraphs = len(graphs)
        n = np.array([int(g[0].numel() - 1) for g in graphs], np.int32)
        nnz = np.array([int(g[1].numel()) for g in graphs], np.int32)
        self.n = n
        self.ws_bytes = capi.gcin_batch_workspace_bytes(n, nnz, hidden, self.flags)
        raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off:off + self.ws_bytes]
        views = [(int(n[i]), int(nnz[i]), g[0].data_ptr(), g[1].data_ptr(), g[2].data_ptr()) for i, g in enumerate(graphs)]
        self.handle = capi.gcin_batch_create(views, self.ws.data_ptr(), self.ws_bytes, self.stream, hidden, self.flags)
        self.nforward = 0  # forwards run so far (a backward belongs to the latest one)

    @property
    def stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def forward(self, params, degree=2, precision=capi.GCIN_BF16, out=None):
        torch = self.torch
        if out is None:
            out = torch.empty(self.ngraphs, 2 * degree + 1, dtype=torch.float32, device=self.device)
        capi.gcin_forward(self.handle, degree, precision, params.data_ptr(), out.data_ptr(), self.stream)
        self.nforward += 1
        return out

    def backward(self, params, dcoeffs, degree=2, precision=capi.GCIN_BF16, grads=None):
        torch = self.torch
        if grads is None:
            grads = torch.empty_like(params)
        capi.gcin_backward(self.handle, degree, precision, params.data_ptr(), dcoeffs.data_ptr(), grads.data_ptr(),
                           self.stream)
        return grads

    def close(self):
        if self.handle:
            capi.gcin_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Predictor:
    """GCIN parameters on the device; predicts per-level smoother coefficients of a solver."""

    def __init__(self, flat: np.ndarray, device, degree: int = 2, precision: int = capi.GCIN_BF16,
                 hidden: int = HIDDEN, diag_levels: int = 0):
        """diag_levels: the number of finest levels whose smoother takes the diagonal form of
        Eq. 5 (f_o = 0), as the network was trained."""
        import torch

        self.torch = torch
        self.device = device
        self.degree = degree
        self.precision = precision
        self.hidden = hidden
        self.diag_levels = int(diag_levels)
        if np.size(flat) != capi.gcin_param_count(degree, hidden):
            raise ValueError(f"{np.size(flat)} parameters do not fit degree {degree}, hidden width {hidden}")
        self.params = torch.from_numpy(np.ascontiguousarray(flat, np.float32)).to(device)

    @classmethod
    def load(cls, path, device, precision: int = capi.GCIN_BF16):
        z = np.load(path, allow_pickle=False)
        hidden = int(z["hidden"]) if "hidden" in z.files else HIDDEN
        diag = int(z["diag_levels"]) if "diag_levels" in z.files else 0
        return cls(z["params"], device, int(z["degree"]), precision, hidden, diag)

    def save(self, path):
        np.savez(path, params=self.params.detach().cpu().numpy(), degree=np.int64(self.degree),
                 hidden=np.int64(self.hidden), diag_levels=np.int64(self.diag_levels))

    def predict(self, hier, ds):
        """Coefficients [nlevels, 2d+1] (float32 CUDA tensor) for a DeviceSolver's levels (an
        inference-only graph batch: no activations are kept). Also records on the solver the
        number of finest levels that take the diagonal form (used by its set_coeffs_device)."""
        ds.diag_levels = self.diag_levels
        batch = GraphBatch([ds.A[l] for l in range(ds.nlevels)], self.device, self.hidden, inference=True)
        out = batch.forward(self.params, self.degree, self.precision)
        self._last_batch = batch
        return out

    def predict_judged(self, hier, ds, b, x=None, **judge_kw):
        """Predict the coefficients, then let the omega-Jacobi AMG judge them on b (DeviceSolver.judge):
        the solver keeps the learned smoother only when it predicts the shorter solve. Returns
        (coefficients, the judge's record)."""
        coeffs = self.predict(hier, ds)
        return coeffs, ds.judge(b, coeffs, self.degree, x=x, diag_levels=self.diag_levels, **judge_kw)


class Trainer:
    """Alg. 1 of the paper on the GPU: batched GCIN inference over every level of every problem,
    per-problem smoother assembly and one (or nvc) V-cycles with the residual-reduction loss,
    hand-written adjoint, GCIN backward, gradient clipping and Adam."""

    def __init__(self, solvers, rhs, predictor: Predictor, lr=1e-3, clip=1.0, nu=(1, 1), nvc=1,
                 cycle_precision=32, streams=1, batched=True):
        """batched: cycle every problem in one block-diagonal context (one launch per level
        operation for the whole mini-batch); otherwise problem by problem, spread over
        `streams` streams. The predictor's diag_levels finest levels of every problem take the
        diagonal form of Eq. 5 (their off-diagonal coefficients get a zero gradient)."""
        import torch

        self.torch = torch
        self.solvers = solvers
        self.batched = batched
        self.rhs = rhs
        self.pred = predictor
        self.lr, self.clip, self.nu, self.nvc = lr, clip, nu, nvc
        self.cycle_precision = cycle_precision
        dev = predictor.device
        graphs, self.slices = [], []
        for ds in solvers:
            self.slices.append((len(graphs), len(graphs) + ds.nlevels))
            graphs += [ds.A[l] for l in range(ds.nlevels)]
        self.batch = GraphBatch(graphs, dev, predictor.hidden)
        d = predictor.degree
        n = predictor.params.numel()
        self.m = torch.zeros(n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=dev)
        self.grads = torch.zeros(n, dtype=torch.float32, device=dev)
        self.scratch = torch.empty(capi.adam_scratch_bytes(), dtype=torch.uint8, device=dev)
        self.gnorm = torch.zeros(1, dtype=torch.float32, device=dev)
        self.losses = torch.zeros(len(solvers), dtype=torch.float64, device=dev)
        self.wmean = torch.full((len(solvers),), 1.0 / len(solvers), dtype=torch.float64, device=dev)
        self.dc64 = torch.zeros(self.batch.ngraphs, 2 * d + 1, dtype=torch.float64, device=dev)
        self.dc32 = torch.zeros(self.batch.ngraphs, 2 * d + 1, dtype=torch.float32, device=dev)
        self.step_count = 0
        # the problems' cycles and adjoints are independent: with streams > 1 they are spread
        # over that many streams (default priority) between two event joins
        self.side = [torch.cuda.Stream(device=dev) for _ in range(streams)] if streams > 1 and not batched else []
        self.bsolver = None
        for ds in solvers:
            ds.diag_levels = predictor.diag_levels
        if batched:
            from .solver import BatchSolver

            self.bsolver = BatchSolver([ds.hier for ds in solvers], dev.index or 0)
            self.bsolver.diag_levels = predictor.diag_levels
            assert self.bsolver.ngraphs == self.batch.ngraphs
        # fork / join events live as long as the trainer: an event must outlive the waits
        # queued on it
        self.fork = torch.cuda.Event()
        self.joins = [torch.cuda.Event() for _ in self.side]

    @property
    def rhs(self):
        return self._rhs

    @rhs.setter
    def rhs(self, value):
        self._rhs = list(value)
        self.f_cat = self.torch.cat(self._rhs) if self.batched else None

    def loss_and_grad(self):
        """Batch-mean loss (device tensor of per-problem losses) and d loss / d coefficients."""
        torch = self.torch
        d = self.pred.degree
        coeffs = self.batch.forward(self.pred.params, d, self.pred.precision)
        stream = self.batch.stream
        if self.bsolver is not None:
            self.bsolver.set_coeffs_device(coeffs, d, stream)
            self.bsolver.loss_adjoint(self.f_cat, self.losses, self.dc64, self.nu, self.cycle_precision, self.nvc,
                                      stream)
            capi.amgg_cast_scale_f64_f32(self.dc64.data_ptr(), self.dc32.data_ptr(), self.dc64.numel(),
                                         1.0 / len(self.solvers), stream)
            return coeffs
        if self.side:
            main = torch.cuda.current_stream(self.pred.device)  # the stream `stream` names
            self.fork.record(main)
            for s in self.side:
                s.wait_event(self.fork)
        for p, ds in enumerate(self.solvers):
            a, b = self.slices[p]
            st = self.side[p % len(self.side)].cuda_stream if self.side else stream
            ds.set_coeffs_device(coeffs[a:b], d, stream=st)
            capi.amgg_vcycle_loss_adjoint(ds.ctx, self.nu[0], self.nu[1], self.cycle_precision, self.nvc,
                                          self.rhs[p].data_ptr(), 0, self.losses[p:p + 1].data_ptr(),
                                          self.dc64[a:b].data_ptr(), st)
        for s, join in zip(self.side, self.joins):
            join.record(s)
            main.wait_event(join)
        capi.amgg_cast_scale_f64_f32(self.dc64.data_ptr(), self.dc32.data_ptr(), self.dc64.numel(),
                                     1.0 / len(self.solvers), stream)
        return coeffs

    def step(self):
        """One step of Alg. 1: forward, batch-mean loss, gradients, clipping and Adam. Batched, the
        gradient flows through the autograd Functions GCIN and VCycleLoss (the batch mean enters as
        the weights 1/|batch| of the per-problem losses); one problem at a time, the same library
        calls are made directly."""
        d = self.pred.degree
        if self.bsolver is not None:
            from .autograd import GCIN, VCycleLoss

            torch = self.torch
            P = self.pred.params.detach().requires_grad_()
            coeffs = GCIN.apply(P, self.batch, d, self.pred.precision)
            losses = VCycleLoss.apply(coeffs, self.bsolver, self.f_cat, self.nu, self.cycle_precision, self.nvc)
            torch.autograd.backward(losses, grad_tensors=self.wmean)
            grads = self.grads = P.grad  # the step's gradient (before clipping), kept for inspection
            self.losses = losses.detach()
        else:
            self.loss_and_grad()
            self.batch.backward(self.pred.params, self.dc32, d, self.pred.precision, self.grads)
            grads = self.grads
        self.step_count += 1
        capi.adam_step(self.pred.params.data_ptr(), grads.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                       self.pred.params.numel(), self.lr, 0.9, 0.999, 1e-8, self.step_count, self.clip,
                       self.gnorm.data_ptr(), self.scratch.data_ptr(), self.batch.stream)
        return self.losses
