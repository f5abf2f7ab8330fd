"""torch.autograd.Function wrappers of the predictor and of the V-cycle loss (plumbing: every
arithmetic step runs in libamggnn; these classes only route tensors between its calls).

GCIN        forward = gcin_forward over a training graph batch (Sec. 3.2, Eqs. 6-10; Alg. 1,
            step 6); backward = gcin_backward. The batch keeps the activations of its last
            forward only, so a backward must follow its own forward with no other forward of the
            same batch in between (checked).
VCycleLoss  forward = amgg_vcycle_loss_adjoint, or its block form for a BatchSolver: the loss of
            Sec. 3.3, Eq. 11 of each problem after nvc V-cycles from u = 0 with the smoother
            assembled from the given coefficients (Eq. 5; Alg. 1, steps 8-11). The library's
            adjoint recomputes each level's iterates from the forward sweep, so one call returns
            the losses together with their gradients with respect to the coefficient rows; the
            backward applies the chain rule to those (amgg_chain_loss_grad).

Typical use (one step of Alg. 1, steps 6-13):
    coeffs = GCIN.apply(params, batch, degree, precision)
    losses = VCycleLoss.apply(coeffs, batch_solver, f, (1, 1), 32, 1)
    torch.autograd.backward(losses, grad_tensors=weights)   # e.g. 1/|batch| each: the batch mean
    params.grad  ->  adam_step
"""
from __future__ import annotations

import torch

from . import capi


class GCIN(torch.autograd.Function):
    """coeffs [ngraphs, 2d+1] (FP32) = GCIN(params) over a training GraphBatch."""

    @staticmethod
    def forward(ctx, params, batch, degree, precision):
        if batch.flags & capi.GCIN_INFERENCE and params.requires_grad:
            raise ValueError("GCIN: an inference-only batch keeps nothing for a backward")
        coeffs = batch.forward(params.detach(), degree, precision)
        ctx.batch, ctx.degree, ctx.precision = batch, degree, precision
        ctx.forward_id = batch.nforward
        ctx.save_for_backward(params)
        return coeffs

    @staticmethod
    def backward(ctx, dcoeffs):
        (params,) = ctx.saved_tensors
        if ctx.batch.nforward != ctx.forward_id:
            raise RuntimeError("GCIN backward: the batch ran another forward since this one")
        g = ctx.batch.backward(params.detach(), dcoeffs.to(torch.float32).contiguous(), ctx.degree, ctx.precision)
        return g, None, None, None


class VCycleLoss(torch.autograd.Function):
    """losses (FP64, one per problem) = Eq. 11 loss of nvc V-cycles with the smoother of `coeffs`
    (FP32 [rows, 2d+1]: one row per level of a DeviceSolver, or one per level graph of every
    problem of a BatchSolver, problem-major)."""

    @staticmethod
    def forward(ctx, coeffs, solver, f, nu=(1, 1), precision=32, nvc=1):
        c = coeffs.detach().contiguous()
        if c.dtype != torch.float32 or c.dim() != 2 or c.shape[1] % 2 != 1:
            raise ValueError("VCycleLoss: coefficients must be a float32 [rows, 2d+1] tensor")
        degree = (c.shape[1] - 1) // 2
        dev = c.device
        stream = torch.cuda.current_stream(dev).cuda_stream
        dc = torch.empty(c.shape[0], c.shape[1], dtype=torch.float64, device=dev)  # written whole by the library
        if hasattr(solver, "nblk"):  # BatchSolver: one block-diagonal hierarchy of several problems
            solver.set_coeffs_device(c, degree, stream)
            losses = torch.empty(solver.nblk, dtype=torch.float64, device=dev)
            solver.loss_adjoint(f, losses, dc, nu, precision, nvc, stream)
            ctx.row_problem = solver.row_problem
        else:  # DeviceSolver: one problem, one coefficient row per level
            solver.set_coeffs_device(c, degree, stream)
            losses = torch.empty(1, dtype=torch.float64, device=dev)
            capi.amgg_vcycle_loss_adjoint(solver.ctx, nu[0], nu[1], precision, nvc, f.data_ptr(), 0,
                                          losses.data_ptr(), dc.data_ptr(), stream)
            ctx.row_problem = None
        ctx.save_for_backward(dc)
        return losses

    @staticmethod
    def backward(ctx, dloss):
        (dc,) = ctx.saved_tensors
        dloss = dloss.to(torch.float64).contiguous()
        out = torch.empty(dc.shape, dtype=torch.float32, device=dc.device)
        rp = ctx.row_problem
        capi.amgg_chain_loss_grad(dc.shape[0], dc.shape[1], dc.data_ptr(), 0 if rp is None else rp.data_ptr(),
                                  dloss.data_ptr(), out.data_ptr(), torch.cuda.current_stream(dc.device).cuda_stream)
        return out, None, None, None, None, None
