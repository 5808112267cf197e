"""Reverse-mode differentiation over the C ABI (torch.autograd.Functions).

* ``apply(A, x, adjoint=False)``: y = A x (or A^H x), differentiable in x;
  the vector-Jacobian product of a linear map is its adjoint, A^H G.
* ``circulant_apply(c, x, adjoint=False)``: y = C(c) x (or C(c)^H x),
  differentiable in the generator c and in x. The generator gradient is a
  circular cross-correlation (``fm_circulant_grad_generator``).
* ``unrolled_fista(c, b, rows, lam, L, iters, checkpoint)``: x_K of K FISTA
  steps on A = S_rows C(c) (the solver of eq. (8) on the row-selected
  circulant), differentiable in c and b. The forward pass keeps (x_k, y_k)
  every ``checkpoint`` steps; the backward pass recomputes each segment from
  its checkpoint and runs the reverse sweep with ``fm_fista_step_vjp``,
  operator applications and generator gradients. L and lam are constants.

Gradients follow PyTorch's convention for complex tensors. All arithmetic
runs in the HIP library; this module only sequences the calls and owns the
buffers (torch device memory).
"""

from __future__ import annotations

import torch

from . import capi
from .operators import Circulant, Operator, Product, SelectRows, _dt, _stream


def _as_block(x: torch.Tensor) -> torch.Tensor:
    xb = x.unsqueeze(0) if x.dim() == 1 else x
    return xb if xb.stride(-1) == 1 and xb.stride(0) == xb.shape[1] else xb.contiguous()


# ---------------------------------------------------------------- y = A x
class _OperatorApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, op, adjoint):
        ctx.op = op
        ctx.adjoint = adjoint
        return op.apply(x.detach(), adjoint)

    @staticmethod
    def backward(ctx, g):
        return ctx.op.apply(g.contiguous(), not ctx.adjoint), None, None


def apply(op: Operator, x: torch.Tensor, adjoint: bool = False) -> torch.Tensor:
    """A x (or A^H x) with gradient A^H G (or A G) for x."""
    return _OperatorApply.apply(x, op, adjoint)


# ---------------------------------------------------------------- generator gradient
def grad_generator(inp: torch.Tensor, g: torch.Tensor, adjoint: bool, out: torch.Tensor | None = None,
                   accumulate: bool = False) -> torch.Tensor:
    """Gradient of the generator c for y = C(c) inp (adjoint=False) or
    w = C(c)^H inp (adjoint=True), given the upstream gradient g of y / w,
    summed over the columns."""
    ib, gb = _as_block(inp), _as_block(g)
    if ib.shape != gb.shape or ib.dtype != gb.dtype:
        raise ValueError("input and upstream gradient must have the same shape and dtype")
    ncols, n = ib.shape
    if out is None:
        out = torch.empty(n, dtype=ib.dtype, device=ib.device)
    capi.fm_circulant_grad_generator(n, ncols, capi.FM_ADJ if adjoint else capi.FM_FWD, ib, n, gb, n, out,
                                     1 if accumulate else 0, _dt(ib.dtype), _stream())
    return out


class _CirculantApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, x, adjoint):
        op = Circulant(c.detach())
        ctx.op = op
        ctx.adjoint = adjoint
        ctx.vec = x.dim() == 1
        xb = _as_block(x.detach())
        ctx.save_for_backward(xb)
        y = op.apply(xb, adjoint)
        return y.squeeze(0) if ctx.vec else y

    @staticmethod
    def backward(ctx, g):
        (xb,) = ctx.saved_tensors
        gb = _as_block(g)
        gc = gx = None
        if ctx.needs_input_grad[1]:
            gx = ctx.op.apply(gb, not ctx.adjoint)
            if ctx.vec:
                gx = gx.squeeze(0)
        if ctx.needs_input_grad[0]:
            gc = grad_generator(xb, gb, ctx.adjoint)
        return gc, gx, None


def circulant_apply(c: torch.Tensor, x: torch.Tensor, adjoint: bool = False) -> torch.Tensor:
    """C(c) x (or C(c)^H x), differentiable in c and x."""
    return _CirculantApply.apply(c, x, adjoint)


# ---------------------------------------------------------------- unrolled FISTA
class _Problem:
    """A = S C(c) (S omitted without rows) and the buffers of one solve."""

    def __init__(self, c, rows, ncols):
        n = c.numel()
        self.n, self.ncols, self.dtype, self.dev = n, ncols, c.dtype, c.device
        self.dt = _dt(c.dtype)
        self.C = Circulant(c.detach().contiguous())
        self.S = SelectRows(n, rows, c.dtype) if rows is not None else None
        self.A = Product(self.S, self.C) if self.S is not None else self.C
        self.m = self.A.shape[0]

    def block(self, nrows=None, ncols=None):
        return torch.empty((ncols or self.ncols, nrows or self.n), dtype=self.dtype, device=self.dev)

    def axpby(self, alpha, x, beta, y, out):
        r = x.shape[1]
        capi.fm_axpby(r, self.ncols, alpha, x, r, beta, y, r, out, r, self.dt, _stream())

    def gradient(self, y, b, r, v, g):
        """g = A^H (A y - b) through r = A y - b and v = S^H r (without a
        selection v is r itself and r is not used)."""
        if self.S is None:
            r = v
        self.A.apply(y, out=r)
        self.axpby(1.0, r, -1.0, b, r)
        if self.S is not None:
            self.S.apply(r, adjoint=True, out=v)
        self.C.apply(v, adjoint=True, out=g)

    def step(self, y, g, x_old, x_new, y_new, z, lam, L, k, momentum):
        capi.fm_fista_step(self.n, self.ncols, y, g, x_old, x_new, y_new, z, self.n, lam, L, k, int(momentum),
                           self.dt, _stream())


class _UnrolledFista(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, b, rows, lam, L, iters, checkpoint, momentum):
        bb = _as_block(b.detach())
        ncols = bb.shape[0]
        P = _Problem(c, rows, ncols)
        if bb.shape[1] != P.m:
            raise ValueError(f"b must have {P.m} rows")
        lam = lam.detach().to(device=P.dev, dtype=torch.float64).contiguous()
        if lam.numel() == 1:
            lam = lam.expand(ncols).contiguous()
        if L is None:
            L = capi.fm_op_norm_bound(P.A.handle, _stream())
        x = torch.zeros((ncols, P.n), dtype=P.dtype, device=P.dev)
        y = x.clone()
        xn, yn, g, v = P.block(), P.block(), P.block(), P.block()
        r = P.block(P.m)
        ckpts = []
        for k in range(iters):
            if k % checkpoint == 0:
                ckpts.append((x.clone(), y.clone()))
            P.gradient(y, bb, r, v, g)
            P.step(y, g, x, xn, yn, None, lam, L, k, momentum)
            x, xn = xn, x
            y, yn = yn, y
        ctx.P, ctx.lam, ctx.L, ctx.momentum, ctx.ckpts = P, lam, float(L), int(momentum), ckpts
        ctx.iters, ctx.checkpoint, ctx.bb = iters, checkpoint, bb
        return x

    @staticmethod
    def backward(ctx, gx_out):
        P, lam, L, mom = ctx.P, ctx.lam, ctx.L, ctx.momentum
        K, seg = ctx.iters, ctx.checkpoint
        need_c, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        nc, n, m = P.ncols, P.n, P.m
        xbar = _as_block(gx_out).clone()        # gradient of x_{k+1}
        ybar = torch.zeros_like(xbar)            # gradient of y_{k+1}
        gc = torch.zeros(n, dtype=P.dtype, device=P.dev) if need_c else None
        gb = torch.zeros((nc, m), dtype=P.dtype, device=P.dev) if need_b else None
        rbar, t, g, r = P.block(m), P.block(), P.block(), P.block(m)
        for s0 in range((K - 1) // seg * seg, -1, -seg):
            s1 = min(s0 + seg, K)
            # Recompute the segment from its checkpoint. Step k keeps
            #   Y[k] = [y_k; gbar_k]  and  U[k] = [u_k; v_k]   (2 ncols x n each)
            # so that one correlation call sums both generator terms,
            # corr(u_k, y_k) (forward use) + corr(v_k, gbar_k) (adjoint use).
            x0, y0 = ctx.ckpts[s0 // seg]
            x, xs = x0.clone(), P.block()
            Y = [P.block(ncols=2 * nc) for _ in range(s0, s1)]
            U = [P.block(ncols=2 * nc) for _ in range(s0, s1)]
            Z = [P.block() for _ in range(s0, s1)]
            Y[0][:nc].copy_(y0)  # device copy of the checkpoint
            for k in range(s0, s1):
                j = k - s0
                P.gradient(Y[j][:nc], ctx.bb, r, U[j][nc:], g)
                yn = Y[j + 1][:nc] if k + 1 < s1 else P.block()
                P.step(Y[j][:nc], g, x, xs, yn, Z[j], lam, L, k, mom)
                x, xs = xs, x
            for k in range(s1 - 1, s0 - 1, -1):
                j = k - s0
                gbar = Y[j][nc:]
                # xbar <- gz (gradient of z_k), ybar <- -beta_k ybar (x_k part), gbar = -gz/L
                capi.fm_fista_step_vjp(n, nc, Z[j], xbar, ybar, xbar, gbar, ybar, n, lam, L, k, mom,
                                       P.dt, _stream())
                u = U[j][:nc]
                if P.S is not None:
                    P.A.apply(gbar, out=rbar)                  # rbar = A gbar
                    P.S.apply(rbar, adjoint=True, out=u)       # u = S^H rbar
                else:
                    P.A.apply(gbar, out=u)                     # rbar = u = A gbar
                    rbar = u
                P.C.apply(u, adjoint=True, out=t)              # A^H rbar
                P.axpby(1.0, xbar, 1.0, t, xbar)               # gradient of y_k
                if need_b:
                    P.axpby(1.0, gb, -1.0, rbar, gb)
                if need_c:
                    grad_generator(Y[j], U[j], adjoint=False, out=gc, accumulate=True)
                xbar, ybar = ybar, xbar
        return gc, gb, None, None, None, None, None, None


def unrolled_fista(c: torch.Tensor, b: torch.Tensor, rows: torch.Tensor | None, lam, L: float | None = None,
                   iters: int = 20, checkpoint: int = 5, momentum: bool = True) -> torch.Tensor:
    """x_K of ``iters`` FISTA steps for min 1/2||S C(c) x - b||^2 + lam_j ||x||_1
    per column of b (shape (ncols, m)), from x_0 = 0; differentiable in c and b.
    rows: int32 GPU tensor of selected rows (None: no selection). lam: float
    or per-column tensor. L: step constant (default: the structural bound
    max_k |DFT(c)_k|^2)."""
    if not torch.is_tensor(lam):
        lam = torch.tensor([float(lam)], dtype=torch.float64, device=c.device)
    return _UnrolledFista.apply(c, b, rows, lam, L, int(iters), int(checkpoint), bool(momentum))
