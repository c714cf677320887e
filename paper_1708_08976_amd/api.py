"""User-facing API in PyTorch's dimension order.

A C-contiguous tensor X of shape (S_0, ..., S_{N-1}) is the paper's tensor
with dims (S_{N-1}, ..., S_0) in the natural linearisation (the paper's mode
0 is torch's last axis).  Here `mode` and the factor list follow torch's
axes: factors[m] has shape (S_m, R) and mttkrp(X, factors, m) has shape
(S_m, R).  The mapping to the C-ABI's paper order happens only in this file.

Every call runs the HIP library; nothing here computes the operation itself.
"""
import torch

from . import _abi


class SplitBF16Tensor:
    """A float32 tensor stored as two bfloat16 planes (hi, lo) with value
    hi + lo: the input format of the split-precision MTTKRP."""

    def __init__(self, planes, shape):
        self.planes = planes
        self.shape = tuple(int(s) for s in shape)
        self.device = planes.device

    @classmethod
    def from_float(cls, x):
        x = x.contiguous()
        return cls(_abi.split_bf16(x), x.shape)

    def numel(self):
        n = 1
        for s in self.shape:
            n *= s
        return n


def _paper(X, factors):
    if isinstance(X, SplitBF16Tensor):
        shape, buf, dt = X.shape, X.planes, _abi.CPM_BF16X2
    else:
        shape, buf = tuple(X.shape), X.contiguous()
        dt = _abi.CPM_F64 if X.dtype == torch.float64 else _abi.CPM_F32
    N = len(shape)
    if len(factors) != N:
        raise ValueError("need %d factors, got %d" % (N, len(factors)))
    dims = tuple(reversed(shape))
    pf = [None if f is None else f.contiguous() for f in reversed(factors)]
    return buf, dims, pf, dt, N


def mttkrp(X, factors, mode, out=None):
    """MTTKRP for torch axis `mode`: out[i, c] = sum over entries with index i
    on that axis of X * prod of the other factors' rows."""
    buf, dims, pf, dt, N = _paper(X, factors)
    return _abi.mttkrp(buf, dims, pf, N - 1 - mode, out=out, dtype=dt)


def cp_als_step(X, factors, xnorm2=-1.0, want_fit=True):
    """One CP-ALS sweep updating `factors` in place (the paper's mode order
    0..N-1, i.e. torch axes from last to first).  Returns the fit."""
    buf, dims, pf, dt, N = _paper(X, factors)
    return _abi.cp_als_step(buf, dims, pf, dtype=dt, xnorm2=xnorm2, want_fit=want_fit)


def cp_grad(X, factors, xnorm2=-1.0):
    """(gradients in torch axis order, loss tensor) of 1/2||X - [[U]]||^2."""
    buf, dims, pf, dt, N = _paper(X, factors)
    grads, loss = _abi.cp_grad(buf, dims, pf, xnorm2=xnorm2, dtype=dt)
    return list(reversed(grads)), loss


def residual2(X, factors):
    """||X - [[U]]||_F^2 as a float64 GPU scalar, the model recomputed on the
    fly while X streams once (float32 or split-bf16 tensors)."""
    buf, dims, pf, dt, N = _paper(X, factors)
    return _abi.residual2(buf, dims, pf, dtype=dt)


def xnorm2(X):
    buf, dims, _, dt, _ = _paper(X, [None] * len(X.shape))
    return _abi.xnorm2(buf, dims, dtype=dt)


class CPLoss(torch.autograd.Function):
    """f(U_0..U_{N-1}) = 1/2 ||X - [[U]]||_F^2 for a fixed tensor X.

    forward: by default one MTTKRP (the last paper mode) and the Grams give
    f by ||X||^2 - 2 <M, U> + sum(Hadamard of the Grams); with exact=True
    the residual is recomputed entry by entry in one pass over X
    (cpm_residual2; float32 and split-bf16 tensors), which loses nothing to
    cancellation when the model fits closely.  Either way X - [[U]] is never
    stored.  backward: the hand-written gradient U_n H_n - MTTKRP_n for
    every factor, recomputing the MTTKRPs.  X gets no gradient.
    """

    @staticmethod
    def forward(ctx, X, xnorm2, exact, *factors):
        buf, dims, pf, dt, N = _paper(X, factors)
        xn = -1.0 if xnorm2 is None else float(xnorm2)
        if exact:
            loss = _abi.residual2(buf, dims, pf, dtype=dt).mul_(0.5)
        else:
            _, loss = _abi.cp_grad(buf, dims, pf, grads=False, xnorm2=xn, dtype=dt)
        ctx.X = X
        ctx.xnorm2 = xn
        ctx.save_for_backward(*factors)
        return loss

    @staticmethod
    def backward(ctx, g):
        factors = ctx.saved_tensors
        buf, dims, pf, dt, N = _paper(ctx.X, factors)
        grads, _ = _abi.cp_grad(buf, dims, pf, xnorm2=ctx.xnorm2, dtype=dt)
        scale = g.to(grads[0].dtype)
        out = [gr.mul_(scale) for gr in reversed(grads)]
        return (None, None, None) + tuple(out)


def cp_loss(X, factors, xnorm2=None, exact=False):
    return CPLoss.apply(X, xnorm2, bool(exact), *factors)
