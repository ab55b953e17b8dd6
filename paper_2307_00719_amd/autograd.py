"""TR fit loss 1/2 ||TR(G) - X||_F^2 as a torch.autograd.Function.

Forward and backward both run in libtrstream.so on torch's current HIP
stream.  The backward returns, for every core, G_{n(2)} Q_n - P_n (the
normal-equation form of the gradient, Sec. 3.1) scaled by the incoming
gradient; subchains are rebuilt on the fly, never stored.
"""

import torch

from . import _lib


def _colmajor(x):
    return _lib._colmajor_torch(x)


def _colmajor_empty(shape, dtype, device):
    strides, acc = [], 1
    for s in shape:
        strides.append(acc)
        acc *= s
    return torch.empty_strided(tuple(shape), tuple(strides), dtype=dtype, device=device)


def _dt(t):
    if t.dtype == torch.float64:
        return _lib.TR_F64
    if t.dtype == torch.float32:
        return _lib.TR_F32
    raise TypeError("TR fit loss supports float32 and float64 tensors")


class TRFitLoss(torch.autograd.Function):
    """loss = TRFitLoss.apply(X, G_1, ..., G_N) with X of shape (I_1..I_N)
    and G_n of shape (R_n, I_n, R_{n+1}) on one HIP device; loss is a
    float64 scalar tensor."""

    @staticmethod
    def forward(ctx, X, *cores):
        if not X.is_cuda:
            raise RuntimeError("TRFitLoss runs on the HIP device only")
        dt = _dt(X)
        dims = list(X.shape)
        ranks = [int(G.shape[0]) for G in cores]
        Xc = _colmajor(X.detach())
        cs = [_colmajor(G.detach().to(X.dtype)) for G in cores]
        wsb = _lib.tr_workspace_bytes(dims, ranks, dt)
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=X.device)
        loss = torch.empty((), dtype=torch.float64, device=X.device)
        stream = torch.cuda.current_stream(X.device).cuda_stream
        _lib.tr_fit_loss_fwd(dims, ranks, dt, Xc.data_ptr(), [c.data_ptr() for c in cs],
                             loss.data_ptr(), ws.data_ptr(), wsb, stream)
        ctx.save_for_backward(Xc, *cs)
        ctx.meta = (dims, ranks, dt, [G.dtype for G in cores])
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        Xc, *cs = ctx.saved_tensors
        dims, ranks, dt, dtypes = ctx.meta
        wsb = _lib.tr_workspace_bytes(dims, ranks, dt)
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=Xc.device)
        grads = [_colmajor_empty(c.shape, c.dtype, c.device) for c in cs]
        stream = torch.cuda.current_stream(Xc.device).cuda_stream
        scale = float(grad_out)
        _lib.tr_fit_loss_bwd(dims, ranks, dt, Xc.data_ptr(), [c.data_ptr() for c in cs], scale,
                             [g.data_ptr() for g in grads], ws.data_ptr(), wsb, stream)
        out = [g.to(d) for g, d in zip(grads, dtypes)]
        return (None, *out)


def tr_fit_loss(X, cores):
    return TRFitLoss.apply(X, *cores)
