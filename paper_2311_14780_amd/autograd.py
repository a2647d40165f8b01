"""torch.autograd.Function wrappers around the C ABI.

``PtychoLoss`` returns the scalar loss of Eq. 1's model against the measured
patterns; its backward multiplies the library's hand-written gradients
(object, probe, positions, power coefficients, background and, for a tensor
of exact sampling ratios, dL/d alpha, i.e. the propagation distance) by the
incoming gradient.
The forward call already computes the gradients (one fused pass), so the
backward is a scaling only.

``PtychoForward`` returns the predicted patterns I'_k; its backward is the
vector-Jacobian product, computed by the same library call with the VJP loss
kind (the upstream gradient takes the place of the measured patterns).

Complex gradients follow PyTorch's convention for real-valued losses,
G = dL/dRe + i dL/dIm, which is also the library's.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import binding as B


_KEYS = ("g_object", "g_probe", "g_pos", "g_sigma", "g_background", "g_ratio")


def _zeros_like_grads(problem: B.Problem, need):
    """need: flags for object, probe, positions, sigma, background, ratio."""
    dev = problem.object.device
    need = tuple(need) + (False,) * (6 - len(need))
    g = dict(loss=torch.zeros(1, device=dev))
    if need[0]:
        g["g_object"] = torch.zeros_like(problem.object)
    if need[1]:
        g["g_probe"] = torch.zeros_like(problem.probe)
    if need[2]:
        g["g_pos"] = torch.zeros(problem.K, 2, device=dev)
    if need[3]:
        g["g_sigma"] = torch.zeros(problem.K, device=dev)
    if need[4]:
        g["g_background"] = torch.zeros(problem.N, problem.N, device=dev)
    if need[5]:
        g["g_ratio"] = torch.zeros(problem.L, device=dev)
    return g


def _pads_of(pads, ratio):
    """A tensor of exact ratios (floats) replaces the pads."""
    if ratio is None:
        return tuple(pads)
    return tuple(float(a) for a in ratio.detach().cpu().tolist())


class _Workspace:
    """Caches one device workspace per (device, size)."""

    def __init__(self):
        self.buf: Optional[torch.Tensor] = None

    def get(self, problem: B.Problem, which: int, chunk: int = 0) -> torch.Tensor:
        n = B.ptycho_workspace_bytes([problem], which, chunk)
        if self.buf is None or self.buf.numel() < n or self.buf.device != problem.object.device:
            self.buf = torch.empty(n, dtype=torch.uint8, device=problem.object.device)
        return self.buf


_WS = _Workspace()


class PtychoLossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, obj, probe, pos, sigma, background, ratio, measured, mask, resample, pads,
                kind, eps, scale, chunk, reg):
        prob = B.Problem(object=obj.detach().contiguous(), probe=probe.detach().contiguous(),
                         pos=pos.detach().contiguous(), pads=_pads_of(pads, ratio),
                         measured=measured.contiguous(),
                         sigma=None if sigma is None else sigma.detach().contiguous(),
                         background=None if background is None else background.detach().contiguous(),
                         mask=mask, resample=resample)
        ng = ctx.needs_input_grad
        need = (ng[0], ng[1], ng[2], sigma is not None and ng[3],
                background is not None and ng[4], ratio is not None and ng[5])
        g = _zeros_like_grads(prob, need)
        ws = _WS.get(prob, 1, chunk)
        B.ptycho_loss_grad([prob], [g], kind=kind, eps=eps, scale=scale, workspace=ws, **reg)
        ctx.save_for_backward(*(g[k] for k in _KEYS if k in g))
        ctx.have = tuple(k in g for k in _KEYS)
        ctx.ratio_like = None if ratio is None else (ratio.device, ratio.dtype)
        return g["loss"][0]

    @staticmethod
    def backward(ctx, gout):
        saved = list(ctx.saved_tensors)
        out = [saved.pop(0) * gout if have else None for have in ctx.have]
        if out[5] is not None:  # the ratios may be host data
            out[5] = out[5].to(device=ctx.ratio_like[0], dtype=ctx.ratio_like[1])
        return tuple(out) + (None,) * 9


def ptycho_loss(obj, probe, pos, pads, measured, sigma=None, background=None, mask=None,
                resample=None, kind: int = B.LOSS_AMPLITUDE, eps: float = 1e-6,
                scale: float = 1.0, chunk: int = 0, ratio: Optional[torch.Tensor] = None,
                **reg) -> torch.Tensor:
    """Scalar loss, differentiable w.r.t. obj, probe, pos, sigma, background and
    ``ratio`` (a tensor of exact sampling ratios alpha_l that replaces ``pads``;
    alpha_l is proportional to the propagation distance z).  ``reg``:
    noise_var (mixed-noise loss), l1, tv, tv_eps (amplitude regularisers)."""
    return PtychoLossFn.apply(obj, probe, pos, sigma, background, ratio, measured, mask,
                              resample, tuple(pads), int(kind), float(eps), float(scale),
                              int(chunk), dict(reg))


class PtychoForwardFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, obj, probe, pos, sigma, background, ratio, pads, mask, resample, chunk):
        prob = B.Problem(object=obj.detach().contiguous(), probe=probe.detach().contiguous(),
                         pos=pos.detach().contiguous(), pads=_pads_of(pads, ratio),
                         sigma=None if sigma is None else sigma.detach().contiguous(),
                         background=None if background is None else background.detach().contiguous(),
                         mask=mask, resample=resample)
        out = torch.empty(prob.K, prob.N, prob.N, device=obj.device)
        ws = _WS.get(prob, 0, chunk)
        B.ptycho_forward([prob], [out], ws)
        ctx.prob = prob
        ctx.chunk = chunk
        ng = ctx.needs_input_grad
        ctx.need = (ng[0], ng[1], ng[2], sigma is not None and ng[3],
                    background is not None and ng[4], ratio is not None and ng[5])
        ctx.ratio_like = None if ratio is None else (ratio.device, ratio.dtype)
        return out

    @staticmethod
    def backward(ctx, gout):
        prob = ctx.prob
        prob.measured = gout.contiguous().float()
        g = _zeros_like_grads(prob, ctx.need)
        ws = _WS.get(prob, 1, ctx.chunk)
        B.ptycho_loss_grad([prob], [g], kind=B.LOSS_VJP, eps=0.0, scale=1.0, workspace=ws)
        prob.measured = None
        gr = g.get("g_ratio")
        if gr is not None:
            gr = gr.to(device=ctx.ratio_like[0], dtype=ctx.ratio_like[1])
        return (g.get("g_object"), g.get("g_probe"), g.get("g_pos"), g.get("g_sigma"),
                g.get("g_background"), gr, None, None, None, None)


def ptycho_forward(obj, probe, pos, pads, sigma=None, background=None, mask=None, resample=None,
                   chunk: int = 0, ratio: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Predicted patterns I'_k [K][N][N], differentiable w.r.t. obj, probe,
    pos, sigma, background and ``ratio`` (exact sampling ratios replacing
    ``pads``)."""
    return PtychoForwardFn.apply(obj, probe, pos, sigma, background, ratio, tuple(pads), mask,
                                 resample, int(chunk))
