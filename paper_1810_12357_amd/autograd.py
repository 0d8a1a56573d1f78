"""torch.autograd.Function over the library's recorded advance and adjoint.

Forward: write per-system K and G into the parameters, write T^0, run
``l2t_advance_recorded`` (FP32C sub-steps, checkpoints every ``ckpt_every``),
read T^N.  Backward: ``l2t_adjoint`` (hand-written reverse sub-step kernel with
checkpointed recomputation) returns dL/dT^0, dL/dK and dL/dG.  Marshalling
only; all arithmetic runs in the HIP library.
"""
from __future__ import annotations

import torch

from . import l2t as L


class L2TAdvance(torch.autograd.Function):
    """T^N = advance(T^0; K, g) for every system of a ``l2t.Context``.

    T0: float64 tensor on the GPU with all systems' atoms concatenated in
    caller order; K, g: float64 tensors of shape (n_systems,).
    """

    @staticmethod
    def forward(ctx, T0, K, g, context: "L.Context", n_substeps: int, ckpt_every: int):
        h = context.h
        sizes = [s.n for s in context.systems]
        Kc = K.detach().double().cpu().numpy()
        gc = g.detach().double().cpu().numpy()
        off = 0
        T0d = T0.detach().contiguous()
        for s, sy in enumerate(context.systems):
            p = dict(sy.params, K=float(Kc[s]), g=float(gc[s]))
            L.l2t_set_params(h, s, p)
            L.l2t_set_field(h, s, L.L2T_FIELD_TE, T0d[off:off + sizes[s]])
            off += sizes[s]
        L.l2t_advance_recorded(h, int(n_substeps), int(ckpt_every))
        # the context keeps one recording: a later recorded forward replaces it
        gen = getattr(context, "_recording", 0) + 1
        context._recording = gen
        TN = torch.empty_like(T0d)
        off = 0
        for s in range(len(sizes)):
            L.l2t_get_field(h, s, L.L2T_FIELD_TE, TN[off:off + sizes[s]])
            off += sizes[s]
        ctx.context = context
        ctx.n_sys = len(sizes)
        ctx.recording = gen
        return TN

    @staticmethod
    def backward(ctx, grad_TN):
        if getattr(ctx.context, "_recording", None) != ctx.recording:
            raise RuntimeError("this forward's recording was replaced by a later recorded "
                               "advance of the same context; run backward before the next forward")
        w = grad_TN.detach().double().contiguous()
        dT0 = torch.empty_like(w)
        dK, dg = L.l2t_adjoint(ctx.context.h, w, ctx.n_sys, dL_dT0=dT0)
        dev = grad_TN.device
        return (dT0, torch.from_numpy(dK).to(dev), torch.from_numpy(dg).to(dev), None, None, None)


def advance(T0, K, g, context, n_substeps: int, ckpt_every: int = 100):
    return L2TAdvance.apply(T0, K, g, context, n_substeps, ckpt_every)
