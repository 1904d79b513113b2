"""torch.autograd binding of an HH population (Methods, "Gradient learning
support": the neuron as a module stepped over time and differentiated;
"Engineering optimization": manual gradients with re-computation).

Forward runs hh_step_n over the dense input with checkpoints every
ckpt_every steps and the level output; backward runs hh_backward, the
adjoint with the surrogate derivative of the level.  Both are libhh
kernels; this module only allocates the buffers and routes the gradients.
"""
from __future__ import annotations

import torch

from . import hh


class HHFunction(torch.autograd.Function):
    """r = HHFunction.apply(I, x0, cm, model, ckpt_every=50, beta=0.2)

    I: [T][n] dense input current (float32, device); x0: [n_state][n]
    initial state (not modified); cm: the per-neuron capacitance tensor [N]
    the model was built with, or None for the model's scalar C; model: an
    hh.Model without synapses.  Returns r [n] = (1/T) sum_t H(V_t - v_th),
    the fraction of steps at or above threshold.  Gradients: dL/dI [T][n],
    dL/dx0 [n_state][n] and dL/dcm [N] (summed over the batch), with
    dH/dV replaced by beta s (1 - s), s = sigmoid(beta (V - v_th))."""

    @staticmethod
    def forward(ctx, I, x0, cm, model, ckpt_every=50, beta=0.2):
        T, n = I.shape
        Ic = I.detach().contiguous()
        st = x0.detach().clone()
        nck = (T + ckpt_every - 1) // ckpt_every
        ck = torch.empty((nck, model.n_state, n), dtype=torch.float32, device=I.device)
        lv = torch.zeros(n, dtype=torch.float32, device=I.device)
        model.step_n(st, T, 0, i_dense=Ic, ckpt=ck, ckpt_every=ckpt_every, level=lv)
        ctx.save_for_backward(ck, Ic)
        ctx.model, ctx.ckpt_every, ctx.beta, ctx.has_cm = model, ckpt_every, beta, cm is not None
        return hh.level_rate(lv, T, torch.empty_like(lv))

    @staticmethod
    def backward(ctx, dr):
        ck, Ic = ctx.saved_tensors
        M = ctx.model
        T, n = Ic.shape
        dI = torch.zeros_like(Ic)
        dx0 = torch.zeros((M.n_state, n), dtype=torch.float32, device=Ic.device)
        dC = torch.zeros(M.N, dtype=torch.float32, device=Ic.device) if ctx.has_cm else None
        M.backward(ck, ctx.ckpt_every, Ic, T, dI, dL_dlevel=dr.detach().float().contiguous(),
                   beta=ctx.beta, dCm=dC, dx0=dx0)
        status, bad = M.check()
        if status != 0:
            raise RuntimeError("adjoint failed: status %d (neuron %d)" % (status, bad))
        return dI, dx0, dC, None, None, None
