"""torch.autograd bridge: receiver traces as a differentiable function of the
per-node permittivity and the source amplitudes.

Forward: one library run from zero fields with soft sources and receivers,
checkpointing the state every ceil(sqrt(T)) steps.  Backward: the library's
discrete adjoint (segment recomputation from the checkpoints, reverse sweep
with the transposed operators), returning dJ/deps_r and dJ/da in FP64.
"""
import math

import numpy as np
import torch


class AdjointProblem:
    """Fixed parts of a differentiable run: solver, T, sources, receivers."""

    def __init__(self, solver, T, src_nodes, src_wave, rcv_nodes, ckpt_every=None):
        self.solver = solver
        self.T = int(T)
        self.src_nodes = np.asarray(src_nodes)
        self.src_wave = np.asarray(src_wave, dtype=np.float64)
        self.rcv_nodes = np.asarray(rcv_nodes)
        self.ckpt_every = int(ckpt_every or math.ceil(math.sqrt(self.T)))


class MaxwellFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_r, amp, prob):
        s = prob.solver
        N = s.N
        st = s.state(np.zeros((N, s.fe)), np.zeros((N, s.fh)), eps_r=eps_r.detach().double().cpu().numpy())
        amp_np = amp.detach().double().cpu().numpy()
        out = s.run(st, prob.T, src=(prob.src_nodes, amp_np, prob.src_wave), rcv=prob.rcv_nodes,
                    ckpt_every=prob.ckpt_every)
        ctx.prob = prob
        ctx.st = st
        ctx.amp = amp_np
        ctx.ckpt = out["ckpt"]
        ctx.eps_meta = (eps_r.dtype, eps_r.device)
        ctx.amp_meta = (amp.dtype, amp.device)
        return out["traces"].clone()

    @staticmethod
    def backward(ctx, grad_traces):
        prob = ctx.prob
        s = prob.solver
        g_eps, g_amp = s.adjoint(ctx.st, prob.T, ctx.ckpt, prob.ckpt_every, grad_traces.detach(),
                                 src=(prob.src_nodes, ctx.amp, prob.src_wave), rcv=prob.rcv_nodes)
        ge = torch.as_tensor(g_eps).to(dtype=ctx.eps_meta[0], device=ctx.eps_meta[1])
        ga = torch.as_tensor(g_amp).to(dtype=ctx.amp_meta[0], device=ctx.amp_meta[1])
        return ge, ga, None
