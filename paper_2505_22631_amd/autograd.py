"""torch.autograd.Function over the schedule adjoint kernels.

RelaxedCut.apply(K, Ks, sigma, problem, theta0, seeds, q, dt, checkpoint_every,
step0) returns the relaxed cut sum_{i<j} w_ij (1 - cos(th_i - th_j)) / 2
(w = -J) at the final phases of the fixed-noise trajectory, summed over
replicas and instances, as an FP64 scalar tensor.  Its backward runs the
adjoint kernel from the checkpoints the forward kept, so K, Ks and sigma
(FP32 [steps] on the GPU) receive exact trajectory gradients.
"""
from __future__ import annotations

import torch

from . import oim_adjoint_backward, oim_adjoint_checkpoint_words, oim_adjoint_forward


class RelaxedCut(torch.autograd.Function):
    @staticmethod
    def forward(ctx, K, Ks, sigma, problem, theta0, seeds, q, dt, checkpoint_every, step0=0):
        R = int(theta0.shape[0])
        steps = int(K.shape[0])
        words = oim_adjoint_checkpoint_words(problem.handle, q=q, R=R, steps=steps, dt=dt,
                                             checkpoint_every=checkpoint_every)
        ckpt = torch.empty(max(words, 1), dtype=torch.uint32, device=theta0.device)
        RI = R * int(problem.info["n_instances"])
        loss = torch.empty(RI, dtype=torch.float64, device=theta0.device)
        oim_adjoint_forward(problem.handle, problem.n, theta0, K, Ks, sigma, seeds, ckpt, q=q,
                            dt=dt, checkpoint_every=checkpoint_every, step0=step0, loss=loss)
        ctx.save_for_backward(K, Ks, sigma, seeds, ckpt)
        ctx.cfg = (problem, R, q, dt, checkpoint_every, step0)
        return loss.sum()

    @staticmethod
    def backward(ctx, grad_out):
        K, Ks, sigma, seeds, ckpt = ctx.saved_tensors
        problem, R, q, dt, C, step0 = ctx.cfg
        steps = int(K.shape[0])
        dev = K.device
        gK, gKs, gS = (torch.empty(steps, dtype=torch.float64, device=dev) for _ in range(3))
        oim_adjoint_backward(problem.handle, R, K, Ks, sigma, seeds, ckpt, gK, gKs, gS, q=q,
                             dt=dt, checkpoint_every=C, step0=step0)
        g = grad_out.to(torch.float64)
        return ((g * gK).to(K.dtype), (g * gKs).to(Ks.dtype), (g * gS).to(sigma.dtype),
                None, None, None, None, None, None, None)


def relaxed_cut(problem, theta0, K, Ks, sigma, seeds, *, q, dt, checkpoint_every=64, step0=0):
    return RelaxedCut.apply(K, Ks, sigma, problem, theta0, seeds, q, dt, checkpoint_every, step0)
