"""torch.autograd hook for the reflection loss of a 1D plasma profile.

RLoss.apply(wp2, problem, xref, steps) returns L = sum_f |R(f)|^2 with
R = (X - xref)/xref the reflection at probe 0 after `steps` steps, as a 0-d
tensor; its backward returns grad_output * dL/d(wp2) from the library's
discrete adjoint (sqrt(T) checkpoints).  The forward run stores the
checkpoints the backward recomputes from; torch only carries the tensors.
"""
from __future__ import annotations

import numpy as np
import torch

from .plasma import FdtdPlasma
from .workloads import Problem1D


class RLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, wp2: torch.Tensor, problem: Problem1D, xref: np.ndarray, steps: int,
                precision: str = "f32", probe: int = 0):
        p = problem.copy(wp2=wp2.detach().to("cpu", torch.float64).numpy().copy())
        h = FdtdPlasma(p, precision=precision, exec="tiled", checkpoint=steps)
        h.run(steps)
        loss = h.loss_r2(np.asarray(xref).reshape(1, -1), probe)[0]
        ctx.h, ctx.steps, ctx.xref, ctx.probe = h, steps, xref, probe
        ctx.wp2_meta = (wp2.dtype, wp2.device)
        return torch.tensor(loss, dtype=torch.float64, device=wp2.device)

    @staticmethod
    def backward(ctx, grad_out):
        h = ctx.h
        _, g = h.grad_r2(ctx.steps, np.asarray(ctx.xref).reshape(1, -1), ctx.probe)
        h.close()
        dtype, device = ctx.wp2_meta
        gt = torch.from_numpy(g).to(device=device, dtype=dtype)
        return grad_out.to(dtype) * gt, None, None, None, None, None


def reflection_loss(wp2: torch.Tensor, problem: Problem1D, xref, steps: int,
                    precision: str = "f32", probe: int = 0) -> torch.Tensor:
    return RLoss.apply(wp2, problem, xref, steps, precision, probe)
