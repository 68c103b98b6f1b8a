"""``torch.autograd.Function`` for <C>(beta, gamma): forward and the library's reverse sweep.

The forward calls ``qaoa_expect_grad`` when the angles need a gradient (the reverse sweep
runs on the device right after the forward evolution, no per-layer states are stored) and
keeps the gradient; ``backward`` scales it by the incoming gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from .api import Mixer, Problem, _stream
from ._lib import QAOA_FP32


class QAOAExpectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, angles: torch.Tensor, problem: Problem, mixer: Mixer, precision: int = QAOA_FP32):
        a = angles.detach().to("cpu", torch.float64).contiguous().numpy()
        p = a.size // mixer.angles_per_layer
        if ctx.needs_input_grad[0]:
            e, g = _lib.qaoa_expect_grad(problem.handle, mixer.handle, p, a, 0, precision, _stream(None))
            ctx.save_for_backward(torch.from_numpy(g).to(angles.device, angles.dtype))
        else:
            e = _lib.qaoa_expect(problem.handle, mixer.handle, p, a, 0, precision, _stream(None))
        return torch.tensor(e, dtype=angles.dtype, device=angles.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None


def qaoa_expectation(angles: torch.Tensor, problem: Problem, mixer: Mixer, precision: int = QAOA_FP32):
    return QAOAExpectation.apply(angles, problem, mixer, precision)
