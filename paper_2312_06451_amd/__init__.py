"""MI355X (gfx950) QAOA statevector library: Python side of libqaoa.so.

Every step of the evolution runs in the HIP kernels of ``csrc/``; this package marshals
arguments through the C ABI (``_lib``), wraps handles in small classes (``api``) and offers a
``torch.autograd.Function`` for d<C>/d(beta, gamma) (``autograd``). PyTorch is used only for
device memory (optional initial states, state outputs) and the current stream.
"""
from ._lib import QAOA_FP32, QAOA_FP64, QAOAError, lib  # noqa: F401
from .api import (Context, Mixer, Problem, angle_opts, basinhopping, expect, expect_batched, expect_grad,  # noqa: F401
                  expect_grad_batched, expect_grad_pairs, expect_pairs, find_angles, find_angles_multi,
                  find_angles_random, minimize, state)
