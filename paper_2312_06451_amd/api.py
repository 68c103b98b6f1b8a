"""Handle classes over the C ABI (argument marshalling only)."""
from __future__ import annotations

import weakref

import numpy as np

from . import _lib
from ._lib import QAOA_FP32, QAOA_FP64


def _stream(stream):
    """HIP stream handle for a call: an int, a torch stream, or torch's current stream."""
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return int(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Context:
    """One HIP device and the scratch vectors evaluations reuse."""

    def __init__(self, device: int = 0):
        self.handle = _lib.qaoa_ctx_create(device)
        self.device = device
        self._children = weakref.WeakSet()

    def set_autotune(self, enable: bool = True):
        """Turn the tile-pass plan tuner on or off (``qaoa_ctx_set_autotune``)."""
        _lib.qaoa_ctx_set_autotune(self.handle, enable)

    def plans(self) -> str:
        """The chosen tile-pass plans as text (``qaoa_plans_text``)."""
        return _lib.qaoa_plans_text(self.handle)

    def save_plans(self, path: str):
        _lib.qaoa_plans_save(self.handle, path)

    def load_plans(self, path: str):
        _lib.qaoa_plans_load(self.handle, path)

    def close(self):
        """Destroy the context; problems and mixers still open on it are closed first."""
        if self.handle:
            for ch in list(self._children):
                ch.close()
            _lib.qaoa_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Cost diagonal C(x) over the feasible states, tabulated on the device: a (weighted)
    MaxCut instance (``Problem(ctx, n, u, v, w)``, ``Problem.from_graph``) or any list of
    values (``Problem.from_values``)."""

    def __init__(self, ctx: Context, n: int, u=None, v=None, w=None, hamming_k: int = -1, stream=None,
                 _handle=None):
        self.ctx = ctx
        if _handle is None:
            _handle = _lib.qaoa_cost_table(ctx.handle, n, u, v, w, hamming_k, _stream(stream))
        self.handle = _handle
        ctx._children.add(self)
        info = _lib.qaoa_problem_info(self.handle)
        self.n = info["n"]
        self.hamming_k = info["hamming_k"]
        self.size = info["size"]
        self.max_value = info["max_value"]

    @classmethod
    def from_graph(cls, ctx: Context, g, hamming_k: int = -1, stream=None):
        return cls(ctx, g.n, g.u, g.v, g.w, hamming_k, stream)

    @classmethod
    def from_values(cls, ctx: Context, n: int, values, hamming_k: int = -1, stream=None):
        """C(x) = values[i] for the i-th feasible state (all 2^n strings, or the weight-k
        strings in increasing order)."""
        h = _lib.qaoa_problem_from_values(ctx.handle, n, hamming_k, values, _stream(stream))
        return cls(ctx, n, hamming_k=hamming_k, _handle=h)

    def table(self, stream=None) -> np.ndarray:
        return _lib.qaoa_problem_copy_table(self.handle, _stream(stream))

    @classmethod
    def degeneracies_of_graph(cls, ctx: Context, g, hamming_k: int = -1, stream=None):
        """MaxCut degeneracies counted on the device without a table (Grover mixer only)."""
        h = _lib.qaoa_cost_degeneracies(ctx.handle, g.n, g.u, g.v, g.w, hamming_k, _stream(stream))
        return cls(ctx, g.n, hamming_k=hamming_k, _handle=h)

    def degeneracies(self, stream=None):
        """(distinct values, how many feasible states take each)."""
        return _lib.qaoa_problem_degeneracies(self.handle, _stream(stream))

    def values(self, stream=None) -> np.ndarray:
        """C(x) over the feasible states as FP64."""
        return _lib.qaoa_problem_copy_values(self.handle, _stream(stream))

    def close(self):
        if self.handle:
            _lib.qaoa_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mixer:
    """H_M: ``Mixer.x(ctx, n)`` (sum of X_q), ``Mixer.clique(ctx, n, k)`` or
    ``Mixer.grover(ctx, n, hamming_k)`` (|psi0><psi0|)."""

    def __init__(self, ctx: Context, handle: int, kind: str, n: int, k: int = -1):
        self.ctx, self.handle, self.kind, self.n, self.k = ctx, handle, kind, n, k
        # angles per layer of an angle set: beta and gamma, or n betas and gamma (multi-angle)
        self.angles_per_layer = n + 1 if kind == "x_multiangle" else 2
        ctx._children.add(self)

    @classmethod
    def x(cls, ctx: Context, n: int):
        return cls(ctx, _lib.qaoa_mixer_x(ctx.handle, n), "x", n)

    @classmethod
    def ring(cls, ctx: Context, n: int, k: int, stream=None):
        return cls(ctx, _lib.qaoa_mixer_ring(ctx.handle, n, k, _stream(stream)), "ring", n, k)

    @classmethod
    def matrix(cls, ctx: Context, n: int, H, hamming_k: int = -1, stream=None):
        """Any real symmetric mixer matrix over the feasible states (eigendecomposed once)."""
        return cls(ctx, _lib.qaoa_mixer_matrix(ctx.handle, n, hamming_k, H, _stream(stream)), "matrix", n, hamming_k)

    @classmethod
    def from_eigen(cls, ctx: Context, n: int, V, D, hamming_k: int = -1, stream=None):
        """A mixer V diag(D) V^T from a stored eigendecomposition (no eigensolver)."""
        h = _lib.qaoa_mixer_from_eigen(ctx.handle, n, hamming_k, V, D, _stream(stream))
        return cls(ctx, h, "eigen", n, hamming_k)

    def eigen(self, stream=None):
        """(V, D) of a clique, ring or matrix mixer: eigenvectors as columns of V."""
        from math import comb
        N = (1 << self.n) if self.k < 0 else comb(self.n, self.k)
        return _lib.qaoa_mixer_eigen(self.handle, N, _stream(stream))

    @classmethod
    def x_orders(cls, ctx: Context, n: int, orders):
        """sum over k in orders of all k-body products of X (Eq. (2)); [1] is the transverse field."""
        return cls(ctx, _lib.qaoa_mixer_x_orders(ctx.handle, n, list(orders)), "x_orders", n)

    @classmethod
    def x_terms(cls, ctx: Context, n: int, masks, coefs):
        """sum_t coefs[t] prod_{i in masks[t]} X_i (at most 10 terms)."""
        return cls(ctx, _lib.qaoa_mixer_x_terms(ctx.handle, n, list(masks), list(coefs)), "x_terms", n)

    @classmethod
    def x_multiangle(cls, ctx: Context, n: int):
        """prod_q e^{-i beta_{k,q} X_q}: angle sets [beta_{1,0..n-1}, ..., beta_{p,0..n-1}, gamma_1..gamma_p]."""
        return cls(ctx, _lib.qaoa_mixer_x_multiangle(ctx.handle, n), "x_multiangle", n)

    def info(self) -> dict:
        return _lib.qaoa_mixer_info(self.handle)

    @classmethod
    def grover(cls, ctx: Context, n: int, hamming_k: int = -1):
        return cls(ctx, _lib.qaoa_mixer_grover(ctx.handle, n, hamming_k), "grover", n, hamming_k)

    @classmethod
    def clique(cls, ctx: Context, n: int, k: int, stream=None):
        return cls(ctx, _lib.qaoa_mixer_clique(ctx.handle, n, k, _stream(stream)), "clique", n, k)

    def close(self):
        if self.handle:
            _lib.qaoa_mixer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t):
    if t is None:
        return 0
    return int(t.data_ptr())


def expect(problem: Problem, mixer: Mixer, angles, psi0=None, precision: int = QAOA_FP32, stream=None) -> float:
    a = np.asarray(angles, dtype=np.float64).reshape(-1)
    return _lib.qaoa_expect(problem.handle, mixer.handle, a.size // mixer.angles_per_layer, a, _ptr(psi0), precision,
                            _stream(stream))


def expect_grad(problem: Problem, mixer: Mixer, angles, psi0=None, precision: int = QAOA_FP32, stream=None):
    a = np.asarray(angles, dtype=np.float64).reshape(-1)
    return _lib.qaoa_expect_grad(problem.handle, mixer.handle, a.size // mixer.angles_per_layer, a, _ptr(psi0),
                                 precision,
                                 _stream(stream))


def state(problem: Problem, mixer: Mixer, angles, out, psi0=None, precision: int = QAOA_FP32, stream=None):
    """Write psi_p into the device tensor ``out`` (complex64 / complex128, feasible-set length)."""
    a = np.asarray(angles, dtype=np.float64).reshape(-1)
    _lib.qaoa_state(problem.handle, mixer.handle, a.size // mixer.angles_per_layer, a, _ptr(out), _ptr(psi0), precision,
                    _stream(stream))
    return out


def expect_batched(problems, mixers, angles, precision: int = QAOA_FP32, stream=None):
    a = np.asarray(angles, dtype=np.float64)
    p = a.shape[-1] // mixers[0].angles_per_layer
    return _lib.qaoa_expect_batched([x.handle for x in problems], [m.handle for m in mixers], p, a,
                                    precision, _stream(stream), set_len=a.shape[-1])


def expect_grad_batched(problems, mixers, angles, precision: int = QAOA_FP32, stream=None):
    a = np.asarray(angles, dtype=np.float64)
    p = a.shape[-1] // mixers[0].angles_per_layer
    return _lib.qaoa_expect_grad_batched([x.handle for x in problems], [m.handle for m in mixers], p, a,
                                         precision, _stream(stream), set_len=a.shape[-1])


# ---------------------------------------------------------------- angle finding (Sec. 2.3)

def angle_opts(**kw):
    """qaoa_angle_opts with the library defaults, overridden by keyword (maximize, precision,
    max_iter, gtol, n_chains, n_hops, step, temperature, seed, max_sets_per_call)."""
    o = _lib.qaoa_angle_opts_default()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown angle-finding option {k!r}")
        setattr(o, k, v)
    return o


def minimize(problem: Problem, mixer: Mixer, starts, stream=None, **opts):
    """BFGS from every row of ``starts`` (n_starts x 2p) as one batch: (optima, <C>, steps)."""
    s = np.asarray(starts, dtype=np.float64)
    p = s.shape[-1] // 2
    return _lib.qaoa_minimize(problem.handle, mixer.handle, p, s, angle_opts(**opts), _stream(stream))


def basinhopping(problem: Problem, mixer: Mixer, x0, stream=None, **opts):
    """Basinhopping from ``x0`` (2p angles): (best angles, best <C>)."""
    a = np.asarray(x0, dtype=np.float64).reshape(-1)
    return _lib.qaoa_basinhopping(problem.handle, mixer.handle, a.size // 2, a, angle_opts(**opts),
                                  _stream(stream))


def find_angles(problem: Problem, mixer: Mixer, p: int, file=None, stream=None, **opts):
    """Iterative angle finding up to p rounds, resuming from / saving to ``file``:
    (list of per-round angle arrays, array of <C> per round)."""
    out, vals = _lib.qaoa_find_angles(problem.handle, mixer.handle, p, angle_opts(**opts), file,
                                      _stream(stream))
    return [out[r - 1, :2 * r].copy() for r in range(1, p + 1)], vals


def find_angles_multi(problems, mixers, p: int, files=None, stream=None, **opts):
    """find_angles for many instances at once (one launch per optimiser step for all of them):
    per instance, (list of per-round angle arrays, array of <C> per round)."""
    out, vals = _lib.qaoa_find_angles_multi([x.handle for x in problems], [m.handle for m in mixers], p,
                                            angle_opts(**opts), files, _stream(stream))
    return [([out[i, r - 1, :2 * r].copy() for r in range(1, p + 1)], vals[i]) for i in range(len(problems))]


def expect_pairs(problems, mixers, angles, precision: int = QAOA_FP32, stream=None):
    """<C> of pair i = (problems[i], mixers[i], angles[i])."""
    a = np.asarray(angles, dtype=np.float64)
    return _lib.qaoa_expect_pairs([x.handle for x in problems], [m.handle for m in mixers],
                                  a.shape[-1] // mixers[0].angles_per_layer, a, precision, _stream(stream),
                                  set_len=a.shape[-1])


def expect_grad_pairs(problems, mixers, angles, precision: int = QAOA_FP32, stream=None):
    a = np.asarray(angles, dtype=np.float64)
    return _lib.qaoa_expect_grad_pairs([x.handle for x in problems], [m.handle for m in mixers],
                                       a.shape[-1] // mixers[0].angles_per_layer, a, precision, _stream(stream),
                                       set_len=a.shape[-1])


def find_angles_random(problem: Problem, mixer: Mixer, p: int, restarts: int = 100, stream=None, **opts):
    """Random local-minima search: (best angles, best <C>, <C> of every restart)."""
    return _lib.qaoa_find_angles_random(problem.handle, mixer.handle, p, restarts, angle_opts(**opts),
                                        _stream(stream))
