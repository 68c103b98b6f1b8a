"""ctypes binding of libqaoa.so: the C ABI of include/qaoa.h, same names, marshalling only.

The library must have been built (``python paper_2312_06451_amd/build.py`` or
``__graft_entry__.build()``). There is no fallback: if it is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqaoa.so")

QAOA_OK = 0
QAOA_ERR_INVALID_ARG = -1
QAOA_ERR_OUT_OF_MEMORY = -2
QAOA_ERR_HIP = -3
QAOA_ERR_UNSUPPORTED = -4
QAOA_FP32 = 0
QAOA_FP64 = 1

EXPORTED = [
    "qaoa_ctx_create", "qaoa_ctx_destroy", "qaoa_cost_table", "qaoa_problem_copy_table",
    "qaoa_problem_info", "qaoa_problem_destroy", "qaoa_mixer_x", "qaoa_mixer_clique",
    "qaoa_mixer_destroy", "qaoa_expect", "qaoa_expect_grad", "qaoa_state", "qaoa_expect_batched",
    "qaoa_expect_grad_batched", "qaoa_status_string", "qaoa_last_error", "qaoa_profile_enable",
    "qaoa_profile_read", "qaoa_problem_from_values", "qaoa_problem_copy_values", "qaoa_mixer_grover",
    "qaoa_cost_degeneracies", "qaoa_problem_degeneracies", "qaoa_mixer_ring", "qaoa_mixer_matrix",
    "qaoa_mixer_eigen", "qaoa_mixer_from_eigen", "qaoa_angle_opts_default", "qaoa_minimize",
    "qaoa_basinhopping", "qaoa_find_angles", "qaoa_find_angles_random", "qaoa_find_angles_multi",
    "qaoa_expect_pairs", "qaoa_expect_grad_pairs", "qaoa_mixer_x_orders", "qaoa_mixer_x_terms",
    "qaoa_mixer_x_multiangle", "qaoa_mixer_info", "qaoa_stream_copy",
    "qaoa_expect_grad_pairs_noalloc", "qaoa_ctx_set_autotune", "qaoa_plans_text", "qaoa_plans_save",
    "qaoa_plans_load",
]
KERNEL_CLASSES = {"fwd_pass": 0, "rev_pass": 1, "small": 2, "dense": 3, "other": 4, "grover": 5,
                  "count_states": 6, "xmix": 7}


class qaoa_angle_opts(ctypes.Structure):
    """Mirror of struct qaoa_angle_opts (include/qaoa.h)."""
    _fields_ = [("maximize", ctypes.c_int), ("precision", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("gtol", ctypes.c_double), ("n_chains", ctypes.c_int), ("n_hops", ctypes.c_int),
                ("step", ctypes.c_double), ("temperature", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("max_sets_per_call", ctypes.c_int)]


class QAOAError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


_lib = None

c_int, c_void_p, c_double, c_size_t = ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_size_t
c_int64 = ctypes.c_int64
P = ctypes.POINTER


def lib() -> ctypes.CDLL:
    """Load libqaoa.so (raises OSError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch enumerates HIP devices on its own first use; if this library initialises the HIP
    # runtime before that, torch later reports no GPU. Let torch look first when present.
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it first (paper_2312_06451_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    i32p = P(ctypes.c_int32)
    L.qaoa_ctx_create.argtypes = [c_int, P(c_void_p)]
    L.qaoa_ctx_destroy.argtypes = [c_void_p]
    L.qaoa_cost_table.argtypes = [c_void_p, c_int, c_int, i32p, i32p, i32p, c_int, P(c_void_p), c_void_p]
    L.qaoa_problem_copy_table.argtypes = [c_void_p, P(c_int64), c_size_t, c_void_p]
    L.qaoa_problem_from_values.argtypes = [c_void_p, c_int, c_int, P(c_double), c_size_t, P(c_void_p), c_void_p]
    L.qaoa_problem_copy_values.argtypes = [c_void_p, P(c_double), c_size_t, c_void_p]
    L.qaoa_problem_info.argtypes = [c_void_p, P(c_int), P(c_int), P(c_int64), P(c_int64)]
    L.qaoa_problem_destroy.argtypes = [c_void_p]
    L.qaoa_mixer_x.argtypes = [c_void_p, c_int, P(c_void_p)]
    L.qaoa_mixer_clique.argtypes = [c_void_p, c_int, c_int, P(c_void_p), c_void_p]
    L.qaoa_mixer_grover.argtypes = [c_void_p, c_int, c_int, P(c_void_p)]
    L.qaoa_mixer_ring.argtypes = [c_void_p, c_int, c_int, P(c_void_p), c_void_p]
    L.qaoa_mixer_x_orders.argtypes = [c_void_p, c_int, P(c_int), c_int, P(c_void_p)]
    L.qaoa_mixer_x_terms.argtypes = [c_void_p, c_int, P(ctypes.c_uint64), P(c_double), c_int, P(c_void_p)]
    L.qaoa_mixer_x_multiangle.argtypes = [c_void_p, c_int, P(c_void_p)]
    L.qaoa_mixer_info.argtypes = [c_void_p, P(c_int), P(c_int), P(c_int)]
    L.qaoa_mixer_eigen.argtypes = [c_void_p, P(c_double), P(c_double), c_size_t, c_void_p]
    L.qaoa_mixer_from_eigen.argtypes = [c_void_p, c_int, c_int, P(c_double), P(c_double), P(c_void_p), c_void_p]
    L.qaoa_mixer_matrix.argtypes = [c_void_p, c_int, c_int, P(c_double), P(c_void_p), c_void_p]
    L.qaoa_cost_degeneracies.argtypes = [c_void_p, c_int, c_int, i32p, i32p, i32p, c_int, P(c_void_p), c_void_p]
    L.qaoa_problem_degeneracies.argtypes = [c_void_p, P(c_double), P(c_int64), c_size_t, P(c_size_t), c_void_p]
    L.qaoa_mixer_destroy.argtypes = [c_void_p]
    L.qaoa_expect.argtypes = [c_void_p, c_void_p, c_int, P(c_double), c_void_p, c_int, P(c_double), c_void_p]
    L.qaoa_expect_grad.argtypes = [c_void_p, c_void_p, c_int, P(c_double), c_void_p, c_int,
                                   P(c_double), P(c_double), c_void_p]
    L.qaoa_state.argtypes = [c_void_p, c_void_p, c_int, P(c_double), c_void_p, c_int, c_void_p, c_void_p]
    L.qaoa_expect_batched.argtypes = [P(c_void_p), P(c_void_p), c_int, c_int, c_int, P(c_double), c_int,
                                      P(c_double), c_void_p]
    L.qaoa_expect_grad_batched.argtypes = [P(c_void_p), P(c_void_p), c_int, c_int, c_int, P(c_double),
                                           c_int, P(c_double), P(c_double), c_void_p]
    L.qaoa_profile_enable.argtypes = [c_void_p, c_int]
    L.qaoa_profile_read.argtypes = [c_void_p, c_int, P(c_int64), P(c_double), P(c_double), P(c_double)]
    L.qaoa_stream_copy.argtypes = [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.qaoa_ctx_set_autotune.argtypes = [c_void_p, c_int]
    L.qaoa_plans_text.argtypes = [c_void_p, ctypes.c_char_p, c_size_t, P(c_size_t)]
    L.qaoa_plans_save.argtypes = [c_void_p, ctypes.c_char_p]
    L.qaoa_plans_load.argtypes = [c_void_p, ctypes.c_char_p]
    opts_p = P(qaoa_angle_opts)
    L.qaoa_angle_opts_default.argtypes = [opts_p]
    L.qaoa_minimize.argtypes = [c_void_p, c_void_p, c_int, c_int, P(c_double), P(c_double), P(c_int), opts_p,
                                c_void_p]
    L.qaoa_basinhopping.argtypes = [c_void_p, c_void_p, c_int, P(c_double), opts_p, P(c_double), P(c_double),
                                    c_void_p]
    L.qaoa_find_angles.argtypes = [c_void_p, c_void_p, c_int, opts_p, ctypes.c_char_p, P(c_double), P(c_double),
                                   c_void_p]
    L.qaoa_find_angles_multi.argtypes = [P(c_void_p), P(c_void_p), c_int, c_int, opts_p, P(ctypes.c_char_p),
                                         P(c_double), P(c_double), c_void_p]
    L.qaoa_expect_pairs.argtypes = [P(c_void_p), P(c_void_p), c_int, c_int, P(c_double), c_int, P(c_double),
                                    c_void_p]
    L.qaoa_expect_grad_pairs.argtypes = [P(c_void_p), P(c_void_p), c_int, c_int, P(c_double), c_int,
                                         P(c_double), P(c_double), c_void_p]
    L.qaoa_expect_grad_pairs_noalloc.argtypes = [P(c_void_p), P(c_void_p), c_int, c_int, P(c_double), c_int,
                                                 P(c_double), P(c_double), c_void_p]
    L.qaoa_find_angles_random.argtypes = [c_void_p, c_void_p, c_int, c_int, opts_p, P(c_double), P(c_double),
                                          P(c_double), c_void_p]
    L.qaoa_status_string.argtypes = [c_int]
    L.qaoa_status_string.restype = ctypes.c_char_p
    L.qaoa_last_error.argtypes = []
    L.qaoa_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("qaoa_status_string", "qaoa_last_error", "qaoa_angle_opts_default"):
            getattr(L, name).restype = c_int
    L.qaoa_angle_opts_default.restype = None
    _lib = L
    return L


def check(status: int, where: str) -> None:
    if status != QAOA_OK:
        L = lib()
        detail = L.qaoa_last_error().decode(errors="replace")
        raise QAOAError(status, where, f"{L.qaoa_status_string(status).decode()}: {detail}")


# ---------------------------------------------------------------- same-name wrappers

def qaoa_ctx_create(hip_device: int) -> int:
    out = c_void_p()
    check(lib().qaoa_ctx_create(hip_device, ctypes.byref(out)), "qaoa_ctx_create")
    return out.value


def qaoa_ctx_destroy(ctx: int) -> None:
    check(lib().qaoa_ctx_destroy(ctx), "qaoa_ctx_destroy")


def _i32(a):
    import numpy as np
    arr = np.ascontiguousarray(a, dtype=np.int32)
    return arr, arr.ctypes.data_as(P(ctypes.c_int32))


def qaoa_cost_table(ctx: int, n: int, u, v, w=None, hamming_k: int = -1, stream: int = 0) -> int:
    ua, up = _i32(u)
    va, vp = _i32(v)
    if w is None:
        wp = None
    else:
        wa, wp = _i32(w)
    out = c_void_p()
    check(lib().qaoa_cost_table(ctx, n, int(ua.size), up, vp, wp, hamming_k, ctypes.byref(out), stream),
          "qaoa_cost_table")
    return out.value


def qaoa_problem_from_values(ctx: int, n: int, hamming_k: int, values, stream: int = 0) -> int:
    import numpy as np
    va = np.ascontiguousarray(values, dtype=np.float64)
    out = c_void_p()
    check(lib().qaoa_problem_from_values(ctx, n, hamming_k, va.ctypes.data_as(P(c_double)), va.size,
                                         ctypes.byref(out), stream), "qaoa_problem_from_values")
    return out.value


def qaoa_problem_copy_values(prob: int, stream: int = 0):
    import numpy as np
    info = qaoa_problem_info(prob)
    out = np.zeros(info["size"], dtype=np.float64)
    check(lib().qaoa_problem_copy_values(prob, out.ctypes.data_as(P(c_double)), out.size, stream),
          "qaoa_problem_copy_values")
    return out


def qaoa_problem_copy_table(prob: int, stream: int = 0):
    import numpy as np
    info = qaoa_problem_info(prob)
    out = np.zeros(info["size"], dtype=np.int64)
    check(lib().qaoa_problem_copy_table(prob, out.ctypes.data_as(P(c_int64)), out.size, stream),
          "qaoa_problem_copy_table")
    return out


def qaoa_problem_info(prob: int) -> dict:
    n, k, size, mx = c_int(), c_int(), c_int64(), c_int64()
    check(lib().qaoa_problem_info(prob, ctypes.byref(n), ctypes.byref(k), ctypes.byref(size),
                                  ctypes.byref(mx)), "qaoa_problem_info")
    return {"n": n.value, "hamming_k": k.value, "size": size.value, "max_value": mx.value}


def qaoa_problem_destroy(prob: int) -> None:
    check(lib().qaoa_problem_destroy(prob), "qaoa_problem_destroy")


def qaoa_mixer_x(ctx: int, n: int) -> int:
    out = c_void_p()
    check(lib().qaoa_mixer_x(ctx, n, ctypes.byref(out)), "qaoa_mixer_x")
    return out.value


def qaoa_mixer_ring(ctx: int, n: int, k: int, stream: int = 0) -> int:
    out = c_void_p()
    check(lib().qaoa_mixer_ring(ctx, n, k, ctypes.byref(out), stream), "qaoa_mixer_ring")
    return out.value


def qaoa_mixer_matrix(ctx: int, n: int, hamming_k: int, matrix, stream: int = 0) -> int:
    import numpy as np
    m = np.ascontiguousarray(matrix, dtype=np.float64)
    out = c_void_p()
    check(lib().qaoa_mixer_matrix(ctx, n, hamming_k, m.ctypes.data_as(P(c_double)), ctypes.byref(out), stream),
          "qaoa_mixer_matrix")
    return out.value


def qaoa_mixer_eigen(mix: int, N: int, stream: int = 0):
    """(V, D): eigenvectors as columns of V (N x N) and eigenvalues."""
    import numpy as np
    Vt = np.zeros((N, N), dtype=np.float64)   # row j = eigenvector j
    D = np.zeros(N, dtype=np.float64)
    check(lib().qaoa_mixer_eigen(mix, Vt.ctypes.data_as(P(c_double)), D.ctypes.data_as(P(c_double)), N, stream),
          "qaoa_mixer_eigen")
    return Vt.T.copy(), D


def qaoa_mixer_from_eigen(ctx: int, n: int, hamming_k: int, V, D, stream: int = 0) -> int:
    import numpy as np
    Vt = np.ascontiguousarray(np.asarray(V, dtype=np.float64).T)   # row j = eigenvector j
    Da = np.ascontiguousarray(D, dtype=np.float64)
    out = c_void_p()
    check(lib().qaoa_mixer_from_eigen(ctx, n, hamming_k, Vt.ctypes.data_as(P(c_double)), Da.ctypes.data_as(P(c_double)),
                                      ctypes.byref(out), stream), "qaoa_mixer_from_eigen")
    return out.value


def qaoa_mixer_x_orders(ctx: int, n: int, orders) -> int:
    o = (c_int * len(orders))(*[int(x) for x in orders])
    out = c_void_p()
    check(lib().qaoa_mixer_x_orders(ctx, n, o, len(orders), ctypes.byref(out)), "qaoa_mixer_x_orders")
    return out.value


def qaoa_mixer_x_terms(ctx: int, n: int, masks, coefs) -> int:
    m = (ctypes.c_uint64 * len(masks))(*[int(x) for x in masks])
    c = (c_double * len(coefs))(*[float(x) for x in coefs])
    out = c_void_p()
    check(lib().qaoa_mixer_x_terms(ctx, n, m, c, len(masks), ctypes.byref(out)), "qaoa_mixer_x_terms")
    return out.value


def qaoa_mixer_x_multiangle(ctx: int, n: int) -> int:
    out = c_void_p()
    check(lib().qaoa_mixer_x_multiangle(ctx, n, ctypes.byref(out)), "qaoa_mixer_x_multiangle")
    return out.value


def qaoa_mixer_info(mix: int) -> dict:
    n, k, apl = c_int(), c_int(), c_int()
    check(lib().qaoa_mixer_info(mix, ctypes.byref(n), ctypes.byref(k), ctypes.byref(apl)), "qaoa_mixer_info")
    return {"n": n.value, "hamming_k": k.value, "angles_per_layer": apl.value}


def qaoa_mixer_grover(ctx: int, n: int, hamming_k: int = -1) -> int:
    out = c_void_p()
    check(lib().qaoa_mixer_grover(ctx, n, hamming_k, ctypes.byref(out)), "qaoa_mixer_grover")
    return out.value


def qaoa_cost_degeneracies(ctx: int, n: int, u, v, w=None, hamming_k: int = -1, stream: int = 0) -> int:
    ua, up = _i32(u)
    va, vp = _i32(v)
    if w is None:
        wp = None
    else:
        wa, wp = _i32(w)
    out = c_void_p()
    check(lib().qaoa_cost_degeneracies(ctx, n, int(ua.size), up, vp, wp, hamming_k, ctypes.byref(out), stream),
          "qaoa_cost_degeneracies")
    return out.value


def qaoa_problem_degeneracies(prob: int, stream: int = 0):
    """(values, counts) of the distinct costs taken by at least one feasible state."""
    import numpy as np
    cnt = c_size_t()
    check(lib().qaoa_problem_degeneracies(prob, None, None, 0, ctypes.byref(cnt), stream), "qaoa_problem_degeneracies")
    vals = np.zeros(cnt.value, dtype=np.float64)
    counts = np.zeros(cnt.value, dtype=np.int64)
    check(lib().qaoa_problem_degeneracies(prob, vals.ctypes.data_as(P(c_double)), counts.ctypes.data_as(P(c_int64)),
                                          cnt.value, ctypes.byref(cnt), stream), "qaoa_problem_degeneracies")
    return vals, counts


def qaoa_mixer_clique(ctx: int, n: int, k: int, stream: int = 0) -> int:
    out = c_void_p()
    check(lib().qaoa_mixer_clique(ctx, n, k, ctypes.byref(out), stream), "qaoa_mixer_clique")
    return out.value


def qaoa_mixer_destroy(mix: int) -> None:
    check(lib().qaoa_mixer_destroy(mix), "qaoa_mixer_destroy")


def _f64(a):
    import numpy as np
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return arr, arr.ctypes.data_as(P(c_double))


def qaoa_expect(prob: int, mix: int, p: int, angles, d_psi0: int = 0, precision: int = QAOA_FP32,
                stream: int = 0) -> float:
    aa, ap = _f64(angles)
    out = c_double()
    check(lib().qaoa_expect(prob, mix, p, ap, d_psi0 or None, precision, ctypes.byref(out), stream),
          "qaoa_expect")
    return out.value


def qaoa_expect_grad(prob: int, mix: int, p: int, angles, d_psi0: int = 0,
                     precision: int = QAOA_FP32, stream: int = 0):
    import numpy as np
    aa, ap = _f64(angles)
    out = c_double()
    g = np.zeros(aa.size, dtype=np.float64)
    check(lib().qaoa_expect_grad(prob, mix, p, ap, d_psi0 or None, precision, ctypes.byref(out),
                                 g.ctypes.data_as(P(c_double)), stream), "qaoa_expect_grad")
    return out.value, g


def qaoa_state(prob: int, mix: int, p: int, angles, d_out: int, d_psi0: int = 0,
               precision: int = QAOA_FP32, stream: int = 0) -> None:
    aa, ap = _f64(angles)
    check(lib().qaoa_state(prob, mix, p, ap, d_psi0 or None, precision, d_out, stream), "qaoa_state")


def _ptrs(handles):
    arr = (c_void_p * len(handles))(*handles)
    return arr


def qaoa_expect_batched(probs, mixers, p: int, angles, precision: int = QAOA_FP32, stream: int = 0,
                        set_len: int = 0):
    import numpy as np
    aa, ap = _f64(angles)
    n_sets = aa.size // (set_len or 2 * p)
    out = np.zeros((len(probs), n_sets), dtype=np.float64)
    check(lib().qaoa_expect_batched(_ptrs(probs), _ptrs(mixers), len(probs), n_sets, p, ap, precision,
                                    out.ctypes.data_as(P(c_double)), stream), "qaoa_expect_batched")
    return out


def qaoa_expect_grad_batched(probs, mixers, p: int, angles, precision: int = QAOA_FP32, stream: int = 0,
                             set_len: int = 0):
    import numpy as np
    aa, ap = _f64(angles)
    L = set_len or 2 * p
    n_sets = aa.size // L
    out = np.zeros((len(probs), n_sets), dtype=np.float64)
    g = np.zeros((len(probs), n_sets, L), dtype=np.float64)
    check(lib().qaoa_expect_grad_batched(_ptrs(probs), _ptrs(mixers), len(probs), n_sets, p, ap, precision,
                                         out.ctypes.data_as(P(c_double)), g.ctypes.data_as(P(c_double)),
                                         stream), "qaoa_expect_grad_batched")
    return out, g


def qaoa_expect_pairs(probs, mixers, p: int, angles, precision: int = QAOA_FP32, stream: int = 0,
                      set_len: int = 0):
    """<C> of pair i = (probs[i], mixers[i], angles[i])."""
    import numpy as np
    aa, ap = _f64(angles)
    n = len(probs)
    if aa.size != n * (set_len or 2 * p) or len(mixers) != n:
        raise ValueError("one mixer and 2p angles per pair")
    out = np.zeros(n, dtype=np.float64)
    check(lib().qaoa_expect_pairs(_ptrs(probs), _ptrs(mixers), n, p, ap, precision,
                                  out.ctypes.data_as(P(c_double)), stream), "qaoa_expect_pairs")
    return out


def qaoa_expect_grad_pairs(probs, mixers, p: int, angles, precision: int = QAOA_FP32, stream: int = 0,
                           set_len: int = 0):
    import numpy as np
    aa, ap = _f64(angles)
    n = len(probs)
    L = set_len or 2 * p
    if aa.size != n * L or len(mixers) != n:
        raise ValueError("one mixer and 2p angles per pair")
    out = np.zeros(n, dtype=np.float64)
    g = np.zeros((n, L), dtype=np.float64)
    check(lib().qaoa_expect_grad_pairs(_ptrs(probs), _ptrs(mixers), n, p, ap, precision,
                                       out.ctypes.data_as(P(c_double)), g.ctypes.data_as(P(c_double)), stream),
          "qaoa_expect_grad_pairs")
    return out, g


def qaoa_expect_grad_pairs_noalloc(probs, mixers, p: int, angles, precision: int = QAOA_FP32, stream: int = 0):
    """The allocation-free paired fwd+grad (whole-state transverse-field pairs only)."""
    import numpy as np
    aa, ap = _f64(angles)
    n = len(probs)
    if aa.size != n * 2 * p or len(mixers) != n:
        raise ValueError("one mixer and 2p angles per pair")
    out = np.zeros(n, dtype=np.float64)
    g = np.zeros((n, 2 * p), dtype=np.float64)
    check(lib().qaoa_expect_grad_pairs_noalloc(_ptrs(probs), _ptrs(mixers), n, p, ap, precision,
                                               out.ctypes.data_as(P(c_double)), g.ctypes.data_as(P(c_double)),
                                               stream), "qaoa_expect_grad_pairs_noalloc")
    return out, g


def qaoa_profile_enable(ctx: int, enable: bool = True) -> None:
    check(lib().qaoa_profile_enable(ctx, 1 if enable else 0), "qaoa_profile_enable")


def qaoa_profile_read(ctx: int, kernel_class: int) -> dict:
    n, ms, by, fl = c_int64(), c_double(), c_double(), c_double()
    check(lib().qaoa_profile_read(ctx, kernel_class, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                  ctypes.byref(fl)), "qaoa_profile_read")
    return {"launches": n.value, "ms": ms.value, "bytes": by.value, "flops": fl.value}


def qaoa_stream_copy(ctx: int, src: int, dst: int, nbytes: int, stream: int = 0) -> None:
    check(lib().qaoa_stream_copy(ctx, src, dst, nbytes, stream), "qaoa_stream_copy")


def qaoa_ctx_set_autotune(ctx: int, enable: bool = True) -> None:
    check(lib().qaoa_ctx_set_autotune(ctx, 1 if enable else 0), "qaoa_ctx_set_autotune")


def qaoa_plans_text(ctx: int) -> str:
    need = c_size_t()
    check(lib().qaoa_plans_text(ctx, None, 0, ctypes.byref(need)), "qaoa_plans_text")
    buf = ctypes.create_string_buffer(need.value)
    check(lib().qaoa_plans_text(ctx, buf, need.value, None), "qaoa_plans_text")
    return buf.value.decode()


def qaoa_plans_save(ctx: int, path: str) -> None:
    check(lib().qaoa_plans_save(ctx, os.fsencode(path)), "qaoa_plans_save")


def qaoa_plans_load(ctx: int, path: str) -> None:
    check(lib().qaoa_plans_load(ctx, os.fsencode(path)), "qaoa_plans_load")


# ---------------------------------------------------------------- angle finding

def qaoa_angle_opts_default() -> qaoa_angle_opts:
    o = qaoa_angle_opts()
    lib().qaoa_angle_opts_default(ctypes.byref(o))
    return o


def qaoa_minimize(prob: int, mix: int, p: int, starts, opts: qaoa_angle_opts, stream: int = 0):
    """(optima [n_starts][2p], <C> there [n_starts], accepted steps [n_starts])."""
    import numpy as np
    xs = np.array(starts, dtype=np.float64, order="C").reshape(-1, 2 * p)
    vals = np.zeros(xs.shape[0], dtype=np.float64)
    its = np.zeros(xs.shape[0], dtype=np.int32)
    check(lib().qaoa_minimize(prob, mix, p, xs.shape[0], xs.ctypes.data_as(P(c_double)),
                              vals.ctypes.data_as(P(c_double)), its.ctypes.data_as(P(c_int)), ctypes.byref(opts),
                              stream), "qaoa_minimize")
    return xs, vals, its


def qaoa_basinhopping(prob: int, mix: int, p: int, x0, opts: qaoa_angle_opts, stream: int = 0):
    import numpy as np
    xa, xp = _f64(x0)
    out = np.zeros(2 * p, dtype=np.float64)
    val = c_double()
    check(lib().qaoa_basinhopping(prob, mix, p, xp, ctypes.byref(opts), out.ctypes.data_as(P(c_double)),
                                  ctypes.byref(val), stream), "qaoa_basinhopping")
    return out, val.value


def qaoa_find_angles(prob: int, mix: int, p_max: int, opts: qaoa_angle_opts, checkpoint_path=None,
                     stream: int = 0):
    """(angles [p_max][2 p_max], row r-1 holding round r's 2r angles; values [p_max])."""
    import numpy as np
    out = np.zeros((p_max, 2 * p_max), dtype=np.float64)
    vals = np.zeros(p_max, dtype=np.float64)
    path = os.fsencode(checkpoint_path) if checkpoint_path is not None else None
    check(lib().qaoa_find_angles(prob, mix, p_max, ctypes.byref(opts), path, out.ctypes.data_as(P(c_double)),
                                 vals.ctypes.data_as(P(c_double)), stream), "qaoa_find_angles")
    return out, vals


def qaoa_find_angles_random(prob: int, mix: int, p: int, n_restarts: int, opts: qaoa_angle_opts, stream: int = 0):
    """(best angles [2p], best <C>, <C> of every restart's optimum [n_restarts])."""
    import numpy as np
    out = np.zeros(2 * p, dtype=np.float64)
    allv = np.zeros(n_restarts, dtype=np.float64)
    val = c_double()
    check(lib().qaoa_find_angles_random(prob, mix, p, n_restarts, ctypes.byref(opts), out.ctypes.data_as(P(c_double)),
                                        ctypes.byref(val), allv.ctypes.data_as(P(c_double)), stream),
          "qaoa_find_angles_random")
    return out, val.value, allv


def qaoa_find_angles_multi(probs, mixers, p_max: int, opts: qaoa_angle_opts, checkpoint_paths=None,
                           stream: int = 0):
    """(angles [n][p_max][2 p_max], values [n][p_max]) for n instances solved together."""
    import numpy as np
    n = len(probs)
    out = np.zeros((n, p_max, 2 * p_max), dtype=np.float64)
    vals = np.zeros((n, p_max), dtype=np.float64)
    paths = None
    if checkpoint_paths is not None:
        paths = (ctypes.c_char_p * n)(*[os.fsencode(x) if x is not None else None for x in checkpoint_paths])
    check(lib().qaoa_find_angles_multi(_ptrs(probs), _ptrs(mixers), n, p_max, ctypes.byref(opts), paths,
                                       out.ctypes.data_as(P(c_double)), vals.ctypes.data_as(P(c_double)), stream),
          "qaoa_find_angles_multi")
    return out, vals
