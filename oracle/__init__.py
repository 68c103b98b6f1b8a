"""Python wrapper of the plain FP64 CPU oracle (``oracle/qaoa_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the benchmark's
CPU-baseline leg, never by the product library. It shares no code with the GPU path.

The C file holds the arithmetic (cost table, Eq. (1) evolution with the transverse-field or
clique mixer, <C>, adjoint gradient). This wrapper adds argument marshalling and a second,
independent gradient route: central finite differences with one Richardson step, built
only on the forward <C>.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qaoa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (IEEE FP64, OpenMP); returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fcx-limited-range", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        c128p = np.ctypeslib.ndpointer(np.complex128, flags="C_CONTIGUOUS")
        L.orc_binom.restype = ctypes.c_int64
        L.orc_binom.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_states.restype = ctypes.c_int64
        L.orc_states.argtypes = [ctypes.c_int, ctypes.c_int, u64p]
        L.orc_cost_table.restype = ctypes.c_int64
        L.orc_cost_table.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, i32p, ctypes.c_int, i64p]
        L.orc_apply_phase.argtypes = [ctypes.c_int64, ctypes.c_double, f64p, c128p]
        L.orc_apply_x_mixer.argtypes = [ctypes.c_int, ctypes.c_double, c128p]
        L.orc_apply_x_sum.argtypes = [ctypes.c_int, c128p, c128p]
        L.orc_clique_neighbours.restype = ctypes.c_int64
        L.orc_clique_neighbours.argtypes = [ctypes.c_int, ctypes.c_int, u64p, ctypes.c_int64, i64p]
        L.orc_apply_clique_mixer.argtypes = [ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int64,
                                             ctypes.c_double, c128p]
        L.orc_expect.restype = ctypes.c_double
        L.orc_expect.argtypes = [ctypes.c_int64, f64p, c128p, ctypes.POINTER(ctypes.c_double)]
        vp = ctypes.c_void_p
        L.orc_qaoa_state.restype = ctypes.c_int
        L.orc_qaoa_state.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, f64p, f64p, vp, c128p]
        L.orc_qaoa_expect.restype = ctypes.c_int
        L.orc_qaoa_expect.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, f64p, f64p, vp,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.orc_qaoa_grad.restype = ctypes.c_int
        L.orc_qaoa_grad.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, f64p, f64p, vp,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), f64p]
        i = ctypes.c_int
        L.orc_qaoa_state_m.restype = ctypes.c_int
        L.orc_qaoa_state_m.argtypes = [i, i, i, i, f64p, f64p, vp, c128p]
        L.orc_qaoa_expect_m.restype = ctypes.c_int
        L.orc_qaoa_expect_m.argtypes = [i, i, i, i, f64p, f64p, vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
        L.orc_qaoa_grad_m.restype = ctypes.c_int
        L.orc_qaoa_grad_m.argtypes = [i, i, i, i, f64p, f64p, vp, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), f64p]
        L.orc_apply_grover_mixer.argtypes = [ctypes.c_int64, ctypes.c_double, c128p]
        L.orc_ring_neighbours.restype = ctypes.c_int64
        L.orc_ring_neighbours.argtypes = [ctypes.c_int, ctypes.c_int, u64p, ctypes.c_int64, i64p]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_cost_values.restype = ctypes.c_int
        L.orc_cost_values.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, i32p, u64p, ctypes.c_int64, i64p]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def binom(n: int, k: int) -> int:
    return int(lib().orc_binom(n, k))


def states(n: int, k: int = -1) -> np.ndarray:
    """Feasible set S in the oracle's order: all 0..2^n-1, or weight-k integers ascending."""
    N = (1 << n) if k < 0 else binom(n, k)
    out = np.zeros(N, dtype=np.uint64)
    lib().orc_states(n, k, out)
    return out


def cost_table(n: int, u, v, w=None, k: int = -1) -> np.ndarray:
    """MaxCut table C(x) = sum_e w_e [x_u != x_v] over S (int64)."""
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ones_like(u) if w is None else np.ascontiguousarray(w, dtype=np.int32)
    N = (1 << n) if k < 0 else binom(n, k)
    out = np.zeros(N, dtype=np.int64)
    r = lib().orc_cost_table(n, int(u.size), u, v, w, k, out)
    if r != N:
        raise ValueError("oracle rejected the graph")
    return out


def cost_values(n: int, u, v, w, xs) -> np.ndarray:
    """C(x) at the given basis strings (for sampled checks of tables too large to build)."""
    u = np.ascontiguousarray(u, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.int32)
    w = np.ones_like(u) if w is None else np.ascontiguousarray(w, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    out = np.zeros(xs.size, dtype=np.int64)
    if lib().orc_cost_values(n, int(u.size), u, v, w, xs, xs.size, out):
        raise ValueError("oracle rejected the graph")
    return out


def graph_table(g, k: int = -1) -> np.ndarray:
    return cost_table(g.n, g.u, g.v, g.w, k)


def _psi0_ptr(psi0, N):
    if psi0 is None:
        return None, None
    a = np.ascontiguousarray(psi0, dtype=np.complex128)
    if a.size != N:
        raise ValueError("psi0 has the wrong length")
    return a, a.ctypes.data


def _check(n, k, angles, table):
    """The cost is any list of values over the feasible states (integers from cost_table, or
    arbitrary reals); the evolution takes it as FP64."""
    angles = np.ascontiguousarray(angles, dtype=np.float64)
    table = np.ascontiguousarray(table, dtype=np.float64)
    N = (1 << n) if k < 0 else binom(n, k)
    if table.size != N or angles.size % 2:
        raise ValueError("bad table or angle length")
    return angles, table, N, angles.size // 2


def _code(grover, ring):
    return 1 if grover else (2 if ring else 0)


def state(n: int, table, angles, k: int = -1, psi0=None, grover: bool = False, ring: bool = False) -> np.ndarray:
    """psi_p of Eq. (1) (complex128, order of ``states``). Mixer: X (k < 0) or clique
    (k >= 0); ``grover=True``: the Grover mixer on the same states (Sec. 2.4); ``ring=True``:
    the ring mixer on weight k."""
    angles, table, N, p = _check(n, k, angles, table)
    keep, ptr = _psi0_ptr(psi0, N)
    out = np.zeros(N, dtype=np.complex128)
    if lib().orc_qaoa_state_m(n, k, _code(grover, ring), p, angles, table, ptr, out):
        raise RuntimeError("oracle failed")
    return out


def expect(n: int, table, angles, k: int = -1, psi0=None, grover: bool = False, ring: bool = False):
    """(E, Nrm): E = sum |psi_p|^2 C, Nrm = sum |psi_p|^2."""
    angles, table, N, p = _check(n, k, angles, table)
    keep, ptr = _psi0_ptr(psi0, N)
    E, Nr = ctypes.c_double(), ctypes.c_double()
    if lib().orc_qaoa_expect_m(n, k, _code(grover, ring), p, angles, table, ptr, ctypes.byref(E), ctypes.byref(Nr)):
        raise RuntimeError("oracle failed")
    return E.value, Nr.value


def grad(n: int, table, angles, k: int = -1, psi0=None, grover: bool = False, ring: bool = False):
    """(E, Nrm, g) with g = [d/dbeta_1..p, d/dgamma_1..p] from the adjoint recursion."""
    angles, table, N, p = _check(n, k, angles, table)
    keep, ptr = _psi0_ptr(psi0, N)
    E, Nr = ctypes.c_double(), ctypes.c_double()
    g = np.zeros(2 * p, dtype=np.float64)
    if lib().orc_qaoa_grad_m(n, k, _code(grover, ring), p, angles, table, ptr, ctypes.byref(E), ctypes.byref(Nr), g):
        raise RuntimeError("oracle failed")
    return E.value, Nr.value, g


def dense_mixer_grad(table, angles, H, psi0=None):
    """Eq. (1) with a mixer given as a real symmetric matrix H on the feasible states
    (Sec. 2.1: any mixer can be handed over as a matrix): each round psi <- expm(-i b H)
    (e^{-i g C} psi), expm by scipy; <C> and the adjoint gradient as in the C oracle, in plain
    dense FP64 linear algebra. Returns (E, Nrm, g)."""
    import scipy.linalg
    angles = np.asarray(angles, dtype=np.float64)
    C = np.asarray(table, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    N, p = C.size, angles.size // 2
    psi = np.full(N, 1 / np.sqrt(N), dtype=np.complex128) if psi0 is None else np.array(psi0, dtype=np.complex128)
    U = [scipy.linalg.expm(-1j * angles[r] * H) for r in range(p)]
    for r in range(p):
        psi = U[r] @ (np.exp(-1j * angles[p + r] * C) * psi)
    pr = np.abs(psi) ** 2
    E, Nr = float(np.sum(pr * C)), float(np.sum(pr))
    phi, lam = psi.copy(), C * psi
    g = np.zeros(2 * p)
    for r in range(p - 1, -1, -1):
        g[r] = 2 * np.imag(np.vdot(lam, H @ phi))
        phi, lam = U[r].conj().T @ phi, U[r].conj().T @ lam
        g[p + r] = 2 * np.imag(np.vdot(lam, C * phi))
        ph = np.exp(1j * angles[p + r] * C)
        phi, lam = ph * phi, ph * lam
    return E, Nr, g


def ring_neighbours(n: int, k: int) -> np.ndarray:
    """[C(n,k), ring edges] neighbour indices of the ring mixer on weight k (-1: no swap)."""
    st = states(n, k)
    deg = n if n >= 3 else (1 if n == 2 else 0)
    nb = np.zeros(st.size * max(deg, 1), dtype=np.int64)
    lib().orc_ring_neighbours(n, k, st, st.size, nb)
    return nb.reshape(st.size, max(deg, 1))[:, :deg]


def degeneracies(table):
    """Distinct values of C over the feasible states and how many states take each (Sec. 2.4)."""
    vals, counts = np.unique(np.asarray(table), return_counts=True)
    return vals, counts


def fd_grad(n: int, table, angles, k: int = -1, psi0=None, h: float = 1e-3, grover: bool = False,
            ring: bool = False) -> np.ndarray:
    """Central finite differences with one Richardson step (error O(h^4)), forward-only."""
    angles = np.asarray(angles, dtype=np.float64)
    g = np.zeros(angles.size)
    for j in range(angles.size):
        def f(d):
            a = angles.copy()
            a[j] += d
            return expect(n, table, a, k, psi0, grover, ring)[0]
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        g[j] = (4 * d2 - d1) / 3
    return g


def apply_phase(table, gamma: float, psi: np.ndarray) -> None:
    """In place: psi(x) *= e^{-i gamma C(x)}."""
    lib().orc_apply_phase(int(psi.size), float(gamma), np.ascontiguousarray(table, dtype=np.float64), psi)


def apply_x_mixer(n: int, beta: float, psi: np.ndarray) -> None:
    """In place: psi <- prod_q e^{-i beta X_q} psi."""
    lib().orc_apply_x_mixer(n, float(beta), psi)


def apply_grover_mixer(beta: float, psi: np.ndarray) -> None:
    """In place: psi += (e^{-i beta} - 1) <psi0|psi> psi0 over len(psi) states."""
    lib().orc_apply_grover_mixer(int(psi.size), float(beta), psi)


def apply_x_sum(n: int, psi: np.ndarray) -> np.ndarray:
    out = np.zeros_like(psi)
    lib().orc_apply_x_sum(n, psi, out)
    return out


def clique_neighbours(n: int, k: int) -> np.ndarray:
    st = states(n, k)
    deg = k * (n - k)
    nb = np.zeros(st.size * max(deg, 1), dtype=np.int64)
    lib().orc_clique_neighbours(n, k, st, st.size, nb)
    return nb.reshape(st.size, max(deg, 1))[:, :deg]


def apply_clique_mixer(n: int, k: int, beta: float, psi: np.ndarray, nb=None) -> None:
    """In place: psi <- e^{-i beta H_clique} psi on the weight-k subspace (Taylor series)."""
    if nb is None:
        nb = clique_neighbours(n, k)
    nbf = np.ascontiguousarray(nb, dtype=np.int64).reshape(-1)
    if nbf.size == 0:
        nbf = np.zeros(1, dtype=np.int64)
    lib().orc_apply_clique_mixer(n, k, nbf, int(psi.size), float(beta), psi)
