"""Plain FP64 reference for mixers built from products of Pauli X (Sec. 2.1, Eq. (2)) and for
multi-angle mixers (Sec. 3: several mixers per layer, each with its own angle).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: shares no code with the library.

A mixer H_M = sum_t c_t prod_{i in S_t} X_i is diagonal after a Hadamard on every qubit
(H Z H = X): e^{-i b H_M} = W e^{-i b f(Z)} W with W the normalised Walsh-Hadamard transform
and f(Z) the diagonal with entries d(y) = sum_t c_t (-1)^{|y & S_t|} (Z_i = (-1)^{y_i}). The
symmetric mixers sum_{|S| = k} X_S (k-body terms over all k-subsets) have d(y) = K_k(|y|), the
Krawtchouk polynomial K_k(w) = sum_j (-1)^j C(w, j) C(n - w, k - j); k = 1 is the transverse
field. Multi-angle per qubit: layer k applies prod_q e^{-i beta_{k,q} X_q}, here applied qubit
by qubit as 2 x 2 rotations (not through W).

Angle layouts: single-angle mixers [beta_1..beta_p, gamma_1..gamma_p]; per-qubit multi-angle
[beta_{1,0..n-1}, ..., beta_{p,0..n-1}, gamma_1..gamma_p].
"""
from __future__ import annotations

from math import comb

import numpy as np


def krawtchouk(n: int, k: int, w: int) -> int:
    return sum((-1) ** j * comb(w, j) * comb(n - w, k - j) for j in range(0, k + 1))


def popcounts(n: int) -> np.ndarray:
    y = np.arange(1 << n, dtype=np.int64)
    c = np.zeros(1 << n, dtype=np.int64)
    for i in range(n):
        c += (y >> i) & 1
    return c


def diag_orders(n: int, orders) -> np.ndarray:
    """d(y) of sum_{k in orders} sum_{|S| = k} prod_{i in S} X_i."""
    w = popcounts(n)
    table = np.array([sum(krawtchouk(n, k, v) for k in orders) for v in range(n + 1)], dtype=np.float64)
    return table[w]


def diag_terms(n: int, masks, coefs) -> np.ndarray:
    """d(y) of sum_t coefs[t] prod_{i: bit i of masks[t]} X_i."""
    y = np.arange(1 << n, dtype=np.int64)
    d = np.zeros(1 << n, dtype=np.float64)
    for m, c in zip(masks, coefs):
        par = np.zeros(1 << n, dtype=np.int64)
        for i in range(n):
            if (int(m) >> i) & 1:
                par ^= (y >> i) & 1
        d += c * (1 - 2 * par)
    return d


def wht(psi: np.ndarray) -> np.ndarray:
    """Normalised Walsh-Hadamard transform: a Hadamard on every qubit."""
    v = np.array(psi, dtype=np.complex128)
    n = v.size.bit_length() - 1
    for q in range(n):
        v = v.reshape(-1, 2, 1 << q)
        a, b = v[:, 0, :].copy(), v[:, 1, :].copy()
        v[:, 0, :] = (a + b) / np.sqrt(2)
        v[:, 1, :] = (a - b) / np.sqrt(2)
        v = v.reshape(-1)
    return v


def apply_x_rotation(psi: np.ndarray, q: int, beta: float) -> np.ndarray:
    """e^{-i beta X_q} psi."""
    v = psi.reshape(-1, 2, 1 << q)
    a, b = v[:, 0, :].copy(), v[:, 1, :].copy()
    c, s = np.cos(beta), np.sin(beta)
    out = np.empty_like(v)
    out[:, 0, :] = c * a - 1j * s * b
    out[:, 1, :] = -1j * s * a + c * b
    return out.reshape(-1)


def apply_x(psi: np.ndarray, q: int) -> np.ndarray:
    """X_q psi."""
    return psi.reshape(-1, 2, 1 << q)[:, ::-1, :].reshape(-1).copy()


def _mixer(psi, beta, d):
    return wht(np.exp(-1j * beta * d) * wht(psi))


def grad(n: int, table, angles, d=None, multiangle: bool = False, psi0=None):
    """(E, Nrm, g) of Eq. (1) with the X-product mixer of diagonal d (single angle per layer),
    or with per-qubit angles (multiangle=True); g in the angle layout of the module docstring.
    The gradient is the adjoint recursion: lam = C psi_p, then layer by layer backwards
    dE/dtheta = 2 Im <lam| A |psi> for a factor e^{-i theta A} at the point just after it."""
    C = np.asarray(table, dtype=np.float64)
    a = np.asarray(angles, dtype=np.float64)
    N = 1 << n
    m = n if multiangle else 1
    p = a.size // (m + 1)
    betas = a[:p * m].reshape(p, m)
    gammas = a[p * m:]
    psi = np.full(N, 1 / np.sqrt(N), dtype=np.complex128) if psi0 is None else np.array(psi0, dtype=np.complex128)
    after_phase = []
    for k in range(p):
        psi = np.exp(-1j * gammas[k] * C) * psi
        after_phase.append(psi.copy())
        if multiangle:
            for q in range(n):
                psi = apply_x_rotation(psi, q, betas[k, q])
        else:
            psi = _mixer(psi, betas[k, 0], d)
    E = float(np.sum(np.abs(psi) ** 2 * C))
    Nr = float(np.sum(np.abs(psi) ** 2))
    gb = np.zeros((p, m))
    gg = np.zeros(p)
    lam = C * psi
    for k in range(p - 1, -1, -1):
        if multiangle:
            phi = psi
            for q in range(n - 1, -1, -1):
                # the rotations commute, so every X_q term is taken at the layer's end point
                gb[k, q] = 2 * np.imag(np.vdot(lam, apply_x(phi, q)))
            for q in range(n):
                lam = apply_x_rotation(lam, q, -betas[k, q])
        else:
            gb[k, 0] = 2 * np.imag(np.vdot(lam, wht(d * wht(psi))))
            lam = _mixer(lam, -betas[k, 0], d)
        psi = after_phase[k]
        gg[k] = 2 * np.imag(np.vdot(lam, C * psi))
        lam = np.exp(1j * gammas[k] * C) * lam
        psi = np.exp(1j * gammas[k] * C) * psi
    return E, Nr, np.concatenate([gb.reshape(-1), gg])


def dense_x_products(n: int, masks, coefs) -> np.ndarray:
    """The 2^n x 2^n matrix sum_t coefs[t] prod_{i in S_t} X_i, built entry by entry:
    <x| X_S |z> = 1 exactly when z = x XOR S."""
    N = 1 << n
    H = np.zeros((N, N))
    for m, c in zip(masks, coefs):
        for x in range(N):
            H[x, x ^ int(m)] += c
    return H


def all_masks_of_order(n: int, k: int):
    from itertools import combinations
    return [sum(1 << i for i in S) for S in combinations(range(n), k)]
