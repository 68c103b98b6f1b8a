"""Independent constructions that pin the oracle (test code, not part of the oracle).

* ``maxcut_p1``: closed-form p=1 MaxCut expectation of Wang, Hadfield, Jiang and Rieffel
  (Phys. Rev. A 97, 022304, 2018), for H_M = sum X_q, phase e^{-i gamma C}, C = number of cut
  edges, and its analytic derivative in (beta, gamma).
* ``dense_*``: brute-force 2^n x 2^n constructions from Pauli matrices with
  ``scipy.linalg.expm`` (matrix exponential of the full Hamiltonian, not the oracle's
  per-qubit loop or Taylor series).
* ``johnson_spectrum``: closed-form eigenvalues of the clique mixer on weight-k strings
  (Johnson-scheme adjacency times 2).
* ``cycle_edge``: per-edge cut probability of p-round QAOA on a cycle of at least 2p + 3
  vertices, from the light cone (Farhi, Goldstone and Gutmann, arXiv:1411.4028): the middle
  edge of the path of 2p + 2 vertices, by dense matrix exponentials, and its gradient by
  central differences.
* ``light_cone_expect``: <C> of p-round QAOA on any graph as a sum of per-edge terms, each
  evaluated on the vertices within distance p of its edge (the same light cone), with the
  mixer applied by ``scipy.sparse.linalg.expm_multiply`` on the sparse sum of X built entry
  by entry (not the oracle's qubit-by-qubit rotations); the gradient by central differences.
* ``cycle_edge_blocks``: the cycle's edge term of ``cycle_edge`` at any depth (the path of
  2p + 2 vertices: 18 qubits at p = 8, beyond dense 2^m x 2^m matrices), with the mixer
  applied block by block: the X_q commute, so e^{-i b sum_q X_q} is the product over blocks
  of at most 6 qubits of the dense matrix exponential of that block's sum of X (built from
  Pauli Kronecker products), each applied to the state reshaped so the block is one axis.
"""
from __future__ import annotations

from math import comb

import numpy as np
import scipy.linalg

X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def _op_on(n, ops):
    """Kronecker product with ops[q] on qubit q (qubit q = bit q of the basis index)."""
    m = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):        # most significant qubit leftmost
        m = np.kron(m, ops.get(q, I2))
    return m


def dense_x_mixer_hamiltonian(n):
    return sum(_op_on(n, {q: X}) for q in range(n))


def dense_clique_hamiltonian(n):
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for i in range(n):
        for j in range(i + 1, n):
            H += _op_on(n, {i: X, j: X}) + _op_on(n, {i: Y, j: Y})
    return H


def dense_evolve(H_M, table, angles, psi0):
    """Eq. (1) by dense matrix exponentials: psi <- expm(-i b H_M) diag(e^{-i g C}) psi."""
    p = len(angles) // 2
    psi = np.array(psi0, dtype=np.complex128)
    for r in range(p):
        psi = np.exp(-1j * angles[p + r] * np.asarray(table, dtype=np.float64)) * psi
        psi = scipy.linalg.expm(-1j * angles[r] * H_M) @ psi
    return psi


def maxcut_p1(n, edges, beta, gamma):
    """Closed-form p=1 <C> for unweighted MaxCut, and (d/dbeta, d/dgamma)."""
    nbrs = [set() for _ in range(n)]
    for a, b in edges:
        nbrs[a].add(b)
        nbrs[b].add(a)
    s4b, c4b = np.sin(4 * beta), np.cos(4 * beta)
    s2b2, ds2b2 = np.sin(2 * beta) ** 2, 2 * np.sin(4 * beta)
    sg, cg = np.sin(gamma), np.cos(gamma)
    c2g, s2g = np.cos(2 * gamma), np.sin(2 * gamma)

    def pw(x, k):
        return x ** k

    def dpw(x, k, dx):          # d/dgamma x^k where dx = dx/dgamma
        return k * x ** (k - 1) * dx if k > 0 else 0.0

    E = dEb = dEg = 0.0
    for a, b in edges:
        du, dv = len(nbrs[a]) - 1, len(nbrs[b]) - 1
        f = len(nbrs[a] & nbrs[b])
        S = sg * (pw(cg, du) + pw(cg, dv))
        dS = cg * (pw(cg, du) + pw(cg, dv)) + sg * (dpw(cg, du, -sg) + dpw(cg, dv, -sg))
        ex = du + dv - 2 * f
        T = pw(cg, ex) * (1 - pw(c2g, f))
        dT = dpw(cg, ex, -sg) * (1 - pw(c2g, f)) - pw(cg, ex) * dpw(c2g, f, -2 * s2g)
        E += 0.5 + 0.25 * s4b * S - 0.25 * s2b2 * T
        dEb += 0.25 * 4 * c4b * S - 0.25 * ds2b2 * T
        dEg += 0.25 * s4b * dS - 0.25 * s2b2 * dT
    return E, dEb, dEg


def johnson_spectrum(n, k):
    """Eigenvalues of sum_{i<j} X_iX_j + Y_iY_j on weight k, with multiplicities."""
    out = []
    for j in range(min(k, n - k) + 1):
        lam = 2 * ((k - j) * (n - k - j) - j)
        mult = comb(n, j) - (comb(n, j - 1) if j > 0 else 0)
        out += [lam] * mult
    return np.sort(np.array(out, dtype=np.float64))


def dense_ring_hamiltonian(n):
    """sum_i X_i X_{i+1} + Y_i Y_{i+1} with i + 1 mod n (one edge for n = 2)."""
    H = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    edges = [(i, (i + 1) % n) for i in range(n)] if n >= 3 else [(0, 1)]
    for i, j in edges:
        H += _op_on(n, {i: X, j: X}) + _op_on(n, {i: Y, j: Y})
    return H


def cycle_edge(p, angles, h=1e-5):
    """(value, gradient) of the cut probability of one edge of a cycle C_n, n >= 2p + 3, after
    p rounds at `angles` ([beta_1..p, gamma_1..p]): after p rounds the edge term involves only
    the qubits within distance p of the edge and the edges touching qubits within distance
    p - 1, i.e. the path of 2p + 2 vertices with the edge in the middle."""
    m = 2 * p + 2
    xs = np.arange(1 << m)
    bit = lambda q: (xs >> q) & 1
    path_cost = sum(bit(i) ^ bit(i + 1) for i in range(m - 1)).astype(np.float64)
    mid_cut = (bit(p) ^ bit(p + 1)).astype(np.float64)
    H = dense_x_mixer_hamiltonian(m)
    psi0 = np.full(1 << m, 2.0 ** (-m / 2), dtype=np.complex128)

    def value(a):
        psi = dense_evolve(H, path_cost, a, psi0)
        return float(np.sum(np.abs(psi) ** 2 * mid_cut))

    a = np.asarray(angles, dtype=np.float64)
    g = np.array([(value(a + h * e) - value(a - h * e)) / (2 * h) for e in np.eye(2 * p)])
    return value(a), g


def sparse_x_mixer_hamiltonian(m):
    """sum_q X_q on m qubits, sparse, entry by entry: <x| X_q |z> = 1 exactly when z = x XOR 2^q."""
    import scipy.sparse as sp
    N = 1 << m
    rows = np.repeat(np.arange(N), m)
    cols = (np.arange(N)[:, None] ^ (1 << np.arange(m))[None, :]).reshape(-1)
    return sp.csr_matrix((np.ones(N * m), (rows, cols)), shape=(N, N))


def light_cone_expect(n, u, v, w, p, angles, h=1e-5, components=None):
    """(<C>, gradient) of p-round QAOA for C = sum_e w_e [x_u != x_v] on the graph (u, v, w) at
    `angles` ([beta_1..p, gamma_1..p]). After p rounds the term of edge e involves only the
    qubits within distance p of e, and the phase terms of edges outside that ball commute with
    it, so each term is evolved on the subgraph induced by its ball (<= 2 + 4 + ... qubits on a
    3-regular graph) from the uniform superposition. `components` limits the central
    differences to those gradient entries (all by default; the others are returned as NaN)."""
    from scipy.sparse.linalg import expm_multiply
    u = np.asarray(u); v = np.asarray(v); w = np.asarray(w, dtype=np.float64)
    adj = [[] for _ in range(n)]
    for a_, b_ in zip(u, v):
        adj[int(a_)].append(int(b_)); adj[int(b_)].append(int(a_))
    terms = []
    for e in range(u.size):
        dist = {int(u[e]): 0, int(v[e]): 0}
        front = [int(u[e]), int(v[e])]
        for d in range(1, p + 1):
            nxt = []
            for x in front:
                for y in adj[x]:
                    if y not in dist:
                        dist[y] = d
                        nxt.append(y)
            front = nxt
        ball = sorted(dist)
        loc = {x: i for i, x in enumerate(ball)}
        m = len(ball)
        xs = np.arange(1 << m)
        bit = lambda q: (xs >> q) & 1
        cost = np.zeros(1 << m)
        for a_, b_, ww in zip(u, v, w):
            if int(a_) in loc and int(b_) in loc:
                cost += ww * (bit(loc[int(a_)]) ^ bit(loc[int(b_)]))
        cut = w[e] * (bit(loc[int(u[e])]) ^ bit(loc[int(v[e])])).astype(np.float64)
        terms.append((m, cost, cut, sparse_x_mixer_hamiltonian(m)))

    def value(a):
        tot = 0.0
        for m, cost, cut, H in terms:
            psi = np.full(1 << m, 2.0 ** (-m / 2), dtype=np.complex128)
            for k in range(p):
                psi = np.exp(-1j * a[p + k] * cost) * psi
                psi = expm_multiply((-1j * a[k]) * H, psi)
            tot += float(np.sum(np.abs(psi) ** 2 * cut))
        return tot

    a = np.asarray(angles, dtype=np.float64)
    g = np.full(2 * p, np.nan)
    for i in (range(2 * p) if components is None else components):
        e = np.eye(2 * p)[i]
        g[i] = (value(a + h * e) - value(a - h * e)) / (2 * h)
    return value(a), g


def _block_mixers(m, beta, block=6):
    """[(lo, hi, expm(-i beta sum_{lo <= q < hi} X_q))] covering qubits 0..m-1."""
    out = []
    for lo in range(0, m, block):
        hi = min(m, lo + block)
        out.append((lo, hi, scipy.linalg.expm(-1j * beta * dense_x_mixer_hamiltonian(hi - lo))))
    return out


def _apply_block(psi, m, lo, hi, U):
    """psi <- (I (x) U (x) I) psi with U on qubits lo..hi-1 (qubit q = bit q of the index)."""
    t = psi.reshape(1 << (m - hi), 1 << (hi - lo), 1 << lo)
    return np.einsum("ij,ajb->aib", U, t).reshape(-1)


def cycle_edge_blocks(p, angles, h=1e-5, components=None, block=6):
    """(value, gradient) of the cut probability of one edge of a cycle C_n, n >= 2p + 3, after
    p rounds (the light cone of ``cycle_edge``: the middle edge of the path of 2p + 2
    vertices), for any p. The mixer of each round is the product over qubit blocks of dense
    block exponentials (``_block_mixers``). `components` limits the central differences to
    those gradient entries (all by default; the others are NaN)."""
    m = 2 * p + 2
    xs = np.arange(1 << m)
    bit = lambda q: (xs >> q) & 1
    path_cost = sum(bit(i) ^ bit(i + 1) for i in range(m - 1)).astype(np.float64)
    mid_cut = (bit(p) ^ bit(p + 1)).astype(np.float64)

    def value(a):
        psi = np.full(1 << m, 2.0 ** (-m / 2), dtype=np.complex128)
        for r in range(p):
            psi = np.exp(-1j * a[p + r] * path_cost) * psi
            for lo, hi, U in _block_mixers(m, a[r], block):
                psi = _apply_block(psi, m, lo, hi, U)
        return float(np.sum(np.abs(psi) ** 2 * mid_cut))

    a = np.asarray(angles, dtype=np.float64)
    g = np.full(2 * p, np.nan)
    for i in (range(2 * p) if components is None else components):
        e = np.eye(2 * p)[i]
        g[i] = (value(a + h * e) - value(a - h * e)) / (2 * h)
    return value(a), g
