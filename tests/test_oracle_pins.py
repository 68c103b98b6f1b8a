"""Pins of the FP64 CPU oracle against what the paper and mathematics fix (CPU only).

Each test would fail for a plausible slip in the oracle: a wrong bit index or XOR in the
table (sum identity, complete-graph closed form), a wrong sign or a missing factor in the
mixer (dense expm, Eq. (2) form, closed form), a swapped round order (dense brute force at
p >= 2, and at n > 8 the light cone on cycles), or a wrong inner product in the adjoint
(closed-form derivative, finite differences, zero-gradient identities).
"""
from math import comb

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads
from tests import pins


def _er(n, seed, weights=None):
    return workloads.erdos_renyi(n, seed, 0.5, weights)


# ---------------------------------------------------------------- cost table (step a)

@pytest.mark.parametrize("g", [workloads.random_regular_graph(10, 3, 7), _er(12, 3, (1, 4)),
                               workloads.random_regular_graph(16, 3, 11)])
def test_table_sum_identity(g):
    # every edge is cut in exactly half of all 2^n strings: sum_x C(x) = W 2^(n-1)
    t = oracle.graph_table(g)
    assert t.sum() == g.total_weight * 2 ** (g.n - 1)


def test_table_complement_symmetry():
    g = _er(11, 5, (1, 4))
    t = oracle.graph_table(g)
    x = np.arange(1 << g.n)
    assert np.array_equal(t, t[x ^ ((1 << g.n) - 1)])


def test_table_complete_graph_closed_form():
    # K_n: a string with h ones cuts exactly h (n - h) edges
    n = 9
    iu, ju = np.triu_indices(n, 1)
    t = oracle.cost_table(n, iu, ju)
    h = np.array([bin(x).count("1") for x in range(1 << n)])
    assert np.array_equal(t, h * (n - h))


def test_table_single_edge_is_bit_xor():
    n = 7
    for a, b in [(0, 6), (3, 4), (5, 1)]:
        t = oracle.cost_table(n, [a], [b])
        x = np.arange(1 << n)
        assert np.array_equal(t, ((x >> a) ^ (x >> b)) & 1)


def test_table_hamming_weight_subspace():
    g = _er(12, 9, (1, 3))
    for k in (1, 5, 6):
        st = oracle.states(g.n, k)
        assert st.size == comb(g.n, k)
        assert np.all(np.diff(st.astype(np.int64)) > 0)              # increasing order
        assert all(bin(int(x)).count("1") == k for x in st[:50])
        tk = oracle.cost_table(g.n, g.u, g.v, g.w, k)
        # an edge is cut by exactly 2 C(n-2, k-1) weight-k strings
        assert tk.sum() == g.total_weight * 2 * comb(g.n - 2, k - 1)
        assert np.array_equal(tk, oracle.graph_table(g)[st.astype(np.int64)])


# ---------------------------------------------------------------- X mixer (step c)

@pytest.mark.parametrize("n", [1, 3, 6])
def test_x_mixer_matches_dense_expm(n):
    rng = np.random.default_rng(n)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    beta = 0.7312
    want = scipy.linalg.expm(-1j * beta * pins.dense_x_mixer_hamiltonian(n)) @ psi
    got = psi.copy()
    oracle.apply_x_mixer(n, beta, got)
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def test_x_mixer_equation_2_hadamard_form():
    # Eq. (2): e^{-i b sum X} = H^n diag(e^{-i b (n - 2|y|)}) H^n
    n = 7
    Hd = scipy.linalg.hadamard(1 << n) / 2 ** (n / 2)
    pop = np.array([bin(y).count("1") for y in range(1 << n)])
    beta = 2.2
    rng = np.random.default_rng(3)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    want = Hd @ (np.exp(-1j * beta * (n - 2 * pop)) * (Hd @ psi))
    got = psi.copy()
    oracle.apply_x_mixer(n, beta, got)
    assert np.max(np.abs(got - want)) < 1e-12


def test_x_sum_is_sum_of_flips():
    n = 6
    rng = np.random.default_rng(4)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    want = pins.dense_x_mixer_hamiltonian(n) @ psi
    assert np.max(np.abs(oracle.apply_x_sum(n, psi) - want)) < 1e-12


def test_norm_preserved():
    W = workloads.workload("maxcut3reg_n10_p3")
    g = W.graphs[0]
    t = oracle.graph_table(g)
    rng = np.random.default_rng(0)
    for _ in range(3):
        a = rng.uniform(-np.pi, np.pi, 10)
        E, N = oracle.expect(g.n, t, a)
        assert abs(N - 1) < 1e-13


# ---------------------------------------------------------------- <C> (step d), Eq. (1)

P1_GRAPHS = [workloads.random_regular_graph(10, 3, 1), workloads.random_regular_graph(12, 3, 2),
             _er(8, 17), _er(9, 18), workloads.random_regular_graph(8, 5, 3)]


@pytest.mark.parametrize("g", P1_GRAPHS)
def test_p1_closed_form_expectation_and_gradient(g):
    t = oracle.graph_table(g)
    edges = list(zip(g.u.tolist(), g.v.tolist()))
    rng = np.random.default_rng(g.n)
    for _ in range(4):
        beta, gamma = rng.uniform(0, np.pi, 2)
        Ecf, dbeta, dgamma = pins.maxcut_p1(g.n, edges, beta, gamma)
        E, N, gr = oracle.grad(g.n, t, [beta, gamma])
        assert abs(E - Ecf) < 1e-12 * max(1, abs(Ecf))
        assert abs(gr[0] - dbeta) < 1e-11 * max(1, abs(dbeta))
        assert abs(gr[1] - dgamma) < 1e-11 * max(1, abs(dgamma))


def test_zero_angles_give_uniform_mean():
    g = _er(10, 21, (1, 4))
    t = oracle.graph_table(g)
    rng = np.random.default_rng(1)
    p = 3
    for which in ("beta", "gamma"):
        a = rng.uniform(0, np.pi, 2 * p)
        if which == "beta":
            a[:p] = 0
        else:
            a[p:] = 0
        E, N, gr = oracle.grad(g.n, t, a)
        assert abs(E - g.total_weight / 2) < 1e-12 * g.total_weight
        # at beta = 0 nothing depends on gamma; at gamma = 0 nothing depends on beta
        zero = gr[p:] if which == "beta" else gr[:p]
        assert np.max(np.abs(zero)) < 1e-12 * g.total_weight


def test_symmetries():
    g = workloads.random_regular_graph(10, 3, 5)
    t = oracle.graph_table(g)
    rng = np.random.default_rng(2)
    p = 3
    a = rng.uniform(0, np.pi, 2 * p)
    E, N, gr = oracle.grad(g.n, t, a)
    # beta_k -> beta_k + pi/2 multiplies the state by a product of X's (C(x) = C(~x))
    b = a.copy(); b[1] += np.pi / 2
    assert abs(oracle.expect(g.n, t, b)[0] - E) < 1e-12
    # gamma_k -> gamma_k + 2 pi (integer C)
    b = a.copy(); b[p + 2] += 2 * np.pi
    assert abs(oracle.expect(g.n, t, b)[0] - E) < 1e-12
    # (beta, gamma) -> (-beta, -gamma) is complex conjugation: same <C>, gradient flips sign
    E2, N2, gr2 = oracle.grad(g.n, t, -a)
    assert abs(E2 - E) < 1e-12
    assert np.max(np.abs(gr2 + gr)) < 1e-11


@pytest.mark.parametrize("n,p", [(5, 2), (7, 3), (8, 2)])
def test_state_matches_dense_bruteforce(n, p):
    g = _er(n, 100 + n, (1, 3))
    t = oracle.graph_table(g)
    a = workloads.random_angles(p, 1, 7 + n)[0]
    psi0 = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    want = pins.dense_evolve(pins.dense_x_mixer_hamiltonian(n), t, a, psi0)
    got = oracle.state(n, t, a)
    assert np.max(np.abs(got - want)) < 1e-13


def test_custom_initial_state():
    n, p = 6, 2
    g = _er(n, 55)
    t = oracle.graph_table(g)
    rng = np.random.default_rng(8)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    a = rng.uniform(0, np.pi, 2 * p)
    want = pins.dense_evolve(pins.dense_x_mixer_hamiltonian(n), t, a, psi0)
    assert np.max(np.abs(oracle.state(n, t, a, psi0=psi0) - want)) < 1e-13


# ---------------------------------------------------------------- gradient (adjoint vs FD)

def test_adjoint_gradient_matches_finite_differences():
    W = workloads.workload("maxcut3reg_n10_p3")
    g = W.graphs[0]
    t = oracle.graph_table(g)
    for a in workloads.random_angles(4, 3, 99):
        E, N, gr = oracle.grad(g.n, t, a)
        fd = oracle.fd_grad(g.n, t, a)
        assert np.max(np.abs(gr - fd)) < 1e-9 * max(1, np.max(np.abs(gr)))


@pytest.mark.parametrize("n,p", [(12, 2), (15, 3)])
def test_cycle_light_cone_pins_large_n(n, p):
    """Light cone (Farhi, Goldstone and Gutmann, arXiv:1411.4028): after p rounds the term of
    edge (u, v) involves only the qubits within distance p of the edge and the edges touching
    qubits within distance p - 1. On the cycle C_n (n >= 2p + 3) every edge therefore sees a
    path of 2p + 2 vertices, so <C>(C_n) = n * P(middle edge cut) on the path P_{2p+2}, the
    latter by dense matrix exponentials on 2p + 2 qubits. Pins the oracle's evolution and its
    adjoint gradient at p >= 2 and n > 8, where no other closed form or brute force reaches."""
    u = np.arange(n)
    t = oracle.cost_table(n, u, (u + 1) % n)
    for a in workloads.random_angles(p, 2, 4100 + n):
        E, Nr, g = oracle.grad(n, t, a)
        ev, fd = pins.cycle_edge(p, a)
        assert abs(E / Nr - n * ev) < 1e-11 * n
        assert np.max(np.abs(g / Nr - n * fd)) < 1e-7 * n


def test_light_cone_pins_weighted_regular_graph_p2():
    """The same light cone on a graph that is not a cycle: a weighted random 3-regular graph
    on 20 vertices at p = 2, where each edge's ball holds at most 14 qubits. Every edge term is
    evolved on its ball with scipy's expm_multiply on the sparse sum of X; their weighted sum
    pins the oracle's <C> and its adjoint gradient (central differences of the sum)."""
    g = workloads.random_regular_graph(20, 3, 4200)
    w = np.random.default_rng(4201).integers(1, 4, g.u.size).astype(np.int32)
    t = oracle.cost_table(20, g.u, g.v, w)
    for a in workloads.random_angles(2, 1, 4202):
        E, Nr, gr = oracle.grad(20, t, a)
        ev, fd = pins.light_cone_expect(20, g.u, g.v, w, 2, a)
        scale = float(w.sum())
        assert abs(E / Nr - ev) < 1e-10 * scale
        assert np.max(np.abs(gr / Nr - fd)) < 1e-7 * scale


def test_light_cone_pins_circular_ladder_p3():
    """p = 3 on a graph that is not a cycle: the circular ladder (prism) on 2 x 10 vertices,
    3-regular with weights 1..3, where the ball of radius 3 around any edge holds 14 qubits
    (8 consecutive rungs' worth, no wrap-around). <C> and the d/dbeta_1 entry of the gradient
    from the light-cone sum."""
    L = 10
    u = [i for i in range(L)] + [i for i in range(L)] + [L + i for i in range(L)]
    v = [(i + 1) % L for i in range(L)] + [L + i for i in range(L)] + [L + (i + 1) % L for i in range(L)]
    u, v = np.array([min(a, b) for a, b in zip(u, v)]), np.array([max(a, b) for a, b in zip(u, v)])
    w = np.random.default_rng(4301).integers(1, 4, u.size).astype(np.int32)
    n = 2 * L
    t = oracle.cost_table(n, u, v, w)
    a = workloads.random_angles(3, 1, 4302)[0]
    E, Nr, gr = oracle.grad(n, t, a)
    ev, fd = pins.light_cone_expect(n, u, v, w, 3, a, components=[0])
    scale = float(w.sum())
    assert abs(E / Nr - ev) < 1e-10 * scale
    assert abs(gr[0] / Nr - fd[0]) < 1e-7 * scale


def test_cycle_light_cone_pins_headline_depth():
    """The light cone at the benchmark's depth p = 8: on the cycles C_20 and C_24 (both
    >= 2p + 3) <C> is n times the middle-edge cut probability of the path of 18 vertices,
    evolved with the mixer as a product of dense exponentials over blocks of qubits
    (``pins.cycle_edge_blocks``; 2^18 amplitudes, no oracle code). Pins the oracle's <C> and
    three entries of its adjoint gradient (d/dbeta_1, d/dbeta_8, d/dgamma_1; central
    differences of the light-cone value) at the p of the headline workload."""
    p = 8
    a = workloads.random_angles(p, 1, 4800)[0]
    comps = [0, p - 1, p]
    ev, fd = pins.cycle_edge_blocks(p, a, components=comps)
    for n in (20, 24):
        u = np.arange(n)
        t = oracle.cost_table(n, u, (u + 1) % n)
        E, Nr, g = oracle.grad(n, t, a)
        assert abs(E / Nr - n * ev) < 1e-10 * n
        for i in comps:
            assert abs(g[i] / Nr - n * fd[i]) < 1e-7 * n


# ---------------------------------------------------------------- clique mixer

@pytest.mark.parametrize("n,k", [(4, 2), (6, 3), (7, 2)])
def test_clique_matrix_is_pauli_sum_restricted(n, k):
    H = pins.dense_clique_hamiltonian(n)
    st = oracle.states(n, k).astype(np.int64)
    # no leakage: H maps weight-k strings only to weight-k strings
    mask = np.zeros(1 << n, bool); mask[st] = True
    assert np.max(np.abs(H[np.ix_(~mask, mask)])) == 0
    Hk = H[np.ix_(st, st)]
    nb = oracle.clique_neighbours(n, k)
    M = np.zeros((st.size, st.size))
    for r in range(st.size):
        for j in nb[r]:
            M[r, j] += 2
    assert np.max(np.abs(Hk - M)) < 1e-14


@pytest.mark.parametrize("n,k", [(8, 4), (10, 5), (10, 3)])
def test_clique_johnson_spectrum(n, k):
    nb = oracle.clique_neighbours(n, k)
    N = nb.shape[0]
    M = np.zeros((N, N))
    for r in range(N):
        M[r, nb[r]] += 2
    ev = np.linalg.eigvalsh(M)
    assert np.max(np.abs(np.sort(ev) - pins.johnson_spectrum(n, k))) < 1e-10


def test_clique_mixer_matches_expm():
    n, k = 8, 4
    nb = oracle.clique_neighbours(n, k)
    N = nb.shape[0]
    M = np.zeros((N, N))
    for r in range(N):
        M[r, nb[r]] += 2
    rng = np.random.default_rng(1)
    psi = rng.normal(size=N) + 1j * rng.normal(size=N)
    for beta in (0.3, 2.9):
        want = scipy.linalg.expm(-1j * beta * M) @ psi
        got = psi.copy()
        oracle.apply_clique_mixer(n, k, beta, got, nb)
        assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_clique_dicke_state_is_top_eigenvector():
    # the Dicke state has eigenvalue 2k(n-k): at gamma = 0 it only picks up a phase
    g = _er(10, 31)
    n, k = 10, 5
    t = oracle.cost_table(n, g.u, g.v, g.w, k)
    a = np.array([0.4, 1.3, 0.0, 0.0])
    E, N = oracle.expect(n, t, a, k=k)
    assert abs(E - g.total_weight * 2 * comb(n - 2, k - 1) / comb(n, k)) < 1e-12 * g.total_weight


def test_clique_qaoa_matches_full_space_bruteforce():
    n, k, p = 8, 4, 3
    g = _er(n, 41)
    st = oracle.states(n, k).astype(np.int64)
    tfull = oracle.graph_table(g)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[st] = 1 / np.sqrt(st.size)                     # Dicke state |D^n_k>
    a = workloads.random_angles(p, 1, 5)[0]
    want = pins.dense_evolve(pins.dense_clique_hamiltonian(n), tfull, a, psi0)
    got = oracle.state(n, tfull[st], a, k=k)
    assert np.max(np.abs(want[st] - got)) < 1e-12
    mask = np.ones(1 << n, bool); mask[st] = False
    assert np.max(np.abs(want[mask])) < 1e-12          # evolution never leaves weight k


def test_clique_gradient_matches_finite_differences():
    n, k, p = 8, 4, 2
    g = _er(n, 43)
    t = oracle.cost_table(n, g.u, g.v, g.w, k)
    a = workloads.random_angles(p, 1, 6)[0]
    E, N, gr = oracle.grad(n, t, a, k=k)
    fd = oracle.fd_grad(n, t, a, k=k)
    assert np.max(np.abs(gr - fd)) < 1e-8 * max(1, np.max(np.abs(gr)))


# ---------------------------------------------------------------- arbitrary objective values

def _real_table(N, seed, distinct=None):
    """Real, non-integer, complement-asymmetric values (optionally drawn from a small set)."""
    rng = np.random.default_rng(seed)
    if distinct is None:
        return rng.normal(1.5, 2.0, N)
    pool = rng.normal(0.0, 3.0, distinct)
    return pool[rng.integers(0, distinct, N)]


@pytest.mark.parametrize("n,p", [(5, 3), (7, 2)])
def test_real_asymmetric_cost_matches_dense_bruteforce(n, p):
    # Sec. 3: the objective is any list of values over the states; Eq. (1) by dense expm
    t = _real_table(1 << n, 300 + n)
    assert np.max(np.abs(t - t[::-1])) > 0.1                      # C(~x) != C(x)
    a = workloads.random_angles(p, 1, 301 + n)[0]
    psi0 = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    want = pins.dense_evolve(pins.dense_x_mixer_hamiltonian(n), t, a, psi0)
    assert np.max(np.abs(oracle.state(n, t, a) - want)) < 1e-13
    E, N = oracle.expect(n, t, a)
    assert abs(E - np.sum(np.abs(want) ** 2 * t)) < 1e-12 * np.sum(np.abs(t))


def test_real_cost_gradient_matches_finite_differences():
    n, p = 8, 3
    t = _real_table(1 << n, 310, distinct=40)
    a = workloads.random_angles(p, 1, 311)[0]
    E, N, gr = oracle.grad(n, t, a)
    fd = oracle.fd_grad(n, t, a)
    assert np.max(np.abs(gr - fd)) < 1e-9 * max(1, np.max(np.abs(gr)))
    # a constant shift of C shifts <C> and leaves the gradient unchanged (the adjoint starts
    # from (C + s) psi_p; the extra s psi_p term has real inner products)
    E2, N2, gr2 = oracle.grad(n, t + 7.25, a)
    assert abs(E2 / N2 - E / N - 7.25) < 1e-12
    assert np.max(np.abs(gr2 - gr)) < 1e-11 * max(1, np.max(np.abs(gr)))


def test_real_cost_clique_matches_full_space_bruteforce():
    n, k, p = 7, 3, 2
    st = oracle.states(n, k).astype(np.int64)
    tfull = _real_table(1 << n, 320)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[st] = 1 / np.sqrt(st.size)
    a = workloads.random_angles(p, 1, 321)[0]
    want = pins.dense_evolve(pins.dense_clique_hamiltonian(n), tfull, a, psi0)
    got = oracle.state(n, tfull[st], a, k=k)
    assert np.max(np.abs(want[st] - got)) < 1e-12


# ---------------------------------------------------------------- Grover mixer (Sec. 2.4)

def _projector_uniform(N):
    u = np.full(N, 1 / np.sqrt(N), dtype=np.complex128)
    return np.outer(u, u.conj())


@pytest.mark.parametrize("N", [64, 70])
def test_grover_mixer_matches_expm(N):
    rng = np.random.default_rng(N)
    psi = rng.normal(size=N) + 1j * rng.normal(size=N)
    for beta in (0.3, 1.7, -2.4):
        want = scipy.linalg.expm(-1j * beta * _projector_uniform(N)) @ psi
        got = psi.copy()
        oracle.apply_grover_mixer(beta, got)
        assert np.max(np.abs(got - want)) < 1e-13


@pytest.mark.parametrize("n,k,p", [(6, -1, 3), (8, 3, 2)])
def test_grover_qaoa_matches_dense(n, k, p):
    N = (1 << n) if k < 0 else comb(n, k)
    t = _real_table(N, 330 + n)
    a = workloads.random_angles(p, 1, 331 + n)[0]
    psi0 = np.full(N, 1 / np.sqrt(N), dtype=np.complex128)
    want = pins.dense_evolve(_projector_uniform(N), t, a, psi0)
    assert np.max(np.abs(oracle.state(n, t, a, k=k, grover=True) - want)) < 1e-13


def test_grover_fair_sampling():
    # states with equal cost keep equal amplitudes (Sec. 2.4, third property)
    g = _er(10, 77, (1, 3))
    t = oracle.graph_table(g)
    psi = oracle.state(10, t, workloads.random_angles(4, 1, 78)[0], grover=True)
    for c in np.unique(t):
        cls = psi[t == c]
        assert np.max(np.abs(cls - cls[0])) < 1e-14


def test_grover_p1_closed_form_from_degeneracies():
    # p = 1: psi(x) = (e^{-i g C(x)} + (e^{-i b} - 1) F(g)) / sqrt(N) with F(g) the mean of
    # e^{-i g C} over the states, so <C> = sum_c m_c c |e^{-i g c} + (e^{-i b} - 1) F|^2 / N
    g = _er(9, 79, (1, 4))
    t = oracle.graph_table(g)
    vals, cnt = oracle.degeneracies(t)
    assert cnt.sum() == 1 << 9 and np.array_equal(vals, np.unique(t))
    N = cnt.sum()
    for b, gm in ((0.4, 1.1), (2.2, 0.35), (1.57, 2.9)):
        F = np.sum(cnt * np.exp(-1j * gm * vals)) / N
        amp = np.exp(-1j * gm * vals) + (np.exp(-1j * b) - 1) * F
        want = np.sum(cnt * vals * np.abs(amp) ** 2) / N
        E, Nr = oracle.expect(9, t, [b, gm], grover=True)
        assert abs(E - want) < 1e-12 * abs(want) and abs(Nr - 1) < 1e-13


def test_grover_gradient_matches_finite_differences():
    for n, k in ((8, -1), (9, 4)):
        N = (1 << n) if k < 0 else comb(n, k)
        t = _real_table(N, 340 + n, distinct=25)
        a = workloads.random_angles(3, 1, 341 + n)[0]
        E, Nr, gr = oracle.grad(n, t, a, k=k, grover=True)
        fd = oracle.fd_grad(n, t, a, k=k, grover=True)
        assert np.max(np.abs(gr - fd)) < 1e-9 * max(1, np.max(np.abs(gr)))


# ---------------------------------------------------------------- ring mixer, matrix mixers

@pytest.mark.parametrize("n,k", [(5, 2), (6, 3), (2, 1)])
def test_ring_matrix_is_pauli_sum_restricted(n, k):
    st = oracle.states(n, k).astype(np.int64)
    Hd = pins.dense_ring_hamiltonian(n)[np.ix_(st, st)]
    nb = oracle.ring_neighbours(n, k)
    Hn = np.zeros((st.size, st.size))
    for r in range(st.size):
        for j in nb[r]:
            if j >= 0:
                Hn[j, r] += 2.0
    assert np.max(np.abs(Hd - Hn)) == 0
    # the Pauli sum never leaves weight k
    full = pins.dense_ring_hamiltonian(n)
    off = np.setdiff1d(np.arange(1 << n), st)
    assert np.max(np.abs(full[np.ix_(off, st)])) == 0


def test_ring_qaoa_matches_full_space_bruteforce():
    n, k, p = 7, 3, 3
    st = oracle.states(n, k).astype(np.int64)
    tfull = _real_table(1 << n, 350)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[st] = 1 / np.sqrt(st.size)
    a = workloads.random_angles(p, 1, 351)[0]
    want = pins.dense_evolve(pins.dense_ring_hamiltonian(n), tfull, a, psi0)
    got = oracle.state(n, tfull[st], a, k=k, ring=True)
    assert np.max(np.abs(want[st] - got)) < 1e-12


def test_ring_gradient_and_dense_matrix_reference():
    n, k, p = 8, 4, 2
    st = oracle.states(n, k).astype(np.int64)
    t = _real_table(st.size, 360, distinct=30)
    a = workloads.random_angles(p, 1, 361)[0]
    E, N, gr = oracle.grad(n, t, a, k=k, ring=True)
    assert np.max(np.abs(gr - oracle.fd_grad(n, t, a, k=k, ring=True))) < 1e-9 * max(1, np.max(np.abs(gr)))
    # the dense-matrix reference (scipy expm on the restricted matrix) agrees with the C
    # oracle's sparse Taylor path, for the ring and the clique mixer
    for H, kw in ((pins.dense_ring_hamiltonian(n), {"ring": True}), (pins.dense_clique_hamiltonian(n), {})):
        Hr = np.real(H[np.ix_(st, st)])
        E0, N0, g0 = oracle.grad(n, t, a, k=k, **kw)
        E1, N1, g1 = oracle.dense_mixer_grad(t, a, Hr)
        assert abs(E0 - E1) < 1e-12 * np.sum(np.abs(t)) and np.max(np.abs(g0 - g1)) < 1e-11 * max(1, np.max(np.abs(g0)))
