"""Pins of the X-product and per-qubit multi-angle oracle (Sec. 2.1 Eq. (2); Sec. 3). Each
would fail for a plausible slip: a wrong sign or factor in the Walsh-Hadamard transform or in
the diagonal (dense brute force, k = 1 equal to the transverse field, X^{(x)n} closed form),
a wrong Krawtchouk term (symmetric sums built from all k-subsets), a wrong order or a
transposed rotation (dense expm at p >= 2), or a wrong inner product in the adjoint (finite
differences, equal per-qubit angles summing to the single-angle derivative)."""
import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads
from oracle import xmixers as X


def _dense_evolve(H_M, table, betas, gammas):
    N = table.size
    psi = np.full(N, 1 / np.sqrt(N), dtype=np.complex128)
    for b, g in zip(betas, gammas):
        psi = np.exp(-1j * g * table) * psi
        psi = scipy.linalg.expm(-1j * b * H_M) @ psi
    return psi


@pytest.mark.parametrize("n,orders", [(5, [1]), (5, [2]), (6, [1, 3]), (4, [4]), (6, [2, 4, 5])])
def test_orders_diagonal_matches_dense(n, orders):
    masks = [m for k in orders for m in X.all_masks_of_order(n, k)]
    H = X.dense_x_products(n, masks, [1.0] * len(masks))
    d = X.diag_orders(n, orders)
    W = np.array([X.wht(np.eye(1 << n)[i]) for i in range(1 << n)]).T
    assert np.allclose(W @ np.diag(d) @ W, H, atol=1e-12)
    assert np.allclose(X.diag_terms(n, masks, [1.0] * len(masks)), d)


def test_krawtchouk_values():
    # K_1(w) = n - 2w; K_n(w) = (-1)^w; sum_k K_k(w) = 2^n [w = 0]
    for n in (3, 6, 9):
        for w in range(n + 1):
            assert X.krawtchouk(n, 1, w) == n - 2 * w
            assert X.krawtchouk(n, n, w) == (-1) ** w
            assert sum(X.krawtchouk(n, k, w) for k in range(n + 1)) == (2 ** n if w == 0 else 0)


@pytest.mark.parametrize("n,masks,coefs,p", [
    (5, [0b1, 0b110, 0b10101], [1.0, -0.5, 2.0], 2),
    (6, [0b111111, 0b11, 0b100100], [0.3, 1.0, -1.2], 3),
])
def test_terms_evolution_matches_dense(n, masks, coefs, p):
    g = workloads.erdos_renyi(n, 2700 + n, 0.5, (1, 3))
    t = oracle.graph_table(g).astype(np.float64)
    a = workloads.random_angles(p, 1, 2701)[0]
    d = X.diag_terms(n, masks, coefs)
    E, Nr, _ = X.grad(n, t, a, d=d)
    psi = _dense_evolve(X.dense_x_products(n, masks, coefs), t, a[:p], a[p:])
    assert abs(E - np.sum(np.abs(psi) ** 2 * t)) <= 1e-11 * t.max() and abs(Nr - 1) <= 1e-12


def test_order_one_is_the_transverse_field():
    n = 7
    g = workloads.erdos_renyi(n, 2710, 0.5, (1, 3))
    t = oracle.graph_table(g)
    for a in workloads.random_angles(3, 3, 2711):
        E, Nr, gr = X.grad(n, t, a, d=X.diag_orders(n, [1]))
        E0, N0, g0 = oracle.grad(n, t, a)
        assert abs(E - E0) <= 1e-11 * t.max() and np.max(np.abs(gr - g0)) <= 1e-10 * np.max(np.abs(g0))


def test_all_qubit_product_closed_form():
    # e^{-i b X^{(x)n}} = cos b I - i sin b X^{(x)n}; p = 1 from the uniform state (an eigenvector
    # of X^{(x)n} with eigenvalue 1 after the phase is not needed: check the state directly)
    n = 5
    rng = np.random.default_rng(2720)
    t = rng.integers(0, 7, 1 << n).astype(np.float64)
    b, gm = 0.37, 0.81
    psi = np.exp(-1j * gm * t) / np.sqrt(1 << n)
    flipped = psi[::-1]                         # X^{(x)n} maps x to its complement
    want = np.cos(b) * psi - 1j * np.sin(b) * flipped
    d = X.diag_orders(n, [n])
    got = X._mixer(psi, b, d)
    assert np.allclose(got, want, atol=1e-14)


@pytest.mark.parametrize("multi", [False, True])
def test_gradient_matches_finite_differences(multi):
    n, p = 6, 3
    g = workloads.erdos_renyi(n, 2730, 0.5, (1, 3))
    t = oracle.graph_table(g).astype(np.float64)
    rng = np.random.default_rng(2731)
    a = rng.uniform(0, np.pi, p * (n + 1) if multi else 2 * p)
    d = None if multi else X.diag_terms(n, [0b11, 0b101010, 0b1], [1.0, 0.7, -0.4])
    E, Nr, gr = X.grad(n, t, a, d=d, multiangle=multi)
    h = 1e-6
    fd = np.array([(X.grad(n, t, a + h * e, d=d, multiangle=multi)[0] -
                    X.grad(n, t, a - h * e, d=d, multiangle=multi)[0]) / (2 * h) for e in np.eye(a.size)])
    assert np.max(np.abs(gr - fd)) <= 1e-7 * np.max(np.abs(fd))


def test_multiangle_reduces_to_single_angle():
    n, p = 6, 3
    g = workloads.erdos_renyi(n, 2740, 0.5, (1, 3))
    t = oracle.graph_table(g)
    a = workloads.random_angles(p, 1, 2741)[0]
    ma = np.concatenate([np.repeat(a[:p], n), a[p:]])
    E, Nr, gm = X.grad(n, t, ma, multiangle=True)
    E0, N0, g0 = oracle.grad(n, t, a)
    assert abs(E - E0) <= 1e-12 * t.max()
    # the single-angle derivative is the sum of the per-qubit ones
    assert np.allclose(gm[:p * n].reshape(p, n).sum(axis=1), g0[:p], atol=1e-11)
    assert np.allclose(gm[p * n:], g0[p:], atol=1e-11)


def test_multiangle_matches_dense_per_qubit():
    n, p = 4, 2
    rng = np.random.default_rng(2750)
    t = rng.integers(0, 5, 1 << n).astype(np.float64)
    a = rng.uniform(0, np.pi, p * (n + 1))
    psi = np.full(1 << n, 1 / 4, dtype=np.complex128)
    for k in range(p):
        psi = np.exp(-1j * a[p * n + k] * t) * psi
        Hk = X.dense_x_products(n, [1 << q for q in range(n)], a[k * n:(k + 1) * n])
        psi = scipy.linalg.expm(-1j * Hk) @ psi
    E, Nr, _ = X.grad(n, t, a, multiangle=True)
    assert abs(E - np.sum(np.abs(psi) ** 2 * t)) <= 1e-12 * t.max()
