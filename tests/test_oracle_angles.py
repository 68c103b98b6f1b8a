"""Pins of the oracle's angle-finding routines (Sec. 2.3; CPU only).

Each would fail for a plausible slip: a wrong constant or shift in the counter-based
generator (published SplitMix64 outputs), a wrong weight or index in the round seeding
(INTERP keeps endpoints and resamples straight lines exactly), a wrong sign or transposition
in the BFGS update or the line search (Rosenbrock and quadratic minima, known closed forms),
a broken acceptance rule in basinhopping (a double well whose global minimum is known), or a
seeding that loses the previous round (the zero layer is the identity, and rounds never get
worse)."""
import numpy as np
import pytest
import scipy.optimize

import oracle
import workloads
from oracle import angles as A
from tests import pins


def test_splitmix64_published_outputs():
    # Outputs 1-3 of SplitMix64 from state 0 (the generator of Steele, Lea and Flood, 2014).
    assert A.splitmix64_sequence(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_draws_are_uniform_and_keyed():
    u = np.array([A.uniform(7, 3, c, h, j) for c in range(20) for h in range(-1, 9) for j in range(10)])
    assert np.all((u >= 0) & (u < 1))
    assert abs(u.mean() - 0.5) < 0.03 and abs(u.var() - 1 / 12) < 0.01
    assert len(set(u.tolist())) == u.size                      # distinct keys, distinct draws
    assert A.uniform(7, 3, 1, 2, 0) != A.uniform(8, 3, 1, 2, 0) != A.uniform(7, 4, 1, 2, 0)


@pytest.mark.parametrize("q", [1, 2, 3, 7])
def test_interp_endpoints_and_lines(q):
    rng = np.random.default_rng(q)
    a = rng.uniform(0, 1, q)
    b = A.interp(a)
    assert b.size == q + 1 and b[0] == a[0] and b[-1] == a[-1]
    if q >= 2:
        u, v = 0.3, 1.1                                        # a straight line sampled at q points
        line = u + v * np.arange(q) / (q - 1)
        assert np.allclose(A.interp(line), u + v * np.arange(q + 1) / q, atol=1e-15)
    assert np.allclose(A.interp(np.full(q, 0.7)), 0.7, atol=1e-15)
    if q == 2:
        assert np.allclose(b, [a[0], (a[0] + a[1]) / 2, a[1]])


def test_bfgs_rosenbrock_and_quadratic():
    def rosen(x):
        f = 100 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
        g = np.array([-400 * x[0] * (x[1] - x[0] ** 2) - 2 * (1 - x[0]), 200 * (x[1] - x[0] ** 2)])
        return f, g
    x, f, it = A.bfgs(rosen, [-1.2, 1.0], gtol=1e-8, max_iter=500)
    assert np.allclose(x, [1, 1], atol=1e-7) and f < 1e-14 and 10 < it < 200
    rng = np.random.default_rng(5)
    M = rng.normal(size=(6, 6))
    Q = M @ M.T + 6 * np.eye(6)
    b = rng.normal(size=6)
    x, f, it = A.bfgs(lambda x: (0.5 * x @ Q @ x - b @ x, Q @ x - b), np.zeros(6), gtol=1e-10, max_iter=200)
    assert np.allclose(x, np.linalg.solve(Q, b), atol=1e-9) and it <= 40


def test_basinhopping_finds_the_global_well():
    # f = 0.05 x^2 - cos(3 x): global minimum -1 at x = 0, local minima near +-2.1, +-4.2
    fun = lambda x: (0.05 * x[0] ** 2 - np.cos(3 * x[0]), np.array([0.1 * x[0] + 3 * np.sin(3 * x[0])]))
    x, f, _ = A.bfgs(fun, [4.3])
    assert abs(x[0]) > 3.5                                     # plain BFGS stays in its well
    bx, bf = A.basinhopping(fun, [[4.3], [4.3]], 1, seed=11, n_hops=30, step=1.5, temperature=0.5)
    assert abs(bx[0]) < 1e-6 and abs(bf + 1) < 1e-12
    # temperature 0 accepts improvements only: the best is never above the first minimum
    bx0, bf0 = A.basinhopping(fun, [[4.3]], 1, seed=11, n_hops=5, step=0.3, temperature=0.0)
    assert bf0 <= f + 1e-15


def test_zero_layer_is_the_identity():
    g = workloads.erdos_renyi(7, 2301, 0.5, (1, 3))
    t = oracle.graph_table(g)
    for a in workloads.random_angles(2, 3, 2302):
        e1, _ = oracle.expect(7, t, a)
        e2, _ = oracle.expect(7, t, A.pad_zero_layer(a))
        assert abs(e1 - e2) <= 1e-12 * abs(e1)


def test_round_one_reaches_the_closed_form_optimum():
    # p = 1 MaxCut: the closed-form <C>(beta, gamma) on a dense grid, polished, is the global optimum
    n = 7
    g = workloads.erdos_renyi(n, 2311, 0.5)
    edges = list(zip(g.u.tolist(), g.v.tolist()))
    bs, gs = np.linspace(0, np.pi, 181), np.linspace(0, 2 * np.pi, 361)
    grid = np.array([[pins.maxcut_p1(n, edges, b, c)[0] for c in gs] for b in bs])
    i, j = np.unravel_index(np.argmax(grid), grid.shape)
    res = scipy.optimize.minimize(lambda x: -pins.maxcut_p1(n, edges, x[0], x[1])[0], [bs[i], gs[j]],
                                  jac=lambda x: -np.array(pins.maxcut_p1(n, edges, x[0], x[1])[1:]),
                                  method="BFGS", options={"gtol": 1e-12})
    best = -res.fun
    t = oracle.graph_table(g)
    ang, vals = A.find_angles(lambda r: A.Objective(n, t), 1, seed=3, n_chains=4, n_hops=4)
    assert abs(vals[0] - best) <= 1e-9 * best
    e, dEb, dEg = pins.maxcut_p1(n, edges, *ang[0])
    assert abs(e - vals[0]) <= 1e-9 * best and max(abs(dEb), abs(dEg)) < 1e-5


def test_rounds_never_get_worse_and_end_at_optima():
    n = 6
    g = workloads.erdos_renyi(n, 2321, 0.5, (1, 3))
    t = oracle.graph_table(g)
    ang, vals = A.find_angles(lambda r: A.Objective(n, t), 3, seed=5, n_chains=3, n_hops=2, gtol=1e-7)
    assert np.all(np.diff(vals) >= -1e-12)
    for r, a in enumerate(ang, start=1):
        assert a.size == 2 * r
        E, Nr, gr = oracle.grad(n, t, a)
        assert abs(E / Nr - vals[r - 1]) <= 1e-12 * vals[r - 1]
        assert np.max(np.abs(gr)) < 1e-5
    # minimisation: the same problem with maximize=False finds values below the mean
    _, lo = A.find_angles(lambda r: A.Objective(n, t, maximize=False), 1, seed=5, n_chains=3, n_hops=2,
                          maximize=False)
    assert lo[0] < np.mean(t) < vals[0]


def test_random_restarts_take_the_best():
    n = 6
    g = workloads.erdos_renyi(n, 2331, 0.5)
    t = oracle.graph_table(g)
    x, v, allv = A.find_angles_random(A.Objective(n, t), 2, 6, seed=9)
    assert v == np.max(allv) and allv.size == 6
    assert abs(oracle.expect(n, t, x)[0] - v) <= 1e-12 * v
