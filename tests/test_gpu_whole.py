"""GPU parity of the register-resident whole-state kernel (n = 12, 13 in FP32; n = 12 in
FP64) against the FP64 oracle: one-byte and two-byte tables, symmetric (MaxCut) and
asymmetric value tables, angles on both sides of |sin beta| = |cos beta| (the flipped and the
plain rotation form), p from 1 to 10, single and batched calls. Tolerances: FP32 1e-5, FP64
1e-10, relative to max|C| for <C> and to max|g| for the gradient."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
TOL = {0: 1e-5, 1: 1e-10}


@pytest.fixture(scope="module")
def q():
    import paper_2312_06451_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def _angles(p, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0, np.pi, (3, 2 * p))
    a[1, :p] = rng.uniform(np.pi / 4 + 0.05, 3 * np.pi / 4 - 0.05, p)   # flipped rotation form
    a[2, :p] = rng.uniform(-np.pi / 4 + 0.05, np.pi / 4 - 0.05, p)     # plain form
    return a


def _check(q, P, M, n, table, angles, precisions=(0, 1)):
    scale = float(np.max(np.abs(table)))
    for prec in precisions:
        if prec == 1 and n > 12:
            continue
        e, g = q.expect_grad_batched([P], [M], angles, precision=prec)
        for s, a in enumerate(angles):
            E, Nr, g0 = oracle.grad(n, table, a)
            assert abs(e[0, s] - E / Nr) <= TOL[prec] * scale, (prec, s, e[0, s], E / Nr)
            assert np.max(np.abs(g[0, s] - g0 / Nr)) <= TOL[prec] * max(np.max(np.abs(g0 / Nr)), 1e-3), (prec, s)
            e1, g1 = q.expect_grad(P, M, a, precision=prec)
            assert e1 == e[0, s] and np.array_equal(g1, g[0, s])


@pytest.mark.parametrize("n,p", [(12, 1), (12, 4), (12, 10), (13, 3), (13, 8)])
def test_maxcut_one_byte_table(q, ctx, n, p):
    g = workloads.erdos_renyi(n, 2600 + n + p, 0.5)
    t = oracle.graph_table(g)
    _check(q, q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n), n, t, _angles(p, 2610 + p))


@pytest.mark.parametrize("n,p", [(12, 3), (13, 2)])
def test_weighted_two_byte_table(q, ctx, n, p):
    g = workloads.erdos_renyi(n, 2620 + n, 0.5, (1, 30))      # max cut above 255: two-byte table
    t = oracle.graph_table(g)
    assert t.max() > 255
    _check(q, q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n), n, t, _angles(p, 2621))


@pytest.mark.parametrize("n,distinct", [(12, 40), (12, 700), (13, 300)])
def test_asymmetric_value_tables(q, ctx, n, distinct):
    rng = np.random.default_rng(2630 + distinct)
    vals = rng.normal(0.0, 3.0, distinct)[rng.integers(0, distinct, 1 << n)]
    P = q.Problem.from_values(ctx, n, vals)
    _check(q, P, q.Mixer.x(ctx, n), n, vals, _angles(3, 2631))


def test_mixed_batch_of_sizes(q, ctx):
    """Problems of n = 9..14 in one batched call: the register kernel takes n = 12, 13, the LDS
    kernel the smaller ones, the tile passes n = 14; all against the oracle."""
    gs = [workloads.erdos_renyi(n, 2640 + n, 0.5, (1, 3)) for n in (9, 12, 13, 12, 14, 11)]
    P = [q.Problem.from_graph(ctx, g) for g in gs]
    M = [q.Mixer.x(ctx, g.n) for g in gs]
    a = _angles(4, 2641)
    e, gr = q.expect_grad_batched(P, M, a)
    for i, g in enumerate(gs):
        t = oracle.graph_table(g)
        for s in range(a.shape[0]):
            E, Nr, g0 = oracle.grad(g.n, t, a[s])
            assert abs(e[i, s] - E / Nr) <= 1e-5 * t.max()
            assert np.max(np.abs(gr[i, s] - g0 / Nr)) <= 1e-5 * np.max(np.abs(g0 / Nr))
