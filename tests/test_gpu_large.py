"""n = 32 (2^32 amplitudes: 32 GiB per complex64 vector): the large transverse-field
workload, MaxCut on a random 3-regular graph. The host oracle cannot hold the state (64 GiB
per FP64 vector), so parity here rests on properties that hold at any size: the p=1
closed form and its derivative, the beta = 0 identities, the FP64 GPU path (compared
component by component with the FP32 path at p=16), and the table against the oracle's
definition at sampled strings plus its sum identity."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c5():
    import paper_2312_06451_amd as q
    ctx = q.Context(0)
    W = workloads.workload("maxcut3reg_n32_p16")
    g = W.graphs[0]
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, 32)
    yield q, ctx, W, g, P, M
    P.close(); M.close(); ctx.close()


def test_n32_table_sampled(c5):
    """The 2^32-entry table (64-bit indexing) copied back whole: sampled entries on both sides
    of 2^31 equal the oracle's definition evaluated at those strings, the complement pairs
    agree, and the sum is the identity sum_x C(x) = W 2^(n-1)."""
    q, ctx, W, g, P, M = c5
    assert P.size == 1 << 32 and P.max_value <= g.m
    t = P.table()
    rng = np.random.default_rng(5100)
    xs = np.concatenate([np.arange(0, 1 << 32, 1000003, dtype=np.uint64),
                         rng.integers(1 << 31, 1 << 32, 20000, dtype=np.uint64),
                         np.array([0, (1 << 31) - 1, 1 << 31, (1 << 32) - 1], dtype=np.uint64)])
    want = oracle.cost_values(g.n, g.u, g.v, g.w, xs)
    assert np.array_equal(t[xs.astype(np.int64)], want)
    comp = (xs ^ np.uint64((1 << 32) - 1)).astype(np.int64)
    assert np.array_equal(t[comp], want)
    assert int(t.sum(dtype=np.int64)) == g.total_weight * 2 ** (g.n - 1)
    assert int(t.max()) == P.max_value
    del t


def test_n32_p1_closed_form(c5):
    from tests import pins
    q, ctx, W, g, P, M = c5
    edges = list(zip(g.u.tolist(), g.v.tolist()))
    beta, gamma = 0.37, 2.2
    E, db, dg = pins.maxcut_p1(32, edges, beta, gamma)
    for prec, tol in ((0, 1e-5), (1, 1e-12)):
        e, gr = q.expect_grad(P, M, [beta, gamma], precision=prec)
        assert abs(e - E) / abs(E) < tol
        assert np.max(np.abs(gr - [db, dg])) < tol * max(abs(db), abs(dg))


def test_n32_p16_fp32_vs_fp64(c5):
    q, ctx, W, g, P, M = c5
    a = W.angles[0]
    e32, g32 = q.expect_grad(P, M, a, precision=0)
    e64, g64 = q.expect_grad(P, M, a, precision=1)
    print("n32 p16: E32", e32, "E64", e64, "rel", abs(e32 - e64) / abs(e64),
          "grad", np.max(np.abs(g32 - g64)) / np.max(np.abs(g64)))
    assert abs(e32 - e64) / abs(e64) < 1e-5
    assert np.max(np.abs(g32 - g64)) < 1e-5 * np.max(np.abs(g64))
    a0 = a.copy(); a0[:16] = 0.0
    e0 = q.expect(P, M, a0, precision=0)
    assert abs(e0 - g.total_weight / 2) < 1e-5 * g.total_weight
