"""GPU parity of the Grover mixer (Sec. 2.4): evaluations on the cost classes against the FP64
oracle's full-vector evolution, state export, batching, and the degeneracy counts (from a
stored table, and table-free over all states or a Hamming-weight subspace) against the
oracle's histogram and, at n = 34, against exact moment identities of the MaxCut cost.

The class evaluation runs in FP64 for either precision argument: tolerance 1e-11."""
from math import comb

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.fixture(scope="module")
def q():
    import paper_2312_06451_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def real_values(N, seed, distinct=50):
    rng = np.random.default_rng(seed)
    pool = rng.normal(0.5, 3.0, distinct)
    return pool[rng.integers(0, distinct, N)]


def close(q, P, M, n, t, a, k=-1):
    E0, N0, g0 = oracle.grad(n, t, a, k=k, grover=True)
    for prec in (0, 1):
        e, gr = q.expect_grad(P, M, a, precision=prec)
        assert abs(e - E0 / N0) <= TOL * np.max(np.abs(t)), (e, E0 / N0)
        assert np.max(np.abs(gr - g0 / N0)) <= TOL * max(1.0, np.max(np.abs(g0))), (gr, g0)
        assert abs(q.expect(P, M, a, precision=prec) - e) <= 1e-13 * max(1.0, abs(e))


@pytest.mark.parametrize("n,k", [(12, -1), (18, -1), (12, 5), (16, 8)])
def test_grover_graph_vs_oracle(q, ctx, n, k):
    g = workloads.erdos_renyi(n, 900 + n, 0.5, (1, 3))
    t = oracle.graph_table(g, k)
    P, M = q.Problem.from_graph(ctx, g, hamming_k=k), q.Mixer.grover(ctx, n, k)
    vals, cnt = P.degeneracies()
    v0, c0 = oracle.degeneracies(t)
    assert np.array_equal(vals, v0.astype(np.float64)) and np.array_equal(cnt, c0)
    for a in workloads.random_angles(6, 2, 910 + n):
        close(q, P, M, n, t, a, k)


def test_grover_real_values_and_state(q, ctx):
    import torch
    n, p = 12, 5
    t = real_values(1 << n, 920)
    P, M = q.Problem.from_values(ctx, n, t), q.Mixer.grover(ctx, n)
    a = workloads.random_angles(p, 1, 921)[0]
    close(q, P, M, n, t, a)
    want = oracle.state(n, t, a, grover=True)
    for prec, dt, tol in ((0, torch.complex64, 1e-6), (1, torch.complex128, 1e-12)):
        out = torch.empty(1 << n, dtype=dt, device="cuda")
        q.state(P, M, a, out, precision=prec)
        torch.cuda.synchronize()
        assert np.max(np.abs(out.cpu().numpy() - want)) * np.sqrt(1 << n) < tol


def test_grover_batched_with_other_mixers(q, ctx):
    g1 = workloads.erdos_renyi(14, 930, 0.5)
    g2 = workloads.random_regular_graph(16, 3, 931)
    P1, P2 = q.Problem.from_graph(ctx, g1), q.Problem.from_graph(ctx, g2)
    Mg, Mx = q.Mixer.grover(ctx, 14), q.Mixer.x(ctx, 16)
    angles = workloads.random_angles(4, 5, 932)
    for prec in (0, 1):
        Eb, Gb = q.expect_grad_batched([P1, P2], [Mg, Mx], angles, precision=prec)
        for s in range(5):
            e1, g1s = q.expect_grad(P1, Mg, angles[s], precision=prec)
            e2, g2s = q.expect_grad(P2, Mx, angles[s], precision=prec)
            assert abs(Eb[0, s] - e1) <= 1e-12 * abs(e1) and np.allclose(Gb[0, s], g1s, rtol=0, atol=1e-12 * np.max(np.abs(g1s)))
            assert abs(Eb[1, s] - e2) <= 1e-6 * abs(e2)


@pytest.mark.parametrize("n,k,wr", [(20, -1, None), (18, -1, (1, 9)), (16, 7, None), (14, 6, (2, 5)),
                                    (24, -1, None), (26, -1, (1, 3)), (27, -1, (2, 2)), (25, -1, (1, 6))])
def test_table_free_degeneracies(q, ctx, n, k, wr):
    g = workloads.erdos_renyi(n, 940 + n, 0.5, wr)
    Pd = q.Problem.degeneracies_of_graph(ctx, g, hamming_k=k)
    vals, cnt = Pd.degeneracies()
    v0, c0 = oracle.degeneracies(oracle.graph_table(g, k))
    assert np.array_equal(vals, v0.astype(np.float64)) and np.array_equal(cnt, c0)
    # the Grover evaluation on the counted classes equals the tabulated one
    Pt = q.Problem.from_graph(ctx, g, hamming_k=k)
    M = q.Mixer.grover(ctx, n, k)
    for a in workloads.random_angles(5, 2, 950 + n):
        e1, g1 = q.expect_grad(Pd, M, a)
        e2, g2 = q.expect_grad(Pt, M, a)
        # same classes, same FP64 rounds: agreement to rounding, on the scale of <C>
        scale = max(abs(e2), np.max(np.abs(g2)))
        assert abs(e1 - e2) <= 1e-12 * abs(e2) and np.max(np.abs(g1 - g2)) <= 1e-12 * scale


@pytest.mark.parametrize("n,kind", [(26, "reg3"), (27, "sparse"), (27, "sparse12")])
def test_table_free_degeneracies_block_walk(q, ctx, n, kind):
    # 2^(n-20) states per thread, walked in pairs of 32-step blocks; sparse graphs keep the
    # histogram in per-thread columns (one or two edge-weight classes)
    if kind == "reg3":
        g = workloads.random_regular_graph(n, 3, 970 + n)
    else:
        g = workloads.erdos_renyi(n, 975 + n, 0.08, (1, 2) if kind == "sparse12" else None)
    assert g.w.sum() <= 63
    Pd = q.Problem.degeneracies_of_graph(ctx, g)
    vals, cnt = Pd.degeneracies()
    v0, c0 = oracle.degeneracies(oracle.graph_table(g, -1))
    assert np.array_equal(vals, v0.astype(np.float64)) and np.array_equal(cnt, c0)


@pytest.mark.parametrize("n,kind", [(30, "reg3"), (31, "dense"), (32, "sparse13"), (30, "sparse14")])
def test_table_free_degeneracies_vs_table_histogram(q, ctx, n, kind):
    # larger walks (2^10 .. 2^12 states per thread: every high-qubit flip of the block walk)
    # against the histogram of the stored cost table, itself checked against the oracle above;
    # sparse13 (67 bins) and sparse14 (109 bins: one workgroup per CU) keep per-thread columns,
    # dense (585 bins) the shared histogram
    if kind == "reg3":
        g = workloads.random_regular_graph(n, 3, 980 + n)
    elif kind == "dense":
        g = workloads.erdos_renyi(n, 980 + n, 0.5, (1, 4))
    elif kind == "sparse14":
        g = workloads.erdos_renyi(n, 950 + n, 0.09, (1, 4))
        assert 80 < g.w.sum() + 1 <= 160
    else:
        g = workloads.erdos_renyi(n, 980 + n, 0.07, (1, 3))
    vals, cnt = q.Problem.degeneracies_of_graph(ctx, g).degeneracies()
    Pt = q.Problem.from_graph(ctx, g)
    vt, ct = Pt.degeneracies()
    Pt.close()
    assert np.array_equal(vals, vt) and np.array_equal(cnt, ct)
    assert int(cnt.sum()) == 2 ** n


def test_table_free_degeneracies_n34_moments(q, ctx):
    # over all 2^n strings the cut indicators of the edges are pairwise independent fair bits:
    # sum_c m_c = 2^n, sum_c c m_c = W 2^(n-1), sum_c (2c - W)^2 m_c = 2^n sum_e w_e^2
    for seed, wr in ((960, None), (961, (1, 7))):
        g = workloads.random_regular_graph(34, 3, seed) if wr is None else workloads.erdos_renyi(34, seed, 0.12, wr)
        Pd = q.Problem.degeneracies_of_graph(ctx, g)
        vals, cnt = Pd.degeneracies()
        c = [int(v) for v in vals]
        m = [int(x) for x in cnt]
        W = int(g.w.sum())
        assert sum(m) == 2 ** 34
        assert sum(ci * mi for ci, mi in zip(c, m)) == W * 2 ** 33
        assert sum((2 * ci - W) ** 2 * mi for ci, mi in zip(c, m)) == 2 ** 34 * int((g.w.astype(np.int64) ** 2).sum())
        assert Pd.size == 2 ** 34


def test_grover_errors(q, ctx):
    import torch
    from paper_2312_06451_amd import _lib
    g = workloads.random_regular_graph(14, 3, 970)
    Pd = q.Problem.degeneracies_of_graph(ctx, g)
    Mx, Mg = q.Mixer.x(ctx, 14), q.Mixer.grover(ctx, 14)
    a = [0.3, 0.7]
    with pytest.raises(q.QAOAError) as ei:
        q.expect(Pd, Mx, a)
    assert ei.value.status == _lib.QAOA_ERR_UNSUPPORTED
    with pytest.raises(q.QAOAError) as ei:
        Pd.table()
    assert ei.value.status == _lib.QAOA_ERR_UNSUPPORTED
    Pt = q.Problem.from_graph(ctx, g)
    psi0 = torch.full((1 << 14,), 2 ** -7, dtype=torch.complex64, device="cuda")
    with pytest.raises(q.QAOAError) as ei:
        q.expect(Pt, Mg, a, psi0=psi0)
    assert ei.value.status == _lib.QAOA_ERR_UNSUPPORTED
    with pytest.raises(q.QAOAError):
        q.expect(Pt, q.Mixer.grover(ctx, 14, 7), a)     # subspace differs
