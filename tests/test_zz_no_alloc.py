"""The allocation-free paired fwd+grad entry point (qaoa_expect_grad_pairs_noalloc) against
the allocating one (qaoa_expect_grad_pairs) on the same pairs: two calls in a row, the second
with fewer pairs and a smaller p, both precisions, pairs of mixed n and table width (the
register-resident kernel at n = 12, 13 and the LDS kernel below). The same kernels run on the
same inputs, so results must be identical; both are also within the FP32 / FP64 bar of the
FP64 oracle on a few pairs."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _pairs(q, ctx, ns, seed, weighted_every=3):
    probs, mixers, graphs = [], [], []
    for j, n in enumerate(ns):
        wr = (1, 4) if j % weighted_every == 0 else None
        g = workloads.erdos_renyi(n, seed + j, 0.5, wr)
        probs.append(q.Problem.from_graph(ctx, g))
        mixers.append(q.Mixer.x(ctx, n))
        graphs.append(g)
    return probs, mixers, graphs


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_pairs_match_allocating_call(prec):
    import paper_2312_06451_amd as q
    from paper_2312_06451_amd import _lib
    ctx = q.Context(0)
    top = 13 if prec == 0 else 12
    calls = [(list(range(6, top + 1)) * 6, 10, 9100), ([top, 9, top - 1, 5], 3, 9200)]
    for ns, p, seed in calls:
        probs, mixers, graphs = _pairs(q, ctx, ns, seed)
        a = workloads.random_angles(p, len(ns), seed + 50)
        hp = [P.handle for P in probs]
        hm = [M.handle for M in mixers]
        e0, g0 = _lib.qaoa_expect_grad_pairs(hp, hm, p, a, prec)
        e1, g1 = _lib.qaoa_expect_grad_pairs_noalloc(hp, hm, p, a, prec)
        assert np.array_equal(e0, e1) and np.array_equal(g0, g1)
        tol = 1e-5 if prec == 0 else 1e-12
        for i in (0, len(ns) - 1):
            t = oracle.graph_table(graphs[i])
            E, Nr, gr = oracle.grad(graphs[i].n, t, a[i])
            assert abs(e1[i] - E / Nr) <= tol * abs(E / Nr)
            assert np.max(np.abs(g1[i] - gr / Nr)) <= tol * np.max(np.abs(gr / Nr))
        for P in probs:
            P.close()
        for M in mixers:
            M.close()
    ctx.close()


def test_noalloc_rejects_what_it_cannot_hold():
    import paper_2312_06451_amd as q
    from paper_2312_06451_amd import _lib
    ctx = q.Context(0)
    g = workloads.erdos_renyi(10, 9300, 0.5)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, 10)
    p = 1000                                   # 200 pairs at p = 1000 need 6.4 MB > 4 MiB
    a = workloads.random_angles(p, 200, 9301)
    with pytest.raises(q.QAOAError):
        _lib.qaoa_expect_grad_pairs_noalloc([P.handle] * 200, [M.handle] * 200, p, a, 0)
    g2 = workloads.random_regular_graph(16, 3, 9302)   # n = 16 is not a whole-state pair
    P2, M2 = q.Problem.from_graph(ctx, g2), q.Mixer.x(ctx, 16)
    with pytest.raises(q.QAOAError):
        _lib.qaoa_expect_grad_pairs_noalloc([P2.handle], [M2.handle], 2, workloads.random_angles(2, 1, 9303), 0)
    for h in (P, M, P2, M2):
        h.close()
    ctx.close()
