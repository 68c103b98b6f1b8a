"""GPU parity of mixers built from Pauli-X products (Eq. (2)) and of per-qubit multi-angle
mixers against the FP64 oracle (``oracle.xmixers``): symmetric k-body sums, term lists,
per-qubit angles; one and several transform passes (n <= 12 and n > 12); FP32 (1e-5) and FP64
(1e-10), relative to max|C| for <C> and to max|g| for the gradient. At n = 24 the transverse
field written as the order-1 sum is compared with the rotation kernels, an independent path."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import xmixers as X

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


def _check(q, P, M, n, t, angles, d=None, multi=False, precisions=(0, 1)):
    scale = float(np.max(np.abs(t)))
    for prec in precisions:
        for a in angles:
            E, Nr, g0 = X.grad(n, t, a, d=d, multiangle=multi)
            e, g = q.expect_grad(P, M, a, precision=prec)
            assert abs(e - E / Nr) <= TOL[prec] * scale, (prec, e, E / Nr)
            assert g.shape == g0.shape
            assert np.max(np.abs(g - g0 / Nr)) <= TOL[prec] * max(np.max(np.abs(g0)), 1e-3), (prec, g, g0)
            assert abs(q.expect(P, M, a, precision=prec) - e) <= 1e-12 * scale


@pytest.mark.parametrize("n,orders,p", [(8, [1], 3), (10, [2], 2), (12, [1, 3], 2), (14, [2], 2), (17, [1, 2, 5], 2)])
def test_orders_vs_oracle(q, ctx, n, orders, p):
    g = workloads.erdos_renyi(n, 2800 + n, 0.5, (1, 3))
    t = oracle.graph_table(g)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x_orders(ctx, n, orders)
    _check(q, P, M, n, t, workloads.random_angles(p, 2, 2801 + n), d=X.diag_orders(n, orders))


@pytest.mark.parametrize("n,masks,coefs", [(9, [0b1, 0b110, 0b101010101], [1.0, -0.5, 2.0]),
                                            (13, [0b1111111111111, 0b11, 0b1000000000001, 0b1010], [0.3, 1.0, -1.2, 0.8])])
def test_terms_vs_oracle(q, ctx, n, masks, coefs):
    rng = np.random.default_rng(2810 + n)
    vals = rng.normal(0.0, 2.0, 60)[rng.integers(0, 60, 1 << n)]
    P, M = q.Problem.from_values(ctx, n, vals), q.Mixer.x_terms(ctx, n, masks, coefs)
    _check(q, P, M, n, vals, workloads.random_angles(3, 2, 2811), d=X.diag_terms(n, masks, coefs))


@pytest.mark.parametrize("n,p", [(6, 2), (11, 3), (15, 2)])
def test_multiangle_vs_oracle(q, ctx, n, p):
    g = workloads.erdos_renyi(n, 2820 + n, 0.5, (1, 3))
    t = oracle.graph_table(g)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x_multiangle(ctx, n)
    assert M.info()["angles_per_layer"] == n + 1
    rng = np.random.default_rng(2821 + n)
    _check(q, P, M, n, t, rng.uniform(0, np.pi, (2, p * (n + 1))), multi=True)


def test_multiangle_equal_angles_is_the_transverse_field(q, ctx):
    n, p = 16, 3
    g = workloads.erdos_renyi(n, 2830, 0.5, (1, 3))
    P, Mx, Mm = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n), q.Mixer.x_multiangle(ctx, n)
    a = workloads.random_angles(p, 1, 2831)[0]
    ma = np.concatenate([np.repeat(a[:p], n), a[p:]])
    for prec in (0, 1):
        e0, g0 = q.expect_grad(P, Mx, a, precision=prec)
        e1, g1 = q.expect_grad(P, Mm, ma, precision=prec)
        assert abs(e0 - e1) <= TOL[prec] * 40
        assert np.allclose(g1[:p * n].reshape(p, n).sum(axis=1), g0[:p], atol=TOL[prec] * 40 * n)
        assert np.allclose(g1[p * n:], g0[p:], atol=TOL[prec] * 40)


def test_order_one_at_n24_matches_rotation_kernels(q, ctx):
    n, p = 24, 2
    g = workloads.random_regular_graph(n, 3, 2840)
    P, Mx, Mo = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n), q.Mixer.x_orders(ctx, n, [1])
    a = workloads.random_angles(p, 2, 2841)
    for prec in (0, 1):
        e0, g0 = q.expect_grad_batched([P], [Mx], a, precision=prec)
        e1, g1 = q.expect_grad_batched([P], [Mo], a, precision=prec)
        assert np.max(np.abs(e0 - e1)) <= TOL[prec] * 36
        assert np.max(np.abs(g0 - g1)) <= TOL[prec] * np.max(np.abs(g0))


def test_batched_and_paired_equal_single_calls(q, ctx):
    n = 13
    gs = [workloads.erdos_renyi(n, 2850 + i, 0.5, (1, 3)) for i in range(2)]
    P = [q.Problem.from_graph(ctx, g) for g in gs]
    Mo, Mt = q.Mixer.x_orders(ctx, n, [2, 3]), q.Mixer.x_terms(ctx, n, [0b111, 0b1000000000001], [1.0, -2.0])
    a = workloads.random_angles(3, 3, 2851)
    e, g = q.expect_grad_batched(P, [Mo, Mt], a)
    for i, M in enumerate((Mo, Mt)):
        for s in range(3):
            e1, g1 = q.expect_grad(P[i], M, a[s])
            assert e[i, s] == e1 and np.array_equal(g[i, s], g1)
    Mm = q.Mixer.x_multiangle(ctx, n)
    am = np.random.default_rng(2852).uniform(0, np.pi, (3, 2 * (n + 1)))
    ep, gp = q.expect_grad_pairs([P[0], P[1], P[0]], [Mm] * 3, am)
    for j, i in enumerate((0, 1, 0)):
        e1, g1 = q.expect_grad(P[i], Mm, am[j])
        assert ep[j] == e1 and np.array_equal(gp[j], g1)


def test_state_output(q, ctx):
    import torch
    n, p = 14, 2
    g = workloads.erdos_renyi(n, 2860, 0.5, (1, 3))
    t = oracle.graph_table(g)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x_orders(ctx, n, [1, 2])
    a = workloads.random_angles(p, 1, 2861)[0]
    out = torch.zeros(1 << n, dtype=torch.complex128, device="cuda")
    q.state(P, M, a, out, precision=1)
    psi = out.cpu().numpy()
    d = X.diag_orders(n, [1, 2])
    want = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    for k in range(p):
        want = X._mixer(np.exp(-1j * a[p + k] * t) * want, a[k], d)
    assert np.max(np.abs(psi - want)) <= 1e-12


def test_errors(q, ctx):
    n = 8
    with pytest.raises(q.QAOAError):
        q.Mixer.x_orders(ctx, n, [1, 1])
    with pytest.raises(q.QAOAError):
        q.Mixer.x_orders(ctx, n, [9])
    with pytest.raises(q.QAOAError):
        q.Mixer.x_terms(ctx, n, [1 << 8], [1.0])
    with pytest.raises(q.QAOAError):
        q.Mixer.x_terms(ctx, n, list(range(1, 12)), [1.0] * 11)
    g = workloads.erdos_renyi(n, 2870, 0.5)
    Pk = q.Problem.from_graph(ctx, g, hamming_k=4)
    with pytest.raises(q.QAOAError):
        q.expect(Pk, q.Mixer.x_orders(ctx, n, [1]), [0.1, 0.2])
    P = q.Problem.from_graph(ctx, g)
    Mm, Mx = q.Mixer.x_multiangle(ctx, n), q.Mixer.x(ctx, n)
    with pytest.raises(q.QAOAError):
        q.expect_batched([P, P], [Mm, Mx], np.zeros((1, 9)))
    with pytest.raises(q.QAOAError):
        q.find_angles(P, Mm, 1)


def test_full_size_against_stored_oracle_values(q, ctx):
    """The benchmark's workload and launch configuration (16 angle sets per batched call) at
    n = 24: set 0 against the FP64 oracle values stored by tests/golden/make_golden.py."""
    import json
    import os
    W = workloads.workload("xorders_maxcut3reg_n24_p4")
    G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "xorders_maxcut3reg_n24_p4.json")))
    rec = G["sets"][0]
    assert np.array_equal(np.array(rec["angles"]), W.angles[0])
    g = W.graphs[0]
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x_orders(ctx, g.n, W.extra["orders"])
    for prec in (0, 1):
        e, gr = q.expect_grad_batched([P], [M], W.angles, precision=prec)
        assert abs(e[0, 0] - rec["expect"]) <= TOL[prec] * G["table_max"]
        g0 = np.array(rec["grad"])
        assert np.max(np.abs(gr[0, 0] - g0)) <= TOL[prec] * np.max(np.abs(g0))


@pytest.mark.parametrize("n,orders,p", [(13, [2], 2), (16, [1, 2], 3), (23, [1, 2], 2)])
def test_tile_passes_match_transform_passes(q, monkeypatch, n, orders, p):
    """Mixers diagonal by Hamming weight run on the tile passes (basis change by Y rotations,
    the transform's boundary passes shared with the diagonals) for n above the tile bits (13
    complex64, 12 complex128); with QAOA_XPROD_TILES=0 the same calls take the separate
    Walsh-Hadamard and diagonal kernels. Both against each other for several angle sets and an
    initial state, and the first set against the FP64 oracle where it finishes quickly."""
    g = workloads.erdos_renyi(n, 2870 + n, 0.3, (1, 2))
    t = oracle.graph_table(g)
    A = workloads.random_angles(p, 3, 2871 + n)
    rng = np.random.default_rng(2872 + n)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    res = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("QAOA_XPROD_TILES", mode)
        c = q.Context(0)
        try:
            P, M = q.Problem.from_graph(c, g), q.Mixer.x_orders(c, n, orders)
            out = []
            for prec in (0, 1):
                e, gr = q.expect_grad_batched([P], [M], A, precision=prec)
                import torch
                dt = torch.complex64 if prec == 0 else torch.complex128
                s0 = torch.tensor(psi0, dtype=dt, device="cuda")
                e0, g0 = q.expect_grad(P, M, A[0], psi0=s0, precision=prec)
                out.append((e[0], gr[0], e0, g0))
            res[mode] = out
        finally:
            c.close()
    scale = float(np.max(np.abs(t)))
    for prec in (0, 1):
        e1, g1, e1s, g1s = res["1"][prec]
        e0, g0, e0s, g0s = res["0"][prec]
        assert np.max(np.abs(e1 - e0)) <= TOL[prec] * scale
        assert np.max(np.abs(g1 - g0)) <= TOL[prec] * max(np.max(np.abs(g0)), 1e-3)
        assert abs(e1s - e0s) <= TOL[prec] * scale
    # From a random initial state the gradient is far below the cost scale (cancellation over
    # the whole state), while the rounding of each term scales with the costs: each path's
    # FP32 gradient against its own FP64 one, with the error floor at 1e-3 of the cost scale.
    for mode in ("1", "0"):
        g32, g64 = res[mode][0][3], res[mode][1][3]
        assert np.max(np.abs(g32 - g64)) <= TOL[0] * max(np.max(np.abs(g64)), 1e-3 * scale), mode
    assert np.max(np.abs(res["1"][1][3] - res["0"][1][3])) <= TOL[1] * max(np.max(np.abs(res["0"][1][3])), 1e-3)
    if n <= 16:
        E, Nr, gref = X.grad(n, t, A[0], d=X.diag_orders(n, orders))
        for prec in (0, 1):
            e1, g1 = res["1"][prec][0], res["1"][prec][1]
            assert abs(e1[0] - E / Nr) <= TOL[prec] * scale
            assert np.max(np.abs(g1[0] - gref / Nr)) <= TOL[prec] * max(np.max(np.abs(gref)), 1e-3)


@pytest.mark.parametrize("n,masks,coefs", [(15, [0b11, 0b101000000000001, 0b111111100000000, 0b1010], [1.0, -0.7, 0.4, 1.3]),
                                            (22, [(1 << 22) - 1, 0b11 << 20, 0b1001, 1 << 17], [0.2, 1.0, -1.5, 0.6])])
def test_terms_on_tile_passes(q, monkeypatch, n, masks, coefs):
    """Term-list mixers (index = parities of y against the masks) on the tile passes against the
    separate transform and diagonal kernels (QAOA_XPROD_TILES=0), FP32 and FP64, and against
    the FP64 oracle at n = 15. The masks span the tiles' contiguous, strided and register bits."""
    rng = np.random.default_rng(2890 + n)
    vals = rng.integers(0, 40, 1 << n).astype(np.float64)
    A = workloads.random_angles(2, 2, 2891 + n)
    res = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("QAOA_XPROD_TILES", mode)
        c = q.Context(0)
        try:
            P, M = q.Problem.from_values(c, n, vals), q.Mixer.x_terms(c, n, masks, coefs)
            res[mode] = [q.expect_grad_batched([P], [M], A, precision=prec) for prec in (0, 1)]
        finally:
            c.close()
    scale = float(np.max(np.abs(vals)))
    for prec in (0, 1):
        (e1, g1), (e0, g0) = res["1"][prec], res["0"][prec]
        assert np.max(np.abs(e1 - e0)) <= TOL[prec] * scale
        assert np.max(np.abs(g1 - g0)) <= TOL[prec] * max(np.max(np.abs(g0)), 1e-3)
    if n <= 16:
        E, Nr, gref = X.grad(n, vals, A[0], d=X.diag_terms(n, masks, coefs))
        for prec in (0, 1):
            e1, g1 = res["1"][prec]
            assert abs(e1[0, 0] - E / Nr) <= TOL[prec] * scale
            assert np.max(np.abs(g1[0, 0] - gref / Nr)) <= TOL[prec] * max(np.max(np.abs(gref)), 1e-3)


@pytest.mark.parametrize("n,p,nsets,distinct", [(14, 1, 1, 300), (19, 1, 5, 30), (20, 3, 2, 700)])
def test_tile_passes_edge_cases(q, monkeypatch, n, p, nsets, distinct):
    """Edge cases of the X-product tile passes against the transform path: one layer (the plan
    is then the first pass, the fused end-of-sweep pass and their reverses), one angle set,
    cost tables of 16-bit indices (more than 255 distinct values), k-body sums and term lists."""
    rng = np.random.default_rng(2900 + n)
    vals = rng.normal(0.0, 3.0, distinct)[rng.integers(0, distinct, 1 << n)]
    A = workloads.random_angles(p, nsets, 2901 + n)
    res = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("QAOA_XPROD_TILES", mode)
        c = q.Context(0)
        try:
            P = q.Problem.from_values(c, n, vals)
            Ms = [q.Mixer.x_orders(c, n, [1, 3]), q.Mixer.x_terms(c, n, [0b111, 1 << (n - 1), (1 << n) - 1], [0.5, -1.0, 0.25])]
            res[mode] = [[q.expect_grad_batched([P], [M], A, precision=prec) for prec in (0, 1)] for M in Ms]
        finally:
            c.close()
    scale = float(np.max(np.abs(vals)))
    for m in range(2):
        for prec in (0, 1):
            (e1, g1), (e0, g0) = res["1"][m][prec], res["0"][m][prec]
            assert e1.shape == (1, nsets) and g1.shape == (1, nsets, 2 * p)
            assert np.max(np.abs(e1 - e0)) <= TOL[prec] * scale, (m, prec)
            assert np.max(np.abs(g1 - g0)) <= TOL[prec] * max(np.max(np.abs(g0)), 1e-3 * scale), (m, prec)


def test_multiangle_full_size_against_stored_oracle_values(q, ctx):
    """The per-qubit multi-angle workload in its benchmark launch configuration (n = 24, p = 4,
    16 angle sets per batched call): set 0 against the FP64 oracle values stored by
    tests/golden/make_golden.py."""
    import json
    import os
    W = workloads.workload("multiangle_maxcut3reg_n24_p4")
    G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "multiangle_maxcut3reg_n24_p4.json")))
    rec = G["sets"][0]
    assert np.array_equal(np.array(rec["angles"]), W.angles[0])
    g = W.graphs[0]
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x_multiangle(ctx, g.n)
    for prec in (0, 1):
        e, gr = q.expect_grad_batched([P], [M], W.angles, precision=prec)
        assert abs(e[0, 0] - rec["expect"]) <= TOL[prec] * G["table_max"]
        g0 = np.array(rec["grad"])
        assert np.max(np.abs(gr[0, 0] - g0)) <= TOL[prec] * np.max(np.abs(g0))


@pytest.mark.parametrize("n,p,nsets", [(13, 2, 2), (14, 2, 3), (23, 2, 2)])
def test_multiangle_on_tile_passes(q, monkeypatch, n, p, nsets):
    """Per-qubit multi-angle mixers on the tile passes (diagonal factored into a per-thread and
    a per-register part, n + 1 gradient sums per layer) against the transform path
    (QAOA_XPROD_TILES=0), complex64 and complex128, and against the FP64 oracle at n <= 14."""
    g = workloads.erdos_renyi(n, 2920 + n, 0.3, (1, 3))
    t = oracle.graph_table(g)
    A = np.random.default_rng(2921 + n).uniform(0.0, np.pi, size=(nsets, p * (n + 1)))
    res = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("QAOA_XPROD_TILES", mode)
        c = q.Context(0)
        try:
            P, M = q.Problem.from_graph(c, g), q.Mixer.x_multiangle(c, n)
            res[mode] = [q.expect_grad_batched([P], [M], A, precision=prec) for prec in (0, 1)]
        finally:
            c.close()
    scale = float(np.max(np.abs(t)))
    for prec in (0, 1):
        (e1, g1), (e0, g0) = res["1"][prec], res["0"][prec]
        assert g1.shape == (1, nsets, p * (n + 1))
        assert np.max(np.abs(e1 - e0)) <= TOL[prec] * scale, prec
        assert np.max(np.abs(g1 - g0)) <= TOL[prec] * max(np.max(np.abs(g0)), 1e-3), prec
    if n <= 14:
        E, Nr, gref = X.grad(n, t, A[0], multiangle=True)
        for prec in (0, 1):
            e1, g1 = res["1"][prec]
            assert abs(e1[0, 0] - E / Nr) <= TOL[prec] * scale
            assert np.max(np.abs(g1[0, 0] - gref / Nr)) <= TOL[prec] * max(np.max(np.abs(gref)), 1e-3)


@pytest.mark.parametrize("kind", ["orders", "terms", "multiangle"])
def test_tile_passes_in_place_sweep(q, monkeypatch, kind):
    """The X-product tile passes' gradient with the reverse sweep undoing the state in place
    (QAOA_GRAD_CHECKPOINT=0, the fallback when the forward checkpoints do not fit) against the
    sweep that reads the checkpoints and against the transform path, both precisions."""
    n, p = 15, 2
    g = workloads.erdos_renyi(n, 2950, 0.3, (1, 2))
    t = oracle.graph_table(g)
    width = p * (n + 1) if kind == "multiangle" else 2 * p
    A = np.random.default_rng(2951).uniform(0.0, np.pi, size=(2, width))

    def mixer(c):
        if kind == "orders":
            return q.Mixer.x_orders(c, n, [1, 2])
        if kind == "terms":
            return q.Mixer.x_terms(c, n, [0b111, 1 << 14, (1 << 15) - 1], [0.5, -1.0, 0.25])
        return q.Mixer.x_multiangle(c, n)

    res = {}
    for tiles, ckpt in (("1", "0"), ("1", "1"), ("0", "1")):
        monkeypatch.setenv("QAOA_XPROD_TILES", tiles)
        monkeypatch.setenv("QAOA_GRAD_CHECKPOINT", ckpt)
        c = q.Context(0)
        try:
            P, M = q.Problem.from_graph(c, g), mixer(c)
            res[(tiles, ckpt)] = [q.expect_grad_batched([P], [M], A, precision=prec) for prec in (0, 1)]
        finally:
            c.close()
    scale = float(np.max(np.abs(t)))
    for ref in (("1", "1"), ("0", "1")):
        for prec in (0, 1):
            (e1, g1), (e0, g0) = res[("1", "0")][prec], res[ref][prec]
            assert np.max(np.abs(e1 - e0)) <= TOL[prec] * scale, (ref, prec)
            assert np.max(np.abs(g1 - g0)) <= TOL[prec] * max(np.max(np.abs(g0)), 1e-3), (ref, prec)
