"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Tolerances (element by element or per scalar):
  * cost table: bit-exact;
  * QAOA_FP64: <C> within 1e-12 relative; gradient within 1e-11 * max|g_ref| (an inf-norm
    relative bound: single components can be ~0, e.g. d/dgamma at beta = 0);
  * QAOA_FP32: <C> within 1e-5 relative, gradient within 1e-5 * max|g_ref| (the bound the
    FP32 form targets); states within 1e-5 of the oracle's unit-norm amplitudes scaled
    by 2^(n/2).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def q():
    import paper_2312_06451_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _gerr(g, ref):
    return float(np.max(np.abs(np.asarray(g) - ref)) / max(np.max(np.abs(ref)), 1e-300))


TOL = {0: (1e-5, 1e-5), 1: (1e-12, 1e-11)}   # precision -> (<C> rel, grad inf-rel)


# ---------------------------------------------------------------- step (a): table

@pytest.mark.parametrize("case", ["reg10", "er16w", "k12w_u16", "reg20"])
def test_table_bit_exact(q, ctx, case):
    if case == "reg10":
        g = workloads.random_regular_graph(10, 3, 1)
    elif case == "er16w":
        g = workloads.erdos_renyi(16, 5, 0.5, (1, 4))
    elif case == "k12w_u16":
        iu, ju = np.triu_indices(12, 1)
        w = (np.arange(iu.size) % 4) + 1          # total weight 165 -> max cut > ... uint16 path
        w = w * 2
        g = workloads.Graph(12, iu.astype(np.int32), ju.astype(np.int32), w.astype(np.int32))
    else:
        g = workloads.random_regular_graph(20, 3, 4)
    P = q.Problem.from_graph(ctx, g)
    want = oracle.graph_table(g)
    got = P.table()
    assert got.dtype == np.int64 and np.array_equal(got, want)
    assert P.max_value == want.max()


def test_table_hamming_weight_bit_exact(q, ctx):
    g = workloads.erdos_renyi(16, 4016, 0.5)
    for k in (1, 8, 15):
        P = q.Problem.from_graph(ctx, g, hamming_k=k)
        want = oracle.cost_table(g.n, g.u, g.v, g.w, k)
        assert np.array_equal(P.table(), want)


def test_table_full_size_sampled(q, ctx):
    # n = 28 (2^28 entries): every 4099th entry plus the complement pairs, and the sum identity
    W = workloads.workload("maxcut3reg_n28_p8")
    g = W.graphs[0]
    P = q.Problem.from_graph(ctx, g)
    t = P.table()
    xs = np.arange(0, 1 << 28, 4099, dtype=np.uint64)
    assert np.array_equal(t[xs.astype(np.int64)], oracle.cost_values(g.n, g.u, g.v, g.w, xs))
    assert int(t.sum()) == g.total_weight * 2 ** (g.n - 1)


# ---------------------------------------------------------------- whole-state path (n <= 13)

@pytest.mark.parametrize("prec", [1, 0])
def test_small_n10_expect_and_grad(q, ctx, prec):
    W = workloads.workload("maxcut3reg_n10_p3")
    g = W.graphs[0]
    t = oracle.graph_table(g)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, g.n)
    for a in [W.angles[0]] + list(workloads.random_angles(3, 3, 77)):
        E0, N0, g0 = oracle.grad(g.n, t, a)
        e = q.expect(P, M, a, precision=prec)
        e2, gr = q.expect_grad(P, M, a, precision=prec)
        assert _rel(e, E0 / N0) < TOL[prec][0]
        assert _rel(e2, E0 / N0) < TOL[prec][0]
        assert _gerr(gr, g0 / N0) < TOL[prec][1]


@pytest.mark.parametrize("n,prec", [(13, 0), (12, 1), (5, 0), (1, 1)])
def test_small_edges(q, ctx, n, prec):
    g = workloads.erdos_renyi(n, 50 + n, 0.5, (1, 3)) if n > 1 else workloads.Graph(
        1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    t = oracle.graph_table(g)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    a = workloads.random_angles(4, 1, n)[0]
    E0, N0, g0 = oracle.grad(n, t, a)
    e, gr = q.expect_grad(P, M, a, precision=prec)
    assert abs(e - E0 / N0) <= TOL[prec][0] * max(1.0, abs(E0))
    assert np.max(np.abs(gr - g0 / N0)) <= TOL[prec][1] * max(1.0, np.max(np.abs(g0)))


@pytest.mark.parametrize("n,p,prec", [(10, 1024, 0), (10, 1025, 1), (12, 1024, 0), (12, 1025, 0), (12, 1024, 1),
                                      (13, 1024, 0)])
def test_small_parameter_staging_boundary(q, ctx, n, p, prec):
    # p <= 1024: the whole-state kernels read their items and angle sets from host memory
    # (the angle set staged in LDS); p > 1024: both are copied to device memory first. FP32
    # bound: each of the p layers adds at most ~1.2e-7 relative rounding to the amplitudes,
    # so 2e-4 at p = 1024 (the usual 1e-5 is for p <= 100); FP64 keeps its bounds.
    g = workloads.erdos_renyi(n, 60 + n, 0.4)
    t = oracle.graph_table(g)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    a = np.random.default_rng(90 + p + n).uniform(0.0, np.pi, 2 * p)
    E0, N0, g0 = oracle.grad(n, t, a)
    e, gr = q.expect_grad(P, M, a, precision=prec)
    te, tg = TOL[prec] if prec == 1 else (2e-4, 2e-4)
    assert _rel(e, E0 / N0) < te
    assert _gerr(gr, g0 / N0) < tg
    assert _rel(q.expect(P, M, a, precision=prec), E0 / N0) < te


# ---------------------------------------------------------------- tile path (n > 13)

TILE_CASES = [(14, 1, 0), (14, 2, 1), (16, 3, 0), (17, 2, 1), (20, 4, 0), (21, 3, 0), (22, 2, 0),
              (22, 3, 1), (23, 5, 0), (14, 1, 1), (13, 2, 1)]


@pytest.mark.parametrize("n,p,prec", TILE_CASES)
def test_tile_expect_and_grad(q, ctx, n, p, prec):
    g = workloads.random_regular_graph(n, 3, 100 + n) if n % 2 == 0 else workloads.erdos_renyi(
        n, 100 + n, 0.5, (1, 4))
    t = oracle.graph_table(g)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    for a in workloads.random_angles(p, 2, 200 + n + p):
        E0, N0, g0 = oracle.grad(n, t, a)
        e = q.expect(P, M, a, precision=prec)
        e2, gr = q.expect_grad(P, M, a, precision=prec)
        assert _rel(e, E0 / N0) < TOL[prec][0], (e, E0)
        assert _rel(e2, E0 / N0) < TOL[prec][0], (e2, E0)
        assert _gerr(gr, g0 / N0) < TOL[prec][1], (gr, g0)


@pytest.mark.parametrize("n,prec", [(14, 0), (15, 1), (18, 0), (22, 0)])
def test_tile_state_elementwise(q, ctx, n, prec):
    import torch
    g = workloads.erdos_renyi(n, 300 + n, 0.5, (1, 2))
    t = oracle.graph_table(g)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    a = workloads.random_angles(3, 1, 400 + n)[0]
    want = oracle.state(n, t, a)
    out = torch.empty(1 << n, dtype=torch.complex64 if prec == 0 else torch.complex128, device="cuda")
    q.state(P, M, a, out, precision=prec)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.complex128)
    scale = 2 ** (n / 2)
    tol = 1e-5 if prec == 0 else 1e-12
    assert np.max(np.abs(got - want)) * scale < tol


@pytest.mark.parametrize("prec", [0, 1])
def test_tile_custom_initial_state(q, ctx, prec):
    import torch
    n, p = 15, 2
    g = workloads.erdos_renyi(n, 500, 0.5)
    t = oracle.graph_table(g)
    rng = np.random.default_rng(5)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    a = workloads.random_angles(p, 1, 501)[0]
    E0, N0, g0 = oracle.grad(n, t, a, psi0=psi0)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    d = torch.tensor(psi0, dtype=torch.complex64 if prec == 0 else torch.complex128, device="cuda")
    e, gr = q.expect_grad(P, M, a, psi0=d, precision=prec)
    assert _rel(e, E0 / N0) < TOL[prec][0]
    assert _gerr(gr, g0 / N0) < TOL[prec][1]


def test_tile_angle_edge_cases(q, ctx):
    # beta at exactly pi/4 (tan = 1, form switch), pi/2 (cos = 0), 0; gamma = 0; negative angles
    n = 16
    g = workloads.random_regular_graph(n, 3, 9)
    t = oracle.graph_table(g)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    for a in ([np.pi / 4, np.pi / 2, 0.3, 0.0], [0.0, 0.0, 1.0, 2.0], [-1.2, 2.9, -0.4, 0.0],
              [3 * np.pi / 4, -np.pi / 4, 1e-9, 7.0]):
        E0, N0, g0 = oracle.grad(n, t, np.array(a))
        for prec in (0, 1):
            e, gr = q.expect_grad(P, M, np.array(a), precision=prec)
            assert _rel(e, E0 / N0) < TOL[prec][0]
            assert np.max(np.abs(gr - g0 / N0)) <= TOL[prec][1] * max(1.0, np.max(np.abs(g0)))


# ---------------------------------------------------------------- full size (n = 28, p = 8)

def _golden(name):
    with open(os.path.join(HERE, "golden", name + ".json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def c2(q, ctx):
    W = workloads.workload("maxcut3reg_n28_p8")
    g = W.graphs[0]
    return W, g, q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, g.n)


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_n28_p8_vs_oracle(q, c2, prec):
    W, g, P, M = c2
    G = _golden("maxcut3reg_n28_p8")
    assert G["edges"][0] == g.u.tolist() and G["edges"][1] == g.v.tolist()
    s = G["sets"][0]
    assert np.allclose(s["angles"], W.angles[0], rtol=0, atol=0)
    e, gr = q.expect_grad(P, M, W.angles[0], precision=prec)
    print("n28 p8 prec", prec, "rel err E", _rel(e, s["expect"]), "grad", _gerr(gr, np.array(s["grad"])))
    assert _rel(e, s["expect"]) < TOL[prec][0]
    assert _gerr(gr, np.array(s["grad"])) < TOL[prec][1]
    e_only = q.expect(P, M, W.angles[0], precision=prec)
    assert _rel(e_only, s["expect"]) < TOL[prec][0]


def test_full_size_n28_p1_closed_form(q, c2):
    from tests import pins
    W, g, P, M = c2
    edges = list(zip(g.u.tolist(), g.v.tolist()))
    for beta, gamma in [(0.3, 0.7), (2.1, 1.3), (0.9, 2.8)]:
        E, db, dg = pins.maxcut_p1(g.n, edges, beta, gamma)
        for prec in (0, 1):
            e, gr = q.expect_grad(P, M, [beta, gamma], precision=prec)
            assert _rel(e, E) < TOL[prec][0]
            assert np.max(np.abs(gr - [db, dg])) < TOL[prec][1] * max(abs(db), abs(dg))


def test_full_size_n28_identities(q, c2):
    W, g, P, M = c2
    a = W.angles[0].copy()
    p = 8
    a0 = a.copy(); a0[:p] = 0.0                     # beta = 0: uniform mean, d/dgamma = 0
    e, gr = q.expect_grad(P, M, a0, precision=0)
    assert _rel(e, g.total_weight / 2) < 1e-6
    assert np.max(np.abs(gr[p:])) < 1e-5
    e1, g1 = q.expect_grad(P, M, a, precision=0)      # (beta, gamma) -> -(beta, gamma)
    e2, g2 = q.expect_grad(P, M, -a, precision=0)
    assert _rel(e2, e1) < 2e-6
    assert np.max(np.abs(g1 + g2)) < 2e-5 * np.max(np.abs(g1))


def test_full_size_cycle_light_cone(q, ctx):
    """MaxCut on the cycle C_28 at p = 3 in the n = 28 launch configuration of the benchmark
    (tile passes, complex64 and complex128) against a property that holds at any size: by the
    light cone, <C> = 28 times the middle-edge cut probability of the path of 8 vertices, and
    the same for the gradient (dense matrices on 8 qubits, no oracle)."""
    from tests import pins
    n, p = 28, 3
    u = np.arange(n, dtype=np.int32)
    v = (u + 1) % n
    g = workloads.Graph(n, np.minimum(u, v).astype(np.int32), np.maximum(u, v).astype(np.int32), np.ones(n, dtype=np.int32))
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    for a in workloads.random_angles(p, 2, 4128):
        ev, eg = pins.cycle_edge(p, a)
        for prec in (0, 1):
            e, gr = q.expect_grad(P, M, a, precision=prec)
            assert _rel(e, n * ev) < TOL[prec][0]
            # the finite differences of the dense value carry ~1e-10 of their own
            assert np.max(np.abs(gr - n * eg)) < max(TOL[prec][1], 1e-9) * n * np.max(np.abs(eg))


def test_full_size_cycle_light_cone_p8(q, ctx):
    """MaxCut on the cycle C_28 at the benchmark's depth p = 8 and in its launch configuration
    (n = 28 tile passes with the checkpoint-reading reverse sweep, complex64 and complex128)
    against the light cone: <C> = 28 times the middle-edge cut probability of the path of 18
    vertices (block-exponential mixer on 2^18 amplitudes, no oracle), and three gradient
    entries against central differences of that value."""
    from tests import pins
    n, p = 28, 8
    u = np.arange(n, dtype=np.int32)
    v = (u + 1) % n
    g = workloads.Graph(n, np.minimum(u, v).astype(np.int32), np.maximum(u, v).astype(np.int32),
                        np.ones(n, dtype=np.int32))
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    a = workloads.random_angles(p, 1, 4800)[0]
    comps = [0, p - 1, p]
    ev, eg = pins.cycle_edge_blocks(p, a, components=comps)
    for prec in (0, 1):
        e, gr = q.expect_grad(P, M, a, precision=prec)
        assert _rel(e, n * ev) < TOL[prec][0]
        scale = n * np.nanmax(np.abs(eg))
        for i in comps:
            # the central differences carry ~1e-10 of their own
            assert abs(gr[i] - n * eg[i]) < max(TOL[prec][1], 1e-9) * scale
    P.close(); M.close()


def test_full_size_weighted_ladder_light_cone(q, ctx):
    """Weighted MaxCut on the circular ladder with 2 x 14 = 28 vertices (3-regular, weights
    1..3) at p = 3, in the n = 28 launch configuration of the benchmark, against the light-cone
    sum: every edge term evolved on its ball of 14 qubits with scipy's expm_multiply (no
    oracle). <C> in both precisions, and d/dbeta_1 against central differences of the sum."""
    from tests import pins
    L, p = 14, 3
    ed = sorted({(min(a, b), max(a, b)) for i in range(L)
                 for a, b in ((i, (i + 1) % L), (i, L + i), (L + i, L + (i + 1) % L))})
    u = np.array([e[0] for e in ed], dtype=np.int32)
    v = np.array([e[1] for e in ed], dtype=np.int32)
    w = np.random.default_rng(4401).integers(1, 4, u.size).astype(np.int32)
    n = 2 * L
    g = workloads.Graph(n, u, v, w)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    a = workloads.random_angles(p, 1, 4402)[0]
    ev, eg = pins.light_cone_expect(n, u, v, w, p, a, components=[0])
    for prec in (0, 1):
        assert _rel(q.expect(P, M, a, precision=prec), ev) < TOL[prec][0]
        e, gr = q.expect_grad(P, M, a, precision=prec)
        assert _rel(e, ev) < TOL[prec][0]
        # the central differences carry ~1e-9 of their own
        assert abs(gr[0] - eg[0]) < max(TOL[prec][1] * np.max(np.abs(gr)), 1e-7 * float(w.sum()))


def test_deterministic_repeat(q, c2):
    W, g, P, M = c2
    r1 = q.expect_grad(P, M, W.angles[0], precision=0)
    r2 = q.expect_grad(P, M, W.angles[0], precision=0)
    assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1])


@pytest.mark.parametrize("mode", ["0", "1"])
def test_gradient_sweep_modes(q, mode, monkeypatch):
    # "0": the reverse sweep undoes every forward pass in place; "1": it reads the forward
    # passes' stored outputs. Both must match the oracle.
    monkeypatch.setenv("QAOA_GRAD_CHECKPOINT", mode)
    c = q.Context(0)
    for n, p, prec in [(16, 3, 0), (22, 2, 1), (21, 4, 0)]:
        g = workloads.random_regular_graph(n, 3, 600 + n) if n % 2 == 0 else workloads.erdos_renyi(
            n, 600 + n, 0.5, (1, 3))
        t = oracle.graph_table(g)
        P, M = q.Problem.from_graph(c, g), q.Mixer.x(c, n)
        a = workloads.random_angles(p, 1, 700 + n)[0]
        E0, N0, g0 = oracle.grad(n, t, a)
        e, gr = q.expect_grad(P, M, a, precision=prec)
        assert _rel(e, E0 / N0) < TOL[prec][0]
        assert _gerr(gr, g0 / N0) < TOL[prec][1]
        P.close(); M.close()
    c.close()
