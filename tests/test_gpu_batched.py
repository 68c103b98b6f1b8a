"""GPU parity of the batched entry points: 8 weighted G(n, 1/2) MaxCut instances with
n ~ U{12..20} (the batched workload's instances), p = 10, many angle sets.

Each (instance, angle set) of a batched call must equal the single evaluation of that
item bit for bit (same kernels, same per-item arithmetic), and a sample of items must
match the FP64 oracle (1e-5 FP32, 1e-12 FP64)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_2312_06451_amd as q
    ctx = q.Context(0)
    W = workloads.workload("batched_er_n12to20_p10", n_sets=16)
    probs = [q.Problem.from_graph(ctx, g) for g in W.graphs]
    mixers = [q.Mixer.x(ctx, g.n) for g in W.graphs]
    yield q, ctx, W, probs, mixers


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_matches_single_and_oracle(setup, prec):
    q, ctx, W, probs, mixers = setup
    A = W.angles
    E, G = q.expect_grad_batched(probs, mixers, A, precision=prec)
    Eo = q.expect_batched(probs, mixers, A, precision=prec)
    assert E.shape == (8, 16) and G.shape == (8, 16, 20)
    tol = 1e-5 if prec == 0 else 1e-12
    for i, g in enumerate(W.graphs):
        t = oracle.graph_table(g)
        for s in (0, 7, 15):
            e1, g1 = q.expect_grad(probs[i], mixers[i], A[s], precision=prec)
            assert E[i, s] == e1 and np.array_equal(G[i, s], g1)
            assert Eo[i, s] == q.expect(probs[i], mixers[i], A[s], precision=prec)
        for s in (3,):
            E0, N0, g0 = oracle.grad(g.n, t, A[s])
            assert abs(E[i, s] - E0 / N0) <= tol * abs(E0)
            assert np.max(np.abs(G[i, s] - g0 / N0)) <= tol * np.max(np.abs(g0))


def test_batched_full_angle_count(setup):
    # 256 angle sets (the workload's size): finite, deterministic, and equal per item to a
    # single evaluation for a few sampled sets
    q, ctx, W, probs, mixers = setup
    A = workloads.workload("batched_er_n12to20_p10").angles
    E1, G1 = q.expect_grad_batched(probs, mixers, A)
    E2, G2 = q.expect_grad_batched(probs, mixers, A)
    assert np.all(np.isfinite(E1)) and np.all(np.isfinite(G1))
    assert np.array_equal(E1, E2) and np.array_equal(G1, G2)
    for i in range(8):
        for s in (0, 255):
            e, g = q.expect_grad(probs[i], mixers[i], A[s])
            assert E1[i, s] == e and np.array_equal(G1[i, s], g)


@pytest.mark.parametrize("prec,side_stream", [(0, False), (0, True), (1, False)])
def test_batched_graph_replays_match_eager(prec, side_stream, monkeypatch):
    """From the second batched call with the same problems, mixers, p, sets and precision on,
    the device work is a captured HIP graph that is replayed with freshly staged parameters.
    Four calls with different angle sets (first: eager, second: capture, then replays), on
    torch's default (null) stream or a side stream, equal a context that never uses graphs bit
    for bit; a call on a larger problem in between (which grows the shared buffers) makes the
    next call fall back to eager work and capture again, with the same results."""
    import torch
    import paper_2312_06451_amd as q
    W = workloads.workload("batched_er_n12to20_p10", n_sets=8)
    sets = [workloads.random_angles(10, 8, 9500 + k) for k in range(5)]
    monkeypatch.setenv("QAOA_BATCH_GRAPH", "0")
    c0 = q.Context(0)
    monkeypatch.delenv("QAOA_BATCH_GRAPH")
    c1 = q.Context(0)
    P0 = [q.Problem.from_graph(c0, g) for g in W.graphs]
    M0 = [q.Mixer.x(c0, g.n) for g in W.graphs]
    P1 = [q.Problem.from_graph(c1, g) for g in W.graphs]
    M1 = [q.Mixer.x(c1, g.n) for g in W.graphs]
    big = workloads.random_regular_graph(22, 3, 9600)
    Pb, Mb = q.Problem.from_graph(c1, big), q.Mixer.x(c1, 22)
    st = torch.cuda.Stream() if side_stream else None
    for k, A in enumerate(sets):
        if k == 3:
            q.expect_grad(Pb, Mb, workloads.random_angles(10, 1, 9601)[0], precision=prec)
        E0, G0 = q.expect_grad_batched(P0, M0, A, precision=prec)
        if st is not None:
            with torch.cuda.stream(st):
                E1, G1 = q.expect_grad_batched(P1, M1, A, precision=prec, stream=st)
        else:
            E1, G1 = q.expect_grad_batched(P1, M1, A, precision=prec)
        assert np.array_equal(E0, E1) and np.array_equal(G0, G1), k
    e, g = q.expect_grad(P1[2], M1[2], sets[-1][5], precision=prec)
    assert E1[2, 5] == e and np.array_equal(G1[2, 5], g)
    for h in P0 + M0 + P1 + M1 + [Pb, Mb]:
        h.close()
    c0.close(); c1.close()
