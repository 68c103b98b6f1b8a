"""GPU parity of the constrained path: clique mixer on the Hamming-weight-k subspace,
eigenbasis products (FP16-split MFMA products in the FP32 form, DGEMM in the FP64 form).

Tolerances: FP32 form <C> 1e-5 relative and gradient 1e-5 of max|g| (at N = 12870 over many
random sets: 1e-5 of the batch's gradient scale, 5e-5 of a set's own, see the balanced-schedule
test); FP64 form 1e-12 for both (the eigendecomposition carries ~1e-13 relative error per eigenpair, which the 2p to
4p products of an evaluation compound; measured at N = 12870: 1e-16 in <C>, 7e-13 in the
gradient)."""
import json
import os
from math import comb

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {0: 1e-5, 1: 1e-12}


@pytest.fixture(scope="module")
def q():
    import paper_2312_06451_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,k,p", [(6, 3, 2), (8, 4, 3), (10, 5, 2), (12, 6, 2), (9, 2, 3)])
def test_clique_small_vs_oracle(q, ctx, n, k, p):
    g = workloads.erdos_renyi(n, 800 + n, 0.5)
    t = oracle.cost_table(n, g.u, g.v, g.w, k)
    P = q.Problem.from_graph(ctx, g, hamming_k=k)
    M = q.Mixer.clique(ctx, n, k)
    assert np.array_equal(P.table(), t)
    for a in workloads.random_angles(p, 2, 900 + n):
        E0, N0, g0 = oracle.grad(n, t, a, k=k)
        for prec in (0, 1):
            e, gr = q.expect_grad(P, M, a, precision=prec)
            assert abs(e - E0 / N0) <= TOL[prec] * abs(E0), (prec, e, E0)
            assert np.max(np.abs(gr - g0 / N0)) <= TOL[prec] * np.max(np.abs(g0)), (prec, gr, g0)
            assert abs(q.expect(P, M, a, precision=prec) - e) <= TOL[prec] * abs(E0)


def test_clique_state_and_initial_state(q, ctx):
    import torch
    n, k, p = 10, 4, 3
    g = workloads.erdos_renyi(n, 77, 0.5)
    t = oracle.cost_table(n, g.u, g.v, g.w, k)
    P, M = q.Problem.from_graph(ctx, g, hamming_k=k), q.Mixer.clique(ctx, n, k)
    a = workloads.random_angles(p, 1, 78)[0]
    want = oracle.state(n, t, a, k=k)
    for prec, dt, tol in ((0, torch.complex64, 1e-5), (1, torch.complex128, 1e-12)):
        out = torch.empty(comb(n, k), dtype=dt, device="cuda")
        q.state(P, M, a, out, precision=prec)
        torch.cuda.synchronize()
        assert np.max(np.abs(out.cpu().numpy() - want)) * np.sqrt(comb(n, k)) < tol
    rng = np.random.default_rng(3)
    psi0 = rng.normal(size=comb(n, k)) + 1j * rng.normal(size=comb(n, k))
    psi0 /= np.linalg.norm(psi0)
    E0, N0, g0 = oracle.grad(n, t, a, k=k, psi0=psi0)
    for prec, dt in ((0, torch.complex64), (1, torch.complex128)):
        d = torch.tensor(psi0, dtype=dt, device="cuda")
        e, gr = q.expect_grad(P, M, a, psi0=d, precision=prec)
        assert abs(e - E0 / N0) <= TOL[prec] * abs(E0)
        assert np.max(np.abs(gr - g0 / N0)) <= TOL[prec] * np.max(np.abs(g0))


def test_clique_identities(q, ctx):
    # gamma = 0: the Dicke state is an eigenvector, so <C> stays the subspace mean for any
    # beta; beta = 0 likewise
    n, k = 12, 6
    g = workloads.erdos_renyi(n, 31, 0.5)
    P, M = q.Problem.from_graph(ctx, g, hamming_k=k), q.Mixer.clique(ctx, n, k)
    mean = g.total_weight * 2 * comb(n - 2, k - 1) / comb(n, k)
    for a in ([0.7, 1.9, 0.0, 0.0], [0.0, 0.0, 2.5, 0.3]):
        for prec in (0, 1):
            assert abs(q.expect(P, M, a, precision=prec) - mean) < 10 * TOL[prec] * mean


@pytest.mark.parametrize("prec", [0, 1])
def test_clique_full_size_vs_oracle(q, ctx, prec):
    path = os.path.join(HERE, "golden", "bisection_g16_k8_p6.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle values for the weight-8 workload not generated")
    G = json.load(open(path))
    W = workloads.workload("bisection_g16_k8_p6", n_sets=8)
    g = W.graphs[0]
    assert G["edges"][0] == g.u.tolist()
    P, M = q.Problem.from_graph(ctx, g, hamming_k=8), q.Mixer.clique(ctx, 16, 8)
    for i, s in enumerate(G["sets"]):
        assert np.array_equal(np.array(s["angles"]), W.angles[i])
        e, gr = q.expect_grad(P, M, W.angles[i], precision=prec)
        print("bisection n16 k8 p6 set", i, "prec", prec, "E err", abs(e - s["expect"]) / abs(s["expect"]),
              "g err", np.max(np.abs(gr - s["grad"])) / np.max(np.abs(s["grad"])))
        assert abs(e - s["expect"]) <= TOL[prec] * abs(s["expect"])
        assert np.max(np.abs(gr - np.array(s["grad"]))) <= TOL[prec] * np.max(np.abs(s["grad"]))
    # the batched call over 8 sets agrees with the single evaluations: bit for bit in the FP32
    # form (every column of the split product is reduced in the same fixed order while the
    # tiles fit one round of workgroups, as here), to rounding in the FP64 form (library DGEMM)
    Eb, Gb = q.expect_grad_batched([P], [M], W.angles, precision=prec)
    for i in (0, 5):
        e, gr = q.expect_grad(P, M, W.angles[i], precision=prec)
        if prec == 0:
            assert Eb[0, i] == e and np.array_equal(Gb[0, i], gr)
        else:
            assert abs(Eb[0, i] - e) <= 1e-13 * abs(e) and np.max(np.abs(Gb[0, i] - gr)) <= 1e-12 * np.max(np.abs(gr))


def test_clique_full_batch_512(q, ctx):
    """The benchmark's launch configuration: all 512 angle sets in one call (products of 12870 x
    12870 by 1024 columns: 408 workgroup tiles, more than one round of the 256 CUs, so the
    products run the XCD-balanced schedule with K-split tiles). Sets 0 and 1 against the stored
    oracle values; every set against the same sets evaluated 256 at a time (the plain schedule,
    one round); the call repeated gives identical results (the tile configuration, the K cuts and
    every summation order are fixed)."""
    path = os.path.join(HERE, "golden", "bisection_g16_k8_p6.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle values for the weight-8 workload not generated")
    G = json.load(open(path))
    W = workloads.workload("bisection_g16_k8_p6")
    assert W.angles.shape[0] == 512
    g = W.graphs[0]
    P, M = q.Problem.from_graph(ctx, g, hamming_k=8), q.Mixer.clique(ctx, 16, 8)
    Eb, Gb = q.expect_grad_batched([P], [M], W.angles, precision=0)
    for i, s in enumerate(G["sets"]):
        assert np.array_equal(np.array(s["angles"]), W.angles[i])
        e_err = abs(Eb[0, i] - s["expect"]) / abs(s["expect"])
        g_err = np.max(np.abs(Gb[0, i] - np.array(s["grad"]))) / np.max(np.abs(s["grad"]))
        print("bisection 512 sets, set", i, "E err", e_err, "g err", g_err, flush=True)
        assert e_err <= TOL[0] and g_err <= TOL[0]
    Eb2, Gb2 = q.expect_grad_batched([P], [M], W.angles, precision=0)
    assert np.array_equal(Eb, Eb2) and np.array_equal(Gb, Gb2)
    halves = [q.expect_grad_batched([P], [M], W.angles[h:h + 256], precision=0) for h in (0, 256)]
    Eh = np.concatenate([e[0] for e, _ in halves])
    Gh = np.concatenate([g_[0] for _, g_ in halves])
    e_dev = np.max(np.abs(Eb[0] - Eh) / np.abs(Eh))
    g_dev = np.max(np.max(np.abs(Gb[0] - Gh), axis=1) / np.max(np.abs(Gh), axis=1))
    print("512 at once vs 2 x 256: E", e_dev, "grad", g_dev, flush=True)
    # two FP32 results, each within TOL of the exact value (split-FP16 products, FP32 sums in
    # different K orders): they agree to 2 TOL
    assert e_dev <= 2 * TOL[0] and g_dev <= 2 * TOL[0]
    P.close(); M.close()


@pytest.fixture(scope="module")
def bisection(q, ctx):
    W = workloads.workload("bisection_g16_k8_p6")
    P, M = q.Problem.from_graph(ctx, W.graphs[0], hamming_k=8), q.Mixer.clique(ctx, 16, 8)
    yield P, M
    P.close(); M.close()


@pytest.mark.parametrize("nsets", [320, 650])
def test_clique_balanced_schedule_shapes(q, bisection, nsets):
    """Other shapes of the XCD-balanced product schedule at N = 12870: 320 sets (5 column
    tiles, super-tiles of 6 row tiles: 9 super-tiles, one more than the XCDs) and 650 sets (11
    column tiles, 2 row tiles per super-tile, 26 super-tiles, up to 5 pieces per XCD). Every set
    of the call, and of the same sets in calls of 100 (one round of tiles: the plain schedule),
    against the FP64 form (DGEMM on the FP64 eigenbasis, 1e-12): <C> to 1e-6 relative; the
    gradient to 1e-5 of the batch's gradient scale (the largest |g| over its sets) and to 5e-5
    of each set's own largest |g|. The FP32 form's gradient error comes from the FP32
    accumulation of the products over N = 12870 terms (about 2e-6 relative per element and
    product, over 4p = 24 products) and is absolute rather than relative per set: measured, at
    most 3.5e-6 of the batch scale, and up to 2.6e-5 of a set's own scale for sets whose
    gradient is small (both schedules alike). The call repeated gives identical results."""
    P, M = bisection
    a = workloads.random_angles(6, nsets, 4400 + nsets)
    E, G = q.expect_grad_batched([P], [M], a, precision=0)
    chunks = [q.expect_grad_batched([P], [M], a[h:h + 100], precision=0) for h in range(0, nsets, 100)]
    Ec = np.concatenate([e[0] for e, _ in chunks])
    Gc = np.concatenate([g_[0] for _, g_ in chunks])
    E64, G64 = q.expect_grad_batched([P], [M], a, precision=1)
    E64, G64 = E64[0], G64[0]
    own = np.max(np.abs(G64), axis=1)
    for name, e, g_ in (("balanced", E[0], G[0]), ("calls of 100", Ec, Gc)):
        e_err = np.max(np.abs(e - E64) / np.abs(E64))
        g_abs = np.max(np.abs(g_ - G64), axis=1)
        print(f"{nsets} sets, {name}: E {e_err:.2e}, grad {g_abs.max() / own.max():.2e} of the batch scale, "
              f"{np.max(g_abs / own):.2e} of a set's own", flush=True)
        assert e_err <= 1e-6
        assert g_abs.max() <= 1e-5 * own.max() and np.all(g_abs <= 5e-5 * own)
    E2, G2 = q.expect_grad_batched([P], [M], a, precision=0)
    assert np.array_equal(E, E2) and np.array_equal(G, G2)
