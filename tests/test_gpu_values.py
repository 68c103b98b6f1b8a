"""GPU parity for objectives given as value lists (qaoa_problem_from_values): real-valued and
complement-asymmetric costs (Sec. 2.1 pre-computation, Sec. 3 objective list) on the
whole-state kernel, both tile plans and the clique path, against the FP64 oracle.

Tolerances: FP32 1e-5 and FP64 1e-11, relative to max|C| for <C> (a real cost can have a mean
near zero) and to max|g| for the gradient."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
TOL = {0: 1e-5, 1: 1e-11}


@pytest.fixture(scope="module")
def q():
    import paper_2312_06451_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(q):
    c = q.Context(0)
    yield c
    c.close()


def real_values(N, seed, distinct=60):
    rng = np.random.default_rng(seed)
    pool = rng.normal(0.3, 3.0, distinct)
    return pool[rng.integers(0, distinct, N)]


def check(q, P, M, n, vals, a, prec, k=-1, psi0=None, d_psi0=None):
    E0, N0, g0 = oracle.grad(n, vals, a, k=k, psi0=psi0)
    e, gr = q.expect_grad(P, M, a, psi0=d_psi0, precision=prec)
    scale = np.max(np.abs(vals))
    assert abs(e - E0 / N0) <= TOL[prec] * scale, (n, prec, e, E0 / N0)
    assert np.max(np.abs(gr - g0 / N0)) <= TOL[prec] * np.max(np.abs(g0 / N0)), (n, prec)
    assert abs(q.expect(P, M, a, psi0=d_psi0, precision=prec) - e) <= TOL[prec] * scale


def test_graph_values_give_graph_results(q, ctx):
    for n, seed in ((10, 1), (16, 2), (22, 3)):
        g = workloads.random_regular_graph(n, 3, 700 + seed)
        t = oracle.graph_table(g)
        Pg, Pv = q.Problem.from_graph(ctx, g), q.Problem.from_values(ctx, n, t.astype(np.float64))
        M = q.Mixer.x(ctx, n)
        assert np.array_equal(Pv.values(), t.astype(np.float64))
        assert np.array_equal(Pg.values(), t.astype(np.float64))
        for a in workloads.random_angles(3, 2, 710 + seed):
            for prec in (0, 1):
                eg, gg = q.expect_grad(Pg, M, a, precision=prec)
                ev, gv = q.expect_grad(Pv, M, a, precision=prec)
                assert abs(eg - ev) <= 1e-12 * abs(eg)
                assert np.max(np.abs(gg - gv)) <= 1e-12 * np.max(np.abs(gg))


@pytest.mark.parametrize("n,p", [(10, 3), (12, 2), (14, 3), (17, 2), (18, 2), (22, 2)])
def test_real_asymmetric_values_vs_oracle(q, ctx, n, p):
    vals = real_values(1 << n, 720 + n)
    assert np.max(np.abs(vals - vals[::-1])) > 0.5
    P, M = q.Problem.from_values(ctx, n, vals), q.Mixer.x(ctx, n)
    assert np.array_equal(P.values(), vals)
    angles = workloads.random_angles(p, 3, 730 + n)
    # the tangent form is used for some rounds and the cotangent form for others
    assert np.any(np.abs(np.tan(angles[:, :p])) > 1) and np.any(np.abs(np.tan(angles[:, :p])) < 1)
    for a in angles:
        for prec in (0, 1):
            check(q, P, M, n, vals, a, prec)


def test_real_values_state_psi0_and_batched(q, ctx):
    import torch
    n, p = 15, 3
    vals = real_values(1 << n, 740)
    P, M = q.Problem.from_values(ctx, n, vals), q.Mixer.x(ctx, n)
    angles = workloads.random_angles(p, 4, 741)
    a = angles[0]
    want = oracle.state(n, vals, a)
    for prec, dt, tol in ((0, torch.complex64, 1e-5), (1, torch.complex128, 1e-11)):
        out = torch.empty(1 << n, dtype=dt, device="cuda")
        q.state(P, M, a, out, precision=prec)
        torch.cuda.synchronize()
        assert np.max(np.abs(out.cpu().numpy() - want)) * np.sqrt(1 << n) < tol
    rng = np.random.default_rng(742)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    for prec, dt in ((0, torch.complex64), (1, torch.complex128)):
        check(q, P, M, n, vals, a, prec, psi0=psi0, d_psi0=torch.tensor(psi0, dtype=dt, device="cuda"))
    # several angle sets and a second (small, symmetric) problem in one batched call
    g = workloads.random_regular_graph(10, 3, 743)
    Pg, Mg = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, 10)
    for prec in (0, 1):
        Eb, Gb = q.expect_grad_batched([P, Pg], [M, Mg], angles, precision=prec)
        for s in range(angles.shape[0]):
            e, gr = q.expect_grad(P, M, angles[s], precision=prec)
            assert abs(Eb[0, s] - e) <= 1e-6 * np.max(np.abs(vals)) and np.allclose(Gb[0, s], gr, rtol=0, atol=1e-6 * np.max(np.abs(gr)))
            e2, g2 = q.expect_grad(Pg, Mg, angles[s], precision=prec)
            assert abs(Eb[1, s] - e2) <= 1e-6 * abs(e2)


def test_real_values_clique(q, ctx):
    n, k, p = 10, 4, 3
    from math import comb
    vals = real_values(comb(n, k), 750)
    P, M = q.Problem.from_values(ctx, n, vals, hamming_k=k), q.Mixer.clique(ctx, n, k)
    assert np.array_equal(P.values(), vals)
    for a in workloads.random_angles(p, 2, 751):
        for prec in (0, 1):
            check(q, P, M, n, vals, a, prec, k=k)


def test_many_distinct_values_and_errors(q, ctx):
    from paper_2312_06451_amd import _lib
    n = 12
    rng = np.random.default_rng(760)
    vals = rng.permutation(np.arange(1 << n) % 1024) * 0.37 - 50.0     # exactly 1024 distinct values
    P, M = q.Problem.from_values(ctx, n, vals), q.Mixer.x(ctx, n)
    assert P.max_value == 1023
    a = workloads.random_angles(2, 1, 761)[0]
    for prec in (0, 1):
        check(q, P, M, n, vals, a, prec)
    too_many = np.arange(1 << n, dtype=np.float64)
    with pytest.raises(q.QAOAError) as ei:
        q.Problem.from_values(ctx, n, too_many)
    assert ei.value.status == _lib.QAOA_ERR_UNSUPPORTED
    bad = vals.copy()
    bad[5] = np.nan
    with pytest.raises(q.QAOAError) as ei:
        q.Problem.from_values(ctx, n, bad)
    assert ei.value.status == _lib.QAOA_ERR_INVALID_ARG
    with pytest.raises(q.QAOAError) as ei:
        q.Problem.from_values(ctx, n, vals[:-1])
    assert ei.value.status == _lib.QAOA_ERR_INVALID_ARG
    # -0.0 and 0.0 are one value
    z = np.zeros(1 << 10)
    z[1::2] = -0.0
    Pz = q.Problem.from_values(ctx, 10, z)
    assert Pz.max_value == 0
