"""GPU: the torch.autograd.Function wrapper returns the library's <C> and d<C>/d(beta, gamma),
and a torch optimiser step on it moves <C> the right way (Sec. 2.3: gradient-based angle
finding maximises <C>); handle lifetimes through the C ABI."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def test_autograd_matches_oracle_and_optimiser_step():
    import torch
    import paper_2312_06451_amd as q
    from paper_2312_06451_amd.autograd import qaoa_expectation
    n, p = 14, 3
    g = workloads.random_regular_graph(n, 3, 611)
    a0 = workloads.random_angles(p, 1, 612)[0]
    t = oracle.graph_table(g)
    E0, N0, g0 = oracle.grad(n, t, a0)
    ctx = q.Context(0)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    for prec, tol in ((q.QAOA_FP32, 1e-5), (q.QAOA_FP64, 1e-11)):
        ang = torch.tensor(a0, dtype=torch.float64, requires_grad=True)
        e = qaoa_expectation(ang, P, M, prec)
        e.backward()
        assert abs(e.item() - E0 / N0) <= tol * abs(E0)
        assert np.max(np.abs(ang.grad.numpy() - g0 / N0)) <= tol * np.max(np.abs(g0))
        # chain rule through a scaling: d(3 <C>)/d angles = 3 g
        ang2 = torch.tensor(a0, dtype=torch.float64, requires_grad=True)
        (3.0 * qaoa_expectation(ang2, P, M, prec)).backward()
        assert np.allclose(ang2.grad.numpy(), 3.0 * ang.grad.numpy(), rtol=1e-12, atol=0)
    # no gradient requested: forward only, same value
    with torch.no_grad():
        e_ng = qaoa_expectation(torch.tensor(a0), P, M, q.QAOA_FP64)
    assert abs(e_ng.item() - E0 / N0) <= 1e-11 * abs(E0)
    # one ascent step of size 1e-3 raises <C> (to first order by 1e-3 |g|^2)
    ang = torch.tensor(a0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.SGD([ang], lr=1e-3, maximize=True)
    e_before = qaoa_expectation(ang, P, M, q.QAOA_FP64)
    e_before.backward()
    opt.step()
    with torch.no_grad():
        e_after = qaoa_expectation(ang, P, M, q.QAOA_FP64)
    assert e_after.item() > e_before.item()
    ctx.close()
    assert P.handle is None and M.handle is None


def test_context_outlives_its_problems():
    import paper_2312_06451_amd as q
    from paper_2312_06451_amd import _lib
    g = workloads.random_regular_graph(10, 3, 5)
    c = _lib.qaoa_ctx_create(0)
    prob = _lib.qaoa_cost_table(c, g.n, g.u, g.v, g.w, -1, 0)
    mix = _lib.qaoa_mixer_x(c, g.n)
    with pytest.raises(q.QAOAError) as ei:
        _lib.qaoa_ctx_destroy(c)
    assert ei.value.status == _lib.QAOA_ERR_INVALID_ARG
    # the context is untouched by the refused call
    assert abs(_lib.qaoa_expect(prob, mix, 1, np.array([0.0, 0.0]), 0, 1, 0) - g.total_weight / 2) < 1e-12
    _lib.qaoa_problem_destroy(prob)
    with pytest.raises(q.QAOAError):
        _lib.qaoa_ctx_destroy(c)
    _lib.qaoa_mixer_destroy(mix)
    _lib.qaoa_ctx_destroy(c)
