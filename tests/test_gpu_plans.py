"""Tile-pass plans: each option of a plan (reverse sweep in place or from checkpoints, tile
cover, low-qubit placement, first-round tile order, which tile takes the round boundaries,
workgroup order) gives the oracle's
results; the tuner's choice is shared by single and batched evaluations (bit-identical) and a
saved plan file reproduces a run bit for bit in a new context. The narrow-run covers (three
tiles instead of four: n = 30..33 in FP32, 29..32 in FP64) are checked at full size against
the cycle light cone, which holds at any size."""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {0: (1e-5, 1e-5), 1: (1e-12, 1e-11)}   # precision -> (<C> rel, grad inf-rel)
OPTS = ("narrow", "narrow_top", "lowbits", "down", "xcd", "ckpt", "swap", "swz")
DEFAULT = dict(narrow=1, narrow_top=1, lowbits=1, down=0, xcd=1, ckpt=-1, swap=0, swz=1)


@pytest.fixture(scope="module")
def q():
    import paper_2312_06451_amd as q
    return q


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _gerr(g, ref):
    return float(np.max(np.abs(np.asarray(g) - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _plan_file(path, n, opts):
    """A plan file that gives every key of n (both precisions, with and without gradient,
    checkpoints fitting or not) the options `opts` (transverse-field mixer)."""
    o = dict(DEFAULT, **opts)
    vals = " ".join(str(o[k]) for k in OPTS)
    with open(path, "w") as f:
        f.write("qaoa-plans 3\n")
        for prec in (0, 1):
            for grad in (0, 1):
                for fits in (0, 1):
                    f.write(f"{n} {prec} {grad} 0 {fits} : {vals}\n")


def _cycle(n):
    u = np.arange(n, dtype=np.int32)
    v = (u + 1) % n
    return workloads.Graph(n, np.minimum(u, v).astype(np.int32), np.maximum(u, v).astype(np.int32),
                           np.ones(n, dtype=np.int32))


@pytest.fixture(scope="module")
def reg22():
    g = workloads.random_regular_graph(22, 3, 2222)
    a = workloads.random_angles(3, 1, 2223)[0]
    E, Nr, G = oracle.grad(22, oracle.graph_table(g), a)
    return g, a, E / Nr, G / Nr


@pytest.mark.parametrize("opts", [{}, {"lowbits": 0}, {"down": 1}, {"xcd": 0}, {"ckpt": 0}, {"swap": 1},
                                  {"swap": 1, "ckpt": 0}, {"down": 1, "lowbits": 0, "xcd": 0, "ckpt": 0}])
def test_plan_options_match_oracle(q, tmp_path, reg22, opts):
    """n = 22, p = 3 (three tiles in both precisions): every option against the FP64 oracle,
    forward and fwd+grad, after loading the plan from a file."""
    g, a, E, G = reg22
    path = str(tmp_path / "plans.txt")
    _plan_file(path, 22, opts)
    ctx = q.Context(0)
    ctx.load_plans(path)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, 22)
    for prec in (0, 1):
        e, gr = q.expect_grad(P, M, a, precision=prec)
        e1 = q.expect(P, M, a, precision=prec)
        print("plan", opts, "prec", prec, "E err", _rel(e, E), "grad err", _gerr(gr, G), flush=True)
        assert _rel(e, E) < TOL[prec][0] and _rel(e1, E) < TOL[prec][0]
        assert _gerr(gr, G) < TOL[prec][1]
    text = ctx.plans()
    assert text.splitlines()[0] == "qaoa-plans 3" and len(text.splitlines()) == 9
    P.close(); M.close(); ctx.close()


def test_tuner_shared_by_single_and_batched(q, tmp_path, reg22):
    """With the tuner on, the first evaluation measures the plan of its key; a batched call over
    several angle sets follows the same plan (bit-identical to single evaluations), and a new
    context that loads the saved plans reproduces both bit for bit."""
    g, a, E, G = reg22
    sets = np.vstack([a, workloads.random_angles(3, 2, 2224)])
    ctx = q.Context(0)
    ctx.set_autotune(True)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, 22)
    e0, g0 = q.expect_grad(P, M, a, precision=0)
    lines = ctx.plans().splitlines()
    print("tuned plans:", lines, flush=True)
    assert len(lines) == 2 and lines[1].startswith("22 0 1 0 ")
    assert _rel(e0, E) < TOL[0][0] and _gerr(g0, G) < TOL[0][1]
    eb, gb = q.expect_grad_batched([P], [M], sets, precision=0)
    assert eb[0, 0] == e0 and np.array_equal(gb[0, 0], g0)
    singles = [q.expect_grad(P, M, s, precision=0) for s in sets]
    for i, (es, gs) in enumerate(singles):
        assert eb[0, i] == es and np.array_equal(gb[0, i], gs)
    path = str(tmp_path / "tuned.txt")
    ctx.save_plans(path)
    ctx2 = q.Context(0)
    ctx2.load_plans(path)
    assert ctx2.plans() == ctx.plans()
    P2, M2 = q.Problem.from_graph(ctx2, g), q.Mixer.x(ctx2, 22)
    e2, g2 = q.expect_grad(P2, M2, a, precision=0)
    assert e2 == e0 and np.array_equal(g2, g0)
    for c, PP, MM in ((ctx, P, M), (ctx2, P2, M2)):
        PP.close(); MM.close(); c.close()


def test_batched_call_does_not_tune(q, reg22):
    """A batched call never tunes: with no plan for its key it follows the fixed rule (bit for
    bit the same as a context that does not tune) and records nothing; a later single
    evaluation tunes the key, and batched calls follow that choice from then on."""
    g, a, E, G = reg22
    sets = np.vstack([a, workloads.random_angles(3, 3, 2225)])
    ctx, ref = q.Context(0), q.Context(0)
    ctx.set_autotune(True)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, 22)
    Pr, Mr = q.Problem.from_graph(ref, g), q.Mixer.x(ref, 22)
    eb, gb = q.expect_grad_batched([P], [M], sets, precision=0)
    er, gr = q.expect_grad_batched([Pr], [Mr], sets, precision=0)
    assert ctx.plans() == "qaoa-plans 3\n"
    assert np.array_equal(eb, er) and np.array_equal(gb, gr)
    assert _rel(eb[0, 0], E) < TOL[0][0] and _gerr(gb[0, 0], G) < TOL[0][1]
    e0, g0 = q.expect_grad(P, M, a, precision=0)
    lines = ctx.plans().splitlines()
    assert len(lines) == 2 and lines[1].startswith("22 0 1 0 ")
    eb2, gb2 = q.expect_grad_batched([P], [M], sets, precision=0)
    assert eb2[0, 0] == e0 and np.array_equal(gb2[0, 0], g0)
    for c, PP, MM in ((ctx, P, M), (ref, Pr, Mr)):
        PP.close(); MM.close(); c.close()


def test_plan_file_rejects_malformed(q, tmp_path):
    ctx = q.Context(0)
    bad = tmp_path / "bad.txt"
    bad.write_text("qaoa-plans 3\n22 0 1 0 1 : 1 1 1 0 1 -1 0\n")   # one option missing
    with pytest.raises(q.QAOAError):
        ctx.load_plans(str(bad))
    bad.write_text("qaoa-plans 3\n22 0 1 0 1 : 1 1 1 0 1 -1 0 2\n")   # layout option out of range
    with pytest.raises(q.QAOAError):
        ctx.load_plans(str(bad))
    bad.write_text("plans\n")
    with pytest.raises(q.QAOAError):
        ctx.load_plans(str(bad))
    assert ctx.plans() == "qaoa-plans 3\n"
    # a version-1 file (no swap field) loads with swap = 0, versions 1 and 2 (no layout field)
    # with swz = 1
    old = tmp_path / "v1.txt"
    old.write_text("qaoa-plans 1\n22 0 1 0 1 : 1 1 1 1 1 -1\n")
    ctx.load_plans(str(old))
    assert ctx.plans().splitlines()[1] == "22 0 1 0 1 : 1 1 1 1 1 -1 0 1"
    old.write_text("qaoa-plans 2\n23 0 1 0 1 : 1 1 1 1 1 -1 1\n")
    ctx.load_plans(str(old))
    assert ctx.plans().splitlines()[2] == "23 0 1 0 1 : 1 1 1 1 1 -1 1 1"
    ctx.close()


@pytest.mark.parametrize("n,prec", [(30, 0), (29, 1)])
def test_narrow_cover_light_cone(q, tmp_path, n, prec):
    """The first sizes whose fewest-tile cover takes narrow runs (FP32 n = 30: 13 + 9 + 8 bits
    with 64- and 128-byte runs; FP64 n = 29: 12 + 9 + 8 bits), fwd+grad on the cycle C_n at
    p = 3 against the light cone (dense evolution of the 8-vertex path, no oracle), with the
    narrow cover in the swizzled layout (the fixed rule) and in the natural one, and with the
    four-tile cover, loaded from plan files. The layout changes addresses only: the two narrow
    runs agree bit for bit."""
    from tests import pins
    p = 3
    g = _cycle(n)
    a = workloads.random_angles(p, 1, 4130 + n)[0]
    ev, eg = pins.cycle_edge(p, a)
    res = {}
    for narrow, swz in ((1, 1), (1, 0), (0, 1)):
        ctx = q.Context(0)
        path = str(tmp_path / f"plans{narrow}{swz}.txt")
        _plan_file(path, n, {"narrow": narrow, "swz": swz})
        ctx.load_plans(path)
        P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
        e, gr = q.expect_grad(P, M, a, precision=prec)
        print(f"n={n} prec={prec} narrow={narrow} swz={swz}: E err {_rel(e, n * ev):.2e} grad err "
              f"{np.max(np.abs(gr - n * eg)) / (n * np.max(np.abs(eg))):.2e}", flush=True)
        assert _rel(e, n * ev) < TOL[prec][0]
        assert np.max(np.abs(gr - n * eg)) < max(TOL[prec][1], 1e-9) * n * np.max(np.abs(eg))
        res[narrow, swz] = (e, gr)
        P.close(); M.close(); ctx.close()
    assert res[1, 1][0] == res[1, 0][0] and np.array_equal(res[1, 1][1], res[1, 0][1])
    assert _rel(res[1, 1][0], res[0, 1][0]) < TOL[prec][0]


@pytest.mark.parametrize("n,prec,weighted", [(30, 0, False), (29, 1, False), (30, 0, True)])
def test_swizzled_layout_bit_identical(q, tmp_path, n, prec, weighted):
    """The swizzled state layout of the narrow covers (the top ten index bits folded into ten
    middle ones; per tile the add form, the XOR form, or the XOR form with cached accesses for
    runs under 128 bytes) against the natural layout, on a random 3-regular (n even) or
    4-regular (n odd) graph at p = 2: <C> and the gradient bit for bit, with the reverse sweep
    from checkpoints and in place, and <C> alone. A wrong address anywhere in the swizzled
    passes (a lost or doubled element, an element read from the wrong place) changes the
    results. A caller's initial state (natural order) runs the natural layout under either
    plan. The weighted case (G(n, 1/2), weights U{1..4}) takes 16-bit tables."""
    import torch
    p = 2
    if weighted:
        g = workloads.erdos_renyi(n, 7300 + n, 0.5, (1, 4))
    else:
        g = workloads.random_regular_graph(n, 3 if n % 2 == 0 else 4, 7300 + n)
    a = workloads.random_angles(p, 1, 7301 + n)[0]
    gen = torch.Generator(device="cuda").manual_seed(7302 + n)
    dt = torch.complex64 if prec == 0 else torch.complex128
    psi0 = torch.randn(1 << n, dtype=dt, device="cuda", generator=gen)
    res = {}
    for swz in (1, 0):
        for ckpt in (-1, 0):
            ctx = q.Context(0)
            path = str(tmp_path / f"plans{swz}{ckpt}.txt")
            _plan_file(path, n, {"swz": swz, "ckpt": ckpt})
            ctx.load_plans(path)
            P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
            assert (P.max_value > 255) == weighted
            res[swz, ckpt] = (q.expect_grad(P, M, a, precision=prec), q.expect(P, M, a, precision=prec),
                              q.expect_grad(P, M, a, psi0=psi0, precision=prec))
            P.close(); M.close(); ctx.close()
    del psi0
    torch.cuda.empty_cache()
    for ckpt in (-1, 0):
        (e1, g1), x1, (f1, h1) = res[1, ckpt]
        (e0, g0), x0, (f0, h0) = res[0, ckpt]
        print(f"n={n} prec={prec} ckpt={ckpt}: E {e1!r} / {e0!r}, expect {x1!r} / {x0!r}", flush=True)
        assert e1 == e0 and np.array_equal(g1, g0) and x1 == x0
        assert f1 == f0 and np.array_equal(h1, h0)
    # the two reverse sweeps agree to rounding
    assert _rel(res[1, -1][0][0], res[1, 0][0][0]) < TOL[prec][0]


def test_n32_cycle_light_cone_p8(q):
    """n = 32 (three tiles with narrow runs, reverse sweep in place) at p = 8 on the cycle C_32
    against the light cone (path of 18 vertices, block-exponential mixer, no oracle): <C> and
    three gradient entries, both precisions."""
    from tests import pins
    n, p = 32, 8
    g = _cycle(n)
    a = workloads.random_angles(p, 1, 4832)[0]
    comps = [0, p - 1, p]
    ev, eg = pins.cycle_edge_blocks(p, a, components=comps)
    ctx = q.Context(0)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, n)
    for prec in (0, 1):
        e, gr = q.expect_grad(P, M, a, precision=prec)
        print(f"n=32 p=8 prec={prec}: E err {_rel(e, n * ev):.2e}", flush=True)
        assert _rel(e, n * ev) < TOL[prec][0]
        scale = n * np.nanmax(np.abs(eg))
        for i in comps:
            assert abs(gr[i] - n * eg[i]) < max(TOL[prec][1], 1e-9) * scale
    P.close(); M.close(); ctx.close()


@pytest.mark.parametrize("narrow_top", [1, 0])
def test_n28_cover_options_vs_golden(q, tmp_path, narrow_top):
    """n = 28, FP32 and FP64, in the benchmark's configuration (random 3-regular graph, p = 8,
    checkpointed reverse sweep): the cover with the extra strided bit in the top tile
    (narrow_top = 1, the fixed rule: B = [0,6) + [13,20), C = [0,5) + [20,28) in FP32) and in
    the middle tile (narrow_top = 0) against the stored oracle values."""
    import json
    here = os.path.dirname(os.path.abspath(__file__))
    G = json.load(open(os.path.join(here, "golden", "maxcut3reg_n28_p8.json")))
    W = workloads.workload("maxcut3reg_n28_p8")
    g = W.graphs[0]
    s = G["sets"][0]
    assert np.array_equal(np.array(s["angles"]), W.angles[0])
    path = str(tmp_path / "plans.txt")
    _plan_file(path, 28, {"narrow_top": narrow_top})
    ctx = q.Context(0)
    ctx.load_plans(path)
    P, M = q.Problem.from_graph(ctx, g), q.Mixer.x(ctx, 28)
    for prec in (0, 1):
        e, gr = q.expect_grad(P, M, W.angles[0], precision=prec)
        print(f"n28 narrow_top={narrow_top} prec={prec}: E err {_rel(e, s['expect']):.2e} "
              f"grad err {_gerr(gr, np.array(s['grad'])):.2e}", flush=True)
        assert _rel(e, s["expect"]) < TOL[prec][0]
        assert _gerr(gr, np.array(s["grad"])) < TOL[prec][1]
    P.close(); M.close(); ctx.close()
