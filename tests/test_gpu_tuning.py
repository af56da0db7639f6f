"""Autotuned launch shapes (pc_tune, pc_set_tuning; marked gpu).

The skeleton of PC-stable does not depend on how the work of a level is cut into items or staged
(Sec. 2.4), so any per-level shapes must give the oracle's skeleton; the tuner keeps, per level,
the fastest shapes it timed, never slower than the context's own (it starts from them).
"""
import numpy as np
import pytest

import oracle
import semgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_08491_amd as pc  # noqa: E402


def _problem(ctx, X, alpha, max_level=-1):
    m, n = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    return (Xd, alpha, max_level, adj, recs, count)


def _check(item, X, alpha, ref):
    Xd, a, ml, adj, recs, count = item
    m, n = X.shape
    G = pc.bits_to_dense(adj.cpu().numpy(), n)
    assert np.array_equal(G, ref.G), np.argwhere(G != ref.G)[:8]
    k = int(count.item())
    seps = pc.decode_sepsets(recs[:k].cpu().numpy(), k)
    assert set(seps) == set(ref.sepsets.as_dict())
    C = oracle.corr(X)
    for (i, j), (l, S) in list(seps.items())[:400]:
        assert oracle.ci_test(C, i, j, list(S), m, alpha)[0], (i, j, S)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tune_keeps_the_oracle_skeleton(prec):
    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    ref = oracle.skeleton_corr(oracle.corr(X), X.shape[0], alpha)
    ctx = pc.Context(precision=prec)
    item = _problem(ctx, X, alpha)
    probs = ctx.problems([item])
    ws = ctx.batch_workspace(probs)
    print(f"tune n1000 {prec}", flush=True)
    t = ctx.pc_tune(probs, ws)
    d = t.as_dict()
    assert d["levels"] == ref.levels_run and d["runs"] >= 30
    for l in range(1, ref.levels_run):
        assert 0 < d["level_ms"][l] <= d["default_ms"][l], (l, d)
    _check(item, X, alpha, ref)               # the outputs of the last tuning run
    r, status = ctx.pc_batch_skeleton(probs, ws)
    assert r == 0 and status == [0]
    _check(item, X, alpha, ref)               # a run with the tuning applied


def test_extreme_shapes_and_graph_capture_keep_the_skeleton():
    """Items of one test per lane, the global-memory gather path and 8 sets per lane at every level
    (planning and level kernels must agree on the item size level by level), eager and captured."""
    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    ref = oracle.skeleton_corr(oracle.corr(X), X.shape[0], alpha)
    ext = pc.pc_tuning.from_dict({"tests_per_lane": [1] * (pc.PC_MAX_LEVEL + 1),
                                   "ranks_per_lane": [8] * (pc.PC_MAX_LEVEL + 1),
                                   "lds_budget": [0] * (pc.PC_MAX_LEVEL + 1),
                                   "set_lanes": [64] * (pc.PC_MAX_LEVEL + 1)})
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = pc.Context(stream=stream, precision="fp32")
        ctx.pc_set_tuning(ext)
        item = _problem(ctx, X, alpha)
        probs = ctx.problems([item])
        ws = ctx.batch_workspace(probs)
        r, status = ctx.pc_batch_skeleton(probs, ws)
        assert r == 0 and status == [0]
        _check(item, X, alpha, ref)
        g = ctx.pc_batch_capture(probs, ws)
        for replay in range(2):
            g.pc_graph_launch()
            r, status = g.pc_graph_results()
            torch.cuda.synchronize()
            assert r == 0 and status == [0]
            _check(item, X, alpha, ref)
        g.close()
        ctx.pc_set_tuning(None)
        for bad in ({"lds_budget": [-2]}, {"set_lanes": [0, 3]}, {"set_lanes": [0, 128]}):
            with pytest.raises(pc.PCError):
                ctx.pc_set_tuning(pc.pc_tuning.from_dict(bad))


def test_set_lanes_keep_the_skeleton():
    """Fewer or more lanes per level-1 and level-2 conditioning set change how many of a short row's
    sets run at once (and so how many speculative tests run), never the skeleton; a whole wavefront
    per set runs fewer level-1 tests than four lanes per set on this short-row workload."""
    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    ref = oracle.skeleton_corr(oracle.corr(X), X.shape[0], alpha)
    tests1 = {}
    for lanes in (4, 16, 64):
        ctx = pc.Context(precision="fp32")
        ctx.pc_set_tuning(pc.pc_tuning.from_dict({"set_lanes": [0, lanes, lanes]}))
        item = _problem(ctx, X, alpha)
        probs = ctx.problems([item])
        ws = ctx.batch_workspace(probs)
        stats = (pc.pc_run_stats * 1)()
        print(f"set_lanes {lanes}", flush=True)
        r, status = ctx.pc_batch_skeleton(probs, ws, stats)
        assert r == 0 and status == [0]
        _check(item, X, alpha, ref)
        tests1[lanes] = int(stats[0].tests[1])
    print("level-1 tests by set_lanes", tests1, flush=True)
    assert tests1[64] < tests1[4]


def test_tuning_cache_round_trip(tmp_path):
    """A tuning stored in a cache file under its workload key is applied by the next pc_tune on the
    same workload without a search (no skeleton runs), and keeps the oracle's skeleton; another
    precision gets a key of its own."""
    import json

    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    ref = oracle.skeleton_corr(oracle.corr(X), X.shape[0], alpha)
    cache = str(tmp_path / "tuning.json")
    ctx = pc.Context(precision="fp32")
    item = _problem(ctx, X, alpha)
    probs = ctx.problems([item])
    ws = ctx.batch_workspace(probs)
    print("tune with a cache file", flush=True)
    t1 = ctx.pc_tune(probs, ws, cache=cache)
    with open(cache) as f:
        assert list(json.load(f)) == [ctx.tuning_key(probs)]
    ctx2 = pc.Context(precision="fp32")
    item2 = _problem(ctx2, X, alpha)
    probs2 = ctx2.problems([item2])
    ws2 = ctx2.batch_workspace(probs2)
    assert ctx2.tuning_key(probs2) == ctx.tuning_key(probs)
    t2 = ctx2.pc_tune(probs2, ws2, cache=cache)
    assert t2.as_dict() == t1.as_dict()
    assert int(item2[5].item()) == 0          # nothing ran: the SepSet counter is untouched
    r, status = ctx2.pc_batch_skeleton(probs2, ws2)
    assert r == 0 and status == [0]
    _check(item2, X, alpha, ref)
    ctx3 = pc.Context(precision="fp64")
    probs3 = ctx3.problems([_problem(ctx3, X, alpha)])
    assert ctx3.tuning_key(probs3) != ctx.tuning_key(probs)


def test_tune_ordered_and_dense_rows():
    """The ordered form (count 1 with an order) on the n = 2000 workload, and the paper's dense
    family at n = 1000, where item size matters most (long rows)."""
    from paper_1812_08491_amd import learn

    X, sem, alpha = semgen.workload("n2000_d10_m1000_apply")
    ref = oracle.skeleton_corr(oracle.corr(X), X.shape[0], alpha)
    ctx = pc.Context(precision="fp32")
    item = _problem(ctx, X, alpha)
    probs = ctx.problems([item])
    ws = ctx.batch_workspace(probs)
    params = learn.load_weights(learn.ROW_WEIGHTS)
    order = ctx.order(None, row_params=params, row_top=2, row_short=learn.ROW_SHORT, row_sort=True,
                      row_split=32)
    print("tune ordered n2000", flush=True)
    t = ctx.pc_tune(probs, ws, order=order)
    _check(item, X, alpha, ref)
    print("tuned n2000 level ms", [round(x, 3) for x in t.as_dict()["level_ms"][:4]],
          "default", [round(x, 3) for x in t.as_dict()["default_ms"][:4]], flush=True)
    Xs, _, alpha_s = semgen.scalability(1000, 0.1, 10000)
    C = oracle.corr(Xs)
    refs = oracle.skeleton_corr(C, Xs.shape[0], alpha_s)
    sctx = pc.Context(precision="fp64")
    sitem = _problem(sctx, Xs, alpha_s)
    sprobs = sctx.problems([sitem])
    sws = sctx.batch_workspace(sprobs)
    print("tune paper scalability n1000", flush=True)
    ts = sctx.pc_tune(sprobs, sws).as_dict()
    print("tuned level ms", [round(x, 3) for x in ts["level_ms"][:4]], "default",
          [round(x, 3) for x in ts["default_ms"][:4]], "tests_per_lane", ts["tests_per_lane"][:4], flush=True)
    assert ts["level_ms"][1] <= ts["default_ms"][1]
    G = pc.bits_to_dense(sitem[3].cpu().numpy(), 1000)
    # near-collinear data: the same pairs as the pc_skeleton path may differ from the oracle
    assert int((G != refs.G).sum()) // 2 <= 50


def test_timed_runs_with_the_tail_kernel():
    """Levels the tail kernel runs record no timing events: a timed call must read back only the
    events it recorded, and leave no error behind for the next call (pc_tune makes 42 timed calls
    in a row; a captured graph with the tail follows)."""
    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    ref = oracle.skeleton_corr(oracle.corr(X), X.shape[0], alpha)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = pc.Context(stream=stream, precision="fp32", timing=1 | 2 | 4 | 8, tail_tests=1 << 30, graph_levels=3)
        item = _problem(ctx, X, alpha)
        probs = ctx.problems([item])
        ws = ctx.batch_workspace(probs)
        for _ in range(2):
            st = (pc.pc_run_stats * 1)()
            r, status = ctx.pc_batch_skeleton(probs, ws, st)
            assert r == 0 and status == [0]
            _check(item, X, alpha, ref)
            d = st[0].as_dict()
            assert d["level_ms"][1] > 0 and d["corr_ms"] > 0
        t = ctx.pc_tune(probs, ws).as_dict()
        assert t["runs"] >= 30
        _check(item, X, alpha, ref)
        g = ctx.pc_batch_capture(probs, ws)
        g.pc_graph_launch()
        r, status = g.pc_graph_results()
        torch.cuda.synchronize()
        assert r == 0 and status == [0]
        _check(item, X, alpha, ref)
        g.close()
