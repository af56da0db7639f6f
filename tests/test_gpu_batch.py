"""GPU parity of the batched entry points (pc_batch_skeleton, pc_batch_capture + pc_graph_launch)
against the FP64 oracle, dataset by dataset (marked gpu)."""
import numpy as np
import pytest

import oracle
import semgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_08491_amd as pc  # noqa: E402


def uneven_batch(count, seed, nmax=200, mmax=2000):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(3, nmax + 1))
        m = int(rng.integers(40, mmax + 1))
        d = float(rng.uniform(2, 8))
        sem = semgen.random_dag(n, semgen.expected_degree_p(n, d), rng)
        out.append((semgen.sample(sem, m, rng), float(rng.choice([0.01, 0.05])), int(rng.integers(-1, 4))))
    return out


def device_problem(ctx, X, alpha, max_level):
    m, n = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    return (Xd, alpha, max_level, adj, recs, count)


def check_one(X, alpha, max_level, item, status):
    m, n = X.shape
    _, _, _, adj, recs, count = item
    ref = oracle.skeleton(X, alpha, max_level=max_level)
    G = pc.bits_to_dense(adj.cpu().numpy(), n)
    assert status == {0: 0, 2: 1}[ref.status]          # oracle warning 2 = pc warning 1
    assert np.array_equal(G, ref.G), (n, m, alpha, max_level)
    k = int(count.item())
    seps = pc.decode_sepsets(recs[:k].cpu().numpy(), k)
    ref_seps = ref.sepsets.as_dict()
    assert set(seps) == set(ref_seps)
    C = oracle.corr(X)
    for e, (l, S) in seps.items():
        assert ref_seps[e][0] == l
        assert oracle.ci_test(C, e[0], e[1], list(S), m, alpha)[0]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_batch_skeleton_matches_oracle(prec):
    batch = uneven_batch(12, seed=40 + len(prec))
    ctx = pc.Context(precision=prec)
    items = [device_problem(ctx, X, a, ml) for X, a, ml in batch]
    probs = ctx.problems(items)
    ws = ctx.batch_workspace(probs)
    stats = (pc.pc_run_stats * len(items))()
    r, status = ctx.pc_batch_skeleton(probs, ws, stats)
    assert r >= 0
    for (X, a, ml), item, st in zip(batch, items, status):
        check_one(X, a, ml, item, st)


def test_graph_replays_match_oracle_with_new_data():
    batch = uneven_batch(8, seed=77)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = pc.Context(stream=stream, precision="fp32")
        items = [device_problem(ctx, X, a, ml) for X, a, ml in batch]
        probs = ctx.problems(items)
        ws = ctx.batch_workspace(probs)
        g = ctx.pc_batch_capture(probs, ws)
        rng = np.random.default_rng(5)
        for replay in range(3):
            if replay > 0:
                # new data of the same shapes, written into the captured buffers
                for k, (X, a, ml) in enumerate(batch):
                    sem = semgen.random_dag(X.shape[1], 0.05, rng)
                    Xn = semgen.sample(sem, X.shape[0], rng)
                    batch[k] = (Xn, a, ml)
                    items[k][0].copy_(torch.from_numpy(Xn))
                # unrelated eager work between replays
                junk = torch.randn(1024, 1024, device="cuda")
                (junk @ junk).sum().item()
            g.pc_graph_launch()
            r, status = g.pc_graph_results()
            assert r >= 0
            for (X, a, ml), item, st in zip(batch, items, status):
                check_one(X, a, ml, item, st)
        g.close()
    torch.cuda.synchronize()


def test_graph_rejects_null_stream():
    ctx = pc.Context(stream=torch.cuda.default_stream(), precision="fp32")
    X = np.random.default_rng(0).standard_normal((50, 5))
    items = [device_problem(ctx, X, 0.05, -1)]
    probs = ctx.problems(items)
    ws = ctx.batch_workspace(probs)
    if torch.cuda.default_stream().cuda_stream == 0:
        with pytest.raises(pc.PCError):
            ctx.pc_batch_capture(probs, ws)


def test_batch_reports_per_dataset_errors():
    batch = uneven_batch(3, seed=3)
    X_bad = batch[1][0].copy()
    X_bad[:, 0] = 1.0
    batch[1] = (X_bad, batch[1][1], batch[1][2])
    ctx = pc.Context(precision="fp32")
    items = [device_problem(ctx, X, a, ml) for X, a, ml in batch]
    probs = ctx.problems(items)
    ws = ctx.batch_workspace(probs)
    r, status = ctx.pc_batch_skeleton(probs, ws)
    assert status[1] == -3 and r == -3
    check_one(*batch[0], items[0], status[0])
    check_one(*batch[2], items[2], status[2])


@pytest.mark.parametrize("tail_tests", [0, 1, 2048, 1 << 20])
def test_graph_continues_past_recorded_levels(tail_tests):
    """A graph that records only 2 levels still yields whole skeletons: the tail kernel recorded
    after them runs the small levels (budget 2048 tests, or 1 << 20: every level up to 8; 0: no
    tail), and pc_graph_results runs whatever the datasets still need on the stream (with budget 1
    the tail hands every level back at once), on every replay."""
    batch = uneven_batch(6, seed=91, nmax=160)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        print(f"graph continuation tail_tests={tail_tests}", flush=True)
        ctx = pc.Context(stream=stream, precision="fp32", graph_levels=2, tail_tests=tail_tests)
        items = [device_problem(ctx, X, a, -1) for X, a, _ in batch]
        probs = ctx.problems(items)
        ws = ctx.batch_workspace(probs)
        g = ctx.pc_batch_capture(probs, ws)
        for replay in range(2):
            g.pc_graph_launch()
            stats = (pc.pc_run_stats * len(items))()
            r, status = g.pc_graph_results(stats)
            assert r >= 0
            assert max(st.levels_run for st in stats) > 3
            for (X, a, _), item, st in zip(batch, items, status):
                check_one(X, a, -1, item, st)
        g.close()
    torch.cuda.synchronize()


def test_batch256_in_one_graph_matches_oracle_on_sample():
    """The 256 uneven datasets (n ~ U[20,400], expected degree ~ U[2,8], m ~ U[200,5000], alpha 0.01)
    captured in one graph, replayed twice (second replay on the same data), then checked dataset by
    dataset against the oracle: the datasets of largest n, largest m and most GPU levels, and a
    seeded sample of 61 more (64 in all). Also every dataset's status and level count."""
    import os
    batch = semgen.batch_problems(256)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = pc.Context(stream=stream, precision="fp32")
        items = [device_problem(ctx, X, a, -1) for X, _, a in batch]
        probs = ctx.problems(items)
        ws = ctx.batch_workspace(probs)
        graph = ctx.pc_batch_capture(probs, ws)
        st = (pc.pc_run_stats * len(items))()
        for _ in range(2):
            graph.pc_graph_launch()
            r, status = graph.pc_graph_results(st)
        torch.cuda.synchronize()
        graph.close()
    assert r == 0 and all(s == 0 for s in status)
    ns = [X.shape[1] for X, _, _ in batch]
    ms = [X.shape[0] for X, _, _ in batch]
    levels = [st[d].levels_run for d in range(len(batch))]
    pick = {int(np.argmax(ns)), int(np.argmax(ms)), int(np.argmax(levels))}
    rng = np.random.default_rng(2560)
    for d in rng.permutation(len(batch)):
        if len(pick) >= 64:
            break
        pick.add(int(d))
    oracle.set_threads(min(16, os.cpu_count() or 1))
    try:
        for d in sorted(pick):
            X, _, a = batch[d]
            print(f"batch256 dataset {d}: n={X.shape[1]} m={X.shape[0]} levels={levels[d]}", flush=True)
            check_one(X, a, -1, items[d], status[d])
    finally:
        oracle.set_threads(1)


@pytest.mark.parametrize("rank", ["abs", "model"])
def test_ordered_graph_replays_match_oracle(rank):
    """pc_batch_capture_ordered: the shared-set order recorded into the graph (|C_ik| ranking, or a
    random row model scoring a short list), two ragged datasets, replayed twice; each skeleton is
    the oracle's and every SepSet passes the oracle's test."""
    from oracle import mlp
    batch = uneven_batch(2, seed=91, nmax=300, mmax=1500)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = pc.Context(stream=stream, precision="fp32", graph_levels=12)
        items = [device_problem(ctx, X, a, ml) for X, a, ml in batch]
        probs = ctx.problems(items)
        ws = ctx.batch_workspace(probs)
        params = torch.from_numpy(mlp.init(np.random.default_rng(9)).astype(np.float32)).cuda()
        order = (ctx.order(None, row_top=3, row_rank="abs") if rank == "abs"
                 else ctx.order(None, row_params=params, row_top=2, row_short=12))
        graph = ctx.pc_batch_capture(probs, ws, order)
        st = (pc.pc_run_stats * len(items))()
        for _ in range(2):
            graph.pc_graph_launch()
            r, status = graph.pc_graph_results(st)
        torch.cuda.synchronize()
        graph.close()
    assert r == 0
    for d, (X, a, ml) in enumerate(batch):
        check_one(X, a, ml, items[d], status[d])
        if st[d].levels_run > 1:
            assert st[d].probe_tests[1] > 0


def test_batch_of_more_problems_than_the_planner_reduces_in_lds():
    """4200 small datasets: past 4096 problems the planning pass folds each problem's maximum
    degree (the stop rule of Algorithm 2) with device atomics instead of in LDS; every dataset must
    still get the oracle's skeleton, SepSets and level count."""
    rng = np.random.default_rng(4200)
    batch = []
    for _ in range(4200):
        n = int(rng.integers(3, 13))
        m = int(rng.integers(40, 201))
        sem = semgen.random_dag(n, semgen.expected_degree_p(n, float(rng.uniform(1.5, 4))), rng)
        batch.append((semgen.sample(sem, m, rng), 0.05, -1))
    ctx = pc.Context(precision="fp32")
    items = [device_problem(ctx, X, a, ml) for X, a, ml in batch]
    probs = ctx.problems(items)
    ws = ctx.batch_workspace(probs)
    stats = (pc.pc_run_stats * len(items))()
    print("batch of 4200 problems", flush=True)
    r, status = ctx.pc_batch_skeleton(probs, ws, stats)
    assert r >= 0
    for (X, a, ml), item, st, s in zip(batch, items, status, stats):
        check_one(X, a, ml, item, st)
        ref = oracle.skeleton(X, a, max_level=ml)
        assert s.levels_run == ref.levels_run
