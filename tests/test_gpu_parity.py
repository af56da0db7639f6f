"""GPU parity of libpc.so against the FP64 CPU oracle (runs on an MI355X; marked gpu).

Every call goes through the C ABI (ctypes binding). Inputs are seeded synthetic SEM data. The bar:
  * C within the stated bound of the FP64 correlation (blocked accumulation with compensated block
    sums, so the bound does not grow with m; u = 2^-24: FP32 37u; BF16x3 (3 + 2^-7) 2^-16 + 195u;
    FP64 1e-12);
  * the adjacency after level 0, after every level and at the end bit-identical to the oracle's;
  * every GPU SepSet passes the oracle's FP64 test at its level, drawn from G' of that level;
  * a re-check queue that overflows completes the level in FP64 with the same skeleton.
"""
import math

import numpy as np
import pytest

import oracle
import semgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_08491_amd as pc  # noqa: E402

U32 = 2.0 ** -24


def eps_c(prec, m):
    # the stated bound on |C - C_64| (blocked accumulation with compensated block sums)
    if prec == "fp32":
        return 37 * U32
    if prec == "bf16x3":
        return (3 + 2.0 ** -7) * 2.0 ** -16 + 195 * U32
    return 1e-12


def sem_data(seed, n, p, m):
    rng = np.random.default_rng(seed)
    sem = semgen.random_dag(n, p, rng)
    return semgen.sample(sem, m, rng)


def gpu_corr(X, alpha, prec, **opt):
    m, n = X.shape
    ctx = pc.Context(precision=prec, **opt)
    ws = ctx.workspace(n, m)
    Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    C = torch.empty((n, n), dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda")
    adj = ctx.adjacency(n)
    ctx.pc_corr(Xt, alpha, ws, C_out=C, adj_out=adj)
    assert ctx.pc_sync_status(ws) == 0
    return ctx, ws, Xt, C.double().cpu().numpy(), pc.bits_to_dense(adj.cpu().numpy(), n)


def check_sepsets(seps, C64, m, alpha, G_before_level):
    for (i, j), (l, S) in seps.items():
        assert i < j and len(S) == l and list(S) == sorted(S)
        Gp = G_before_level[l]
        assert all(Gp[i, s] for s in S) or all(Gp[j, s] for s in S), (i, j, l, S)
        ind, z, t = oracle.ci_test(C64, i, j, list(S), m, alpha)
        assert ind, (i, j, l, S, z, t)


# ---------------------------------------------------------------------------------------------
# Correlation + level 0
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("n,m,seed", [(50, 1000, 1), (130, 333, 2), (64, 64, 3), (2, 4, 4),
                                      (1000, 500, 5), (257, 1999, 6)])
def test_corr_and_level0(prec, n, m, seed):
    X = sem_data(seed, n, min(1.0, 4.0 / max(1, n - 1)), m)
    alpha = 0.01
    print(f"corr prec={prec} n={n} m={m} seed={seed}", flush=True)
    ctx, ws, Xt, C, G0 = gpu_corr(X, alpha, prec)
    C64 = oracle.corr(X)
    err = np.abs(C - C64).max()
    assert err <= eps_c(prec, m), err
    assert np.all(np.diag(C) == 1.0)
    assert np.array_equal(C, C.T)
    Gref, _, _ = oracle.level0(C64, m, alpha)
    assert np.array_equal(G0, Gref)


def test_corr_audit_mode_level0_all_rechecked():
    X = sem_data(11, 200, 0.03, 300)
    ctx, ws, Xt, C, G0 = gpu_corr(X, 0.05, "fp32", force_recheck_all=1)
    Gref, _, _ = oracle.level0(oracle.corr(X), 300, 0.05)
    assert np.array_equal(G0, Gref)


def test_corr_errors():
    X = sem_data(3, 40, 0.1, 100)
    X[:, 7] = 2.5
    ctx = pc.Context(precision="fp32")
    ws = ctx.workspace(40, 100)
    Xt = torch.from_numpy(X).cuda()
    ctx.pc_corr(Xt, 0.01, ws)
    with pytest.raises(pc.PCError) as e:
        ctx.pc_sync_status(ws)
    assert e.value.status == -3
    X = sem_data(3, 40, 0.1, 100)
    X[5, 1] = np.inf
    Xt = torch.from_numpy(X).cuda()
    ctx.pc_corr(Xt, 0.01, ws)
    with pytest.raises(pc.PCError) as e:
        ctx.pc_sync_status(ws)
    assert e.value.status == -4
    with pytest.raises(pc.PCError):
        ctx.pc_corr(Xt[:3].contiguous(), 0.01, ws)       # m < 4


# ---------------------------------------------------------------------------------------------
# One level at a time from the oracle's G'
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec,n,p,m,alpha,seed", [
    ("fp64", 50, 0.05, 1000, 0.01, 1001),
    ("fp32", 60, 0.3, 400, 0.05, 21),
    ("fp32", 150, 0.08, 700, 0.05, 22),
    ("bf16x3", 150, 0.08, 700, 0.05, 23),
    ("fp64", 90, 0.2, 300, 0.05, 24),
])
def test_levels_from_oracle_snapshots(prec, n, p, m, alpha, seed):
    X = sem_data(seed, n, p, m)
    C64 = oracle.corr(X)
    ref = oracle.skeleton_corr(C64, m, alpha, keep_levels=True)
    print(f"levels prec={prec} n={n} seed={seed} levels={ref.levels_run}", flush=True)
    ctx, ws, Xt, C, G0 = gpu_corr(X, alpha, prec)
    assert np.array_equal(G0, ref.G_after[0])
    recs, count = ctx.sepsets(n * n)
    G_before = {}
    for l in range(1, ref.levels_run):
        Gp = ref.G_after[l - 1]
        G_before[l] = Gp
        adj = torch.from_numpy(pc.dense_to_bits(Gp)).cuda()
        st = pc.pc_run_stats()
        status = ctx.pc_level(l, n, m, alpha, adj, recs, count, ws, stats=st)
        assert status == 0
        G = pc.bits_to_dense(adj.cpu().numpy(), n)
        assert np.array_equal(G, ref.G_after[l]), (l, np.argwhere(G != ref.G_after[l])[:5])
    k = int(count.item())
    check_sepsets(pc.decode_sepsets(recs[:k].cpu().numpy(), k), C64, m, alpha, G_before)


# ---------------------------------------------------------------------------------------------
# Whole skeleton
# ---------------------------------------------------------------------------------------------
def run_skeleton(X, alpha, prec, max_level=-1, **opt):
    m, n = X.shape
    ctx = pc.Context(precision=prec, **opt)
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    st = pc.pc_run_stats()
    Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    status = ctx.pc_skeleton(Xt, alpha, adj, recs, count, ws, max_level=max_level, stats=st)
    k = int(count.item())
    G = pc.bits_to_dense(adj.cpu().numpy(), n)
    return G, pc.decode_sepsets(recs[:k].cpu().numpy(), k), st.as_dict(), status


def compare_with_oracle(X, alpha, prec, max_level=-1, **opt):
    m, n = X.shape
    C64 = oracle.corr(X)
    ref = oracle.skeleton_corr(C64, m, alpha, max_level=max_level, keep_levels=True)
    G, seps, st, status = run_skeleton(X, alpha, prec, max_level=max_level, **opt)
    assert status == {0: 0, 2: 1}[ref.status]          # oracle warning 2 = pc warning 1
    assert np.array_equal(G, ref.G), np.argwhere(G != ref.G)[:8]
    assert st["levels_run"] == ref.levels_run
    # same removal level per edge: every oracle record has a GPU record at the same level
    ref_seps = ref.sepsets.as_dict()
    assert set(seps) == set(ref_seps)
    for e, (l, S) in ref_seps.items():
        assert seps[e][0] == l, (e, seps[e], (l, S))
    G_before = {l: ref.G_after[l - 1] for l in range(1, ref.levels_run)}
    check_sepsets(seps, C64, m, alpha, G_before)
    return st, ref


def test_skeleton_n50_fp64():
    X, sem, alpha = semgen.workload("n50_p005_m1000_fp64")
    print("skeleton n50 fp64", flush=True)
    compare_with_oracle(X, alpha, "fp64")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_skeleton_n1000_d4_m500(prec):
    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    print(f"skeleton n1000 {prec}", flush=True)
    st, ref = compare_with_oracle(X, alpha, prec)
    assert st["tests"][0] == 1000 * 999 // 2


@pytest.mark.parametrize("seed", range(4))
def test_skeleton_small_ragged(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 140))
    X = sem_data(500 + seed, n, float(rng.uniform(0.05, 0.4)), int(rng.integers(30, 900)))
    print(f"skeleton ragged seed={seed} n={n}", flush=True)
    compare_with_oracle(X, 0.05, ["fp32", "bf16x3", "fp64", "fp32"][seed])


def test_skeleton_audit_mode_no_violations():
    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    st, ref = compare_with_oracle(X, alpha, "fp32", force_recheck_all=1, recheck_cap=1 << 22)
    assert sum(st["audit_violations"]) == 0
    assert st["rechecks"][1] > 0


def test_skeleton_max_level_and_global_gather_path():
    X = sem_data(77, 120, 0.2, 500)
    compare_with_oracle(X, 0.05, "fp32", max_level=1)
    compare_with_oracle(X, 0.05, "fp32", lds_budget=0)
    compare_with_oracle(X, 0.05, "fp32", ranks_per_lane=1, grid=3)


def factor_data(n, m, seed):
    """One latent factor F = X_0 shared by every other variable (X_i = F + noise): level 0 keeps the
    complete graph, so every row has n - 1 neighbours, and level 1 separates the pairs (i, j) by
    {0}. With n - 1 > 1024 no row's neighbour list fits in LDS: the level kernel takes its
    global-memory placement for every item."""
    rng = np.random.default_rng(seed)
    F = rng.standard_normal(m)
    X = F[:, None] + rng.standard_normal((m, n))
    X[:, 0] = F
    return np.ascontiguousarray(X)


@pytest.mark.parametrize("prec,opt", [("fp32", {}), ("fp64", {}), ("fp32", {"tests_per_lane": 1})])
def test_skeleton_rows_beyond_lds_capacity(prec, opt):
    X = factor_data(1100, 300, 41)
    print(f"rows beyond LDS capacity prec={prec} {opt}", flush=True)
    st, ref = compare_with_oracle(X, 0.001, prec, max_level=1, **opt)
    assert ref.G_after[0].sum(1).min() == 1099
    assert st["tests"][1] >= 604450 - 1100


@pytest.mark.parametrize("prec,tail_tests", [("fp32", 2048), ("fp32", 1), ("fp32", 1 << 24), ("bf16x3", 1 << 24),
                                             ("fp64", 1 << 24)])
def test_skeleton_tail_kernel_modes(prec, tail_tests):
    """The small levels in one work-group per problem: from the first small level the stream run
    looks at (2048), handed back at once (1), or every level up to 8 from level 2 on (a budget
    above any level's test count here)."""
    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    print(f"tail modes prec={prec} tail_tests={tail_tests}", flush=True)
    st, ref = compare_with_oracle(X, alpha, prec, tail_tests=tail_tests)
    assert st["tests"][0] == 1000 * 999 // 2


def test_skeleton_tail_with_rechecks_and_max_level():
    """The tail's FP64 re-checks (audit-free band tests of BF16x3) and a level cap inside it."""
    X = sem_data(19, 300, 0.04, 400)
    for ml in (-1, 3):
        print(f"tail recheck max_level={ml}", flush=True)
        st, ref = compare_with_oracle(X, 0.05, "bf16x3", max_level=ml, tail_tests=1 << 24)


def test_skeleton_sample_limit_warning():
    X = sem_data(5, 12, 0.9, 7)
    compare_with_oracle(X, 0.5, "fp64")


def test_skeleton_deterministic_graph():
    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    G0 = run_skeleton(X, alpha, "fp32")[0]
    for _ in range(4):
        assert np.array_equal(run_skeleton(X, alpha, "fp32")[0], G0)


def test_sepset_capacity_error():
    X = sem_data(9, 60, 0.3, 400)
    m, n = X.shape
    ctx = pc.Context(precision="fp32")
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(1)
    Xt = torch.from_numpy(X).cuda()
    ref = oracle.skeleton(X, 0.05)
    if len(ref.sepsets.i) > 1:
        with pytest.raises(pc.PCError) as e:
            ctx.pc_skeleton(Xt, 0.05, adj, recs, count, ws)
        assert e.value.status == -8
        assert np.array_equal(pc.bits_to_dense(adj.cpu().numpy(), n), ref.G)


def hub_data(parents, m, seed, extra=8):
    """A collider hub with `parents` independent parents (plus unrelated variables): every
    hub-parent edge is a true edge, so the hub keeps its degree and the levels run up to
    parents - 1, through the wavefront-per-set kernel of the deep levels."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, parents + 1 + extra))
    w = rng.choice([-1.0, 1.0], parents) * rng.uniform(0.3, 1.0, parents)
    X[:, parents] = X[:, :parents] @ w + rng.standard_normal(m)
    return np.ascontiguousarray(X)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_skeleton_deep_levels_hub(prec):
    X = hub_data(17, 5000, 31)
    print(f"deep levels prec={prec} n={X.shape[1]} m={X.shape[0]}", flush=True)
    st, ref = compare_with_oracle(X, 0.01, prec)
    assert ref.levels_run >= 17 and st["levels_run"] == ref.levels_run
    assert sum(st["tests"][14:ref.levels_run]) > 0



# ---------------------------------------------------------------------------------------------
# Re-check queue overflow: the run is completed in FP64 from the overflowing level
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_recheck_overflow_completes_level_in_fp64(prec):
    """With every FP32 test sent to the re-check queue (audit mode) and a queue of 2048 entries, level
    1 overflows it: the device stops the level loop, the level is redone in FP64 on its snapshot G'
    and the rest of the skeleton runs in FP64. The result is the oracle's, with status OK."""
    X = sem_data(31, 300, 0.03, 600)
    print(f"overflow {prec}", flush=True)
    st, ref = compare_with_oracle(X, 0.05, prec, force_recheck_all=1, recheck_cap=2048)
    assert st["fp64_from"] == 1


def test_recheck_overflow_at_a_later_level():
    """A queue that holds all of level 1's tests but not level 2's (a collider hub with 20 parents:
    about 20 * 19 tests at level 1, 20 * C(19, 2) at level 2): the run goes on in FP64 from level 2,
    and the re-check launches of levels 3.. (enqueued behind it) leave the stale queue alone."""
    X = hub_data(20, 3000, 41)
    print("overflow at level 2: sizing run", flush=True)
    st, ref = compare_with_oracle(X, 0.01, "fp32", max_level=4, force_recheck_all=1, recheck_cap=1 << 22)
    t1, t2 = st["tests"][1], st["tests"][2]
    assert st["fp64_from"] == 0
    # Every level-1 test is queued in audit mode; pushes <= capacity never overflow (a wavefront
    # tries every slice, and slices only fill up).
    cap = (t1 + 15) // 16 * 16 + 256
    assert cap < t2, (t1, t2)
    print(f"overflow at level 2: cap {cap}", flush=True)
    for graph in (False, True):
        if not graph:
            st, ref = compare_with_oracle(X, 0.01, "fp32", max_level=4, force_recheck_all=1, recheck_cap=cap)
            assert st["fp64_from"] == 2
            continue
        m, n = X.shape
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            gctx = pc.Context(stream=stream, precision="fp32", force_recheck_all=1, recheck_cap=cap)
            gadj = gctx.adjacency(n)
            grecs, gcount = gctx.sepsets(n * n)
            probs = gctx.problems([(torch.from_numpy(X).cuda(), 0.01, 4, gadj, grecs, gcount)])
            gws = gctx.batch_workspace(probs)
            g = gctx.pc_batch_capture(probs, gws)
            gst = (pc.pc_run_stats * 1)()
            g.pc_graph_launch()
            r, status = g.pc_graph_results(gst)
            torch.cuda.synchronize()
            g.close()
        assert r == 0 and status[0] == 0 and gst[0].fp64_from == 2
        assert np.array_equal(pc.bits_to_dense(gadj.cpu().numpy(), n), ref.G)


def test_recheck_overflow_through_pc_level_and_graph():
    """The same completion through pc_level (one level from the oracle's snapshot) and through a
    captured graph (pc_graph_results finishes the overflowed level and the levels after it)."""
    X = sem_data(32, 200, 0.05, 500)
    m, n = X.shape
    alpha = 0.05
    C64 = oracle.corr(X)
    ref = oracle.skeleton_corr(C64, m, alpha, keep_levels=True)
    print("overflow through pc_level", flush=True)
    ctx, ws, Xt, C, G0 = gpu_corr(X, alpha, "fp32", force_recheck_all=1, recheck_cap=1024)
    recs, count = ctx.sepsets(n * n)
    adj = torch.from_numpy(pc.dense_to_bits(ref.G_after[0])).cuda()
    st = pc.pc_run_stats()
    assert ctx.pc_level(1, n, m, alpha, adj, recs, count, ws, stats=st) == 0
    assert st.fp64_from == 1
    assert np.array_equal(pc.bits_to_dense(adj.cpu().numpy(), n), ref.G_after[1])
    print("overflow through a captured graph", flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = pc.Context(stream=stream, precision="fp32", force_recheck_all=1, recheck_cap=1024)
        gadj = gctx.adjacency(n)
        grecs, gcount = gctx.sepsets(n * n)
        probs = gctx.problems([(torch.from_numpy(np.ascontiguousarray(X)).cuda(), alpha, -1, gadj, grecs, gcount)])
        gws = gctx.batch_workspace(probs)
        graph = gctx.pc_batch_capture(probs, gws)
        gst = (pc.pc_run_stats * 1)()
        for replay in range(2):
            graph.pc_graph_launch()
            r, status = graph.pc_graph_results(gst)
            torch.cuda.synchronize()
            assert r == 0 and status[0] == 0 and gst[0].fp64_from == 1
            assert np.array_equal(pc.bits_to_dense(gadj.cpu().numpy(), n), ref.G), replay
        graph.close()
