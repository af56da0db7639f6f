"""GPU checks of the learned conditioning-set ordering (marked gpu):
MLP forward / backward / BCE / Adam kernels against the FP64 reference (oracle/mlp.py), the
feature kernel against values recomputed from the oracle's correlation, and the ordered skeleton
against the oracle for arbitrary model weights (the skeleton must not depend on the order)."""
import itertools
import math

import numpy as np
import pytest

import oracle
import semgen
from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_08491_amd as pc  # noqa: E402


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def test_mlp_forward_backward_bce_adam_match_fp64_reference():
    rng = np.random.default_rng(3)
    ctx = pc.Context(precision="fp32")
    theta = mlp.init(rng) * 0.5
    for rows in (1, 63, 64, 130, 1000):
        X = rng.random((rows, mlp.IN)).astype(np.float32)
        y = (rng.random(rows) < 0.2).astype(np.float32)
        th32 = theta.astype(np.float32)
        p = dev(th32)
        Xd = dev(X)
        scores = torch.empty(rows, device="cuda")
        act = torch.empty((rows, 128), device="cuda")
        ctx.pc_mlp_forward(p, Xd, scores, act)
        s_ref, cache = mlp.forward(th32.astype(np.float64), X.astype(np.float64))
        s = scores.cpu().numpy()
        assert np.allclose(s, s_ref, rtol=1e-4, atol=1e-4 * np.abs(s_ref).max())
        dscore = torch.empty(rows, device="cuda")
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.pc_mlp_bce(scores, dev(y), 3.0, dscore, loss)
        l_ref, ds_ref = mlp.bce(s_ref, y, 3.0)
        assert abs(loss.item() - l_ref) <= 1e-4 * max(1.0, l_ref)
        assert np.allclose(dscore.cpu().numpy(), ds_ref, rtol=1e-3, atol=1e-6 / rows)
        grads = torch.empty(pc.PC_MLP_PARAMS, device="cuda")
        partial = torch.empty(((rows + 63) // 64, pc.PC_MLP_PARAMS), device="cuda")
        ctx.pc_mlp_backward(p, Xd, act, dscore, grads, partial)
        g_ref = mlp.backward(th32.astype(np.float64), cache, ds_ref)
        g = grads.cpu().numpy()
        assert np.abs(g - g_ref).max() <= 1e-4 * max(1e-12, np.abs(g_ref).max()), rows
        m1 = torch.zeros_like(grads)
        m2 = torch.zeros_like(grads)
        ctx.pc_mlp_adam(p, grads, m1, m2, 1, lr=1e-3)
        t_ref, _, _ = mlp.adam(th32.astype(np.float64), g.astype(np.float64), np.zeros(mlp.NPARAMS),
                               np.zeros(mlp.NPARAMS), 1, lr=1e-3)
        assert np.allclose(p.cpu().numpy(), t_ref, atol=2e-6)


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    ctx = pc.Context(precision="fp32")
    rows = 4096
    X = rng.random((rows, mlp.IN)).astype(np.float32)
    y = ((X[:, 3] < 0.2) & (X[:, 1] > 0.3)).astype(np.float32)
    p = dev(mlp.init(rng))
    Xd, yd = dev(X), dev(y)
    scores = torch.empty(rows, device="cuda")
    act = torch.empty((rows, 128), device="cuda")
    ds = torch.empty(rows, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grads = torch.empty(pc.PC_MLP_PARAMS, device="cuda")
    partial = torch.empty((rows // 64, pc.PC_MLP_PARAMS), device="cuda")
    m1, m2 = torch.zeros_like(grads), torch.zeros_like(grads)
    losses = []
    for step in range(1, 301):
        ctx.pc_mlp_forward(p, Xd, scores, act)
        ctx.pc_mlp_bce(scores, yd, 1.0, ds, loss)
        ctx.pc_mlp_backward(p, Xd, act, ds, grads, partial)
        ctx.pc_mlp_adam(p, grads, m1, m2, step, lr=3e-3)
        if step % 50 == 1:
            losses.append(loss.item())
    assert losses[-1] < 0.5 * losses[0], losses


def test_features_match_recomputation():
    X, sem, alpha = semgen.workload("n50_p005_m1000_fp64")
    m, n = X.shape
    C = oracle.corr(X)
    ref = oracle.skeleton_corr(C, m, alpha, keep_levels=True)
    Gp = ref.G_after[1]
    ctx = pc.Context(precision="fp32")
    ws = ctx.workspace(n, m)
    ctx.pc_corr(dev(X, torch.float64), alpha, ws)
    adj = dev(pc.dense_to_bits(Gp), torch.int64)
    deg = Gp.sum(1)
    need = int((deg * (deg - 1)).sum())
    feats = torch.empty((max(need, 1), 8), device="cuda")
    meta = torch.empty((max(need, 1), 3), dtype=torch.int32, device="cuda")
    rows = ctx.pc_features(2, n, m, alpha, adj, feats, meta, ws)
    assert rows == need
    F, M = feats[:rows].cpu().numpy(), meta[:rows].cpu().numpy()
    expect_order = [(i, j, k) for i in range(n) for j in np.flatnonzero(Gp[i])
                    for k in np.flatnonzero(Gp[i]) if k != j]
    assert [tuple(r) for r in M] == expect_order
    for (i, j, k), f in zip(M, F):
        rho = (C[i, j] - C[i, k] * C[j, k]) / math.sqrt((1 - C[i, k] ** 2) * (1 - C[j, k] ** 2))
        want = [abs(C[i, j]), abs(C[i, k]), abs(C[j, k]), abs(rho), deg[i] / 64, deg[j] / 64, deg[k] / 64, 2 / 8]
        assert np.allclose(f, want, atol=2e-4), (i, j, k, f, want)


def ordered_run(X, alpha, params, prec="fp32", **order_kw):
    m, n = X.shape
    ctx = pc.Context(precision=prec)
    order = ctx.order(params, **order_kw)
    ws = ctx.ordered_workspace(n, m, order)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    st = pc.pc_run_stats()
    status = ctx.pc_skeleton_ordered(dev(X, torch.float64), alpha, adj, recs, count, ws, order, stats=st)
    k = int(count.item())
    return (pc.bits_to_dense(adj.cpu().numpy(), n), pc.decode_sepsets(recs[:k].cpu().numpy(), k),
            st.as_dict(), status)


@pytest.mark.parametrize("seed,prec,min_level,top", [(0, "fp32", 1, 4), (1, "fp32", 2, 2), (2, "bf16x3", 2, 8),
                                                     (3, "fp64", 1, 3), (4, "fp32", 3, 5)])
def test_ordered_skeleton_equals_oracle_for_any_weights(seed, prec, min_level, top):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(30, 160))
    sem = semgen.random_dag(n, float(rng.uniform(0.05, 0.25)), rng)
    X = semgen.sample(sem, int(rng.integers(200, 1200)), rng)
    alpha = 0.05
    params = dev(mlp.init(rng) * rng.uniform(0.1, 3.0))
    G, seps, st, status = ordered_run(X, alpha, params, prec, min_level=min_level, top=top)
    C = oracle.corr(X)
    ref = oracle.skeleton_corr(C, X.shape[0], alpha, keep_levels=True)
    assert np.array_equal(G, ref.G)
    ref_seps = ref.sepsets.as_dict()
    assert set(seps) == set(ref_seps)
    for e, (l, S) in seps.items():
        assert ref_seps[e][0] == l
        Gp = ref.G_after[l - 1]
        assert all(Gp[e[0], s] for s in S) or all(Gp[e[1], s] for s in S)
        assert oracle.ci_test(C, e[0], e[1], list(S), X.shape[0], alpha)[0]
    assert sum(st["probe_tests"]) > 0 or st["levels_run"] <= min_level


def test_ordered_skeleton_n1000():
    X, sem, alpha = semgen.workload("n1000_d4_m500_fp32")
    rng = np.random.default_rng(9)
    params = dev(mlp.init(rng))
    G, seps, st, status = ordered_run(X, alpha, params, "fp32", min_level=1, top=4)
    ref = oracle.skeleton(X, alpha)
    assert np.array_equal(G, ref.G)
    assert set(seps) == set(ref.sepsets.as_dict())
    assert st["probe_removed"][1] > 0


def test_training_pipeline_beats_random_order_and_keeps_skeleton():
    """Rows from the plain method on generated SEMs, training on the library's kernels, then the
    trained scorer against a random order on held-out directions, and the learned-order skeleton
    against the plain one."""
    from paper_1812_08491_amd import learn
    data = [(X, a) for X, _, a in semgen.training_sems(40, instance=7, n=100, m=600)]
    X, y = learn.collect(data[:32], 100, 600, cap_per_level=4096, seed=1)
    assert X.shape[0] > 10000 and 0.02 < float(y.mean()) < 0.6
    pos = float(y.sum())
    pw = min(50.0, (y.numel() - pos) / pos)
    coll = learn.RowCollector(100, 600)
    vrows = [r for Xv, a in data[32:] for r in coll.run(Xv, a, None, whole_directions=True)]
    coll.close()
    vX = torch.cat([r[1] for r in vrows])
    vy = torch.cat([r[2] for r in vrows])
    vdir = torch.cat([r[3] + (k << 32) for k, r in enumerate(vrows)])
    tr = learn.Trainer(seed=2, batch=16384)
    v0 = learn.bce_loss(tr, vX, vy, pw)
    for _ in range(8):
        tr.epoch(X, y, pw)
    v1 = learn.bce_loss(tr, vX, vy, pw)
    rec = learn.topq_recall(tr.scores_of(vX), vy, vdir, 4)
    rnd = learn.topq_recall(torch.rand(vX.shape[0], device="cuda"), vy, vdir, 4)
    print(f"val loss {v0:.4f} -> {v1:.4f}; recall@4 trained {rec:.3f} random {rnd:.3f}")
    assert v1 < 0.9 * v0
    assert rec > rnd + 0.1
    X2, _, a2 = next(semgen.training_sems(1, instance=8, n=200, m=1000))
    cmp = learn.compare_orders(X2, a2, tr.params, min_level=1, top=4, repeats=1)
    print({k: cmp[k] for k in ("plain", "learned")})
    assert cmp["same_skeleton"]
    assert sum(cmp["learned"]["probe_removed"]) > 0
    tr.close()


def test_row_features_match_recomputation():
    """Shared-set (row) features and labels of level 1 against values recomputed on the host from
    the same FP32 C and G': the label of k* (largest |C_ik|) is the fraction of the row's other
    edges {k*} separates; that of any other k, the fraction {k} separates and {k*} does not."""
    rng = np.random.default_rng(21)
    n, m, alpha = 90, 400, 0.05
    X = semgen.sample(semgen.random_dag(n, 0.08, rng), m, rng)
    ctx = pc.Context(precision="fp32")
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ctx.pc_corr(dev(X, torch.float64), alpha, ws, C_out=C, adj_out=adj)
    G = pc.bits_to_dense(adj.cpu().numpy(), n).astype(bool)
    Cn = C.cpu().numpy().astype(np.float64)
    deg = G.sum(1)
    need = int(deg.sum())
    feats = torch.empty((need, 8), device="cuda")
    labels = torch.empty(need, device="cuda")
    meta = torch.empty((need, 2), dtype=torch.int32, device="cuda")
    rows = ctx.pc_row_features(1, n, m, alpha, adj, feats, labels, meta, ws)
    assert rows == need
    F, Y, M = feats.cpu().numpy(), labels.cpu().numpy(), meta.cpu().numpy()
    assert [tuple(r) for r in M] == [(i, k) for i in range(n) for k in np.flatnonzero(G[i])]
    th = math.tanh(pc.pc_threshold(alpha, m, 1))

    def sep_bounds(i, k, js):
        # {k} separates (i, j): sure (outside FP32 ties) and possible (ties either way)
        lhs = np.abs(Cn[i, js] - Cn[i, k] * Cn[js, k])
        rhs = th * np.sqrt(np.clip((1 - Cn[i, k] ** 2) * (1 - Cn[js, k] ** 2), 0, None))
        ties = np.abs(lhs - rhs) < 1e-5
        return (lhs <= rhs) & ~ties, (lhs <= rhs) | ties

    checked = 0
    for r, (i, k) in enumerate(M):
        Ni = np.flatnonzero(G[i])
        d = Ni.size
        a = np.abs(Cn[i, Ni])
        p = int(np.flatnonzero(Ni == k)[0])
        ps = int(np.argmax(a))                 # k*: largest |C_ik|, first position on ties
        ks = int(Ni[ps])
        cn = int(np.sum(G[i] & G[k]))
        ckk = 1.0 if p == ps else Cn[ks, k]
        den = (1 - Cn[i, ks] ** 2) * (1 - ckk ** 2)
        rho = 0.0 if p == ps or den <= 0 else min(1.0, abs(Cn[i, k] - Cn[i, ks] * ckk) / math.sqrt(den))
        lift = cn * n / (d * deg[k])
        want = [a[p], a[p] / a.max(), min(lift, 8.0) / 8.0, deg[k] / (d + deg[k]), abs(ckk), rho,
                a.mean() / a.max(), cn / d]
        assert np.allclose(F[r], want, atol=2e-5), (i, k, F[r], want)
        js = Ni[Ni != k]
        sure, maybe = sep_bounds(i, k, js)
        if p != ps:
            # what {k} separates beyond {k*}
            sure_s, maybe_s = sep_bounds(i, ks, js)
            sure_s &= js != ks                 # {k*} is not tested against its own edge
            maybe_s &= js != ks
            sure, maybe = sure & ~maybe_s, maybe & ~sure_s
        lo_, hi_ = int(np.sum(sure)), int(np.sum(maybe))
        assert lo_ / max(d - 1, 1) - 1e-6 <= Y[r] <= hi_ / max(d - 1, 1) + 1e-6, (i, k, Y[r], lo_, hi_)
        checked += 1
    assert checked == rows and Y.sum() > 0


@pytest.mark.parametrize("seed,prec,row_top,with_edge", [(0, "fp32", 4, False), (1, "fp64", 1, False),
                                                         (2, "bf16x3", 16, False), (3, "fp32", 3, True)])
def test_row_order_skeleton_equals_oracle_for_any_weights(seed, prec, row_top, with_edge):
    """The shared-set order (any weights) reorders level 1's sets only: the skeleton is the oracle's,
    every SepSet separates, and the probe part of level 1 ran."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(60, 200))
    X = semgen.sample(semgen.random_dag(n, float(rng.uniform(0.05, 0.2)), rng), int(rng.integers(300, 1500)), rng)
    alpha = 0.05
    row_params = dev(mlp.init(rng) * rng.uniform(0.1, 3.0))
    params = dev(mlp.init(rng)) if with_edge else None
    G, seps, st, status = ordered_run(X, alpha, params, prec, min_level=2, top=4, row_params=row_params,
                                      row_top=row_top)
    C = oracle.corr(X)
    ref = oracle.skeleton_corr(C, X.shape[0], alpha, keep_levels=True)
    assert np.array_equal(G, ref.G)
    ref_seps = ref.sepsets.as_dict()
    assert set(seps) == set(ref_seps)
    for e, (l, S) in seps.items():
        assert ref_seps[e][0] == l
        assert oracle.ci_test(C, e[0], e[1], list(S), X.shape[0], alpha)[0]
    if st["levels_run"] > 1:
        assert st["probe_tests"][1] > 0
        assert st["tests"][1] >= st["probe_tests"][1]


def test_row_order_rows_beyond_scorer_capacity():
    """Rows of more than 512 neighbours are not scored: they keep their order, the ordering pass
    tests their first sets and the level kernel the rest, so the skeleton is still the oracle's."""
    rng = np.random.default_rng(41)
    F = rng.standard_normal(300)
    X = F[:, None] + rng.standard_normal((300, 1100))
    X[:, 0] = F
    X = np.ascontiguousarray(X)
    row_params = dev(mlp.init(np.random.default_rng(6)))
    m, n = X.shape
    ctx = pc.Context(precision="fp32")
    order = ctx.order(None, row_params=row_params, row_top=2)
    ws = ctx.ordered_workspace(n, m, order)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    st = pc.pc_run_stats()
    status = ctx.pc_skeleton_ordered(dev(X, torch.float64), 0.001, adj, recs, count, ws, order, max_level=1,
                                     stats=st)
    assert status == 0
    k = int(count.item())
    G, seps, st = pc.bits_to_dense(adj.cpu().numpy(), n), pc.decode_sepsets(recs[:k].cpu().numpy(), k), st.as_dict()
    C = oracle.corr(X)
    ref = oracle.skeleton_corr(C, m, 0.001, max_level=1)
    assert np.array_equal(G, ref.G)
    ref_seps = ref.sepsets.as_dict()
    assert set(seps) == set(ref_seps)
    assert all(ref_seps[e][0] == l for e, (l, S) in seps.items())
    # about 600 k records: the oracle's FP64 test on a sample of them
    keys = list(seps)
    for t in np.random.default_rng(7).choice(len(keys), 3000, replace=False):
        e = keys[t]
        assert oracle.ci_test(C, e[0], e[1], list(seps[e][1]), m, 0.001)[0]
    assert st["probe_tests"][1] > 0


def test_row_order_n2000_matches_oracle_with_trained_weights():
    """The n = 2000 workload with the trained row model (or fresh weights if none is stored)."""
    import os
    from paper_1812_08491_amd import learn
    X, sem, alpha = semgen.workload("n2000_d10_m1000_apply")
    row = learn.load_weights(learn.ROW_WEIGHTS) if os.path.exists(learn.ROW_WEIGHTS) else dev(
        mlp.init(np.random.default_rng(5)))
    G, seps, st, status = ordered_run(X, alpha, None, "fp32", row_params=row, row_top=4)
    ref = oracle.skeleton(X, alpha)
    assert np.array_equal(G, ref.G)
    assert set(seps) == set(ref.sepsets.as_dict())
    print("level-1 tests", st["tests"][1], "probe", st["probe_tests"][1], "probe removed", st["probe_removed"][1])


# ---------------------------------------------------------------------------------------------
# The BF16 scorer of the shared-set order against the FP64 reference network
# ---------------------------------------------------------------------------------------------
U_BF16 = 2.0 ** -9     # unit roundoff of BF16 (8 stored mantissa bits, round to nearest even)


def _abs_network(theta, F):
    """The network with |weights| and |inputs| (FP64): s_bar bounds every path sum of the score."""
    p = mlp.unpack(np.asarray(theta, np.float64))
    a1 = np.abs(F) @ np.abs(p["W1"]).T + np.abs(p["b1"])
    a2 = a1 @ np.abs(p["W2"]).T + np.abs(p["b2"])
    return a2 @ np.abs(p["W3"]) + abs(p["b3"][0])


def _row_scores(ctx, n, m, alpha, adj, ws, order):
    scores = torch.full((n, n), float("nan"), device="cuda")
    top = torch.full((n, order.row_top), -2, dtype=torch.int32, device="cuda")
    ctx.pc_row_scores(n, m, alpha, adj, order, scores, top, ws)
    return scores.cpu().numpy(), top.cpu().numpy()


def _expected_picks(vals, T):
    """Best first by value, ties to the lower position (the kernel's argmax rounds)."""
    idx = sorted(range(len(vals)), key=lambda q: (-vals[q], q))
    return idx[:T]


@pytest.mark.parametrize("seed,row_short", [(0, 0), (1, 0), (2, 8)])
def test_row_scorer_matches_fp64_network(seed, row_short):
    """k_row_order's BF16 MFMA scores equal the FP64 reference forward (oracle/mlp.py) of the same
    features within the BF16 error bound, and its picks are k* (largest |C_ik|) and then the top of
    its own scores.

    Bound: inputs, W1, W2 and the first hidden layer are rounded to BF16 (relative u = 2^-9 each),
    so |dz1| <= 2u a1 (+ u a1 for rounding h1), |dz2| <= 4u a2 and |ds| <= 4u s_bar to first order,
    where a1, a2, s_bar are the layer sums of the network with |weights| and |inputs|. FP32
    accumulation (at most 64 terms, 2^-24 each) and second-order terms fit in the margin of 6u."""
    rng = np.random.default_rng(500 + seed)
    n, m, alpha = 150, 600, 0.05
    X = semgen.sample(semgen.random_dag(n, 0.12, rng), m, rng)
    ctx = pc.Context(precision="fp32")
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    ctx.pc_corr(dev(X, torch.float64), alpha, ws, adj_out=adj)
    G = pc.bits_to_dense(adj.cpu().numpy(), n).astype(bool)
    need = int(G.sum())
    feats = torch.empty((need, 8), device="cuda")
    labels = torch.empty(need, device="cuda")
    meta = torch.empty((need, 2), dtype=torch.int32, device="cuda")
    assert ctx.pc_row_features(1, n, m, alpha, adj, feats, labels, meta, ws) == need
    F, M = feats.cpu().numpy().astype(np.float64), meta.cpu().numpy()
    theta = mlp.init(rng) * rng.uniform(0.5, 2.0)
    th32 = theta.astype(np.float32)
    T = 3
    params = dev(th32)
    order = ctx.order(None, row_params=params, row_top=T, row_short=row_short)
    S, top = _row_scores(ctx, n, m, alpha, adj, ws, order)
    s_ref, _ = mlp.forward(th32.astype(np.float64), F)
    bound = 6 * U_BF16 * _abs_network(th32, F)
    deg = G.sum(1)
    checked = 0
    for i in range(n):
        rows = np.flatnonzero(M[:, 0] == i)
        if deg[i] < 2:
            continue
        ks = M[rows, 1]
        assert list(ks) == list(np.flatnonzero(G[i]))
        got = S[i, ks].astype(np.float64)
        # k* (largest |C_ik|, first position on ties) always comes first: its score is +inf
        ps = _expected_picks(list(F[rows, 0]), 1)[0]
        assert got[ps] == np.inf
        got[ps] = s_ref[rows][ps]
        if row_short and deg[i] > row_short:
            short = set(_expected_picks(list(F[rows, 0]), row_short))   # |C_ik|, ties: lower position
            inside = np.array([q in short for q in range(len(ks))])
            assert np.all(np.isneginf(got[~inside]))
        else:
            inside = np.ones(len(ks), bool)
        err = np.abs(got[inside] - s_ref[rows][inside])
        assert np.all(err <= bound[rows][inside]), (i, err.max(), bound[rows][inside].max())
        checked += int(inside.sum())
        # picks: k*, then the top of the kernel's own scores, best first, ties to the lower position
        own = got.copy()
        own[ps] = np.inf
        want = [int(ks[q]) for q in _expected_picks(list(own), min(T, len(ks)))]
        assert list(top[i, :len(want)]) == want, (i, top[i], want)
        assert np.all(top[i, len(want):] == -1)
        # and, within the bound, the top of the reference scores among the others
        others = inside.copy()
        others[ps] = False
        if others.sum() >= 1 and T > 1:
            ref_sorted = np.sort(s_ref[rows][others])[::-1]
            kth = ref_sorted[min(T - 1, others.sum()) - 1]
            for k in want[1:]:
                q = int(np.flatnonzero(ks == k)[0])
                assert s_ref[rows][q] >= kth - 2 * bound[rows].max(), (i, k)
    assert checked > 1000


def test_row_scorer_abs_mode_ranks_by_abs_corr():
    """row_rank 'abs': the score of candidate k of node i is |C_ik| itself and the picks are the
    largest |C_ik| (ties to the lower position)."""
    rng = np.random.default_rng(77)
    n, m, alpha = 120, 500, 0.05
    X = semgen.sample(semgen.random_dag(n, 0.1, rng), m, rng)
    ctx = pc.Context(precision="fp32")
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ctx.pc_corr(dev(X, torch.float64), alpha, ws, C_out=C, adj_out=adj)
    G = pc.bits_to_dense(adj.cpu().numpy(), n).astype(bool)
    Cn = C.cpu().numpy()
    order = ctx.order(None, row_top=4, row_rank="abs")
    S, top = _row_scores(ctx, n, m, alpha, adj, ws, order)
    for i in range(n):
        ks = np.flatnonzero(G[i])
        if ks.size < 2:
            continue
        assert np.array_equal(S[i, ks], np.abs(Cn[i, ks]))
        want = [int(ks[q]) for q in _expected_picks(list(np.abs(Cn[i, ks])), min(4, ks.size))]
        assert list(top[i, :len(want)]) == want


@pytest.mark.parametrize("seed,prec,rank,sort,split", [(0, "fp32", "abs", True, 0), (1, "fp32", "abs", True, 16),
                                                       (2, "fp64", "model", True, 8), (3, "bf16x3", "abs", False, 12),
                                                       (4, "fp32", "model", True, 32)])
def test_sorted_and_split_level1_equals_oracle(seed, prec, rank, sort, split):
    """Level 1 with the remaining sets enumerated by descending |C_ik| (a permutation stored after
    each ascending neighbour list; rows with 2 d > n fall back to moving the chosen to the front)
    and/or split into two level-kernel passes: the skeleton is the oracle's, every removal level
    matches and every SepSet separates. Dense and sparse rows are both present (n ~ 60-200)."""
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(60, 200))
    # a dense block (its rows have 2 d > n after level 0) inside a sparse graph
    sem = semgen.random_dag(n, float(rng.uniform(0.05, 0.12)), rng)
    X = semgen.sample(sem, int(rng.integers(300, 1200)), rng)
    k = n // 4
    Z = rng.standard_normal((X.shape[0], 1))
    X[:, :k] += 2.0 * Z
    alpha = 0.05
    row_params = dev(mlp.init(rng))
    kw = dict(row_top=2, row_sort=sort, row_split=split)
    if rank == "abs":
        kw["row_rank"] = "abs"
    else:
        kw.update(row_params=row_params, row_short=8)
    G, seps, st, status = ordered_run(X, alpha, None, prec, **kw)
    C = oracle.corr(X)
    ref = oracle.skeleton_corr(C, X.shape[0], alpha, keep_levels=True)
    assert status == 0
    assert np.array_equal(G, ref.G), np.argwhere(G != ref.G)[:8]
    ref_seps = ref.sepsets.as_dict()
    assert set(seps) == set(ref_seps)
    for e, (l, S) in seps.items():
        assert ref_seps[e][0] == l
        assert oracle.ci_test(C, e[0], e[1], list(S), X.shape[0], alpha)[0], (e, S)
    Gp = ref.G_after[0]
    assert (2 * Gp.sum(1) > n).any() and (2 * Gp.sum(1) <= n).any()


def test_row_labels_from_plain_sepsets():
    """Labels from the SepSets of the plain method (the default training labels of the row model):
    for node i and candidate k, the fraction of the level-1 removals at i whose recorded SepSet is
    {k}. Checked against the records decoded on the host, and every positive label rests on a test
    that the oracle's FP64 test confirms (the record's edge is separated by {k})."""
    from paper_1812_08491_amd import learn

    rng = np.random.default_rng(71)
    sem = semgen.random_dag(100, 6.0 / 99, rng)
    X = semgen.sample(sem, 600, rng)
    alpha = 0.01
    coll = learn.NodeRowCollector(100, 600)
    f, y, mi, mk, C = coll.run(X, alpha)
    rec = coll.plain_level1_records(X, alpha)
    lab = coll.sepset_labels(X, alpha, mi, mk, records=rec).cpu().numpy()
    mi_h, mk_h = mi.cpu().numpy(), mk.cpu().numpy()
    # host recount from the same records
    hits = np.zeros((100, 100))
    by_k = {}
    for i, j, k in rec.cpu().numpy().tolist():
        hits[i, k] += 1
        hits[j, k] += 1
        by_k.setdefault((i, k), []).append(j)
        by_k.setdefault((j, k), []).append(i)
    per = np.maximum(hits.sum(1), 1.0)
    assert np.allclose(lab, hits[mi_h, mk_h] / per[mi_h])
    C64 = oracle.corr(X)
    pos = np.nonzero(lab > 0)[0]
    assert pos.size > 0
    for r in pos[:300]:
        i, k = int(mi_h[r]), int(mk_h[r])
        for j in by_k[(i, k)]:
            assert oracle.ci_test(C64, i, j, [k], 600, alpha)[0], (i, j, k)
    coll.close()
