"""Parity at full workload sizes, where the oracle cannot run the whole skeleton in a test:
sampled outputs it computes one by one, and properties that hold at any size (marked gpu).

  * n=8000 variables, m=2000 samples, expected degree 6, alpha=0.05, BF16x3 correlation, levels
    1-3: sampled entries of C against FP64 (error within the stated bound), level-0 decisions of
    sampled pairs, level-1 decisions of sampled edges recomputed entirely by the oracle (its own
    level-0 neighbour lists, then every size-1 set in both directions), and every sampled SepSet
    record of levels 1-3 passing the oracle's FP64 test.
    The same workload is also checked whole: G after levels 1, 2 and 3 (BF16x3 and FP32) against
    the oracle's stored result (tests/golden/n8000_d6_m2000_levels3.npz, written by
    tests/golden/make_oracle_skeletons.py from the oracle alone; about 100 s of CPU).
  * n=2000 variables, m=1000 samples, expected degree 10: whole skeleton against the oracle, plain
    and with the learned order.
  * Points of the paper's scalability grid (n up to 2000, m 2000-10000, d 0.1-0.5; FP64, and FP32
    completed in FP64 after a re-check queue overflow): every pair on which the GPU and the oracle
    differ is tied to a near-collinear test.
"""
import hashlib
import os
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


@pytest.fixture(scope="module")
def big():
    X, sem, alpha = semgen.workload("n8000_d6_m2000_bf16x3")
    X = np.ascontiguousarray(X)
    return X, np.ascontiguousarray(X.T), alpha


def _bf16x3_bound(m):
    """The stated |C_gpu - C_64| bound of the BF16x3 product: the dropped split terms plus blocked
    FP32 accumulation with compensated block sums (independent of m)."""
    return (3 + 2.0 ** -7) * 2.0 ** -16 + 195 * 2.0 ** -24


def _pair(XT, a, b):
    """Oracle correlation of variables a, b (XT: the data transposed, so the copy is contiguous)."""
    return oracle.corr_pair(np.ascontiguousarray(np.stack((XT[a], XT[b]), 1)), 0, 1)


def _corr_row(XT, a):
    return np.array([1.0 if b == a else _pair(XT, a, b) for b in range(XT.shape[0])])


def test_n8000_bf16x3_corr_error_and_level0_sampled(big):
    X, XT, alpha = big
    m, n = X.shape
    ctx = pc.Context(precision="bf16x3")
    ws = ctx.workspace(n, m)
    Xd = torch.from_numpy(X).cuda()
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    adj = ctx.adjacency(n)
    ctx.pc_corr(Xd, alpha, ws, C_out=C, adj_out=adj)
    ctx.pc_sync_status(ws)
    rng = np.random.default_rng(11)
    a = rng.integers(0, n, 4000)
    b = rng.integers(0, n, 4000)
    keep = a != b
    a, b = a[keep], b[keep]
    Cs = C[torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()].cpu().numpy().astype(np.float64)
    C64 = np.array([_pair(XT, int(i), int(j)) for i, j in zip(a, b)])
    err = np.abs(Cs - C64).max()
    print(f"max |C_bf16x3 - C_64| over {a.size} pairs: {err:.3e} (bound {_bf16x3_bound(m):.3e})")
    assert err <= _bf16x3_bound(m)
    G = adj.cpu().numpy()
    t0 = oracle.tau(alpha, m, 0)
    gpu_edge = (G[a, b >> 6] >> (b & 63).astype(np.int64)) & 1
    for i, j, c, e in zip(a, b, C64, gpu_edge):
        z = oracle.fisher_z(c)
        if abs(z - t0) <= 1e-9 * t0:
            continue     # FP64 tie band: either decision is acceptable
        assert bool(e) == (z > t0), (i, j, c)


def test_n8000_level1_sampled_edges_recomputed_by_oracle(big):
    X, XT, alpha = big
    m, n = X.shape
    ctx = pc.Context(precision="bf16x3")
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    st = pc.pc_run_stats()
    ctx.pc_skeleton(torch.from_numpy(X).cuda(), alpha, adj, recs, count, ws, max_level=1, stats=st)
    G1 = adj.cpu().numpy()
    t0, t1 = oracle.tau(alpha, m, 0), oracle.tau(alpha, m, 1)
    rng = np.random.default_rng(12)
    checked = removed = 0
    rows = {}
    while checked < 12:
        i = int(rng.integers(0, n))
        ci = rows[i] if i in rows else rows.setdefault(i, _corr_row(XT, i))
        Ni = np.flatnonzero([(k != i) and oracle.fisher_z(ci[k]) > t0 for k in range(n)])
        if Ni.size < 2:
            continue
        j = int(rng.choice(Ni))
        cj = rows[j] if j in rows else rows.setdefault(j, _corr_row(XT, j))
        Nj = np.flatnonzero([(k != j) and oracle.fisher_z(cj[k]) > t0 for k in range(n)])
        cands = set(Ni.tolist()) - {j} | (set(Nj.tolist()) - {i})
        indep, tie = False, False
        for k in sorted(cands):
            B = np.array([[1.0, ci[j], ci[k]], [ci[j], 1.0, cj[k]], [ci[k], cj[k], 1.0]])
            ind, z = oracle.ci_test_tau(B, 0, 1, [2], t1)
            tie |= abs(z - t1) <= 1e-9 * t1
            indep |= ind
        gpu_kept = bool((G1[i, j >> 6] >> (j & 63)) & 1)
        if not tie:
            assert gpu_kept == (not indep), (i, j)
        checked += 1
        removed += indep
    print(f"level-1 decisions of {checked} sampled edges match the oracle ({removed} removed)")


def test_n8000_levels_1_to_3_sampled_sepsets_pass_oracle(big):
    X, XT, alpha = big
    m, n = X.shape
    ctx = pc.Context(precision="bf16x3")
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    st = pc.pc_run_stats()
    status = ctx.pc_skeleton(torch.from_numpy(X).cuda(), alpha, adj, recs, count, ws, max_level=3, stats=st)
    d = st.as_dict()
    print("tests per level", d["tests"][:4], "removed", d["removed"][:4], "rechecks", d["rechecks"][:4],
          "status", status)
    k = int(count.item())
    R = recs[:k].cpu().numpy()
    G = pc.bits_to_dense(adj.cpu().numpy(), n)
    rng = np.random.default_rng(13)
    for level in (1, 2, 3):
        sel = np.flatnonzero(R[:, 2] == level)
        assert sel.size == d["removed"][level]
        for r in rng.choice(sel, size=min(300, sel.size), replace=False):
            i, j = int(R[r, 0]), int(R[r, 1])
            S = [int(s) for s in R[r, 3:3 + level]]
            assert i < j and not G[i, j] and len(set(S)) == level and i not in S and j not in S
            V = [i, j] + S
            B = np.eye(len(V))
            for p in range(len(V)):
                for q in range(p + 1, len(V)):
                    B[p, q] = B[q, p] = _pair(XT, V[p], V[q])
            ind, z, t = oracle.ci_test(B, 0, 1, list(range(2, len(V))), m, alpha)
            assert ind or abs(z - t) <= 1e-9 * t, (i, j, S, z, t)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name, X):
    g = np.load(os.path.join(GOLDEN, name), allow_pickle=False)
    assert str(g["digest"]) == hashlib.sha256(np.ascontiguousarray(X, dtype=np.float64).tobytes()).hexdigest(), \
        "stored oracle result is for another input"
    return g


def _dense_edges(E, n):
    G = np.zeros((n, n), np.uint8)
    G[E[:, 0], E[:, 1]] = 1
    return G | G.T


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_n8000_levels_1_to_3_whole_graph_matches_stored_oracle(big, prec):
    """G after each of levels 1, 2, 3 equals the oracle's, bit for bit, and so does the number of
    edges each level removes."""
    X, XT, alpha = big
    m, n = X.shape
    g = _golden("n8000_d6_m2000_levels3.npz", X)
    ctx = pc.Context(precision=prec)
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * n // 4)
    Xd = torch.from_numpy(X).cuda()
    for L in (1, 2, 3):
        print(f"n8000 {prec} max_level {L}", flush=True)
        st = pc.pc_run_stats()
        assert ctx.pc_skeleton(Xd, alpha, adj, recs, count, ws, max_level=L, stats=st) == 0
        G = pc.bits_to_dense(adj.cpu().numpy(), n)
        ref = _dense_edges(g[f"edges_after_{L}"], n)
        assert np.array_equal(G, ref), (L, np.argwhere(G != ref)[:8])
        assert list(st.removed[:L + 1]) == list(g["removed"][:L + 1])
        assert int(count.item()) == int(g["removed"][1:L + 1].sum())


@pytest.fixture(scope="module")
def apply_workload():
    X, sem, alpha = semgen.workload("n2000_d10_m1000_apply")
    ref = oracle.skeleton(X, alpha)
    return np.ascontiguousarray(X), alpha, ref


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_n2000_d10_skeleton_matches_oracle(apply_workload, prec):
    X, alpha, ref = apply_workload
    G, seps, st, status = pc.skeleton(X, alpha, precision=prec)
    assert np.array_equal(G, ref.G)
    assert set(seps) == set(ref.sepsets.as_dict())
    assert st["tests"][0] == ref.tests[0]


def test_n2000_d10_learned_order_matches_oracle(apply_workload):
    X, alpha, ref = apply_workload
    from paper_1812_08491_amd import learn
    params = learn.load_weights() if _have_weights() else torch.from_numpy(
        learn.init_params(np.random.default_rng(5))).cuda()
    cmp = learn.compare_orders(X, alpha, params, min_level=2, top=4, repeats=1)
    assert cmp["same_skeleton"]
    m, n = X.shape
    ctx = pc.Context(precision="fp32")
    order = ctx.order(params, min_level=2, top=4)
    ws = ctx.ordered_workspace(n, m, order)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    ctx.pc_skeleton_ordered(torch.from_numpy(X).cuda(), alpha, adj, recs, count, ws, order)
    assert np.array_equal(pc.bits_to_dense(adj.cpu().numpy(), n), ref.G)
    print({k: cmp[k] for k in ("plain", "learned")})


def _have_weights():
    import os
    from paper_1812_08491_amd import learn
    return os.path.exists(learn.DEFAULT_WEIGHTS)


def _degenerate(A, i, j, S):
    return any(A[np.ix_(V, V)].max() > 1 - 1e-6 for V in ([i] + list(S), [j] + list(S)))


_ORACLE_SCAL = {}


def _scal_oracle(n, p, m):
    if (n, p, m) not in _ORACLE_SCAL:
        _ORACLE_SCAL.clear()
        X, sem, alpha = semgen.scalability(n, p, m)
        C = oracle.corr(X)
        _ORACLE_SCAL[(n, p, m)] = (X, alpha, C, oracle.skeleton_corr(C, m, alpha))
    return _ORACLE_SCAL[(n, p, m)]


@pytest.mark.parametrize("n,p,m,prec", [
    (1000, 0.1, 10000, "fp64"), (1000, 0.1, 10000, "fp32"), (1000, 0.1, 2000, "fp64"),
    (1000, 0.3, 10000, "fp64"), (1000, 0.3, 10000, "fp32"), (1000, 0.5, 10000, "fp64"),
    (2000, 0.1, 10000, "fp64")])
def test_paper_scalability_grid_matches_oracle(n, p, m, prec):
    """Points of the paper's scalability grid (Sec. 5.6, Fig. 10: edge probability p per pair,
    positive weights, m samples). Variances grow along the order (at n = 1000, p = 0.1 about 50
    parents per node), so many late variables are collinear to FP64 rounding: at n = 1000, p = 0.1,
    m = 10000, 179 k pairs have |C| within 1e-12 of 1, and at p = 0.3 three quarters of all pairs.
    There H11 = 1 - C_ik^2 of a level-1 test can round to <= 0 on one side (rho := 0, independent)
    and to a tiny positive value on the other (|rho| >= 1, dependent), so exact parity is not
    defined for those tests: parity partial. Checked: every pair on which the GPU and the oracle
    differ is decided by such a near-collinear test (some |C| > 1 - 1e-6 within {i} u S or {j} u S,
    with S the SepSet of the side that removed it), the same number of levels runs, and every
    sampled GPU SepSet passes the oracle's FP64 test unless it is near-collinear. In FP32 nearly
    every test falls inside the error band, the re-check queue overflows, and the run is completed
    in FP64 from that level (fp64_from)."""
    print(f"paper scalability n={n} p={p} m={m} {prec}", flush=True)
    X, alpha, C, ref = _scal_oracle(n, p, m)
    G, seps, st, status = pc.skeleton(np.ascontiguousarray(X), alpha, precision=prec)
    assert status == 0
    if prec == "fp32":
        assert st["fp64_from"] >= 1
    assert st["levels_run"] == ref.levels_run
    A = np.abs(C - np.eye(n))
    ref_seps = ref.sepsets.as_dict()
    diff = np.argwhere(np.triu(G != ref.G, 1))
    print("pairs that differ:", len(diff), flush=True)
    for i, j in diff:
        i, j = int(i), int(j)
        S = seps[(i, j)][1] if G[i, j] == 0 else ref_seps.get((i, j), (0, ()))[1]
        assert _degenerate(A, i, j, S), ((i, j), int(G[i, j]), S)
    keys = list(seps)
    bad = 0
    for t in np.random.default_rng(3).choice(len(keys), min(2000, len(keys)), replace=False):
        e = keys[t]
        l, S = seps[e]
        if not oracle.ci_test(C, e[0], e[1], list(S), m, alpha)[0]:
            assert _degenerate(A, e[0], e[1], S), (e, S)
            bad += 1
    print("sampled GPU SepSets on near-collinear tests:", bad, flush=True)
