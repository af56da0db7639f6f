"""pc_skeleton_noalloc (the entry point that allocates nothing; its workspace is the library's static
per-GPU array) against pc_skeleton with a caller workspace, on two calls in a row, the second with a
smaller input, so that what the first call left in the shared array cannot leak into the second
(marked gpu). The bar is the parity bar of the rest of the suite: the same adjacency bit for bit,
the same removal level for every removed pair, and every SepSet passing the oracle's FP64 test."""
import numpy as np
import pytest

import oracle
import semgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_08491_amd as pc  # noqa: E402


def _data(seed, n, d, m):
    rng = np.random.default_rng(seed)
    sem = semgen.random_dag(n, semgen.expected_degree_p(n, d), rng)
    return np.ascontiguousarray(semgen.sample(sem, m, rng))


def _run(ctx, X, alpha, noalloc):
    m, n = X.shape
    Xd = torch.from_numpy(X).cuda()
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    st = pc.pc_run_stats()
    if noalloc:
        status = ctx.pc_skeleton_noalloc(Xd, alpha, adj, recs, count, stats=st)
    else:
        ws = ctx.workspace(n, m)
        status = ctx.pc_skeleton(Xd, alpha, adj, recs, count, ws, stats=st)
    k = int(count.item())
    return status, pc.bits_to_dense(adj.cpu().numpy(), n), pc.decode_sepsets(recs[:k].cpu().numpy(), k), st.as_dict()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_workspace_entry_point_on_two_calls(prec):
    ctx = pc.Context(precision=prec)
    # the larger call first (n = 1000 at m = 500 in FP32 is the size class the array is made for),
    # then a smaller one on the array the first call left behind
    cases = [(1, 1000 if prec == "fp32" else 700, 4.0, 500, 0.01), (2, 150, 3.0, 400, 0.05)]
    for seed, n, d, m, alpha in cases:
        print(f"noalloc {prec} n={n} m={m}", flush=True)
        X = _data(seed, n, d, m)
        s0, G0, seps0, st0 = _run(ctx, X, alpha, noalloc=False)
        s1, G1, seps1, st1 = _run(ctx, X, alpha, noalloc=True)
        assert s0 == 0 and s1 == 0
        assert np.array_equal(G1, G0)
        assert st1["levels_run"] == st0["levels_run"]
        assert {e: l for e, (l, S) in seps1.items()} == {e: l for e, (l, S) in seps0.items()}
        C = oracle.corr(X)
        for (i, j), (l, S) in seps1.items():
            assert oracle.ci_test(C, i, j, list(S), m, alpha)[0], (i, j, l, S)


def test_noalloc_rejects_problems_beyond_its_array():
    ctx = pc.Context(precision="fp32")
    X = _data(3, 2000, 2.0, 1000)           # workspace about 131 MiB > 64 MiB
    Xd = torch.from_numpy(X).cuda()
    adj = ctx.adjacency(2000)
    recs, count = ctx.sepsets(16)
    with pytest.raises(pc.PCError) as e:
        ctx.pc_skeleton_noalloc(Xd, 0.01, adj, recs, count)
    assert e.value.status == -5
