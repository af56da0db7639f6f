"""GPU orientation (pc_orient) against the CPU reference (oracle/orient.py), marked gpu.

Both sides take the same skeleton and SepSets (the GPU's own skeleton output, or hand-made ones)
and must give the same arrowhead matrix bit for bit, and the same number of propagation rounds.
"""
import numpy as np
import pytest

import oracle
import semgen
from oracle import orient

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_08491_amd as pc  # noqa: E402


def gpu_skeleton(X, alpha, prec):
    m, n = X.shape
    ctx = pc.Context(precision=prec)
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    status = ctx.pc_skeleton(torch.from_numpy(np.ascontiguousarray(X)).cuda(), alpha, adj, recs, count, ws)
    assert status >= 0
    return ctx, adj, recs, int(count.item())


def compare(ctx, n, adj, recs, nrec):
    arrows = ctx.adjacency(n)
    arrows.fill_(-1)   # every bit must be written
    ws = ctx.orient_workspace(n)
    rounds = ctx.pc_orient(n, adj, recs, nrec, arrows, ws)
    H = pc.bits_to_dense(arrows.cpu().numpy(), n).astype(bool)
    G = pc.bits_to_dense(adj.cpu().numpy(), n).astype(bool)
    seps = pc.decode_sepsets(recs[:max(nrec, 1)].cpu().numpy(), nrec)
    H_ref, rounds_ref = orient.orient(G, orient.sepset_lookup(seps))
    assert np.array_equal(H, H_ref), np.argwhere(H != H_ref)[:8]
    assert rounds == rounds_ref
    assert not (H & ~G).any()
    return H, rounds


@pytest.mark.parametrize("wl,prec", [("n50_p005_m1000_fp64", "fp64"), ("n1000_d4_m500_fp32", "fp32"),
                                     ("n1000_d4_m500_fp32", "bf16x3")])
def test_orientation_of_gpu_skeleton_matches_reference(wl, prec):
    X, sem, alpha = semgen.workload(wl)
    print(f"orient {wl} {prec}", flush=True)
    ctx, adj, recs, k = gpu_skeleton(X, alpha, prec)
    H, rounds = compare(ctx, X.shape[1], adj, recs, k)
    assert H.any()


@pytest.mark.parametrize("seed", range(4))
def test_orientation_ragged_dense_graphs(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(5, 200))
    X = semgen.sample(semgen.random_dag(n, float(rng.uniform(0.05, 0.3)), rng), int(rng.integers(100, 800)), rng)
    print(f"orient ragged seed={seed} n={n}", flush=True)
    ctx, adj, recs, k = gpu_skeleton(X, 0.05, "fp32")
    compare(ctx, n, adj, recs, k)


def test_orientation_n2000_degree10():
    X, sem, alpha = semgen.workload("n2000_d10_m1000_apply")
    print("orient n2000", flush=True)
    ctx, adj, recs, k = gpu_skeleton(X, alpha, "fp32")
    H, rounds = compare(ctx, X.shape[1], adj, recs, k)
    assert rounds >= 1


def _upload(n, edges, seps):
    G = np.zeros((n, n), dtype=np.uint8)
    for a, b in edges:
        G[a, b] = G[b, a] = 1
    adj = torch.from_numpy(pc.dense_to_bits(G)).cuda()
    rows = []
    for (i, j), S in seps.items():
        r = [i, j, len(S)] + list(S) + [-1] * (pc.PC_MAX_LEVEL - len(S))
        rows.append(r)
    recs = torch.tensor(np.array(rows, dtype=np.int32).reshape(-1, 3 + pc.PC_MAX_LEVEL)).cuda()
    return adj, recs, len(rows)


def test_orientation_handmade_rules_and_conflict():
    ctx = pc.Context(precision="fp32")
    # R1 and R2 (two rounds), R3, and colliders in conflict (a bidirected edge), in one graph of
    # disjoint parts; level-0 removals have no record
    edges = [(0, 2), (1, 2), (2, 3), (0, 3),                      # R1 then R2
             (5, 4), (6, 4), (7, 4), (7, 5), (7, 6),              # R3 (c=5, d=6, b=4, a=7)
             (8, 9), (9, 10), (10, 11)]                          # conflicting colliders at 9, 10
    seps = {(1, 3): (2,), (5, 6): (7,)}
    adj, recs, k = _upload(12, edges, seps)
    H, rounds = compare(ctx, 12, adj, recs, k)
    assert H[9, 10] and H[10, 9] and rounds == 2
    # no records at all: every non-adjacent pair separated by the empty set
    adj2, recs2, _ = _upload(12, edges, {(0, 1): ()})
    compare(ctx, 12, adj2, recs2, 0)
