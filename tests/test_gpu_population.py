"""GPU runs on a correlation matrix the caller supplies (pc_skeleton_corr / pc_level_corr; marked gpu).

The CI test of Sec. 4.3 needs only C and a sample size, so a population correlation matrix with a
nominal m = 1e20 runs the tests in the large-sample limit (tau ~ 2.6e-10 at alpha 0.01). There
PC-stable returns the skeleton of the true DAG, and every SepSet d-separates its pair (Sec. 2.4).
These tests hold the GPU path to what brute-force d-separation (tests/ref/dsep.py) and the
hand-worked examples fix, and to the oracle on the same C:
  * 40 random DAGs (n <= 7): skeleton = true skeleton = the oracle's, same removal level per pair,
    every GPU SepSet d-separates its pair;
  * chain / collider / diamond (values worked by hand in tests/test_oracle.py);
  * a variable duplicated exactly, so that conditioning sets holding both copies have a singular
    M2 and take the pseudo-inverse route (Sec. 4.4): exact parity with the oracle at level 2 on
    the complete graph, with the route taken on the GPU (except tests of a copy given its twin,
    which rounding alone decides);
  * pc_level_corr on the oracle's own FP64 sample correlation and snapshots G'.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import semgen
from tests.ref import dsep

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1812_08491_amd as pc  # noqa: E402

M_INF = 1e20


def gpu_skeleton_corr(C, m, alpha, max_level=-1):
    n = C.shape[0]
    ctx = pc.Context(precision="fp64")
    ws = ctx.corr_workspace(n)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    st = pc.pc_run_stats()
    Cd = torch.from_numpy(np.ascontiguousarray(C, dtype=np.float64)).cuda()
    status = ctx.pc_skeleton_corr(Cd, m, alpha, adj, recs, count, ws, max_level=max_level, stats=st)
    k = int(count.item())
    return (pc.bits_to_dense(adj.cpu().numpy(), n), pc.decode_sepsets(recs[:k].cpu().numpy(), k),
            st.as_dict(), status)


@pytest.mark.parametrize("seed", range(40))
def test_large_sample_limit_gpu_matches_dseparation(seed):
    rng = np.random.default_rng(10_000 + seed)       # the DAGs of the oracle's own pin
    n = int(rng.integers(3, 8))
    sem = semgen.random_dag(n, float(rng.uniform(0.2, 0.7)), rng)
    C = dsep.population_corr(sem)
    G, seps, st, status = gpu_skeleton_corr(C, M_INF, 0.01)
    assert status == 0
    truth = sem.skeleton()
    assert np.array_equal(G.astype(bool), truth), (seed, np.argwhere(G.astype(bool) != truth))
    ref = oracle.skeleton_corr(C, M_INF, 0.01)
    assert np.array_equal(G, ref.G)
    assert st["levels_run"] == ref.levels_run
    ref_seps = ref.sepsets.as_dict()
    assert set(seps) == set(ref_seps)
    pa = dsep.parents_of(sem)
    for (i, j), (l, S) in seps.items():
        assert i < j and len(S) == l and ref_seps[(i, j)][0] == l
        assert dsep.d_separated(pa, i, j, S), (seed, i, j, S)
    # level-0 removals carry no record: exactly the marginally independent pairs
    for i, j in itertools.combinations(range(n), 2):
        if not truth[i, j] and (i, j) not in seps:
            assert dsep.d_separated(pa, i, j, ())


def test_chain_collider_diamond_examples():
    # chain X -> Y -> Z (a = 0.8, b = 0.5): level 1 removes X - Z with {Y}
    a, b = 0.8, 0.5
    rxy = a / math.sqrt(1 + a * a)
    ryz = b * math.sqrt(1 + a * a) / math.sqrt(b * b * (1 + a * a) + 1)
    rxz = a * b / math.sqrt(b * b * (1 + a * a) + 1)
    C = np.array([[1, rxy, rxz], [rxy, 1, ryz], [rxz, ryz, 1.0]])
    G, seps, st, _ = gpu_skeleton_corr(C, M_INF, 0.01)
    assert G.tolist() == [[0, 1, 0], [1, 0, 1], [0, 1, 0]]
    assert seps == {(0, 2): (1, (1,))}
    # collider X -> Z <- Y: level 0 removes X - Y (r = 0), and it is not re-added
    vz = a * a + b * b + 1
    C = np.array([[1, 0.0, a / math.sqrt(vz)], [0.0, 1, b / math.sqrt(vz)], [a / math.sqrt(vz), b / math.sqrt(vz), 1.0]])
    G, seps, st, _ = gpu_skeleton_corr(C, M_INF, 0.01)
    assert G.tolist() == [[0, 0, 1], [0, 0, 1], [1, 1, 0]]
    assert seps == {} and st["removed"][0] == 1
    # diamond X -> Y, X -> Z, Y -> W, Z -> W: Y - Z goes at level 1 with {X}, X - W at level 2
    sem = semgen.SEM(n=4, order=np.arange(4),
                     parents=[np.array([], np.int64), np.array([0]), np.array([0]), np.array([1, 2])],
                     weights=[np.array([]), np.array([0.8]), np.array([-0.6]), np.array([0.7, 0.5])])
    G, seps, st, _ = gpu_skeleton_corr(dsep.population_corr(sem), M_INF, 0.01)
    assert G.tolist() == sem.skeleton().astype(np.uint8).tolist()
    assert seps == {(1, 2): (1, (0,)), (0, 3): (2, (1, 2))}


def _duplicated_population(seed, n=9, p=0.45):
    """Population C of a random SEM with variable n-1 an exact copy of variable 0 (C's row and
    column n-1 equal those of 0, C[0, n-1] = 1)."""
    rng = np.random.default_rng(seed)
    sem = semgen.random_dag(n - 1, p, rng)
    C0 = dsep.population_corr(sem)
    C = np.empty((n, n))
    C[:n - 1, :n - 1] = C0
    C[n - 1, :n - 1] = C0[0]
    C[:n - 1, n - 1] = C0[0]
    C[n - 1, n - 1] = 1.0
    return C


@pytest.mark.parametrize("seed", range(4))
def test_pseudo_inverse_route_on_duplicated_variable(seed):
    """Level 2 on the complete graph: every test whose S holds both copies has M2 = C[S,S]
    singular (a zero Cholesky pivot), which both sides send to the Moore-Penrose inverse. The
    GPU level must equal the oracle's level on the same G' exactly."""
    C = _duplicated_population(300 + seed)
    n = C.shape[0]
    alpha, level = 0.01, 2
    Gp = np.ones((n, n), np.uint8) - np.eye(n, dtype=np.uint8)
    G_ref, seps_ref, _, _ = oracle.level(C, M_INF, alpha, level, Gp.copy())
    # Pairs that survive the level were tested with every S, among them S = {0, n-1}, whose M2 is
    # singular: the oracle's partial correlation takes the pseudo-inverse there.
    surv = [(i, j) for i, j in itertools.combinations(range(1, n - 1), 2) if G_ref[i, j]]
    assert surv and all(oracle.pcor(C, i, j, [0, n - 1])[1] for i, j in surv)
    ctx = pc.Context(precision="fp64")
    ws = ctx.corr_workspace(n)
    recs, count = ctx.sepsets(n * n)
    adj = torch.from_numpy(pc.dense_to_bits(Gp)).cuda()
    st = pc.pc_run_stats()
    Cd = torch.from_numpy(np.ascontiguousarray(C)).cuda()
    assert ctx.pc_level_corr(level, Cd, M_INF, alpha, adj, recs, count, ws, stats=st) == 0
    G = pc.bits_to_dense(adj.cpu().numpy(), n)
    # the singular sets went through the re-check kernel's pseudo-inverse
    assert st.rechecks[level] > 0
    k = int(count.item())
    seps = pc.decode_sepsets(recs[:k].cpu().numpy(), k)
    ref_seps = seps_ref.as_dict()
    # Pairs (c, x) with c one copy and the other copy in S have H11 (or H22) = 0 in exact arithmetic
    # (the copy is a linear function of S), so rounding alone decides them on either side (a
    # reading of the paper: near-collinear tests). Every other pair, including all those tested with
    # the singular S = {0, n-1}, must agree exactly.
    twin = {0: n - 1, n - 1: 0}
    for i, j in np.argwhere(np.triu(G != G_ref, 1)):
        i, j = int(i), int(j)
        S = seps[(i, j)][1] if G[i, j] == 0 else ref_seps[(i, j)][1]
        assert any(c in twin and twin[c] in S for c in (i, j)), ((i, j), int(G[i, j]), S)
    for (i, j), (l, S) in seps.items():
        assert l == level and (all(Gp[i, s] for s in S) or all(Gp[j, s] for s in S))
        if not any(c in twin and twin[c] in S for c in (i, j)):
            assert oracle.ci_test(C, i, j, list(S), M_INF, alpha)[0], (i, j, S)


@pytest.mark.parametrize("seed,n,p,m,alpha", [(41, 60, 0.25, 400, 0.05), (42, 120, 0.06, 800, 0.01)])
def test_level_corr_on_oracle_snapshots(seed, n, p, m, alpha):
    """pc_level_corr on the oracle's FP64 sample correlation: every level from the oracle's G'
    gives the oracle's G."""
    rng = np.random.default_rng(seed)
    X = semgen.sample(semgen.random_dag(n, p, rng), m, rng)
    C = oracle.corr(X)
    ref = oracle.skeleton_corr(C, m, alpha, keep_levels=True)
    ctx = pc.Context(precision="fp64")
    ws = ctx.corr_workspace(n)
    recs, count = ctx.sepsets(n * n)
    Cd = torch.from_numpy(np.ascontiguousarray(C)).cuda()
    G, seps, st, status = gpu_skeleton_corr(C, float(m), alpha)
    assert status == 0 and np.array_equal(G, ref.G) and st["levels_run"] == ref.levels_run
    for l in range(1, ref.levels_run):
        adj = torch.from_numpy(pc.dense_to_bits(ref.G_after[l - 1])).cuda()
        assert ctx.pc_level_corr(l, Cd, float(m), alpha, adj, recs, count, ws) == 0
        assert np.array_equal(pc.bits_to_dense(adj.cpu().numpy(), n), ref.G_after[l]), l


def test_given_corr_argument_checks():
    C = torch.eye(5, dtype=torch.float64, device="cuda")
    ctx32 = pc.Context(precision="fp32")
    ws = ctx32.corr_workspace(5)
    adj = ctx32.adjacency(5)
    recs, count = ctx32.sepsets(10)
    with pytest.raises(pc.PCError) as e:
        ctx32.pc_skeleton_corr(C, M_INF, 0.01, adj, recs, count, ws)
    assert e.value.status == -7            # FP64 contexts only
    ctx = pc.Context(precision="fp64")
    ws = ctx.corr_workspace(5)
    with pytest.raises(pc.PCError):
        ctx.pc_skeleton_corr(C, -1.0, 0.01, adj, recs, count, ws)
    # m - l - 3 <= 0 at level 1 (m = 4): level 0 keeps every pair (tau_0 = z = 2.576 and
    # atanh 0.995 = 2.99), level 1 is not run and the call warns
    C2 = torch.from_numpy(np.full((5, 5), 0.995) + 0.005 * np.eye(5)).cuda()
    assert ctx.pc_skeleton_corr(C2, 4.0, 0.01, adj, recs, count, ws) == 1
    assert pc.bits_to_dense(adj.cpu().numpy(), 5).sum() == 20
