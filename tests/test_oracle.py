"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix (CPU only).

Each test compares the oracle with something other than itself: scipy / numpy routines on a
different formula, closed forms, exact distributions, brute-force d-separation in the large-sample
limit, the paper's printed examples, and structural invariants of PC-stable.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy import special, stats

import oracle
import semgen
from tests.ref import dsep, levelcheck

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------------------------------
# Phi^-1 and the threshold of Eq. 6
# ------------------------------------------------------------------------------------------
def test_ppnd_matches_scipy_and_inverts_ndtr():
    ps = np.concatenate([np.logspace(-300, -1, 200), np.linspace(0.01, 0.99, 199),
                         1 - np.logspace(-15, -1, 50)])
    for p in ps:
        x = oracle.ppnd(float(p))
        ref = stats.norm.ppf(p)
        assert abs(x - ref) <= 2e-15 * max(1.0, abs(ref)), (p, x, ref)
        # Phi(Phi^-1(p)) = p, with Phi from scipy's ndtr (a different routine).
        if 1e-250 < p < 0.999:
            assert abs(special.ndtr(x) - p) <= 1e-12 * p, p
    assert oracle.ppnd(0.5) == 0.0
    for p in (2.0 ** -30, 0.0625, 0.125, 0.25, 0.375):     # 1 - p exact in binary
        assert oracle.ppnd(1 - p) == pytest.approx(-oracle.ppnd(p), rel=1e-14)
    assert math.isnan(oracle.ppnd(0.0)) and math.isnan(oracle.ppnd(1.0))


@pytest.mark.parametrize("level", [0, 1, 2, 4])
@pytest.mark.parametrize("m", [10, 14, 30])
def test_threshold_gives_exact_null_rejection_near_alpha(level, m):
    """tau_l = z / sqrt(m - l - 3) (Eq. 6) is Fisher's scaling: under independence, the sample
    partial correlation given l variables from m Gaussian samples is distributed as a sample
    correlation from m - l samples, i.e. t = r sqrt(k / (1 - r^2)) ~ Student t with k = m - l - 2.
    The exact rejection probability P(|atanh r| > tau) must be close to alpha, and closer than the
    neighbouring scalings m - l - 2 and m - l - 4 would give."""
    alpha = 0.05
    k = m - level - 2

    def reject(t):
        r = math.tanh(t)
        return 2 * stats.t.sf(r * math.sqrt(k / (1 - r * r)), k)

    z = stats.norm.ppf(1 - alpha / 2)
    ours = reject(oracle.tau(alpha, m, level))
    assert abs(ours - alpha) < 0.004, ours
    for dof in (m - level - 2, m - level - 4):
        assert abs(ours - alpha) < abs(reject(z / math.sqrt(dof)) - alpha)
    assert math.isnan(oracle.tau(alpha, level + 3, level))


def test_fisher_z_trap_pair():
    """The comparison is on atanh(r), not on r (Eq. 5): m = 100, alpha = 0.05."""
    t = oracle.tau(0.05, 100, 0)
    assert t == pytest.approx(0.199004, abs=1e-6)
    C = np.array([[1.0, 0.197], [0.197, 1.0]])
    assert not oracle.ci_test(C, 0, 1, [], 100, 0.05)[0]      # 0.197 < tau but atanh > tau
    C[0, 1] = C[1, 0] = 0.1
    assert oracle.ci_test(C, 0, 1, [], 100, 0.05)[0]
    assert oracle.fisher_z(0.5) == pytest.approx(math.atanh(0.5), rel=1e-15)
    assert oracle.fisher_z(-1.0) == math.inf


def test_tie_removes_edge():
    """Z <= tau means independent, so an exact tie removes the edge (Sec. 4.3)."""
    for l, C, S in [(0, np.array([[1.0, 0.3], [0.3, 1.0]]), []),
                    (1, np.array([[1.0, 0.3, 0.2], [0.3, 1.0, 0.5], [0.2, 0.5, 1.0]]), [2])]:
        ind, z = oracle.ci_test_tau(C, 0, 1, S, 0.5)
        assert 0 < z < 0.5 and ind
        assert oracle.ci_test_tau(C, 0, 1, S, z)[0]                           # tie: independent
        assert not oracle.ci_test_tau(C, 0, 1, S, math.nextafter(z, 0.0))[0]   # just below: not


# ------------------------------------------------------------------------------------------
# Correlation and partial correlation (Eq. 3-4) and the pseudo-inverse (Sec. 4.4)
# ------------------------------------------------------------------------------------------
def test_corr_matches_numpy_corrcoef():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((137, 23)) @ rng.standard_normal((23, 23)) + 5.0
    C = oracle.corr(X)
    assert np.allclose(C, np.corrcoef(X, rowvar=False), atol=1e-14, rtol=0)
    assert np.all(np.diag(C) == 1.0)
    for a, b in [(0, 1), (5, 22), (9, 9)]:
        assert oracle.corr_pair(X, a, b) == pytest.approx(C[a, b], abs=1e-15)


def test_corr_errors():
    X = np.random.default_rng(0).standard_normal((20, 4))
    X[:, 2] = 3.0
    with pytest.raises(oracle.OracleError):
        oracle.corr(X)
    X = np.random.default_rng(0).standard_normal((20, 4))
    X[3, 1] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.corr(X)


def test_pcor_level1_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(50):
        A = rng.standard_normal((6, 6))
        Sg = A @ A.T + 0.1 * np.eye(6)
        d = np.sqrt(np.diag(Sg))
        C = Sg / np.outer(d, d)
        i, j, k = rng.choice(6, 3, replace=False)
        ref = (C[i, j] - C[i, k] * C[j, k]) / math.sqrt((1 - C[i, k] ** 2) * (1 - C[j, k] ** 2))
        got, used = oracle.pcor(C, int(i), int(j), [int(k)])
        assert not used
        assert got == pytest.approx(ref, abs=1e-13)


def test_pcor_equals_ols_residual_correlation_and_block_inverse():
    """rho(i,j|S) equals the correlation of the OLS residuals of X_i and X_j on X_S (raw data,
    numpy lstsq), and -P12/sqrt(P11 P22) for P the inverse of the whole block."""
    rng = np.random.default_rng(2)
    m, n = 400, 9
    X = rng.standard_normal((m, n)) @ rng.standard_normal((n, n))
    C = oracle.corr(X)
    for _ in range(40):
        l = int(rng.integers(1, 6))
        idx = rng.choice(n, l + 2, replace=False)
        i, j, S = int(idx[0]), int(idx[1]), [int(s) for s in idx[2:]]
        got, used = oracle.pcor(C, i, j, S)
        assert not used
        Z = np.column_stack([np.ones(m), X[:, S]])
        ri = X[:, i] - Z @ np.linalg.lstsq(Z, X[:, i], rcond=None)[0]
        rj = X[:, j] - Z @ np.linalg.lstsq(Z, X[:, j], rcond=None)[0]
        ref = float(ri @ rj / math.sqrt((ri @ ri) * (rj @ rj)))
        assert got == pytest.approx(ref, abs=1e-11)
        assert got == pytest.approx(levelcheck.pcor_block(C, i, j, S), abs=1e-11)


def test_pinv_penrose_conditions():
    rng = np.random.default_rng(3)
    for k, r in [(1, 0), (1, 1), (3, 1), (4, 2), (6, 3), (8, 8)]:
        B = rng.standard_normal((k, r))
        A = B @ B.T
        P = oracle.pinv_sym(A)
        assert np.allclose(A @ P @ A, A, atol=1e-10)
        assert np.allclose(P @ A @ P, P, atol=1e-8)
        assert np.allclose((A @ P).T, A @ P, atol=1e-10)
        assert np.allclose((P @ A).T, P @ A, atol=1e-10)
        assert np.allclose(P, np.linalg.pinv(A, hermitian=True), atol=1e-8)


def test_pcor_rank_deficient_uses_pinv():
    """A duplicated conditioning variable makes M2 singular: the pseudo-inverse path must give the
    same rho as conditioning on the variable once (the column spaces are equal)."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 5)) @ rng.standard_normal((5, 5))
    X = np.column_stack([X, X[:, 2]])          # variable 5 duplicates variable 2
    C = oracle.corr(X)
    C[2, 5] = C[5, 2] = 1.0
    rho, used = oracle.pcor(C, 0, 1, [2, 5])
    assert used
    ref, used1 = oracle.pcor(C, 0, 1, [2])
    assert not used1
    assert rho == pytest.approx(ref, abs=1e-10)


# ------------------------------------------------------------------------------------------
# Hand-worked population examples
# ------------------------------------------------------------------------------------------
def _chain_C(a=0.8, b=0.5):
    rxy = a / math.sqrt(1 + a * a)
    ryz = b * math.sqrt(1 + a * a) / math.sqrt(b * b * (1 + a * a) + 1)
    rxz = a * b / math.sqrt(b * b * (1 + a * a) + 1)
    return np.array([[1, rxy, rxz], [rxy, 1, ryz], [rxz, ryz, 1.0]])


def test_chain_example():
    C = _chain_C()
    assert C[0, 1] == pytest.approx(0.624695, abs=1e-6)
    assert C[0, 2] == pytest.approx(0.336861, abs=1e-6)
    assert abs(oracle.pcor(C, 0, 2, [1])[0]) < 1e-15
    sk = oracle.skeleton_corr(C, 1e20, 0.01)
    assert sk.G.tolist() == [[0, 1, 0], [1, 0, 1], [0, 1, 0]]
    assert sk.sepsets.as_dict() == {(0, 2): (1, (1,))}
    # Fork X <- Y -> Z has the same correlation pattern up to relabelling.
    perm = [1, 0, 2]
    sk2 = oracle.skeleton_corr(C[np.ix_(perm, perm)], 1e20, 0.01)
    assert sk2.G.tolist() == [[0, 1, 1], [1, 0, 0], [1, 0, 0]]


def test_collider_example():
    a, b = 0.8, 0.5
    vz = a * a + b * b + 1
    rxz, ryz = a / math.sqrt(vz), b / math.sqrt(vz)
    C = np.array([[1, 0.0, rxz], [0.0, 1, ryz], [rxz, ryz, 1.0]])
    assert oracle.pcor(C, 0, 1, [2])[0] == pytest.approx(-a * b / math.sqrt((1 + a * a) * (1 + b * b)),
                                                        abs=1e-15)
    assert oracle.pcor(C, 0, 1, [2])[0] == pytest.approx(-0.279372, abs=1e-6)
    sk = oracle.skeleton_corr(C, 1e20, 0.01)
    assert sk.G.tolist() == [[0, 0, 1], [0, 0, 1], [1, 1, 0]]
    assert sk.removed[0] == 1 and sk.sepsets.as_dict() == {}


def test_diamond_example():
    sem = semgen.SEM(n=4, order=np.arange(4),
                     parents=[np.array([], np.int64), np.array([0]), np.array([0]), np.array([1, 2])],
                     weights=[np.array([]), np.array([0.8]), np.array([-0.6]), np.array([0.7, 0.5])])
    C = dsep.population_corr(sem)
    assert abs(oracle.pcor(C, 1, 2, [0])[0]) < 1e-14
    assert oracle.pcor(C, 0, 3, [1])[0] == pytest.approx(-0.205076, abs=1e-6)
    assert oracle.pcor(C, 0, 3, [2])[0] == pytest.approx(0.366083, abs=1e-6)
    assert abs(oracle.pcor(C, 0, 3, [1, 2])[0]) < 1e-14
    sk = oracle.skeleton_corr(C, 1e20, 0.01, keep_levels=True)
    assert sk.G.tolist() == sem.skeleton().astype(np.uint8).tolist()
    assert sk.sepsets.as_dict() == {(1, 2): (1, (0,)), (0, 3): (2, (1, 2))}
    assert sk.G_after[1][0, 3] == 1 and sk.G_after[2][0, 3] == 0


def _read_fig1():
    spec = {}
    for line in open(os.path.join(GOLDEN, "fig1_narrative.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, *rest = line.split()
        spec[key] = rest
    return spec


def test_fig1_narrative_counts():
    """Sec. 2.4 text of Fig. 1: 6 tests at level 0 removing (V1,V2); 12 at level 1 removing
    (V1,V3) and (V2,V3)."""
    spec = _read_fig1()
    parents, weights = [[] for _ in range(4)], [[] for _ in range(4)]
    for e in spec["dag"]:
        uv, w = e.split(":")
        u, v = (int(x) for x in uv.split("->"))
        parents[v].append(u)
        weights[v].append(float(w))
    sem = semgen.SEM(n=4, order=np.array([1, 2, 0, 3]),
                     parents=[np.array(p, np.int64) for p in parents],
                     weights=[np.array(w) for w in weights])
    C = dsep.population_corr(sem)
    sk = oracle.skeleton_corr(C, 1e20, 0.01)
    l0 = dict(x.split("=") for x in spec["level0"])
    l1 = spec["level1"]
    assert sk.tests[0] == int(l0["tests"])
    assert sk.tests[1] == int(l1[0].split("=")[1])
    removed1 = {}
    for x in [l1[1][len("removed="):]] + l1[2:]:
        pair, S = x.split(":")
        a, b = (int(v) for v in pair.split(","))
        removed1[(a, b)] = (1, (int(S),))
    assert sk.sepsets.as_dict() == removed1
    a, b = (int(v) for v in l0["removed"].split(","))
    assert sk.G[a, b] == 0 and (a, b) not in sk.sepsets.as_dict()


# ------------------------------------------------------------------------------------------
# Whole algorithm: large-sample limit against brute-force d-separation
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(40))
def test_large_sample_limit_matches_dseparation(seed):
    rng = np.random.default_rng(10_000 + seed)
    n = int(rng.integers(3, 8))
    sem = semgen.random_dag(n, float(rng.uniform(0.2, 0.7)), rng)
    C = dsep.population_corr(sem)
    sk = oracle.skeleton_corr(C, 1e20, 0.01)
    truth = sem.skeleton()
    assert np.array_equal(sk.G.astype(bool), truth)
    pa = dsep.parents_of(sem)
    for (i, j), (l, S) in sk.sepsets.as_dict().items():
        assert len(S) == l and i < j
        assert dsep.d_separated(pa, i, j, S)
    # Every removed pair is d-separated by some set; every kept pair by none.
    for i, j in itertools.combinations(range(n), 2):
        others = [k for k in range(n) if k not in (i, j)]
        sep_exists = any(dsep.d_separated(pa, i, j, S)
                         for r in range(len(others) + 1) for S in itertools.combinations(others, r))
        assert sep_exists == (not truth[i, j])


# ------------------------------------------------------------------------------------------
# Structural invariants on sampled data
# ------------------------------------------------------------------------------------------
def _small_data(seed, n=14, p=0.35, m=300):
    rng = np.random.default_rng(seed)
    sem = semgen.random_dag(n, p, rng)
    return semgen.sample(sem, m, rng)


@pytest.mark.parametrize("seed", range(6))
def test_each_level_matches_independent_restatement(seed):
    """Per level: an edge is removed iff the numpy re-statement finds a separating S of size l in
    either direction over G' (maximality and soundness), and the stored SepSet is the first one in
    canonical order (direction i first, then lexicographic subsets)."""
    X = _small_data(seed)
    m, n = X.shape
    alpha = 0.05
    C = oracle.corr(X)
    sk = oracle.skeleton_corr(C, m, alpha, keep_levels=True)
    seps = sk.sepsets.as_dict()
    for l in range(1, sk.levels_run):
        Gp, G = sk.G_after[l - 1], sk.G_after[l]
        for i, j in itertools.combinations(range(n), 2):
            if not Gp[i, j]:
                continue
            S, gap = levelcheck.first_separating(C, Gp, i, j, l, m, alpha)
            if gap < 1e-9:
                continue          # decision within FP64 rounding of the threshold: not compared
            assert (S is not None) == (G[i, j] == 0), (l, i, j)
            if S is not None:
                assert seps[(i, j)] == (l, S)
    # The loop stops exactly when no node has enough neighbours (or after the last level).
    last = sk.G_after[-1]
    assert last.sum(1).max() - 1 < sk.levels_run


@pytest.mark.parametrize("seed", range(4))
def test_permutation_invariance(seed):
    """PC-stable is order independent (Sec. 2.4): relabelling the variables relabels G after every
    level."""
    X = _small_data(100 + seed, n=16)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(X.shape[1])
    a = oracle.skeleton(X, 0.05, keep_levels=True)
    b = oracle.skeleton(X[:, perm], 0.05, keep_levels=True)
    assert a.levels_run == b.levels_run
    for Ga, Gb in zip(a.G_after, b.G_after):
        assert np.array_equal(Ga[np.ix_(perm, perm)], Gb)


def test_sepsets_pass_their_test():
    X, sem, alpha = semgen.workload("n50_p005_m1000_fp64")
    C = oracle.corr(X)
    sk = oracle.skeleton_corr(C, X.shape[0], alpha, keep_levels=True)
    for (i, j), (l, S) in sk.sepsets.as_dict().items():
        Gp = sk.G_after[l - 1]
        assert all(Gp[i, s] for s in S) or all(Gp[j, s] for s in S)
        assert oracle.ci_test(C, i, j, list(S), X.shape[0], alpha)[0]
        rho_np = levelcheck.pcor_block(C, i, j, S)
        assert levelcheck.zstat(rho_np) <= levelcheck.tau(alpha, X.shape[0], l) + 1e-12


def test_max_level_cap_and_sample_limit():
    X = _small_data(3, n=12, p=0.5, m=300)
    full = oracle.skeleton(X, 0.05)
    cap = oracle.skeleton(X, 0.05, max_level=1)
    assert cap.levels_run == 2 and full.levels_run >= 2
    assert np.all(cap.G >= full.G)
    # m - l - 3 <= 0 stops with the warning status
    Xs = _small_data(3, n=8, p=0.9, m=6)
    sk = oracle.skeleton(Xs, 0.5)
    assert sk.levels_run <= 3
    if sk.status == oracle.OC_WARN_SAMPLE_LIMIT:
        assert sk.levels_run == 3


def test_threads_give_identical_results():
    """Edges of a level are decided from G' alone (Sec. 2.4), so deciding them on several threads
    must leave the skeleton, the canonical SepSets and the per-level test counts unchanged."""
    X, _, alpha = semgen.workload("n1000_d4_m500_fp32")
    try:
        oracle.set_threads(1)
        a = oracle.skeleton(X, alpha, keep_levels=True)
        oracle.set_threads(4)
        b = oracle.skeleton(X, alpha, keep_levels=True)
    finally:
        oracle.set_threads(1)
    assert np.array_equal(a.G, b.G)
    assert a.tests == b.tests and a.removed == b.removed
    assert a.sepsets.as_dict() == b.sepsets.as_dict()
    assert all(np.array_equal(x, y) for x, y in zip(a.G_after, b.G_after))


def test_dense_sampler_draws_the_same_sem_as_the_sequential_one():
    """semgen.sample_dense (one triangular solve) and semgen.sample (variable by variable in
    topological order) give the same samples from the same noise, up to rounding; the scalability
    grid covers the paper's points (Sec. 5.6)."""
    rng = np.random.default_rng(12)
    sem = semgen.random_dag(80, 0.3, rng, signed=False)
    a = semgen.sample(sem, 400, np.random.default_rng(3))
    b = semgen.sample_dense(sem, 400, np.random.default_rng(3))
    assert np.allclose(a, b, rtol=1e-11, atol=1e-11)
    sem = semgen.random_dag(50, 0.2, rng)
    a = semgen.sample(sem, 300, np.random.default_rng(4))
    b = semgen.sample_dense(sem, 300, np.random.default_rng(4))
    assert np.allclose(a, b, rtol=1e-11, atol=1e-11)
    grid = set(semgen.SCALABILITY_GRID)
    assert {(n, 0.1, 10000) for n in (1000, 2000, 3000, 4000)} <= grid
    assert {(1000, 0.1, m) for m in (2000, 4000, 6000, 8000, 10000)} <= grid
    assert {(1000, d, 10000) for d in (0.1, 0.2, 0.3, 0.4, 0.5)} <= grid


def test_correlation_is_scale_invariant_up_to_extreme_scales():
    """Pearson's r does not depend on the scale of either column. Columns scaled by 10^-100 ..
    10^100 (the dense SEMs of the paper's scalability grid reach standard deviations of 1e100)
    give the correlation of the unscaled data, which numpy's corrcoef fixes; a product of the two
    sums of squares would overflow there."""
    rng = np.random.default_rng(21)
    X = rng.standard_normal((300, 6))
    X[:, 1] += 0.8 * X[:, 0]
    X[:, 2] = X[:, 1] - 0.3 * X[:, 3]
    scales = 10.0 ** np.array([100.0, 90.0, -100.0, 0.0, 75.0, -80.0])
    C = oracle.corr(X * scales)
    assert np.allclose(C, np.corrcoef(X, rowvar=False), rtol=0, atol=1e-13)
    assert abs(C[0, 1]) > 0.5
