"""Pins of the orientation reference (oracle/orient.py) on the CPU.

Hand-made cases for each rule, and, in the large-sample limit, the CPDAG the PC skeleton leads to
against the CPDAG defined by brute force: every DAG with the true skeleton and the true unshielded
colliders (the Markov equivalence class), an edge directed iff all of them agree on it.
"""
import numpy as np
import pytest

import oracle
import semgen
from oracle import orient
from tests.ref import dsep


def _G(n, edges):
    G = np.zeros((n, n), dtype=bool)
    for a, b in edges:
        G[a, b] = G[b, a] = True
    return G


def _arrows(H):
    return {(int(a), int(b)) for a, b in zip(*np.nonzero(H))}


def test_collider_and_non_colliders():
    # 0 - 2 - 1, 0 and 1 separated by {}: collider at 2
    H, _ = orient.orient(_G(3, [(0, 2), (1, 2)]), lambda i, j: ())
    assert _arrows(H) == {(0, 2), (1, 2)}
    # the same skeleton separated by {2} (chain or fork): nothing is oriented
    H, r = orient.orient(_G(3, [(0, 2), (1, 2)]), lambda i, j: (2,))
    assert _arrows(H) == set() and r == 0


def test_rule1_propagates_away_from_a_collider():
    # 0 -> 2 <- 1, 2 - 3 with 3 separated from 0 and 1 by {2}: R1 gives 2 -> 3
    seps = {(0, 1): (), (0, 3): (2,), (1, 3): (2,)}
    H, r = orient.orient(_G(4, [(0, 2), (1, 2), (2, 3)]), lambda i, j: seps[(i, j)])
    assert _arrows(H) == {(0, 2), (1, 2), (2, 3)} and r == 1


def test_rule2_avoids_a_cycle():
    # 0 -> 2 <- 1 (collider), 2 -> 3 (R1 from 0), and 0 - 3: R2 orients 0 -> 3 in the next round
    seps = {(0, 1): (), (1, 3): (2,)}
    H, r = orient.orient(_G(4, [(0, 2), (1, 2), (2, 3), (0, 3)]), lambda i, j: seps[(i, j)])
    assert (2, 3) in _arrows(H) and (0, 3) in _arrows(H) and (3, 0) not in _arrows(H)
    assert r == 2


def test_rule3():
    # c=1 -> b=0 <- d=2 (collider), a=3 adjacent to all three, a - c and a - d undirected:
    # R3 orients a -> b
    seps = {(1, 2): (3,)}
    G = _G(4, [(1, 0), (2, 0), (3, 0), (3, 1), (3, 2)])
    H, _ = orient.orient(G, lambda i, j: seps[(i, j)])
    assert _arrows(H) == {(1, 0), (2, 0), (3, 0)}


def test_conflicting_colliders_make_a_bidirected_edge():
    # 0 - 1 - 2 - 3 with {} separating (0, 2) and (1, 3): colliders at 1 and at 2 put arrowheads
    # at both ends of 1 - 2, which stays bidirected and does not propagate
    seps = {(0, 2): (), (1, 3): (), (0, 3): ()}
    H, _ = orient.orient(_G(4, [(0, 1), (1, 2), (2, 3)]), lambda i, j: seps[(i, j)])
    assert _arrows(H) == {(0, 1), (2, 1), (1, 2), (3, 2)}


def _dag_matrix(sem):
    A = np.zeros((sem.n, sem.n), dtype=bool)
    for v in range(sem.n):
        for p in sem.parents[v]:
            A[int(p), v] = True
    return A


@pytest.mark.parametrize("seed", range(30))
def test_large_sample_limit_equals_equivalence_class_cpdag(seed):
    rng = np.random.default_rng(20_000 + seed)
    n = int(rng.integers(3, 7))
    sem = semgen.random_dag(n, float(rng.uniform(0.3, 0.8)), rng)
    C = dsep.population_corr(sem)
    sk = oracle.skeleton_corr(C, 1e20, 0.01)
    H, _ = orient.orient(sk.G.astype(bool), orient.sepset_lookup(sk.sepsets.as_dict()))
    assert np.array_equal(H, orient.cpdag_brute_force(_dag_matrix(sem)))


def test_orientation_does_not_depend_on_variable_order():
    rng = np.random.default_rng(7)
    sem = semgen.random_dag(12, 0.3, rng)
    X = semgen.sample(sem, 400, rng)
    sk = oracle.skeleton(X, 0.05)
    H, _ = orient.orient(sk.G.astype(bool), orient.sepset_lookup(sk.sepsets.as_dict()))
    perm = rng.permutation(12)
    inv = np.argsort(perm)
    G2 = sk.G.astype(bool)[np.ix_(perm, perm)]
    seps = {}
    for (i, j), (l, S) in sk.sepsets.as_dict().items():
        a, b = sorted((int(inv[i]), int(inv[j])))
        seps[(a, b)] = (l, tuple(int(inv[s]) for s in S))
    H2, _ = orient.orient(G2, orient.sepset_lookup(seps))
    assert np.array_equal(H2, H[np.ix_(perm, perm)])
