"""Orientation of the PC skeleton into a CPDAG: plain CPU reference.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): the product path never imports it.

The skeleton step the paper accelerates is followed, in the PC algorithm, by the orientation step
(Sec. 2.4 names it and leaves it on the CPU): unshielded colliders from the SepSets, then the
rules that propagate orientations (Meek, 1995). Written here with the conventions the library
uses, so the two can be compared bit for bit on the same skeleton and SepSets:

* V-structures. For every unshielded triple i - k - j (i, j not adjacent), k not in SepSet(i, j)
  puts an arrowhead at k on both edges. All triples are judged against the skeleton and SepSets
  alone, so the order of the triples does not matter. An edge that receives arrowheads at both
  ends is bidirected (a conflict between v-structures) and stays so.
* Propagation, in synchronous rounds until nothing changes. In each round every undirected edge
  x - y is tested against the orientation state at the start of the round; x -> y is proposed by
    R1: some a -> x with a, y not adjacent;
    R2: some a with x -> a -> y;
    R3: two non-adjacent c, d with x - c, x - d undirected and c -> y, d -> y.
  Proposals are applied together at the end of the round; an edge proposed in both directions in
  the same round is left undirected. Bidirected edges count neither as directed nor undirected.
  (Meek's fourth rule is not needed without background knowledge.)

Output: a boolean n x n matrix H with H[x, y] true iff the edge x - y has an arrowhead at y.
"""
from __future__ import annotations

import itertools

import numpy as np


def v_structures(G: np.ndarray, sepset) -> np.ndarray:
    """Arrowheads of the unshielded colliders. G: symmetric boolean adjacency (the skeleton);
    sepset(i, j) -> the separating set of the non-adjacent pair (i < j) as a collection of ids."""
    n = G.shape[0]
    H = np.zeros((n, n), dtype=bool)
    for k in range(n):
        nb = np.flatnonzero(G[k])
        for a, b in itertools.combinations(nb, 2):
            i, j = (a, b) if a < b else (b, a)
            if G[i, j]:
                continue
            if k not in set(sepset(i, j)):
                H[i, k] = True
                H[j, k] = True
    return H


def _state(G, H):
    # directed a -> b: arrowhead at b only; undirected: no arrowhead at either end
    dirc = G & H & ~H.T
    und = G & ~H & ~H.T
    return dirc, und


def meek_round(G: np.ndarray, H: np.ndarray) -> np.ndarray:
    """Proposals x -> y of one synchronous round (boolean matrix P, P[x, y] = propose x -> y)."""
    n = G.shape[0]
    dirc, und = _state(G, H)
    P = np.zeros((n, n), dtype=bool)
    for x in range(n):
        for y in np.flatnonzero(und[x]):
            # R1: some a -> x with a, y not adjacent (a != y)
            a1 = dirc[:, x] & ~G[:, y]
            a1[y] = False
            # R2: some a with x -> a -> y
            a2 = dirc[x, :] & dirc[:, y]
            # R3: two non-adjacent c, d among {c : x - c undirected, c -> y}
            cs = np.flatnonzero(und[x, :] & dirc[:, y])
            r3 = any(not G[c, d] for c, d in itertools.combinations(cs, 2))
            if a1.any() or a2.any() or r3:
                P[x, y] = True
    return P


def orient(G: np.ndarray, sepset, max_rounds: int = 10_000):
    """(H, rounds): the arrowhead matrix of the CPDAG and the number of propagation rounds that
    changed something."""
    G = np.asarray(G, dtype=bool)
    H = v_structures(G, sepset)
    rounds = 0
    for _ in range(max_rounds):
        P = meek_round(G, H)
        take = P & ~P.T
        if not take.any():
            break
        H = H | take
        rounds += 1
    return H, rounds


def sepset_lookup(records: dict):
    """sepset(i, j) for a dict {(i, j): (level, S)} of level >= 1 removals; pairs absent from it
    were removed at level 0 and have the empty set."""
    def f(i, j):
        r = records.get((i, j))
        return () if r is None else tuple(r[1])
    return f


# ---- independent definitions used to pin the above (brute force on tiny graphs) ---------------

def dag_v_structures(A: np.ndarray) -> set:
    """Unshielded colliders (i, k, j), i < j, of a DAG with adjacency A[u, v] = u -> v."""
    n = A.shape[0]
    out = set()
    for k in range(n):
        pa = np.flatnonzero(A[:, k])
        for i, j in itertools.combinations(sorted(pa), 2):
            if not A[i, j] and not A[j, i]:
                out.add((i, j, k))
    return out


def _acyclic(A: np.ndarray) -> bool:
    n = A.shape[0]
    indeg = A.sum(0).astype(int)
    stack = [v for v in range(n) if indeg[v] == 0]
    seen = 0
    while stack:
        v = stack.pop()
        seen += 1
        for w in np.flatnonzero(A[v]):
            indeg[w] -= 1
            if indeg[w] == 0:
                stack.append(w)
    return seen == n


def cpdag_brute_force(A: np.ndarray) -> np.ndarray:
    """CPDAG of a DAG by enumerating its Markov equivalence class (Verma and Pearl: same skeleton
    and same unshielded colliders): an edge is directed iff every member orients it the same way.
    Returns the arrowhead matrix H as in orient(). Only for tiny graphs."""
    A = np.asarray(A, dtype=bool)
    n = A.shape[0]
    skel = A | A.T
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if skel[u, v]]
    target = dag_v_structures(A)
    members = []
    for bits in itertools.product((0, 1), repeat=len(edges)):
        B = np.zeros((n, n), dtype=bool)
        for (u, v), b in zip(edges, bits):
            if b:
                B[u, v] = True
            else:
                B[v, u] = True
        if _acyclic(B) and dag_v_structures(B) == target:
            members.append(B)
    H = np.zeros((n, n), dtype=bool)
    for u, v in edges:
        fwd = all(B[u, v] for B in members)
        bwd = all(B[v, u] for B in members)
        if fwd:
            H[u, v] = True
        elif bwd:
            H[v, u] = True
    return H
