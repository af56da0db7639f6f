"""Brute-force d-separation on small DAGs (moralised ancestral graph criterion).

X and Y are d-separated by Z in a DAG iff they are disconnected in the moral graph of the ancestral
set of {X, Y} u Z once Z is deleted (Lauritzen et al., 1990). Independent of the oracle.
"""
import itertools

import numpy as np


def ancestors(parents, nodes):
    out, stack = set(nodes), list(nodes)
    while stack:
        v = stack.pop()
        for u in parents[v]:
            if u not in out:
                out.add(u)
                stack.append(u)
    return out


def d_separated(parents, x, y, Z):
    Z = set(Z)
    anc = ancestors(parents, {x, y} | Z)
    adj = {v: set() for v in anc}
    for v in anc:
        pa = [u for u in parents[v] if u in anc]
        for u in pa:
            adj[u].add(v)
            adj[v].add(u)
        for a, b in itertools.combinations(pa, 2):   # marry parents
            adj[a].add(b)
            adj[b].add(a)
    seen, stack = {x}, [x]
    while stack:
        v = stack.pop()
        if v == y:
            return False
        for w in adj[v]:
            if w not in seen and w not in Z:
                seen.add(w)
                stack.append(w)
    return True


def parents_of(sem):
    return [list(int(u) for u in sem.parents[v]) for v in range(sem.n)]


def population_corr(sem):
    """Population correlation of a linear-Gaussian SEM with unit noise variances."""
    B = sem.weight_matrix()
    A = np.linalg.inv(np.eye(sem.n) - B)      # row vectors: X = N (I - B)^-1
    Sigma = A.T @ A
    d = np.sqrt(np.diag(Sigma))
    return Sigma / np.outer(d, d)
