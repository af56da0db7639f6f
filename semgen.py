"""Seeded synthetic inputs: random DAGs and linear-Gaussian SEM samples.

This module only draws random inputs. It holds none of the PC-stable arithmetic (no correlation, no
CI test), so that both the CPU oracle and the HIP library can be fed from it without sharing code.

Generator (the family of the paper's own synthetic workloads, Sec. 5.6, with signed weights):
  * a uniformly random topological order pi over n variables;
  * for every pair a < b in pi order, an edge pi[a] -> pi[b] with probability p;
  * edge weights: sign +-1 with probability 1/2 each, magnitude U[0.1, 1];
  * X_v = sum_{u in pa(v)} w_uv X_u + N(0, 1), drawn in topological order, m i.i.d. rows.
An "expected degree" d is read as edge probability p = d / (n - 1).

All draws come from numpy's PCG64 (``numpy.random.default_rng(seed)``); a workload's seed is
1000 * config + instance.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class SEM:
    n: int
    order: np.ndarray        # topological order pi (int64, length n)
    parents: list            # parents[v] -> int64 array of parent ids of v
    weights: list            # weights[v] -> float64 array, same length as parents[v]

    def edges(self):
        """Directed edges (u, v, w) of the DAG."""
        out = []
        for v in range(self.n):
            for u, w in zip(self.parents[v], self.weights[v]):
                out.append((int(u), int(v), float(w)))
        return out

    def skeleton(self) -> np.ndarray:
        """Symmetric boolean n x n adjacency of the true DAG's skeleton."""
        A = np.zeros((self.n, self.n), dtype=bool)
        for v in range(self.n):
            A[self.parents[v], v] = True
            A[v, self.parents[v]] = True
        return A

    def weight_matrix(self) -> np.ndarray:
        """B with B[u, v] = weight of u -> v (zero where there is no edge)."""
        B = np.zeros((self.n, self.n))
        for v in range(self.n):
            B[self.parents[v], v] = self.weights[v]
        return B


def random_dag(n: int, p: float, rng: np.random.Generator,
               wmin: float = 0.1, wmax: float = 1.0, signed: bool = True) -> SEM:
    """Erdos-Renyi DAG over a random topological order, with random edge weights."""
    order = rng.permutation(n).astype(np.int64)
    parents, weights = [None] * n, [None] * n
    for b in range(n):
        v = int(order[b])
        if b == 0 or p <= 0.0:
            pa = np.zeros(0, dtype=np.int64)
        else:
            pa = order[:b][rng.random(b) < p]
        mag = rng.uniform(wmin, wmax, size=pa.size)
        if signed:
            sign = np.where(rng.random(pa.size) < 0.5, -1.0, 1.0)
            w = sign * mag
        else:
            w = mag
        parents[v], weights[v] = pa, w
    return SEM(n=n, order=order, parents=parents, weights=weights)


def sample(sem: SEM, m: int, rng: np.random.Generator) -> np.ndarray:
    """m x n float64 samples (row-major: sample r, variable a) drawn in topological order."""
    X = np.empty((m, sem.n), dtype=np.float64)
    noise = rng.standard_normal((sem.n, m))
    for b in range(sem.n):
        v = int(sem.order[b])
        col = noise[b].copy()
        pa = sem.parents[v]
        if pa.size:
            col += X[:, pa] @ sem.weights[v]
        X[:, v] = col
    return X


def sample_dense(sem: SEM, m: int, rng: np.random.Generator) -> np.ndarray:
    """The law of sample() for dense DAGs: with x in topological order, x = B^T x + e, so x solves
    the unit lower-triangular system (I - B^T) x = e for all m samples at once (one BLAS-3 solve
    instead of n gathers of parent columns). Same noise draws as sample(); the values agree with
    it up to rounding."""
    from scipy.linalg import solve_triangular

    n = sem.n
    pos = np.empty(n, dtype=np.int64)
    pos[sem.order] = np.arange(n)
    Lm = np.eye(n)
    for v in range(n):
        pa = sem.parents[v]
        if pa.size:
            Lm[pos[v], pos[pa]] = -sem.weights[v]
    noise = rng.standard_normal((n, m))
    Y = solve_triangular(Lm, noise, lower=True, unit_diagonal=True, check_finite=False)
    X = np.empty((m, n), dtype=np.float64)
    X[:, sem.order] = Y.T
    return X


def expected_degree_p(n: int, d: float) -> float:
    return min(1.0, d / max(1, n - 1))


# ---------------------------------------------------------------------------------------------
# Named workloads. Shapes follow the five workloads this project measures; the values are drawn
# here, never stored.
# ---------------------------------------------------------------------------------------------
WORKLOADS = {
    # name: (config id, n, p or None, expected degree or None, m, alpha)
    "n50_p005_m1000_fp64": (1, 50, 0.05, None, 1000, 0.01),
    "n1000_d4_m500_fp32": (2, 1000, None, 4.0, 500, 0.01),
    "n8000_d6_m2000_bf16x3": (3, 8000, None, 6.0, 2000, 0.05),
    "n2000_d10_m1000_apply": (5, 2000, None, 10.0, 1000, 0.01),
}


def workload(name: str, instance: int = 0):
    """Returns (X, sem, alpha) for a named workload."""
    cfg, n, p, d, m, alpha = WORKLOADS[name]
    rng = np.random.default_rng(1000 * cfg + instance)
    if p is None:
        p = expected_degree_p(n, d)
    sem = random_dag(n, p, rng)
    X = sample(sem, m, rng)
    return X, sem, alpha


def scalability(n: int = 1000, p: float = 0.1, m: int = 10000, instance: int = 0):
    """The paper's own scalability family (Sec. 5.6): every ordered pair gets an edge with
    probability p (a dense graph: about p (n - 1) / 2 parents per node), positive weights U[0.1, 1],
    unit-variance Gaussian noise, m samples. Returns (X, sem, alpha = 0.01)."""
    rng = np.random.default_rng(1000 * 6 + 10 * int(round(p * 100)) + instance)
    sem = random_dag(n, p, rng, signed=False)
    return sample_dense(sem, m, rng), sem, 0.01


# The paper's scalability grid (Sec. 5.6, Fig. 10): n at d = 0.1 and m = 10000; m at n = 1000 and
# d = 0.1; d at n = 1000 and m = 10000. Each entry is (n, p, m).
SCALABILITY_GRID = (
    [(n, 0.1, 10000) for n in (1000, 2000, 3000, 4000)]
    + [(1000, 0.1, m) for m in (2000, 4000, 6000, 8000)]
    + [(1000, p, 10000) for p in (0.2, 0.3, 0.4, 0.5)])


def batch_problems(count: int = 256, instance: int = 0, nmin: int = 20, nmax: int = 400,
                   dmin: float = 2.0, dmax: float = 8.0, mmin: int = 200, mmax: int = 5000):
    """Uneven batch of independent datasets: n ~ U[20,400], degree ~ U[2,8], m ~ U[200,5000]."""
    rng = np.random.default_rng(1000 * 4 + instance)
    probs = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        d = float(rng.uniform(dmin, dmax))
        m = int(rng.integers(mmin, mmax + 1))
        sem = random_dag(n, expected_degree_p(n, d), rng)
        X = sample(sem, m, rng)
        probs.append((X, sem, 0.01))
    return probs


def training_sems(count: int, instance: int = 0, n: int = 200, m: int = 1000,
                  dmin: float = 2.0, dmax: float = 10.0):
    """Training SEMs for the learned ordering: n = 200, degree ~ U[2,10], m = 1000."""
    rng = np.random.default_rng(1000 * 5 + 100 + instance)
    for _ in range(count):
        d = float(rng.uniform(dmin, dmax))
        sem = random_dag(n, expected_degree_p(n, d), rng)
        X = sample(sem, m, rng)
        yield X, sem, 0.01
