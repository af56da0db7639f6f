"""Writes the stored oracle results of the two largest workloads, which the CPU oracle cannot
recompute inside a GPU test run in reasonable time:

  n8000_d6_m2000_levels3.npz   n = 8000, expected degree 6, m = 2000, alpha 0.05, levels 0-3
  n2000_d10_m1000.npz          n = 2000, expected degree 10, m = 1000, alpha 0.01, whole skeleton

Each file holds the SHA-256 of the generated input (so a test can tell that its input is the one
the values were computed from), the oracle's per-level test and removal counts, and the edge list
(i < j, uint16 pairs) of G after every level >= 1, all from oracle/ alone (FP64 Pearson C, then
Algorithm 1 in canonical order).

    python tests/golden/make_oracle_skeletons.py [--threads K]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import semgen  # noqa: E402

SPECS = {
    "n8000_d6_m2000_levels3": ("n8000_d6_m2000_bf16x3", 3),
    "n2000_d10_m1000": ("n2000_d10_m1000_apply", -1),
}


def input_digest(X: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(X, dtype=np.float64).tobytes()).hexdigest()


def edges_of(G: np.ndarray) -> np.ndarray:
    i, j = np.nonzero(np.triu(G, 1))
    return np.stack([i, j], 1).astype(np.uint16)


def make(name: str, threads: int) -> str:
    workload, max_level = SPECS[name]
    X, _, alpha = semgen.workload(workload)
    m, n = X.shape
    oracle.set_threads(threads)
    sk = oracle.skeleton(X, alpha, max_level=max_level, keep_levels=True)
    L = sk.levels_run
    out = {"digest": np.array(input_digest(X)), "workload": np.array(workload), "alpha": np.array(alpha),
           "max_level": np.array(max_level), "tests": np.array(sk.tests[:L], np.int64),
           "removed": np.array(sk.removed[:L], np.int64)}
    for l in range(1, L):
        out[f"edges_after_{l}"] = edges_of(sk.G_after[l])
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, **out)
    return path


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("names", nargs="*", default=list(SPECS))
    a = ap.parse_args()
    for name in a.names:
        print("wrote", make(name, a.threads), flush=True)


if __name__ == "__main__":
    main()
