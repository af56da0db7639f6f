"""The rows-per-set histogram of paper_1812_08491_amd.redundancy against direct enumeration (CPU)."""
import itertools

import numpy as np

from paper_1812_08491_amd.redundancy import set_histogram


def _direct(G, level):
    n = G.shape[0]
    rows = {}
    for i in range(n):
        nb = np.flatnonzero(G[i])
        if nb.size < level + 1:
            continue
        for S in itertools.combinations(nb.tolist(), level):
            rows[S] = rows.get(S, 0) + 1
    return rows


def test_complete_graph_k4_level2():
    G = ~np.eye(4, dtype=bool)
    h = set_histogram(G, 2)
    # every pair is a set of the two rows outside it
    assert h["factors"] == 12 and h["distinct_sets"] == 6 and abs(h["global_saving"] - 0.5) < 1e-12
    assert h["histogram"]["[2,3)"] == {"sets": 6, "factors": 12}


def test_random_graphs_match_enumeration():
    rng = np.random.default_rng(3)
    for level in (2, 3):
        for _ in range(5):
            n = int(rng.integers(5, 40))
            U = np.triu(rng.random((n, n)) < rng.uniform(0.1, 0.5), 1)
            G = U | U.T
            h = set_histogram(G, level)
            rows = _direct(G, level)
            assert h["distinct_sets"] == len(rows)
            assert h["factors"] == sum(rows.values())
            counts = np.array(list(rows.values())) if rows else np.zeros(0, int)
            for key, v in h["histogram"].items():
                lo, hi = (int(key[2:]), 10 ** 9) if key.startswith(">=") else map(int, key[1:-1].split(","))
                sel = (counts >= lo) & (counts < hi)
                assert v == {"sets": int(sel.sum()), "factors": int(counts[sel].sum())}
