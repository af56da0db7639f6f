"""How often a conditioning set repeats across rows of G' (the local vs global sharing question).

The set-sharing kernel factors M2 = C[S,S] once per (row i, set S) and reuses it for every j of the
row. Sharing it across rows as well would need a search of the whole graph for the rows that hold
S; the paper (Sec. 5.5, global against local sharing) measures, at level 2, in how many rows of
A'_G each set appears and finds the counts small. This module measures the same histogram on
G' of a given level, from the library's own skeleton run up to the level before it:

    python -m paper_1812_08491_amd.redundancy [--workload n2000_d10_m1000_apply] [--level 2]

Output: one JSON line with the number of (row, set) factors the local scheme computes, the number
of distinct sets (what a global scheme would compute), and the histogram of rows per set.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

BINS = [1, 2, 3, 5, 10, 20, 40, 80, 160, 10 ** 9]


def set_histogram(G: np.ndarray, level: int) -> dict:
    """Rows per l-subset S over the rows i of G (boolean adjacency) with degree >= l + 1 (the rows
    that test S at level l)."""
    from itertools import combinations
    n = G.shape[0]
    keys = []
    factors = 0
    for i in range(n):
        nb = np.flatnonzero(G[i])
        if nb.size < level + 1:
            continue
        factors += math.comb(nb.size, level)
        if level == 2:
            a, b = np.triu_indices(nb.size, 1)
            keys.append(nb[a].astype(np.int64) * n + nb[b])
        else:
            keys.append(np.array([sum(int(v) * n ** k for k, v in enumerate(S)) for S in combinations(nb, level)],
                                 dtype=np.int64))
    if not keys:
        return {"factors": 0, "distinct_sets": 0, "histogram": {}}
    _, counts = np.unique(np.concatenate(keys), return_counts=True)
    hist = {}
    for lo, hi in zip(BINS[:-1], BINS[1:]):
        sel = (counts >= lo) & (counts < hi)
        hist[f"[{lo},{hi})" if hi < 10 ** 9 else f">={lo}"] = {"sets": int(sel.sum()),
                                                                "factors": int(counts[sel].sum())}
    return {"factors": int(factors), "distinct_sets": int(counts.size),
            "global_saving": 1.0 - counts.size / max(factors, 1),
            "max_rows_per_set": int(counts.max()), "histogram": hist}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="n2000_d10_m1000_apply")
    ap.add_argument("--level", type=int, default=2)
    args = ap.parse_args(argv)
    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import semgen
    from . import _lib as pc

    X, _, alpha = semgen.workload(args.workload)
    m, n = X.shape
    ctx = pc.Context(precision="fp32")
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    # G after level l - 1 is the snapshot G' of level l
    ctx.pc_skeleton(torch.from_numpy(np.ascontiguousarray(X)).cuda(), alpha, adj, recs, count, ws,
                    max_level=args.level - 1)
    G = pc.bits_to_dense(adj.cpu().numpy(), n).astype(bool)
    out = {"workload": args.workload, "level": args.level, "n": n}
    out.update(set_histogram(G, args.level))
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
