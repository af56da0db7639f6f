"""Benchmark: PC-stable skeleton on one MI355X through the C ABI.

One step = one whole skeleton (standardize, correlation GEMM with the level-0 test, then every
level until the stop rule, FP64 re-checks included) of a synthetic linear-Gaussian SEM dataset that
is already resident in HBM: n = 1000 variables, expected degree 4, m = 500 samples, alpha = 0.01,
FP32 CI tests with FP64 re-checks of borderline tests. The skeleton is captured once as a hipGraph
(pc_batch_capture) and each step is one replay; `ms_per_step` is the replay time. The graph records
the levels with many tests (those above TAIL_TESTS in an untimed pc_skeleton run on the same data)
as level kernels, and the small levels after them as the tail kernel (one work-group per problem);
the run asserts that no replay needed the stream continuation of pc_graph_results.

`value` is CI tests per second: the tests the sequential PC-stable enumeration performs on this
input (canonical order, early stop per edge; counted by the CPU oracle in the cpu_baseline leg, on
the same input) divided by the time per step. The tests the GPU evaluated are reported beside it.

Also reported: the same skeleton through pc_skeleton on the stream (with HIP events around the
kernels, which give the roofline of the dominant kernel), plain vs learned conditioning-set order
on n = 2000 (expected degree 10, m = 1000, identical skeleton required), and a captured batch of
256 uneven datasets.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--copy-calibration MiB]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "n1000_d4_m500_fp32"
APPLY_WORKLOAD = "n2000_d10_m1000_apply"
PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix
PEAK_HBM_GBS = 8000.0             # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_level1_n1000_d4_m500.json")
ROW_TOP = 2   # candidates per node the learned order tests first at level 1
TAIL_TESTS = 2048     # levels with more CI tests than this run as level kernels in the graph
TAIL_MAX_LEVEL = 8    # deepest level the tail kernel runs
LEVEL_SOURCES = ["paper_1812_08491_amd/csrc/pc_level.h", "paper_1812_08491_amd/csrc/pc_level_f32.hip",
                 "paper_1812_08491_amd/csrc/pc_citest.h", "paper_1812_08491_amd/csrc/pc_dev.h",
                 "paper_1812_08491_amd/csrc/pc_comb.h"]


def level_source_hash() -> str:
    h = hashlib.sha256()
    for p in LEVEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of k_level<float,1> from the committed PMC summary, or None when the
    level kernel's sources changed after the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != level_source_hash():
        return None
    return float(t["bytes_per_launch"])


def cpu_baseline(X: np.ndarray, alpha: float, min_seconds: float = 10.0, max_reps: int = 30):
    """The FP64 oracle (single-threaded C, as it stands) on the same input, repeated until about
    min_seconds of CPU time; returns (oracle result, seconds per skeleton, runs)."""
    import oracle
    t0 = time.perf_counter()
    ref = oracle.skeleton(X, alpha)
    times = [time.perf_counter() - t0]
    while sum(times) < min_seconds and len(times) < max_reps:
        t0 = time.perf_counter()
        oracle.skeleton(X, alpha)
        times.append(time.perf_counter() - t0)
    return ref, float(np.mean(times)), len(times)


def copy_calibration(mib: int, reps: int = 5) -> None:
    """Device-to-device copies of a known size, for scaling the PMC byte counters."""
    import torch
    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": mib << 20, "reps": reps}))


def write_traffic(fetch_csv: str, write_csv: str, copy_fetch_csv: str, copy_write_csv: str,
                  copy_bytes: int) -> None:
    """Per-launch HBM bytes of k_level<float,1> from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads for a device copy of
    copy_bytes; written to the traffic summary with the hash of the level kernel's sources."""
    import csv

    def per_dispatch(path, kernel):
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if r["Kernel_Name"].startswith(kernel)]
        return float(np.mean(vals)), len(vals)

    fetch, nf = per_dispatch(fetch_csv, "void pcg::k_level<float, 1>")
    write, nw = per_dispatch(write_csv, "void pcg::k_level<float, 1>")
    cf, _ = per_dispatch(copy_fetch_csv, "__amd_rocclr_copyBuffer")
    cw, _ = per_dispatch(copy_write_csv, "__amd_rocclr_copyBuffer")
    f_fetch, f_write = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    out = {"kernel": "k_level<float,1>", "workload": "n=1000, degree 4, m=500, alpha 0.01, fp32",
           "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write, "dispatches": [nf, nw],
           "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": f_fetch, "write_scale": f_write,
           "bytes_per_launch": (fetch * f_fetch + write * f_write) * 1024.0,
           "source_hash": level_source_hash()}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the learned-order and batch legs")
    ap.add_argument("--graph-levels", type=int, default=0,
                    help="levels recorded as level kernels before the tail kernel (0: from TAIL_TESTS)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                         "COPY_WRITE_CSV"))
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, copy_bytes=256 << 20)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              f"multi-GPU path.", file=sys.stderr)
        return 2
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return 0

    import torch

    import paper_1812_08491_amd as pc
    import semgen

    X, sem, alpha = semgen.workload(WORKLOAD)
    m, n = X.shape
    torch.cuda.set_device(0)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()

    # -- the skeleton through pc_skeleton on the stream, HIP events around every kernel phase -------
    stream = torch.cuda.current_stream()
    ctx = pc.Context(stream=stream, precision="fp32", timing=1 | 2 | 4 | 8 | 16)
    ws = ctx.workspace(n, m)
    adj = ctx.adjacency(n)
    recs, count = ctx.sepsets(n * (n - 1) // 2)
    st = pc.pc_run_stats()
    for _ in range(args.warmup):
        ctx.pc_skeleton(Xd, alpha, adj, recs, count, ws, stats=st)
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        status = ctx.pc_skeleton(Xd, alpha, adj, recs, count, ws, stats=st)
        runs.append(st.as_dict())
    torch.cuda.synchronize()
    stream_sec = (time.perf_counter() - t0) / args.steps
    assert status == 0, pc.status_str(status)
    L = runs[-1]["levels_run"]
    # Levels with many tests go to the level kernels, the rest to the tail kernel (levels <= 8).
    big = [l for l in range(1, L) if runs[-1]["tests"][l] > TAIL_TESTS]
    graph_levels = args.graph_levels or max([1] + big)
    if L - 1 > TAIL_MAX_LEVEL:
        graph_levels = max(graph_levels, L - 1)

    # -- timed region: graph replays of the whole skeleton ----------------------------------------
    gstream = torch.cuda.Stream()
    with torch.cuda.stream(gstream):
        # Levels 1 .. graph_levels as level kernels, then the tail kernel (with a budget that
        # covers any level here) up to level 8; a replay needing more would be continued by
        # pc_graph_results, which the check below rules out for the timed replays.
        gctx = pc.Context(stream=gstream, precision="fp32", graph_levels=graph_levels, tail_tests=1 << 30)
        gadj = gctx.adjacency(n)
        grecs, gcount = gctx.sepsets(n * (n - 1) // 2)
        probs = gctx.problems([(Xd, alpha, -1, gadj, grecs, gcount)])
        gws = gctx.batch_workspace(probs)
        graph = gctx.pc_batch_capture(probs, gws)
        for _ in range(args.warmup):
            graph.pc_graph_launch()
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(args.steps):
            graph.pc_graph_launch()
        torch.cuda.synchronize()
        sec_per_step = (time.perf_counter() - g0) / args.steps
        gst = (pc.pc_run_stats * 1)()
        r, gstatus = graph.pc_graph_results(gst)
        graph.close()
    assert r == 0 and gstatus[0] == 0, (r, gstatus)
    G = pc.bits_to_dense(gadj.cpu().numpy(), n)
    gstats = gst[0].as_dict()
    assert gstats["levels_run"] - 1 <= max(graph_levels, TAIL_MAX_LEVEL), "the recorded graph did not cover every level"

    gpu_tests = int(sum(gstats["tests"]))

    same_as_graph = bool(np.array_equal(pc.bits_to_dense(adj.cpu().numpy(), n), G))

    def mean_of(key, lvl=None):
        v = [d[key] if lvl is None else d[key][lvl] for d in runs]
        return float(np.mean(v))

    level_ms = [mean_of("level_ms", l) for l in range(L)]
    kernel_ms = {"prep": mean_of("prep_ms"), "corr_gemm_level0": mean_of("corr_ms"),
                 "compact_plan": [mean_of("compact_ms", l) for l in range(L)],
                 "level": level_ms, "recheck": [mean_of("recheck_ms", l) for l in range(L)]}

    out = {
        "metric": "CI tests/sec and skeleton wall time (PC-stable skeleton, identical to the FP64 oracle)",
        "value": None,
        "unit": "CI tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic linear-Gaussian SEM (seeded), resident in HBM",
        "config": {"workload": "pc_stable_skeleton_n1000_deg4_m500_alpha0.01_fp32_recheck",
                   "n": n, "m": m, "expected_degree": 4, "alpha": alpha, "precision": "fp32+fp64 recheck",
                   "step": "one hipGraph replay of the whole skeleton",
                   "graph_levels": graph_levels, "tail_from_level": graph_levels + 1,
                   "levels_run": gstats["levels_run"], "edges": int(G.sum()) // 2},
        "gpu_tests_per_step": gpu_tests,
        "gpu_executed_tests_per_s": gpu_tests / sec_per_step,
        "per_level_tests": gstats["tests"][:gstats["levels_run"]],
        "rechecks": gstats["rechecks"][:gstats["levels_run"]],
        "stream_ms_per_step": stream_sec * 1e3,
        "stream_same_skeleton": same_as_graph,
        "kernel_ms": kernel_ms,
    }

    # -- roofline of the dominant kernel: the level-1 CI tests (gather bound: per test C_ij and the
    #    entry C[j,S], 4 (l + 1) = 8 bytes at l = 1) --------------------------------------------------
    t1 = runs[-1]["tests"][1]
    l1_s = level_ms[1] * 1e-3
    ach = t1 * 8.0 / l1_s / 1e9
    traffic = measured_traffic()
    out["roofline"] = {"kernel": "k_level<float,1> (level-1 CI tests)", "bound": "hbm",
                       "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                       "traffic": traffic, "algorithmic_bytes": t1 * 8.0, "launch_ms": level_ms[1]}
    corr_s = kernel_ms["corr_gemm_level0"] * 1e-3
    fl = float(m) * n * (n - 1) / corr_s / 1e12
    out["roofline_corr"] = {"kernel": "k_corr<fp32> (SYRK + level-0 test)", "bound": "mfma", "achieved": fl,
                            "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": fl / PEAK_FP32_MFMA_TFLOPS,
                            "launch_ms": kernel_ms["corr_gemm_level0"]}

    if not args.no_extras:
        # -- plain vs learned conditioning-set order (same data, identical skeleton required) ------
        from paper_1812_08491_amd import learn
        Xa, _, alpha_a = semgen.workload(APPLY_WORKLOAD)
        # The shared-set (row) model orders level 1, where this workload's tests are: each node's
        # ROW_TOP best-scored candidates are tested first as sets {k}, then the rest.
        cmp = learn.compare_orders(Xa, alpha_a, None, row_params=learn.load_weights(learn.ROW_WEIGHTS),
                                   row_top=ROW_TOP, repeats=9)
        tp, tl = sum(cmp["plain"]["tests"]), sum(cmp["learned"]["tests"])
        out["learned_vs_plain"] = {
            "workload": "n2000_deg10_m1000_alpha0.01_fp32", "same_skeleton": cmp["same_skeleton"],
            "plain_ms": cmp["plain"]["wall_ms"], "learned_ms": cmp["learned"]["wall_ms"],
            "plain_tests": tp, "learned_tests": tl,
            "plain_tests_per_s": tp / (cmp["plain"]["wall_ms"] * 1e-3),
            "learned_tests_per_s": tl / (cmp["learned"]["wall_ms"] * 1e-3),
            "probe_tests": sum(cmp["learned"]["probe_tests"]),
            "probe_removed": sum(cmp["learned"]["probe_removed"]),
            "level1_tests": [cmp["plain"]["tests"][1], cmp["learned"]["tests"][1]],
            "order": {"form": "shared-set (row) model at level 1", "row_top": ROW_TOP,
                      "weights": "weights/order_row_mlp_n200.npy"}}
        # -- 256 uneven datasets in one captured graph --------------------------------------------
        batch = semgen.batch_problems(256)
        bstream = torch.cuda.Stream()
        with torch.cuda.stream(bstream):
            bctx = pc.Context(stream=bstream, precision="fp32")
            items = []
            for Xb, _, ab in batch:
                mb, nb = Xb.shape
                rb, cb = bctx.sepsets(nb * (nb - 1) // 2)
                items.append((torch.from_numpy(np.ascontiguousarray(Xb)).cuda(), ab, -1, bctx.adjacency(nb), rb, cb))
            bprobs = bctx.problems(items)
            bws = bctx.batch_workspace(bprobs)
            bgraph = bctx.pc_batch_capture(bprobs, bws)
            bst = (pc.pc_run_stats * len(items))()
            for _ in range(2):
                bgraph.pc_graph_launch()
                bgraph.pc_graph_results(bst)
            torch.cuda.synchronize()
            reps = max(3, args.steps // 5)
            b0 = time.perf_counter()
            for _ in range(reps):
                # a replay and its results: levels some datasets need beyond the recorded ones
                # run inside pc_graph_results, so both are timed
                bgraph.pc_graph_launch()
                br, bstatus = bgraph.pc_graph_results(bst)
            torch.cuda.synchronize()
            bms = (time.perf_counter() - b0) / reps * 1e3
            bgraph.close()
        out["batch256_graph"] = {"workload": "256 datasets, n~U[20,400], degree~U[2,8], m~U[200,5000], alpha 0.01",
                                 "ms_per_batch": bms, "status": br,
                                 "tests": int(sum(sum(s.as_dict()["tests"]) for s in bst))}
        # -- orientation of the bench skeleton into a CPDAG (pc_orient) ----------------------------
        nrec = int(gcount.item())
        arrows = gctx.adjacency(n)
        ows = gctx.orient_workspace(n)
        rounds = gctx.pc_orient(n, gadj, grecs, nrec, arrows, ows)
        torch.cuda.synchronize()
        o0 = time.perf_counter()
        oreps = 20
        for _ in range(oreps):
            gctx.pc_orient(n, gadj, grecs, nrec, arrows, ows)
        torch.cuda.synchronize()
        orient_ms = (time.perf_counter() - o0) / oreps * 1e3
        Hg = pc.bits_to_dense(arrows.cpu().numpy(), n).astype(bool)
        out["orientation"] = {"workload": "CPDAG of the bench skeleton (colliders + Meek R1-R3)",
                              "ms": orient_ms, "rounds": rounds,
                              "directed": int((Hg & ~Hg.T).sum()), "bidirected": int((Hg & Hg.T).sum()) // 2,
                              "undirected": int(G.sum()) // 2 - int((Hg & ~Hg.T).sum()) - int((Hg & Hg.T).sum()) // 2}

    if not args.no_extras:
        # -- the paper's scalability family: n = 1000, edge probability 0.1, m = 10000, FP64 --------
        Xs, _, alpha_s = semgen.scalability(1000, 0.1, 10000)
        ms_s, ns_s = Xs.shape
        sctx = pc.Context(precision="fp64")
        sws = sctx.workspace(ns_s, ms_s)
        sadj = sctx.adjacency(ns_s)
        srecs, scount = sctx.sepsets(ns_s * (ns_s - 1) // 2)
        Xsd = torch.from_numpy(np.ascontiguousarray(Xs)).cuda()
        walls = []
        for r in range(4):
            sst = pc.pc_run_stats()
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            sstatus = sctx.pc_skeleton(Xsd, alpha_s, sadj, srecs, scount, sws, stats=sst)
            torch.cuda.synchronize()
            if r:
                walls.append(time.perf_counter() - s0)
        sd = sst.as_dict()
        out["paper_scalability"] = {
            "workload": "n=1000, edge probability 0.1, positive weights, m=10000, alpha 0.01, fp64",
            "ms": float(np.median(walls)) * 1e3, "status": sstatus, "levels_run": sd["levels_run"],
            "gpu_tests": int(sum(sd["tests"])), "edges": int(pc.bits_to_dense(sadj.cpu().numpy(), ns_s).sum()) // 2}
        del Xsd, sws

    if not args.no_cpu_baseline:
        if "orientation" in out:
            # the orientation reference on the same skeleton and SepSets, timed and compared
            from oracle import orient as orient_ref
            seps = pc.decode_sepsets(grecs[:max(nrec, 1)].cpu().numpy(), nrec)
            c0 = time.perf_counter()
            H_ref, rounds_ref = orient_ref.orient(G.astype(bool), orient_ref.sepset_lookup(seps))
            out["orientation"]["cpu_reference_s"] = time.perf_counter() - c0
            out["orientation"]["same_as_reference"] = bool(np.array_equal(H_ref, Hg) and rounds_ref == rounds)
        ref, cpu_sec, reps = cpu_baseline(X, alpha)
        canonical = int(sum(ref.tests))
        out["value"] = canonical / sec_per_step
        out["canonical_tests_per_step"] = canonical
        out["skeleton_equal_to_oracle"] = bool(np.array_equal(G, ref.G))
        out["cpu_baseline"] = {"value": canonical / cpu_sec, "unit": "CI tests/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"whole workload (same input), {reps} runs, {cpu_sec:.3f} s each",
                               "wall_s_per_skeleton": cpu_sec}
    else:
        out["value"] = gpu_tests / sec_per_step
        out["note"] = "value counts GPU-executed tests (cpu baseline skipped)"
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
