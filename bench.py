#!/usr/bin/env python3
"""Benchmark: out-of-core streamed equi-join with zero-copy late materialization on one MI355X.

Workload (default): build 2^26 unique int64 keys with two int32 payloads; probe 2^31 int64 keys
with two int64 payloads (48 GiB) in pinned host memory, 10% of probe rows match; device budget
16 GiB; result = match count and exact int64 SUM of each payload column.  One step is one
vx_join_agg call: build the device hash table from host memory, stream every probe chunk
through the double buffer, gather matching payloads by zero-copy, aggregate, return.

Prints ONE JSON line (rank 0) with the throughput in probe rows/s, the host-link and HBM
roofline fractions (peaks measured live on this machine where the datasheet has no figure),
and the CPU oracle timed on a bounded sample.  The other workloads of the scope ride on the same
line as blocks: the skewed partitioned join (learned splitters against radix-hash, `--no-skew`
leaves it out), the in-memory join (`--no-plain`), the star join with group-by (`--no-star`) and
the 256 batched joins in one graph launch (`--no-batch`).
"""
import argparse
import contextlib
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "probe rows/s + % host-link peak; learned vs hash partitioning, bit-exact"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E datasheet peak
# HBM traffic of a kernel comes from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs, which cannot be
# taken inside this process; each roofline names the profile summary that holds them
# ("traffic_profile") and reports "traffic": null.
PROFILE = {"k_probe_stream": "profiles/k_probe_streamed_join.md",
           "k_probe_plain": "profiles/k_probe_plain_join.md",
           "k_star": "profiles/k_star_star_join.md",
           "batch_graph": "profiles/batch_graph_batched_joins.md",
           "k_pj_stream": "profiles/k_pj_stream_skewed_partitioned_join.md",
           "k_probe_rows": "profiles/k_probe_rows_streamed_join.md",
           "k_rj_probe": "profiles/k_rj_probe_two_table_radix_join.md",
           "sort_run": "profiles/k_digit_scatter_out_of_core_sort.md"}
GiB = 1 << 30


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--log2-build", type=int, default=26)
    ap.add_argument("--log2-probe", type=int, default=31)
    ap.add_argument("--budget-gib", type=float, default=16.0)
    ap.add_argument("--late-mat", type=int, default=-1)
    ap.add_argument("--chunk-rows", type=int, default=0)
    ap.add_argument("--n-buffers", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-skew", action="store_true",
                    help="stream workload: leave out the skewed partitioned join block")
    ap.add_argument("--skew-steps", type=int, default=3,
                    help="stream workload: timed steps per partitioner in the skewed join block")
    ap.add_argument("--no-plain", action="store_true",
                    help="stream workload: leave out the in-memory join block")
    ap.add_argument("--no-star", action="store_true",
                    help="stream workload: leave out the star join block")
    ap.add_argument("--no-batch", action="store_true",
                    help="stream workload: leave out the batched joins block")
    ap.add_argument("--batch-steps", type=int, default=5,
                    help="stream workload: timed steps per variant in the batched joins block")
    ap.add_argument("--workload", default="stream", choices=["stream", "plain", "star", "batch", "skew", "rows", "radix", "sort", "calib"],
                    help="stream (default) is the headline line; the others print their own line")
    ap.add_argument("--method", default="learned", help="skew workload: partitioner to time")
    ap.add_argument("--n-parts", type=int, default=256)
    ap.add_argument("--train-steps", type=int, default=0, help="skew workload: Adam steps (0 = library default)")
    ap.add_argument("--skew-budget-gib", type=float, default=32.0, help="skew workload: device budget")
    ap.add_argument("--skew-scramble", action="store_true",
                    help="skew workload: keys scrambled by a bijection of [0, 2^40) (frequencies kept, order lost)")
    ap.add_argument("--radix-log2", type=int, default=29, help="radix workload: log2 rows of each table")
    ap.add_argument("--radix-budget-gib", type=float, default=4.0, help="radix workload: device budget")
    ap.add_argument("--sort-log2", type=int, default=31, help="sort workload: log2 keys")
    ap.add_argument("--sort-budget-gib", type=float, default=4.0, help="sort workload: device budget")
    return ap.parse_args()


def host_info():
    """What the oracle timings ran on: CPU model, logical CPUs (all, and usable by this process), RAM."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    ram = round(int(line.split()[1]) / (1 << 20), 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "host_cpus_usable": len(os.sched_getaffinity(0)),
            "ram_gib": ram}


def cpu_baseline(log2_build, log2_probe):
    """The oracle (single-threaded, as it stands) on the same workload scaled down 8x:
    2^(b-3) build rows and 2^(p-3) probe rows from the same generators, 10% match.  Also the
    same oracle on all host cores (one build, the probe rows cut into one slice per thread,
    read-only lookups; the C calls release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    import datagen
    import oracle
    nb, np_ = 1 << (log2_build - 3), 1 << (log2_probe - 3)
    bk, b0, b1 = datagen.stream_build(nb)
    pk, p0, p1 = datagen.stream_probe(nb, np_)
    t0 = time.perf_counter()
    one = oracle.join_agg(bk, [b0, b1], pk, [p0, p1])
    dt = time.perf_counter() - t0
    n_thr = max(1, min(16, len(os.sched_getaffinity(0))))
    cut = [np_ * t // n_thr for t in range(n_thr + 1)]
    t0 = time.perf_counter()
    pb = oracle.PreparedBuild(bk, [b0, b1])
    with ThreadPoolExecutor(n_thr) as ex:
        parts = list(ex.map(lambda t: pb.probe(pk[cut[t]:cut[t + 1]], [p0[cut[t]:cut[t + 1]], p1[cut[t]:cut[t + 1]]]),
                            range(n_thr)))
    dt_all = time.perf_counter() - t0
    pb.close()
    if [sum(x) % (1 << 64) for x in zip(*parts)] != one:
        raise SystemExit("threaded oracle run disagrees with the single-threaded one")
    sample = f"same generators scaled 1/8: {nb} build rows, {np_} probe rows (10% match)"
    hi = host_info()
    return ({"value": np_ / dt, "unit": "probe rows/s", "cores": 1, "kind": "oracle",
             "sample": f"{sample}, build + probe in {dt:.1f} s on 1 host thread", **hi},
            {"value": np_ / dt_all, "unit": "probe rows/s", "cores": n_thr, "kind": "oracle",
             "sample": f"{sample}, build on 1 thread + probe on {n_thr} threads in {dt_all:.1f} s", **hi})


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload != "stream":
        out = {"plain": run_plain, "star": run_star, "batch": run_batch, "skew": run_skew,
               "rows": run_rows, "radix": run_radix, "sort": run_sort, "calib": run_calib}[args.workload](args)
        print(json.dumps(out), flush=True)
        return
    import numpy as np
    import torch

    import datagen
    import paper_2502_09541_amd as vx

    nb, np_ = 1 << args.log2_build, 1 << args.log2_probe
    log(f"workload: build {nb} rows, probe {np_} rows, budget {args.budget_gib} GiB")
    ctx = vx.Context(int(args.budget_gib * GiB))
    calib = ctx.calibrate()
    b_peak = calib["h2d_gbs"]
    log(f"measured H2D peak {b_peak:.2f} GB/s, zero-copy granule {calib['zc_granule']} B")

    t0 = time.perf_counter()
    H = {}
    for name, n, dt in (("bk", nb, np.int64), ("b0", nb, np.int32), ("b1", nb, np.int32),
                        ("pk", np_, np.int64), ("p0", np_, np.int64), ("p1", np_, np.int64)):
        H[name] = vx.HostBuffer(n, dt)
    log(f"pinned host columns allocated ({sum(h.n * h.dtype.itemsize for h in H.values()) / GiB:.1f} GiB)"
        f" in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    datagen.stream_build(nb, out=(H["bk"].array, H["b0"].array, H["b1"].array))
    step_rows = 1 << 27
    for r0 in range(0, np_, step_rows):
        r1 = min(np_, r0 + step_rows)
        datagen.stream_probe(nb, r1 - r0, out=(H["pk"].array[r0:r1], H["p0"].array[r0:r1],
                                               H["p1"].array[r0:r1]), row0=r0)
    log(f"generated inputs in {time.perf_counter() - t0:.1f} s")

    def step():
        return ctx.join_plain(H["bk"], [H["b0"], H["b1"]], H["pk"], [H["p0"], H["p1"]],
                              late_mat=args.late_mat, chunk_rows=args.chunk_rows,
                              n_buffers=args.n_buffers)

    for w in range(args.warmup):
        ref, st = step()
        log(f"warmup {w}: {st['total_ms']:.1f} ms, matches {ref[0]}")
    torch.cuda.synchronize()
    results, stats = [], []
    with gc_paused():
        t0 = time.perf_counter()
        for k in range(args.steps):
            r, st = step()
            results.append(r)
            stats.append(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    for k, st in enumerate(stats):
        log(f"step {k}: {st['total_ms']:.1f} ms (build {st['build_ms']:.1f}, probe {st['probe_ms']:.1f})")
    if any(r != results[0] for r in results) or (args.warmup and results[0] != ref):
        raise SystemExit("non-deterministic aggregates across steps")
    ms = wall * 1e3 / args.steps
    value = np_ / (ms / 1e3)

    st = stats[0]
    count = results[0][0]
    # one more step, untimed, with the probe kernels counting the zero-copy granules they move (the
    # count slows the gathers, so the timed steps run without it); same result required
    r_c, st_c = ctx.join_plain(H["bk"], [H["b0"], H["b1"]], H["pk"], [H["p0"], H["p1"]],
                               late_mat=args.late_mat, chunk_rows=args.chunk_rows, n_buffers=args.n_buffers,
                               count_zc=True)
    if r_c != results[0] or (st_c["zc_mask"] and not st_c["zc_counted"]):
        raise SystemExit("the counted step differs from the timed ones")
    # The pipeline is bound by the host link: every step moves the build columns, the probe keys
    # (chunk copies) and the matching rows' payloads (zero-copy gathers) over it.
    # algorithmic bytes: build columns (8 + 4 + 4 B per row), 8 B per probe key, 16 B of payloads
    # per match; wire bytes: the same build columns, the bytes the copy stream moved, and the
    # zero-copy granules the probe kernels counted, times the granule
    alg_bytes = nb * 16 + np_ * 8 + count * 16
    wire_bytes = nb * 16 + st["sdma_bytes"] + st_c["zc_bytes"]
    granule = calib["zc_granule"]
    # the probe kernel itself against HBM (secondary): per row 8 B of key from the chunk buffer
    # and one 16 B table slot, over its average launch time (HIP events on the library's stream)
    kms = sum(s["kernel_ms"] for s in stats)
    klaunch = sum(s["kernel_launches"] for s in stats)
    k_avg_ms = kms / klaunch
    rows_per_launch = np_ / st["kernel_launches"]
    hbm_gbs = 24.0 * rows_per_launch / (k_avg_ms * 1e6)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "probe rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "streamed_join_zero_copy", "build_rows": nb, "probe_rows": np_,
                   "key": "int64", "build_payloads": "2 x int32", "probe_payloads": "2 x int64",
                   "match_frac": 0.1, "probe_host_gib": np_ * 24 / GiB, "device_budget_gib": args.budget_gib,
                   "chunk_rows": st["chunk_rows"], "n_buffers": st["n_buffers"],
                   "late_mat": {-1: "auto", 0: "sdma", 1: "zero-copy", 2: "paper-TH"}[args.late_mat],
                   "zero_copy_columns": bin(st["zc_mask"]).count("1")},
        "roofline": {"bound": "host_link",
                     "kernel": "whole step: build columns read in place, probe-key chunk copies, k_probe's "
                               "zero-copy payload gathers",
                     "achieved": alg_bytes / (ms * 1e6), "peak": b_peak, "unit": "GB/s",
                     "frac": alg_bytes / (ms * 1e6) / b_peak,
                     "traffic": wire_bytes,
                     "peak_kind": "host-to-device copy rate measured in this run (PCIe 5.0 x16, 63 GB/s "
                                  "theoretical); the datasheet gives no achievable figure",
                     "algorithmic_bytes": "per step: 16 B per build row + 8 B per probe key + 16 B of payloads "
                                          "per match",
                     "traffic_kind": "host-link bytes per step: build columns + copy-stream bytes + the zero-copy "
                                     "granules k_probe counts (in one more, untimed step with the count on) x granule"},
        "host_link": {"peak_measured_gbs": b_peak,
                      "achieved_wire_gbs": wire_bytes / (ms * 1e6),
                      "frac_wire": wire_bytes / (ms * 1e6) / b_peak,
                      "achieved_algorithmic_gbs": alg_bytes / (ms * 1e6),
                      "frac_algorithmic": alg_bytes / (ms * 1e6) / b_peak,
                      "wire_bytes_per_step": wire_bytes, "algorithmic_bytes_per_step": alg_bytes,
                      "zero_copy_bytes_counted": st_c["zc_bytes"], "zero_copy_granule": granule,
                      "zero_copy_bytes_binomial_model": st["zc_bytes"],
                      "sdma_bytes_per_step": st["sdma_bytes"]},
        "hbm": {"kernel": "k_probe", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm_gbs / HBM_PEAK_GBS, "traffic": None, "traffic_profile": PROFILE["k_probe_stream"],
                "avg_launch_ms": k_avg_ms, "rows_per_launch": rows_per_launch,
                "algorithmic_bytes": "24 B per probe row (8 B key from the chunk buffer + one 16 B slot)"},
        "result": {"match_count": count, "sums": results[0][1:]},
        "calibration": calib,
    }
    ctx.close()
    for h in H.values():
        h.free()
    del H
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"], out["cpu_baseline_all_cores"] = cpu_baseline(args.log2_build, args.log2_probe)
    if not args.no_skew:
        out["skew_partitioned_join"] = skew_block(args)
    if not args.no_plain:
        out["in_memory_join"] = _sub_block(run_plain, args, 50, 10)
    if not args.no_star:
        out["star_join_groupby"] = _sub_block(run_star, args, 5, 1)
    if not args.no_batch:
        out["batched_joins"] = _sub_block(run_batch, args, args.batch_steps, 1)
    print(json.dumps(out), flush=True)


# --------------------------------------------------------------------------- skewed partitioned join

def _chunks(n, step=1 << 27):
    return [(r0, min(n, r0 + step)) for r0 in range(0, n, step)]


def _skew_inputs(vx, nb, np_, scramble):
    import numpy as np
    import datagen
    bk, bp, pk = vx.HostBuffer(nb, np.int64), vx.HostBuffer(nb, np.int64), vx.HostBuffer(np_, np.int64)
    t0 = time.perf_counter()
    for r0, r1 in _chunks(nb):
        datagen.skew_build(r1 - r0, out=(bk.array[r0:r1], bp.array[r0:r1]), row0=r0)
        if scramble:
            datagen.scramble40(bk.array[r0:r1])
    for r0, r1 in _chunks(np_):
        datagen.skew_probe(r1 - r0, out=pk.array[r0:r1], row0=r0)
        if scramble:
            datagen.scramble40(pk.array[r0:r1])
    log(f"skew: {nb} + {np_} rows generated in {time.perf_counter() - t0:.1f} s")
    return bk, bp, pk


def _skew_time(ctx, vx, torch, bk, bp, pk, methods, args, steps, warmup):
    """Each partitioner timed on the same inputs: warm-up steps, then `steps` timed calls; every
    step's aggregate must be the same for every method."""
    lines, failed = {}, {}
    for method in methods:
        def step():
            return ctx.join_partitioned(bk, [bp], pk, method=method, n_parts=args.n_parts, seed=7,
                                        train_steps=args.train_steps)
        try:
            for _ in range(warmup):
                ref = step()
            torch.cuda.synchronize()
            res = []
            with gc_paused():
                t0 = time.perf_counter()
                for _ in range(steps):
                    res.append(step())
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / steps
        except vx.VxError as e:
            if method == methods[0]:
                raise
            # a control partitioner that cannot run under this budget is reported, not timed
            failed[method] = str(e)
            log(f"skew {method}: {e}")
            continue
        if any(r[0] != res[0][0] for r in res) or (warmup and ref[0] != res[0][0]):
            raise SystemExit(f"skew {method}: non-deterministic results across steps")
        agg, st, used = res[0]
        lines[method] = dict(ms=ms, value=len(pk.array) / (ms / 1e3), agg=agg, st=st, used=used)
        log(f"skew {method}: {ms:.1f} ms/step, partitions {st['n_parts']}, singleton rows {st['singleton_rows']}")
    first = lines[methods[0]]["agg"]
    if any(x["agg"] != first for x in lines.values()):
        raise SystemExit("partitioned join results differ across partitioners")
    return lines, failed


def _skew_line(x):
    st = x["st"]
    return {"ms_per_step": x["ms"], "value": x["value"], "imbalance": st["imbalance"],
            "imbalance_table_partitions": st["imbalance_tables"],
            "imbalance_distinct_keys": st["imbalance_distinct"], "part_ms": st["part_ms"],
            "train_ms": st["train_ms"], "join_ms": st["probe_ms"], "n_parts": st["n_parts"],
            "singleton_rows": st["singleton_rows"],
            "h2d_bytes_per_step": st["sdma_bytes"] + st["zc_bytes"]}


def _skew_checks(ctx, bk, bp, pk, args, with_oracle):
    """Checks of the full-size result that do not use the GPU's other partitioners:
    - the three heaviest keys' singleton partitions against mB(k) mP(k) and sumB(k) mP(k), counted
      from the arrays with numpy;
    - when with_oracle (the cpu_baseline leg): two table partitions against the oracle on the rows
      whose keys fall in them, and the oracle timed on a bounded sample of the workload's rows (the
      first 2^25 build and 2^27 probe rows: a Zipf mix of heavy and light keys, as in the whole)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    M64 = 1 << 64
    nb, np_ = len(bk.array), len(pk.array)
    tot, st, used, per = ctx.join_partitioned(bk, [bp], pk, method="learned", n_parts=args.n_parts, seed=7,
                                              train_steps=args.train_steps, per_partition=True)
    r = ctx.partition(bk, method="learned", n_parts=args.n_parts, seed=7, train_steps=args.train_steps)
    spl = r["splitters"]
    P = len(spl) + 1
    if st["n_parts"] != P or [sum(x) % M64 for x in zip(*per)] != tot:
        raise SystemExit("skew check: per-partition aggregates do not add up to the total")
    single = {int(spl[i - 1]): i for i in range(1, len(spl)) if spl[i] == spl[i - 1] + 1}
    n_thr = max(1, min(16, len(os.sched_getaffinity(0))))
    ex = ThreadPoolExecutor(n_thr)

    def heavy(c, col, pay):
        k = col.array[c[0]:c[1]]
        res = []
        for key in (1, 2, 3):
            m = k == key
            res.append((int(m.sum()), int(pay.array[c[0]:c[1]][m].view(np.uint64).sum(dtype=np.uint64))
                        if pay is not None else 0))
        return res

    hb = list(ex.map(lambda c: heavy(c, bk, bp), _chunks(nb)))
    hp = list(ex.map(lambda c: heavy(c, pk, None), _chunks(np_)))
    heavy_ok = []
    for i, key in enumerate((1, 2, 3)):
        mB, sB, mP = sum(x[i][0] for x in hb), sum(x[i][1] for x in hb), sum(x[i][0] for x in hp)
        ok = key in single and per[single[key]] == [mB * mP % M64, sB * mP % M64]
        if not ok:
            raise SystemExit(f"skew check: singleton partition of key {key} differs from its closed form")
        heavy_ok.append({"key": key, "build_rows": mB, "probe_rows": mP})
    out = {"heavy_key_singletons_closed_form": heavy_ok, "n_parts": P}
    if with_oracle:
        import oracle
        table_parts = [p for p in range(1, P - 1) if p not in single.values()]
        checked = []
        for p in (table_parts[len(table_parts) // 2], table_parts[len(table_parts) // 4]):
            lo, hi = int(spl[p - 1]), int(spl[p])

            def pick(c, col, pay):
                k = col.array[c[0]:c[1]]
                m = (k >= lo) & (k < hi)
                return k[m], (pay.array[c[0]:c[1]][m] if pay is not None else None)

            b = list(ex.map(lambda c: pick(c, bk, bp), _chunks(nb)))
            q = list(ex.map(lambda c: pick(c, pk, None), _chunks(np_)))
            kb, vb = np.concatenate([x[0] for x in b]), np.concatenate([x[1] for x in b])
            kp = np.concatenate([x[0] for x in q])
            if per[p] != oracle.join_agg(kb, [vb], kp, []):
                raise SystemExit(f"skew check: partition {p} differs from the oracle")
            checked.append({"partition": p, "keys": [lo, hi], "build_rows": len(kb), "probe_rows": len(kp)})
        out["oracle_partitions"] = checked
        sb, sp = 1 << 25, 1 << 27
        t0 = time.perf_counter()
        oracle.join_agg(bk.array[:sb], [bp.array[:sb]], pk.array[:sp], [])
        secs = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": sp / secs, "unit": "probe rows/s", "cores": 1, "kind": "oracle",
                               "sample": f"the first {sb} build and {sp} probe rows of the same workload (1/32 of "
                                         f"each side), joined in {secs:.1f} s on 1 host thread", **host_info()}
    ex.shutdown()
    return out


def skew_block(args):
    """The metric's second half on the default line: learned vs radix-hash (and the sample-quantile
    control) on the skewed partitioned join at full size, 2^30 Zipf(1.1) build keys over [1, 2^40]
    with an int64 payload and 2^32 Zipf(1.1) probe keys in pinned host memory, 32 GiB budget."""
    import torch
    import paper_2502_09541_amd as vx
    nb, np_ = 1 << 30, 1 << 32
    bk, bp, pk = _skew_inputs(vx, nb, np_, False)
    try:
        with vx.Context(int(args.skew_budget_gib * GiB)) as ctx:
            b_peak = ctx.calibrate()["h2d_gbs"]
            lines, failed = _skew_time(ctx, vx, torch, bk, bp, pk, ["learned", "radix_hash", "quantile"], args,
                                       args.skew_steps, 1)
            checks = _skew_checks(ctx, bk, bp, pk, args, not args.no_cpu_baseline)
    finally:
        for h in (bk, bp, pk):
            h.free()
    a = lines["learned"]
    out = {"workload": "skewed_partitioned_join", "build_rows": nb, "probe_rows": np_, "zipf_s": 1.1,
           "key_range": "[1, 2^40]", "device_budget_gib": args.skew_budget_gib, "steps": args.skew_steps,
           "warmup": 1, "unit": "probe rows/s", "value": a["value"], "ms_per_step": a["ms"],
           "learned": _skew_line(a),
           "radix_hash": _skew_line(lines["radix_hash"]) if "radix_hash" in lines else {"error": failed["radix_hash"]},
           "sample_quantile": _skew_line(lines["quantile"]) if "quantile" in lines else {"error": failed["quantile"]},
           "learned_speedup_vs_radix_hash": lines["radix_hash"]["ms"] / a["ms"] if "radix_hash" in lines else None,
           "host_link": {"peak_measured_gbs": b_peak,
                         "frac": (a["st"]["sdma_bytes"] + a["st"]["zc_bytes"]) / (a["ms"] * 1e6) / b_peak},
           "result": {"match_count": a["agg"][0], "sum": a["agg"][1]},
           "bit_exact_across_methods": True, "checks": checks}
    if "cpu_baseline" in checks:
        out["cpu_baseline"] = checks.pop("cpu_baseline")
    return out


# --------------------------------------------------------------------------- other workloads
# Each prints its own JSON line (same fields); only the streamed join is the default line.

def _common(metric_unit, value, ms, args, dtype, config, roofline, extra=None):
    out = {"metric": METRIC, "value": value, "unit": metric_unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
           "roofline": roofline}
    if extra:
        out.update(extra)
    return out


@contextlib.contextmanager
def gc_paused():
    """Timed steps run with Python's cyclic garbage collector paused, as timeit runs them: a full
    collection of this process's objects takes tens of milliseconds and would land in whichever
    step happens to trigger it."""
    gc.collect()
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


def _timed(step, args, torch):
    ref = None
    for _ in range(args.warmup):
        ref = step()
    torch.cuda.synchronize()
    res = []
    with gc_paused():
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res.append(step())
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
    first = res[0][0]
    if any(r[0] != first for r in res) or (ref is not None and ref[0] != first):
        raise SystemExit("non-deterministic results across steps")
    return ms, res


def run_rows(args):
    """The streamed join of the default line with its rows materialized: every match writes
    (probe row, 2 build payloads, 2 probe payloads) as int64 into pinned host memory, 40 B per
    output row.  Timed next to the same join reduced to aggregates only."""
    import numpy as np
    import torch
    import datagen
    import paper_2502_09541_amd as vx
    nb, np_ = 1 << args.log2_build, 1 << args.log2_probe
    ctx = vx.Context(int(args.budget_gib * GiB))
    b_peak = ctx.calibrate()["h2d_gbs"]
    H = {}
    for name, n, dt in (("bk", nb, np.int64), ("b0", nb, np.int32), ("b1", nb, np.int32),
                        ("pk", np_, np.int64), ("p0", np_, np.int64), ("p1", np_, np.int64)):
        H[name] = vx.HostBuffer(n, dt)
    datagen.stream_build(nb, out=(H["bk"].array, H["b0"].array, H["b1"].array))
    step_rows = 1 << 27
    for r0 in range(0, np_, step_rows):
        r1 = min(np_, r0 + step_rows)
        datagen.stream_probe(nb, r1 - r0, out=(H["pk"].array[r0:r1], H["p0"].array[r0:r1],
                                               H["p1"].array[r0:r1]), row0=r0)
    cap = int(np_ * 0.1 * 1.01) + (1 << 20)
    O = [vx.HostBuffer(cap, np.uint64)] + [vx.HostBuffer(cap, np.int64) for _ in range(4)]
    out = (O[0].array, [O[1].array, O[2].array], [O[3].array, O[4].array])
    log(f"rows: {np_} probe rows, output capacity {cap} rows ({5 * 8 * cap / GiB:.1f} GiB pinned)")
    t = ctx.build(H["bk"], [H["b0"], H["b1"]])

    def step_rows_():
        return t.probe_rows(H["pk"], [H["p0"], H["p1"]], out=out, cap=cap)

    def step_agg():
        return t.probe(H["pk"], [H["p0"], H["p1"]])

    ms, res = _timed(step_rows_, args, torch)
    ms_agg, res_agg = _timed(step_agg, args, torch)
    agg, st, n_out, _ = res[0]
    if agg != res_agg[0][0] or any(r[0] != agg or r[2] != n_out for r in res):
        raise SystemExit("materialized join disagrees with the aggregate-only join")
    # one more, untimed step with the kernels counting the zero-copy granules they touch
    agg_c, st_c, n_c, _ = t.probe_rows(H["pk"], [H["p0"], H["p1"]], out=out, cap=cap, count_zc=True)
    if agg_c != agg or n_c != n_out or not st_c["zc_counted"]:
        raise SystemExit("counted step disagrees")
    t.destroy()
    ctx.close()
    for h in list(H.values()) + O:
        h.free()
    d2h = n_out * 40
    # dominant kernel: per probe row 8 B key from the chunk buffer + one 16 B slot, as k_probe
    launches = max(1, st["kernel_launches"])
    k_avg = st["kernel_ms"] / launches
    ach = 24.0 * (np_ / launches) / (k_avg * 1e6)
    # the step waits on the host link, as the aggregate-only join does: algorithmic host-to-device
    # bytes as there (16 B per build row, 8 B per probe key, 16 B of payloads per match); the
    # output rows leave in the other direction
    alg = nb * 16 + np_ * 8 + agg[0] * 16
    wire = nb * 16 + st["sdma_bytes"] + st_c["zc_bytes"]
    return _common("probe rows/s", np_ / (ms / 1e3), ms, args, "int64",
                   {"workload": "streamed_join_rows_materialized", "build_rows": nb, "probe_rows": np_,
                    "output_rows": n_out, "output_bytes_per_row": 40, "match_frac": 0.1,
                    "device_budget_gib": args.budget_gib},
                   {"bound": "host_link",
                    "kernel": "whole step: build columns, probe-key chunk copies, k_probe_rows' zero-copy payload "
                              "reads and output row stores",
                    "achieved": alg / (ms * 1e6), "peak": b_peak, "unit": "GB/s", "frac": alg / (ms * 1e6) / b_peak,
                    "traffic": wire, "peak_kind": "host-to-device copy rate measured in this run",
                    "algorithmic_bytes": "host-to-device per step: 16 B per build row + 8 B per probe key + 16 B of "
                                         "payloads per match",
                    "traffic_kind": "host-to-device bytes per step: build columns + copy-stream bytes + the "
                                    "zero-copy granules k_probe_rows counts x granule"},
                   {"hbm": {"kernel": "k_probe_rows", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": ach / HBM_PEAK_GBS, "traffic": None, "traffic_profile": PROFILE["k_probe_rows"],
                            "avg_launch_ms": k_avg, "rows_per_launch": np_ / launches},
                    "host_link": {"peak_measured_gbs": b_peak,
                                  "h2d_gbs": wire / (ms * 1e6),
                                  "zero_copy_bytes_counted": st_c["zc_bytes"],
                                  "zero_copy_bytes_binomial_model": st["zc_bytes"],
                                  "d2h_output_gbs": d2h / (ms * 1e6)},
                    "aggregate_only_ms_per_step": ms_agg,
                    "materialization_cost": ms / ms_agg - 1.0,
                    "result": {"match_count": agg[0], "output_rows": n_out}})


def run_calib(args):
    """The link and memory denominators (vx_calibrate over 4 GiB of pinned memory)."""
    import paper_2502_09541_amd as vx
    ctx = vx.Context(8 * GiB)
    c = ctx.calibrate(4 * GiB)
    ctx.close()
    return {"metric": "host link / device memory calibration", "calibration": c, "n_gpus": 1}


def run_plain(args):
    """In-memory join: 2^20 unique int32 build keys + one int32 payload, 2^24 int32 probes
    (about half match), all device-resident; step = build + probe + aggregate.  The same join
    with its columns in pinned host memory is reported beside it (`host_resident`)."""
    import torch
    import datagen
    import oracle
    import paper_2502_09541_amd as vx
    nb, np_ = 1 << 20, 1 << 24
    bk, bp, pk = datagen.plain_join(nb, np_)
    d = [torch.from_numpy(a).cuda() for a in (bk, bp, pk)]
    ctx = vx.Context(4 * GiB)
    ms, res = _timed(lambda: ctx.join_plain(d[0], [d[1]], d[2]), args, torch)
    agg, st = res[0]
    k_ms = sum(r[1]["kernel_ms"] for r in res) / sum(r[1]["kernel_launches"] for r in res)
    # probe kernel: 4 B key + one 8 B slot per probe row
    achieved = np_ * 12 / (k_ms * 1e6)
    t0 = time.perf_counter()
    exp = oracle.join_agg(bk, [bp], pk, [])
    cpu = time.perf_counter() - t0
    if exp != agg:
        raise SystemExit("plain join result differs from the oracle")
    # the same join with its columns in pinned host memory: the build side is read by zero-copy
    # (its keys are not measured there, so the table is hashed) and the probe keys stream through
    # the chunk pipeline; 8 B per build row and 4 B per probe row cross the host link
    cal = ctx.calibrate()
    hb = []
    for a in (bk, bp, pk):
        h = vx.HostBuffer(len(a), a.dtype)
        h.array[:] = a
        hb.append(h)
    ms_h, res_h = _timed(lambda: ctx.join_plain(hb[0], [hb[1]], hb[2]), args, torch)
    if res_h[0][0] != agg:
        raise SystemExit("host-resident plain join differs from the device-resident one")
    # the same device-resident join through a hash table (the general layout; the dense table above
    # is what this recipe's keys allow)
    ms_x, res_x = _timed(lambda: ctx.join_plain(d[0], [d[1]], d[2], hashed=True), args, torch)
    if res_x[0][0] != agg:
        raise SystemExit("hashed plain join differs from the dense one")
    kx = sum(r[1]["kernel_ms"] for r in res_x) / sum(r[1]["kernel_launches"] for r in res_x)
    hashed_variant = {"ms_per_step": ms_x, "value": np_ / (ms_x / 1e3), "unit": "probe rows/s",
                      "probe_kernel_ms": kx, "table_bytes": res_x[0][1]["table_bytes"]}
    link_bytes = nb * 8 + np_ * 4
    host_variant = {"ms_per_step": ms_h, "value": np_ / (ms_h / 1e3), "unit": "probe rows/s",
                    "link_bytes_per_step": link_bytes, "h2d_peak_measured_gbs": cal["h2d_gbs"],
                    "link_frac": link_bytes / (ms_h * 1e6) / cal["h2d_gbs"]}
    for h in hb:
        h.free()
    ctx.close()
    return _common("probe rows/s", np_ / (ms / 1e3), ms, args, "int32",
                   {"workload": "plain_join_device_resident", "build_rows": nb, "probe_rows": np_,
                    "key": "int32", "build_payloads": "1 x int32"},
                   {"bound": "hbm", "kernel": "k_probe", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None, "traffic_profile": PROFILE["k_probe_plain"], "avg_launch_ms": k_ms,
                    "rows_per_launch": np_},
                   {"result": {"match_count": agg[0], "sum": agg[1]}, "checked_against_oracle": True,
                    "build_ms": st["build_ms"], "probe_ms": st["probe_ms"], "table_bytes": st["table_bytes"],
                    "hash_table": hashed_variant, "host_resident": host_variant,
                    "cpu_baseline": {"value": np_ / cpu, "unit": "probe rows/s", "cores": 1, "kind": "oracle",
                                     "sample": f"the full workload, build + probe in {cpu:.1f} s on 1 host thread",
                                     **host_info()}})


def run_star(args):
    """Star join + GROUP BY: 600,000,000 fact rows (4 int32 foreign keys, 3 int32 measures) in
    pinned host memory; dimensions of 2,556 / 200,000 / 3,000,000 / 2,000,000 rows with filter
    selectivities 1/7, 1/5, 1/25, 1 on the device; 7 x 100 groups."""
    import numpy as np
    import torch
    import datagen
    import oracle
    import paper_2502_09541_amd as vx
    nf = 600_000_000
    rows = datagen.STAR_DIM_ROWS
    dims = datagen.star_dims()
    ddims = [dict(key=torch.from_numpy(x["key"]).cuda(), filt=torch.from_numpy(x["filt"]).cuda(), lo=0, hi=0,
                  group=None if x["group"] is None else torch.from_numpy(x["group"]).cuda()) for x in dims]
    fk = [vx.HostBuffer(nf, np.int32) for _ in range(4)]
    ms_ = [vx.HostBuffer(nf, np.int32) for _ in range(3)]
    step_rows = 1 << 26
    for r0 in range(0, nf, step_rows):
        r1 = min(nf, r0 + step_rows)
        datagen.star_fact(r1 - r0, out=([h.array[r0:r1] for h in fk], [h.array[r0:r1] for h in ms_]), row0=r0)
    log("star: inputs generated")
    ctx = vx.Context(16 * GiB)
    b_peak = ctx.calibrate()["h2d_gbs"]

    def step():
        g, c, sm, st = ctx.join_star(ddims, fk, ms_, groups_cap=4096)
        return (g.tolist(), c.tolist(), sm.tolist()), st

    ms, res = _timed(step, args, torch)
    st = res[0][1]
    k_ms = sum(r[1]["kernel_ms"] for r in res) / sum(r[1]["kernel_launches"] for r in res)
    # one more, untimed step with the kernels counting the zero-copy granules they touch
    g_c, c_c, s_c, st_c = ctx.join_star(ddims, fk, ms_, groups_cap=4096, count_zc=True)
    if (g_c.tolist(), c_c.tolist(), s_c.tolist()) != res[0][0] or not st_c["zc_counted"]:
        raise SystemExit("counted star step disagrees")
    wire = st["sdma_bytes"] + st_c["zc_bytes"]
    # algorithmic link bytes: each fact column is needed only for rows alive when it is read
    # (dimensions probed in ascending filter selectivity, then the 3 measures of survivors)
    sel = sorted(float(np.mean(x["filt"] == 0)) for x in dims)
    alive, alg = 1.0, 0.0
    for sv in sel:
        alg += alive * 4
        alive *= sv
    alg = nf * (alg + alive * 12)
    # CPU oracle on a bounded sample: the first 2^24 fact rows
    n_cpu = 1 << 24
    t0 = time.perf_counter()
    oracle.star_groupby(dims, [h.array[:n_cpu].copy() for h in fk], [h.array[:n_cpu].copy() for h in ms_])
    cpu = time.perf_counter() - t0
    ctx.close()
    out = _common("fact rows/s", nf / (ms / 1e3), ms, args, "int32",
                  {"workload": "star_join_groupby", "fact_rows": nf, "dims": list(rows),
                   "filter_selectivity": ["1/7", "1/5", "1/25", "1"], "groups": len(res[0][0][0]),
                   "chunk_rows": st["chunk_rows"], "zero_copy_columns": bin(st["zc_mask"]).count("1")},
                  # the step waits on the host link: the first foreign key column arrives by chunk
                  # copies, the other columns of the rows still alive by k_star's zero-copy reads
                  {"bound": "host_link",
                   "kernel": "whole step: chunk copies of the first foreign key, k_star's zero-copy reads of the "
                             "other columns for surviving rows",
                   "achieved": alg / (ms * 1e6), "peak": b_peak, "unit": "GB/s", "frac": alg / (ms * 1e6) / b_peak,
                   "traffic": wire,
                   "peak_kind": "host-to-device copy rate measured in this run",
                   "algorithmic_bytes": "per fact row: 4 B of each foreign key column while the row is alive "
                                        "(dimensions in ascending filter selectivity), then 12 B of measures "
                                        "per surviving row",
                   "traffic_kind": "host-link bytes per step: copy-stream bytes + the zero-copy granules k_star "
                                   "counts (in one more, untimed step with the count on) x granule"},
                  {"hbm": {"kernel": "k_star",
                           # per launch: 4 B foreign key from the chunk buffer + one 8 B slot of the first table
                           "achieved": (nf / st["kernel_launches"]) * 12 / (k_ms * 1e6), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": (nf / st["kernel_launches"]) * 12 / (k_ms * 1e6) / HBM_PEAK_GBS,
                           "traffic": None, "traffic_profile": PROFILE["k_star"], "avg_launch_ms": k_ms,
                           "rows_per_launch": nf / st["kernel_launches"]},
                   "host_link": {"peak_measured_gbs": b_peak, "achieved_wire_gbs": wire / (ms * 1e6),
                                 "frac_wire": wire / (ms * 1e6) / b_peak,
                                 "zero_copy_bytes_counted": st_c["zc_bytes"],
                                 "zero_copy_bytes_binomial_model": st["zc_bytes"],
                                 "achieved_algorithmic_gbs": alg / (ms * 1e6),
                                 "frac_algorithmic": alg / (ms * 1e6) / b_peak},
                   "survivors": st["survivors"], "build_ms": st["build_ms"],
                   "cpu_baseline": {"value": n_cpu / cpu, "unit": "fact rows/s", "cores": 1, "kind": "oracle",
                                    "sample": f"first {n_cpu} fact rows in {cpu:.1f} s on 1 host thread",
                                    **host_info()}})
    for h in fk + ms_:
        h.free()
    return out


def run_batch(args):
    """256 independent int32 joins, build sizes log-uniform in 2^10..2^22 (unique keys), probe
    10x..100x the build (about half match), device-resident; one HIP graph launch per step,
    against the per-job baseline of two launches per join."""
    import torch
    import datagen
    import paper_2502_09541_amd as vx
    b, p = datagen.batch_sizes(256)
    jobs = [datagen.batch_job(j, int(b[j]), int(p[j])) for j in range(256)]
    d = [[torch.from_numpy(a).cuda() for a in job] for job in jobs]
    del jobs
    ctx = vx.Context(32 * GiB)
    args3 = ([x[0] for x in d], [x[1] for x in d], [x[2] for x in d])
    rows = int(p.sum())
    log(f"batch: {rows} probe rows over 256 joins; autotuning")
    ms, res = _timed(lambda: ctx.join_batch(*args3, mode=0), args, torch)
    ms1, res1 = _timed(lambda: ctx.join_batch(*args3, mode=1), args, torch)
    if res[0][0] != res1[0][0]:
        raise SystemExit("batched and per-job results differ")
    # the same batch through hash tables (the general layout; these jobs' dense keys allow direct
    # tables), graph and per-job baseline
    log("batch: hash tables for every job")
    ms_h, res_h = _timed(lambda: ctx.join_batch(*args3, mode=0, hashed=True), args, torch)
    ms_h1, res_h1 = _timed(lambda: ctx.join_batch(*args3, mode=1, hashed=True), args, torch)
    if res_h[0][0] != res[0][0] or res_h1[0][0] != res[0][0]:
        raise SystemExit("hashed batch results differ from the direct ones")
    checked = _batch_checks(b, p, res[0][0])
    cpu = _batch_cpu_baseline(b, p, res[0][0])
    st = res[0][1]
    k_ms = sum(r[1]["kernel_ms"] for r in res) / len(res)
    # algorithmic bytes per graph: the join's per-unit figure, as for the in-memory join (a probe
    # row reads its 4 B key and one 8 B table slot; a build row reads 8 B and writes an 8 B slot);
    # beside it the direct tables' own figure, which these dense-key jobs allow (a probe reads its
    # key and, when the key is in its job's range, a 4 B payload; a build row reads its key and
    # payload and writes the payload)
    matches = sum(int(g[0]) for g in res[0][0])
    alg = rows * 12 + int(b.sum()) * 16
    alg_direct = rows * 4 + matches * 4 + int(b.sum()) * 12
    k_ms_h = sum(r[1]["kernel_ms"] for r in res_h) / len(res_h)
    ctx.close()
    return _common("probe rows/s", rows / (ms / 1e3), ms, args, "int32",
                   {"workload": "batched_joins_256", "jobs": 256, "probe_rows": rows, "build_rows": int(b.sum()),
                    "tile_rows": st["chunk_rows"], "block": st["n_buffers"], "load_factor": st["imbalance"],
                    "partitioned_jobs": st["n_parts"], "jobs_probed_from_lds": st["survivors"]},
                   {"bound": "hbm", "kernel": "graph(k_batch_phase build, k_batch_dupcount; k_batch_count, k_batch_scan, k_batch_scatter; k_batch_region)", "achieved": alg / (k_ms * 1e6),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg / (k_ms * 1e6) / HBM_PEAK_GBS,
                    "traffic": None, "traffic_profile": PROFILE["batch_graph"], "avg_launch_ms": k_ms, "rows_per_launch": rows,
                    "algorithmic_bytes": "12 B per probe row (4 B key + one 8 B table slot) + 16 B per build row",
                    "direct_tables": {"bytes_per_launch": alg_direct, "achieved": alg_direct / (k_ms * 1e6),
                                      "frac": alg_direct / (k_ms * 1e6) / HBM_PEAK_GBS,
                                      "algorithmic_bytes": "4 B key per probe row + 4 B payload per match + "
                                                           "12 B per build row"}},
                   {"baseline_separate_launches": {"ms_per_step": ms1, "value": rows / (ms1 / 1e3),
                                                   "launches": res1[0][1]["kernel_launches"]},
                    "speedup_vs_separate_launches": ms1 / ms,
                    "hash_tables": {"ms_per_step": ms_h, "value": rows / (ms_h / 1e3),
                                    "graph_ms": k_ms_h,
                                    "hbm_frac": alg / (k_ms_h * 1e6) / HBM_PEAK_GBS,
                                    "tile_rows": res_h[0][1]["chunk_rows"], "block": res_h[0][1]["n_buffers"],
                                    "load_factor": res_h[0][1]["imbalance"],
                                    "partitioned_jobs": res_h[0][1]["n_parts"],
                                    "jobs_probed_from_lds": res_h[0][1]["survivors"],
                                    "baseline_separate_launches_ms": ms_h1,
                                    "speedup_vs_separate_launches": ms_h1 / ms_h,
                                    "vs_direct_tables": ms_h / ms},
                    "result": {"match_count": matches,
                               "closed_form_checked_jobs": checked},
                    "cpu_baseline": cpu})


def _batch_checks(b, p, got):
    """Sampled jobs of the batch against their closed form: a job's build keys are a permutation of
    0..n_build-1 and its probe keys fall in 0..2*n_build-1, so its COUNT is the number of probe keys
    below n_build and its SUM adds the payload that the permutation gives each of them (mod 2^64).
    Checked: the jobs with the largest build and the largest probe side, the smallest build, and
    five seeded picks."""
    import numpy as np
    import datagen
    M64 = 1 << 64
    pick = {int(np.argmax(b)), int(np.argmax(p)), int(np.argmin(b))}
    pick |= {int(j) for j in np.random.default_rng(0xC4).choice(len(b), 5, replace=False)}
    for j in sorted(pick):
        bk, bp, pk = datagen.batch_job(j, int(b[j]), int(p[j]))
        pay_of_key = np.empty(len(bk), np.int64)
        pay_of_key[bk] = bp
        hit = pk < len(bk)
        exp = [int(hit.sum()), int(pay_of_key[pk[hit]].sum()) % M64]
        if list(got[j]) != exp:
            raise SystemExit(f"batched join {j}: {list(got[j])} against the closed form {exp}")
    return sorted(pick)


def _batch_cpu_baseline(b, p, got):
    """The CPU oracle on a bounded sample of the batch: eight jobs that span its sizes (the middle
    job of each eighth in order of probe size, about 1.2e8 probe rows), joined one after another
    on one host thread; their results must equal the GPU's."""
    import numpy as np
    import datagen
    import oracle
    sample = sorted(int(j) for j in np.argsort(p, kind="stable")[16::32])
    rows, secs = 0, 0.0
    for j in sample:
        bk, bp, pk = datagen.batch_job(j, int(b[j]), int(p[j]))
        t0 = time.perf_counter()
        exp = oracle.join_agg(bk, [bp], pk, [])
        secs += time.perf_counter() - t0
        rows += len(pk)
        if list(got[j]) != exp:
            raise SystemExit(f"batched join {j}: {list(got[j])} against the oracle {exp}")
    return {"value": rows / secs, "unit": "probe rows/s", "cores": 1, "kind": "oracle",
            "sample": f"jobs {sample} of the batch ({rows} probe rows), build + probe in {secs:.1f} s on 1 host "
                      f"thread, results equal to the GPU's", **host_info()}


def _sub_block(run, args, steps, warmup):
    """Another workload's line as a block of the default line: the workload runs with its own
    steps and warmup, and the block keeps its fields except those the headline line carries."""
    sub = argparse.Namespace(**vars(args))
    sub.steps, sub.warmup = steps, warmup
    r = run(sub)
    return {k: v for k, v in r.items()
            if k not in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data")}


def run_skew(args):
    """Skewed partitioned join on its own line: 2^30 Zipf(1.1) int64 build keys over [1, 2^40] with
    an int64 payload, 2^32 Zipf(1.1) probe keys, pinned host memory, device budget
    --skew-budget-gib (32); --method against the sample-quantile and radix-hash controls (a control
    the budget cannot run is reported), optionally with scrambled keys; every method must give the
    same result."""
    import torch
    import paper_2502_09541_amd as vx
    nb, np_ = 1 << 30, 1 << 32
    bk, bp, pk = _skew_inputs(vx, nb, np_, args.skew_scramble)
    methods = [args.method] + [m for m in ("quantile", "radix_hash") if m != args.method]
    try:
        with vx.Context(int(args.skew_budget_gib * GiB)) as ctx:
            b_peak = ctx.calibrate()["h2d_gbs"]
            lines, failed = _skew_time(ctx, vx, torch, bk, bp, pk, methods, args, args.steps, args.warmup)
    finally:
        for h in (bk, bp, pk):
            h.free()
    a = lines[args.method]
    st = a["st"]
    h2d = st["sdma_bytes"] + st["zc_bytes"]
    # dominant kernel: the probe stream (one launch per probe chunk, HIP events on its stream)
    k_avg = st["kernel_ms"] / max(1, st["chunks"])
    ach = (8.0 * np_ + 32.0 * st["survivors"]) / st["chunks"] / (k_avg * 1e6)
    alg = 16 * nb + 8 * np_
    return _common("probe rows/s", a["value"], a["ms"], args, "int64",
                   {"workload": "skewed_partitioned_join", "build_rows": nb, "probe_rows": np_, "zipf_s": 1.1,
                    "key_range": "[1, 2^40]", "device_budget_gib": args.skew_budget_gib,
                    "keys": "scrambled by a bijection of [0, 2^40)" if args.skew_scramble else "Zipf ranks",
                    "method": args.method, "n_parts": st["n_parts"]},
                   # the step waits on the host link: each build and probe column crosses it once
                   {"bound": "host_link",
                    "kernel": "whole step: splitters, pass-1 clustering of the build side, partition builds, "
                              "the probe stream",
                    "achieved": alg / (a["ms"] * 1e6), "peak": b_peak, "unit": "GB/s",
                    "frac": alg / (a["ms"] * 1e6) / b_peak, "traffic": h2d,
                    "peak_kind": "host-to-device copy rate measured in this run",
                    "algorithmic_bytes": "16 B per build row (key, payload) + 8 B per probe key, each read once",
                    "traffic_kind": "host-to-device bytes per step: copy-stream bytes + zero-copy bytes"},
                   {"hbm": {"kernel": "k_pj_stream", "achieved": ach, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                            "traffic_profile": PROFILE["k_pj_stream"], "avg_launch_ms": k_avg,
                            "rows_per_launch": np_ / st["chunks"],
                            "algorithmic_bytes": "8 B per probe key + 32 B table slot per probe row routed to a table"},
                    "host_link": {"peak_measured_gbs": b_peak, "h2d_bytes_per_step": h2d,
                                  "achieved_gbs": h2d / (a["ms"] * 1e6), "frac": h2d / (a["ms"] * 1e6) / b_peak},
                    "result": {"match_count": a["agg"][0], "sum": a["agg"][1]},
                    args.method: _skew_line(a),
                    "radix_hash": _skew_line(lines["radix_hash"]) if "radix_hash" in lines
                    else {"error": failed.get("radix_hash")},
                    "sample_quantile": _skew_line(lines["quantile"]) if "quantile" in lines
                    else {"error": failed.get("quantile")},
                    "speedup_vs_radix_hash": (lines["radix_hash"]["ms"] / a["ms"]) if "radix_hash" in lines
                    else None,
                    "bit_exact_across_methods": True})


def run_radix(args):
    """Two-table radix-partitioned join (the paper's hash-join case study): A and B of 2^29
    rows each, 16 B tuples <int64 key, int64 val> in pinned host memory (8 GiB per table),
    A.key unique (a permutation of [0, 2^29)), B.key a uniform foreign key into A; device budget
    4 GiB, so neither table's hash table fits; result = SUM(A.val + B.val) and the match count."""
    import numpy as np
    import torch
    import datagen
    import oracle
    import paper_2502_09541_amd as vx
    n = 1 << args.radix_log2
    ak, av, bk, bv = (vx.HostBuffer(n, np.int64) for _ in range(4))
    t0 = time.perf_counter()
    step_rows = 1 << 27
    for r0 in range(0, n, step_rows):
        m = min(step_rows, n - r0)
        datagen.radix_a(n, out=(ak.array[r0:r0 + m], av.array[r0:r0 + m]), row0=r0)
        datagen.radix_b(n, m, out=(bk.array[r0:r0 + m], bv.array[r0:r0 + m]), row0=r0)
    log(f"radix: inputs generated in {time.perf_counter() - t0:.1f} s")
    ctx = vx.Context(int(args.radix_budget_gib * GiB))
    cal = ctx.calibrate()
    ms, res = _timed(lambda: ctx.join_radix(ak, [av], bk, [bv]), args, torch)
    agg, st = res[0]
    log(f"radix: {ms:.1f} ms/step, {st['n_parts']} partitions, pass 1 {st['part_ms']:.1f} ms, "
        f"pass 2 {st['probe_ms']:.1f} ms, {st['chunks']} build slices")
    ctx.close()
    # exact check against the generator's closed form: every B row matches the one A row with its key
    a_of_key = np.empty(n, np.uint64)
    a_of_key[ak.array] = av.array.view(np.uint64)
    want = [n, int(a_of_key[bk.array].sum(dtype=np.uint64)), int(bv.array.view(np.uint64).sum(dtype=np.uint64))]
    del a_of_key
    if agg != want:
        raise SystemExit(f"radix join result {agg} differs from the closed form {want}")
    # the oracle on a bounded sample of the same workload: the rows of both tables whose key is
    # below n/16 (a key range, so the sample's join is the whole join restricted to those keys)
    cpu = cpu_all = None
    if not args.no_cpu_baseline:
        lim = n // 16
        ma, mb = ak.array < lim, bk.array < lim
        sak, sav, sbk, sbv = ak.array[ma], av.array[ma], bk.array[mb], bv.array[mb]
        t0 = time.perf_counter()
        got = oracle.join_agg(sak, [sav], sbk, [sbv])
        dt = time.perf_counter() - t0
        if got[0] != len(sbk):
            raise SystemExit("oracle sample: unexpected match count")
        cpu = {"value": (len(sak) + len(sbk)) / dt, "unit": "tuples/s", "cores": 1, "kind": "oracle",
               "sample": f"rows of A and B with key < 2^{args.radix_log2 - 4}: {len(sak)} + {len(sbk)} rows, "
                         f"joined in {dt:.1f} s on 1 host thread", **host_info()}
        # the same oracle on all host cores: the sample's key range cut into one range per thread
        # (each range's join is independent), the C calls run without the GIL
        from concurrent.futures import ThreadPoolExecutor
        n_thr = max(1, min(16, len(os.sched_getaffinity(0))))
        cuts = [lim * t // n_thr for t in range(n_thr + 1)]
        parts_a = [(sak >= cuts[t]) & (sak < cuts[t + 1]) for t in range(n_thr)]
        parts_b = [(sbk >= cuts[t]) & (sbk < cuts[t + 1]) for t in range(n_thr)]
        args_t = [(sak[parts_a[t]], sav[parts_a[t]], sbk[parts_b[t]], sbv[parts_b[t]]) for t in range(n_thr)]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(n_thr) as ex:
            outs = list(ex.map(lambda a: oracle.join_agg(a[0], [a[1]], a[2], [a[3]]), args_t))
        dt_all = time.perf_counter() - t0
        if [sum(x) % (1 << 64) for x in zip(*outs)] != got:
            raise SystemExit("threaded oracle run disagrees with the single-threaded one")
        cpu_all = {"value": (len(sak) + len(sbk)) / dt_all, "unit": "tuples/s", "cores": n_thr, "kind": "oracle",
                   "sample": f"the same sample cut into {n_thr} key ranges, one per thread, in {dt_all:.1f} s",
                   **host_info()}
    for h in (ak, av, bk, bv):
        h.free()
    tuples = 2 * n
    h2d = st["sdma_bytes"] + st["zc_bytes"]
    d2h = st["sdma_bytes"] if st["n_parts"] > 1 and st["zc_bytes"] > 0 else 0   # clustered copies written back
    # dominant kernel: the pass-2 probe (B's rows of a partition read in place from host memory)
    k_avg = st["kernel_ms"] / max(1, st["chunks"])
    rows_per_launch = n / max(1, st["chunks"])
    ach = 16.0 * rows_per_launch / (k_avg * 1e6)
    b_peak = cal["h2d_gbs"]
    # link-time model: pass 1 moves every tuple in and back out (both directions together at the
    # measured duplex rate of copies beside kernel stores to host), pass 2 reads them in again
    t_model = (2 * 16.0 * tuples) / (cal["duplex_zcw_gbs"] * 1e9) + 16.0 * tuples / (b_peak * 1e9)
    return _common("tuples/s", tuples / (ms / 1e3), ms, args, "int64",
                   {"workload": "two_table_radix_join", "rows_a": n, "rows_b": n, "tuple_bytes": 16,
                    "device_budget_gib": args.radix_budget_gib, "n_parts": st["n_parts"],
                    "partition_fn": "raw key bits [0, log2 n_parts)"},
                   {"bound": "host_link", "kernel": "k_rj_probe", "achieved": ach, "peak": b_peak, "unit": "GB/s",
                    "frac": ach / b_peak, "traffic": None, "traffic_profile": PROFILE["k_rj_probe"],
                    "avg_launch_ms": k_avg,
                    "rows_per_launch": rows_per_launch,
                    "algorithmic_bytes": "16 B per B row read in place from pinned host memory"},
                   {"cpu_baseline": cpu, "cpu_baseline_all_cores": cpu_all,
                    "host_link": {"h2d_peak_measured_gbs": b_peak, "duplex_measured_gbs": cal["duplex_zcw_gbs"],
                                  "h2d_bytes_per_step": h2d, "d2h_bytes_per_step": d2h,
                                  "h2d_gbs": h2d / (ms * 1e6), "d2h_gbs": d2h / (ms * 1e6),
                                  "model_ms": t_model * 1e3, "frac_of_model": t_model * 1e3 / ms},
                    "phases": {"pass1_ms": st["part_ms"], "pass2_ms": st["probe_ms"],
                               "pass2_build_kernels_ms": st["build_ms"], "pass2_probe_kernels_ms": st["kernel_ms"],
                               "build_slices": st["chunks"], "imbalance": st["imbalance"]},
                    "result": {"match_count": agg[0], "sum_a_val": agg[1], "sum_b_val": agg[2],
                               "sum_a_plus_b": (agg[1] + agg[2]) % (1 << 64)},
                    "probe_rows_per_s": n / (ms / 1e3), "bit_exact_closed_form": True})


def _fill_sort_keys(h, n):
    import datagen
    step = 1 << 27
    for r0 in range(0, n, step):
        m = min(step, n - r0)
        datagen.sort_keys(m, out=h.array[r0:r0 + m], row0=r0)


def _sort_checks(a):
    """(sorted?, sum mod 2^64, xor) of an int64 array, in slices."""
    import numpy as np
    ok, s, x, prev = True, 0, 0, None
    step = 1 << 27
    for r0 in range(0, len(a), step):
        v = a[r0:r0 + step]
        u = v.view(np.uint64)
        ok = ok and bool(np.all(v[1:] >= v[:-1])) and (prev is None or prev <= v[0])
        prev = v[-1]
        s = (s + int(u.sum(dtype=np.uint64))) % (1 << 64)
        x ^= int(np.bitwise_xor.reduce(u))
    return ok, s, x


def run_sort(args):
    """Out-of-core sort (the paper's sort case study): 2^31 int64 keys uniform over all values in
    pinned host memory (16 GiB), device budget 4 GiB; sorted in place.  Every step sorts the same
    freshly generated input (generation is outside the timed region)."""
    import numpy as np
    import torch
    import oracle
    import paper_2502_09541_amd as vx
    n = 1 << args.sort_log2
    h = vx.HostBuffer(n, np.int64)
    _fill_sort_keys(h, n)
    ok, s_in, x_in = _sort_checks(h.array)
    ctx = vx.Context(int(args.sort_budget_gib * GiB))
    cal = ctx.calibrate()
    times, st = [], None
    for i in range(args.warmup + args.steps):
        if i:
            _fill_sort_keys(h, n)
        torch.cuda.synchronize()
        with gc_paused():
            t0 = time.perf_counter()
            st = ctx.sort(h)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) * 1e3
        if i >= args.warmup:
            times.append(dt)
        log(f"sort step {i}: {dt:.1f} ms (pass 1 {st['part_ms']:.1f}, pass 2 {st['probe_ms']:.1f}, "
            f"{st['chunks']} runs of {st['chunk_rows']})")
    ctx.close()
    ok, s_out, x_out = _sort_checks(h.array)
    if not ok or (s_out, x_out) != (s_in, x_in):
        raise SystemExit("sort output is not the sorted input")
    ms = sum(times) / len(times)
    cpu = None
    if not args.no_cpu_baseline:
        m = n // 16
        sample = np.empty(m, np.int64)
        import datagen
        datagen.sort_keys(m, out=sample)
        t0 = time.perf_counter()
        got = oracle.sort(sample)
        dt = time.perf_counter() - t0
        if not bool(np.all(got[1:] >= got[:-1])):
            raise SystemExit("oracle sample not sorted")
        cpu = {"value": m / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {m} keys of the same generator (1/16), std::sort in {dt:.1f} s on 1 host thread",
               **host_info()}
    h.free()
    runs = st["chunks"]
    # Both passes move every key in and back out over the link at the rate measured for copies in
    # beside kernel stores out: the step is bound by the link.  The GPU's own work, the radix sort
    # of a run (8 digit passes, HIP events), is reported beside it against HBM.
    k_avg = st["kernel_ms"] / max(1, runs)
    rows = st["chunk_rows"]
    ach_hbm = 8 * 24.0 * rows / (k_avg * 1e6)       # per pass: histogram read 8 B, scatter 8 B in + 8 B out
    b_peak = cal["h2d_gbs"]
    duplex = cal["duplex_zcw_gbs"]
    link_bytes = 2 * 2 * 8.0 * n                    # each pass: every key in and back out
    t_model = link_bytes / (duplex * 1e9)
    return _common("keys/s", n / (ms / 1e3), ms, args, "int64",
                   {"workload": "out_of_core_sort", "keys": n, "key_bytes": 8, "distribution": "uniform over int64",
                    "device_budget_gib": args.sort_budget_gib, "runs": runs, "run_keys": rows},
                   {"bound": "host_link", "kernel": "whole step: runs copied in, sorted and stored out (k_store), "
                    "ranges copied in, merged and stored out", "achieved": link_bytes / (ms * 1e6), "peak": duplex,
                    "unit": "GB/s", "frac": link_bytes / (ms * 1e6) / duplex, "traffic": link_bytes,
                    "peak_kind": "copies in beside kernel stores out, measured in this run",
                    "algorithmic_bytes": "per step: 16 B per key in each of the two passes (8 B in, 8 B out)",
                    "hbm_radix_run": {"achieved": ach_hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": ach_hbm / HBM_PEAK_GBS, "avg_launch_ms": k_avg, "rows_per_launch": rows,
                                      "kernels": "8 digit passes of k_digit_hist, the three-launch scan, k_digit_scatter",
                                      "traffic_profile": PROFILE["sort_run"],
                                      "algorithmic_bytes": "24 B per key per digit pass (8 B histogram read, 8 B read + 8 B written by the scatter), 8 passes"}},
                   {"cpu_baseline": cpu,
                    "host_link": {"h2d_peak_measured_gbs": b_peak, "duplex_measured_gbs": cal["duplex_zcw_gbs"],
                                  "link_bytes_per_step": link_bytes, "model_ms": t_model * 1e3,
                                  "frac_of_model": t_model * 1e3 / ms},
                    "phases": {"pass1_ms": st["part_ms"], "pass2_ms": st["probe_ms"], "sort_kernels_ms": st["kernel_ms"],
                               "merge_kernels_ms": st["build_ms"], "runs": runs},
                    "bit_exact": "sorted, same sum mod 2^64 and xor as the input"})


if __name__ == "__main__":
    main()
