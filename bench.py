#!/usr/bin/env python3
"""Benchmarks of the temporal component-matrix library on one MI355X.

Default (--mode exact): one step = one pass of the exact path over the
resident schedule of one network: C <- I, every level of reverse-time row
ORs, then the out- and in-component sizes.  The workload is the
activity-driven network with n = 100,000 nodes and m = 10,000,000 events
(T = 10^6 ticks).  Events, schedule and matrix are in HBM when the timed
region starts; host planning time is reported separately.  Beside the step:
the plain recurrence on the same plan (saturation off; its launch gives the
roofline), and the hashed block: the n = 10^6, m = 10^8 stream with H = 16
end to end at K = 4096, all proxies at K = 65,536 in one launch, and fusion
timed where it intersects (--no-hashed skips it).

Other modes (each prints its own single JSON line):
  --mode hashed    n = 10^6, m = 10^8 activity-driven, H = 16 hashes to
                   K = 4096 super-nodes: all proxies in one persistent launch,
                   then the fusion estimator.
  --mode batched   256 uneven networks (n log-uniform in [500, 20000], m in
                   [10^4, 10^6], uniform-pair and activity-driven) in one
                   persistent autotuned launch under a HIP graph, against
                   the plain kernel run network by network.
  --mode combiner  the learned combiner trained on 64 networks (n = 20,000,
                   m = 10^6) and evaluated on 4 held-out networks
                   (n = 100,000, m = 10^7) against the exact sizes, beside the
                   fusion estimate and the smallest lifted size.
  --mode hll       the HyperLogLog stream at n = 10^6, m = 10^8 (2^b one-byte
                   registers per node instead of n bits), with its accuracy
                   against the exact sizes at n = 10^5, m = 10^7.
  --mode sweep     the paper's synthetic experiment: ER G(n, 2/n) with a
                   Poisson process per link, n from 100 to 10^4 and m from
                   10^4 to 10^7, exact against hashed (H = 5, n_s = 0.3 n):
                   Earth-Mover distance, relative time and memory.
  --mode fusion    fusion alone, on 2*10^5 nodes whose proxy rows are mostly
                   not full (the hashed block's fusion timing).
  --mode online    forward time with online insertion: the n = 10^5,
                   m = 10^7 events in time order, in batches, into a live
                   matrix of in-components, against the resident forward
                   plan (bit for bit).

Each line carries the roofline of the mode's dominant kernel, timed with HIP
events on the stream it runs on, and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# LDS: 256 CUs x 128 bytes per clock x 2.4 GHz
LDS_PEAK_GBS = 256 * 128 * 2.4
METRIC = "events/s (exact & hashed) + % HBM roofline; combiner rel. err vs exact"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2307_04890_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# the kernels of one saturating launch on a network of 16,384+ nodes: the
# zero phase, the forwarding phase, the slice state, the saturating rest
ROWOR_SAT_KERNELS = "k_rowor_global|k_rowor_fwd|k_slice_full_state|k_slice_order"
KERNEL_SOURCES = {"rowor": ("tn_kernels.hip", "tn_internal.h", "tn_device.h", "tn_plan.cpp"),
                  "rowor_plain": ("tn_kernels.hip", "tn_internal.h", "tn_device.h", "tn_plan.cpp"),
                  "batch": ("tn_batch.hip", "tn_batch.h", "tn_batch.cpp", "tn_internal.h"),
                  "recombine": ("tn_hash.hip", "tn_hash.h")}


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counters
    (profiles/<kernel>_<workload>_pmc.json), if they were taken on the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != kernel_source_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("hbm_bytes_per_launch")


def algorithmic_bytes(st: dict, n: int) -> float:
    """Row transfers the definition needs: an undirected pair reads and writes
    two rows (4), a one-way pair reads two and writes one (3), a compound
    gather reads its sources and writes its target; plus the schedule once."""
    row = 8.0 * ((n + 63) // 64)
    sym = st["pairs"] - st["directed_pairs"]
    rows = 4.0 * sym + 3.0 * st["directed_pairs"] + st["gather_sources"] + st["gathers"]
    sched = 8.0 * st["pairs"] + 4.0 * (2 * st["gathers"] + 1 + st["gather_sources"]) \
        + 8.0 * (st["levels"] + 1)
    return rows * row + sched


def base_result(args, value, unit, steps, ms_per_step, config, dtype="u64"):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config}


def timed(ctx, fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    recs = ctx.profile_take()
    ctx.profile(False)
    per = {}
    for name, ms in recs:
        per.setdefault(name, []).append(ms)
    return elapsed, {k: sum(v) / len(v) for k, v in per.items()}, per


# ---------------------------------------------------------------------------
def cpu_baseline_exact(n, s, d, t, budget_s: float, forward: bool = False):
    import oracle
    recurrence = oracle.forward_matrix if forward else oracle.reverse_matrix
    what = "forward-time" if forward else "reverse-time"
    nwords = (n + 63) // 64
    t0 = time.perf_counter()
    recurrence(n, s, d, t, w0=0, nw=min(16, nwords))
    probe = time.perf_counter() - t0
    k = min(nwords, max(16, int(16 * budget_s / max(probe, 1e-3))))
    t0 = time.perf_counter()
    recurrence(n, s, d, t, w0=0, nw=k)
    dt = time.perf_counter() - t0
    full_equiv = dt * nwords / k
    rec = {"value": s.shape[0] / full_equiv, "unit": "events/s", "cores": 1, "kind": "oracle",
           "sample": f"{what} recurrence on word columns [0,{k}) of {nwords} "
                     f"({100.0 * k / nwords:.1f}% of the matrix), all {s.shape[0]} events; "
                     f"{dt:.2f} s single-threaded, scaled to the full width",
           "seconds": dt, "host_nproc": os.cpu_count()}
    # the same oracle on every host core: word columns are independent, so
    # each thread runs it on its own column range (the calls release the GIL)
    import concurrent.futures as cf
    threads = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16"))))
    ka = min(nwords, k * threads)
    cuts = [ka * i // threads for i in range(threads + 1)]
    parts = [(cuts[i], cuts[i + 1] - cuts[i]) for i in range(threads) if cuts[i + 1] > cuts[i]]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(len(parts)) as ex:
        list(ex.map(lambda p: recurrence(n, s, d, t, w0=p[0], nw=p[1]), parts))
    dta = time.perf_counter() - t0
    rec["all_cores"] = {"value": s.shape[0] / (dta * nwords / ka), "unit": "events/s",
                        "cores": len(parts), "kind": "oracle",
                        "sample": f"word columns [0,{ka}) of {nwords} split over {len(parts)} "
                                  f"threads; {dta:.2f} s wall, scaled to the full width",
                        "seconds": dta}
    return rec


def counter_roofline(traffic, ms, kernel, dense, dense_gbs, rows_in):
    """Roofline of a launch that skips saturated rows: the HBM bytes rocprofv3
    counted per launch (FETCH_SIZE + WRITE_SIZE, committed profile of the
    same kernel source) over its mean time.  The plain recurrence's bytes
    are no measure of such a launch (most rows are never moved), so they are
    reported apart, as a dense equivalent."""
    achieved = traffic / (ms * 1e-3) / 1e9 if traffic else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
            "kernel": kernel, "avg_launch_ms": ms, "rows_in": rows_in,
            "basis": "counted HBM bytes per launch / mean launch time (saturated rows are "
                     "skipped; null when no profile of the current source is committed)",
            "dense_equivalent": {"bytes": dense, "GBs": dense_gbs,
                                 "note": "the plain recurrence's row transfers over the same "
                                         "time: not a bandwidth, it exceeds the peak"}}


def run_exact(args):
    import numpy as np
    import torch

    import paper_2307_04890_amd as tn
    import tn_inputs as T

    workload = args.workload or "activity_n100000_m10M"
    spec = T.WORKLOADS[workload]
    n = spec["n"]
    log(f"[bench] generating {workload}")
    s, d, t = T.make_workload(workload)
    m = int(s.shape[0])
    log("[bench] planning on the host")
    t0 = time.perf_counter()
    plan = tn.Plan(n, s, d, t)
    plan_wall = time.perf_counter() - t0
    st = plan.stats
    log(f"[bench] plan: {st['levels']} levels, {st['pairs']} pairs, {st['gathers']} gathers, "
        f"{st['host_seconds']:.2f} s host")
    ctx = tn.get_context()
    C = tn.api.alloc_matrix(n)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    inn = torch.empty(n, dtype=torch.int32, device="cuda")
    cp = tn.api._dp

    def step():
        # the row-OR, then the sizes from the matrix and the slice state the
        # execution left (slices left all ones are counted without a read)
        tn._lib.check(tn.lib.tn_plan_execute_sizes(ctx.bind_stream(), plan.h, cp(C), C.stride(0),
                                                   int(args.slice_words), cp(out), cp(inn)))

    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib)
    elapsed, kms, _ = timed(ctx, step, args.steps, args.warmup)
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s")
    alg = algorithmic_bytes(st, n)
    # what the saturating kernel actually had to move: its own counters of
    # row words loaded and stored (saturated rows skipped), plus the schedule
    ld_w, st_w = ctx.last_traffic()
    moved = 8.0 * (ld_w + st_w) + 16.0 * st["ops"] + 4.0 * (st["op_levels"] + 1)
    o, i = out.cpu().numpy(), inn.cpu().numpy()
    assert o.sum() == i.sum(), "sum of out-sizes differs from sum of in-sizes"
    # the plain leg: the same plan with saturation off, so that every op moves
    # its rows (the forwarded kernel); its launches give the roofline
    if args.no_plain:
        pkms, pper, pld, pst = {"rowor": float("nan")}, {}, 0, 0
    else:
        ctx.saturation(False)
        try:
            p_elapsed, pkms, pper = timed(ctx, lambda: plan.execute(C, slice_words=args.slice_words),
                                          max(2, args.steps // 2), 1)
            pld, pst = ctx.last_traffic()
        finally:
            ctx.saturation(True)
        # (the tests compare whole matrices; here the sizes of both legs)
        tn._lib.check(tn.lib.tn_component_sizes(ctx.bind_stream(), n, cp(C), C.stride(0), cp(out),
                                                cp(inn)))
        assert np.array_equal(out.cpu().numpy(), o) and np.array_equal(inn.cpu().numpy(), i), \
            "plain recurrence differs from the saturating kernel"
    plain_ms = pkms["rowor"]
    achieved = alg / (plain_ms * 1e-3) / 1e9
    plain_traffic = load_traffic("rowor_plain", workload)
    sat_ms = kms["rowor"]
    sat_traffic = load_traffic("rowor", workload)
    config = {"workload": workload, "n": n, "m": m, "T": spec["T"], "generator": spec["kind"],
              "seed": spec["seed"], "flags": "undirected,strict-ties", "ld_words": C.stride(0),
              "slice_words": args.slice_words or "auto", "parallelism": "single-gpu"}
    r = base_result(args, m * args.steps / elapsed, "events/s", args.steps,
                    1e3 * elapsed / args.steps, config)
    r["value_note"] = ("one step = identity + the saturating row-OR kernel (rows that are all "
                       "ones in a column slice are not moved again; the matrix is bit-identical "
                       "to the plain recurrence) + out- and in-sizes (tn_plan_execute_sizes: "
                       "the columns of slices the execution left all ones are counted from its "
                       "slice state, the rest from the matrix)")
    r["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": plain_traffic,
                     "kernel": "k_rowor_fwd (the plain recurrence, saturation off: every op "
                               "applied, each level's results forwarded through LDS)",
                     "algorithmic_bytes": alg, "avg_launch_ms": plain_ms,
                     "traffic_frac": (plain_traffic / (plain_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                      if plain_traffic else None),
                     "row_bytes_moved": 8.0 * (pld + pst),
                     "note": "algorithmic bytes = 4 row transfers per undirected pair (the "
                             "plain recurrence) + the schedule once, over the mean launch time; "
                             "traffic = rocprofv3 FETCH_SIZE + WRITE_SIZE per launch"}
    r["plain"] = {"events_per_s": m / (plain_ms * 1e-3), "avg_launch_ms": plain_ms,
                  "launch_ms_all": pper.get("rowor", []),
                  "row_words_loaded": pld, "row_words_stored": pst}
    if args.no_plain:
        r["roofline"] = r["plain"] = None
    r["saturating"] = {"kernel": "k_rowor_global zero phase, k_rowor_fwd until the ops reach "
                                 "9 n, k_slice_full_state and k_slice_order on narrower "
                                 "slices, k_rowor_global for the rest",
                       "avg_launch_ms": sat_ms, "moved_bytes": moved,
                       "moved_achieved": moved / (sat_ms * 1e-3) / 1e9,
                       "moved_frac": moved / (sat_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "traffic": sat_traffic,
                       "traffic_frac": (sat_traffic / (sat_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                        if sat_traffic else None),
                       "dense_equivalent_frac": alg / (sat_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "dense_equivalent_note": "the plain recurrence's bytes over the "
                                                "saturating launch: not a bandwidth (saturated "
                                                "rows are skipped), so it exceeds 1",
                       "levels": st["op_levels"],
                       "us_per_level": 1e3 * sat_ms / max(1, st["op_levels"])}
    r["kernels_ms"] = kms
    r["plan"] = {"levels": st["levels"], "op_levels": st["op_levels"], "ops": st["ops"],
                 "pairs": st["pairs"], "gathers": st["gathers"],
                 "host_seconds": st["host_seconds"], "wall_seconds": plan_wall,
                 "end_to_end_events_per_s": m / (st["host_seconds"] + 1e-3 * sum(kms.values()))}
    r["mean_out_size"] = float(o.mean())
    # the whole job from host events: streamed one-shot build (planning on
    # host threads overlapped with the device, stop at saturation) + sizes
    plan.close()
    if args.no_end_to_end:
        return r
    ee = []
    for rep in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C2, sst = tn.build_component_matrix_streamed(n, s, d, t, C=C)
        tn._lib.check(tn.lib.tn_component_sizes(ctx.bind_stream(), n, cp(C2), C2.stride(0),
                                                cp(out), cp(inn)))
        torch.cuda.synchronize()
        ee.append(time.perf_counter() - t0)
    assert np.array_equal(out.cpu().numpy(), o), "streamed build differs from the plan"
    r["end_to_end"] = {"events_per_s": m / min(ee), "seconds": min(ee), "seconds_all": ee,
                       "what": "host events -> streamed build (host planning overlapped with "
                               "the device, stop once every slice is full) -> sizes",
                       "stream": sst}
    del C, C2
    torch.cuda.empty_cache()
    if not args.no_hashed:
        r["hashed"] = hashed_block(args)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a column sample")
        r["cpu_baseline"] = cpu_baseline_exact(n, s, d, t, args.cpu_budget)
    return r


def run_online(args):
    """Forward-time streaming with online insertion (Sec. 3.5): the events of
    the 10^5-node workload arrive in time order, in batches, into a live
    matrix whose rows are in-components; against the resident forward plan
    (Algorithm 1 as printed, Sec. 3.1), bit for bit."""
    import numpy as np
    import torch

    import paper_2307_04890_amd as tn
    import tn_inputs as T

    workload = args.workload or "activity_n100000_m10M"
    spec = T.WORKLOADS[workload]
    n = spec["n"]
    log(f"[bench] generating {workload}")
    s, d, t = T.make_workload(workload)
    m = int(s.shape[0])
    ctx = tn.get_context()
    log("[bench] forward plan on the host")
    t0 = time.perf_counter()
    plan = tn.Plan(n, s, d, t, flags=tn.FORWARD)
    plan_wall = time.perf_counter() - t0
    st = plan.stats
    C = tn.api.alloc_matrix(n)
    elapsed, kms, _ = timed(ctx, lambda: plan.execute(C), args.steps, args.warmup)
    alg = algorithmic_bytes(st, n)
    # the plain leg (saturation off: every op moves its rows) gives the roofline
    ctx.saturation(False)
    try:
        C0 = tn.api.alloc_matrix(n)
        _, pkms, _ = timed(ctx, lambda: plan.execute(C0), max(2, args.steps // 2), 1)
        pld, pst = ctx.last_traffic()
    finally:
        ctx.saturation(True)
    assert torch.equal(C0, C), "plain forward recurrence differs from the saturating kernel"
    del C0
    achieved = alg / (pkms["rowor"] * 1e-3) / 1e9
    plan.close()
    # batch boundaries at the first event of a time step (a batch starts
    # strictly after the last time step applied)
    B = max(1, args.online_batches)
    cuts = [0] + [int(np.searchsorted(t, t[m * k // B], side="left")) for k in range(1, B)] + [m]
    cuts = sorted(set(cuts))
    C2 = tn.api.alloc_matrix(n)
    runs = []
    for rep in range(2):
        on = tn.Online(n, flags=tn.FORWARD, C=C2)
        lat, stats = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in zip(cuts[:-1], cuts[1:]):
            t1 = time.perf_counter()
            stats.append(on.insert(s[a:b], d[a:b], t[a:b]))
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t1)
        total = time.perf_counter() - t0
        on.close()
        runs.append((total, lat, stats))
    assert torch.equal(C2, C), "online insertion differs from the forward plan"
    total, lat, stats = min(runs, key=lambda x: x[0])
    config = {"workload": workload + "_forward_online", "n": n, "m": m, "T": spec["T"],
              "generator": spec["kind"], "seed": spec["seed"], "batches": len(cuts) - 1,
              "flags": "forward,undirected,strict-ties", "parallelism": "single-gpu"}
    r = base_result(args, m / total, "events/s", len(cuts) - 1, 1e3 * total / (len(cuts) - 1),
                    config)
    r["value_note"] = ("online insertion end to end from host events: every batch planned on "
                       "host threads and applied to the live matrix (one step = one batch)")
    r["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_rowor_fwd on the resident forward plan, saturation off "
                               "(every op applied)",
                     "algorithmic_bytes": alg, "avg_launch_ms": pkms["rowor"],
                     "row_bytes_moved": 8.0 * (pld + pst),
                     "saturating_launch_ms": kms["rowor"], "levels": st["op_levels"]}
    r["kernels_ms"] = kms
    r["forward_plan"] = {"events_per_s": m * args.steps / elapsed, "levels": st["levels"],
                         "op_levels": st["op_levels"], "ops": st["ops"],
                         "host_seconds": st["host_seconds"], "wall_seconds": plan_wall}
    r["online"] = {"seconds": total, "seconds_all": [x[0] for x in runs],
                   "batch_latency_ms": [1e3 * x for x in lat],
                   "batches": [{k: v for k, v in x.items() if k != "seconds"} for x in stats]}
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a column sample")
        r["cpu_baseline"] = cpu_baseline_exact(n, s, d, t, args.cpu_budget, forward=True)
    return r


def calibrate_copy(mib):
    import torch
    nbytes = mib << 20
    a = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy: {nbytes} bytes read, {nbytes} bytes written")


# ---------------------------------------------------------------------------
def run_hashed(args):
    import numpy as np
    import torch

    import paper_2307_04890_amd as tn
    import tn_inputs as T

    workload = args.workload or "activity_n1M_m100M"
    spec = T.WORKLOADS[workload]
    n, H, K = spec["n"], args.hashes, args.buckets
    log(f"[bench] generating {workload}")
    s, d, t = T.make_workload(workload)
    m = int(s.shape[0])
    A = T.hash_coefficients(H, seed=1003)
    ctx = tn.get_context()
    ctx.profile(True)
    t0 = time.perf_counter()
    bucket, count, proxies = tn.hash_compress(n, s, d, t, A, K)
    torch.cuda.synchronize()
    compress_wall = time.perf_counter() - t0
    hash_ms = sum(ms for k, ms in ctx.profile_take() if k == "hash")
    ctx.profile(False)
    stats, tiles, lds_tiles = proxies.stats()
    log(f"[bench] hashed and planned {H} proxies in {compress_wall:.2f} s; {tiles} tiles "
        f"({lds_tiles} in LDS); levels per proxy {np.mean([x['levels'] for x in stats]):.0f}")
    ldK = tn.words(K)
    P = torch.empty((H, K, ldK), dtype=torch.int64, device="cuda")
    Ps = [P[j] for j in range(H)]
    t0 = time.perf_counter()
    proxies.execute(Ps)  # tunes the tile shape, captures the graph
    torch.cuda.synchronize()
    tune_wall = time.perf_counter() - t0
    _, tiles, lds_tiles = proxies.stats()  # of the tuned shape
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib)

    def step():
        proxies.execute(Ps)
        tn.recombine(P, bucket, count, n)

    elapsed, kms, per = timed(ctx, step, args.steps, args.warmup)
    est, lifted = tn.recombine(P, bucket, count, n)
    proxy_ms = kms["batch"]
    rec_ms = sum(float(np.sum(v)) for k, v in per.items() if k in ("recombine", "aux")) / args.steps
    dense = sum(algorithmic_bytes(x, K) for x in stats)
    achieved = dense / (proxy_ms * 1e-3) / 1e9
    config = {"workload": workload, "n": n, "m": m, "T": spec["T"], "generator": spec["kind"],
              "seed": spec["seed"], "H": H, "K": K, "hash_seed": 1003,
              "flags": "undirected,strict-ties", "parallelism": "single-gpu"}
    r = base_result(args, m / (proxy_ms * 1e-3), "events/s", args.steps,
                    1e3 * elapsed / args.steps, config)
    r["value_note"] = "m / time of the one launch that builds all H proxies"
    # where the proxy rows live in the tuned shape: LDS-resident slices
    # (K = 4096), or global-memory tiles streaming through L2 and HBM
    lds_bound = 2 * lds_tiles >= tiles
    pmc_key = f"{workload}_K{K}"
    r["roofline"] = counter_roofline(load_traffic("batch", pmc_key), proxy_ms,
                                     "k_batch_persistent", dense, achieved,
                                     "lds" if lds_bound else "global")
    r["hashed"] = {"H_times_m_events_per_s": H * m / (proxy_ms * 1e-3),
                   "recombine_ms": rec_ms,
                   "end_to_end_ms": 1e3 * compress_wall + proxy_ms + rec_ms,
                   "hash_kernel_ms": hash_ms, "host_compress_wall_s": compress_wall,
                   "autotune_and_capture_s": tune_wall, "tiles": tiles, "lds_tiles": lds_tiles,
                   "shape": proxies.shape(),
                   "mean_estimate": float(est.float().mean().item())}
    r["kernels_ms"] = kms
    if args.no_end_to_end:
        return r
    # the whole job from host events: hashing, the streamed proxy build
    # (chunks planned on host threads, stop once every tile is full), fusion
    P2 = torch.empty_like(P)
    ee = []
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b2, c2, P2, sst = tn.hash_build_proxies(n, s, d, t, A, K, P=P2)
        est2, _ = tn.recombine(P2, b2, c2, n)
        torch.cuda.synchronize()
        ee.append(time.perf_counter() - t0)
    assert torch.equal(P2, P) and torch.equal(est2, est), "streamed proxies differ"
    r["end_to_end"] = {"events_per_s": m / min(ee), "seconds": min(ee), "seconds_all": ee,
                       "what": "host events -> hash -> streamed proxy build -> fusion",
                       "stream": sst}
    if not args.no_cpu_baseline:
        import oracle
        log("[bench] timing the CPU oracle on one proxy column slice")
        b0 = bucket[0].cpu().numpy().view(np.uint32)
        hs, hd = b0[s], b0[d]
        nwk = tn.words(K)
        t0 = time.perf_counter()
        oracle.reverse_matrix(K, hs, hd, t, w0=0, nw=1)
        dt = time.perf_counter() - t0
        full = dt * nwk * H
        r["cpu_baseline"] = {"value": m / full, "unit": "events/s", "cores": 1, "kind": "oracle",
                             "sample": f"proxy 0 of {H}, word column 0 of {nwk}, all {m} events; "
                                       f"{dt:.2f} s single-threaded, scaled by {nwk * H}",
                             "seconds": dt, "host_nproc": os.cpu_count()}
    proxies.close()
    return r


# ---------------------------------------------------------------------------
FUSION_WORKLOAD = "fusion_activity_n200000_m40000_K4096"


def fusion_timing(args):
    """Fusion (Sec. 4.2) timed where it intersects: 2*10^5 nodes, 4*10^4
    activity-driven events, H = 16 hashes to K = 4096 super-nodes, so that
    proxy rows are mostly not full and every estimate is below n.  The
    AND/popcount kernel reads one word per (node, chunk of 64 nodes, hash)
    from the lifted tables it stages in LDS: its algorithmic bytes are
    8 * nlist * ceil(n/64) * H for the nlist nodes whose rows are not full
    in every hash."""
    import numpy as np
    import torch

    import paper_2307_04890_amd as tn
    import tn_inputs as T

    n, m, Tm, H, K = 200_000, 40_000, 400_000, 16, 4096
    s, d, t = T.activity_driven(n, m, Tm, seed=K + H)
    A = T.hash_coefficients(H, seed=K + 1)
    ctx = tn.get_context()
    bucket, count, P, _ = tn.hash_build_proxies(n, s, d, t, A, K)
    # nodes whose proxy rows are full in every hash skip the AND (est = n)
    Ph = P.cpu().numpy().view(np.uint64)[:, :, :tn.words(K)]
    full_rows = (Ph == np.uint64(0xFFFFFFFFFFFFFFFF)).all(axis=2)
    bh = bucket.cpu().numpy().view(np.uint32)
    node_full = full_rows[np.arange(H)[:, None], bh].all(axis=0)
    nlist = int(n - node_full.sum())
    nq = (n + 63) // 64
    and_bytes = 8.0 * nlist * nq * H
    elapsed, kms, per = timed(ctx, lambda: tn.recombine(P, bucket, count, n), 3, 1)
    est, _ = tn.recombine(P, bucket, count, n)
    e = est.cpu().numpy()
    est_ms = float(np.sum(per.get("recombine", [0.0]))) / 3
    aux_ms = float(np.sum(per.get("aux", [0.0]))) / 3
    traffic = load_traffic("recombine", FUSION_WORKLOAD)
    return {"workload": FUSION_WORKLOAD, "n": n, "m": m, "T": Tm, "H": H, "K": K,
            "nodes_not_full": nlist, "estimates_below_n": float((e < n).mean()),
            "mean_estimate": float(e.mean()),
            "call_ms": 1e3 * elapsed / 3, "recombine_est_ms": est_ms, "other_kernels_ms": aux_ms,
            "and_bytes": and_bytes, "bound": "lds",
            "achieved_GBs": and_bytes / (est_ms * 1e-3) / 1e9,
            "frac": and_bytes / (est_ms * 1e-3) / 1e9 / LDS_PEAK_GBS,
            "traffic": traffic,
            "traffic_frac": (traffic / (est_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None),
            "note": "k_recombine_est: the AND words come from lifted tables staged in LDS "
                    "(LDS peak 256 CU x 128 B/clk x 2.4 GHz); traffic = rocprofv3 FETCH_SIZE + "
                    "WRITE_SIZE of its dispatches, against HBM"}


def hashed_block(args):
    """The hashed half of the metric (Sec. 4.3) in the default run: the
    10^6-node, 10^8-event activity-driven stream hashed with H = 16, (a) end
    to end from host events at K = 4096 (hash, streamed proxy build, fusion),
    (b) all 16 proxies at K = 65,536 in one launch (8 GiB of proxies, HBM
    bound), and (c) fusion timed where it intersects."""
    import numpy as np
    import torch

    import paper_2307_04890_amd as tn
    import tn_inputs as T

    out = {}
    wl = "activity_n1M_m100M"
    spec = T.WORKLOADS[wl]
    n, H = spec["n"], 16
    log(f"[bench] generating {wl}")
    t0 = time.perf_counter()
    s, d, t = T.make_workload(wl, progress=lambda msg: log(f"[bench] {wl}: {msg}"))
    out["generate_s"] = time.perf_counter() - t0
    m = int(s.shape[0])
    A = T.hash_coefficients(H, seed=1003)
    ctx = tn.get_context()
    K = 4096
    P = torch.empty((H, K, tn.words(K)), dtype=torch.int64, device="cuda")
    ee = []
    for rep in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bucket, count, P, sst = tn.hash_build_proxies(n, s, d, t, A, K, P=P)
        est, _ = tn.recombine(P, bucket, count, n)
        torch.cuda.synchronize()
        ee.append(time.perf_counter() - t0)
    out["end_to_end_K4096"] = {
        "workload": wl, "n": n, "m": m, "H": H, "K": K, "hash_seed": 1003,
        "events_per_s": m / min(ee), "seconds": min(ee), "seconds_all": ee,
        "what": "host events -> hash -> streamed proxy build -> fusion", "stream": sst,
        "mean_estimate": float(est.float().mean().item())}
    del P, bucket, count, est
    log("[bench] hashed: the K = 65536 proxies in one launch")
    K = 65536
    t0 = time.perf_counter()
    bucket, count, proxies = tn.hash_compress(n, s, d, t, A, K)
    torch.cuda.synchronize()
    compress_s = time.perf_counter() - t0
    stats, _, _ = proxies.stats()
    P = torch.empty((H, K, tn.words(K)), dtype=torch.int64, device="cuda")
    Ps = [P[j] for j in range(H)]
    proxies.execute(Ps)  # tunes the tile shape, captures the graph
    _, tiles, lds_tiles = proxies.stats()
    elapsed, kms, per = timed(ctx, lambda: proxies.execute(Ps), 3, 0)
    pms = kms["batch"]
    dense = sum(algorithmic_bytes(x, K) for x in stats)
    traffic = load_traffic("batch", f"{wl}_K{K}")
    out["proxies_K65536"] = {
        "workload": wl, "H": H, "K": K, "kernel": "k_batch_persistent (global-memory tiles)",
        "events_per_s": m / (pms * 1e-3), "H_times_m_events_per_s": H * m / (pms * 1e-3),
        "avg_launch_ms": pms, "launch_ms_all": per.get("batch", []), "traffic": traffic,
        "traffic_frac": traffic / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
        "dense_equivalent_bytes": dense,
        "dense_equivalent_frac": dense / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "dense_equivalent_note": "row transfers of the plain recurrence on the 16 proxy streams; "
                                 "saturated rows are skipped, so not a bandwidth",
        "tiles": tiles, "lds_tiles": lds_tiles, "host_hash_and_plan_s": compress_s}
    proxies.close()
    del P, Ps, bucket, count
    torch.cuda.empty_cache()
    log("[bench] hashed: fusion where it intersects")
    out["fusion"] = fusion_timing(args)
    return out


def run_fusion(args):
    """--mode fusion: the fusion timing alone (for profiles of its kernels)."""
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib)
    f = fusion_timing(args)
    config = {"workload": f["workload"], "n": f["n"], "m": f["m"], "T": f["T"], "H": f["H"],
              "K": f["K"], "generator": "activity", "parallelism": "single-gpu"}
    r = base_result(args, f["n"] / (f["call_ms"] * 1e-3), "nodes/s", 3, f["call_ms"], config)
    r["value_note"] = "fusion estimates of every node per second (one tn_recombine call)"
    r["roofline"] = {"bound": "lds", "achieved": f["achieved_GBs"], "peak": LDS_PEAK_GBS,
                     "unit": "GB/s", "frac": f["frac"], "traffic": f["traffic"],
                     "kernel": "k_recombine_est", "algorithmic_bytes": f["and_bytes"],
                     "avg_launch_ms": f["recombine_est_ms"]}
    r["fusion"] = f
    return r


# ---------------------------------------------------------------------------
def run_batched(args):
    import numpy as np
    import torch

    import paper_2307_04890_amd as tn
    import tn_inputs as T

    specs = T.batched_suite(args.networks, seed=4000)
    log(f"[bench] generating {len(specs)} networks")
    nets = [(sp.n,) + sp.generate() for sp in specs]
    m_total = sum(int(x[1].shape[0]) for x in nets)
    ctx = tn.get_context()
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib)
    t0 = time.perf_counter()
    b = tn.Batch(nets)
    plan_wall = time.perf_counter() - t0
    stats, tiles, lds_tiles = b.stats()
    Cs = b.alloc()
    t0 = time.perf_counter()
    b.execute(Cs)  # tunes and captures
    torch.cuda.synchronize()
    tune_wall = time.perf_counter() - t0
    _, tiles, lds_tiles = b.stats()  # of the tuned shape
    elapsed, kms, _ = timed(ctx, lambda: b.execute(Cs), args.steps, args.warmup)
    batch_ms = kms["batch"]
    # the plain one-network kernel, network by network, on the same matrices
    plans = [tn.Plan(n, s, d, t) for (n, s, d, t) in nets]

    def plain():
        for p, C in zip(plans, Cs):
            p.execute(C)

    p_elapsed, pkms, pper = timed(ctx, plain, 1, 1)
    plain_ms = 1e3 * p_elapsed
    dense = sum(algorithmic_bytes(x, sp.n) for x, sp in zip(stats, specs))
    achieved = dense / (batch_ms * 1e-3) / 1e9
    config = {"workload": f"batched_{len(specs)}_uneven", "networks": len(specs),
              "n_range": [500, 20000], "m_range": [10_000, 1_000_000], "m_total": m_total,
              "generators": "uniform pairs (even b) and activity-driven (odd b)",
              "flags": "undirected,strict-ties", "parallelism": "single-gpu"}
    r = base_result(args, m_total / (batch_ms * 1e-3), "events/s", args.steps,
                    1e3 * elapsed / args.steps, config)
    # the tuned shape decides where the rows live: LDS-resident slices, or
    # global-memory tiles whose rows stream through L2 and HBM
    lds_bound = 2 * lds_tiles >= tiles
    r["roofline"] = counter_roofline(load_traffic("batch", config["workload"]), batch_ms,
                                     "k_batch_persistent", dense, achieved,
                                     "lds" if lds_bound else "global")
    r["batched"] = {"graph_launch_ms": batch_ms, "plain_network_by_network_ms": plain_ms,
                    "speedup_vs_plain": plain_ms / batch_ms, "tiles": tiles,
                    "lds_tiles": lds_tiles, "shape": b.shape(), "host_plan_wall_s": plan_wall,
                    "autotune_and_capture_s": tune_wall}
    for p in plans:
        p.close()
    if not args.no_cpu_baseline:
        import oracle
        log("[bench] timing the CPU oracle on a sample of the networks")
        t0 = time.perf_counter()
        done_m = 0
        k = 0
        while time.perf_counter() - t0 < args.cpu_budget and k < len(nets):
            n, s, d, t = nets[k]
            oracle.reverse_matrix(n, s, d, t)
            done_m += int(s.shape[0])
            k += 1
        dt = time.perf_counter() - t0
        r["cpu_baseline"] = {"value": done_m / dt, "unit": "events/s", "cores": 1,
                             "kind": "oracle",
                             "sample": f"full matrices of the first {k} of {len(nets)} networks "
                                       f"({done_m} events), {dt:.2f} s single-threaded",
                             "seconds": dt, "host_nproc": os.cpu_count()}
    b.close()
    return r


# ---------------------------------------------------------------------------
def run_combiner(args):
    import numpy as np
    import torch

    import paper_2307_04890_amd as tn
    import tn_inputs as T
    from paper_2307_04890_amd import combiner as cb

    H, K = args.hashes, args.buckets
    ctx = tn.get_context()

    def features(n, m, Tm, seed, hseed):
        s, d, t = T.activity_driven(n, m, Tm, seed=seed)
        f = cb.hashed_features(n, s, d, t, T.hash_coefficients(H, seed=hseed), K)
        exact = cb.exact_out_sizes(n, s, d, t)
        lifted_min = f["lifted"].min(dim=0).values
        return f["x"], exact, f["est"], lifted_min

    def evaluate(train, heldouts, tag):
        """Train on `train` = (n, m, T) networks, evaluate on each (n, m, T)
        of `heldouts`."""
        t0 = time.perf_counter()
        xs, ys = [], []
        for i in range(args.train_networks):
            x, exact, _, _ = features(*train, 5000 + i, 7000 + i)
            xs.append(x)
            ys.append(torch.log(exact.float() / train[0]))
        log(f"[bench] {tag}: {args.train_networks} training networks")
        X, Y = torch.cat(xs).contiguous(), torch.cat(ys).contiguous()
        data_s = time.perf_counter() - t0
        comb = cb.Combiner(seed=1)
        g = T.rng(2)
        orders = [g.permutation(X.shape[0]) for _ in range(args.epochs)]
        ctx.profile(True)
        t0 = time.perf_counter()
        losses = comb.fit(X, Y, orders, batch=4096, lr=1e-3)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        recs = ctx.profile_take()
        ctx.profile(False)
        bwd = [ms for k, ms in recs if k == "mlp_backward"]
        evals = []
        for heldout in heldouts:
            errs = {"combiner_clamped": [], "combiner": [], "fusion_estimate": [],
                    "min_lifted": []}
            sizes = []
            for i in range(args.heldout_networks):
                n = heldout[0]
                x, exact, est, lmin = features(*heldout, 6000 + i, 8000 + i)
                e = exact.cpu().numpy()
                sizes.append(e)
                errs["combiner_clamped"].append(
                    cb.relative_errors(comb.predict(x, n, est=est).cpu().numpy(), e))
                errs["combiner"].append(cb.relative_errors(comb.predict(x, n).cpu().numpy(), e))
                errs["fusion_estimate"].append(cb.relative_errors(est.cpu().numpy(), e))
                errs["min_lifted"].append(cb.relative_errors(lmin.cpu().numpy(), e))
            log(f"[bench] {tag}: {args.heldout_networks} held-out networks {heldout}")
            summary = {k: {q: float(np.mean([r[q] for r in v])) for q in v[0]}
                       for k, v in errs.items()}
            allsz = np.concatenate(sizes)
            evals.append({"heldout": {"n": heldout[0], "m": heldout[1], "T": heldout[2],
                                      "networks": args.heldout_networks},
                          "exact_size_quantiles": [float(q) for q in
                                                   np.percentile(allsz, [1, 10, 50, 90, 99])],
                          "errors": summary})
        return {"train": {"n": train[0], "m": train[1], "T": train[2],
                          "networks": args.train_networks, "rows": int(X.shape[0])},
                "evaluations": evals, "errors": evals[0]["errors"],
                "exact_size_quantiles": evals[0]["exact_size_quantiles"],
                "dataset_seconds": data_s, "train_seconds": train_s,
                "first_loss": losses[0], "final_loss": float(np.mean(losses[-50:])),
                "steps": len(bwd), "bwd_ms": float(np.sum(bwd)),
                "train_rows": int(X.shape[0])}

    # the stated workload: n = 20,000, m = 10^6 training networks, held-out
    # n = 100,000 networks at the exact workload's density
    main = evaluate((20_000, 1_000_000, 100_000), [(100_000, 10_000_000, 1_000_000)], "stated")
    # the same sizes at 1.2 events per node, where out-components spread;
    # held out at the same events per node, and at the same events per
    # super-node (m / K) as the training networks
    sparse = evaluate((20_000, 24_000, 20_000),
                      [(100_000, 120_000, 100_000), (100_000, 24_000, 100_000)], "sparse")
    steps = main["steps"]
    # forward+backward FLOPs per sample: 2 * (16*64 + 64*64 + 64) * 3
    flop = 2.0 * (16 * 64 + 64 * 64 + 64) * 3 * main["train_rows"] * args.epochs
    achieved = flop / (main["bwd_ms"] * 1e-3) / 1e12
    config = {"workload": "combiner_train64_n20000_m1M_eval4_n100000_m10M", "H": H, "K": K,
              "train_rows": main["train_rows"], "epochs": args.epochs, "batch": 4096,
              "lr": 1e-3, "parallelism": "single-gpu"}
    r = base_result(args, main["errors"]["combiner_clamped"]["mean"], "mean relative error",
                    steps, 1e3 * main["train_seconds"] / max(steps, 1), config, dtype="f32")
    r["higher_is_better"] = False
    r["errors"] = main["errors"]
    r["roofline"] = {"bound": "alu", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s",
                     "frac": achieved / 157.3, "traffic": None, "kernel": "k_mlp_backward",
                     "avg_launch_ms": main["bwd_ms"] / max(steps, 1)}
    r["combiner"] = {k: main[k] for k in ("dataset_seconds", "train_seconds", "first_loss",
                                          "final_loss", "exact_size_quantiles")}
    r["combiner"]["note"] = ("at this density every node reaches every node: exact sizes, "
                             "estimates and predictions all equal n")
    r["sparse"] = sparse
    if not args.no_cpu_baseline:
        from oracle import mlp as ref
        xs_ = np.zeros((4096, 16))
        ys_ = np.zeros(4096)
        p = ref.init(1).astype(np.float64)
        g = T.rng(3)
        xs_[:] = g.normal(size=xs_.shape)
        ys_[:] = g.normal(size=ys_.shape)
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < min(args.cpu_budget, 5.0):
            ref.grad(p, xs_, ys_)
            k += 1
        dt = time.perf_counter() - t0
        r["cpu_baseline"] = {"value": k * 4096 / dt, "unit": "samples/s (forward+backward)",
                             "cores": 1, "kind": "oracle",
                             "sample": f"{k} float64 gradient evaluations of a 4096-row batch",
                             "seconds": dt, "host_nproc": os.cpu_count()}
    return r


def run_sweep(args):
    """The paper's synthetic experiment (Sec. 3.5 setting, Sec. 4.4 criteria):
    ER G(n, 2/n) with a Poisson process on each link; for each (n, m), the
    exact out-component size distribution against the hashed one (H = 5
    hashes to n_s = 0.3 n super-nodes): Earth-Mover distance, relative time
    and relative memory.  Both sides run end to end from host events."""
    import numpy as np
    import torch

    import paper_2307_04890_amd as tn
    import tn_inputs as T
    from paper_2307_04890_amd.evaluate import emd_1d, relative_memory

    ns = [100, 200, 500, 1000, 2000, 5000, 10000]
    ms = [m for m in (10**4, 10**5, 10**6, 10**7, 10**8)
          if args.sweep_min_m <= m <= args.sweep_max_m]
    H = 5
    rows = []
    tot_events = tot_exact = 0.0

    def best_of(fn, reps=2):
        ts, out = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return min(ts), out

    for i, n in enumerate(ns):
        for j, m in enumerate(ms):
            jj = [10**4, 10**5, 10**6, 10**7, 10**8].index(m)  # seeds as in the full grid
            s, d, t = T.er_poisson(n, m, 100 * m, seed=100 * i + jj)
            K = max(1, int(round(0.3 * n)))
            A = T.hash_coefficients(H, seed=7000 + 100 * i + jj)

            def exact():
                C, st = tn.build_component_matrix_streamed(n, s, d, t)
                out, _ = tn.component_sizes(C, n, inn=False)
                return out, st

            def hashed():
                b, c, P, st = tn.hash_build_proxies(n, s, d, t, A, K)
                est, _ = tn.recombine(P, b, c, n, lifted=False)
                return est, st

            te, (out, est_st) = best_of(exact)
            th, (est, hst) = best_of(hashed)
            o = out.cpu().numpy().astype(np.float64)
            e = est.cpu().numpy().astype(np.float64)
            emd = emd_1d(o, e)
            rows.append({"n": n, "m": m, "K": K, "exact_s": te, "hashed_s": th,
                         "relative_time": th / te,
                         "relative_memory": relative_memory(n, K, H),
                         "emd": emd, "emd_over_n": emd / n,
                         "mean_exact": float(o.mean()), "mean_estimate": float(e.mean()),
                         "exact_chunks_run": est_st["chunks_run"], "chunks": est_st["chunks"],
                         "hashed_chunks_run": hst["chunks_run"]})
            tot_events += m
            tot_exact += te
            log(f"[bench] sweep n={n} m={m}: exact {te * 1e3:.1f} ms, hashed {th * 1e3:.1f} ms, "
                f"EMD {emd:.2f} ({emd / n:.4f} n)")
    config = {"workload": "er_poisson_sweep", "n": ns, "m": ms, "H": H, "n_s": "0.3 n",
              "T": "100 m", "graph": "G(n, 2/n)", "parallelism": "single-gpu"}
    r = base_result(args, tot_events / tot_exact, "events/s", len(rows), 1e3 * tot_exact / len(rows),
                    config)
    r["value_note"] = ("exact path end to end from host events (streamed build + out-sizes), "
                       "summed over the sweep")
    r["sweep"] = rows
    return r


def run_hll(args):
    """HyperLogLog stream (Sec. 3.4) at the n = 10^6, m = 10^8 workload, where
    the exact matrix would take 125 GB: registers of 2^b bytes per node,
    resident plan; accuracy against the exact sizes at n = 10^5, m = 10^7."""
    import numpy as np
    import torch

    import paper_2307_04890_amd as tn
    import tn_inputs as T

    b = args.hll_log2s
    workload = args.workload or "activity_n1M_m100M"
    spec = T.WORKLOADS[workload]
    n = spec["n"]
    log(f"[bench] generating {workload}")
    s, d, t = T.make_workload(workload)
    m = int(s.shape[0])
    h = T.hll_node_hashes(n, seed=11)
    ctx = tn.get_context()
    t0 = time.perf_counter()
    plan = tn.Plan(n, s, d, t, tn.HLL)
    plan_wall = time.perf_counter() - t0
    st = plan.stats
    log(f"[bench] plan: {st['levels']} levels, {st['pairs']} pairs, {st['gathers']} gathers, "
        f"{plan_wall:.1f} s")
    M = torch.empty((n, 1 << b), dtype=torch.uint8, device="cuda")
    est = torch.empty(n, dtype=torch.float64, device="cuda")
    # the same outputs every step: the plan replays its captured level launches
    elapsed, kms, _ = timed(ctx, lambda: plan.hll(h, b, M=M, est=est), args.steps, args.warmup)
    torch.cuda.synchronize()
    e = est.cpu().numpy()
    stream_ms = kms["rowor"]
    # row transfers of the level stream: an undirected pair reads and writes
    # two rows, a one-way pair reads two and writes one, a gather reads its
    # sources and writes, reads and writes its scratch row and target
    row = float(1 << b)
    sym = st["pairs"] - st["directed_pairs"]
    moved = row * (4.0 * sym + 3.0 * st["directed_pairs"] + st["gather_sources"] +
                   3.0 * st["gathers"]) + st["device_bytes"]
    config = {"workload": workload, "n": n, "m": m, "T": spec["T"], "generator": spec["kind"],
              "seed": spec["seed"], "registers": 1 << b, "flags": "undirected,strict-ties",
              "parallelism": "single-gpu"}
    r = base_result(args, m * args.steps / elapsed, "events/s", args.steps,
                    1e3 * elapsed / args.steps, config)
    r["value_note"] = ("resident TN_HLL plan: register init + HLL stream + estimates per step; "
                       "the stream stops once every row equals the register-wise maximum over "
                       "all nodes (nothing can change after that)")
    # the whole stream, saturation off: every level runs (the roofline)
    M0 = torch.empty_like(M)
    ctx.saturation(False)
    try:
        _, pkms, _ = timed(ctx, lambda: plan.hll(h, b, M=M0, est=est), 2, 1)
    finally:
        ctx.saturation(True)
    assert torch.equal(M0, M), "the stream with and without the saturation stop differ"
    del M0
    plain_ms = pkms["rowor"]
    r["roofline"] = {"bound": "hbm", "achieved": moved / (plain_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": moved / (plain_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_hll_level + k_hll_gathers_write, every level (saturation "
                               "off; one launch per level, replayed from HIP graphs)",
                     "algorithmic_bytes": moved,
                     "bytes_note": "register rows the level stream must read and write, plus "
                                   "the schedule once", "avg_launch_ms": plain_ms,
                     "levels": st["levels"],
                     "us_per_level": 1e3 * plain_ms / max(1, st["levels"])}
    r["saturating"] = {"stream_ms": stream_ms, "speedup": plain_ms / stream_ms,
                       "us_per_stream_level": 1e3 * stream_ms / max(1, st["levels"]),
                       "note": "mean over every level of the stream; the levels after the "
                               "stop cost nothing"}
    r["kernels_ms"] = kms
    r["hll"] = {"registers_bytes": n * (1 << b), "exact_matrix_bytes": n * ((n + 63) // 64) * 8,
                "plan_wall_s": plan_wall, "mean_estimate": float(e.mean()),
                "estimate_quantiles": [float(q) for q in np.percentile(e, [1, 50, 99])]}
    plan.close()
    # the same stream as the row-OR kernel's level loop on an ops plan (one
    # workgroup per register word column), for comparison
    t0 = time.perf_counter()
    oplan = tn.Plan(n, s, d, t)
    oplan_wall = time.perf_counter() - t0
    _, okms, _ = timed(ctx, lambda: oplan.hll(h, b), 1, 1)
    M2, _ = oplan.hll(h, b)
    assert torch.equal(M, M2), "the two register streams differ"
    r["hll"]["ops_plan"] = {"stream_ms": okms["rowor"], "op_levels": oplan.stats["op_levels"],
                            "plan_wall_s": oplan_wall}
    oplan.close()
    del M2
    # accuracy against exact sizes on the 10^5-node workload
    s2, d2, t2 = T.make_workload("activity_n100000_m10M")
    n2 = 100_000
    h2 = T.hll_node_hashes(n2, seed=12)
    _, est2 = tn.hll_build(n2, s2, d2, t2, h2, b)
    C2, _ = tn.build_component_matrix_streamed(n2, s2, d2, t2)
    out2, _ = tn.component_sizes(C2, n2, inn=False)
    ex = out2.cpu().numpy().astype(np.float64)
    rel = est2.cpu().numpy() / ex - 1.0
    r["hll"]["accuracy_n100000_m10M"] = {
        "mean_relative_error": float(np.mean(np.abs(rel))), "bias": float(np.mean(rel)),
        "std": float(np.std(rel)), "expected_std": 1.04 / np.sqrt(1 << b),
        "mean_exact": float(ex.mean())}
    return r


# ---------------------------------------------------------------------------
# rocprofv3 summaries (run on the CSV files a profiled bench run wrote)
def _read_csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def summarize_pmc(fetch_csv, write_csv, kernel, workload, command, calib_mib, last=0,
                  match=None, per_launch=1):
    """HBM bytes per launch of `kernel`: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch, one --pmc run each), each scaled by what the same counter read
    for the plain device copy of calib_mib MiB in the same run.  last > 0
    keeps only the kernel's last `last` dispatches (the timed ones, after
    autotuning); a launch is `per_launch` consecutive dispatches."""
    match = match or {"rowor": ROWOR_SAT_KERNELS, "rowor_plain": "k_rowor_fwd",
                      "batch": "k_batch_persistent", "recombine": "k_recombine_est"}[kernel]
    alts = match.split("|")
    out = {"kernel": match, "workload": workload, "command": command,
           "kernel_source_sha": kernel_source_hash(KERNEL_SOURCES[kernel])}
    known_kib = calib_mib * 1024.0
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _read_csv(path) if r["Counter_Name"] == name]
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
                  or "elementwise" in r["Kernel_Name"]]
        # the calibration copy is the largest copy dispatch of the run
        calib = max(copies) if copies else float("nan")
        vals = [float(r["Counter_Value"]) for r in rows
                if any(a in r["Kernel_Name"] for a in alts)]
        if last:
            vals = vals[-last:]
        factor = known_kib / calib
        launches = max(len(vals) / per_launch, 1)
        out[name] = {"kib_per_dispatch": vals, "calibration_kib": calib, "factor": factor,
                     "dispatches_per_launch": per_launch,
                     "bytes_per_launch": 1024.0 * factor * sum(vals) / launches}
    out["hbm_bytes_per_launch"] = out["FETCH_SIZE"]["bytes_per_launch"] + \
        out["WRITE_SIZE"]["bytes_per_launch"]
    return out


def summarize_trace(stats_csv, command, top=12, trace_csv=None, match=None, last=0,
                    per_launch=1):
    """Per-kernel stats of a --kernel-trace --stats run; with trace_csv, match
    and last, also the mean duration of the last `last` dispatches of the
    kernels whose names contain `match` (alternatives separated by '|'; the
    timed ones, after autotuning), summed over each launch of `per_launch`
    consecutive dispatches."""
    rows = _read_csv(stats_csv)
    lines = [f"command: {command}", "",
             f"{'calls':>6} {'avg ms':>10} {'total ms':>10} {'%':>6}  kernel"]
    for r in rows[:top]:
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e6:10.3f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}  "
                     f"{r['Name'][:110]}")
    if trace_csv and match and last:
        alts = match.split("|")
        ds = [(int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
              for r in _read_csv(trace_csv) if any(a in r["Kernel_Name"] for a in alts)]
        ds.sort()
        tail = [d for _, d in ds[-last:]]
        k = max(1, per_launch)
        groups = [sum(tail[i:i + k]) for i in range(0, len(tail) - k + 1, k)]
        what = f"launches of {k} dispatches" if k > 1 else "dispatches"
        lines += ["", f"last {len(groups)} {what} of {match} (the timed launches): "
                      f"mean {sum(groups) / max(len(groups), 1) / 1e6:.3f} ms, each "
                      + ", ".join(f"{d / 1e6:.3f}" for d in groups) + " ms"]
        if k > 1:
            lines.append("  dispatch durations: " + ", ".join(f"{d / 1e6:.3f}" for d in tail) + " ms")
    return "\n".join(lines) + "\n"


def main():
    if len(sys.argv) > 1 and sys.argv[1] in ("--summarize-pmc", "--summarize-trace"):
        what = sys.argv[1]
        sp = argparse.ArgumentParser()
        sp.add_argument("--fetch")
        sp.add_argument("--write")
        sp.add_argument("--stats")
        sp.add_argument("--trace")
        sp.add_argument("--kernel", default="rowor")
        sp.add_argument("--workload", default="activity_n100000_m10M")
        sp.add_argument("--command", required=True)
        sp.add_argument("--calib-mib", type=int, default=1024)
        sp.add_argument("--last", type=int, default=0)
        sp.add_argument("--match", default=None, help="kernel name substring")
        sp.add_argument("--per-launch", type=int, default=1)
        sp.add_argument("--out", required=True)
        a = sp.parse_args(sys.argv[2:])
        if what == "--summarize-pmc":
            rec = summarize_pmc(a.fetch, a.write, a.kernel, a.workload, a.command, a.calib_mib,
                                a.last, a.match, a.per_launch)
            with open(a.out, "w") as f:
                json.dump(rec, f, indent=1)
        else:
            with open(a.out, "w") as f:
                f.write(summarize_trace(a.stats, a.command, trace_csv=a.trace, match=a.match,
                                        last=a.last, per_launch=a.per_launch))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="exact",
                    choices=["exact", "hashed", "batched", "combiner", "sweep", "hll", "online",
                             "fusion"])
    ap.add_argument("--online-batches", type=int, default=10,
                    help="event batches of the online mode")
    ap.add_argument("--hll-log2s", type=int, default=8,
                    help="log2 of the HyperLogLog registers per node (--mode hll)")
    ap.add_argument("--sweep-max-m", type=float, default=1e7,
                    help="largest event count of the ER + Poisson sweep")
    ap.add_argument("--sweep-min-m", type=float, default=0,
                    help="smallest event count of the ER + Poisson sweep")
    ap.add_argument("--workload", default=None)
    ap.add_argument("--slice-words", type=int, default=0)
    ap.add_argument("--no-end-to-end", action="store_true",
                    help="exact and hashed modes: skip the streamed end-to-end runs (for "
                         "profiles of the resident launches alone)")
    ap.add_argument("--no-hashed", action="store_true",
                    help="exact mode: skip the hashed block (the 10^6-node stream)")
    ap.add_argument("--no-plain", action="store_true",
                    help="exact mode: skip the plain leg (for profiles of the saturating "
                         "launches alone; the line then has no roofline)")
    ap.add_argument("--hashes", type=int, default=16)
    ap.add_argument("--buckets", type=int, default=4096)
    ap.add_argument("--networks", type=int, default=256)
    ap.add_argument("--train-networks", type=int, default=64)
    ap.add_argument("--heldout-networks", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of single-thread oracle work for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "column sharding is a design, not built here", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    run = {"exact": run_exact, "hashed": run_hashed, "batched": run_batched,
           "combiner": run_combiner, "sweep": run_sweep, "hll": run_hll,
           "online": run_online, "fusion": run_fusion}[args.mode]
    print(json.dumps(run(args)), flush=True)


if __name__ == "__main__":
    main()
