#!/usr/bin/env python
"""Throughput of the batched LP solver on one MI355X.

Workload (one step): solve 50,000 type-1 LPs with m = n = 100 (A~U(1,10),
b~U(10,100), c~U(1,10), seed 1002), inputs resident in HBM, persistent
size-binned kernels.  Prints ONE JSON line with LPs/s, the same batch's
one-LP-per-launch rate on a sample, LPs/s of the other workload classes,
the roofline of the dominant kernel (HIP events recorded by the library on
the solve's stream) and the CPU oracle's rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
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

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (256 CUs x 128 flop/clk x 2.4 GHz)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
PEAK_LDS_GBS = 78643.2    # 256 CUs x 128 B/clk x 2.4 GHz
METRIC = "LPs/sec per size class, batched persistent vs one-LP-per-launch, obj relerr\u22641e-9"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dominant_kernel__type1_m100_n100_K50000.json")
KERNEL_SOURCES = ["paper_1609_08114_amd/csrc/simplex_reg.hip", "paper_1609_08114_amd/csrc/simplex_blk.hpp",
                  "paper_1609_08114_amd/csrc/simplex_cols.hpp", "paper_1609_08114_amd/csrc/simplex_lane.hpp",
                  "paper_1609_08114_amd/csrc/simplex_lane.hip",
                  "paper_1609_08114_amd/csrc/simplex_common.hpp", "paper_1609_08114_amd/csrc/blp_kernels.hpp",
                  "paper_1609_08114_amd/csrc/variants.hpp"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def time_solver(blp, torch, db, steps, warmup, profile=True, warm_ms=0.0, step_times=None, kernel_avg=False,
                **kw):
    """Warm up (`warmup` solves, and with `warm_ms` > 0 at least that much wall
    time, synchronising after 1, 2, 4, ... up to 16 solves), then time `steps` solves enqueued
    back to back on one stream (one synchronisation at each end); returns (ms
    per step, per-class kernel ms of the last timed step from the HIP events
    the library records around each kernel class (zeros without `profile`),
    last outputs, bins).  With `step_times` (a list), HIP events recorded on
    the stream between the back-to-back steps add each step's device time to
    it.  With `kernel_avg`, a second loop of `steps` profiled solves (each read
    back) replaces the per-class kernel ms by their average over those steps."""
    s = blp.Solver(profile=profile, **kw)
    stream = torch.cuda.Stream()
    out = None  # output tensors: allocated by the first solve, reused by every later one
    for _ in range(warmup):
        out = s.solve(db, stream=stream, outputs=out)
    if warm_ms > 0:
        w0, n = time.perf_counter(), 1
        while (time.perf_counter() - w0) * 1e3 < warm_ms:
            for _ in range(n):
                out = s.solve(db, stream=stream, outputs=out)
            torch.cuda.synchronize()
            n = min(16, 2 * n)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if step_times is not None else None
    t0 = time.perf_counter()
    if evs:
        evs[0].record(stream)
    for i in range(steps):
        out = s.solve(db, stream=stream, outputs=out)
        if evs:
            evs[i + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if evs:
        step_times.extend(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    kms = blp.blp_last_kernel_ms(s.h)
    if kernel_avg and profile:
        acc = np.zeros_like(kms)
        for _ in range(steps):
            out = s.solve(db, stream=stream, outputs=out)
            acc += blp.blp_last_kernel_ms(s.h)
        kms = acc / steps
    bins = blp.blp_last_bins(s.h)
    s.close()
    return (t1 - t0) * 1e3 / steps, kms, out, bins


TIMER_LIB = os.path.join(ROOT, "paper_1609_08114_amd", "libblp_timers.so")


def _timer_child(K: int) -> None:
    """Run in a child process with BLP_LIBRARY naming the phase-timer build:
    one solve of the headline batch; closing the handle prints the phase
    cycle counters (summed over the LP's first wave, per LP and per pivot)."""
    import torch

    import lpgen
    import paper_1609_08114_amd as blp
    db = blp.DeviceBatch.from_host(lpgen.config(2, range(K)))
    s = blp.Solver()
    s.solve(db)
    torch.cuda.synchronize()
    s.close()


def phase_timers(K: int) -> dict | None:
    """Per-phase cycles of the headline solve from the phase-timer build (a
    child process), or None if that build is absent.  For the column-split
    kernel the four pivot phases are: candidate (the wave's Step 1, column
    publication and Step 2), exchange (candidate record, the barrier, the
    winner), pivot row (publication and division) and update (mirrors and
    the rank-1 update of the tile)."""
    import re
    import subprocess
    if not os.path.exists(TIMER_LIB):
        return None
    env = dict(os.environ, BLP_LIBRARY=TIMER_LIB)
    r = subprocess.run([sys.executable, "-c", f"import bench; bench._timer_child({K})"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    m = re.search(r"\[blp timers\] LPs (\d+) pivots (\d+) \| cycles per LP: load ([\d.]+) extract ([\d.]+) \| "
                  r"per pivot: price ([\d.]+) pubcol ([\d.]+) ratio ([\d.]+) pivot ([\d.]+)", r.stderr)
    if r.returncode != 0 or not m:
        log(f"phase timers: no counters (rc {r.returncode}): {r.stderr[-400:]}")
        return None
    lps, piv = int(m.group(1)), int(m.group(2))
    load, extract, cand, exch, prow, upd = (float(m.group(i)) for i in range(3, 9))
    per_pivot = cand + exch + prow + upd
    per_lp = load + extract + per_pivot * piv / max(lps, 1)
    return {"lps": lps, "pivots": piv, "unit": "cycles of one wave (s_memtime), per LP and per pivot",
            "per_lp": {"load": round(load), "extract": round(extract)},
            "per_pivot": {"candidate": round(cand), "exchange": round(exch), "pivot_row": round(prow),
                          "update": round(upd)},
            "update_share_of_pivot": round(upd / per_pivot, 4) if per_pivot > 0 else None,
            "pivot_loop_share_of_lp": round(per_pivot * piv / max(lps, 1) / per_lp, 4) if per_lp > 0 else None}


def rate_one_per_launch(blp, torch, lpgen, cfg, ids, **kw):
    hb = lpgen.config(cfg, ids) if not isinstance(cfg, tuple) else lpgen.config(cfg[0], ids, part=cfg[1])
    db = blp.DeviceBatch.from_host(hb)
    ms, _, out, _ = time_solver(blp, torch, db, 1, 1, mode=blp.BLP_MODE_ONE_PER_LAUNCH)
    return hb.count / (ms / 1e3), ms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=50_000)
    ap.add_argument("--one-per-launch-sample", type=int, default=50_000)
    ap.add_argument("--cpu-sample", type=int, default=50_000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-classes", action="store_true")
    ap.add_argument("--no-host", action="store_true")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic file from the counter_collection.csv of a FETCH_SIZE and a WRITE_SIZE "
                         "run of --counter-pass, then exit")
    ap.add_argument("--counter-pass", action="store_true",
                    help="only a 1 GiB device copy followed by one persistent solve of the batch "
                         "(the workload of the HBM-counter runs)")
    ap.add_argument("--counter-workload", default="2", choices=["2", "3", "box5", "box28"],
                    help="--counter-pass: the headline batch (2), workload 3 at its 10,000 LPs, or the "
                         "4,000,000 n=5 / 6,000,000 n=28 hyperbox batches of workload 5")
    ap.add_argument("--counter-table", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the HBM bytes of every kernel of two counter runs (scaled by the copy), then exit")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(*args.traffic_from, batch=args.batch)
        return
    if args.counter_table:
        print(json.dumps(counter_table(*args.counter_table), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the batch shards across GPUs "
              "with no exchange, so run one process per GPU instead.", file=sys.stderr)
        sys.exit(2)

    import torch

    import lpgen
    import paper_1609_08114_amd as blp
    assert torch.cuda.is_available(), "needs a GPU"

    if args.counter_pass:
        counter_pass(blp, torch, lpgen, args.batch, args.counter_workload)
        return

    # ------------------------------------------------------------ main line
    K = args.batch
    log(f"generating {K} type-1 LPs 100x100")
    t = time.perf_counter()
    hb = lpgen.config(2, range(K))
    log(f"generated in {time.perf_counter() - t:.1f}s; copying to HBM")
    db = blp.DeviceBatch.from_host(hb)
    torch.cuda.synchronize()
    log("timing persistent mode")
    # the timed steps run as a caller would run them, without the library's
    # per-class timing events; the kernel times come from a separate
    # profiled pass over the same batch
    step_ms = []
    ms, _, out, bins = time_solver(blp, torch, db, args.steps, args.warmup, profile=False, step_times=step_ms)
    _, kms, _, _ = time_solver(blp, torch, db, args.steps, 1, profile=True, kernel_avg=True)
    status = out["status"][:K].cpu().numpy()
    iters = out["iters"][:K].cpu().numpy().astype(np.int64)
    obj = out["obj"][:K].cpu().numpy()
    value = K / (ms / 1e3)
    log(f"persistent: {ms:.3f} ms/step, {value:,.0f} LPs/s, statuses {np.bincount(status, minlength=5)}")

    # dominant kernel (largest device time) and its roofline
    names = [v[0] for v in blp.variants()] + ["streaming", "hyperbox", "binning"]
    dom = int(np.argmax(kms))
    dom_ms = float(kms[dom])
    m = n = 100
    # Work per pivot as executed: the kernel stores the condensed tableau,
    # the n nonbasic columns and the rhs of the m constraint rows and the
    # objective row, (m + 1)(n + 1) entries, one FMA each (the basic columns
    # of the full tableau of Sec. 3.1 are unit vectors and are not stored).
    # The full tableau, (m + 1)(n + m + 1) entries, is reported as context.
    executed = float(iters.sum()) * 2.0 * (m + 1) * (n + 1)
    full = float(iters.sum()) * 2.0 * (m + 1) * (n + m + 1)
    achieved = executed / (dom_ms / 1e3) / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("kernel_source_hash") == kernel_source_hash() and tf.get("batch") == K:
            traffic = tf.get("bytes_per_launch")
    input_bytes = K * 8.0 * (m * n + m + n) + K * (m + 2 * 4 + 8 + 8 * (m + n))
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
                "kernel": names[dom], "kernel_ms": round(dom_ms, 4),
                "kernel_ms_note": f"mean of {args.steps} profiled solves (HIP events on the solve's stream)",
                "flops_per_pivot": 2 * (m + 1) * (n + 1), "pivots": int(iters.sum()), "executed_flops": executed,
                "context_full_tableau_flops": full,
                "context_full_tableau_frac": round(full / (dom_ms / 1e3) / 1e12 / PEAK_FP64_TFLOPS, 4),
                "hbm_input_bytes": input_bytes,
                "hbm_frac_of_input_read": round(input_bytes / (dom_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}

    # per-phase cycles of the same solve (phase-timer build, child process)
    timers = phase_timers(K)
    if timers:
        roofline["phase_cycles"] = timers
        log(f"phase timers: {timers}")
    # the same batch with its recorded pivots replayed (no Steps 1 and 2)
    if names[dom] == "b4_r112_c112":
        roofline["pivot_replay"] = pivot_replay(blp, torch, db, K, obj, dom_ms, (m + 1) * (n + 1))
        log(f"pivot replay: {roofline['pivot_replay']}")

    # ------------------------------------------------- one LP per launch
    S = min(args.one_per_launch_sample, K)
    log(f"one-LP-per-launch on the first {S} LPs")
    sub = db if S == K else blp.DeviceBatch.from_host(lpgen.config(2, range(S)))
    ms1, _, out1, _ = time_solver(blp, torch, sub, 1, 1, mode=blp.BLP_MODE_ONE_PER_LAUNCH)
    rate1 = S / (ms1 / 1e3)
    assert np.array_equal(out1["obj"][:S].cpu().numpy().view(np.int64), obj[:S].view(np.int64))
    log(f"one-per-launch: {rate1:,.0f} LPs/s")

    # --------------------------------- end to end from pinned host memory
    host = None
    if not args.no_host:
        log("end to end from pinned host memory")
        host = rate_host_resident(blp, torch, hb, obj)
        log(f"host-resident: {host}")

    # -------------------------------------------------- other size classes
    per_class = {}
    if not args.no_classes:
        per_class = bench_classes(blp, torch, lpgen)

    # ---------------------- shared constraints, many objectives (Sec. 7)
    shared = None
    if not args.no_classes:
        shared = bench_shared(blp, torch, lpgen)

    # ------------------- captured launch sequences against eager launches
    graphs = lanes = None
    if not args.no_classes:
        graphs = graph_replay(blp, torch, lpgen)
        lanes = lane_scaling(blp, torch, lpgen)

    # -------------------- pivot rules: RPC (Sec. 4.2) against LPC, same batch
    rules = None
    if not args.no_classes:
        rules = pivot_rules(blp, torch, db, K, obj, iters, value)

    # ------------------------------------------- layout ablation (Sec. 4.3)
    ablation = None
    if not args.no_classes:
        ablation = layout_ablation(blp, torch, lpgen)

    # ------------------------------------------------------- CPU baseline
    cpu = None
    parity = None
    if not args.no_cpu:
        import oracle
        C = min(args.cpu_sample, K)
        ids = np.arange(C)
        sample = lpgen.config(2, ids)
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"CPU oracle on {C} LPs, {cores} threads, repeated for about {args.cpu_seconds:.0f} s")
        reps, dt = 0, 0.0
        while reps < 1 or (dt < args.cpu_seconds and reps < 50):
            t = time.perf_counter()
            ref = oracle.solve_batch(sample)
            dt += time.perf_counter() - t
            reps += 1
        cpu = {"value": round(C * reps / dt, 1), "unit": "LPs/s", "cores": cores, "kind": "oracle",
               "sample": f"first {C} LPs of the 50,000-LP batch (type 1, m=n=100) solved {reps} times, "
                         "OpenMP one LP per thread",
               "seconds": round(dt, 3), "single_core": oracle_single_core(1000), "host": host_cpu()}
        rel = np.abs(obj[:C] - ref["obj"]) / np.maximum(1.0, np.abs(ref["obj"]))
        parity = {"checked": C, "status_mismatch": int((status[:C] != ref["status"]).sum()),
                  "max_obj_relerr": float(rel.max()),
                  "iters_mismatch": int((iters[:C] != ref["iters"]).sum()),
                  "obj_bit_identical": int((obj[:C].view(np.int64) == ref["obj"].view(np.int64)).sum())}
        log(f"oracle: {cpu['value']:,.0f} LPs/s; parity {parity}")

    line = {
        "metric": METRIC,
        "value": round(value, 1), "unit": "LPs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "type-1 dense LPs, m=n=100 (tableau 101x101 condensed, 101x201 full), "
                               "A~U(1,10) b~U(10,100) c~U(1,10), seed 1002",
                   "batch": K, "m": 100, "n": 100, "mode": "persistent"},
        "end_to_end_pinned_host": host,
        "step_ms": {"mean": round(float(np.mean(step_ms)), 4), "median": round(float(np.median(step_ms)), 4),
                    "min": round(float(np.min(step_ms)), 4), "max": round(float(np.max(step_ms)), 4),
                    "runs": len(step_ms), "note": "device time of each timed step (HIP events between steps)"},
        "one_per_launch": {"value": round(rate1, 1), "unit": "LPs/s",
                           "sample": "all LPs" if S == K else f"first {S} LPs",
                           "speedup_persistent": round(value / rate1, 2)},
        "statuses": np.bincount(status, minlength=5).tolist(),
        "pivots_per_lp": round(float(iters.mean()), 3),
        "bins": {names[i]: int(bins[i]) for i in range(len(bins)) if bins[i]},
        "kernel_ms": {names[i]: round(float(kms[i]), 4) for i in range(len(kms)) if kms[i] > 0},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "per_class": per_class,
        "layout_ablation": ablation,
        "shared_constraints": shared,
        "pivot_rules": rules,
        "graph_replay": graphs,
        "lane_kernel_scaling": lanes,
    }
    print(json.dumps(line), flush=True)


def pivot_replay(blp, torch, db, K, obj, fused_ms, entries, runs=5) -> dict:
    """Cross-check of the update time from the phase counters: the batch is
    solved once recording every LP's pivots (leaving row, entering slot), then
    `runs` times replaying them, so Steps 1 and 2 (pricing and the ratio test)
    are skipped while the load, the column and row exchanges, the division,
    the rank-1 updates and the extraction run as in the fused kernel."""
    stride = 1 + 2 * 128
    tr = torch.empty(K * stride, dtype=torch.int32, device="cuda")
    s = blp.Solver(profile=True)
    stream = torch.cuda.Stream()
    v = [x[0] for x in blp.variants()].index("b4_r112_c112")
    rec = s.pivot_trace(db, tr, stride, False, stream=stream)
    torch.cuda.synchronize()
    rec_ms = float(blp.blp_last_kernel_ms(s.h)[v])
    cnt = tr.view(K, stride)[:, 0].cpu().numpy()
    out = None
    ts = []
    for _ in range(runs):
        out = s.pivot_trace(db, tr, stride, True, stream=stream, outputs=out)
        torch.cuda.synchronize()
        ts.append(float(blp.blp_last_kernel_ms(s.h)[v]))
    st = out["status"][:K].cpu().numpy()
    same = bool(np.array_equal(out["obj"][:K].cpu().numpy().view(np.int64), obj.view(np.int64)))
    s.close()
    piv = float(cnt[cnt > 0].sum())
    med = float(np.median(ts))
    return {"lps": K, "replayed": int((st == 0).sum()), "pivots": int(piv), "stride": stride,
            "record_kernel_ms": round(rec_ms, 4), "replay_kernel_ms": _stats(ts), "fused_kernel_ms": round(fused_ms, 4),
            "replay_over_fused": round(med / fused_ms, 4), "search_share_of_fused": round(1.0 - med / fused_ms, 4),
            "replay_fma_tflops": round(piv * 2.0 * entries / (med / 1e3) / 1e12, 3),
            "obj_identical_to_solve": same,
            "note": "replay: Steps 1 and 2 read from the record; load, exchanges, division, update, extraction kept"}


def host_cpu() -> dict:
    """The host's logical CPU count and model (the oracle's cores)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def oracle_single_core(C: int) -> dict | None:
    """The oracle on one thread (a child process with OMP_NUM_THREADS=1)
    over the first C LPs of the headline batch, repeated for about 2 s."""
    import subprocess
    code = ("import time, numpy as np, lpgen, oracle\n"
            f"b = lpgen.config(2, np.arange({C}))\n"
            "reps, dt = 0, 0.0\n"
            "while reps < 1 or dt < 2.0:\n"
            "    t = time.perf_counter(); oracle.solve_batch(b); dt += time.perf_counter() - t; reps += 1\n"
            f"print({C} * reps / dt)\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=300)
        return {"value": round(float(r.stdout.strip().splitlines()[-1]), 1), "unit": "LPs/s", "cores": 1,
                "sample": f"first {C} LPs of the headline batch, one thread"}
    except Exception as e:  # reported, never fatal to the bench line
        log(f"single-core oracle: {e}")
        return None


def rate_host_resident(blp, torch, hb, ref_obj, steps=3):
    """LPs/s including the PCIe copies: inputs in pinned host memory, results
    back in pinned host memory, pieces alternating on two streams."""
    import ctypes
    K = hb.count

    def pinned(a):
        t = torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
        return t

    keep = [pinned(a) for a in (hb.m, hb.n, hb.kind, hb.a_off, hb.row_off, hb.col_off, hb.A, hb.b, hb.sense,
                                hb.c, hb.l, hb.u)]
    outs = [torch.empty(K, dtype=torch.int32).pin_memory(), torch.empty(K, dtype=torch.int32).pin_memory(),
            torch.empty(K, dtype=torch.float64).pin_memory(), torch.empty(hb.c.size, dtype=torch.float64).pin_memory(),
            torch.empty(max(1, hb.b.size), dtype=torch.float64).pin_memory()]
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    b = blp.blp_batch(K, 0, 0, *[P(t) for t in keep])
    o = blp.blp_outputs(*[P(t) for t in outs])
    s = blp.Solver()
    blp.blp_solve_batch_host(s.h, b, o, 0)
    t0 = time.perf_counter()
    for _ in range(steps):
        blp.blp_solve_batch_host(s.h, b, o, 0)
    dt = (time.perf_counter() - t0) / steps
    s.close()
    same = bool(np.array_equal(outs[2].numpy().view(np.int64), ref_obj.view(np.int64)))
    in_bytes = sum(t.numel() * t.element_size() for t in keep)
    out_bytes = sum(t.numel() * t.element_size() for t in outs)
    return {"value": round(K / dt, 1), "unit": "LPs/s", "ms": round(dt * 1e3, 3), "pcie_bytes": in_bytes + out_bytes,
            "obj_identical_to_resident": same}


def _read_counter(path, counter):
    import csv
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def counter_table(fetch_csv: str, write_csv: str) -> dict:
    """HBM bytes per dispatch of every kernel of a FETCH_SIZE and a
    WRITE_SIZE run, each scaled so that the run's 1 GiB device copy reads
    and writes 1 GiB."""
    f = _read_counter(fetch_csv, "FETCH_SIZE")
    w = _read_counter(write_csv, "WRITE_SIZE")
    copy = next(k for k in f if "copyBuffer" in k or "copy" in k.lower())
    kib = float(1 << 20)
    ff, fw = kib / f[copy][0], kib / w[copy][0]
    out = {"fetch_factor": round(ff, 4), "write_factor": round(fw, 4), "kernels": {}}
    for k in f:
        if k == copy:
            continue
        fb = [v * ff * 1024.0 for v in f[k]]
        wb = [v * fw * 1024.0 for v in w.get(k, [0.0])]
        out["kernels"][k.split("(")[0][:120]] = {"dispatches": len(fb), "fetch_bytes_max": max(fb),
                                                "write_bytes_max": max(wb)}
    return out


def write_traffic(fetch_csv: str, write_csv: str, batch: int) -> None:
    """HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc
    runs of --counter-pass, each counter scaled by what it reads for the
    1 GiB device copy of the same run."""
    f = _read_counter(fetch_csv, "FETCH_SIZE")
    w = _read_counter(write_csv, "WRITE_SIZE")
    copy = next(k for k in f if "copyBuffer" in k or "copy" in k.lower())
    kib = float(1 << 20)  # the copy moves 1 GiB each way
    ff, fw = kib / f[copy][0], kib / w[copy][0]
    simplex = [k for k in f if "simplex_" in k]
    dom = max(simplex, key=lambda k: f[k][0])
    fetch_b = f[dom][0] * ff * 1024.0
    write_b = w[dom][0] * fw * 1024.0
    out = {"kernel": dom, "batch": batch, "kernel_source_hash": kernel_source_hash(),
           "fetch_factor": round(ff, 4), "write_factor": round(fw, 4),
           "fetch_bytes": fetch_b, "write_bytes": write_b, "bytes_per_launch": fetch_b + write_b}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(out))


def counter_pass(blp, torch, lpgen, K, workload="2"):
    """The workload of the HBM byte-counter runs: one plain device copy of
    1 GiB (the calibration of FETCH_SIZE/WRITE_SIZE) and one persistent solve
    of the K-LP headline batch, of workload 3 (10,000 LPs) or of a full
    hyperbox batch of workload 5."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    if workload == "3":
        hb, K = lpgen.config(3, range(10_000)), 10_000
    elif workload.startswith("box"):
        K = 4_000_000 if workload == "box5" else 6_000_000
        hb = lpgen.config(5, range(K), part=workload)
    else:
        hb = lpgen.config(2, range(K))
    db = blp.DeviceBatch.from_host(hb)
    s = blp.Solver()
    s.solve(db)
    torch.cuda.synchronize()
    s.close()
    log(f"counter pass done: copy of {1 << 30} bytes, one solve of {K} LPs (workload {workload})")


def bench_shared(blp, torch, lpgen, K=50_000) -> dict:
    """One workload-2 polytope (m = n = 100) queried in K directions, as in
    support-function sampling: directions swept around a circle, and random
    unit directions.  blp_solve_shared (phase 1 once, warm starts) against
    the same K LPs solved independently by blp_solve_batch (the oracle
    comparison of this mode is in the tests), and the time of its adjoint
    blp_backward_shared."""
    dev = torch.device("cuda")
    lp = lpgen.config(2, [0]).lp(0)
    A, b, sense = lp["A"], lp["b"], lp["sense"]
    m, n = A.shape
    rng = np.random.default_rng(1007)
    u, v = rng.normal(size=(2, n))
    t = np.linspace(0.0, 2.0 * np.pi, K, endpoint=False)
    sweep = np.cos(t)[:, None] * u + np.sin(t)[:, None] * v
    G = rng.normal(size=(K, n))
    rand = G / np.linalg.norm(G, axis=1, keepdims=True)
    Ad = torch.from_numpy(np.ascontiguousarray(A).ravel()).to(dev)
    bd = torch.from_numpy(b).to(dev)
    sd = torch.from_numpy(sense).to(dev)
    res = {"polytope": "workload-2 LP 0, m=n=100", "lps": K}
    for name, C in (("circle_sweep", sweep), ("random_directions", rand)):
        Cd = torch.from_numpy(np.ascontiguousarray(C)).to(dev)
        s = blp.Solver()
        out = s.solve_shared(Ad, bd, sd, Cd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            out = s.solve_shared(Ad, bd, sd, Cd)
        torch.cuda.synchronize()
        ms_sh = (time.perf_counter() - t0) * 1e3 / reps
        # the adjoint of the sweep: dC, db and dA summed over the objectives
        g = torch.from_numpy(rng.uniform(0.0, 1.0, size=K)).to(dev)
        s.backward_shared(out, m, n, g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            s.backward_shared(out, m, n, g)
        torch.cuda.synchronize()
        ms_bw = (time.perf_counter() - t0) * 1e3 / reps
        s.close()
        obj_sh = out["obj"][:K].cpu().numpy()
        it_sh = out["iters"][:K].cpu().numpy()
        st_sh = out["status"][:K].cpu().numpy()
        # the same LPs, independently
        hb = lpgen.make_batch(1002, np.zeros(K, np.int64), np.ones(K, np.int32), np.full(K, m), np.full(K, n))
        hb.A = np.tile(A.ravel(), K)
        hb.b = np.tile(b, K)
        hb.sense = np.tile(sense, K)
        hb.c = np.ascontiguousarray(C).ravel()
        db = blp.DeviceBatch.from_host(hb)
        ms_ind, _, out_i, _ = time_solver(blp, torch, db, 3, 1)
        obj_i = out_i["obj"][:K].cpu().numpy()
        st_i = out_i["status"][:K].cpu().numpy()
        it_i = out_i["iters"][:K].cpu().numpy()
        del db
        ok = st_i == 0
        rel = np.abs(obj_sh[ok] - obj_i[ok]) / np.maximum(1.0, np.abs(obj_i[ok]))
        entry = {"shared_lps_per_s": round(K / (ms_sh / 1e3), 1), "shared_ms": round(ms_sh, 3),
                 "independent_lps_per_s": round(K / (ms_ind / 1e3), 1), "independent_ms": round(ms_ind, 3),
                 "speedup": round(ms_ind / ms_sh, 2), "pivots_per_lp_shared": round(float(it_sh.mean()), 2),
                 "pivots_per_lp_independent": round(float(it_i.mean()), 2),
                 "status_mismatch": int((st_sh != st_i).sum()), "max_obj_relerr_vs_independent": float(rel.max()),
                 "backward_ms": round(ms_bw, 3),
                 "backward_GBps": round(K * 8.0 * (2 * n + m + 1) / (ms_bw / 1e3) / 1e9, 1)}
        res[name] = entry
        log(f"shared {name}: {entry}")
    return res


def pivot_rules(blp, torch, db, K, obj_lpc, iters_lpc, rate_lpc, seed=12345) -> dict:
    """The random-positive-coefficient rule (Sec. 4.2) on the same resident
    batch as the headline LPC run: LPs/s, pivots per LP and agreement of the
    optima (both rules reach the same optimum; the pivot paths differ)."""
    log("pivot rules: RPC on the headline batch")
    ms, _, out, _ = time_solver(blp, torch, db, 3, 1, pivot_rule=blp.BLP_RULE_RPC, seed=seed)
    st = out["status"][:K].cpu().numpy()
    it = out["iters"][:K].cpu().numpy().astype(np.int64)
    ob = out["obj"][:K].cpu().numpy()
    rel = np.abs(ob - obj_lpc) / np.maximum(1.0, np.abs(obj_lpc))
    rate = K / (ms / 1e3)
    return {"lps": K, "seed": seed,
            "lpc": {"lps_per_s": round(rate_lpc, 1), "pivots_per_lp": round(float(iters_lpc.mean()), 3)},
            "rpc": {"lps_per_s": round(rate, 1), "ms": round(ms, 3), "pivots_per_lp": round(float(it.mean()), 3),
                    "statuses": np.bincount(st, minlength=5).tolist()},
            "lpc_over_rpc": round(rate_lpc / rate, 3),
            "max_obj_relerr_rpc_vs_lpc": float(rel[st == 0].max()) if (st == 0).any() else None}


def layout_ablation(blp, torch, lpgen, K=512) -> dict:
    """The streaming kernel on workload 3 (type-2 LPs, m = n = 200, tableau
    202 x 301 in HBM) with the coalesced column-major workspace against the
    row-major one under the same thread mapping (Sec. 4.3's comparison)."""
    hb = lpgen.config(3, range(K))
    db = blp.DeviceBatch.from_host(hb)
    res = {"lps": K, "workload": "type-2 m=n=200, streaming kernel"}
    objs = {}
    for name, lay in (("column_major", blp.BLP_LAYOUT_COLUMN), ("row_major", blp.BLP_LAYOUT_ROW)):
        log(f"layout ablation: {name}")
        ms, kms, out, _ = time_solver(blp, torch, db, 1, 1, variant=-2, layout=lay)
        res[name] = {"ms": round(ms, 3), "lps_per_s": round(K / (ms / 1e3), 1),
                     "kernel_ms": round(float(kms[len(blp.variants())]), 3)}
        objs[name] = out["obj"][:K].cpu().numpy().view(np.int64)
    res["row_over_column"] = round(res["row_major"]["kernel_ms"] / res["column_major"]["kernel_ms"], 2)
    res["bit_identical"] = bool(np.array_equal(objs["column_major"], objs["row_major"]))
    return res


def _stats(ts) -> dict:
    return {"mean_ms": round(float(np.mean(ts)), 4), "median_ms": round(float(np.median(ts)), 4),
            "min_ms": round(float(np.min(ts)), 4), "max_ms": round(float(np.max(ts)), 4), "runs": len(ts)}


# Workloads at their stated sizes: (name, config, part, LPs, one-LP-per-launch
# LPs (None: all of them), timed runs)
CLASS_PLAN = [
    ("type1_5x5", 1, None, 1_000, None, 10),
    ("type1_20..150", 5, "simplex", 20_000, None, 10),
    ("type2_200x200", 3, None, 10_000, 50, 10),
    ("mixed_5..300", 4, None, 200_000, 200, 5),
    ("hyperbox_n5", 5, "box5", 4_000_000, 0, 10),
    ("hyperbox_n28", 5, "box28", 6_000_000, 0, 10),
]


def bench_classes(blp, torch, lpgen, plan=None) -> dict:
    """Every workload at its stated size: persistent LPs/s (mean and median
    of the timed runs' device times, HIP events between back-to-back runs),
    the kernel classes it used, one-LP-per-launch on all of its LPs or on a
    stated leading subset, and for the mixed batch the autotuned rate; for
    workload 5 also the backward pass (LPs/s, bytes and HBM fraction)."""
    res = {}
    names = [v[0] for v in blp.variants()] + ["streaming", "hyperbox", "binning"]
    for name, cfg, part, n_batch, n_single, runs in (plan or CLASS_PLAN):
        log(f"class {name}: generating {n_batch} LPs")
        t0 = time.perf_counter()
        hb = lpgen.config(cfg, range(n_batch), part=part) if part else lpgen.config(cfg, range(n_batch))
        log(f"class {name}: generated in {time.perf_counter() - t0:.1f} s; copying to HBM")
        db = blp.DeviceBatch.from_host(hb)
        # kernel classes and their device times from one profiled solve
        ms1, kms, _, bins = time_solver(blp, torch, db, 1, 1)
        log(f"class {name}: one profiled solve {ms1:.2f} ms")
        # short classes: warm-up of at least 100 ms of wall time, then the
        # timed runs back to back (no profiling events)
        warm = max(1, min(32, int(np.ceil(20.0 / max(ms1, 1e-3)))))
        ts = []
        ms, _, out, _ = time_solver(blp, torch, db, runs, warm if ms1 < 100 else 0, profile=False,
                                    warm_ms=100.0 if ms1 < 100 else 0.0, step_times=ts)
        st = np.bincount(out["status"][:n_batch].cpu().numpy(), minlength=5).tolist()
        med = float(np.median(ts))
        entry = {"lps": n_batch, "persistent_lps_per_s": round(n_batch / (med / 1e3), 1),
                 "persistent_lps_per_s_mean": round(n_batch / (float(np.mean(ts)) / 1e3), 1),
                 "wall_ms_per_run": round(ms, 3), "device_ms": _stats(ts), "statuses": st,
                 "bins": {names[i]: int(bins[i]) for i in range(len(bins)) if bins[i]},
                 "kernel_ms": {names[i]: round(float(kms[i]), 4) for i in range(len(kms)) if kms[i] > 0}}
        if part and part.startswith("box"):
            # Eq. (7) streams c, l, u in and x, obj, status, iters out
            n = int(hb.n[0])
            kb = float(kms[len(blp.variants()) + 1])
            byt = n_batch * (24.0 * n + 8.0 * n + 16.0)
            entry.update({"kernel_ms": round(kb, 4), "algorithmic_bytes": byt, "GBps": round(byt / kb / 1e6, 1),
                          "hbm_frac": round(byt / kb / 1e6 / PEAK_HBM_GBS, 4),
                          "note": "batch larger than the 256 MB last-level cache; bytes are the algorithmic "
                                  "stream (HBM counters of the same kernels in profiles/)"})
        if cfg == 3:
            # the streaming kernel reads and writes each stored tableau entry
            # once per pivot (ldk x (n + n_art + 1) in phase 1, the artificial
            # columns skipped in phase 2); part of it hits the L2 and the
            # last-level cache, so this is a tableau stream, not HBM traffic
            m, n = int(hb.m[0]), int(hb.n[0])
            sense = hb.sense.reshape(n_batch, m) != 0
            b = hb.b.reshape(n_batch, m)
            nart = ((np.where(sense, -b, b)) < 0).sum(axis=1)
            it = out["iters"][:n_batch].cpu().numpy().astype(np.float64)
            gms = float(kms[len(blp.variants())])
            stored = float((it * 16.0 * (m + 2) * (n + nart + 1)).sum())
            entry.update({"streaming_kernel_ms": round(gms, 3), "pivots_per_lp": round(float(it.mean()), 1),
                          "tableau_stream_GBps_l2_mall_hbm": round(stored / gms / 1e6, 1),
                          "tableau_stream_note": "16 B per stored entry per pivot (phase-1 width, an upper "
                                                 "bound); served by L2, the last-level cache and HBM"})
        if n_single is None or n_single > 0:
            S = n_batch if n_single is None else n_single
            sub = db if S == n_batch else blp.DeviceBatch.from_host(
                lpgen.config(cfg, range(S), part=part) if part else lpgen.config(cfg, range(S)))
            log(f"class {name}: one LP per launch on {S} LPs")
            ms1, _, _, _ = time_solver(blp, torch, sub, 1, 0, mode=blp.BLP_MODE_ONE_PER_LAUNCH)
            entry["one_per_launch_lps_per_s"] = round(S / (ms1 / 1e3), 1)
            entry["one_per_launch_sample"] = "all LPs" if S == n_batch else f"first {S} LPs"
            entry["speedup"] = round(entry["persistent_lps_per_s"] / entry["one_per_launch_lps_per_s"], 2)
            del sub
        if cfg == 4:
            entry["autotuned"] = autotune_gain(blp, torch, db, n_batch, med)
        if cfg == 5:
            entry["backward"] = bench_backward(blp, torch, lpgen, hb, db, part)
        res[name] = entry
        log(f"  {name}: {entry}")
        del db, hb, out
        torch.cuda.empty_cache()
    return res


def lane_scaling(blp, torch, lpgen) -> dict:
    """Tiny LPs (workload 1's recipe, 5 x 5) at several batch sizes: the
    automatic choice (one LP per lane once the batch is large enough) against
    one LP per wave forced (variant w1_r8_c8); device ms per step, median."""
    names = [v[0] for v in blp.variants()]
    w1 = names.index("w1_r8_c8")
    res = {}
    for K in (1_000, 16_384, 200_000):
        db = blp.DeviceBatch.from_host(lpgen.config(1, range(K)))
        e = {}
        for mode, kw in (("automatic", {}), ("one_lp_per_wave", {"variant": w1})):
            ts = []
            _, _, out, bins = time_solver(blp, torch, db, 20, 5, profile=False, warm_ms=50.0, step_times=ts, **kw)
            med = float(np.median(ts))
            e[mode] = {"median_ms": round(med, 4), "lps_per_s": round(K / (med / 1e3), 1),
                       "bins": {names[i]: int(bins[i]) for i in range(len(names)) if bins[i]}}
        e["automatic_over_one_per_wave"] = round(e["one_lp_per_wave"]["median_ms"] / e["automatic"]["median_ms"], 3)
        res[f"K{K}"] = e
        log(f"lane scaling K={K}: {e}")
    return res


def graph_replay(blp, torch, lpgen, runs=50) -> dict:
    """Captured launch sequence (hipGraph, replayed per batch signature)
    against eager launches, on batches solved over and over: small batches,
    where launch overheads weigh most.  Device time per step from HIP events
    between back-to-back steps; results identical either way."""
    res = {}
    for name, hb in (("type1_5x5_x1000", lpgen.config(1, range(1000))),
                     ("mixed_20..150_x2000", lpgen.config(5, range(2000), part="simplex")),
                     ("mixed_5..300_x500", lpgen.config(4, range(500)))):
        db = blp.DeviceBatch.from_host(hb)
        e = {}
        objs = {}
        for mode, graph in (("eager", False), ("graph", True)):
            ts = []
            ms, _, out, _ = time_solver(blp, torch, db, runs, 5, profile=False, warm_ms=50.0, step_times=ts,
                                        graph=graph)
            e[mode] = {"median_ms": round(float(np.median(ts)), 4), "wall_ms_per_step": round(ms, 4)}
            objs[mode] = out["obj"][:hb.count].cpu().numpy().view(np.int64)
        e["graph_over_eager"] = round(e["graph"]["median_ms"] / e["eager"]["median_ms"], 3)
        e["identical"] = bool(np.array_equal(objs["eager"], objs["graph"]))
        res[name] = e
        log(f"graph replay {name}: {e}")
    return res


def autotune_gain(blp, torch, db, K, base_ms, sample=256, runs=3) -> dict:
    """The autotuner on the batch itself (a calibration sample per size bin,
    every variant able to hold the bin), then the tuned solve timed."""
    s = blp.Solver()
    t0 = time.perf_counter()
    s.autotune(db, sample=sample)
    tune_s = time.perf_counter() - t0
    remap = blp.blp_tuning(s.h)
    s.close()
    names = [v[0] for v in blp.variants()] + ["streaming"]
    changed = {names[v]: names[w] for v, w in enumerate(remap) if w != v}
    # a tuned handle: load the remap through a cache file
    import tempfile
    s = blp.Solver()
    path = os.path.join(tempfile.mkdtemp(), "tune.json")
    s.autotune(db, sample=sample, cache_path=path)
    s.close()
    deep = json.load(open(path)).get("streaming_deep")
    ts = []
    ms, _, out, _ = time_solver(blp, torch, db, runs, 0, profile=False, step_times=ts, tune_cache=path)
    med = float(np.median(ts))
    return {"sample_per_bin": sample, "tuning_s": round(tune_s, 2), "remap": changed,
            "streaming_loads_in_flight": {1: 32, 0: 8}.get(deep, "automatic"),
            "device_ms": _stats(ts), "lps_per_s": round(K / (med / 1e3), 1),
            "gain_vs_untuned": round(base_ms / med, 3)}


def bench_backward(blp, torch, lpgen, hb, db, part, runs=10) -> dict:
    """blp_backward after a solve of the batch: loss = sum w_k opt_k with
    w ~ U(0, 1); LPs/s and the algorithmic HBM bytes (simplex: read status,
    g, x, y, write dc, db, dA; hyperbox: read status, g, c, x, write dc, dl,
    du)."""
    K = hb.count
    s = blp.Solver()
    out = s.solve(db)
    w = torch.from_numpy(lpgen.weights(lpgen.SEEDS[5] + 100, np.arange(K))).to("cuda")
    grads = s.backward(w)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(runs + 1)]
    evs[0].record(stream)
    for i in range(runs):
        grads = s.backward(w, out=grads)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    ts = [evs[i].elapsed_time(evs[i + 1]) for i in range(runs)]
    s.close()
    m = hb.m.astype(np.float64)
    n = hb.n.astype(np.float64)
    if part == "simplex":
        byt = float((12.0 + 8.0 * (m + n) + 8.0 * (m * n + m + n)).sum())
    else:
        byt = float((12.0 + 16.0 * n + 24.0 * n).sum())
    med = float(np.median(ts))
    # (the gradient buffers are allocated and zeroed once, by the untimed
    # first call, and rewritten by each timed one)
    return {"lps": K, "device_ms": _stats(ts), "lps_per_s": round(K / (med / 1e3), 1), "algorithmic_bytes": byt,
            "GBps": round(byt / med / 1e6, 1), "hbm_frac": round(byt / med / 1e6 / PEAK_HBM_GBS, 4)}


if __name__ == "__main__":
    main()
