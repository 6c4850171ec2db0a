#!/usr/bin/env python3
"""Benchmark of the FP16 block-floating-point FFT path on one MI355X.

Headline (one JSON line on stdout): fused FP16-BFP range compression of a
2048-pulse x 4096-sample synthetic echo (5 LFM targets, 20 dB noise): per
pulse a forward FFT, the matched-filter product, the exact 2^-12 prescale
folded into the conjugate, and the inverse FFT, one HBM read and one HBM
write per pulse.  GFLOP/s use the paper's convention, 5 N log2 N per
transform (two transforms per pulse), from GPU event timestamps.

A step is one kernel launch over one 2048-pulse batch.  The batches rotate
through 16 distinct input/output buffer pairs (1 GiB in total), so the
working set cannot sit in the 256 MB last-level cache and every step streams
from HBM.  Secondary figures (FP32 path, other precision modes, plain FFT at
N = 4096, SQNR against the FP64 oracle, the oracle's own CPU throughput) are
added to the same line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP16-BFP FFT GFLOP/s (5N·log2N) + SAR frames/s at stated SQNR vs FP32 path"
# headline precision mode and the kernel that carries it
HEAD_MODE = "fp16"
RADIX_PLANS_4096 = {0: "16 16 16, 16 values per thread", 1: "8 8 8 8, 8 values per thread"}


def head_kernel_text(t):
    """The headline kernel the autotuner chose (rows.hip)."""
    if t is None:
        return "row_kernel (rows.hip), default tuning"
    if t["rows_per_thread"] == 1 and t["radix_plan"] == 0 and t["blocks_per_cu"] != 0 \
            and t["engine"] != "matrix cores":
        # persistent grids of the pure-FP16 compression at 4096 points: the
        # pipelined form with one LDS buffer per row
        kern = "row_kernel_rr<ModeFP16, 12, OP_COMPRESS, V_PLAIN, RR = 1, NB = 1, PIPE>"
    elif t["rows_per_thread"] > 1 or t["radix_plan"] == 1:
        kern = "row_kernel_rr<ModeFP16, 12, OP_COMPRESS, V_PLAIN>"
    else:
        kern = "row_kernel<ModeFP16, 12, OP_COMPRESS, V_PLAIN>"
    grid = ("one workgroup per row group" if t["blocks_per_cu"] == 0 else
            "the default grid" if t["blocks_per_cu"] < 0 else
            f"a persistent grid of {t['blocks_per_cu']} workgroups per CU")
    return (f"{kern} (rows.hip), {t['engine']}, radix plan "
            f"{t['radix_plan']} ({RADIX_PLANS_4096[t['radix_plan']]}), {t['rows_per_thread']} row(s) per "
            f"thread, {grid}; " + ("chosen by the library autotuner on the rotating buffers"
                                   if t["tuned_ms"] is not None else "set by --tuning"))


MODE_TEXT = {
    "fp16": "pure FP16 (packed half2 arithmetic, FP16 LDS and twiddles)",
    "fp16_mul_fp32_acc": "FP16 multiply / FP32 accumulate (radix-16 butterflies on the matrix cores)",
}
HBM_PEAK_GBS = 8000.0
# bytes of one stored complex value per precision mode
STORE_BYTES = {"fp32": 8, "fp16": 4, "fp16_fp32": 4, "fp16_mul_fp32_acc": 4, "e4m3": 2, "e5m2": 2}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "range_compress_2048x4096_traffic.json")


def measured_traffic(mode):
    """HBM bytes per launch of the fused compression from the committed PMC
    summary, or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources") != KERNEL_SOURCES or \
            kernel_source_sha256() != rec.get("kernel_source_sha256"):
        return None
    m = rec.get("modes", {}).get(mode)
    return None if m is None else m["traffic_bytes"]


KERNEL_SOURCES = ["rows.hip", "fft_engine.hpp", "fft_device.hpp", "fft_mfma.hpp", "internal.hpp"]


def kernel_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_28451_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_summary(specs):
    """Turn rocprofv3 --pmc databases of `bench.py --kernel-only <mode>` runs
    into the committed traffic record.  specs: [(mode, fetch_dir, write_dir)],
    each dir holding one run with FETCH_SIZE resp. WRITE_SIZE.  Per counter
    the kernel's mean KiB per dispatch is scaled by known bytes / KiB of the
    device copy that the same run performs (the compression's bytes: half
    read, half written; 32 MiB each way in the 4-byte storage modes)."""
    import glob
    import sqlite3

    def means(d):
        dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
        if len(dbs) != 1:
            raise SystemExit(f"expected one rocprofv3 database under {d}, found {len(dbs)}")
        con = sqlite3.connect(dbs[0])
        rows = con.execute("select kernel_name, value from counters_collection").fetchall()
        agg = {}
        for name, v in rows:
            agg.setdefault(name, []).append(float(v))
        kern = [k for k in agg if "bfp::row_kernel" in k]
        copy = [k for k in agg if "bfp::copy_kernel" in k]
        if not kern or len(copy) != 1:
            raise SystemExit(f"no row kernel / copy kernel dispatches in {dbs[0]}")
        k = max(kern, key=lambda n: len(agg[n]))
        return k, sum(agg[k]) / len(agg[k]), sum(agg[copy[0]]) / len(agg[copy[0]])

    rec = {"workload": "fused range compression, 2048 x 4096 (FP16, FP32 or FP8 storage)",
           "source": "profiles/range_compress_2048x4096_hbm_traffic.md",
           "kernel_sources": KERNEL_SOURCES, "kernel_source_sha256": kernel_source_sha256(),
           "modes": {}}
    lines = ["| mode | kernel | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | copy FETCH / WRITE KiB |",
             "|---|---|---|---|---|"]
    notes = []
    for mode, fdir, wdir in specs:
        algo = 2 * 2048 * 4096 * STORE_BYTES[mode]
        copy_kib = algo // 2 // 1024  # the copy moves the compression's bytes, half each way
        kf, f_kib, cf = means(fdir)
        kw, w_kib, cw = means(wdir)
        ff, fw = copy_kib / cf, copy_kib / cw
        traffic = int(round(f_kib * ff * 1024 + w_kib * fw * 1024))
        rec["modes"][mode] = {"traffic_bytes": traffic, "algorithmic_bytes": algo,
                              "fetch_factor": round(ff, 4),
                              "write_factor": round(fw, 4), "kernel": kf}
        lines.append(f"| {mode} | `{kf[:70]}` | {f_kib:.1f} | {w_kib:.1f} | {cf:.1f} / {cw:.1f} |")
        notes.append(f"- {mode}: fetch {f_kib:.0f} KiB x {ff:.3f} + write {w_kib:.0f} KiB x {fw:.3f} = "
                     f"{traffic} B ({traffic / algo:.3f} x algorithmic {algo} B)")
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print("\n".join(lines + [""] + notes))


def trace_summary(d, top=12, tail=None):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (its database).
    tail: only the last `tail` dispatches of the library's own kernels (the
    timed region of a run that also autotunes and stages inputs)."""
    import glob
    import sqlite3
    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if len(dbs) != 1:
        raise SystemExit(f"expected one rocprofv3 database under {d}, found {len(dbs)}")
    con = sqlite3.connect(dbs[0])
    if tail:
        disp = [r for r in con.execute("select name, duration from kernels order by start").fetchall()
                if "bfp::" in r[0] or r[0].startswith("_ZN3bfp")][-tail:]
        agg = {}
        for name, dur in disp:
            agg.setdefault(name, []).append(dur)
        rows = sorted(((k, len(v), sum(v), sum(v) / len(v), min(v), max(v)) for k, v in agg.items()),
                      key=lambda r: -r[2])
    else:
        rows = con.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                           "max(duration) from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    out = ["| kernel | calls | average us | min us | max us | share of GPU time |",
           "|---|---|---|---|---|---|"]
    for name, n, tot, avg, mn, mx in rows[:top]:
        name = name if len(name) <= 90 else name[:87] + "..."
        out.append(f"| `{name}` | {n} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | "
                   f"{100.0 * tot / total:.1f}% |")
    print("\n".join(out))


def _finite_or_none(x, nd):
    """Rounded float, or None where a collapsed image gives no finite figure
    (the JSON line stays strict)."""
    x = float(x)
    return round(x, nd) if np.isfinite(x) else None


def fft_flops(n, transforms):
    import math
    return 5.0 * n * math.log2(n) * transforms


def time_launches(launch, n_sets, steps, warmup):
    """Run `launch(i)` (kernel launches on the current stream) for warmup +
    steps iterations rotating over n_sets buffer sets.  The timed steps are
    issued back to back between one pair of events on that stream; returns
    (average ms per step, total timed ms)."""
    import torch
    for i in range(warmup):
        launch(i % n_sets)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for i in range(steps):
        launch(i % n_sets)
    ev1.record()
    torch.cuda.synchronize()
    total = ev0.elapsed_time(ev1)
    return total / steps, total


def rotating_sets(make, n_sets):
    return [make(i) for i in range(n_sets)]


def tuning_record(plan, ms):
    e, b, rr, pl = plan.get_tuning_ex()
    return {"engine": "matrix cores" if e == 0 else "vector ALU", "blocks_per_cu": b,
            "rows_per_thread": rr, "radix_plan": pl,
            "tuned_ms": None if ms is None else round(ms, 5)}


def parse_tuning(text):
    """'engine,blocks_per_cu,rows_per_thread,radix_plan' -> 4-tuple of ints."""
    t = tuple(int(v) for v in text.split(","))
    if len(t) != 4:
        raise SystemExit("--tuning takes engine,blocks_per_cu,rows_per_thread,radix_plan")
    return t


def bench_compress(mode, rows, n, steps, warmup, min_bytes=1 << 30, adaptive=False, tune=True,
                   fixed=None, blocks=1):
    """Fused range compression in `mode`, rotating buffers totalling >= min_bytes
    (adaptive: the per-row adaptive block shift, with its exponent rows).
    tune: the library's autotuner picks engine, grid, rows per thread and
    radix plan on the same rotating buffers before the timed steps; fixed
    (a tuning 4-tuple) sets them instead, so that a profiled run holds the
    one kernel configuration only.  blocks > 1: that many timed blocks of
    `steps` launches, the median block reported (secondary rows: a single
    block of this workload has measured up to 15% off on a box)."""
    import torch
    from paper_2605_28451_amd import api, scenes
    sc = scenes.range_scene(seed=2, n_pulses=rows, n=n)
    fmt = api.storage_format(mode)
    echo0 = api.to_device(sc.echo, fmt)
    set_bytes = 2 * echo0.numel() * echo0.element_size()
    n_sets = max(1, -(-min_bytes // set_bytes))
    ins = [echo0 if i == 0 else echo0.clone() for i in range(n_sets)]
    outs = [torch.empty_like(echo0) for _ in range(n_sets)]
    plan = api.FFTPlan(n, rows, mode)
    H = api.filter_tensor(sc.replica, n, mode)

    exps = [torch.empty(rows, dtype=torch.int32, device="cuda") for _ in range(n_sets)]
    if fixed is not None:
        plan.set_tuning_ex(*fixed)
        tuning = tuning_record(plan, None)
    elif tune and not adaptive:
        tuning = tuning_record(plan, plan.autotune_on(2, ins, outs, H, reps=10))
    else:
        tuning = None

    def launch(i):
        if adaptive:
            plan.range_compress_adaptive(ins[i], H, out=outs[i], row_exp=exps[i])
        else:
            plan.range_compress(ins[i], H, out=outs[i])

    timed = sorted(time_launches(launch, n_sets, steps, warmup) for _ in range(max(1, blocks)))
    ms, total = timed[len(timed) // 2]
    res = {
        "mode": mode, "rows": rows, "n": n, "buffer_sets": n_sets, "timed_blocks": max(1, blocks),
        "working_set_mib": round(n_sets * set_bytes / 2 ** 20, 1),
        "ms_per_launch": ms,
        "ms_total": total,
        "bytes_per_launch": set_bytes,
        "tuning": tuning,
    }
    res["gflops"] = fft_flops(n, 2 * rows) / (res["ms_per_launch"] * 1e-3) / 1e9
    res["hbm_gbs"] = set_bytes / (res["ms_per_launch"] * 1e-3) / 1e9
    # parity sample: first 64 pulses of the first output
    torch.cuda.synchronize()
    res["_sample_out"] = api.to_host(outs[0][:64], fmt)
    res["_sample_in"] = scenes.quantize(sc.echo[:64], fmt)
    res["_sample_in_raw"] = sc.echo[:64]
    res["_replica"] = sc.replica
    del ins, outs, echo0
    plan.close()
    torch.cuda.empty_cache()
    return res


def bench_fft(mode, rows, n, steps, warmup, min_bytes=1 << 30, inverse=False, tune=True):
    import torch
    from paper_2605_28451_amd import api, scenes
    fmt = api.storage_format(mode)
    x0 = api.to_device(scenes.gaussian_rows(1, 64, n), fmt)
    x0 = x0.repeat((rows + 63) // 64, 1, 1)[:rows].contiguous()
    set_bytes = 2 * x0.numel() * x0.element_size()
    n_sets = max(1, -(-min_bytes // set_bytes))
    ins = [x0 if i == 0 else x0.clone() for i in range(n_sets)]
    outs = [torch.empty_like(x0) for _ in range(n_sets)]
    plan = api.FFTPlan(n, rows, mode)
    tuning = tuning_record(plan, plan.autotune_on(1 if inverse else 0, ins, outs, reps=10)) if tune else None
    if inverse:
        launch = lambda i: plan.inverse_bfp(ins[i], out=outs[i])  # noqa: E731
    else:
        launch = lambda i: plan.forward(ins[i], out=outs[i])  # noqa: E731
    ms, total = time_launches(launch, n_sets, steps, warmup)
    res = {"mode": mode, "op": "inverse_bfp" if inverse else "forward", "rows": rows, "n": n,
           "buffer_sets": n_sets, "ms_per_launch": ms, "tuning": tuning,
           "gflops": fft_flops(n, rows) / (ms * 1e-3) / 1e9,
           "hbm_gbs": set_bytes / (ms * 1e-3) / 1e9}
    res["hbm_frac"] = res["hbm_gbs"] / HBM_PEAK_GBS
    del ins, outs, x0
    plan.close()
    torch.cuda.empty_cache()
    return res


_ORACLE_FRAMES = {}


def frame_vs_oracle(sc, mode, img, pts):
    """The GPU frame against the FP64 oracle's frame of the same storage-
    rounded echo and filters: unaligned SQNR and the largest per-target
    differences of PSLR, ISLR, SNR (dB) and IRW (samples)."""
    import numpy as np
    import oracle
    from paper_2605_28451_amd import api, metrics, scenes
    n = img.shape[0]
    fmt, ffmt = api.storage_format(mode), api.filter_format(mode)
    if (fmt, ffmt) not in _ORACLE_FRAMES:
        Hr = scenes.quantize(oracle.matched_filter(sc.range_replica, n), ffmt)
        Ha = scenes.quantize(oracle.matched_filter(sc.azimuth_replica, n), ffmt)
        ref = oracle.sar_image(scenes.quantize(sc.echo, fmt), Hr, Ha)
        _ORACLE_FRAMES[(fmt, ffmt)] = (ref, [metrics.point_target(ref, r0, a0, noise_patch=(r0 + 300, a0 + 300))
                                             for (r0, a0) in sc.targets])
    ref, ref_pts = _ORACLE_FRAMES[(fmt, ffmt)]
    d = {k: max(abs(p[k] - q[k]) for p, q in zip(pts, ref_pts))
         for k in ("pslr_range", "pslr_azimuth", "islr_range", "islr_azimuth", "snr", "irw_range",
                   "irw_azimuth")}
    return {"sqnr_db": _finite_or_none(metrics.sqnr_db(ref, img), 2),
            "max_abs_delta_pslr_db": _finite_or_none(max(d["pslr_range"], d["pslr_azimuth"]), 3),
            "max_abs_delta_islr_db": _finite_or_none(max(d["islr_range"], d["islr_azimuth"]), 3),
            "max_abs_delta_snr_db": _finite_or_none(d["snr"], 3),
            "max_abs_delta_irw_samples": _finite_or_none(max(d["irw_range"], d["irw_azimuth"]), 4)}


def bench_sar_frame(mode, steps, warmup, n_frames=4, graph=True, fused_ct=False, streams=1, tune=True):
    """Full 4096x4096 range-Doppler frame: fused range compression, LDS-tiled
    corner turn, fused azimuth compression (fused_ct: the corner turn folded
    into the range compression's store, no separate pass).  n_frames
    independent frame buffer sets rotate (4 x 256 MiB for FP16) and two
    rounds over them (8 frames: a replay carries a fixed cost on the device)
    are captured once in a HIP graph.  streams > 1: the
    frames of a replay are dealt round-robin to that many streams (default
    priority) forked and joined inside the graph, so independent frames run
    concurrently (frame k's memory-bound corner turn beside frame k+1's
    compressions); each frame's three steps stay in order on its stream."""
    import torch
    from paper_2605_28451_amd import api
    fmt = api.storage_format(mode)
    sc = _sar_scene()
    n = 4096
    echo0 = api.to_device(sc.echo, fmt)
    echoes = [echo0] + [echo0.clone() for _ in range(n_frames - 1)]
    rcs = [torch.empty_like(echo0) for _ in range(n_frames)]
    rcts = [torch.empty_like(echo0) for _ in range(n_frames)]
    imgs = [torch.empty_like(echo0) for _ in range(n_frames)]
    rplan = api.FFTPlan(n, n, mode)
    aplan = api.FFTPlan(n, n, mode)
    Hr = api.filter_tensor(sc.range_replica, n, mode)
    Ha = api.filter_tensor(sc.azimuth_replica, n, mode)

    def frame(i):
        if fused_ct:
            rplan.range_compress(echoes[i], Hr, out=rcts[i], transposed=True)
        else:
            rplan.range_compress(echoes[i], Hr, out=rcs[i])
            api.corner_turn(rcs[i], fmt, out=rcts[i])
        aplan.azimuth_compress(rcts[i], Ha, out=imgs[i])

    for i in range(max(warmup, n_frames)):
        frame(i % n_frames)
    torch.cuda.synchronize()
    tuning = None
    if tune and not fused_ct:
        # both compressions tuned on the frame's own rotating buffers (the
        # transposed store keeps its default grid)
        tr = tuning_record(rplan, rplan.autotune_on(2, echoes, rcs, Hr, reps=5))
        ta = tuning_record(aplan, aplan.autotune_on(2, rcts, imgs, Ha, reps=5))
        tuning = {"range": tr, "azimuth": ta}
        for i in range(n_frames):
            frame(i)
        torch.cuda.synchronize()
    per_graph = 2 * n_frames
    reps = max(1, -(-steps // per_graph))
    if graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        side = [torch.cuda.Stream() for _ in range(streams - 1)]
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                if streams == 1:
                    for i in range(per_graph):
                        frame(i % n_frames)
                else:
                    lanes = [s] + side
                    for q in side:
                        q.wait_stream(s)  # fork
                    for i in range(per_graph):
                        with torch.cuda.stream(lanes[i % streams]):
                            frame(i % n_frames)
                    for q in side:
                        s.wait_stream(q)  # join
        torch.cuda.current_stream().wait_stream(s)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / (reps * per_graph)
    else:
        ms, total = time_launches(frame, n_frames, reps * n_frames, 0)
    # RC r/w, (CT r/w,) AC r/w
    bytes_frame = (4 if fused_ct else 6) * echo0.numel() * echo0.element_size()
    res = {"mode": mode, "ms_per_frame": ms, "frames_per_s": 1e3 / ms,
           "hbm_gbs": bytes_frame / (ms * 1e-3) / 1e9, "bytes_per_frame": bytes_frame,
           "gflops": fft_flops(n, 4 * n) / (ms * 1e-3) / 1e9, "graph": graph,
           "frames_rotating": n_frames, "frames_per_replay": per_graph if graph else None,
           "corner_turn": "fused into the range store" if fused_ct
           else "separate LDS-tiled pass", "concurrent_streams": streams, "tuning": tuning}
    torch.cuda.synchronize()
    res["_img"] = api.to_host(imgs[0], fmt)
    res["_scene"] = sc
    del echoes, rcs, rcts, imgs
    torch.cuda.empty_cache()
    return res


def bench_uneven(mode, steps, warmup, with_sqnr=True):
    """The 20,000-transform uneven batch (N log-uniform in 256..16384,
    random directions) in one launch: the plan's grid autotuned on the
    batch, 8 launches captured in a HIP graph over two rotating buffer sets;
    eager launches timed beside it; SQNR per size and direction against the
    FP64 oracle."""
    import numpy as np
    import torch
    from paper_2605_28451_amd import api, scenes
    ub = scenes.uneven_batch(seed=4, count=20000)
    fmt = api.storage_format(mode)
    x0 = api.to_device(ub.x, fmt)
    sets = 2
    ins = [x0, x0.clone()]
    outs = [torch.empty_like(x0) for _ in range(sets)]
    plan = api.UnevenPlan(ub.log2n, ub.inverse, mode)
    tuned_ms = plan.autotune_on(0, ins[0], outs[0], reps=10)
    tuning = plan.get_tuning()
    # the median of three timed blocks: single blocks of this workload vary
    # by up to 10% between blocks on one box
    ms_eager = sorted(time_launches(lambda i: plan.execute(ins[i], out=outs[i]), sets, steps,
                                    warmup)[0] for _ in range(3))[1]
    # a replay carries a fixed cost on the device (measured ≈ 8 us beside
    # one large kernel): 16 launches per replay, alternating the two sets
    # (measured per launch: 152-155 us with one per replay, 148-150 with 8,
    # 148 with 16, eager 148)
    per_graph = 16
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for i in range(per_graph):
                plan.execute(ins[i % sets], out=outs[i % sets])
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    reps = max(1, -(-steps // per_graph))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    blocks = []
    for _ in range(3):
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        blocks.append(e0.elapsed_time(e1) / (reps * per_graph))
    ms = sorted(blocks)[1]
    sizes = (1 << ub.log2n.astype("int64"))
    flops = float(np.sum(5.0 * sizes * ub.log2n))
    bytes_ = 2 * x0.numel() * x0.element_size()
    res = {"mode": mode, "transforms": 20000, "ms_per_launch": ms, "ms_per_launch_eager": ms_eager,
           "graph": "16 launches per replay over 2 rotating buffer sets (queue reset, when the grid "
                    "claims from the queue, and the kernel); median of 3 timed blocks",
           "autotuned_workgroups_per_cu": tuning[1], "autotune_ms": tuned_ms,
           "gflops": flops / (ms * 1e-3) / 1e9, "hbm_gbs": bytes_ / (ms * 1e-3) / 1e9,
           "bytes_per_launch": bytes_}
    if with_sqnr:
        import oracle
        from paper_2605_28451_amd.metrics import sqnr_db
        xq = api.to_host(ins[0], fmt)
        y = api.to_host(outs[0], fmt)
        per = {}
        for e in range(8, 15):
            for inv in (0, 1):
                idx = np.nonzero((ub.log2n == e) & (ub.inverse == inv))[0]
                if idx.size == 0:
                    continue
                nn = 1 << e
                sel = (ub.offsets[idx][:, None] + np.arange(nn)[None]).ravel()
                ref = oracle.fft(xq[sel].reshape(idx.size, nn), inverse=bool(inv))
                per[f"{nn}_{'inverse_bfp' if inv else 'forward'}"] = {
                    "transforms": int(idx.size),
                    "sqnr_db_vs_fp64_oracle": round(sqnr_db(ref, y[sel].reshape(idx.size, nn)), 2)}
        res["sqnr_by_size"] = per
    del ins, outs, x0
    torch.cuda.empty_cache()
    return res


def bench_autofocus(steps, lr_max=2.5, lr_min=0.02, with_oracle=True, per_replay=5):
    """`steps` Adam steps (cosine learning-rate schedule from lr_max to
    lr_min, read on the device) of entropy autofocus on the 4096x4096 frame
    with the injected per-pulse phase error: ms per step (graph replays of
    `per_replay` iterations each, and eager), entropy and azimuth PSLR/ISLR
    before and after, beside the image
    the FP64 oracle forms with the true correction, and the GPU gradient at
    phase 0 against FP64 central differences of the oracle's entropy."""
    import numpy as np
    import torch
    from paper_2605_28451_amd import api, metrics, scenes
    from paper_2605_28451_amd.autofocus import (AutofocusLoop, AutofocusPlan, cosine_schedule,
                                                entropy_and_grad)
    n = 4096
    perr = scenes.autofocus_phase_error(seed=5, n_pulse=n)
    sc = scenes.sar_scene(seed=3, phase_error=perr)
    mode = "fp16_fp32"
    rplan = api.FFTPlan(n, n, mode)
    Hr = api.filter_tensor(sc.range_replica, n, mode)
    rc = rplan.range_compress(api.to_device(sc.echo, "fp16"), Hr)
    rct = api.corner_turn(rc, "fp16")
    plan = AutofocusPlan(n, n, mode)
    Ha = api.filter_tensor(sc.azimuth_replica, n, mode)
    sched = cosine_schedule(steps, lr_max, lr_min)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    k = per_replay if steps % per_replay == 0 else 1

    def run(graph):
        """`steps` iterations from phase 0 (library kernels only; k captured
        iterations per replay when graph)."""
        phi = torch.zeros(n, dtype=torch.float32, device="cuda")
        loop = AutofocusLoop(plan, rct, Ha, phi, graph=graph, lr_schedule=sched,
                             iterations_per_step=k if graph else 1)
        E0 = float(loop.entropy())
        img0 = api.to_host(loop.img, "fp32")
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps // loop.k):
            loop.step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        E = float(loop.entropy())
        return ms, E0, E, img0, api.to_host(loop.img, "fp32"), phi

    ms, E0, E, img0, img1, phi_g = run(graph=True)
    ms_eager, _, E_eager, _, _, phi_e = run(graph=False)
    # the image, entropy and phase gradient alone (no update), back to back
    img = torch.empty((n, n, 2), dtype=torch.float32, device="cuda")
    stats = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.empty(n, dtype=torch.float32, device="cuda")
    e0.record()
    for _ in range(steps):
        entropy_and_grad(plan, rct, Ha, phi_g, img=img, stats=stats, grad=grad)
    e1.record()
    torch.cuda.synchronize()
    ms_grad = e0.elapsed_time(e1) / steps

    def az(im):
        pts = [metrics.point_target(im, r0, a0, search=64) for (r0, a0) in sc.targets]
        return (float(np.mean([p["pslr_azimuth"] for p in pts])),
                float(np.mean([p["islr_azimuth"] for p in pts])))

    out = {"ms_per_step": ms, "ms_per_step_eager": ms_eager, "ms_per_gradient": ms_grad,
           "graph_equals_eager": bool(torch.equal(phi_g, phi_e)), "steps": steps,
           "iterations_per_replay": k,
           "lr_schedule": f"cosine {lr_max} -> {lr_min} over {steps} steps (device-side)",
           "entropy_before": E0, "entropy_after": float(E)}
    out["pslr_azimuth_db_before"], out["islr_azimuth_db_before"] = az(img0)
    out["pslr_azimuth_db_after"], out["islr_azimuth_db_after"] = az(img1)
    if with_oracle:
        import oracle
        rct_h = api.to_host(rct, "fp16")
        Haq = scenes.quantize(oracle.matched_filter(sc.azimuth_replica, n), "fp16")
        E_true, _, img_true = oracle.autofocus(rct_h, Haq, -perr, want_image=True)
        out["entropy_focused_oracle"] = float(E_true)
        out["pslr_azimuth_db_focused_oracle"], out["islr_azimuth_db_focused_oracle"] = az(img_true)
        # the GPU gradient at phase 0 against the FP64 analytic gradient and
        # FP64 central differences of the oracle's entropy (3 largest pulses)
        z = torch.zeros(n, dtype=torch.float32, device="cuda")
        _, g_gpu, _ = entropy_and_grad(plan, rct, Ha, z)
        g_gpu = g_gpu.cpu().numpy().astype(np.float64)
        _, g_ref = oracle.autofocus(rct_h, Haq, np.zeros(n))
        fd_err, h = 0.0, 1e-4
        for m in np.argsort(-np.abs(g_ref))[:3]:
            pp = np.zeros(n); pp[m] = h
            fd = (oracle.autofocus(rct_h, Haq, pp)[0] - oracle.autofocus(rct_h, Haq, -pp)[0]) / (2 * h)
            fd_err = max(fd_err, abs(g_gpu[m] - fd) / abs(fd))
        out["gradient_rel_err_vs_fp64_analytic"] = float(np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref))
        out["gradient_max_rel_err_vs_fp64_central_differences"] = float(fd_err)
    out["_img0"], out["_img1"], out["_scene"] = img0, img1, sc
    return out


def cpu_baseline(sample_in, replica, n, sample_out):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload."""
    import numpy as np
    import oracle
    from paper_2605_28451_amd.metrics import sqnr_db
    from paper_2605_28451_amd import scenes
    H = oracle.matched_filter(replica, n)
    Hq = scenes.quantize(H, "fp16")
    rows = sample_in.shape[0]
    oracle.compress(sample_in[:4], Hq)  # warm the library
    reps = 0
    t0 = time.perf_counter()
    while True:
        ref = oracle.compress(sample_in, Hq)
        reps += 1
        if time.perf_counter() - t0 > 10.0:
            break
    dt = (time.perf_counter() - t0) / reps
    gflops = fft_flops(n, 2 * rows) / dt / 1e9
    sq = sqnr_db(ref, sample_out, align=True)
    sq_raw = sqnr_db(ref, sample_out, align=False)
    cores = oracle.num_threads()
    # context: the same oracle on one thread (a quarter of the sample; one
    # warm-up call after the thread change, then the best of three), and
    # numpy's FP64 FFT (pocketfft) for the same two transforms per pulse
    oracle.set_threads(1)
    try:
        oracle.compress(sample_in[:16], Hq)
        dt1 = 1e30
        for _ in range(3):
            t1 = time.perf_counter()
            oracle.compress(sample_in[:16], Hq)
            dt1 = min(dt1, time.perf_counter() - t1)
    finally:
        oracle.set_threads(cores)
    t2 = time.perf_counter()
    for _ in range(3):
        np.conj(np.fft.fft(np.conj(np.fft.fft(sample_in, axis=1) * Hq) / n, axis=1))
    dt2 = (time.perf_counter() - t2) / 3
    return {
        "value": gflops, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
        "sample": f"{rows} pulses x {n} of the same range-compression workload, repeated "
                  f"{reps}x ({dt * 1e3:.1f} ms per pass), FP64 recursive radix-2, OpenMP over pulses",
        "value_1_thread": fft_flops(n, 2 * 16) / dt1 / 1e9,
        "numpy_fft_fp64_gflops": fft_flops(n, 2 * rows) / dt2 / 1e9,
    }, sq, sq_raw


_MIGRATION_SCENE = []
_SAR_SCENE = []


def _sar_scene():
    """The 4096x4096 point-target frame (seed 3), generated once per process."""
    if not _SAR_SCENE:
        from paper_2605_28451_amd import scenes
        _SAR_SCENE.append(scenes.sar_scene(seed=3))
    return _SAR_SCENE[0]


def cpu_oracle_workloads(reps=3):
    """Context beside the CPU baseline: the FP64 oracle as it stands (all host
    threads) on the other workloads the GPU path is timed on, best of `reps`:
    the 64 x 4096 BFP round trip (forward, then normalised inverse), one
    4096 x 4096 range-Doppler frame, and the 20,000-transform uneven batch
    (transforms grouped by length and direction before the timed calls)."""
    import numpy as np
    import oracle
    from paper_2605_28451_amd import scenes

    def best(fn):
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            t.append(time.perf_counter() - t0)
        return min(t)

    res = {"threads": oracle.num_threads()}
    x = scenes.quantize(scenes.gaussian_rows(1, 64, 4096), "fp16")
    dt = best(lambda: oracle.fft(oracle.fft(x), inverse=True))
    res["round_trip_64x4096"] = {"ms": round(dt * 1e3, 3),
                                 "gflops": round(fft_flops(4096, 128) / dt / 1e9, 2)}
    sc = _sar_scene()
    echo = scenes.quantize(sc.echo, "fp16")
    Hr = scenes.quantize(oracle.matched_filter(sc.range_replica, 4096), "fp16")
    Ha = scenes.quantize(oracle.matched_filter(sc.azimuth_replica, 4096), "fp16")
    dt = best(lambda: oracle.sar_image(echo, Hr, Ha))
    res["sar_frame_4096"] = {"ms": round(dt * 1e3, 1), "frames_per_s": round(1.0 / dt, 2),
                             "gflops": round(fft_flops(4096, 4 * 4096) / dt / 1e9, 2)}
    ub = scenes.uneven_batch(seed=4, count=20000)
    xq = scenes.quantize(ub.x, "fp16")
    groups = []
    for e in np.unique(ub.log2n):
        for d in (0, 1):
            idx = np.nonzero((ub.log2n == e) & (ub.inverse == d))[0]
            if idx.size:
                n = 1 << int(e)
                rows = np.stack([xq[o:o + n] for o in ub.offsets[idx]])
                groups.append((rows, bool(d)))
    dt = best(lambda: [oracle.fft(r, inverse=d) for r, d in groups])
    flops = float(np.sum(5.0 * (1 << ub.log2n.astype(np.int64)) * ub.log2n))
    res["uneven_20000"] = {"ms": round(dt * 1e3, 1), "gflops": round(flops / dt / 1e9, 2)}
    return res


def _migration_scene():
    """The RCMC scene, generated once per process (about 3 s of numpy)."""
    if not _MIGRATION_SCENE:
        from paper_2605_28451_amd import scenes
        _MIGRATION_SCENE.append(scenes.migration_scene())
    return _MIGRATION_SCENE[0]


def bench_rcmc_frame(mode, steps, warmup, n_frames=4, streams=1):
    """4096x4096 range-Doppler frame with range cell migration correction:
    corner turn, azimuth FFT, corner turn, migration-corrected range
    compression per Doppler bin, corner turn, azimuth BFP inverse with H_a
    (12 passes over 64 MiB in FP16), n_frames rotating buffer sets, one HIP
    graph per replay (streams > 1: frames dealt to that many streams forked
    and joined inside the graph, as in bench_sar_frame); plus the focus
    metrics of the first image."""
    import torch
    from paper_2605_28451_amd import api, scenes, metrics
    fmt = api.storage_format(mode)
    sc = _migration_scene()
    n = 4096
    echo0 = api.to_device(sc.echo, fmt)
    echoes = [echo0] + [echo0.clone() for _ in range(n_frames - 1)]
    bufs = [[torch.empty_like(echo0) for _ in range(2)] for _ in range(n_frames)]
    aplan = api.FFTPlan(n, n, mode)
    rplan = api.FFTPlan(n, n, mode)
    Hr = api.filter_tensor(sc.range_replica, n, mode)
    Ha = api.filter_tensor(sc.azimuth_replica, n, mode)
    shift = torch.tensor(sc.rcmc_shift.astype(np.float32), device="cuda")

    def frame(i):
        a, b = bufs[i]
        api.corner_turn(echoes[i], fmt, out=a)
        aplan.forward(a, out=b)
        api.corner_turn(b, fmt, out=a)
        rplan.range_compress_rcmc(a, Hr, shift, out=b)
        api.corner_turn(b, fmt, out=a)
        aplan.inverse_bfp(a, Ha, out=b)

    for i in range(warmup):
        frame(i % n_frames)
    torch.cuda.synchronize()
    per_graph = 2 * n_frames  # two rounds over the sets per replay
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    side = [torch.cuda.Stream() for _ in range(streams - 1)]
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            lanes = [s] + side
            for q in side:
                q.wait_stream(s)
            for i in range(per_graph):
                with torch.cuda.stream(lanes[i % streams]):
                    frame(i % n_frames)
            for q in side:
                s.wait_stream(q)
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    reps = max(1, -(-steps // per_graph))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (reps * per_graph)
    img = api.to_host(bufs[0][1], fmt)
    pts = [metrics.point_target(img, r0, a0, noise_patch=(r0 + 300, a0 + 300)) for (r0, a0) in sc.targets]
    bytes_frame = 12 * echo0.numel() * echo0.element_size()
    del echoes, bufs
    aplan.close()
    rplan.close()
    torch.cuda.empty_cache()
    return {"mode": mode, "concurrent_streams": streams, "ms_per_frame": round(ms, 5),
            "frames_per_s": round(1e3 / ms, 1),
            "hbm_gbs": round(bytes_frame / (ms * 1e-3) / 1e9, 1), "bytes_per_frame": bytes_frame,
            "migration_edge_bins": sc.migration_edge_bins,
            "pslr_range_db_mean": round(float(np.mean([p["pslr_range"] for p in pts])), 3),
            "pslr_azimuth_db_mean": round(float(np.mean([p["pslr_azimuth"] for p in pts])), 3),
            "irw_azimuth_mean": round(float(np.mean([p["irw_azimuth"] for p in pts])), 4)}


def adaptive_shift_quality(rows=256, scales=(0, -12, -16)):
    """Pure FP16 compression of the range scene's echo scaled by 2^s, fixed
    and adaptive block shift, each against the GPU FP32 path on the same
    FP16-rounded echo (SQNR, dB)."""
    from paper_2605_28451_amd import api, scenes
    from paper_2605_28451_amd.metrics import sqnr_db
    sc = scenes.range_scene(seed=2, n_pulses=rows)
    p16 = api.FFTPlan(4096, rows, "fp16")
    p32 = api.FFTPlan(4096, rows, "fp32")
    H16 = api.filter_tensor(sc.replica, 4096, "fp16")
    H32 = api.filter_tensor(sc.replica, 4096, "fp32")
    out = {}
    for ls in scales:
        e16 = scenes.quantize(sc.echo * 2.0 ** ls, "fp16")
        ref = api.to_host(p32.range_compress(api.to_device(e16, "fp32"), H32), "fp32")
        d16 = api.to_device(e16, "fp16")
        fixed = api.to_host(p16.range_compress(d16, H16), "fp16")
        y, ex = p16.range_compress_adaptive(d16, H16)
        ad = api.to_host(y, "fp16") * np.ldexp(1.0, ex.cpu().numpy().astype(np.int64))[:, None]
        out[f"scale_2^{ls}"] = {"fixed_sqnr_db": round(sqnr_db(ref, fixed), 2),
                                "adaptive_sqnr_db": round(sqnr_db(ref, ad), 2)}
    p16.close()
    p32.close()
    return out


def weighted_frame_metrics(mode, taper):
    """Point-target metrics of one 4096x4096 frame whose range and azimuth
    matched filters are weighted (taper: ("taylor", nbar, sll_db) or
    ("hamming",)); the kernels are those of the timed frame, so only the
    image quality is reported."""
    import torch
    from paper_2605_28451_amd import api, scenes, metrics
    sc = _sar_scene()
    n = 4096
    fmt = api.storage_format(mode)
    kind, rest = taper[0], taper[1:]
    wl, wa = api.window(kind, 1024, *rest), api.window(kind, 512, *rest)
    rplan = api.FFTPlan(n, n, mode)
    aplan = api.FFTPlan(n, n, mode)
    Hr = api.filter_tensor(scenes.weighted_range_replica(n, wl), n, mode)
    Ha = api.filter_tensor(scenes.weighted_azimuth_replica(n, wa), n, mode)
    rc = rplan.range_compress(api.to_device(sc.echo, fmt), Hr)
    img = api.to_host(aplan.azimuth_compress(api.corner_turn(rc, fmt), Ha), fmt)
    torch.cuda.synchronize()
    rplan.close()
    aplan.close()
    return [metrics.point_target(img, r0, a0, noise_patch=(r0 + 300, a0 + 300))
            for (r0, a0) in sc.targets]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="headline only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--kernel-only", default=None,
                    help="profiling mode: run only the fused range-compression kernel of the "
                         "given precision (e.g. fp16) for --steps launches, then a plain device "
                         "copy of the same bytes (counter calibration); prints no JSON")
    ap.add_argument("--section", default=None, choices=("sar_frame", "uneven", "autofocus"),
                    help="profiling mode: run only one secondary workload (the 4096x4096 FP16 SAR "
                         "frame graph, the 20,000-transform uneven batch, or the 4096x4096 "
                         "autofocus loop) for --steps steps; prints its figures, no JSON line")
    ap.add_argument("--uneven-size", type=int, default=None, metavar="L",
                    help="profiling mode: 128 MiB of forward transforms of 2^L points (FP16) through "
                         "the uneven kernel (one workgroup per item) and then through the row kernel, "
                         "--steps launches each; prints no JSON")
    ap.add_argument("--tuning", default=None, metavar="E,B,R,P",
                    help="with --quick or --kernel-only: set the compression plan's tuning (engine "
                         "0 = matrix cores / 1 = vector, blocks per CU, rows per thread, radix plan) "
                         "instead of autotuning, so a profiled run holds one kernel configuration")
    ap.add_argument("--traffic-summary", nargs="+", metavar="MODE:FETCH_DIR:WRITE_DIR", default=None,
                    help="write the HBM traffic record from rocprofv3 --pmc runs of --kernel-only "
                         "(no GPU needed) and print its table")
    ap.add_argument("--trace-tail", type=int, default=None, metavar="K",
                    help="with --trace-summary: only the last K dispatches of the library's kernels")
    ap.add_argument("--trace-summary", metavar="DIR", default=None,
                    help="print the kernel table of a rocprofv3 --kernel-trace --stats run (no GPU needed)")
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(args.trace_summary, tail=args.trace_tail)
        return
    if args.traffic_summary:
        traffic_summary([tuple(a.split(":")) for a in args.traffic_summary])
        return
    if args.gpus != 1:
        print(f"bench.py: this path runs on one GPU; --gpus {args.gpus} is not supported "
              "(batches and SAR frames would shard by row or frame, with no exchange between GPUs)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2605_28451_amd import api
    if not torch.cuda.is_available() or api.device_count() < 1:
        print("bench.py: no gfx950 GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    n, rows = 4096, 2048
    fixed = parse_tuning(args.tuning) if args.tuning else None
    if fixed is not None and not (args.quick or args.kernel_only):
        raise SystemExit("--tuning applies to --quick and --kernel-only runs only")
    if args.uneven_size is not None:
        if not 8 <= args.uneven_size <= 14:
            raise SystemExit("--uneven-size takes 8..14")
        e = args.uneven_size
        nn, c = 1 << e, (1 << 25) >> e
        from paper_2605_28451_amd import scenes
        x = api.to_device(scenes.gaussian_rows(1, 64, nn), "fp16").repeat(c // 64, 1, 1).contiguous()
        o = torch.empty_like(x)
        up = api.UnevenPlan(np.full(c, e, np.int32), np.zeros(c, np.uint8), "fp16")
        up.set_tuning(1, 64)
        ms_u, _ = time_launches(lambda i: up.execute(x.view(-1, 2), out=o.view(-1, 2)), 1, args.steps,
                                args.warmup)
        rp = api.FFTPlan(nn, c, "fp16")
        ms_r, _ = time_launches(lambda i: rp.forward(x, out=o), 1, args.steps, args.warmup)
        print(f"[uneven-size] n={nn} transforms={c}: uneven kernel {ms_u * 1e3:.1f} us, "
              f"row kernel {ms_r * 1e3:.1f} us", file=sys.stderr, flush=True)
        return
    if args.kernel_only:
        r = bench_compress(args.kernel_only, rows, n, args.steps, args.warmup, fixed=fixed)
        print(f"[kernel-only] {args.kernel_only} compress: {r['ms_per_launch']:.4f} ms/launch "
              f"{r['hbm_gbs']:.0f} GB/s algorithmic ({r['bytes_per_launch']} B/launch)",
              file=sys.stderr, flush=True)
        buf_in = torch.empty(r["bytes_per_launch"] // 2, dtype=torch.uint8, device="cuda")
        buf_out = torch.empty_like(buf_in)
        ms, _ = time_launches(lambda i: api.device_copy(buf_in, buf_out), 1, args.steps, args.warmup)
        print(f"[kernel-only] device copy of {buf_in.numel()} B: {ms:.4f} ms, "
              f"{2 * buf_in.numel() / (ms * 1e-3) / 1e9:.0f} GB/s (read + write)",
              file=sys.stderr, flush=True)
        return
    if args.section:
        if args.section == "sar_frame":
            r = bench_sar_frame("fp16", args.steps, args.warmup)
        elif args.section == "uneven":
            r = bench_uneven("fp16", args.steps, args.warmup, with_sqnr=False)
        else:
            r = bench_autofocus(args.steps, with_oracle=False)
        print(f"[section] {args.section}: " + json.dumps(
            {k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()
             if not k.startswith("_")}), file=sys.stderr, flush=True)
        return
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)  # noqa: E731

    log("headline: fused FP16-BFP range compression 2048x4096")
    head = bench_compress(HEAD_MODE, rows, n, args.steps, args.warmup, fixed=fixed)
    log(f"  {head['gflops']:.0f} GFLOP/s, {head['hbm_gbs']:.0f} GB/s")
    out = {
        "metric": METRIC,
        "value": round(head["gflops"], 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_total"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16",
        "data": "synthetic",
        "config": {
            "workload": "SAR range compression: 2048 pulses x 4096 range samples, complex FP16, "
                        "LFM chirp 1024 samples b=0.8, 5 point targets + 20 dB AWGN; forward FFT, "
                        "x conj(H), 2^-12 prescale folded into the conjugate, inverse FFT (fused)",
            "precision": MODE_TEXT[HEAD_MODE],
            "buffer_sets": head["buffer_sets"],
            "working_set_mib": head["working_set_mib"],
            "tuning": head["tuning"],
            "flop_convention": "5 N log2 N per transform, 2 transforms per pulse",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(head["hbm_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(head["hbm_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(HEAD_MODE),
            "kernel": head_kernel_text(head["tuning"]),
            "algorithmic_bytes_per_launch": head["bytes_per_launch"],
        },
    }
    if not args.no_cpu:
        log("cpu baseline: FP64 oracle on 64 pulses")
        cb, sq, sq_raw = cpu_baseline(head["_sample_in"], head["_replica"], n, head["_sample_out"])
        out["cpu_baseline"] = cb
        out["sqnr_db_vs_fp64_oracle"] = round(sq, 2)
        out["sqnr_db_vs_fp64_oracle_unaligned"] = round(sq_raw, 2)
        # the paper's convention: the oracle on the unquantised FP64 echo and
        # filter, so the figure also carries the storage rounding of both
        import oracle
        from paper_2605_28451_amd.metrics import sqnr_db
        ref_raw = oracle.compress(head["_sample_in_raw"], oracle.matched_filter(head["_replica"], n))
        out["sqnr_db_vs_fp64_oracle_unquantised_input"] = round(sqnr_db(ref_raw, head["_sample_out"],
                                                                         align=True), 2)
    if not args.quick:
        modes = {}
        for mode in ("fp32", "fp16_fp32", "fp16_mul_fp32_acc", "e4m3", "e5m2"):
            log(f"range compression mode={mode}")
            r = bench_compress(mode, rows, n, args.steps, args.warmup, blocks=3)
            modes[mode] = {"gflops": round(r["gflops"], 1), "hbm_gbs": round(r["hbm_gbs"], 1),
                           "ms_per_launch": round(r["ms_per_launch"], 5), "timed": "median of 3 blocks",
                           "tuning": r["tuning"]}
        out["range_compress_modes"] = modes
        out["fp16_over_fp32"] = round(head["gflops"] / modes["fp32"]["gflops"], 3)
        fft = {}
        for mode, b in (("fp16", 65536), ("fp32", 32768), ("fp16_fp32", 65536),
                        ("fp16_mul_fp32_acc", 65536)):
            log(f"plain forward FFT n=4096 batch={b} mode={mode}")
            r = bench_fft(mode, b, n, args.steps, args.warmup)
            fft[mode] = {k: round(v, 4) if isinstance(v, float) else v for k, v in r.items()}
        for name, inv in (("fp16_rows16384", False), ("fp16_inverse_bfp_rows16384", True)):
            log(f"plain {'BFP inverse' if inv else 'forward'} FFT n=4096 batch=16384 mode=fp16 "
                "(2 rotating sets, 1 GiB working set)")
            r = bench_fft("fp16", 16384, n, args.steps, args.warmup, inverse=inv)
            fft[name] = {k: round(v, 4) if isinstance(v, float) else v for k, v in r.items()}
        by_n = {}
        for e in range(8, 15):
            nn = 1 << e
            log(f"plain forward / BFP inverse FFT n={nn} batch={(1 << 25) // nn} mode=fp16")
            for inv in (False, True):
                r = bench_fft("fp16", (1 << 25) // nn, nn, args.steps, args.warmup, inverse=inv)
                by_n[f"{nn}_{'inverse_bfp' if inv else 'forward'}"] = {
                    "rows": r["rows"], "us_per_launch": round(r["ms_per_launch"] * 1e3, 2),
                    "gflops": round(r["gflops"], 1), "hbm_frac": round(r["hbm_frac"], 4),
                    "tuning": r["tuning"]}
        out["fft_fp16_by_n"] = by_n
        log("plain forward FFT n=4096 batch=64 (latency-bound shape)")
        r = bench_fft("fp16", 64, n, args.steps, args.warmup, min_bytes=0)
        fft["fp16_batch64"] = {k: round(v, 4) if isinstance(v, float) else v for k, v in r.items()}
        fft["fp16_batch64"]["note"] = ("the 64 x 4096 round-trip workload's shape: 1 MiB each way, "
                                       "bound by launch latency, not by HBM")
        out["fft_n4096"] = fft
        # the same ratio on the plain forward FFT (1 GiB each way, both modes)
        out["fp16_over_fp32_plain_fft"] = round(fft["fp16"]["gflops"] / fft["fp32"]["gflops"], 3)
        from paper_2605_28451_amd import metrics as _m  # noqa: F401  (metrics of the GPU image only)
        sar = {}
        imgs = {}
        for mode in ("fp16", "fp32", "fp16_fp32", "fp16_mul_fp32_acc", "e4m3", "e5m2"):
            log(f"SAR frame 4096x4096 mode={mode} (graph)")
            r = bench_sar_frame(mode, args.steps, args.warmup)
            sar[mode] = {k: (round(v, 4) if isinstance(v, float) else v)
                         for k, v in r.items() if not k.startswith("_")}
            imgs[mode] = r["_img"]
            sc = r["_scene"]
            pts = [_m.point_target(r["_img"], r0, a0, noise_patch=(r0 + 300, a0 + 300))
                   for (r0, a0) in sc.targets]
            sar[mode]["image"] = {
                k: _finite_or_none(np.mean([p[key] for p in pts]), nd)
                for k, key, nd in (("pslr_range_db_mean", "pslr_range", 3),
                                   ("pslr_azimuth_db_mean", "pslr_azimuth", 3),
                                   ("snr_db_mean", "snr", 2))}
            if not args.no_cpu:
                sar[mode]["image"]["vs_fp64_oracle"] = frame_vs_oracle(sc, mode, r["_img"], pts)
        sar_fp16_img = imgs["fp16"]
        sar["fp16_metrics"] = sar["fp16"]["image"]
        # image SQNR of every mode against the FP32 path's image (real scale aligned)
        for mode in imgs:
            if mode != "fp32":
                sar[mode]["image"]["sqnr_db_vs_fp32_path"] = _finite_or_none(
                    _m.sqnr_db(imgs["fp32"], imgs[mode], align=True), 2)
        del imgs
        log("SAR frame 4096x4096 mode=fp16, corner turn fused into the range store (graph)")
        r = bench_sar_frame("fp16", args.steps, args.warmup, fused_ct=True)
        sar["fp16_fused_corner_turn"] = {k: (round(v, 4) if isinstance(v, float) else v)
                                         for k, v in r.items() if not k.startswith("_")}
        sar["fp16_fused_corner_turn"]["image_equals_separate_corner_turn"] = bool(
            np.array_equal(r["_img"], sar_fp16_img))
        for nst in (2, 4):
            log(f"SAR frame 4096x4096 mode=fp16, {nst} frames concurrently on {nst} streams (graph)")
            r = bench_sar_frame("fp16", args.steps, args.warmup, streams=nst)
            sar[f"fp16_{nst}_streams"] = {k: (round(v, 4) if isinstance(v, float) else v)
                                          for k, v in r.items() if not k.startswith("_")}
            sar[f"fp16_{nst}_streams"]["image_equals_one_stream"] = bool(np.array_equal(r["_img"], sar_fp16_img))
        out["sar_frame_4096"] = sar
        out["sar_frames_per_s_fp16"] = max(sar[k]["frames_per_s"] for k in
                                           ("fp16", "fp16_fused_corner_turn", "fp16_2_streams", "fp16_4_streams"))
        log("weighted SAR frames (Taylor nbar=5, -40 dB): image quality per mode")
        wq = {"taper": "Taylor, nbar = 5, -40 dB, range (1024) and azimuth (512) filters"}
        wpts = {m: weighted_frame_metrics(m, ("taylor", 5, 40.0))
                for m in ("fp32", "fp16_fp32", "fp16_mul_fp32_acc", "fp16")}
        for m, pts in wpts.items():
            shift = max(max(abs(p[k] - q[k]) for k in ("pslr_range", "pslr_azimuth"))
                        for p, q in zip(pts, wpts["fp32"]))
            wq[m] = {"pslr_range_db_mean": round(float(np.mean([p["pslr_range"] for p in pts])), 3),
                     "pslr_azimuth_db_mean": round(float(np.mean([p["pslr_azimuth"] for p in pts])), 3),
                     "islr_range_db_mean": round(float(np.mean([p["islr_range"] for p in pts])), 3),
                     "max_pslr_shift_vs_fp32_path_db": round(float(shift), 3)}
        out["sar_frame_4096_weighted"] = wq
        log("adaptive block shift: fused compression 2048x4096 fp16, time and quality")
        r = bench_compress("fp16", 2048, 4096, args.steps, args.warmup, adaptive=True)
        out["range_compress_adaptive_shift"] = {
            "ms_per_launch": round(r["ms_per_launch"], 5),
            "ms_per_launch_fixed_shift": round(head["ms_per_launch"], 5),
            "hbm_gbs": round(r["hbm_gbs"], 1),
            "sqnr_vs_fp32_path_by_echo_scale": adaptive_shift_quality()}
        log("RCMC frame 4096x4096 (hyperbolic migration 6.4 bins), fp16 and fp32 (graph)")
        out["sar_frame_4096_rcmc"] = {m: bench_rcmc_frame(m, args.steps, args.warmup)
                                      for m in ("fp16", "fp32")}
        out["sar_frame_4096_rcmc"]["fp16_2_streams"] = bench_rcmc_frame("fp16", args.steps, args.warmup,
                                                                        streams=2)
        log("uneven batch 20000 transforms fp16")
        ub = bench_uneven("fp16", args.steps, args.warmup)
        out["uneven_20000"] = {k: round(v, 4) if isinstance(v, float) else v for k, v in ub.items()}
        log("autofocus 50 Adam steps 4096x4096")
        af = bench_autofocus(50, with_oracle=not args.no_cpu)
        out["autofocus_4096"] = {
            k: (round(v, 4) if isinstance(v, float) else v) for k, v in af.items() if not k.startswith("_")}
        out["autofocus_4096"]["step"] = ("image + entropy, fused phase gradient, Adam (library kernels), "
                                         "several iterations per HIP graph replay (iterations_per_replay)")
        if not args.no_cpu:
            log("cpu oracle on the other workloads (context)")
            out["cpu_baseline"]["other_workloads"] = cpu_oracle_workloads()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
