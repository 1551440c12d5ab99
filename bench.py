#!/usr/bin/env python3
"""Throughput of bulk xorgens generation on one MI355X.

Workload (one step): 1024 independent streams (stream i seeded from 42 + i),
2^20 outputs each as uint32, then 2^20 more each as FP32 uniforms in [0, 1)
by the top-24-bit mapping; each type written contiguously to HBM by one plain
launch in the stream-major layout (xg_generate_*: stream i's outputs at
out[i * 2^20 + t]).  A step produces 2^31 random numbers.  The streams advance
across steps, so every step generates new numbers.  The bulk-fill layout
(xg_fill_*: 64-word chunks of the streams interleaved, so the wavefronts write
one dense region) is timed beside it and reported under "bulk_fill".

Prints one JSON line: RN/s of the whole job, the roofline of the uint32
kernel (HBM write bound, per-launch duration from HIP events on the launch
stream), and the CPU oracle timed on the host's cores on one full step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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

STREAMS = 1024
N = 1 << 20
SEED = 42
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stream_major_u32.json")
DEFAULT_THROUGHPUT_SHAPE = (4, 8, 2, 1)  # waves_per_block, unroll, blocks_per_cu, store_words
VALU_FILE = os.path.join(ROOT, "profiles", "valu_fused_moments.json")
# VALU issue capacity: 256 CUs x 4 SIMDs at 2.4 GHz, each SIMD issuing one
# wave64 instruction per 4 cycles for 32-bit integer and conversion work (16
# lanes per cycle, 39.3e12 lane operations/s), per 2 cycles for FP32 add /
# mul / FMA (the published 157.3 TFLOP/s) and per 8 cycles for transcendentals.
SIMD_CYCLES_PER_S = 256 * 4 * 2.4e9
# The bulk and normal kernels' source: the kernel file and the headers it
# includes.  The committed counter records are used only while it matches.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1108_0486_amd", "csrc", f)
                  for f in ("xg_kernels.hip", "xg_device.h", "xg_normal.h", "xg_internal.h", "xg_host.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per uint32 launch from the committed rocprofv3 counter runs,
    or None when they are absent or were taken on another kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def measured_valu():
    """VALU wave instructions per fused-moments launch (SQ_INSTS_VALU, from
    the committed rocprofv3 counter run) and the minimum issue time of that
    instruction mix, or None when absent or taken on another kernel source."""
    try:
        with open(VALU_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    insts = rec["valu_wave_insts_per_launch"]
    mix, cyc = rec["main_loop_valu_mix"], rec["issue_cycles_per_wave_instruction"]
    return insts, insts * sum(f * cyc[k] for k, f in mix.items()) / SIMD_CYCLES_PER_S


def host_threads() -> int:
    """Host cores this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


# The method's own work per normal pair (independent of the kernel's
# instruction mix): two generator words at 13 integer operations each
# (recurrence 9, Weyl 1, tempering 2, combine 1); two uniform maps (a shift and
# an integer-to-float conversion at the 32-bit rate, an FP32 scale); one FP32
# multiply for -2 ln u; two FP32 multiplies (rho cos, rho sin); four FP32
# moment updates (fused kernel only); and four transcendentals (log, sqrt,
# sin, cos).  Issue cycles per wave64 instruction on one SIMD: 4 for 32-bit
# integer and conversion, 2 for FP32 add / mul / FMA, 8 for transcendentals.
FUSED_PAIR_OPS = {"int32": 2 * 13 + 2 + 2, "fp32": 2 + 1 + 2 + 4, "transcendental": 4}
FUSED_OPS_PER_PAIR = sum(FUSED_PAIR_OPS.values())
FUSED_CYCLES_PER_64_PAIRS = 4 * FUSED_PAIR_OPS["int32"] + 2 * FUSED_PAIR_OPS["fp32"] + 8 * FUSED_PAIR_OPS["transcendental"]


def fused_algorithmic_floor(pairs: int):
    """(operations, minimum seconds) of the fused normal moments over `pairs`
    pairs at full VALU issue on every SIMD."""
    return FUSED_OPS_PER_PAIR * pairs, pairs / 64 * FUSED_CYCLES_PER_64_PAIRS / SIMD_CYCLES_PER_S


def normals_floor(pairs: int):
    """The same without the four moment updates (the unfused normals)."""
    cycles = FUSED_CYCLES_PER_64_PAIRS - 2 * 4
    return (FUSED_OPS_PER_PAIR - 4) * pairs, pairs / 64 * cycles / SIMD_CYCLES_PER_S


def cpu_baseline(threads: int):
    """The oracle on one full step of the workload (u32 and f32 of all 1024
    streams), in slices of at least 64 streams (and at least one per thread)
    to bound host memory."""
    import numpy as np
    from oracle import oracle as O

    slice_ = max(64, threads)
    while STREAMS % slice_:
        slice_ += 1
    t0 = time.perf_counter()
    total = 0
    for first in range(0, STREAMS, slice_):
        st = O.OracleStreams(SEED, slice_, first=first)
        st.u32(N, threads=threads)
        st.f32(N, threads=threads)
        total += 2 * slice_ * N
    dt = time.perf_counter() - t0
    del np
    return {"value": total / dt, "unit": "RN/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "one full step: 1024 streams x (2^20 uint32 + 2^20 FP32), plain sequential C oracle, "
                      "one POSIX thread per share of streams (includes per-slice seeding, %.1f s)" % dt}


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it: model name, vendor, family /
    model / stepping, and the logical CPUs it lists."""
    fields, cpus = {}, 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    continue
                k, v = (x.strip() for x in line.split(":", 1))
                if k == "processor":
                    cpus += 1
                fields.setdefault(k, v)
    except OSError:
        return "unknown"
    return "%s (%s, family %s model %s stepping %s; %d logical CPUs listed, %d usable here)" % (
        fields.get("model name", "unknown"), fields.get("vendor_id", "?"), fields.get("cpu family", "?"),
        fields.get("model", "?"), fields.get("stepping", "?"), cpus, host_threads())


# The paper's own throughput (Section 3, Table 1), for context only: other
# hardware (NVIDIA GTX 480 and one GPU of a GTX 295, CUDA 3.2), repeated
# generation of 10^8 numbers; the paper does not say what was stored.
PAPER_TABLE1 = {"source": "Section 3, Table 1 (context, not a target)",
                "xorgensGP_GTX480_rn_per_s": 17.7e9, "xorgensGP_GTX295_rn_per_s": 9.1e9,
                "hardware": "NVIDIA GeForce GTX 480; one GPU of a GeForce GTX 295; CUDA 3.2"}


RAGGED_KEY = "ragged65536/u32"


def _graph_ms(torch, g, reps=5):
    g.replay()
    torch.cuda.synchronize()
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.replay()
    e.record()
    torch.cuda.synchronize()
    return a.elapsed_time(e) / reps


def extra_ragged_batch(torch, dev, shape=None, per_stream=True):
    """65536 streams, lengths log-uniform in [2^10, 2^20] (seed 7), uint32:
    the one-call batch (xg_generate_batch: the table in stream order, grouped
    and ordered on the device, served by one persistent launch) captured in a
    HIP graph, with the shape the autotuner stored in the tuning cache under
    RAGGED_KEY; the host-planned batch kernel alone in the same shape; and one
    plain launch per stream on the same GPU."""
    from paper_1108_0486_amd import workloads as W
    from paper_1108_0486_amd import xg
    from paper_1108_0486_amd.batch import Batch, PlannedBatch
    from paper_1108_0486_amd.streams import XorgensStreams

    lengths = W.ragged_lengths()
    off = W.csr_offsets(lengths)
    total = int(off[-1])
    S = len(lengths)
    reqs = [(i, int(lengths[i]), int(off[i]), 0) for i in range(S)]
    gs = XorgensStreams(S, seed=SEED, device=dev)
    b = Batch(gs, reqs, total)
    t0 = time.perf_counter()
    recs = []
    if shape is None:
        best, recs = b.autotune(reps=1, tune_key=RAGGED_KEY)
    else:
        best = tuple(shape)
        arch, cus = xg.xg_tune_identity(gs.ctx)
        xg.xg_tune_cache_put(arch, cus, xg.XG_FAMILY_R128_W32, RAGGED_KEY, best)
    tune_s = time.perf_counter() - t0
    # the library's default for this many queue items (8 or more per compute unit)
    default_ms = [r[4] for r in recs if r[:4] == DEFAULT_THROUGHPUT_SHAPE]
    batch_ms = _graph_ms(torch, b.capture_graph(tune_key=RAGGED_KEY))
    err = b.error_flag()
    out = b.out
    del b
    pb = PlannedBatch(gs, reqs, total, out=out)
    kernel_ms = _graph_ms(torch, pb.capture_graph(tune=best))
    err |= pb.error_flag()
    del pb
    res = {
        "workload": "65536 streams, n_i = floor(2^(10 + 10 U_i)) (U from seed 7), uint32, CSR offsets",
        "total_rn": total,
        "path": "xg_generate_batch (one call: device grouping and ordering, then the persistent launch), "
                "captured in a HIP graph, shape from the tuning cache key %r" % RAGGED_KEY,
        "batched_graph_ms": batch_ms,
        "batched_rn_per_s": total / (batch_ms * 1e-3),
        "batched_frac_of_hbm_peak": 4 * total / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "batch_kernel_graph_ms": kernel_ms,
        "batch_kernel_frac_of_hbm_peak": 4 * total / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "device_planning_ms": batch_ms - kernel_ms,
        "autotuned_shape": {"waves_per_block": best[0], "unroll": best[1], "blocks_per_cu": best[2],
                            "store_words": best[3]},
        "default_shape": list(DEFAULT_THROUGHPUT_SHAPE),
        "default_shape_ms": default_ms[0] if default_ms else None,
        "autotune_s": tune_s,
        "autotune_candidates": len(recs),
        "error_flag": err,
    }
    if per_stream:
        # baseline: one plain launch per stream (one wavefront each), in order on one stream
        stream = torch.cuda.current_stream()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        t0 = time.perf_counter()
        for i in range(S):
            gs.u32(int(lengths[i]), first=i, count=1, out=out[int(off[i]):int(off[i + 1])], stream=stream)
        e.record()
        torch.cuda.synchronize()
        res["per_stream_plain_wall_s"] = time.perf_counter() - t0
        res["per_stream_plain_launches_ms"] = a.elapsed_time(e)
        res["speedup_batched_vs_per_stream"] = res["per_stream_plain_launches_ms"] / batch_ms
    del gs, out
    torch.cuda.empty_cache()
    return res


def extra_fused_moments(torch, dev):
    """4096 streams x 2^18 normals reduced in-kernel to sums of z and z^2."""
    from paper_1108_0486_amd import workloads as W
    from paper_1108_0486_amd.streams import XorgensStreams

    S, N = W.FUSED_STREAMS, W.FUSED_N
    gs = XorgensStreams(S, seed=SEED, device=dev)
    sums = torch.empty((S, 2), dtype=torch.float32, device=dev)
    # 40 warm-up launches: from idle, ALU-heavy launches first run fast, then
    # dip for a few dozen launches while the power management settles.
    for _ in range(40):
        gs.moments(N, out=sums)
    reps = 20
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        gs.moments(N, out=sums)
    e.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(e) / reps
    zs = torch.empty((S, N), dtype=torch.float32, device=dev)
    for _ in range(20):
        gs.normal(N, out=zs)
    a.record()
    for _ in range(10):
        gs.normal(N, out=zs)
    e.record()
    torch.cuda.synchronize()
    unfused_ms = a.elapsed_time(e) / 10
    del zs, gs
    torch.cuda.empty_cache()
    # the FP64 oracle on a sample of the same workload (host cores)
    from oracle import oracle as O
    threads = host_threads()
    sample = 64
    st = O.OracleStreams(SEED, sample)
    t0 = time.perf_counter()
    st.moments(N, threads=threads)
    dt = time.perf_counter() - t0
    cpu = {"value": sample * N / dt, "unit": "normals/s", "cores": threads, "kind": "oracle",
           "sample": "64 of the 4096 streams x 2^18 FP64 Box-Muller normals and their sums (%.2f s)" % dt}
    pairs = S * N // 2
    ops, t_min = fused_algorithmic_floor(pairs)
    roof = {"bound": "alu", "achieved": ops / (ms * 1e-3) / 1e9, "peak": ops / t_min / 1e9,
            "unit": "Gop/s (the method's operations: %d per normal pair, weighted by their VALU issue "
                    "rates)" % FUSED_OPS_PER_PAIR,
            "frac": t_min / (ms * 1e-3), "ops_per_pair": dict(FUSED_PAIR_OPS),
            "issue_cycles_per_64_pairs": FUSED_CYCLES_PER_64_PAIRS, "min_ms": t_min * 1e3}
    valu = measured_valu()
    issue = None
    if valu is not None:
        insts, t_issue = valu
        issue = {"valu_wave_insts_per_launch": insts, "min_issue_ms_of_this_mix": t_issue * 1e3,
                 "frac": t_issue / (ms * 1e-3),
                 "note": "how busy the VALU is with the kernel's own instructions (not the method's work)"}
    unfused_ops, unfused_t = normals_floor(pairs)
    return {"workload": "4096 streams x 2^18 FP32 normals (Box-Muller), sums of z and z^2 in-kernel",
            "kernel_ms": ms, "rn_per_s": S * N / (ms * 1e-3), "roofline": roof, "issue_efficiency": issue,
            "cpu_oracle": cpu,
            "unfused_normals_ms": unfused_ms, "unfused_rn_per_s": S * N / (unfused_ms * 1e-3),
            "unfused_roofline": {"hbm_floor_ms": 4 * S * N / (HBM_PEAK_GBS * 1e9) * 1e3,
                                 "alu_floor_ms": unfused_t * 1e3,
                                 "frac_of_hbm_peak": 4 * S * N / (unfused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "frac_of_larger_floor": max(4 * S * N / (HBM_PEAK_GBS * 1e9), unfused_t)
                                 / (unfused_ms * 1e-3)}}


def _member_ragged_batch(torch, dev, fam):
    """The ragged workload (65536 streams, uint32, CSR offsets) served by one
    persistent launch of a further member's batch kernel, autotuned, replayed
    in a HIP graph."""
    from paper_1108_0486_amd import workloads as W
    from paper_1108_0486_amd.batch import Batch
    from paper_1108_0486_amd.streams import XorgensStreams

    lengths = W.ragged_lengths()
    off = W.csr_offsets(lengths)
    total = int(off[-1])
    S = len(lengths)
    gs = XorgensStreams(S, seed=SEED, device=dev, family=fam)
    b = Batch(gs, [(i, int(lengths[i]), int(off[i]), 0) for i in range(S)], total)
    best, recs = b.autotune(reps=1)
    g = b.capture_graph(tune=best)
    g.replay()
    torch.cuda.synchronize()
    reps = 5
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.replay()
    e.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(e) / reps
    res = {"total_rn": total, "batched_graph_ms": ms, "batched_rn_per_s": total / (ms * 1e-3),
           "batched_frac_of_hbm_peak": 4 * total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "autotuned_shape": {"waves_per_block": best[0], "unroll": best[1], "blocks_per_cu": best[2]},
           "error_flag": b.error_flag()}
    del b, g, gs
    torch.cuda.empty_cache()
    return res


def extra_family_members(torch, dev):
    """The two further members (r = 64, s = 33; two streams per wavefront):
    4 GiB per launch in the bulk-fill layout and stream-major, per output
    type, at 2048 streams (1024 wavefronts, one per SIMD) and 1024 streams."""
    from paper_1108_0486_amd import xg
    from paper_1108_0486_amd.streams import XorgensStreams

    res = {}
    for fam, name, wbytes, kinds in [
            (xg.XG_FAMILY_R64_W32, "r64_w32 (n=2048)", 4, ("u32", "f32")),
            (xg.XG_FAMILY_R64_W64, "r64_w64 (n=4096)", 8, ("u64", "f64"))]:
        rec = {}
        for S in (2048, 1024):
            n = (4 << 30) // (wbytes * S)
            gs = XorgensStreams(S, seed=SEED, device=dev, family=fam)
            dt = torch.int32 if wbytes == 4 else torch.int64
            out = torch.empty(S * n, dtype=dt, device=dev)
            row = {}
            for kind in kinds:
                for layout in ("fill", "stream_major"):
                    f = getattr(gs, ("fill_" if layout == "fill" else "") + kind)
                    o = out if layout == "fill" else out.view(S, n)
                    if kind in ("f32", "f64"):
                        o = o.view(torch.float32 if wbytes == 4 else torch.float64)
                    for _ in range(30):        # past the clock transient of a fresh launch series
                        f(n, out=o)
                    reps = 20
                    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    torch.cuda.synchronize()
                    a.record()
                    for _ in range(reps):
                        f(n, out=o)
                    e.record()
                    torch.cuda.synchronize()
                    ms = a.elapsed_time(e) / reps
                    gbs = wbytes * S * n / (ms * 1e-3) / 1e9
                    row["%s_%s" % (layout, kind)] = {"ms": ms, "GBs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
                                                     "values_per_s": S * n / (ms * 1e-3)}
            rec["%d streams x %d" % (S, n)] = row
            del out, gs
            torch.cuda.empty_cache()
        res[name] = rec
    res["r64_w32 (n=2048) ragged batch"] = _member_ragged_batch(torch, dev, xg.XG_FAMILY_R64_W32)
    # the 32-bit member's fused normal moments on the fused workload's shape
    S, n = 4096, 1 << 18
    gs = XorgensStreams(S, seed=SEED, device=dev, family=xg.XG_FAMILY_R64_W32)
    sums = torch.empty((S, 2), dtype=torch.float32, device=dev)
    for _ in range(10):
        gs.moments(n, out=sums)
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(20):
        gs.moments(n, out=sums)
    e.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(e) / 20
    res["r64_w32 (n=2048) fused moments 4096 x 2^18"] = {"kernel_ms": ms, "rn_per_s": S * n / (ms * 1e-3)}
    del gs, sums
    # the 64-bit member's FP64 normals: 2048 streams x 2^18 doubles (4 GiB)
    S, n = 2048, 1 << 18
    gs = XorgensStreams(S, seed=SEED, device=dev, family=xg.XG_FAMILY_R64_W64)
    z = torch.empty((S, n), dtype=torch.float64, device=dev)
    for _ in range(10):
        gs.normal_f64(n, out=z)
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(20):
        gs.normal_f64(n, out=z)
    e.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(e) / 20
    res["r64_w64 (n=4096) FP64 normals 2048 x 2^18"] = {"kernel_ms": ms, "rn_per_s": S * n / (ms * 1e-3),
                                                        "GBs": 8 * S * n / (ms * 1e-3) / 1e9}
    del gs, z
    return res


def extra_serving(torch, dev, num_requests: int):
    """10^5 device-resident streams; Poisson arrivals at 20k req/s (seed 11);
    N log-uniform in [2^8, 2^24]; dtype uniform over {u32, f32, normal};
    8 GiB output pool, 4 lanes, requests longer than 2^16 words served as
    jumped segments; against one plain launch per request (FIFO) on a prefix
    of the same trace."""
    from paper_1108_0486_amd import workloads as W
    from paper_1108_0486_amd.serve import Server, run_trace, run_trace_plain_fifo
    from paper_1108_0486_amd.streams import XorgensStreams

    trace = W.serving_trace(num_requests)
    seg = 1 << 16
    # Warm the process (code objects, pinned staging, allocator) with a
    # throwaway server on a short prefix, so the timed replay is steady state.
    gw = XorgensStreams(W.SERVE_STREAMS, seed=SEED + 7, device=dev)
    warm = Server(gw, pool_elems=1 << 28, num_lanes=4, max_batch=8192, segment_words=seg)
    run_trace(warm, trace[:300], timeout_s=120)
    warm.close()
    del warm, gw
    gs = XorgensStreams(W.SERVE_STREAMS, seed=SEED, device=dev)
    srv = Server(gs, pool_elems=1 << 31, num_lanes=4, max_batch=8192, segment_words=seg)
    full, _, _ = run_trace(srv, trace, timeout_s=600)
    srv.close()
    prefix = trace[:2000]
    gs2 = XorgensStreams(W.SERVE_STREAMS, seed=SEED, device=dev)
    srv2 = Server(gs2, pool_elems=1 << 31, num_lanes=4, max_batch=8192, segment_words=seg)
    served_prefix, _, _ = run_trace(srv2, prefix, timeout_s=300)
    srv2.close()
    gs3 = XorgensStreams(W.SERVE_STREAMS, seed=SEED, device=dev)
    plain_prefix = run_trace_plain_fifo(gs3, prefix, max_n=1 << 24, timeout_s=300)
    del srv, srv2, gs, gs2, gs3
    torch.cuda.empty_cache()
    return {"workload": "10^5 streams, %d requests, Poisson 20k req/s (seed 11), N = floor(2^(8 + 16 U)), "
                        "dtype in {u32, f32, normal}, 8 GiB pool, 4 lanes, 2^16-word segments; the process is "
                        "warmed on a 300-request prefix with a throwaway server first" % num_requests,
            "served": full,
            "prefix_2000": {"served": served_prefix, "plain_fifo": plain_prefix}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # Untimed warm-up: from an idle GPU the first few dozen bulk launches run
    # through a power-management transient (measured: a dip from ~600 to
    # ~900 us per launch that settles back over ~40 launches), so the default
    # warm-up (4 launches per step) is long enough for the timed region to see
    # the settled state.
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--waves-per-block", type=int, default=None)
    ap.add_argument("--unroll", type=int, default=None)
    ap.add_argument("--store-words", type=int, default=None)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the ragged-batch, fused-moments, family and serving measurements")
    ap.add_argument("--extras", default="ragged,fused,family,serving",
                    help="comma-separated subset of the extra measurements to run")
    ap.add_argument("--serve-requests", type=int, default=200_000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference for HBM byte counters)")
    ap.add_argument("--only-extras", action="store_true",
                    help="run only the chosen extras and print their JSON (for profiling one workload)")
    ap.add_argument("--ragged-shape", default=None,
                    help="waves_per_block,unroll,blocks_per_cu,store_words for the ragged batch (no autotune)")
    ap.add_argument("--no-per-stream", action="store_true",
                    help="skip the ragged batch's one-launch-per-stream baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(streams are independent and would shard by stream id with no exchange)", file=sys.stderr)
        return 2

    import torch
    from paper_1108_0486_amd.streams import XorgensStreams

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ragged_shape = tuple(int(v) for v in args.ragged_shape.split(",")) if args.ragged_shape else None
    extra_runs = [("ragged_batch", "ragged",
                   lambda: extra_ragged_batch(torch, dev, ragged_shape, not args.no_per_stream)),
                  ("fused_moments", "fused", lambda: extra_fused_moments(torch, dev)),
                  ("family_members", "family", lambda: extra_family_members(torch, dev)),
                  ("serving", "serving", lambda: extra_serving(torch, dev, args.serve_requests))]
    if args.only_extras:
        chosen = set(args.extras.split(","))
        res = {}
        for key, name, f in extra_runs:
            if name in chosen:
                print("extra: %s" % key, file=sys.stderr, flush=True)
                res[key] = f()
        print(json.dumps({"extras": res}), flush=True)
        return 0
    gs = XorgensStreams(STREAMS, seed=SEED, device=dev)
    if args.waves_per_block or args.unroll or args.store_words:
        wpb, un, sw = gs.plain_tune()
        gs.set_plain_tune(args.waves_per_block or wpb, args.unroll or un, args.store_words or sw)
    out_u = torch.empty((STREAMS, N), dtype=torch.int32, device=dev)
    out_f = torch.empty((STREAMS, N), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def timed(launch_u, launch_f, steps):
        """Per-launch event times (ms) of `steps` steps, and the wall time
        between synchronisations."""
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            launch_u()
            ev[k][1].record(stream)
            ev[k][2].record(stream)
            launch_f()
            ev[k][3].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return (sum(e[0].elapsed_time(e[1]) for e in ev) / steps,
                sum(e[2].elapsed_time(e[3]) for e in ev) / steps, wall)

    fill_u = lambda: gs.fill_u32(N, out=out_u.view(-1), stream=stream)       # noqa: E731
    fill_f = lambda: gs.fill_f32(N, out=out_f.view(-1), stream=stream)       # noqa: E731
    gen_u = lambda: gs.u32(N, out=out_u, stream=stream)                      # noqa: E731
    gen_f = lambda: gs.f32(N, out=out_f, stream=stream)                      # noqa: E731

    for _ in range(args.warmup):
        fill_u()
        fill_f()
        gen_u()
        gen_f()
    torch.cuda.synchronize()

    K = args.steps
    u32_ms, f32_ms, wall = timed(gen_u, gen_f, K)
    fill_u32_ms, fill_f32_ms, _ = timed(fill_u, fill_f, max(5, K // 2))
    rn_per_step = 2 * STREAMS * N
    ms_per_step = wall * 1e3 / K
    bytes_per_launch = 4 * STREAMS * N
    achieved = bytes_per_launch / (u32_ms * 1e-3) / 1e9

    # Practical write ceiling on the same buffer: torch's own fill kernel.
    fill_ms = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        out_u.fill_(7)
        b.record(stream)
        torch.cuda.synchronize()
        fill_ms.append(a.elapsed_time(b))
    fill_gbs = bytes_per_launch / (sorted(fill_ms)[2] * 1e-3) / 1e9
    # ... and the library's hand-written write-only kernel (16-byte nt stores).
    from paper_1108_0486_amd import xg as _xg
    h = stream.cuda_stream
    for _ in range(10):
        _xg.xg_fill_value(out_u.data_ptr(), STREAMS * N, 7, h)
    wv = []
    for _ in range(10):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        _xg.xg_fill_value(out_u.data_ptr(), STREAMS * N, 7, h)
        b.record(stream)
        torch.cuda.synchronize()
        wv.append(a.elapsed_time(b))
    write_only_gbs = bytes_per_launch / (sorted(wv)[5] * 1e-3) / 1e9

    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    traffic = measured_traffic()
    threads = host_threads()
    cpu = None if args.no_cpu_baseline else cpu_baseline(threads)
    del out_u, out_f
    torch.cuda.empty_cache()
    extras = None
    if not args.no_extras:
        chosen = set(args.extras.split(","))
        extras = {key: f() for key, name, f in extra_runs if name in chosen}

    wpb, un, sw = gs.plain_tune()
    line = {
        "metric": "RN/s (32-bit) and % of HBM write BW",
        "value": rn_per_step / (ms_per_step * 1e-3),
        "unit": "RN/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "bulk uniform generation: 1024 xorgens streams (seed 42 + i) x 2^20 outputs, "
                        "uint32 then FP32 [0,1) (top-24-bit), one plain launch per type, written contiguously "
                        "to HBM stream-major (stream i at out[i * 2^20 + t])",
            "layout": "stream-major (xg_generate_u32 / xg_generate_f32)",
            "streams": STREAMS,
            "outputs_per_stream_per_type": N,
            "rn_per_step": rn_per_step,
            "params": "(r,s,a,b,c,d)=(128,65,15,14,12,17), w=32, omega=0x9E3779B9, gamma=16",
            "launch": {"waves_per_block": wpb or "auto: 4 (one stream per SIMD)",
                       "unroll": un or "auto: 2 for the stream-major launches", "store_words": sw},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_generate<u32> (xg_generate_u32, stream-major)",
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": u32_ms,
        },
        "kernels_ms": {"stream_major_u32": u32_ms, "stream_major_f32": f32_ms,
                       "fill_u32": fill_u32_ms, "fill_f32": fill_f32_ms},
        "f32_GBs": bytes_per_launch / (f32_ms * 1e-3) / 1e9,
        "bulk_fill": {
            "layout": "bulk-fill (xg_fill_u32 / xg_fill_f32): 64-word chunks of the streams interleaved",
            "rn_per_s_kernels": rn_per_step / ((fill_u32_ms + fill_f32_ms) * 1e-3),
            "u32_GBs": bytes_per_launch / (fill_u32_ms * 1e-3) / 1e9,
            "u32_frac_of_peak": bytes_per_launch / (fill_u32_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "f32_GBs": bytes_per_launch / (fill_f32_ms * 1e-3) / 1e9,
        },
        "fill_ceiling_GBs": fill_gbs,
        "frac_of_fill_ceiling": achieved / fill_gbs,
        "write_only_kernel_GBs": write_only_gbs,
        "frac_of_write_only_kernel": achieved / write_only_gbs,
        "cpu_baseline": cpu,
        "paper_context": dict(PAPER_TABLE1, value_over_gtx480=rn_per_step / (ms_per_step * 1e-3) / 17.7e9),
        "extras": extras,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
