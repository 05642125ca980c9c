"""Benchmark: batched V-MT19937-32 generation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (one step): 65,536 independent V-MT19937-32 generators (M = 16
lanes), seeded by init_by_array with 4-word keys from splitmix64(42), each
asked for a log-uniform number of uint32 in [1e3, 1e7) (splitmix64(43)):
about 287 GB of output per step. States stay resident in HBM; each step
continues every stream. The output of a step is larger than HBM, so it is
written in rounds into an output arena (every round's tasks get disjoint
slices; the next round overwrites the arena, as a consumer that drains each
round would). One round = one persistent-kernel launch over its tasks,
longest first.

The persistent kernel's launch shape is autotuned first on a sample of the
task lengths; each step is one replay of a HIP graph holding every round's
launch.

Printed: ONE JSON line with the output GB/s of the step (value), the
roofline of the persistent kernel (HIP events on its stream), the plain form
(one launch per generator, same kernel), single-stream rates of the other
configurations, lane de-phasing (init) cost, and the oracle's rate on the
host as cpu_baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "output GB/s vs HBM-write roofline, batched vs plain; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0
N_GEN = 65536
M_LANES = 16
STATE_WIN_BYTES = 624 * 16 * 4  # window of one V-MT19937-32 (M = 16) state

# HBM bytes per launch of the batch kernel from rocprofv3 FETCH_SIZE (x2.0) and
# WRITE_SIZE (x1.0), scaled by a 4 GiB device copy; valid only for the kernel
# code (kernel_fingerprint) and the launch shapes they were taken with
# (profiles/batch_mt32_m16_counters.md): threads per workgroup, store bytes,
# workgroups per CU -> (bytes read, bytes written).
COUNTERS = {
    "kernel_fingerprint": "2fbb6e123c2646db2298973bca40abb13454322095e63202f3ff065d64f6ccd5",
    "shapes": {
        (512, 16, 2): (877944533, 96283548128),
        (512, 8, 2): (878033707, 96283547808),
        (256, 16, 2): (878094549, 96283547797),
        (256, 8, 3): (878342400, 96283564277),
        (960, 16, 2): (878137984, 96283549333),
    },
}


def kernel_fingerprint() -> str:
    """sha256 of the kernel source without comments and whitespace (comment
    edits do not invalidate counters taken on the same code)."""
    import hashlib
    import re

    with open(os.path.join(ROOT, "paper_2309_16682_amd", "csrc", "vmt_kernels.hip")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return hashlib.sha256(re.sub(r"\s+", "", src).encode()).hexdigest()


def counter_traffic(shape) -> int | None:
    key = (shape.threads, shape.store_bytes, shape.wg_per_cu)
    if kernel_fingerprint() != COUNTERS["kernel_fingerprint"] or key not in COUNTERS["shapes"]:
        return None
    return sum(COUNTERS["shapes"][key])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--generators", type=int, default=N_GEN)
    ap.add_argument("--arena-gib", type=float, default=96.0)
    ap.add_argument("--plain-sample", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-threads", type=int, default=16, help="host threads for the oracle baseline (capped by the CPUs)")
    ap.add_argument("--skip-secondary", action="store_true")
    ap.add_argument("--skip-serving", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--only-batch", action="store_true", help="time the batched step only (for profiling)")
    ap.add_argument("--only-serving", action="store_true", help="run the serving section only")
    ap.add_argument("--only-check", action="store_true", help="run the linear-complexity self-check section only")
    ap.add_argument("--only-jumps", action="store_true", help="run the jump section only")
    ap.add_argument("--only-variants", type=str, default=None,
                    help="run these batched family lines only (comma-separated names, e.g. mt64_M8_u64, or 'all')")
    ap.add_argument("--only-single", type=str, default=None,
                    help="run these single-stream configurations only (comma-separated names, e.g. sfmt_M4_2^28_u32)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--single-shape", type=str, default=None,
                    help="with --only-single: LANES_PER_WG,SPLIT_LOG2 instead of autotuning the generate family")
    ap.add_argument("--no-graph", action="store_true", help="launch the rounds eagerly instead of replaying a graph")
    ap.add_argument("--no-pattern", action="store_true", help="skip timing the output pattern without the twist")
    ap.add_argument("--tune-sample", type=int, default=8192)
    ap.add_argument("--shape", type=str, default=None,
                    help="fix the batch shape as threads_variant,store_bytes,wg_per_cu (no autotuning)")
    ap.add_argument("--calibrate", action="store_true",
                    help="only a 4 GiB device copy and fill: the counter scale and the measured write ceiling")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds: float, threads: int) -> dict:
    """The oracle, as it is, on the host's cores: V-MT19937-32 (M = 16) streams
    keyed like the batch serve the batch's request lengths, request i on
    thread i mod T (each thread its own streams; the oracle's C calls run
    without the interpreter lock). Also the oracle's single-thread rate on the
    batch sample and on the single-stream configurations."""
    import threading

    from oracle import pyoracle as O
    from paper_2309_16682_amd.workload import batch_keys, batch_lengths
    from tests import golden_io

    keys = batch_keys(4 * threads, seed=42)
    lens = batch_lengths(N_GEN, seed=43)
    gJ = golden_io.lane_poly(0, M_LANES)

    def serve(t, T, budget, out, start=None):
        streams = [O.VStream(0, M_LANES, O.seed_state(0, key=k), gJ) for k in keys[4 * t : 4 * t + 4]]
        if start is not None:
            start.wait()  # every thread's streams are seeded: the timed parts run side by side
        done = reqs = 0
        i = t
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget:
            streams[reqs % 4].generate(int(lens[i % N_GEN]))
            done += int(lens[i % N_GEN])
            reqs += 1
            i += T
        out[t] = (done, reqs, time.perf_counter() - t0)

    res = [None] * threads
    start = threading.Barrier(threads)
    workers = [threading.Thread(target=serve, args=(t, threads, seconds, res, start)) for t in range(threads)]
    for w in workers:
        w.start()
    for w in workers:
        w.join()
    wall = max(r[2] for r in res)  # the timed part (streams are seeded before the barrier)
    done = sum(r[0] for r in res)
    reqs = sum(r[1] for r in res)
    one = [None]
    serve(0, 1, min(3.0, seconds), one)
    single = {}
    for name, variant, M, seed, n, eb in (("mt32_M16_u32", 0, 16, 5489, 1 << 22, 4), ("mt64_M8_u64", 1, 8, 5489, 1 << 21, 8),
                                          ("sfmt_M4_u32", 2, 4, 1234, 1 << 22, 4), ("sfmt_M64_u32", 2, 64, 1234, 1 << 22, 4)):
        st = O.VStream(variant, M, O.seed_state(variant, seed=seed), golden_io.lane_poly(variant, M))
        t1 = time.perf_counter()
        st.generate(n)
        single[name] = round(n * eb / (time.perf_counter() - t1) / 1e9, 4)
    return {
        "value": round(done * 4 / wall / 1e9, 4),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"oracle V-MT19937-32 (M=16) serving the batch workload's request lengths from 4 init_by_array "
        f"generators per thread on {threads} threads: {reqs} requests, {done} uint32 in {wall:.1f} s",
        "host": f"{cpu_model()}, {os.cpu_count()} CPUs visible",
        "single_thread_GBps": round(one[0][0] * 4 / one[0][2] / 1e9, 4),
        "single_thread_single_stream_GBps": single,
    }


def calibrate(torch, ctx=None, gib: int = 4, reps: int = 3) -> dict:
    """A plain device copy (read n + write n bytes), fill (torch's 16-byte
    vector stores), hipMemsetAsync and the library's own 16-byte fills
    (4 KiB pieces in address order; two contiguous regions per CU, plain and
    nontemporal) of `gib` GiB: the copy's FETCH_SIZE / WRITE_SIZE readings
    give the counters' scale, the fill and memset rates the write ceilings
    measured on this device."""
    n = gib << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty(n, dtype=torch.uint8, device="cuda")
    out = {"bytes": n}
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so")  # the HIP runtime torch has loaded
    hip.hipMemsetAsync.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p]
    hip.hipMemsetAsync.restype = ctypes.c_int
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def memset():
        assert hip.hipMemsetAsync(ctypes.c_void_p(dst.data_ptr()), 7, n, stream) == 0

    legs = [("copy", lambda: dst.copy_(src), 2 * n), ("fill", lambda: dst.fill_(7), n), ("memset", memset, n)]
    if ctx is not None:
        from paper_2309_16682_amd import vmt

        legs += [("fill_pieces", lambda: vmt.vmt_calib_fill(ctx, dst), n),
                 ("fill_regions", lambda: vmt.vmt_calib_fill(ctx, dst, regions=True), n),
                 ("fill_regions_nt", lambda: vmt.vmt_calib_fill(ctx, dst, regions=True, nontemporal=True), n)]
    for name, fn, moved in legs:
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name + "_GBps"] = round(moved * reps / (a.elapsed_time(b) * 1e-3) / 1e9, 1)
    return out


# Ceilings of the self-check kernel. Dense form: VALU issue, 256 CUs x 4 SIMDs x 16 lanes per clock x
# 2.4 GHz = 39.3 T lane-ops/s, and one three-input XOR (v_bitop3_b32) folds two terms of the
# recurrence: at most 78.6 T term-XORs/s. Sparse form: every term of every offset reads one 4-byte
# word from LDS, 256 CUs x 128 B/clock x 2.4 GHz = 78.6 TB/s.
CHECK_PEAK_TERMS = 2 * 256 * 4 * 16 * 2.4e9
LDS_PEAK_BYTES = 256 * 128 * 2.4e9


SINGLE_STREAMS = (
    ("mt32_M16_2^24_u32", 0, 16, 5489, 1 << 24, "u32"),
    ("mt32_M1_2^24_u32 (the std::mt19937 stream)", 0, 1, 5489, 1 << 24, "u32"),
    ("mt64_M8_2^26_u64", 1, 8, 5489, 1 << 26, "u64"),
    ("mt64_M8_2^26_f64", 1, 8, 5489, 1 << 26, "f64"),
    ("sfmt_M4_2^28_u32", 2, 4, 1234, 1 << 28, "u32"),
    ("sfmt_M64_2^28_u32", 2, 64, 1234, 1 << 28, "u32"),
    ("sfmt_M64_2^28_f32", 2, 64, 1234, 1 << 28, "f32"),
    ("sfmt607_M64_2^28_u32", 3, 64, 1234, 1 << 28, "u32"),
    ("sfmt11213_M16_2^28_u32", 7, 16, 1234, 1 << 28, "u32"),
)


def single_streams(ctx, torch, args, only=None) -> dict:
    """Workloads 1-3 (one generator each, after autotuning the generate family):
    output GB/s of one call of n elements, state resident in HBM."""
    from paper_2309_16682_amd import vmt

    dev = torch.device("cuda:0")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sec = {}
    for name, variant, M, seed, n, kind in SINGLE_STREAMS:
        if only and name.split(" ")[0] not in only:
            continue
        okind = {"u32": vmt.VMT_OUT_U32, "u64": vmt.VMT_OUT_U64, "f64": vmt.VMT_OUT_F64, "f32": vmt.VMT_OUT_F32}[kind]
        lpw = split = None
        if args.single_shape:  # a fixed shape (profiling one configuration): lanes per workgroup, log2 chunk
            lpw, split = (int(x) for x in args.single_shape.split(","))
            vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, variant, M, okind, lanes_per_wg=lpw, split_log2=split)
        elif not args.no_autotune:
            b, tried = vmt.vmt_autotune(ctx, vmt.VMT_FAMILY_GENERATE, variant, M, okind, [n], reps=2)
            lpw = b.lanes_per_wg
            split = b.split_log2
            log(f"{name} autotune: " + ", ".join(
                f"{'lpw=%d' % t.lanes_per_wg if t.split_log2 == 255 else 'split=2^%d/lpw=%d' % (t.split_log2, t.lanes_per_wg)}: "
                f"{t.gbps:.1f}" for t in tried))
        st = vmt.new_state(variant, M)
        vmt.vmt_init_genrand(ctx, variant, seed, M, st)
        esz = 8 if kind in ("u64", "f64") else 4
        # successive calls write to a rotation of output buffers totalling at least 1 GiB, so that no call's
        # output still sits in the 256 MB last-level cache when the next one is timed
        nbuf = max(2, -(-(1 << 30) // (n * esz)))
        outs = [torch.empty(n * esz, dtype=torch.uint8, device=dev) for _ in range(nbuf)]
        fn = {"u32": vmt.vmt_generate_u32, "u64": vmt.vmt_generate_u64, "f64": vmt.vmt_uniform_f64,
              "f32": vmt.vmt_uniform_f32}[kind]
        fn(ctx, st, n, outs[-1])
        torch.cuda.synchronize()
        reps = max(nbuf, 2 if variant in vmt.SFMT_FAMILY and M <= 16 else 3)
        e0.record()
        for r in range(reps):
            fn(ctx, st, n, outs[r % nbuf])
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) * 1e-3 / reps
        shp = vmt.vmt_shape_get(ctx, vmt.VMT_FAMILY_GENERATE, variant, M, okind)
        gbps = n * esz / s / 1e9
        sec[name] = {"GB/s": round(gbps, 2), "ms": round(s * 1e3, 3),
                     "lanes_per_wg": shp.lanes_per_wg,
                     "split": "never" if shp.split_log2 == 255 else (
                         "auto" if shp.split_log2 == 0 else f"chunks of 2^{shp.split_log2} lane steps"),
                     "output_rotation": f"{nbuf} buffers, {nbuf * n * esz / 2**30:.2f} GiB",
                     # whole call (copies, jumps, generation, position fix-ups) against the HBM write peak
                     "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(gbps / HBM_PEAK_GBS, 4), "scope": "whole call, output bytes"}}
        log(f"{name}: {sec[name]}")
        del outs
    return sec


# Batched lines of the other generator families: 65,536 lanes' worth of generators (65,536 / M of them) seeded
# init_genrand(i + 1) in one batched call, each asked for a log-uniform number of elements in
# [M/16 * 1e3, M/16 * 1e7) (the headline batch's volume per lane), one launch of a batch plan over them.
# name, variant, lanes, output kind, bytes per element
BATCH_VARIANTS = (
    ("mt64_M8_u64", 1, 8, 1, 8),
    ("mt64_M8_f64", 1, 8, 3, 8),
    ("sfmt_M4_u32", 2, 4, 0, 4),
    ("sfmt_M4_f32", 2, 4, 2, 4),
    ("sfmt_M64_u32", 2, 64, 0, 4),
    ("sfmt_M64_f32", 2, 64, 2, 4),
)


def batched_variants(ctx, torch, args, only=None) -> dict:
    """Output GB/s and roofline of one batch-plan launch per family (mean of
    `reps` launches timed with HIP events on the stream they run on; the
    states continue from launch to launch, the outputs are overwritten)."""
    from paper_2309_16682_amd import vmt
    from paper_2309_16682_amd.workload import batch_lengths

    res = {}
    run_stream = torch.cuda.Stream()
    for name, variant, M, kind, esz in BATCH_VARIANTS:
        if only and name not in only:
            continue
        G = 65536 // M
        lens = batch_lengths(G, seed=47, lo=1e3 * M / 16, hi=1e7 * M / 16)
        sb = vmt.vmt_state_bytes(variant, M)
        pool = torch.empty(G * sb, dtype=torch.uint8, device="cuda")
        states = [pool[i * sb : (i + 1) * sb] for i in range(G)]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        vmt.vmt_init_genrand_batch(ctx, variant, [i + 1 for i in range(G)], M, states)
        e1.record()
        torch.cuda.synchronize()
        init_ms = e0.elapsed_time(e1)
        tune = None
        if variant not in vmt.SFMT_FAMILY and not args.no_autotune:  # the MT persistent kernel has launch shapes
            sample = np.random.default_rng(17).choice(lens, size=min(4096, G), replace=False)
            best, _ = vmt.vmt_autotune(ctx, vmt.VMT_FAMILY_BATCH, variant, M, kind, sample, reps=2)
            tune = {"threads": best.threads, "store_bytes": best.store_bytes, "wg_per_cu": best.wg_per_cu}
        offs = np.concatenate([[0], np.cumsum((lens * esz + 255) // 256 * 256)]).astype(np.int64)
        arena = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")
        plan = vmt.vmt_batch_plan_create(ctx, states, [int(x) for x in lens],
                                         [arena.data_ptr() + int(o) for o in offs[:-1]], kind)
        try:
            with torch.cuda.stream(run_stream):
                vmt.vmt_batch_plan_launch(plan, run_stream)
            torch.cuda.synchronize()
            reps = 3
            e0.record(run_stream)
            for _ in range(reps):
                vmt.vmt_batch_plan_launch(plan, run_stream)
            e1.record(run_stream)
            torch.cuda.synchronize()
        finally:
            vmt.vmt_batch_plan_destroy(plan)
        ms = e0.elapsed_time(e1) / reps
        out_bytes = int(lens.sum()) * esz
        alg = out_bytes + 2 * (sb - 256) * G
        res[name] = {
            "generators": G, "lanes": M, "elements": int(lens.sum()), "output_bytes": out_bytes,
            "lengths": f"log-uniform [{1e3 * M / 16:g}, {1e7 * M / 16:g}) elements (splitmix64(47))",
            "seeding": f"init_genrand(i + 1), one batched call: {init_ms:.1f} ms",
            "ms_per_launch": round(ms, 3), "GB/s": round(out_bytes / (ms * 1e-3) / 1e9, 1),
            "shape": tune,
            "roofline": {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "alg_bytes_per_launch": alg,
                         "kernel": ("batch_mt_kernel" if variant == 1 else "batch_sfmt_kernel")},
        }
        log(f"batched {name}: {res[name]}")
        del arena, pool, states
        torch.cuda.empty_cache()
    return res


# Jumps by 2^100 steps per lane: one state, and batches of states (the sliced grouped form up to 1,024 lane jumps,
# the per-coefficient form beyond). name, variant, lanes, states
JUMP_CASES = (
    ("mt32_M16_1state", 0, 16, 1),
    ("mt64_M8_1state", 1, 8, 1),
    ("sfmt_M4_1state", 2, 4, 1),
    ("mt64_M8_128states", 1, 8, 128),
    ("mt32_M16_256states", 0, 16, 256),
)


def jumps(ctx, torch, reps: int = 10, k: int = 100) -> dict:
    """Time vmt_jump_pow2 / vmt_jump_pow2_batch by 2^k. Algorithmic LDS reads
    per lane jump: one window (2,496 bytes for every variant) per nonzero
    group of 4 coefficients of g = t^(2^k) mod mu (grouped form, up to 1,024
    lane jumps per call) or per set coefficient (beyond); against the LDS
    peak of 256 CUs x 128 B/clock x 2.4 GHz."""
    from paper_2309_16682_amd import vmt

    res = {}
    for name, variant, M, count in JUMP_CASES:
        g = vmt.vmt_jump_poly(ctx, variant, 1 << k)
        nib = sum(1 for i in range(0, g.bit_length(), 4) if (g >> i) & 15)
        bits = bin(g).count("1")
        lanes = M * count
        grouped = lanes <= 1024
        win = (vmt.vmt_state_bytes(variant, M) - 256) // M  # bytes of one lane's window
        lds = (nib if grouped else bits) * win
        sb = vmt.vmt_state_bytes(variant, M)
        pool = torch.empty(count * sb, dtype=torch.uint8, device="cuda")
        states = [pool[i * sb : (i + 1) * sb] for i in range(count)]
        vmt.vmt_init_genrand_batch(ctx, variant, [i + 1 for i in range(count)], M, states)
        call = (lambda: vmt.vmt_jump_pow2(ctx, states[0], k)) if count == 1 else (
            lambda: vmt.vmt_jump_pow2_batch(ctx, states, [k] * count))
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rate = lanes * lds / (ms * 1e-3)
        res[name] = {"lane_jumps": lanes, "ms_per_call": round(ms, 4), "us_per_lane_jump": round(ms * 1e3 / lanes, 3),
                     "form": "grouped, sliced over a workgroup per lane" if grouped else "per coefficient",
                     "set_coefficients": bits, "nonzero_groups": nib, "lds_bytes_per_lane_jump": lds,
                     "roofline": {"bound": "lds", "achieved": round(rate / 1e9, 1), "peak": LDS_PEAK_BYTES / 1e9,
                                  "unit": "GB/s", "frac": round(rate / LDS_PEAK_BYTES, 4),
                                  "scope": "whole call (jump kernel and position fix-up)"}}
        log(f"jump {name}: {res[name]}")
        del pool, states
    return res


def call_size_sweep(ctx, torch) -> dict:
    """Workload 1's call-size sweep: one V-MT19937-32 (M = 16) state, calls of
    1 .. 2^20 elements (powers of 4), each timed over repeated back-to-back
    calls: per-call time (launch overhead at the small end) and output GB/s."""
    from paper_2309_16682_amd import vmt

    # the default shape (lanes per workgroup and splitting chosen per call), not one tuned for 2^24 elements
    vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, vmt.VMT_MT32, 16, vmt.VMT_OUT_U32)
    st = vmt.new_state(vmt.VMT_MT32, 16)
    vmt.vmt_init_genrand(ctx, vmt.VMT_MT32, 7, 16, st)
    out = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for lg in range(0, 21, 2):
        n = 1 << lg
        reps = 200 if n <= 4096 else 50
        vmt.vmt_generate_u32(ctx, st, n, out)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            vmt.vmt_generate_u32(ctx, st, n, out)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        res[f"2^{lg}"] = {"us_per_call": round(us, 2), "GB/s": round(4 * n / us / 1e3, 3)}
    log(f"call-size sweep: {res}")
    return res


def self_check(ctx, torch, reps: int = 3) -> dict:
    """Time vmt_check_stream on single streams: term-XORs = set coefficients x checked offsets."""
    from paper_2309_16682_amd import vmt

    res = {}
    for name, variant, M, seed, n, kind, esz, wpe, S in (
        ("mt32_M16_2^24_u32", vmt.VMT_MT32, 16, 5489, 1 << 24, vmt.VMT_OUT_U32, 4, 1, 1),
        ("mt64_M8_2^26_u64", vmt.VMT_MT64, 8, 5489, 1 << 26, vmt.VMT_OUT_U64, 8, 2, 2),
        ("sfmt_M4_2^28_u32", vmt.VMT_SFMT, 4, 1234, 1 << 28, vmt.VMT_OUT_U32, 4, 1, 4),
    ):
        A = vmt.vmt_check_poly(ctx, variant, M)
        deg, terms = A.bit_length() - 1, bin(A).count("1")
        st = vmt.new_state(variant, M)
        vmt.vmt_init_genrand(ctx, variant, seed, M, st)
        out = torch.empty(n * esz, dtype=torch.uint8, device="cuda")
        (vmt.vmt_generate_u64 if esz == 8 else vmt.vmt_generate_u32)(ctx, st, n, out)
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        stream = torch.cuda.current_stream()
        vmt.vmt_check_stream(ctx, variant, M, kind, out, n, cnt, stream=stream)  # uploads A, warms up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            vmt.vmt_check_stream(ctx, variant, M, kind, out, n, cnt, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / reps
        nw = n * wpe
        offsets = nw - deg * S
        rate = terms * offsets / sec
        dense = terms * 8 > deg  # the library's choice of form
        res[name] = {"failing_offsets": int(cnt.item()), "words": nw, "ms": round(sec * 1e3, 3),
                     "Gwords_per_s": round(nw / sec / 1e9, 3), "set_coefficients": terms,
                     "form": "dense" if dense else "sparse", "term_xors_per_s": float(f"{rate:.4g}")}
        if dense:
            res[name]["roofline"] = {"bound": "alu", "achieved": float(f"{rate / 1e12:.4g}"),
                                     "peak": CHECK_PEAK_TERMS / 1e12, "unit": "T term-XORs/s",
                                     "frac": round(rate / CHECK_PEAK_TERMS, 3)}
        else:
            lds = 4 * rate
            res[name]["roofline"] = {"bound": "lds", "achieved": round(lds / 1e9, 1), "peak": LDS_PEAK_BYTES / 1e9,
                                     "unit": "GB/s", "frac": round(lds / LDS_PEAK_BYTES, 3)}
        log(f"self-check {name}: {res[name]}")
        del out
    return res


def serving(ctx, seconds: float, warm: float, mode: int, n_streams: int = 4, chunk: int = 1 << 20,
            rate: float = 20000.0) -> dict:
    """Serving configuration: 4096 device-resident V-MT19937-64 (M = 8)
    states seeded init_genrand(i + 1); Poisson arrivals at 20k requests/s,
    request sizes log-uniform in [4 KiB, 256 MiB] of uint64, 10% of requests
    a jump by 2^k with k uniform in [32, 256], 16 GiB admission budget. Requests
    arriving in the first `warm` seconds run but are not counted."""
    import torch

    from paper_2309_16682_amd import vmt
    from paper_2309_16682_amd.workload import serving_trace

    n_states, Mv = 4096, 8
    sb = vmt.vmt_state_bytes(vmt.VMT_MT64, Mv)
    pool = torch.empty(n_states * sb, dtype=torch.uint8, device="cuda")
    states = [pool[i * sb : (i + 1) * sb] for i in range(n_states)]
    vmt.vmt_init_genrand_batch(ctx, vmt.VMT_MT64, [i + 1 for i in range(n_states)], Mv, states)
    torch.cuda.synchronize()
    budget = 16 * 2**30
    arena = torch.empty(budget, dtype=torch.uint8, device="cuda")
    trace = serving_trace(seconds + warm, rate_per_s=rate, n_states=n_states, min_bytes=4096,
                          max_bytes=256 << 20, elem_bytes=8, jump_fraction=0.1, kmin=32, kmax=256, seed=11)
    reqs = [(r.t_arrival, r.state, 0 if r.kind == "gen" else 1, r.nelem if r.kind == "gen" else 0, r.k) for r in trace]
    srv = vmt.vmt_server_create(ctx, states, arena, budget, budget, vmt.VMT_OUT_U64, n_streams=n_streams, mode=mode,
                                chunk_elems=chunk)
    try:
        res, wall = vmt.vmt_server_run(srv, reqs, realtime=True)
    finally:
        vmt.vmt_server_destroy(srv)
    t_arr = np.array([r[0] for r in reqs])
    kind = np.array([r[2] for r in reqs])
    cnt = np.array([r[3] for r in reqs], dtype=np.float64)
    ok = res["status"] == 0
    counted = ok & (t_arr >= warm)
    lat = (res["t_done"] - t_arr) * 1e3
    wait = (res["t_admit"] - t_arr) * 1e3
    g = counted & (kind == 0)
    j = counted & (kind == 1)
    gen_bytes = float((cnt[g] * 8).sum())
    span = float(res["t_done"][counted].max() - warm)
    offered = float(sum(8 * r[3] for r in reqs if r[0] >= warm)) / seconds
    out = {
        "offered_requests_per_s": rate,
        "offered_GB/s": round(offered / 1e9, 2),
        "mode": {0: "continuous batching, long requests as successive bounded tasks",
                 4: "continuous batching, long requests split by jump-ahead into chunks run side by side",
                 1: "plain (one launch per request)"}[mode] if chunk else (
                     "continuous batching, one task per request" if mode == 0 else "plain (one launch per request)"),
        "chunk_elems": chunk,
        "requests": int(counted.sum()),
        "generate_requests": int(g.sum()),
        "jump_requests": int(j.sum()),
        "GB/s": round(gen_bytes / span / 1e9, 2),
        "requests_per_s": round(float(counted.sum()) / span, 1),
        "p50_ms": round(float(np.percentile(lat[g], 50)), 3),
        "p99_ms": round(float(np.percentile(lat[g], 99)), 3),
        "mean_ms": round(float(lat[g].mean()), 3),
        "jump_p50_ms": round(float(np.percentile(lat[j], 50)), 3) if j.any() else None,
        "jump_p99_ms": round(float(np.percentile(lat[j], 99)), 3) if j.any() else None,
        "admit_wait_p99_ms": round(float(np.percentile(wait[counted], 99)), 3),
        "launches": int(res["launch"].max() + 1),
        "wall_s": round(wall, 2),
    }
    del arena, pool
    torch.cuda.empty_cache()
    return out


def serving_capacity(ctx, seconds: float = 2.0, warm: float = 0.5) -> dict:
    """The serving workload at rising arrival rates (same request mix): a rate
    is sustained when the loop completes requests at >= 97 % of the offered
    rate and the p99 wait for admission stays under 50 ms. The capacity is the
    highest sustained rate, with its delivered GB/s as a fraction of 8 TB/s."""
    out = {}
    # splitting with chunks of 2^20 (the 20k rows above) and 2^21 elements: larger chunks need fewer jumps per
    # request (more capacity) and leave the largest requests on fewer workgroups (longer p99 at low load)
    for label, mode, chunk, rates in (("batched_split", 4, 1 << 20, (20e3, 40e3, 60e3, 80e3, 160e3)),
                                      ("batched_split_chunk2^21", 4, 1 << 21, (20e3, 40e3, 60e3, 80e3, 100e3, 160e3)),
                                      ("batched", 0, 1 << 20, (20e3, 40e3, 60e3, 80e3, 160e3)),
                                      ("plain", 1, 0, (500.0, 1e3, 2e3, 4e3))):
        rows = []
        for rate in rates:
            r = serving(ctx, seconds, warm, mode, chunk=chunk, rate=rate)
            r["sustained"] = bool(r["requests_per_s"] >= 0.97 * rate and r["admit_wait_p99_ms"] < 50.0)
            rows.append({k: r[k] for k in ("offered_requests_per_s", "offered_GB/s", "requests_per_s", "GB/s",
                                           "p50_ms", "p99_ms", "jump_p99_ms", "admit_wait_p99_ms", "sustained")})
            log(f"serving capacity {label} at {rate:g} req/s: {rows[-1]}")
            if not r["sustained"]:
                break
        ok = [x for x in rows if x["sustained"]]
        best = max(ok, key=lambda x: x["GB/s"]) if ok else None
        out[label] = {"rates": rows,
                      "capacity_requests_per_s": best["requests_per_s"] if best else None,
                      "capacity_GB/s": best["GB/s"] if best else None,
                      "capacity_frac_of_hbm": round(best["GB/s"] / HBM_PEAK_GBS, 4) if best else None,
                      "p50_ms_at_capacity": best["p50_ms"] if best else None,
                      "p99_ms_at_capacity": best["p99_ms"] if best else None}
    out["rule"] = ("sustained: completed requests/s >= 0.97 x offered and admission-wait p99 < 50 ms; "
                   f"{seconds:g} s per rate after {warm:g} s warm-up; the sweep of a mode stops at its first "
                   "unsustained rate")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(
            f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
            "(independent generators shard across GPUs with no communication)",
            file=sys.stderr,
        )
        sys.exit(2)

    import torch

    from paper_2309_16682_amd import vmt
    from paper_2309_16682_amd.workload import batch_keys, batch_lengths, plan_rounds

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate:
        ctx = vmt.vmt_ctx_create(0)
        print(json.dumps(calibrate(torch, ctx)), flush=True)
        vmt.vmt_ctx_destroy(ctx)
        return
    if args.only_single:
        ctx = vmt.vmt_ctx_create(0)
        print(json.dumps({"single_stream": single_streams(ctx, torch, args, args.only_single.split(",")),
                          "call_size_sweep_mt32_M16": call_size_sweep(ctx, torch)}), flush=True)
        vmt.vmt_ctx_destroy(ctx)
        return
    if args.only_variants:
        ctx = vmt.vmt_ctx_create(0)
        only = None if args.only_variants == "all" else args.only_variants.split(",")
        print(json.dumps({"batched_variants": batched_variants(ctx, torch, args, only)}), flush=True)
        vmt.vmt_ctx_destroy(ctx)
        return
    if args.only_jumps:
        ctx = vmt.vmt_ctx_create(0)
        print(json.dumps({"jumps": jumps(ctx, torch)}), flush=True)
        vmt.vmt_ctx_destroy(ctx)
        return
    if args.only_check:
        ctx = vmt.vmt_ctx_create(0)
        print(json.dumps({"self_check": self_check(ctx, torch)}), flush=True)
        vmt.vmt_ctx_destroy(ctx)
        return
    if args.only_serving:
        ctx = vmt.vmt_ctx_create(0)
        out = {m: serving(ctx, args.serve_seconds, 1.0, mode, chunk=c) for m, mode, c in
               (("batched_split", 4, 1 << 20), ("batched", 0, 1 << 20), ("batched_unchunked", 0, 0))}
        out["capacity"] = serving_capacity(ctx)
        print(json.dumps({"serving": out}), flush=True)
        return
    stream = torch.cuda.current_stream()
    ctx = vmt.vmt_ctx_create(0)

    ceiling = calibrate(torch, ctx)  # measured write ceiling on this device, before the big allocations
    torch.cuda.empty_cache()
    log(f"device copy/fill: {ceiling}")

    G = args.generators
    keys = batch_keys(G, seed=42)
    lens = batch_lengths(G, seed=43)
    sb = vmt.vmt_state_bytes(vmt.VMT_MT32, M_LANES)
    state_pool = torch.empty(G * sb, dtype=torch.uint8, device=dev)
    states = [state_pool[i * sb : (i + 1) * sb] for i in range(G)]

    # ---- lane de-phasing: seeding + M-1 jump-aheads per generator (device)
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    vmt.vmt_init_by_array(ctx, vmt.VMT_MT32, keys[0], M_LANES, states[0])  # builds the lane table
    torch.cuda.synchronize()
    host_poly_s = time.perf_counter() - t0
    e0.record()
    vmt.vmt_init_by_array_batch(ctx, keys, M_LANES, states)
    e1.record()
    torch.cuda.synchronize()
    init_ms = e0.elapsed_time(e1)
    log(f"init: {G} generators in {init_ms:.1f} ms (+{host_poly_s:.2f} s host polynomials)")

    # ---- autotune the persistent kernel's launch shape on a sample of the task lengths
    tune = None
    if args.shape:
        tv, sw, wpc = (int(x) for x in args.shape.split(","))
        vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_BATCH, vmt.VMT_MT32, M_LANES, vmt.VMT_OUT_U32, threads_variant=tv,
                          store_bytes=sw, wg_per_cu=wpc)
    elif not args.no_autotune:
        sample_lens = np.random.default_rng(17).choice(lens, size=min(args.tune_sample, G), replace=False)
        t0 = time.perf_counter()
        best, tried = vmt.vmt_autotune(ctx, vmt.VMT_FAMILY_BATCH, vmt.VMT_MT32, M_LANES, vmt.VMT_OUT_U32, sample_lens,
                                       reps=2)
        tune = {
            "sample": f"{len(sample_lens)} task lengths drawn from the workload, "
            f"{float(sample_lens.sum()) * 4 / 1e9:.1f} GB of output per trial",
            "seconds": round(time.perf_counter() - t0, 2),
            "best": {k: (round(v, 1) if k == "gbps" else v) for k, v in best.as_dict().items()},
            "tried": [[t.threads, t.store_bytes, t.wg_per_cu, round(t.gbps, 1)] for t in tried],
            "tried_columns": ["threads", "store_bytes", "wg_per_cu", "GB/s"],
        }
        log(f"autotune: best {tune['best']} of {len(tried)} shapes in {tune['seconds']} s")
    shape = vmt.vmt_shape_get(ctx, vmt.VMT_FAMILY_BATCH, vmt.VMT_MT32, M_LANES, vmt.VMT_OUT_U32)

    # ---- arena and rounds
    free, _ = torch.cuda.mem_get_info()
    arena_bytes = int(min(args.arena_gib * 2**30, free - 16 * 2**30))
    arena_bytes = max(arena_bytes, 1 << 30)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    rounds, offs = plan_rounds(lens, arena_bytes, 4)
    base = arena.data_ptr()
    plans = []
    round_alg_bytes = []
    for idx in rounds:
        sp = [states[int(i)].data_ptr() for i in idx]
        ln = [int(lens[i]) for i in idx]
        op = [base + offs[int(i)] for i in idx]
        plans.append(vmt.vmt_batch_plan_create(ctx, sp, ln, op, vmt.VMT_OUT_U32))
        round_alg_bytes.append(sum(ln) * 4 + len(idx) * 2 * STATE_WIN_BYTES)
    step_out_bytes = int(lens.sum()) * 4
    log(f"rounds: {len(plans)} over a {arena_bytes / 2**30:.1f} GiB arena; {step_out_bytes / 1e9:.1f} GB per step")

    # one step = every round's persistent launch, captured once into a HIP graph and replayed
    run_stream = torch.cuda.Stream()
    graph = None
    if not args.no_graph:
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(run_stream):
            with torch.cuda.graph(graph, stream=run_stream):
                for p in plans:
                    vmt.vmt_batch_plan_launch(p)
        torch.cuda.synchronize()

    def step():
        with torch.cuda.stream(run_stream):
            if graph is not None:
                graph.replay()
            else:
                for p in plans:
                    vmt.vmt_batch_plan_launch(p)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(run_stream)
        step()
        b.record(run_stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    step_ms = [a.elapsed_time(b) for a, b in evs]
    # events bracket each replay on the stream the kernels run on; a replay is
    # the rounds' launches back to back, so the mean launch duration is the
    # event time over the number of launches (gaps between them included)
    kern_ms_total = float(np.sum(step_ms))
    launch_ms_mean = kern_ms_total / (args.steps * len(plans))
    alg_total = sum(round_alg_bytes) * args.steps
    achieved = alg_total / (kern_ms_total * 1e-3) / 1e9
    value = step_out_bytes / (ms_per_step * 1e-3) / 1e9
    log(f"batched: {ms_per_step:.2f} ms/step, {value:.1f} GB/s output; kernel avg {launch_ms_mean:.3f} ms/launch")

    # the ceiling of this output pattern: the same plans and launch shape with the twist left out
    # (vmt_batch_plan_write_pattern: same queue, stores and state traffic; states unchanged)
    pattern_ms = None
    if not args.no_pattern:
        with torch.cuda.stream(run_stream):
            for p in plans:
                vmt.vmt_batch_plan_write_pattern(p, run_stream)
        torch.cuda.synchronize()
        pa, pb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        preps = 2
        pa.record(run_stream)
        for _ in range(preps):
            for p in plans:
                vmt.vmt_batch_plan_write_pattern(p, run_stream)
        pb.record(run_stream)
        torch.cuda.synchronize()
        pattern_ms = pa.elapsed_time(pb) / (preps * len(plans))
        log(f"write pattern without the twist: {pattern_ms:.3f} ms/launch")

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"batched V-MT19937-32, M=16 lanes, {G} generators (init_by_array keys from "
            f"splitmix64(42)), log-uniform request lengths in [1e3,1e7) uint32 (splitmix64(43)), "
            f"persistent kernel, longest first, one HIP graph per step",
            "generators": G,
            "lanes": M_LANES,
            "elements_per_step": int(lens.sum()),
            "output_bytes_per_step": step_out_bytes,
            "rounds": len(plans),
            "arena_gib": round(arena_bytes / 2**30, 1),
            "launch": "hipGraph replay" if graph is not None else "eager launches",
            "shape": {"threads": shape.threads, "store_bytes": shape.store_bytes,
                      "wg_per_cu": shape.wg_per_cu or "max"},
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": counter_traffic(shape),
            "kernel": "batch_mt_kernel<MT32, 16 lanes, u32>",
            "avg_launch_ms": round(launch_ms_mean, 4),
            "measured_fill_GBps": ceiling["fill_GBps"],
            "measured_memset_GBps": ceiling["memset_GBps"],
            "frac_of_measured_fill": round(achieved / ceiling["fill_GBps"], 4),
            # the library's own fills: 4 KiB pieces in address order, and two contiguous regions per CU
            # written side by side (the pattern of many independent output streams)
            "measured_fill_pieces_GBps": ceiling.get("fill_pieces_GBps"),
            "measured_fill_regions_GBps": ceiling.get("fill_regions_GBps"),
            "measured_fill_regions_nt_GBps": ceiling.get("fill_regions_nt_GBps"),
            "frac_of_fill_regions": round(achieved / ceiling["fill_regions_GBps"], 4)
            if ceiling.get("fill_regions_GBps") else None,
            "pattern_ceiling_GBps": round(np.mean(round_alg_bytes) / (pattern_ms * 1e-3) / 1e9, 1) if pattern_ms else None,
            "frac_of_pattern_ceiling": round(launch_ms_mean and pattern_ms / launch_ms_mean, 4) if pattern_ms else None,
            "alg_bytes_per_launch": int(np.mean(round_alg_bytes)),
        },
        "init": {"generators": G, "device_ms": round(init_ms, 2), "lane_jumps": G * (M_LANES - 1),
                 "host_poly_s": round(host_poly_s, 3)},
        "autotune": tune,
    }
    if args.only_batch:
        print(json.dumps(result), flush=True)
        return

    # ---- plain form: one launch per generator (same kernel family), sample
    rng = np.random.default_rng(5)
    sample = rng.choice(G, size=min(args.plain_sample, G), replace=False)
    out_base = arena
    # the plain form: one workgroup per generator, one launch each, no splitting
    vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, vmt.VMT_MT32, M_LANES, vmt.VMT_OUT_U32, lanes_per_wg=M_LANES,
                      split_log2=255)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    off = 0
    plain_bytes = 0
    for i in sample:
        n = int(lens[i])
        view = out_base[off : off + n * 4]
        vmt.vmt_generate_u32(ctx, states[int(i)], n, view)
        off += ((n * 4 + 255) // 256) * 256
        plain_bytes += n * 4
    e1.record()
    torch.cuda.synchronize()
    vmt.vmt_shape_set(ctx, vmt.VMT_FAMILY_GENERATE, vmt.VMT_MT32, M_LANES, vmt.VMT_OUT_U32)
    plain_s = e0.elapsed_time(e1) * 1e-3
    result["plain"] = {
        "value": round(plain_bytes / plain_s / 1e9, 3),
        "unit": "GB/s",
        "form": "one vmt_generate_u32 launch per generator (one workgroup, no splitting), same stream",
        "sample": f"{len(sample)} random generators of the batch, {plain_bytes / 1e9:.2f} GB",
        "speedup_batched_vs_plain": round(value / (plain_bytes / plain_s / 1e9), 1),
    }
    log(f"plain: {result['plain']['value']} GB/s")

    # ---- single-stream configurations (one generator each)
    if not args.skip_secondary:
        torch.cuda.empty_cache()
        result["single_stream"] = single_streams(ctx, torch, args)
        result["call_size_sweep_mt32_M16"] = call_size_sweep(ctx, torch)
        result["self_check"] = self_check(ctx, torch)
        result["jumps"] = jumps(ctx, torch)

    arena = out_base = None  # the batch arena is not needed any more
    torch.cuda.empty_cache()
    if not args.skip_secondary:
        result["batched_variants"] = batched_variants(ctx, torch, args)
    if not args.skip_serving:
        result["serving"] = {
            "config": "4096 V-MT19937-64 (M=8) states, Poisson 20k req/s, log-uniform 4 KiB-256 MiB uint64, "
            f"10% jumps by 2^k (k in [32,256]), 16 GiB budget, 4 streams, {args.serve_seconds:g} s after 1 s warm-up "
            f"(plain: {max(args.serve_seconds / 10, 0.5):g} s after 0.2 s); chunks of 2^20 elements",
            "batched_split": serving(ctx, args.serve_seconds, 1.0, 4),
            "batched": serving(ctx, args.serve_seconds, 1.0, 0),
            "batched_unchunked": serving(ctx, args.serve_seconds, 1.0, 0, chunk=0),
            # the plain form cannot keep up with the offered rate: a shorter trace keeps its run bounded
            "plain": serving(ctx, max(args.serve_seconds / 10, 0.5), 0.2, 1, chunk=0),
        }
        result["serving"]["capacity"] = serving_capacity(ctx)
        log(f"serving: {result['serving']}")

    result["cpu_baseline"] = cpu_baseline(args.cpu_seconds, max(1, min(os.cpu_count() or 1, args.cpu_threads)))
    log(f"cpu baseline: {result['cpu_baseline']['value']} GB/s")
    for p in plans:
        vmt.vmt_batch_plan_destroy(p)
    vmt.vmt_ctx_destroy(ctx)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
