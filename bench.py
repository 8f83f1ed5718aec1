#!/usr/bin/env python3
"""Benchmark: Fast-SSC decoding of the (32768, 29492) polar code, int8 LLRs.

One step = one batched decode launch of 4,096 frames (channel LLRs already
resident in HBM; the steps cycle over 4 copies of the frames so that none
finds its rows in the Infinity Cache), the workload on which the paper
quotes its 26 us / 1.13 Gb/s single-core figure for this code.  Prints one
JSON line:

  value        information throughput (Gb/s) of the batched decode;
  latency_us   p50/p99 frame latency of a batched launch (submit -> done);
  plain        the same frames decoded with one launch per frame (and with
               the layout the autotuner picks for one frame per launch);
  roofline     algorithmic HBM bytes (LLR in + info bits out) per launch
               over the decode kernel's mean duration vs 8 TB/s (and vs a
               measured plain copy of 1 GiB);
  valu         the bound that actually holds: the kernel's vector-ALU
               instructions per frame (committed counter summary) at one
               wave64 instruction per 4 cycles on each of the 1,024 SIMDs at
               2.4 GHz, as a time floor per launch vs the measured time;
  cpu_baseline the CPU oracle on a bounded sample on this host's cores;
  mixed_batch  the 65,536-frame mixed-code workload in one persistent,
               autotuned launch (information Gb/s, launch time, FER);
  serving      the continuous-batching server under Poisson arrivals at
               10/50/90% of the batch capacity: Gb/s and p50/p99 latency.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "info Gbps/GPU + p50/p99 frame latency (µs), (32768,29492) int8 vs plain"
HBM_PEAK_GBS = 8000.0


def make_inputs(code, seed, frames, ebn0_db):
    from paper_1504_00353_amd import synth
    fr = code.frozen()
    idx = np.arange(frames)
    bits = synth.info_bits(seed, idx, code.k)
    x = synth.unpack_bits(code.encode(synth.pack_bits(bits)), code.n)
    z = synth.noise(seed, idx, code.n)
    llr = synth.quantize6(synth.awgn_llr(x, z, ebn0_db, code.k / code.n))
    return fr, bits, llr


def kernel_source_hash():
    """Hash of the sources that make up the decode kernel; HBM counter
    readings are only valid for the kernel they were taken on."""
    h = hashlib.sha256()
    for f in ("decode_ops.h", "opcodes.h", "decode.hip", "unrolled.cpp", "plan.h", "construct.cpp"):
        with open(os.path.join(ROOT, "paper_1504_00353_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_file(kernel):
    name = "polar_unrolled" if kernel == "unrolled" else "decode_kernel"
    return os.path.join(ROOT, "profiles", "%s_i8_32768x29492_hbm_traffic.txt" % name)


def measured_traffic(frames, kernel):
    """HBM bytes per launch from the committed counter summary: FETCH_SIZE
    and WRITE_SIZE of the decode kernel, each scaled by the same counter's
    reading on a plain copy of known size.  None when there is no summary
    for this frame count or the kernel sources changed since it was taken."""
    path = pmc_file(kernel)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                a, b = line.split(":", 1)
                kv[a.strip()] = b.strip()
    try:
        if kv.get("kernel_source_hash") != kernel_source_hash() or int(kv["frames"]) != frames:
            return None
        copy_bytes = float(kv["copy_bytes"])
        fetch = float(kv["decode_fetch_kib"]) * copy_bytes / float(kv["copy_fetch_kib"])
        write = float(kv["decode_write_kib"]) * copy_bytes / float(kv["copy_write_kib"])
    except (KeyError, ValueError, ZeroDivisionError):
        return None
    return fetch + write


VALU_CLOCK_GHZ = 2.4
VALU_SIMDS = 1024  # 256 CUs x 4 SIMDs; a wave64 VALU instruction takes 4 cycles on a 16-lane SIMD


def valu_view(frames, kernel, mean_kernel_ms):
    """Vector-ALU floor of one launch from the committed counter summary
    (SQ_INSTS_VALU per wave), or None when the summary is missing or was
    taken on other kernel sources."""
    if kernel != "unrolled":
        return None
    path = os.path.join(ROOT, "profiles", "polar_unrolled_i8_32768x29492_valu.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                a, b = line.split(":", 1)
                kv[a.strip()] = b.strip().split()[0]
    try:
        if kv.get("kernel_source_hash") != kernel_source_hash():
            return None
        per_frame = float(kv["valu_insts_per_frame"])
    except (KeyError, ValueError):
        return None
    floor_ms = frames * per_frame * 4.0 / VALU_SIMDS / (VALU_CLOCK_GHZ * 1e9) * 1e3
    return {"bound": "alu", "valu_insts_per_frame": round(per_frame, 1), "clock_ghz": VALU_CLOCK_GHZ,
            "floor_ms": round(floor_ms, 4), "frac": round(floor_ms / mean_kernel_ms, 4),
            "what": "frames x VALU instructions x 4 cycles / 1024 SIMDs / clock, over the mean kernel time"}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Measured HBM bandwidth of a plain device copy (bytes read + written
    per second, GB/s): the practical ceiling beside the 8 TB/s peak."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def copy_calibration(nbytes, reps):
    """A plain copy of known size (read nbytes, write nbytes) for scaling
    the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.randint(-128, 127, (nbytes,), dtype=torch.int8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps,
                      "kernel": "elementwise bitwise_not int8 (reads and writes each byte once)"}), flush=True)


def mixed_batch_bench(steps, pool_frames=4096, frames=65536, seed=3):
    """The mixed workload in one persistent launch: 65,536 frames, code
    uniform over N in {256, ..., 32768} x R in {0.5, 0.83, 0.9}, Eb/N0
    uniform 2-5 dB per frame, int8.  The LLRs of pool_frames distinct frames
    are generated; the 65,536 descriptors pick among them."""
    import torch
    from paper_1504_00353_amd import Batch, Code, synth, workloads as W
    codes = [Code(n, k, d, llr="i8", prepare=False) for n, k, d in W.MIXED["codes"]]
    batch = Batch(codes)
    idx = np.arange(pool_frames)
    cidx, ebn0 = synth.frame_params(seed, idx, [list(range(len(codes))), W.MIXED["ebn0_db"]])
    cidx = np.asarray(cidx, np.int32)
    ebn0 = np.asarray(ebn0)
    sizes = np.array([codes[c].n for c in cidx], np.int64)
    poffs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.zeros(int(sizes.sum()), np.int8)
    infos = [None] * pool_frames
    for c, code in enumerate(codes):
        sel = np.flatnonzero(cidx == c)
        if sel.size == 0:
            continue
        bits = synth.info_bits(seed, sel, code.k)
        x = synth.unpack_bits(code.encode(synth.pack_bits(bits)), code.n)
        l = synth.quantize6(synth.awgn_llr(x, synth.noise(seed, sel, code.n), ebn0[sel], code.k / code.n))
        for j, f in enumerate(sel):
            flat[poffs[f]:poffs[f] + code.n] = l[j]
            infos[f] = bits[j]
    pick = np.random.default_rng(seed).integers(0, pool_frames, size=frames)
    code_idx = cidx[pick]
    rb = np.array([codes[c].row_bytes for c in code_idx], np.int64)
    bo = np.concatenate([[0], np.cumsum(rb)[:-1]]).astype(np.int64)
    batch.set_frames(code_idx, poffs[pick], bo)
    llr = torch.from_numpy(flat).cuda()
    out = torch.zeros(int(rb.sum()), dtype=torch.uint8, device="cuda")
    shape = batch.tune(llr, out)
    stream = torch.cuda.current_stream()
    batch.decode(llr, out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        batch.decode(llr, out)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    info_bits = float(sum(codes[c].k for c in code_idx))
    o = out.cpu().numpy()
    fe = 0
    for i in range(frames):
        f = pick[i]
        got = synth.unpack_bits(o[bo[i]:bo[i] + rb[i]][None], codes[code_idx[i]].k)[0]
        fe += int((got != infos[f]).any())
    return {"frames": frames, "distinct_frames": pool_frames, "codes": len(codes),
            "value": round(info_bits * steps / wall / 1e9, 3), "unit": "Gbps",
            "mean_kernel_ms": round(float(np.mean(ms)), 4),
            "launch_ms": {"p50": round(percentile(ms, 50), 4), "p99": round(percentile(ms, 99), 4)},
            "fer": round(fe / frames, 5), "launch_shape": shape}


def serving_bench(seconds=1.0, loads=(0.1, 0.5, 0.9), seed=4, pool=64, capacity_frames=16384, streams=3):
    """Requests of 1..64 frames (code uniform over N in {1024, 4096, 32768} x
    R in {0.5, ..., 0.9}, Eb/N0 uniform 2-5 dB) with Poisson arrivals at
    fractions of the measured batch capacity, replayed by the library's
    native load generator against the continuous-batching server; LLRs and
    results device-resident.  Latency = arrival -> completion seen by the
    server's poll loop."""
    import torch
    from paper_1504_00353_amd import Batch, Code, Server, synth, workloads as W
    codes = [Code(n, k, d, llr="i8", prepare=False) for n, k, d in W.SERVING["codes"]]
    batch = Batch(codes)
    rng = np.random.default_rng(seed)
    # device pool: `pool` channel frames per code, back to back
    offs, parts, o = [], [], 0
    for c, code in enumerate(codes):
        idx = np.arange(pool) + 100000 * c
        bits = synth.info_bits(seed, idx, code.k)
        x = synth.unpack_bits(code.encode(synth.pack_bits(bits)), code.n)
        eb = rng.uniform(*W.SERVING["ebn0_db"], size=pool)
        parts.append(synth.quantize6(synth.awgn_llr(x, synth.noise(seed, idx, code.n), eb, code.k / code.n)).ravel())
        offs.append(o)
        o += pool * code.n
    flat = torch.from_numpy(np.concatenate(parts)).cuda()
    base = flat.data_ptr()
    ns = np.array([c.n for c in codes])
    rbs = np.array([c.row_bytes for c in codes])
    ks = np.array([c.k for c in codes])
    # batch capacity on this mix (frames/s), autotuned
    cidx = rng.integers(0, len(codes), size=capacity_frames).astype(np.int32)
    start = rng.integers(0, pool, size=capacity_frames)
    lo = np.array([offs[c] + s * ns[c] for c, s in zip(cidx, start)], np.int64)
    bo = np.concatenate([[0], np.cumsum(rbs[cidx])[:-1]]).astype(np.int64)
    out = torch.zeros(int(rbs[cidx].sum()), dtype=torch.uint8, device="cuda")
    batch.set_frames(cidx, lo, bo)
    batch.tune(flat, out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(5):
        e0.record()
        batch.decode(flat, out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    cap_fps = capacity_frames / (float(np.median(ts)) / 1e3)
    mean_frames = 32.5
    srv = Server(batch, slots_per_class=8192, streams=streams)
    ring = 8192  # result regions reused round robin (results of finished requests get overwritten)
    out_ring = torch.zeros(ring * 64 * int(rbs.max()), dtype=torch.uint8, device="cuda")
    results = []
    for load in loads:
        rate = load * cap_fps / mean_frames
        n = max(int(rate * seconds), 50)
        arrival = np.cumsum(rng.exponential(1.0 / rate, size=n))
        c = rng.integers(0, len(codes), size=n).astype(np.int32)
        f = rng.integers(1, 65, size=n).astype(np.int32)
        s0 = rng.integers(0, pool - f + 1)
        lp = (base + np.array(offs, np.int64)[c] + s0 * ns[c]).astype(np.uint64)
        bp = (out_ring.data_ptr() + (np.arange(n) % ring) * 64 * int(rbs.max())).astype(np.uint64)
        done = srv.run_trace(arrival, c, f, lp, bp)
        torch.cuda.synchronize()
        lat = (done - arrival) * 1e6
        span = float(done.max() - arrival[0])
        info = float((ks[c] * f).sum())
        results.append({"offered_load": load, "requests": n, "frames": int(f.sum()),
                        "offered_frames_per_s": round(load * cap_fps), "value": round(info / span / 1e9, 3),
                        "unit": "Gbps",
                        "latency_us": {"p50": round(percentile(lat, 50), 1), "p99": round(percentile(lat, 99), 1)},
                        "frame_latency_us": {"p50": round(float(np.percentile(np.repeat(lat, f), 50)), 1),
                                             "p99": round(float(np.percentile(np.repeat(lat, f), 99)), 1)}})
    srv.close()
    return {"batch_capacity_frames_per_s": round(cap_fps), "capacity_launch": batch.launch_shape(),
            "loads": results, "what": "Poisson arrivals, 1..64 frames per request, device-resident LLRs and results"}



def usable_cores():
    """CPU model and the cores this process may use: the affinity mask,
    further limited by a cgroup CPU quota where one is set."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = len(os.sched_getaffinity(0))
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, per = fh.read().split()[:2]
            if q != "max":
                quota = float(q) / float(per)
    except (OSError, ValueError):
        pass
    cores = n if quota is None else max(1, min(n, int(quota)))
    return {"cpu_model": model, "affinity_cpus": n, "cgroup_quota_cpus": quota, "usable": cores}


def gen_frames(code, seed, frame_ids, ebn0_db, llr="i8", threads=8):
    """LLR rows (6-bit int8 or float32) and information bits of the given
    frame indices of one code."""
    from paper_1504_00353_amd import inputs, synth
    l32, info = inputs.channel_frames(code, seed, frame_ids, ebn0_db, threads)
    return (synth.quantize6(l32) if llr == "i8" else l32), info


def timed_launches(fn, reps, stream):
    """Mean and median of reps launches of fn timed with events on the
    launch stream (after one untimed launch)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    return float(np.mean(ms)), float(np.median(ms)), wall


def roof(bytes_per_launch, mean_ms, kernel):
    gbs = bytes_per_launch / (mean_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 5), "kernel": kernel, "bytes_per_launch": int(bytes_per_launch),
            "mean_kernel_ms": round(mean_ms, 4)}


def single_code_config(wl, reps=10, frames=None):
    """One workload of a single code: its frames resident, reps launches of
    the unrolled kernel; information Gb/s, FER and the HBM roofline."""
    import torch
    from paper_1504_00353_amd import Code, synth
    n, k, d = wl["codes"][0]
    frames = frames or wl["frames"]
    code = Code(n, k, d, algo=wl["algo"], llr=wl["llr"], kernel="unrolled")
    llr_np, info = gen_frames(code, wl["seed"], np.arange(frames), wl["ebn0_db"], wl["llr"])
    llr = torch.from_numpy(llr_np).cuda()
    out = torch.empty((frames, code.row_bytes), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    mean_ms, med_ms, wall = timed_launches(lambda: code.decode(llr, out=out), reps, stream)
    fer = float(np.mean((synth.unpack_bits(out.cpu().numpy(), k) != info).any(axis=1)))
    elem = 1 if wl["llr"] == "i8" else 4
    bpf = n * elem + (k + 7) // 8
    res = {"workload": wl["name"], "frames": frames, "algo": wl["algo"], "llr": wl["llr"],
           "value": round(float(k) * frames * reps / wall / 1e9, 3), "unit": "Gbps",
           "ms_per_launch": round(mean_ms, 4), "fer": round(fer, 5), "bytes_per_frame": bpf,
           "roofline": roof(bpf * frames, mean_ms, "polar_unrolled (%s)" % ("int8" if elem == 1 else "float"))}
    code.close()
    return res


def mixed_distinct_config(reps=5, frames=65536, seed=3):
    """The mixed workload with every descriptor on its own LLR row: 65,536
    distinct frames (code uniform over the 15 (N, R) pairs, Eb/N0 uniform
    2-5 dB per frame), about 715 MB of int8 LLRs, one persistent launch."""
    import torch
    from paper_1504_00353_amd import Batch, Code, synth, workloads as W
    codes = [Code(n, k, d, llr="i8", prepare=False) for n, k, d in W.MIXED["codes"]]
    batch = Batch(codes)
    idx = np.arange(frames)
    cidx, ebn0 = synth.frame_params(seed, idx, [list(range(len(codes))), W.MIXED["ebn0_db"]])
    cidx = np.asarray(cidx, np.int32)
    ebn0 = np.asarray(ebn0)
    sizes = np.array([codes[c].n for c in cidx], np.int64)
    rb = np.array([codes[c].row_bytes for c in cidx], np.int64)
    bo = np.concatenate([[0], np.cumsum(rb)[:-1]]).astype(np.int64)
    llr = torch.empty(int(sizes.sum()), dtype=torch.int8, device="cuda")
    offs = np.zeros(frames, np.int64)
    info = [None] * len(codes)
    sels = []
    pos = 0
    for c, code in enumerate(codes):  # each frame its own row; the rows of one code side by side
        sel = np.flatnonzero(cidx == c)
        sels.append(sel)
        if sel.size == 0:
            continue
        l, info[c] = gen_frames(code, seed, sel, ebn0[sel])
        offs[sel] = pos + np.arange(sel.size, dtype=np.int64) * code.n
        llr[pos:pos + l.size] = torch.from_numpy(l.reshape(-1)).cuda()
        pos += l.size
    out = torch.zeros(int(rb.sum()), dtype=torch.uint8, device="cuda")
    batch.set_frames(cidx, offs, bo)
    shape = batch.tune(llr, out)
    stream = torch.cuda.current_stream()
    mean_ms, med_ms, wall = timed_launches(lambda: batch.decode(llr, out), reps, stream)
    o = out.cpu().numpy()
    fe = 0
    for c, sel in enumerate(sels):
        if sel.size:
            rows = np.stack([o[bo[i]:bo[i] + rb[i]] for i in sel])
            fe += int((synth.unpack_bits(rows, codes[c].k) != info[c]).any(axis=1).sum())
    ks = np.array([codes[c].k for c in cidx], np.int64)
    total_bytes = int(sizes.sum() + rb.sum())
    return {"workload": W.MIXED["name"], "frames": frames, "distinct_frames": frames,
            "llr_bytes": int(sizes.sum()), "value": round(float(ks.sum()) * reps / wall / 1e9, 3), "unit": "Gbps",
            "ms_per_launch": round(mean_ms, 4), "fer": round(fe / frames, 5), "launch_shape": shape,
            "roofline": roof(total_bytes, mean_ms, "polar_batch (int8)")}


def stress_config(replays=20, frames=262144, distinct=4096):
    """Throughput stress: 262,144 frames per launch of (32768,29492) and of
    (4096,3686), int8, Eb/N0 4.5 dB, the register/LDS layout picked by the
    autotuner on this launch, the launch captured in a HIP graph and
    replayed; median replay time.  Every frame has its own LLR row (8 GiB
    and 1 GiB); the row contents repeat a set of `distinct` generated
    frames."""
    import torch
    from paper_1504_00353_amd import Code, synth, workloads as W
    wl = W.STRESS
    res = []
    for n, k, d in wl["codes"]:
        code = Code(n, k, d, algo="fastssc", llr="i8", kernel="unrolled", prepare=False)
        nd = min(distinct * (32768 // n), frames)
        l_np, info = gen_frames(code, wl["seed"], np.arange(nd), wl["ebn0_db"])
        src = torch.from_numpy(l_np).cuda()
        llr = src.repeat(frames // nd, 1)
        del src
        out = torch.empty((frames, code.row_bytes), dtype=torch.uint8, device="cuda")
        # the autotuner picks the register/LDS layout on this launch size
        chosen = code.tune_layout(llr, out=out)
        layout = dict(code.layouts()[chosen], index=chosen)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):
                code.decode(llr, out=out, stream=s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            code.decode(llr, out=out, stream=s)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(replays)]
        cur = torch.cuda.current_stream()
        for a, b in ev:
            a.record(cur)
            g.replay()
            b.record(cur)
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in ev]
        med = float(np.median(ms))
        dec = synth.unpack_bits(out[:nd].cpu().numpy(), k)
        same = bool(torch.equal(out[:nd], out[nd:2 * nd])) if frames >= 2 * nd else True
        bpf = n + (k + 7) // 8
        res.append({"code": [n, k], "frames": frames, "distinct_frames": nd, "replays": replays, "layout": layout,
                    "median_replay_ms": round(med, 4), "value": round(float(k) * frames / (med / 1e3) / 1e9, 3),
                    "unit": "Gbps", "fer": round(float(np.mean((dec != info).any(axis=1))), 5),
                    "repeated_rows_equal": same,
                    "roofline": roof(bpf * frames, float(np.mean(ms)), "polar_unrolled (int8), graph replay")})
        del llr, out, g
        torch.cuda.empty_cache()
        code.close()
    return {"workload": wl["name"], "codes": res, "what": "hipGraph-captured launch, median of replays"}


def percentile(v, p):
    return float(np.percentile(np.asarray(v, np.float64), p))


def cpu_baseline(frozen, llr, seconds=10.0):
    """Plain CPU oracle (int8 Fast-SSC) on this host: all-core throughput
    over repeated passes of a frame sample, plus a one-core latency."""
    import oracle
    threads = usable_cores()["usable"]
    sample = llr[:512]
    # one core
    t0 = time.perf_counter()
    oracle.decode(frozen, sample[:32], "fastssc", nthreads=1)
    one_core_us = (time.perf_counter() - t0) / 32 * 1e6
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        oracle.decode(frozen, sample, "fastssc", nthreads=threads)
        done += sample.shape[0]
    dt = time.perf_counter() - t0
    return done, dt, threads, one_core_us


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=4096)
    ap.add_argument("--plain-frames", type=int, default=256)
    ap.add_argument("--latency-runs", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-code batch measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-server measurement")
    ap.add_argument("--serving-seconds", type=float, default=1.0)
    ap.add_argument("--host-steps", type=int, default=10, help="steps of the PCIe-inclusive measurement (0: skip)")
    ap.add_argument("--prewarm-seconds", type=float, default=0.25,
                    help="untimed decode launches before the warmup steps, so the timed steps run at the "
                         "GPU's steady clock (short runs start below it)")
    ap.add_argument("--kernel", choices=["unrolled", "schedule"], default="unrolled",
                    help="generated per-code kernel (default) or the schedule-interpreting one")
    ap.add_argument("--input-copies", type=int, default=4,
                    help="timed steps cycle over this many copies of the frames at distinct addresses "
                         "(default 4: 537 MB, more than the 256 MB Infinity Cache, so no step finds its "
                         "channel rows left in the cache by the step before; 1: the same frames every step)")
    ap.add_argument("--layout", type=int, default=0,
                    help="register/LDS layout of the unrolled kernel (index into Code.layouts(); 0: default rule)")
    ap.add_argument("--only", choices=["sc_f32", "fastssc_f32", "mixed", "stress"], default=None,
                    help="run just this one workload configuration (profiling) and print its object")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workload configurations")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain copy of BYTES bytes (counter calibration)")
    args = ap.parse_args()
    if args.input_copies < 1:
        ap.error("--input-copies must be at least 1")

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py decodes on one GPU only: frames are independent, so more GPUs would "
              "each run this same single-GPU decode on their own share (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration, max(args.steps, 1))
        return

    import torch
    from paper_1504_00353_amd import Code, synth, workloads as W

    config_runs = {"sc_f32": lambda: single_code_config(W.SC_1024),
                   "fastssc_f32": lambda: single_code_config(W.FSSC_32K_F32),
                   "mixed": mixed_distinct_config, "stress": stress_config}
    if args.only:
        print(json.dumps({args.only: config_runs[args.only]()}), flush=True)
        return

    n, k, design, ebn0 = 32768, 29492, 4.0, 4.0
    frames = args.frames
    code = Code(n, k, design, algo="fastssc", llr="i8", kernel=args.kernel,
                layout=args.layout if args.kernel == "unrolled" else 0)
    frozen, info, llr_np = make_inputs(code, seed=2, frames=frames, ebn0_db=ebn0)
    dev = torch.device("cuda", 0)
    llr = torch.from_numpy(llr_np).to(dev)
    # --input-copies C: the timed steps cycle over C copies of the frames at
    # distinct device addresses (C x 134 MB); with the default 4 (537 MB) a
    # step's channel rows are not left in the 256 MB Infinity Cache by the
    # steps before it
    llr_steps = [llr] + [llr.clone() for _ in range(args.input_copies - 1)]
    out = torch.empty((frames, code.row_bytes), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    t_pre = time.perf_counter()
    while time.perf_counter() - t_pre < args.prewarm_seconds:
        for i in range(16):
            code.decode(llr_steps[i % len(llr_steps)], out=out)
        torch.cuda.synchronize()
    for i in range(args.warmup):
        code.decode(llr_steps[i % len(llr_steps)], out=out)
    torch.cuda.synchronize()

    # timed region: K batched launches, events on the launch stream
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        code.decode(llr_steps[i % len(llr_steps)], out=out)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_per_step = wall * 1e3 / args.steps
    info_bits = float(k) * frames * args.steps
    gbps = info_bits / wall / 1e9

    decoded = synth.unpack_bits(out.cpu().numpy(), k)
    fer = float(np.mean((decoded != info).any(axis=1)))

    # batched frame latency: submit -> completion of a launch, one at a time
    lat = []
    for _ in range(args.latency_runs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        code.decode(llr, out=out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e6)

    # plain: one launch per frame, back to back, same frames
    pf = min(args.plain_frames, frames)
    plain = None
    if pf > 0:
        outs1 = torch.empty((pf, code.row_bytes), dtype=torch.uint8, device=dev)
        for i in range(min(3, pf)):
            code.decode(llr[i:i + 1], out=outs1[i:i + 1])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(pf):
            code.decode(llr[i:i + 1], out=outs1[i:i + 1])
        torch.cuda.synchronize()
        plain_wall = time.perf_counter() - t
        plain_gbps = float(k) * pf / plain_wall / 1e9
        assert torch.equal(outs1, out[:pf]), "plain and batched decodes differ"
        plat = []
        for i in range(min(pf, 100)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            code.decode(llr[i:i + 1], out=outs1[i:i + 1])
            torch.cuda.synchronize()
            plat.append((time.perf_counter() - t) * 1e6)
        plain = {"value": round(plain_gbps, 4), "unit": "Gbps", "frames": pf,
                 "latency_us": {"p50": round(percentile(plat, 50), 2), "p99": round(percentile(plat, 99), 2)},
                 "bits_equal_batched": True}
        if args.kernel == "unrolled":
            # the same single-frame launches with the register/LDS layout the
            # autotuner picks for one frame per launch (latency, not occupancy)
            lc = Code(n, k, design, algo="fastssc", llr="i8", kernel="unrolled", prepare=False)
            chosen = lc.tune_layout(llr[:1])
            tl = []
            for i in range(min(pf, 100)):
                torch.cuda.synchronize()
                t = time.perf_counter()
                lc.decode(llr[i:i + 1], out=outs1[i:i + 1])
                torch.cuda.synchronize()
                tl.append((time.perf_counter() - t) * 1e6)
            assert torch.equal(outs1[:min(pf, 100)], out[:min(pf, 100)]), "latency-tuned decode differs"
            plain["latency_tuned"] = {"layout": dict(lc.layouts()[chosen], index=chosen),
                                      "latency_us": {"p50": round(percentile(tl, 50), 2),
                                                     "p99": round(percentile(tl, 99), 2)},
                                      "what": "one frame per launch, layout tuned on one frame"}
            lc.close()

    # host-inclusive: LLRs from pinned host memory, bits back to it (PCIe), per step
    host = None
    if args.host_steps > 0:
        h_llr = torch.from_numpy(llr_np).pin_memory()
        h_out = torch.empty((frames, code.row_bytes), dtype=torch.uint8).pin_memory()
        d_llr = torch.empty_like(llr)
        for _ in range(2):
            d_llr.copy_(h_llr, non_blocking=True)
            code.decode(d_llr, out=out)
            h_out.copy_(out, non_blocking=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.host_steps):
            d_llr.copy_(h_llr, non_blocking=True)
            code.decode(d_llr, out=out)
            h_out.copy_(out, non_blocking=True)
        torch.cuda.synchronize()
        hw = (time.perf_counter() - t) / args.host_steps
        assert torch.equal(h_out, out.cpu()), "host-inclusive decode differs"
        host = {"value": round(float(k) * frames / hw / 1e9, 3), "unit": "Gbps", "ms_per_step": round(hw * 1e3, 4),
                "what": "pinned host LLRs -> device, decode, bits -> pinned host, one stream (PCIe-inclusive; "
                        "not the headline value)"}
        del h_llr, h_out, d_llr

    bytes_per_frame = n * 1 + (k + 7) // 8
    mean_kernel_s = float(np.mean(kernel_ms)) / 1e3
    achieved = bytes_per_frame * frames / mean_kernel_s / 1e9
    traffic = measured_traffic(frames, args.kernel)
    copy_gbs = copy_bandwidth()

    result = {
        "metric": METRIC,
        "value": round(gbps, 3),
        "unit": "Gbps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "prewarm_s": args.prewarm_seconds,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic: uniform info bits, BPSK over AWGN at 4.0 dB, 6-bit LLRs in int8",
        "config": {"workload": "fastssc_32768_29492_i8", "N": n, "K": k, "design_ebn0_db": design,
                   "ebn0_db": ebn0, "frames_per_step": frames, "algo": "fast-ssc",
                   "kernel": args.kernel, "layout": dict(code.layouts()[args.layout], index=args.layout)
                   if args.kernel == "unrolled" else None, "input_copies": args.input_copies},
        "latency_us": None if not lat else
        {"p50": round(percentile(lat, 50), 2), "p99": round(percentile(lat, 99), 2),
         "what": "batched launch of %d frames, submit to completion" % frames},
        "plain": plain,
        "host_inclusive": host,
        "fer": fer,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": None if traffic is None else round(traffic),
                     "kernel": "polar_unrolled (int8)" if args.kernel == "unrolled" else "decode_kernel<int8>",
                     "bytes_per_frame": bytes_per_frame,
                     "mean_kernel_ms": round(mean_kernel_s * 1e3, 4),
                     "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 5)},
        "valu": valu_view(frames, args.kernel, mean_kernel_s * 1e3),
    }
    if not args.no_mixed and args.kernel == "unrolled":
        result["mixed_batch"] = mixed_batch_bench(max(args.steps // 2, 3))
    if not args.no_serving and args.kernel == "unrolled":
        result["serving"] = serving_bench(args.serving_seconds)
    if not args.no_configs and args.kernel == "unrolled":
        result["configs"] = {name: run() for name, run in config_runs.items()}
    if not args.no_cpu:
        done, dt, threads, one_core_us = cpu_baseline(frozen, llr_np, args.cpu_seconds)
        result["cpu_baseline"] = {"value": round(done * k / dt / 1e9, 5), "unit": "Gbps", "cores": threads,
                                  "kind": "oracle", "host": usable_cores(),
                                  "sample": "%d frames (512 distinct, repeated) of this workload, int8 Fast-SSC, "
                                            "%.1f s" % (done, dt),
                                  "one_core_latency_us": round(one_core_us, 1)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
