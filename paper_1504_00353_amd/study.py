"""Algorithm and quantisation study on one MI355X (the shape of the paper's
Table 4 and Fig. 5, on this hardware): decoding speed of plain SC vs
Fast-SSC and of the schedule vs the unrolled kernel on the same codes, and
frame-error rates of 8-bit fixed point vs float32 LLRs.

    python -m paper_1504_00353_amd.study [--frames F] [--fer-frames M]

Frames are synthetic and generated on the host: seeded uniform
information bits, the codeword from the library's encoder (polar_encode),
BPSK over AWGN (``inputs.channel_frames``); LLRs as in the benchmark (6-bit
quantiser for int8; the int8 and float32 FER columns decode the same
channel samples).  Prints markdown tables.
"""
import argparse
import os

import numpy as np

from . import inputs, synth

SEED = 2015
THREADS = min(16, len(os.sched_getaffinity(0)))


def channel_frames(code, frames, ebn0_db, llr, first=0, seed=SEED):
    """(information bits, LLR tensor on the GPU) of frames first ..
    first + frames - 1 of the study's stream for this code."""
    import torch
    l32, info = inputs.channel_frames(code, seed, np.arange(first, first + frames), ebn0_db, THREADS)
    l = synth.quantize6(l32) if llr == "i8" else l32
    return info, torch.from_numpy(l).cuda()


def frame_errors(out, info):
    return int((synth.unpack_bits(out.cpu().numpy(), info.shape[1]) != info).any(axis=1).sum())


def speed(code, l, prewarm_s=0.25):
    import time
    import torch
    code.decode(l)
    torch.cuda.synchronize()
    t0 = time.perf_counter()  # untimed launches first: the GPU clock ramps up
    while time.perf_counter() - t0 < prewarm_s:
        code.decode(l)
        torch.cuda.synchronize()
    t = []
    for _ in range(25):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        code.decode(l)
        e1.record()
        torch.cuda.synchronize()
        t.append(e0.elapsed_time(e1))
    batch_ms = float(np.median(t))
    one = []
    for i in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        code.decode(l[i:i + 1])
        e1.record()
        torch.cuda.synchronize()
        one.append(e0.elapsed_time(e1))
    return code.k * l.shape[0] / batch_ms / 1e6, float(np.median(one)) * 1e3


def main():
    import torch
    from paper_1504_00353_amd import Code
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=4096)
    ap.add_argument("--fer-frames", type=int, default=100000)
    args = ap.parse_args()

    print("## Decoding speed (int8, %d frames per launch; latency = one frame per launch, kernel time)\n" % args.frames)
    print("| code | algorithm | kernel | info Gb/s | latency us | ops |")
    print("|---|---|---|---|---|---|")
    for n, k, d in ((1024, 512, 2.5), (2048, 1707, 4.0), (32768, 29492, 4.0)):
        for algo in ("sc", "fastssc"):
            for kernel in ("schedule", "unrolled"):
                if algo == "sc" and n > 2048:
                    continue  # plain SC schedules of N = 32768 are ~65,000 ops
                code = Code(n, k, d, algo=algo, llr="i8", kernel=kernel)
                _, l = channel_frames(code, args.frames, d, "i8")
                gbps, lat = speed(code, l)
                print("| (%d,%d) | %s | %s | %.1f | %.1f | %d |" % (n, k, "SC" if algo == "sc" else "Fast-SSC", kernel,
                                                                     gbps, lat, len(code.schedule())))
                code.close()

    print("\n## Fused leaf-pair nodes (P_01, 0SPC, RepSPC, Rep-R1) on vs off, int8 Fast-SSC, %d frames\n" % args.frames)
    print("| code | kernel | fused | device ops | info Gb/s | latency us |")
    print("|---|---|---|---|---|---|")
    for n, k, d in ((1024, 512, 2.5), (4096, 3686, 4.0), (32768, 29492, 4.0)):
        for kernel in ("schedule", "unrolled"):
            for fused in (False, True):
                code = Code(n, k, d, llr="i8", kernel=kernel, fused=fused)
                _, l = channel_frames(code, args.frames, d, "i8")
                gbps, lat = speed(code, l)
                print("| (%d,%d) | %s | %s | %d | %.1f | %.1f |" % (n, k, kernel, "yes" if fused else "no",
                                                                   len(code.device_schedule()), gbps, lat))
                code.close()

    print("\n## Frame-error rate, Fast-SSC, int8 (6-bit) vs float32 LLRs, %d frames per point\n" % args.fer_frames)
    print("| code | Eb/N0 dB | FER int8 | FER float32 |")
    print("|---|---|---|---|")
    for n, k, d, pts in ((1024, 512, 2.5, (1.5, 2.0, 2.5, 3.0)), (2048, 1707, 4.0, (3.5, 4.0, 4.5)),
                         (32768, 29492, 4.0, (4.0, 4.25, 4.5))):
        codes = {llr: Code(n, k, d, llr=llr) for llr in ("i8", "f32")}
        for eb in pts:
            errs = {"i8": 0, "f32": 0}
            chunk = max(1, min(args.fer_frames, (1 << 27) // n))
            first = 0
            while first < args.fer_frames:
                m = min(chunk, args.fer_frames - first)
                # one set of channel samples, decoded from float32 and from 6-bit int8 LLRs
                l32, info = inputs.channel_frames(codes["f32"], SEED + int(eb * 1000), np.arange(first, first + m),
                                                  eb, THREADS)
                for llr, code in codes.items():
                    l = synth.quantize6(l32) if llr == "i8" else l32
                    errs[llr] += frame_errors(code.decode(torch.from_numpy(l).cuda()), info)
                first += m
            fer = {llr: e / args.fer_frames for llr, e in errs.items()}
            print("| (%d,%d) | %.2f | %.2e | %.2e |" % (n, k, eb, fer["i8"], fer["f32"]))


if __name__ == "__main__":
    main()
