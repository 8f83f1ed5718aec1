"""Algorithm and quantisation study on one MI355X (the shape of the paper's
Table 4 and Fig. 5, on this hardware): decoding speed of plain SC vs
Fast-SSC and of the schedule vs the unrolled kernel on the same codes, and
frame-error rates of 8-bit fixed point vs float32 LLRs.

    python -m paper_1504_00353_amd.study [--frames F] [--fer-frames M]

Frames are synthetic: uniform information bits, BPSK over AWGN, generated
on the GPU with torch (random codewords, encoded with the butterfly of
Sec. II-A in torch ops); LLRs as in the benchmark (6-bit quantiser for
int8).  Prints markdown tables.
"""
import argparse
import time

import numpy as np


def encode_torch(u):
    """x = u G_N over the last axis (x[i] ^= x[i + h] for bit h of i clear)."""
    x = u.clone()
    n = x.shape[1]
    h = 1
    while h < n:
        v = x.view(x.shape[0], n // (2 * h), 2, h)
        v[:, :, 0, :] ^= v[:, :, 1, :]
        h *= 2
    return x


def channel_frames(code, frames, ebn0_db, llr, gen):
    import torch
    frozen = torch.from_numpy(code.frozen().astype(bool)).cuda()
    info = torch.randint(0, 2, (frames, code.k), generator=gen, device="cuda", dtype=torch.uint8)
    u = torch.zeros((frames, code.n), dtype=torch.uint8, device="cuda")
    u[:, ~frozen] = info
    x = encode_torch(u)
    rate = code.k / code.n
    sigma = (1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))) ** 0.5
    y = (1.0 - 2.0 * x.double()) + sigma * torch.randn(x.shape, generator=gen, device="cuda", dtype=torch.float64)
    l = (2.0 * y / sigma ** 2).float()
    if llr == "i8":
        q = torch.sign(2.0 * l) * torch.floor(torch.abs(2.0 * l) + 0.5)
        l = torch.clamp(q, -31, 31).to(torch.int8)
    return info, l.contiguous()


def unpack(out, k):
    import torch
    bits = torch.stack([(out >> b) & 1 for b in range(8)], dim=2).reshape(out.shape[0], -1)
    return bits[:, :k]


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
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2015)

    print("## Decoding speed (int8, %d frames per launch; latency = one frame per launch, kernel time)\n" % args.frames)
    print("| code | algorithm | kernel | info Gb/s | latency us | ops |")
    print("|---|---|---|---|---|---|")
    for n, k, d in ((1024, 512, 2.5), (2048, 1707, 4.0), (32768, 29492, 4.0)):
        for algo in ("sc", "fastssc"):
            for kernel in ("schedule", "unrolled"):
                if algo == "sc" and n > 2048:
                    continue  # plain SC schedules of N = 32768 are ~65,000 ops
                code = Code(n, k, d, algo=algo, llr="i8", kernel=kernel)
                _, l = channel_frames(code, args.frames, d, "i8", gen)
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
                _, l = channel_frames(code, args.frames, d, "i8", gen)
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
            fer = {}
            for llr, code in codes.items():
                errs, done = 0, 0
                g2 = torch.Generator(device="cuda")
                g2.manual_seed(int(eb * 1000) + n)
                chunk = max(1, min(args.fer_frames, (1 << 28) // (n * 8)))
                while done < args.fer_frames:
                    m = min(chunk, args.fer_frames - done)
                    info, l = channel_frames(code, m, eb, llr, g2)
                    out = code.decode(l)
                    errs += int((unpack(out, k) != info).any(dim=1).sum())
                    done += m
                fer[llr] = errs / done
            print("| (%d,%d) | %.2f | %.2e | %.2e |" % (n, k, eb, fer["i8"], fer["f32"]))


if __name__ == "__main__":
    main()
