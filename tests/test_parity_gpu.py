"""GPU decode == oracle, element by element.

int8: decoded bits and the leaf-LLR trace are bit-exact against the 8-bit
saturating oracle.  float32: bits and trace are bit-exact against the
float32 oracle (same operations in the same order); the float64 side of
the float contract is in test_float_contract_gpu.py.
"""
import numpy as np
import pytest

import oracle
from frames import make_frames
from paper_1504_00353_amd import Code, synth, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def gpu_decode(code, llr, trace=False):
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    if trace:
        out, tr = code.decode_trace(t)
        torch.cuda.synchronize()
        return out.cpu().numpy(), tr.cpu().numpy()
    out = code.decode(t)
    torch.cuda.synchronize()
    return out.cpu().numpy(), None


def packed_info(frozen, u_hat):
    return synth.pack_bits(u_hat[:, np.asarray(frozen) == 0])


def check_parity(code, frozen, llr, algo, trace=True, label=""):
    u, _, t = oracle.decode(frozen, llr, algo, trace=trace, nthreads=8)
    bits, tr = gpu_decode(code, llr, trace=trace)
    expect = packed_info(frozen, u)
    bad = np.flatnonzero((bits != expect).any(axis=1))
    assert bad.size == 0, "%s: %d frames differ, first %s" % (label, bad.size, bad[:5])
    if trace:
        diff = np.flatnonzero((tr != t).any(axis=1))
        assert diff.size == 0, "%s: trace differs in %d frames" % (label, diff.size)
    return u


def random_llrs(rng, frames, n, kind):
    if kind == "i8":
        return rng.integers(-128, 128, size=(frames, n)).astype(np.int8)
    if kind == "i8small":  # many zeros and ties
        return rng.integers(-3, 4, size=(frames, n)).astype(np.int8)
    return rng.normal(0.3, 3.0, size=(frames, n)).astype(np.float32)


def random_mask(n, rng, p):
    m = (rng.random(n) < p).astype(np.uint8)
    if m.all():
        m[rng.integers(0, n)] = 0
    return m


@pytest.mark.parametrize("algo", ["fastssc", "sc"])
@pytest.mark.parametrize("kind", ["i8", "i8small", "f32"])
def test_listing1_code(algo, kind):
    fr = np.array([1, 1, 0, 0, 1, 0, 0, 0], np.uint8)
    code = Code(frozen=fr, algo=algo, llr="f32" if kind == "f32" else "i8")
    rng = np.random.default_rng(1)
    check_parity(code, fr, random_llrs(rng, 333, 8, kind), algo, label="listing1")


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 8192])
@pytest.mark.parametrize("algo", ["fastssc", "sc"])
@pytest.mark.parametrize("kind", ["i8", "i8small", "f32"])
def test_random_masks(n, algo, kind):
    """Arbitrary frozen sets exercise every node kind, including a Rate-0
    right child under a non-frozen left child."""
    if algo == "sc" and n > 2048:
        pytest.skip("plain SC covered up to N = 2048 here")
    rng = np.random.default_rng(n * 7 + len(kind) + (3 if algo == "sc" else 0))
    for p in (0.1, 0.5, 0.9):
        fr = random_mask(n, rng, p)
        code = Code(frozen=fr, algo=algo, llr="f32" if kind == "f32" else "i8")
        check_parity(code, fr, random_llrs(rng, 67, n, kind), algo, label="mask n=%d p=%.1f" % (n, p))


CODES = [(64, 32, 2.5), (256, 128, 2.5), (256, 230, 4.0), (1024, 512, 2.5), (1024, 922, 4.0),
         (4096, 3400, 4.0), (4096, 3686, 4.0), (16384, 14746, 4.0), (32768, 27197, 4.0), (32768, 29492, 4.0)]


@pytest.mark.parametrize("n,k,d", CODES)
@pytest.mark.parametrize("llr", ["i8", "f32"])
def test_constructed_codes_channel_frames(n, k, d, llr):
    code = Code(n, k, d, llr=llr)
    fr = code.frozen()
    frames = 130 if n <= 4096 else 40
    _, _, l = make_frames(fr, 77, frames, d - 0.5, llr)
    check_parity(code, fr, l, "fastssc", label="(%d,%d) %s" % (n, k, llr))


@pytest.mark.parametrize("kernel", ["schedule", "unrolled"])
def test_sc_1024_512_float32_full_workload(kernel):
    """(1024,512), plain SC, float32, 10,000 frames at 2.5 dB."""
    code = Code(1024, 512, 2.5, algo="sc", llr="f32", kernel=kernel)
    fr = code.frozen()
    _, _, l = make_frames(fr, 1, 10000, 2.5, "f32")
    check_parity(code, fr, l, "sc", label="sc-1024")


def test_schedule_kernel_lds_limit_independent_of_prepare_order():
    """A (32768,29492) float code on the schedule kernel (132 KB of LDS per
    frame) prepared before a (1024,512) one still decodes afterwards: the
    kernel's dynamic-LDS limit does not follow the last prepared code."""
    big = Code(32768, 29492, 4.0, llr="f32", kernel="schedule")
    small = Code(1024, 512, 2.5, llr="f32", kernel="schedule")
    fr = big.frozen()
    _, _, l = make_frames(fr, 5, 8, 4.0, "f32")
    check_parity(big, fr, l, "fastssc", trace=False, label="32k f32 after 1k")
    frs = small.frozen()
    _, _, ls = make_frames(frs, 6, 8, 2.5, "f32")
    check_parity(small, frs, ls, "fastssc", trace=False, label="1k f32")


@pytest.mark.parametrize("kernel", ["schedule", "unrolled"])
@pytest.mark.parametrize("llr", ["i8", "f32"])
def test_fastssc_32768_29492_full_workload(llr, kernel):
    """(32768,29492) Fast-SSC, 4,096 frames at 4.0 dB, every frame."""
    code = Code(32768, 29492, 4.0, llr=llr, kernel=kernel)
    fr = code.frozen()
    _, _, l = make_frames(fr, 2, 4096, 4.0, llr)
    check_parity(code, fr, l, "fastssc", trace=True, label="32k " + llr)


@pytest.mark.parametrize("kernel", ["schedule", "unrolled"])
@pytest.mark.parametrize("n,k", [(4096, 3686), (32768, 29492)])
def test_stress_launch_262144_frames_sampled(n, k, kernel):
    """One launch of 262,144 frames (a pool of 2,048 distinct frames tiled);
    sampled frames against the oracle, and every tile identical."""
    code = Code(n, k, 4.0, llr="i8", kernel=kernel)
    fr = code.frozen()
    pool = 2048
    _, _, l = make_frames(fr, 5, pool, 4.5, "i8")
    u, _, _ = oracle.decode(fr, l, "fastssc", nthreads=8)
    expect = packed_info(fr, u)
    frames = 262144
    dev = torch.from_numpy(l).cuda().repeat(frames // pool, 1)
    out = code.decode(dev)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    rng = np.random.default_rng(0)
    idx = rng.choice(frames, size=4096, replace=False)
    assert np.array_equal(out[idx], expect[idx % pool])
    assert (out.reshape(frames // pool, pool, -1) == expect[None]).all()


@pytest.mark.parametrize("n,k", [(4096, 3686), (32768, 29492)])
def test_stress_launch_graph_replays(n, k):
    """The stress workload as a captured HIP graph of the unrolled decode
    (262,144 frames per launch), replayed with eager work and
    synchronisation in between: every replay equals the oracle on sampled
    frames and tile by tile."""
    code = Code(n, k, 4.0, llr="i8", kernel="unrolled")
    fr = code.frozen()
    pool = 2048
    _, _, l = make_frames(fr, 6, pool, 4.5, "i8")
    u, _, _ = oracle.decode(fr, l, "fastssc", nthreads=8)
    expect = packed_info(fr, u)
    frames = 262144
    dev = torch.from_numpy(l).cuda().repeat(frames // pool, 1)
    out = torch.zeros((frames, code.row_bytes), dtype=torch.uint8, device="cuda")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        code.decode(dev, out=out, stream=s)  # eager launch before capture
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            code.decode(dev, out=out, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    rng = np.random.default_rng(1)
    for rep in range(3):
        out.fill_(0x5A)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        idx = rng.choice(frames, size=2048, replace=False)
        assert np.array_equal(o[idx], expect[idx % pool]), "replay %d" % rep
        assert (o.reshape(frames // pool, pool, -1) == expect[None]).all(), "replay %d" % rep
        del junk


@pytest.mark.parametrize("n,k", [(64, 64), (4096, 4096), (64, 1), (32768, 1), (64, 63), (8192, 8191), (2, 1), (2, 2)])
@pytest.mark.parametrize("kind", ["i8", "f32"])
def test_degenerate_codes(n, k, kind):
    """Root is a Rate-1, repetition or SPC node; N = 2."""
    code = Code(n, k, 3.0, llr="f32" if kind == "f32" else "i8")
    fr = code.frozen()
    rng = np.random.default_rng(n + k)
    check_parity(code, fr, random_llrs(rng, 65, n, kind), "fastssc", label="(%d,%d)" % (n, k))


def test_extreme_and_zero_llrs():
    code = Code(1024, 922, 4.0, llr="i8")
    fr = code.frozen()
    rng = np.random.default_rng(3)
    l = np.zeros((8, 1024), np.int8)
    l[1] = 127
    l[2] = -128
    l[3] = -127
    l[4] = rng.choice([-128, 127], size=1024)
    l[5] = rng.choice([-128, 0, 127], size=1024)
    l[6] = rng.choice([-1, 0, 1], size=1024)
    l[7] = rng.integers(-128, 128, size=1024)
    check_parity(code, fr, l, "fastssc", label="extremes")


def test_noiseless_recovery_on_gpu():
    for (n, k, d) in [(1024, 512, 2.5), (32768, 29492, 4.0)]:
        for llr in ("i8", "f32"):
            code = Code(n, k, d, llr=llr)
            fr = code.frozen()
            bits = synth.info_bits(8, np.arange(16), k)
            x = oracle.encode(synth.scatter_info(bits, fr))
            sign = 1 - 2 * x.astype(np.int32)
            l = (sign * 31).astype(np.int8) if llr == "i8" else (sign * 8.0).astype(np.float32)
            out, _ = gpu_decode(code, l)
            assert np.array_equal(out, synth.pack_bits(bits))


def test_zero_frames_is_noop():
    code = Code(256, 128, 2.5)
    t = torch.zeros((0, 256), dtype=torch.int8, device="cuda")
    out = code.decode(t)
    torch.cuda.synchronize()
    assert out.shape == (0, 16)


def _unrolled_specs():
    from paper_1504_00353_amd import build
    return [t for t in build._kernel_specs() if t[1] != "mask" and len(t) == 5]


@pytest.mark.parametrize("name", workloads.UNROLLED_MASKS_F32)
def test_unrolled_kernel_masks_float(name):
    """Float LLRs on frozen sets with leaves at the top stages: the float
    generated kernels (virtual top stage where the root's children are
    inner) against the float32 oracle (bits and trace) and the schedule
    kernel."""
    n, fr = workloads.UNROLLED_MASKS[name]
    fr = np.asarray(fr, np.uint8)
    code = Code(frozen=fr, llr="f32", kernel="unrolled")
    ref = Code(frozen=fr, llr="f32", kernel="schedule")
    rng = np.random.default_rng(n + 3 * len(name))
    l = random_llrs(rng, 24, n, "f32")
    check_parity(code, fr, l, "fastssc", label="unrolled float mask %s" % name)
    b1, _ = gpu_decode(code, l)
    b0, _ = gpu_decode(ref, l)
    assert np.array_equal(b0, b1)


@pytest.mark.parametrize("name", sorted(workloads.UNROLLED_MASKS))
@pytest.mark.parametrize("kind", ["i8", "i8small"])
def test_unrolled_kernel_masks(name, kind):
    """Frozen sets with Rate-0, Rate-1, repetition and SPC nodes at the
    widest stages (held in registers by the generated int8 kernels of
    N >= 16384): bits and trace against the oracle, bits against the
    schedule kernel."""
    n, fr = workloads.UNROLLED_MASKS[name]
    fr = np.asarray(fr, np.uint8)
    code = Code(frozen=fr, kernel="unrolled")
    ref = Code(frozen=fr, kernel="schedule")
    rng = np.random.default_rng(n + len(name))
    l = random_llrs(rng, 48, n, kind)
    check_parity(code, fr, l, "fastssc", label="unrolled mask %s" % name)
    b1, _ = gpu_decode(code, l)
    b0, _ = gpu_decode(ref, l)
    assert np.array_equal(b0, b1)


@pytest.mark.parametrize("spec", _unrolled_specs(), ids=lambda t: "%d_%d_%s_%s" % (t[0], t[1], t[3], t[4]))
def test_unrolled_kernel_codes(spec):
    """Every code with a prebuilt unrolled kernel: bits and leaf-LLR trace
    against the oracle, and bits identical to the schedule kernel, on
    channel frames plus extreme and tied LLRs."""
    n, k, d, algo, llr = spec
    code = Code(n, k, d, algo=algo, llr=llr, kernel="unrolled")
    ref = Code(n, k, d, algo=algo, llr=llr, kernel="schedule")
    fr = code.frozen()
    frames = 96 if n >= 16384 else 300
    _, _, l = make_frames(fr, 11, frames, d, llr)
    rng = np.random.default_rng(n + k)
    kind = "f32" if llr == "f32" else "i8"
    l = np.concatenate([l, random_llrs(rng, 16, n, kind)] + ([random_llrs(rng, 16, n, "i8small")] if kind == "i8" else []))
    check_parity(code, fr, l, algo, label="unrolled %s" % (spec,))
    b1, _ = gpu_decode(code, l)
    b0, _ = gpu_decode(ref, l)
    assert np.array_equal(b0, b1)


@pytest.mark.parametrize("frames", [1, 3, 4, 5, 65])
def test_unrolled_ragged_frame_counts(frames):
    """Frame counts that leave the last block partly empty."""
    code = Code(1024, 512, 2.5, llr="i8", kernel="unrolled")
    fr = code.frozen()
    _, _, l = make_frames(fr, 12, frames, 2.5, "i8")
    check_parity(code, fr, l, "fastssc", label="unrolled ragged %d" % frames)


@pytest.mark.parametrize("spec", workloads.UNROLLED_UNFUSED, ids=lambda t: "%d_%d_%s" % (t[0], t[1], t[4]))
@pytest.mark.parametrize("kernel", ["schedule", "unrolled"])
def test_fused_nodes_identical_to_separate_ops(spec, kernel):
    """The fused leaf-pair nodes (P_01, 0SPC, RepSPC, Rep-R1) compute what the
    separate f / leaf / g / leaf / combine ops compute: bits and trace equal
    with the fusion on and off, and equal to the oracle."""
    n, k, d, algo, llr = spec
    on = Code(n, k, d, algo=algo, llr=llr, kernel=kernel, fused=True)
    off = Code(n, k, d, algo=algo, llr=llr, kernel=kernel, fused=False)
    fr = on.frozen()
    _, _, l = make_frames(fr, 21, 64 if n >= 16384 else 256, d, llr)
    rng = np.random.default_rng(n + 5)
    extra = [random_llrs(rng, 16, n, "f32" if llr == "f32" else "i8")]
    if llr == "i8":
        extra.append(random_llrs(rng, 16, n, "i8small"))
    l = np.concatenate([l] + extra)
    check_parity(on, fr, l, algo, label="fused %s %s" % (kernel, spec))
    b1, t1 = gpu_decode(on, l, trace=True)
    b0, t0 = gpu_decode(off, l, trace=True)
    assert np.array_equal(b0, b1)
    assert np.array_equal(t0.view(np.uint8), t1.view(np.uint8))


@pytest.mark.parametrize("llr", ["i8", "i8small", "f32"])
@pytest.mark.parametrize("fused", [True, False])
def test_leaf_pair_mask_schedule_kernel(llr, fused):
    """Every leaf-pair pattern at every child size (the fused ops' node
    sizes 4..64), through the schedule kernel, fused and not."""
    n, fr = workloads.UNROLLED_MASKS["m2k_leaf_pairs"]
    fr = np.asarray(fr, np.uint8)
    code = Code(frozen=fr, llr="f32" if llr == "f32" else "i8", fused=fused)
    rng = np.random.default_rng(77 + len(llr))
    check_parity(code, fr, random_llrs(rng, 200, n, llr), "fastssc", label="pairs %s %s" % (llr, fused))


@pytest.mark.parametrize("spec", workloads.UNROLLED_LAYOUTS, ids=lambda t: "%d_%d_%s" % (t[0], t[1], t[4]))
def test_every_layout_matches_oracle(spec):
    """Each register/LDS layout the autotuner can pick decodes the same bits
    and leaf LLRs as the oracle; the tuner leaves the code prepared with one
    of them and decoding the same bits."""
    n, k, d, algo, llr = spec
    probe = Code(n, k, d, algo=algo, llr=llr, kernel="unrolled", prepare=False)
    count = len(probe.layouts())
    fr = probe.frozen()
    _, _, l = make_frames(fr, 21, 64 if n >= 16384 else 200, d, llr)
    rng = np.random.default_rng(n)
    l = np.concatenate([l, random_llrs(rng, 8, n, "f32" if llr == "f32" else "i8")])
    bits = []
    for i in range(count):
        code = Code(n, k, d, algo=algo, llr=llr, kernel="unrolled", layout=i)
        check_parity(code, fr, l, algo, label="layout %d of %s" % (i, spec))
        bits.append(gpu_decode(code, l)[0])
        code.close()
    tuned = Code(n, k, d, algo=algo, llr=llr, kernel="unrolled", prepare=False)
    t = torch.from_numpy(np.ascontiguousarray(l)).cuda()
    chosen = tuned.tune_layout(t)
    assert 0 <= chosen < count
    b, _ = gpu_decode(tuned, l)
    assert np.array_equal(b, bits[0])
