"""Seeded synthetic channel inputs for polar decoding workloads.

This module draws random numbers and shapes them into channel inputs; it
holds no encoding or decoding arithmetic, so both the GPU path and the CPU
oracle can consume exactly the same bytes from it.  The codeword x = u G_N
is computed by the caller (the oracle's encoder in tests, the library's
encoder in the benchmark).

Channel model (the simulation chain of Sec. III "Methodology"): BPSK
(0 -> +1, 1 -> -1) over AWGN with sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)),
LLR = 2 y / sigma^2 computed in float64 and rounded once to float32.  The
6-bit quantiser maps an LLR to clamp(round_half_away(2 LLR), -31, 31) and
stores it as int8 (one fractional bit, symmetric range).

Random streams are counter based: numpy's Philox4x64 keyed by
(seed, stream id) with the frame index in the counter, so frame f of a
workload is the same whatever batch it is drawn in.
"""
import numpy as np

_INFO_STREAM = 1
_NOISE_STREAM = 2
_PARAM_STREAM = 3


def _rng(seed, stream, frame):
    key = (int(seed) << 8) | int(stream)
    bitgen = np.random.Philox(key=key, counter=[0, int(frame), 0, 0])
    return np.random.Generator(bitgen)


def info_bits(seed, frames, k):
    """Uniform i.i.d. information bits, [len(frames), k] of 0/1 bytes."""
    frames = np.atleast_1d(frames)
    out = np.empty((frames.shape[0], k), np.uint8)
    for j, f in enumerate(frames):
        out[j] = _rng(seed, _INFO_STREAM, f).integers(0, 2, size=k, dtype=np.uint8)
    return out


def noise(seed, frames, n):
    """Standard normal samples, [len(frames), n] float64."""
    frames = np.atleast_1d(frames)
    out = np.empty((frames.shape[0], n), np.float64)
    for j, f in enumerate(frames):
        out[j] = _rng(seed, _NOISE_STREAM, f).standard_normal(n)
    return out


def frame_params(seed, frames, choices):
    """Per-frame uniform picks: for each entry of ``choices`` (a list of
    option lists, or (lo, hi) float tuples) one value per frame."""
    frames = np.atleast_1d(frames)
    cols = []
    for c, opt in enumerate(choices):
        col = []
        for f in frames:
            g = _rng(seed, _PARAM_STREAM, (int(f) << 4) | c)
            if isinstance(opt, tuple):
                col.append(float(g.uniform(opt[0], opt[1])))
            else:
                col.append(opt[int(g.integers(0, len(opt)))])
        cols.append(col)
    return cols


def scatter_info(bits, frozen):
    """Place information bits at the non-frozen indices; u_F = 0."""
    bits = np.atleast_2d(bits)
    info = np.flatnonzero(np.asarray(frozen) == 0)
    if bits.shape[1] != info.shape[0]:
        raise ValueError("got %d info bits for a code with %d" % (bits.shape[1], info.shape[0]))
    u = np.zeros((bits.shape[0], np.asarray(frozen).shape[0]), np.uint8)
    u[:, info] = bits
    return u


def sigma(ebn0_db, rate):
    return float(np.sqrt(1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))))


def awgn_llr(x, z, ebn0_db, rate):
    """LLR = 2 y / sigma^2 with y = (1 - 2x) + sigma z, float32 [frames, n].

    ``ebn0_db`` may be a scalar or one value per frame.
    """
    x = np.atleast_2d(x)
    z = np.atleast_2d(z)
    s = np.asarray([sigma(e, rate) for e in np.atleast_1d(ebn0_db)], np.float64)
    if s.shape[0] == 1:
        s = np.full(x.shape[0], s[0])
    s = s.reshape(-1, 1)
    y = (1.0 - 2.0 * x.astype(np.float64)) + s * z
    return (2.0 * y / (s * s)).astype(np.float32)


def quantize6(llr):
    """6-bit symmetric saturating quantiser with one fractional bit -> int8."""
    v = 2.0 * np.asarray(llr, np.float64)
    q = np.sign(v) * np.floor(np.abs(v) + 0.5)
    return np.clip(q, -31, 31).astype(np.int8)


def pack_bits(bits):
    """[frames, n] 0/1 bytes -> [frames, ceil(n/8)] bytes, LSB first."""
    return np.packbits(np.atleast_2d(bits).astype(np.uint8), axis=1, bitorder="little")


def unpack_bits(packed, n):
    return np.unpackbits(np.atleast_2d(packed), axis=1, count=n, bitorder="little")
