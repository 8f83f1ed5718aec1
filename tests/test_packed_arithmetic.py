"""The int8 kernels compute f and g on packed 16-bit lanes holding 256 x the
LLR, with "loose" intermediates (exact multiples of 256, or 32767 standing
for +127).  This models those packed operations in numpy (16-bit
saturation and wrap-around included) and checks them against the 8-bit
definitions of eq. (1) and eq. (2) with Listing 4's saturation (channel
-128 read as -127): every single op over all int8 pairs, and the two-level
chains of the fused root-child ops over sampled and edge quadruples."""
import itertools

import numpy as np


def sat16(x):
    return np.clip(x, -32768, 32767)


def wrap16(x):
    return (x + 32768) % 65536 - 32768


# packed-lane models of the kernel's operations
def fx(a, b):  # max(min(a, b), sat(0 - max(a, b)))
    return np.maximum(np.minimum(a, b), sat16(0 - np.maximum(a, b)))


def gx(a, b, s):  # sat_lo(add_sat(b, a * s)), the product wrapping in 16 bits
    return np.maximum(sat16(b + wrap16(a * s)), -32512)


def chanx(a):
    return np.maximum(a, -32512)


def tight(a):
    return np.minimum(a, 32512)


def pack(w):  # the high byte, as a signed int8
    return w >> 8


# 8-bit definitions
def clamp_chan(x):
    return np.maximum(x, -127)


def f_def(a, b):
    return np.sign(a) * np.sign(b) * np.minimum(np.abs(a), np.abs(b))


def g_def(a, b, s):
    return np.clip(b + s * a, -127, 127)


V = np.arange(-128, 128)
A, B = (x.ravel() for x in np.meshgrid(V, V, indexing="ij"))


def test_single_ops_exhaustive():
    # f on channel values (no clamp needed), and sign agreement aside from zero
    r = pack(fx(A * 256, B * 256))
    e = f_def(clamp_chan(A), clamp_chan(B))
    nz = e != 0
    assert (r[nz] == e[nz]).all() and (r[~nz] == 0).all()
    for s in (1, -1):
        assert (pack(gx(chanx(A * 256), chanx(B * 256), s)) == g_def(clamp_chan(A), clamp_chan(B), s)).all()


def test_fused_chains_sampled_and_edges():
    rng = np.random.default_rng(0)
    edge = np.array([-128, -127, -126, -100, -64, -2, -1, 0, 1, 2, 63, 100, 126, 127])
    q = np.concatenate([rng.integers(-128, 128, size=(200_000, 4)), np.array(list(itertools.product(edge, repeat=4)))])
    a0, a1, b0, b1 = (q[:, i] for i in range(4))
    inner_ops = {"F": None, "G+": 1, "G-": -1}
    for yc, ys in inner_ops.items():
        for xc, xs in inner_ops.items():
            if ys is None:
                x, y = fx(a0 * 256, a1 * 256), fx(b0 * 256, b1 * 256)
                xr, yr = f_def(clamp_chan(a0), clamp_chan(a1)), f_def(clamp_chan(b0), clamp_chan(b1))
            else:
                x, y = gx(chanx(a0 * 256), chanx(a1 * 256), ys), gx(chanx(b0 * 256), chanx(b1 * 256), ys)
                xr, yr = g_def(clamp_chan(a0), clamp_chan(a1), ys), g_def(clamp_chan(b0), clamp_chan(b1), ys)
            # loose values: exact multiples of 256 in range, or 32767
            for w in (x, y):
                assert ((w >= -32512) & (w <= 32767) & ((w % 256 == 0) | (w == 32767))).all()
            if xs is None:
                r, er = fx(x, y), f_def(xr, yr)
                nz = er != 0
                assert (pack(r)[nz] == er[nz]).all() and (pack(r)[~nz] == 0).all(), (yc, xc)
            else:
                r = gx(tight(x), tight(y), xs)
                assert (pack(r) == g_def(xr, yr, xs)).all(), (yc, xc)
