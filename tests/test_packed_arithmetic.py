"""The int8 kernels compute f and g on packed 16-bit lanes.  A 32-bit word
holds four int8 LLRs; read as two 16-bit lanes, its odd bytes are the high
bytes, so each lane is 256 v + e with v the odd LLR and e in [0, 255] the
even one ("garbled": the high byte is the value, the low byte is noise).
The even LLRs are moved into the high bytes with a zero low byte ("clean").
Results are kept garbled; their high bytes are packed back into words.

This models those packed operations in numpy (16-bit saturation included)
and checks them against the 8-bit definitions of eq. (1) and eq. (2) with
Listing 4's saturation (channel -128 read as -127): every single op over all
int8 pairs with edge and sampled noise bytes, and the two-level chains of the
fused root-child ops over sampled and edge quadruples.  The multiply-add of
g is exact before it saturates (checked on the device for every pair of
multiples of 256 and both signs)."""
import itertools

import numpy as np


def sat16(x):
    return np.clip(x, -32768, 32767)


# packed-lane models of the kernel's operations
def neg(a):  # 255 - a, saturating: the value -v, noise 255 - e
    return sat16(255 - a)


def fx(a, b):  # max(min(a, b), neg(max(a, b))); a, b clean or garbled
    return np.maximum(np.minimum(a, b), neg(np.maximum(a, b)))


def gx(a, b, s):  # max(mad_sat(a, s, b), -32512); a clean, b clean or garbled
    return np.maximum(sat16(b + a * s), -32512)


def chanx(a):  # channel -128 read as -127; clean or garbled
    return np.maximum(a, -32512)


def clean(a):  # drop the noise byte
    return (a >> 8) << 8


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
EDGE_NOISE = (0, 1, 2, 127, 128, 253, 254, 255)


def lanes(v, e):
    """16-bit lane holding value v with noise byte e (e = 0: clean)."""
    return v * 256 + e


def test_single_ops_exhaustive():
    rng = np.random.default_rng(1)
    noise = [(ea, eb) for ea in EDGE_NOISE for eb in EDGE_NOISE]
    noise += [(rng.integers(0, 256, A.shape), rng.integers(0, 256, A.shape)) for _ in range(4)]
    ef = f_def(clamp_chan(A), clamp_chan(B))
    nz = ef != 0
    for ea, eb in noise:
        a, b = lanes(A, ea), lanes(B, eb)
        # f on channel or stored values, either operand garbled
        r = pack(fx(a, b))
        assert (r[nz] == ef[nz]).all() and (r[~nz] == 0).all()
        # g: a clean, b garbled (channel values through chanx)
        for s in (1, -1):
            r = pack(gx(chanx(lanes(A, 0)), chanx(b), s))
            assert (r == g_def(clamp_chan(A), clamp_chan(B), s)).all()
            # a garbled, made clean first
            r = pack(gx(chanx(clean(a)), chanx(b), s))
            assert (r == g_def(clamp_chan(A), clamp_chan(B), s)).all()


def test_results_stay_in_range():
    """f and g results never read as -128 (stored bytes are in [-127, 127])."""
    for ea, eb in itertools.product(EDGE_NOISE, EDGE_NOISE):
        a, b = lanes(A, ea), lanes(B, eb)
        assert (pack(fx(a, b)) >= -127).all()
        for s in (1, -1):
            assert (pack(gx(chanx(lanes(A, 0)), chanx(b), s)) >= -127).all()


def test_fused_chains_sampled_and_edges():
    rng = np.random.default_rng(0)
    edge = np.array([-128, -127, -126, -100, -64, -2, -1, 0, 1, 2, 63, 100, 126, 127])
    q = np.concatenate([rng.integers(-128, 128, size=(200_000, 4)), np.array(list(itertools.product(edge, repeat=4)))])
    a0, a1, b0, b1 = (q[:, i] for i in range(4))
    inner_ops = {"F": None, "G+": 1, "G-": -1}
    for odd in (False, True):  # even lanes are clean; odd lanes carry noise
        e = [rng.integers(0, 256, q.shape[0]) if odd else 0 for _ in range(4)]
        c00, c01, c10, c11 = lanes(a0, e[0]), lanes(a1, e[1]), lanes(b0, e[2]), lanes(b1, e[3])
        for yc, ys in inner_ops.items():
            for xc, xs in inner_ops.items():
                if ys is None:
                    x, y = fx(c00, c01), fx(c10, c11)
                    xr, yr = f_def(clamp_chan(a0), clamp_chan(a1)), f_def(clamp_chan(b0), clamp_chan(b1))
                else:
                    x = gx(chanx(clean(c00)), chanx(c01), ys)
                    y = gx(chanx(clean(c10)), chanx(c11), ys)
                    xr, yr = g_def(clamp_chan(a0), clamp_chan(a1), ys), g_def(clamp_chan(b0), clamp_chan(b1), ys)
                assert (pack(x) == xr).all() and (pack(y) == yr).all(), (yc, odd)
                if xs is None:
                    r, er = fx(x, y), f_def(xr, yr)
                    nz = er != 0
                    assert (pack(r)[nz] == er[nz]).all() and (pack(r)[~nz] == 0).all(), (yc, xc)
                else:
                    r = gx(clean(x), y, xs)
                    assert (pack(r) == g_def(xr, yr, xs)).all(), (yc, xc)
