"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a value
printed in the paper, a brute-force computation on tiny inputs, a closed
form derived independently, or an invariant.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from bounds import forward_error_scale
from frames import make_frames

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def kron_generator(n):
    """G_N = F_2^{(x) log2 N} built with numpy's Kronecker product."""
    F = np.array([[1, 0], [1, 1]], np.int64)
    G = np.array([[1]], np.int64)
    while G.shape[0] < n:
        G = np.kron(G, F)
    return G


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- encoder

def test_g4_matrix_as_printed():
    """Sec. II-A prints G_4; row j is the codeword of the unit vector e_j."""
    g4 = np.array([[int(v) for v in r] for r in read_golden("g4_matrix.txt")], np.uint8)
    rows = oracle.encode(np.eye(4, dtype=np.uint8))
    assert np.array_equal(rows, g4)


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64, 128, 256])
def test_encoder_is_kronecker_power(n):
    rng = np.random.default_rng(n)
    u = rng.integers(0, 2, size=(20, n), dtype=np.uint8)
    expect = (u.astype(np.int64) @ kron_generator(n)) % 2
    assert np.array_equal(oracle.encode(u), expect.astype(np.uint8))


# ---------------------------------------------------------- schedule / tree

def test_listing1_schedule_of_8_5_code():
    """Listing 1: the unrolled Fast-SSC decoder of the (8,5) code of Fig. 2."""
    rows = read_golden("listing1_8_5.txt")
    frozen = np.zeros(8, np.uint8)
    frozen[[int(v) for v in rows[0][1:]]] = 1
    expect = [(r[0], int(r[1])) for r in rows[1:]]
    assert oracle.schedule(frozen, "fastssc") == expect


def test_sc_schedule_walks_every_node():
    """Plain SC (Sec. II-C): F, G, Combine at every internal node of the full
    tree and one decision per information bit."""
    frozen = oracle.construct(64, 32, 2.5)
    ops = oracle.schedule(frozen, "sc")
    count = {}
    for name, _ in ops:
        count[name] = count.get(name, 0) + 1
    assert count == {"F": 63, "G": 63, "Combine": 63, "Info": 32}


# ------------------------------------------------------------- f and g

def maxlog_pair(a, b):
    """Max-log LLR of x0 xor x1 for the length-2 kernel, by enumerating the
    four hypotheses (metric ((1-2x0)a + (1-2x1)b)/2, kept doubled)."""
    best = {0: None, 1: None}
    for x0, x1 in itertools.product((0, 1), repeat=2):
        m = (1 - 2 * x0) * a + (1 - 2 * x1) * b
        p = x0 ^ x1
        best[p] = m if best[p] is None else max(best[p], m)
    return (best[0] - best[1]) / 2


def maxlog_u1(a, b, u0):
    """LLR of u1 given u0 for x = (u0 xor u1, u1), by enumeration."""
    best = {}
    for u1 in (0, 1):
        x0, x1 = u0 ^ u1, u1
        best[u1] = (1 - 2 * x0) * a + (1 - 2 * x1) * b
    return (best[0] - best[1]) / 2


def test_f_is_maxlog_parity_llr_int8_exhaustive():
    """eq. (1) min-sum f equals the max-log LLR of a parity, exactly, for
    every pair of int8 LLRs in the symmetric range."""
    vals = range(-127, 128)
    for a in vals:
        for b in vals:
            assert oracle.f_i8(a, b) == maxlog_pair(a, b)


def test_g_is_llr_of_u1_int8_exhaustive_with_saturation():
    """eq. (2) g equals the exact LLR of u1 given u0 = beta; the 8-bit form
    saturates symmetrically to [-127, 127] (Listing 4)."""
    vals = range(-127, 128)
    for beta in (0, 1):
        for a in vals:
            for b in vals:
                expect = int(np.clip(maxlog_u1(a, b, beta), -127, 127))
                assert oracle.g_i8(a, b, beta) == expect


def test_f_g_float_match_kernel_llrs():
    rng = np.random.default_rng(7)
    for a, b in rng.normal(0, 4, size=(2000, 2)):
        assert oracle.f_f64(a, b) == pytest.approx(maxlog_pair(a, b), rel=1e-12, abs=1e-15)
        for beta in (0, 1):
            assert oracle.g_f64(a, b, beta) == pytest.approx(maxlog_u1(a, b, beta), rel=0, abs=1e-12)


# ------------------------------------------------ constituent-code decoders

def code_words(kind, n):
    allw = np.array(list(itertools.product((0, 1), repeat=n)), np.uint8)
    if kind == "rate1":
        return allw
    if kind == "rep":
        return np.array([[0] * n, [1] * n], np.uint8)
    if kind == "spc":
        return allw[allw.sum(axis=1) % 2 == 0]
    raise ValueError(kind)


def spc_words_from_generator(n):
    """Rows 1..n-1 of G_n span the constituent code of an SPC node."""
    G = kron_generator(n)[1:]
    msgs = np.array(list(itertools.product((0, 1), repeat=n - 1)), np.int64)
    return np.unique((msgs @ G) % 2, axis=0).astype(np.uint8)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_spc_code_is_even_weight_code(n):
    words = spc_words_from_generator(n)
    assert np.array_equal(words, np.unique(code_words("spc", n), axis=0))


def rep_words_from_generator(n):
    G = kron_generator(n)[n - 1:]
    return np.unique((np.array([[0], [1]]) @ G) % 2, axis=0).astype(np.uint8)


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_rep_code_is_repetition_code(n):
    assert np.array_equal(rep_words_from_generator(n), code_words("rep", n))


@pytest.mark.parametrize("kind,n", [("rate1", 1), ("rate1", 2), ("rate1", 4), ("rate1", 8), ("rate1", 16),
                                    ("rep", 2), ("rep", 4), ("rep", 8), ("rep", 16),
                                    ("spc", 4), ("spc", 8), ("spc", 16)])
@pytest.mark.parametrize("dtype", ["i8", "f64"])
def test_node_decoder_is_ml(kind, n, dtype):
    """Rate-1, repetition and SPC node rules (Sec. II-D, II-E) return a
    codeword of the constituent code that attains the ML metric
    sum (1 - 2 c_i) alpha_i (ties allowed), checked by brute force."""
    words = code_words(kind, n)
    sign = 1 - 2 * words.astype(np.int64)
    rng = np.random.default_rng(1000 * n + len(kind))
    for trial in range(300):
        if dtype == "i8":
            alpha = rng.integers(-128, 128, size=n).astype(np.int8)
            if trial % 3 == 0:   # many ties and zeros
                alpha = rng.integers(-2, 3, size=n).astype(np.int8)
            metric = sign @ alpha.astype(np.int64)
        else:
            alpha = rng.normal(0, 3, size=n)
            metric = sign.astype(np.float64) @ alpha
        beta = oracle.node(kind, alpha)
        hit = np.flatnonzero((words == beta).all(axis=1))
        assert hit.size == 1, "not a codeword of the constituent code"
        assert metric[hit[0]] == metric.max()


def test_spc_flips_lowest_index_on_ties():
    """Listing 2 returns the first lane equal to the minimum: the lowest
    index is flipped when several |alpha| tie."""
    beta = oracle.node("spc", np.array([3, -1, 1, -1, 5, 1, 7, 9], np.int8))
    # hard decisions 0 1 0 1 0 0 0 0 have even parity -> unchanged
    assert beta.tolist() == [0, 1, 0, 1, 0, 0, 0, 0]
    beta = oracle.node("spc", np.array([3, -1, 1, 1, 5, 1, 7, 9], np.int8))
    # odd parity; |alpha| = 1 at indices 1, 2, 3, 5 -> flip index 1
    assert beta.tolist() == [0, 0, 0, 0, 0, 0, 0, 0]
    beta = oracle.node("spc", np.array([0.5, -2.0, 0.25, 0.25], np.float64))
    assert beta.tolist() == [0, 1, 1, 0]


def test_hard_decision_of_zero_is_zero():
    """eq. (4) and the repetition rule decide 0 for a zero input."""
    assert oracle.node("rate1", np.array([0, 0], np.int8)).tolist() == [0, 0]
    assert oracle.node("rep", np.array([3, -3, 1, -1], np.int8)).tolist() == [0, 0, 0, 0]
    assert oracle.node("rate1", np.array([-0.0, 0.0], np.float64)).tolist() == [0, 0]


# ---------------------------------------------------------- whole decoders

def random_r0_r1_rep_mask(n, rng):
    """A frozen mask whose Fast-SSC tree has only Rate-0, Rate-1 and
    repetition leaves."""
    if n >= 2 and rng.random() < 0.35:
        return np.array([1] * (n - 1) + [0], np.uint8)
    if n == 1 or rng.random() < 0.2:
        return np.full(n, rng.integers(0, 2), np.uint8)
    return np.concatenate([random_r0_r1_rep_mask(n // 2, rng), random_r0_r1_rep_mask(n // 2, rng)])


@pytest.mark.parametrize("n", [8, 32, 128, 512])
def test_fastssc_equals_sc_on_rate0_rate1_rep_trees(n):
    """Rate-0/Rate-1 pruning and the repetition rule reproduce SC exactly
    when LLRs have no exact ties (float64 Gaussian inputs); the halving-tree
    repetition sum is SC's own G_0R cascade."""
    rng = np.random.default_rng(n)
    for _ in range(20):
        frozen = random_r0_r1_rep_mask(n, rng)
        if frozen.all():
            continue
        llr = rng.normal(0.5, 2.0, size=(16, n))
        u_sc, x_sc, _ = oracle.decode(frozen, llr, "sc")
        u_fs, x_fs, _ = oracle.decode(frozen, llr, "fastssc")
        assert np.array_equal(u_sc, u_fs)
        assert np.array_equal(x_sc, x_fs)
        l32 = llr.astype(np.float32)
        assert np.array_equal(oracle.decode(frozen, l32, "sc")[0], oracle.decode(frozen, l32, "fastssc")[0])


CODES = [(8, 5, 2.0), (64, 32, 2.5), (256, 128, 2.5), (1024, 512, 2.5), (1024, 922, 4.0),
         (4096, 3686, 4.0), (32768, 29492, 4.0)]


@pytest.mark.parametrize("n,k,d", CODES)
def test_noiseless_recovery(n, k, d):
    """With reliable LLRs every decoder returns the transmitted u and x."""
    frozen = oracle.construct(n, k, d)
    rng = np.random.default_rng(n + k)
    u = np.zeros((4, n), np.uint8)
    u[:, frozen == 0] = rng.integers(0, 2, size=(4, k))
    x = oracle.encode(u)
    sign = 1 - 2 * x.astype(np.int64)
    algos = ["fastssc", "sc"] if n <= 4096 else ["fastssc"]
    for llr in (sign.astype(np.int8) * 31, sign.astype(np.float32) * 8.0, sign.astype(np.float64) * 8.0):
        for algo in algos:
            u_hat, x_hat, _ = oracle.decode(frozen, llr, algo)
            assert np.array_equal(u_hat, u)
            assert np.array_equal(x_hat, x)


@pytest.mark.parametrize("n,k,d", CODES[:6])
@pytest.mark.parametrize("llr", ["i8", "f32"])
def test_frozen_bits_decode_to_zero_and_u_is_transform_of_x(n, k, d, llr):
    frozen = oracle.construct(n, k, d)
    u, x, l = make_frames(frozen, 11, 32, d - 1.0, llr)
    for algo in ("fastssc", "sc"):
        u_hat, x_hat, _ = oracle.decode(frozen, l, algo)
        assert not u_hat[:, frozen == 1].any()
        assert np.array_equal(oracle.encode(u_hat), x_hat)


def test_fer_falls_with_snr():
    frozen = oracle.construct(256, 128, 2.5)
    fer = []
    for snr in (0.5, 2.0, 3.5):
        u, _, l = make_frames(frozen, 21, 300, snr, "f32")
        u_hat, _, _ = oracle.decode(frozen, l, "fastssc")
        fer.append(np.mean((u_hat != u).any(axis=1)))
    assert fer[0] > fer[1] > fer[2]
    assert fer[0] > 0.3 and fer[2] < 0.1


@pytest.mark.parametrize("n,k,d,algo", [(1024, 512, 2.5, "sc"), (4096, 3686, 4.0, "fastssc"),
                                        (32768, 29492, 4.0, "fastssc")])
def test_float32_oracle_tracks_float64(n, k, d, algo):
    """Same float32 channel values into both precisions: decisions identical,
    leaf LLRs within 1e-5 of the forward-error scale."""
    frozen = oracle.construct(n, k, d)
    frames = 8 if n > 4096 else 32
    _, _, l32 = make_frames(frozen, 31, frames, d, "f32")
    u32, _, t32 = oracle.decode(frozen, l32, algo, trace=True)
    u64, _, t64 = oracle.decode(frozen, l32.astype(np.float64), algo, trace=True)
    assert np.array_equal(u32, u64)
    scale = forward_error_scale(l32.astype(np.float64))
    err = np.abs(t32.astype(np.float64) - t64)
    assert (err <= 1e-5 * scale + 1e-30).all()


# ------------------------------------------------------------- construction

def bec_erasure_bruteforce(n, eps):
    """Exact probability that genie-aided SC cannot determine u_i on the
    BEC(eps), by enumerating every erasure pattern."""
    G = kron_generator(n)
    probs = np.zeros(n)
    vs = np.array(list(itertools.product((0, 1), repeat=n)), np.int64)
    cw = (vs @ G) % 2
    for pattern in itertools.product((0, 1), repeat=n):
        e = np.array(pattern, bool)   # True = erased
        p = eps ** e.sum() * (1 - eps) ** (n - e.sum())
        seen = ~e
        for i in range(n):
            # u_i undetermined iff some v with v_<i = 0, v_i = 1 maps to a
            # codeword that is zero on every unerased position
            cand = (vs[:, :i] == 0).all(axis=1) & (vs[:, i] == 1)
            if ((cw[cand][:, seen] == 0).all(axis=1)).any():
                probs[i] += p
    return probs


@pytest.mark.parametrize("n", [2, 4, 8])
@pytest.mark.parametrize("eps", [0.5, 0.2, 0.7])
def test_bhattacharyya_recursion_is_exact_on_bec(n, eps):
    """For the BEC, z -> 2z - z^2 and z -> z^2 are exact erasure
    probabilities; the index order (first index bit = root split) matches
    a brute-force genie-aided SC over all erasure patterns."""
    z = np.exp(oracle.bhattacharyya(n, np.log(eps)))
    assert np.allclose(z, bec_erasure_bruteforce(n, eps), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("n,k,d", CODES[1:] + [(256, 212, 4.0), (16384, 14746, 4.0), (32768, 27197, 4.0)])
def test_construction_invariants(n, k, d):
    frozen = oracle.construct(n, k, d)
    assert int((frozen == 0).sum()) == k
    # bit channel i + 2^b (bit b of i clear) is never less reliable than i
    idx = np.arange(n)
    h = 1
    while h < n:
        lo = idx[(idx & h) == 0]
        assert not (frozen[lo + h] & (frozen[lo] == 0)).any()
        h *= 2


# ------------------------------------------- construction channel parameter

def awgn_bhattacharyya_numeric(rate, ebn0_db):
    """Bhattacharyya parameter of BPSK (0 -> +1, 1 -> -1) over AWGN at the
    given Eb/N0, from its definition: the integral over y of
    sqrt(p(y | +1) p(y | -1)), with noise variance 1 / (2 R Eb/N0),
    integrated numerically."""
    from scipy import integrate
    sigma2 = 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))

    def density(y, s):
        return np.exp(-(y - s) ** 2 / (2 * sigma2)) / np.sqrt(2 * np.pi * sigma2)

    z, err = integrate.quad(lambda y: np.sqrt(density(y, 1.0) * density(y, -1.0)), -np.inf, np.inf,
                            epsabs=0, epsrel=1e-12, limit=200)
    assert err < 1e-10 * z
    return z


@pytest.mark.parametrize("n,k,d", [(1024, 512, 2.5), (32768, 29492, 4.0), (4096, 3686, 4.0),
                                   (256, 128, 2.5), (1024, 850, 4.0), (64, 16, 0.0), (16384, 15565, 6.0)])
def test_design_channel_is_bpsk_awgn_bhattacharyya(n, k, d):
    """Sec. II-A construction: the channel the oracle starts its reliability
    recursion from is the Bhattacharyya parameter of BPSK over AWGN at the
    design Eb/N0 of a rate-K/N code (checked against the numerically
    integrated definition, not a closed form), and the frozen set is the
    N - K channels of largest ln z, ties frozen at the lower index."""
    lnz, lnz0 = oracle.construct_reliability(n, k, d)
    assert lnz0 == pytest.approx(np.log(awgn_bhattacharyya_numeric(k / n, d)), rel=1e-9, abs=0)
    assert np.array_equal(lnz, oracle.bhattacharyya(n, lnz0))
    order = sorted(range(n), key=lambda i: (lnz[i], -i))  # most reliable first, higher index first on ties
    expect = np.ones(n, np.uint8)
    expect[order[:k]] = 0
    assert np.array_equal(oracle.construct(n, k, d), expect)


def test_fastssc_tree_sizes_match_independent_count():
    """The oracle's Fast-SSC schedule of the benchmark codes has the sizes
    counted independently of it (tests/golden/fastssc_sizes.txt): number of
    node functions, leaves of each kind and the elements they cover, f and
    G_0R elements.  Pins construction, node classification and pruning at
    full size together."""
    import collections
    rows = read_golden("fastssc_sizes.txt")
    assert rows
    for row in rows:
        n, k, d = int(row[0]), int(row[1]), float(row[2])
        sched = oracle.schedule(oracle.construct(n, k, d), "fastssc")
        count = collections.Counter(name for name, _ in sched)
        elems = collections.Counter()
        for name, size in sched:
            elems[name] += size // 2 if name in ("F", "G", "G_0R", "Combine", "Combine_0R") else size
        got = [len(sched), count["Info"], count["Repetition"], count["SPC"],
               elems["Info"], elems["Repetition"], elems["SPC"], elems["F"], elems["G_0R"]]
        for want, have in zip(row[3:], got):
            if want != "-":
                assert int(want) == have, (n, k, row, got)


@pytest.mark.parametrize("n,k,d,algo", [(64, 32, 2.5, "fastssc"), (64, 32, 2.5, "sc"),
                                        (1024, 512, 2.5, "fastssc"), (1024, 512, 2.5, "sc"),
                                        (4096, 3686, 4.0, "fastssc")])
def test_channel_minus128_is_read_as_minus127(n, k, d, algo):
    """Listing 4 keeps 8-bit LLRs in the symmetric range [-127, 127]; a
    channel value of -128 (representable in int8) is read as -127: decoding a
    frame that contains -128 gives the bits and leaf LLRs of the same frame
    with -127 in its place."""
    frozen = oracle.construct(n, k, d)
    rng = np.random.default_rng(n + k + len(algo))
    llr = rng.integers(-128, 128, size=(24, n)).astype(np.int8)
    llr[:8] = np.where(rng.random((8, n)) < 0.3, np.int8(-128), llr[:8])   # dense -128
    llr[8:16] = rng.choice(np.array([-128, -127, 127, 1, -1, 0], np.int8), size=(8, n))
    assert (llr == -128).any()
    u, x, t = oracle.decode(frozen, llr, algo, trace=True)
    u2, x2, t2 = oracle.decode(frozen, np.maximum(llr, np.int8(-127)), algo, trace=True)
    assert np.array_equal(u, u2)
    assert np.array_equal(x, x2)
    assert np.array_equal(t, t2)
    assert t.min() >= -127
