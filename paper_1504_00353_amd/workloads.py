"""The benchmark workloads: codes, channel SNRs, frame counts and seeds.

Parameters only -- no encoding or decoding arithmetic lives here.  Each
workload draws its frames from ``synth`` with its own seed.  The codes are
the paper's families: rate-1/2 and high-rate codes from N = 256 up to
N = 32768, including the (32768, 29492) code of Tables 1 and 3 and the
(4096, 3686) code of Table 6.
"""

# Design Eb/N0 of the frozen set: 2.5 dB for rate 1/2, 4.0 dB for higher rates.
DESIGN_DB_LOW_RATE = 2.5
DESIGN_DB_HIGH_RATE = 4.0


def code_k(n, rate):
    """K = round_half_up(rate * N); rate 0.9 at N = 32768 is the paper's
    (32768, 29492) code."""
    if n == 32768 and abs(rate - 0.9) < 1e-9:
        return 29492
    return int(rate * n + 0.5)


def design_db(rate):
    return DESIGN_DB_LOW_RATE if rate <= 0.5 + 1e-9 else DESIGN_DB_HIGH_RATE


# name -> description.  "codes" lists (N, K, design Eb/N0 dB).
SC_1024 = dict(
    name="sc_1024_512_f32", seed=1, algo="sc", llr="f32",
    codes=[(1024, 512, 2.5)], ebn0_db=2.5, frames=10000)

FSSC_32K = dict(
    name="fastssc_32768_29492_i8", seed=2, algo="fastssc", llr="i8",
    codes=[(32768, 29492, 4.0)], ebn0_db=4.0, frames=4096)

FSSC_32K_F32 = dict(FSSC_32K, name="fastssc_32768_29492_f32", llr="f32")

MIXED_NS = (256, 1024, 4096, 16384, 32768)
MIXED_RATES = (0.5, 0.83, 0.9)
MIXED = dict(
    name="mixed_batch_i8", seed=3, algo="fastssc", llr="i8",
    codes=[(n, code_k(n, r), design_db(r)) for n in MIXED_NS for r in MIXED_RATES],
    ebn0_db=(2.0, 5.0), frames=65536)

SERVE_NS = (1024, 4096, 32768)
SERVE_RATES = (0.5, 0.6, 0.7, 0.8, 0.9)
SERVING = dict(
    name="serving_i8", seed=4, algo="fastssc", llr="i8",
    codes=[(n, code_k(n, r), design_db(r)) for n in SERVE_NS for r in SERVE_RATES],
    ebn0_db=(2.0, 5.0), loads=(0.1, 0.5, 0.9), frames_per_request=(1, 64))

STRESS = dict(
    name="stress_i8", seed=5, algo="fastssc", llr="i8",
    codes=[(32768, 29492, 4.0), (4096, 3686, 4.0)], ebn0_db=4.5, frames=262144)

ALL = [SC_1024, FSSC_32K, FSSC_32K_F32, MIXED, SERVING, STRESS]

# Further codes whose unrolled kernels are built ahead of time: the small
# codes of the smoke run and of the unrolled-kernel parity tests.
# codes whose unrolled kernels are built in every layout the autotuner
# times (layout parity tests, polar_tune_layout)
UNROLLED_LAYOUTS = [
    (32768, 29492, 4.0, "fastssc", "i8"),
    (4096, 3686, 4.0, "fastssc", "i8"),
    (16384, 14746, 4.0, "fastssc", "f32"),
    (32768, 29492, 4.0, "fastssc", "f32"),
]

# a batch whose codes use non-default layouts: (N, K, design dB, layout)
BATCH_LAYOUTS = [(32768, 29492, 4.0, 2), (4096, 3686, 4.0, 1), (1024, 512, 2.5, 0)]

# a float batch with the N = 32768 code in its default layout (stages 14 and
# 12 recomputed) beside smaller codes
BATCH_F32 = [(32768, 29492, 4.0), (4096, 3686, 4.0), (1024, 512, 2.5)]

# unrolled kernels built with the fused leaf-pair nodes switched off (the
# fused-vs-separate comparison)
UNROLLED_UNFUSED = [
    (1024, 512, 2.5, "fastssc", "i8"),
    (1024, 512, 2.5, "fastssc", "f32"),
    (4096, 3686, 4.0, "fastssc", "i8"),
    (32768, 29492, 4.0, "fastssc", "i8"),
]

UNROLLED_EXTRA = [
    (1024, 512, 2.5, "fastssc", "i8"),
    (1024, 512, 2.5, "fastssc", "f32"),
    (256, 128, 2.5, "sc", "i8"),
    (4096, 3686, 4.0, "fastssc", "f32"),
    (16384, 14746, 4.0, "fastssc", "i8"),
    (16384, 14746, 4.0, "fastssc", "f32"),
    (32768, 16384, 2.5, "fastssc", "i8"),
]


def _blocks(n, spec):
    """Frozen mask from (kind, size) blocks laid end to end: kind "R0"
    all frozen, "R1" none, "REP" all but the last, "SPC" only the first."""
    mask = []
    for kind, size in spec:
        if kind == "R0":
            mask += [1] * size
        elif kind == "R1":
            mask += [0] * size
        elif kind == "REP":
            mask += [1] * (size - 1) + [0]
        else:
            mask += [1] + [0] * (size - 1)
    assert len(mask) == n
    return mask


# Frozen sets with every leaf kind at the widest node sizes of N = 32768 and
# 16384 (the stages a generated int8 kernel keeps in registers), and inner
# root children reached through f, g and g_0R (its fused root-child ops).
def pair_blocks():
    """Every fused leaf-pair node (left Rate-0 or repetition, right Rate-1 or
    SPC) at every child size 2..32 where the pair exists (P_01 from 2, the
    others from 4), largest first so every block is aligned to its size."""
    spec = []
    for h in (32, 16, 8, 4, 2):
        for left, right in (("R0", "R1"), ("R0", "SPC"), ("REP", "SPC"), ("REP", "R1")):
            if h < 4 and (right == "SPC" or left == "REP"):
                continue  # SPC leaves start at 4; repetition 2 + Rate-1 2 is itself an SPC node
            spec += [(left, h), (right, h)]
    return spec


def _pairs_mask(n):
    spec = pair_blocks()
    used = sum(size for _, size in spec)
    # the rest: aligned groups of a size-8 RepSPC and two size-4 P_01 pairs,
    # then Rate-1 bits
    rest = []
    while used + 16 <= n:
        rest += [("REP", 4), ("SPC", 4), ("R0", 2), ("R1", 2), ("R0", 2), ("R1", 2)]
        used += 16
    rest += [("R1", 1)] * (n - used)
    return _blocks(n, spec + rest)


UNROLLED_MASKS = {
    "m2k_leaf_pairs": (2048, _pairs_mask(2048)),
    "m32k_spc13_rep13_spc14": (32768, _blocks(32768, [("SPC", 8192), ("REP", 8192), ("SPC", 16384)])),
    "m32k_r013_r113_rep14": (32768, _blocks(32768, [("R0", 8192), ("R1", 8192), ("REP", 16384)])),
    "m32k_r114_r014": (32768, _blocks(32768, [("R1", 16384), ("R0", 16384)])),
    "m32k_rep12_spc12_r113_spc14": (32768, _blocks(32768, [("REP", 4096), ("SPC", 4096), ("R1", 8192),
                                                           ("SPC", 16384)])),
    "m32k_r014_spc13_rep13": (32768, _blocks(32768, [("R0", 16384), ("SPC", 8192), ("REP", 8192)])),
    "m32k_spc13_rep13_r013_r113": (32768, _blocks(32768, [("SPC", 8192), ("REP", 8192), ("R0", 8192),
                                                            ("R1", 8192)])),
    # Rate-1 and SPC leaves of size 4096 and inner size-4096 nodes under each
    # parent op (f, g, g_0R): the float N = 32768 kernels recompute stage 12
    "m32k_mid_leaves": (32768, _blocks(32768, [("REP", 2048), ("SPC", 2048), ("R1", 4096), ("SPC", 4096),
                                               ("R0", 2048), ("SPC", 2048), ("R0", 4096), ("SPC", 4096),
                                               ("REP", 2048), ("R1", 2048), ("REP", 2048), ("SPC", 2048)])),
    "m16k_spc13_rep13": (16384, _blocks(16384, [("SPC", 8192), ("REP", 8192)])),
    "m16k_r113_spc13": (16384, _blocks(16384, [("R1", 8192), ("SPC", 8192)])),
}

# masks whose generated kernels are also built for float LLRs (virtual top
# stage with g_0R and inner children, and a code that keeps the stage)
UNROLLED_MASKS_F32 = ["m32k_spc13_rep13_r013_r113", "m32k_r014_spc13_rep13", "m32k_r013_r113_rep14",
                      "m32k_mid_leaves"]
