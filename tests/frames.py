"""Test helper: seeded channel frames for a code, encoded by the oracle.

Inputs come from the shared seeded generator; the codeword is computed by
the oracle's encoder, so no input or expected value here depends on the GPU
library.
"""
import numpy as np

import oracle
from paper_1504_00353_amd import synth


def make_frames(frozen, seed, frames, ebn0_db, llr="i8"):
    """Returns (u, x, llr) for frame indices ``frames`` (int or array)."""
    frozen = np.asarray(frozen, np.uint8)
    n = frozen.shape[0]
    k = int((frozen == 0).sum())
    idx = np.arange(frames) if np.isscalar(frames) else np.asarray(frames)
    bits = synth.info_bits(seed, idx, k)
    u = synth.scatter_info(bits, frozen)
    x = oracle.encode(u)
    z = synth.noise(seed, idx, n)
    l32 = synth.awgn_llr(x, z, ebn0_db, k / n)
    if llr == "f32":
        return u, x, l32
    if llr == "i8":
        return u, x, synth.quantize6(l32)
    raise ValueError(llr)
