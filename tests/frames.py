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


def make_mixed(frozens, seed, frames, ebn0_range, llr="i8"):
    """Frames of several codes in one flat LLR buffer: the code of each frame
    and its Eb/N0 (uniform over ``ebn0_range``) are per-frame seeded picks.
    Returns (code index [frames], llr offsets, flat llr, expected u list)."""
    idx = np.arange(frames)
    code_idx, ebn0 = synth.frame_params(seed, idx, [list(range(len(frozens))), ebn0_range])
    code_idx = np.asarray(code_idx, np.int32)
    ebn0 = np.asarray(ebn0, np.float64)
    sizes = np.array([len(frozens[c]) for c in code_idx], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.zeros(int(sizes.sum()), np.int8 if llr == "i8" else np.float32)
    us = [None] * frames
    for c, fr in enumerate(frozens):
        sel = np.flatnonzero(code_idx == c)
        if sel.size == 0:
            continue
        fr = np.asarray(fr, np.uint8)
        n = fr.shape[0]
        k = int((fr == 0).sum())
        bits = synth.info_bits(seed, sel, k)
        u = synth.scatter_info(bits, fr)
        x = oracle.encode(u)
        z = synth.noise(seed, sel, n)
        l32 = synth.awgn_llr(x, z, ebn0[sel], k / n)
        l = synth.quantize6(l32) if llr == "i8" else l32
        for j, f in enumerate(sel):
            flat[offs[f]:offs[f] + n] = l[j]
            us[f] = u[j]
    return code_idx, offs, flat, us
