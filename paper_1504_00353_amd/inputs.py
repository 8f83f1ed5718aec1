"""Channel frames of one code for the benchmark and the study: seeded
information bits and noise from ``synth``, the codeword from the library's
own encoder (polar_encode, on the host), BPSK over AWGN as in ``synth``.

No decoding arithmetic here; the encoder is the library's, which the tests
hold to the oracle's (tests/test_library_host.py)."""
import concurrent.futures as cf

import numpy as np

from . import synth


def channel_frames(code, seed, frame_ids, ebn0_db, threads=8):
    """Float32 channel LLRs [len(frame_ids), N] and the information bits
    [len(frame_ids), K] of the given frame indices of ``code`` (frame f is
    the same whatever batch it is drawn in).  ``ebn0_db``: a scalar or one
    value per frame.  Chunks of frames run on ``threads`` threads."""
    frame_ids = np.atleast_1d(np.asarray(frame_ids))
    eb = np.broadcast_to(np.asarray(ebn0_db, np.float64), frame_ids.shape)
    llr = np.empty((frame_ids.shape[0], code.n), np.float32)
    info = np.empty((frame_ids.shape[0], code.k), np.uint8)

    def work(lo):
        hi = min(lo + step, frame_ids.shape[0])
        ids = frame_ids[lo:hi]
        bits = synth.info_bits(seed, ids, code.k)
        x = synth.unpack_bits(code.encode(synth.pack_bits(bits)), code.n)
        llr[lo:hi] = synth.awgn_llr(x, synth.noise(seed, ids, code.n), eb[lo:hi], code.k / code.n)
        info[lo:hi] = bits

    step = max(1, min(1024, (1 << 22) // code.n))
    with cf.ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(work, range(0, frame_ids.shape[0], step)))
    return llr, info
