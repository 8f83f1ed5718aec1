"""The float32 contract against the float64 oracle at full workload size.

The GPU float32 decoders compute every message with one binary32 operation
in a fixed order; the float64 oracle is the reference precision.  On the
float workloads -- (1024,512) plain SC over 10,000 frames at 2.5 dB and
(32768,29492) Fast-SSC over 4,096 frames at 4.0 dB -- the GPU's decoded
bits equal the float64 oracle's on every frame, and every leaf LLR is
within 1e-5 of the float64 value relative to its forward-error scale
(eqs. (1)-(2): the bound of the magnitudes that reach that position).  A
bit disagreement would have to sit on a near-tie (|alpha64| below the
tolerance); such positions are counted and reported.
"""
import numpy as np
import pytest

import oracle
from bounds import forward_error_scale
from frames import make_frames
from paper_1504_00353_amd import Code, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def check_against_f64(code, frozen, llr, algo, chunk):
    """Returns (frames with differing bits, near-tie leaf positions, worst
    relative trace error) over all frames, in chunks."""
    bad_frames, near_ties, worst = 0, 0, 0.0
    for a in range(0, llr.shape[0], chunk):
        sub = np.ascontiguousarray(llr[a:a + chunk])
        t = torch.from_numpy(sub).cuda()
        out, tr = code.decode_trace(t)
        torch.cuda.synchronize()
        bits, tr = out.cpu().numpy(), tr.cpu().numpy().astype(np.float64)
        l64 = sub.astype(np.float64)
        u64, _, t64 = oracle.decode(frozen, l64, algo, trace=True, nthreads=8)
        expect = synth.pack_bits(u64[:, np.asarray(frozen) == 0])
        bad_frames += int((bits != expect).any(axis=1).sum())
        scale = forward_error_scale(l64)
        leaf = frozen == 0  # the trace covers every position under a decision node
        err = np.abs(tr - t64)
        ok = err <= TOL * scale
        # positions under Rate-0 nodes are untouched on both sides (zero)
        assert ok.all(), "trace beyond 1e-5 of the forward-error scale in %d positions" % int((~ok).sum())
        near_ties += int(((np.abs(t64) < TOL * scale) & (scale > 0) & leaf[None, :]).sum())
        rel = err / np.maximum(scale, 1e-300)
        worst = max(worst, float(rel.max()))
        del t, out
    return bad_frames, near_ties, worst


def test_sc_1024_512_f32_equals_float64_oracle_all_frames():
    """Config: (1024,512) plain SC, float32 LLRs, 10,000 frames at 2.5 dB."""
    code = Code(1024, 512, 2.5, algo="sc", llr="f32", kernel="unrolled")
    fr = code.frozen()
    _, _, l = make_frames(fr, 1, 10000, 2.5, "f32")
    bad, ties, worst = check_against_f64(code, fr, l, "sc", 2500)
    print("(1024,512) SC f32 vs f64: %d frames differ, %d near-tie positions, worst trace error %.2e of scale"
          % (bad, ties, worst))
    assert bad == 0


def test_fastssc_32768_29492_f32_equals_float64_oracle_all_frames():
    """Config: (32768,29492) Fast-SSC, float32 LLRs, 4,096 frames at 4.0 dB."""
    code = Code(32768, 29492, 4.0, llr="f32", kernel="unrolled")
    fr = code.frozen()
    _, _, l = make_frames(fr, 2, 4096, 4.0, "f32")
    bad, ties, worst = check_against_f64(code, fr, l, "fastssc", 256)
    print("(32768,29492) Fast-SSC f32 vs f64: %d frames differ, %d near-tie positions, worst trace error %.2e "
          "of scale" % (bad, ties, worst))
    assert bad == 0
