"""The allocation-free batch entry point (polar_batch_decode_frames_noalloc):
its output equals polar_batch_set_frames + polar_batch_decode on the same
frames, on two calls in a row (the second smaller, so stale descriptors of
the first would show), frames with bad entries are skipped, and sizes over
the fixed descriptor array are refused."""
import ctypes

import numpy as np
import pytest

from frames import make_mixed
from paper_1504_00353_amd import Batch, Code, binding, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIXED = workloads.MIXED
SENTINEL = 0xA5


@pytest.fixture(scope="module")
def mixed():
    codes = [Code(n, k, d, llr="i8", prepare=False) for n, k, d in MIXED["codes"]]
    batch = Batch(codes)
    return codes, batch, [c.frozen() for c in codes]


def layout(codes, code_idx):
    rb = np.array([codes[c].row_bytes for c in code_idx], np.int64)
    return np.concatenate([[0], np.cumsum(rb)[:-1]]).astype(np.int64), rb, int(rb.sum())


def reference(batch, code_idx, offs, bo, llr, total):
    batch.set_frames(code_idx, offs, bo)
    bits = torch.full((total,), SENTINEL, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    batch.decode(llr, bits)
    torch.cuda.synchronize()
    return bits.cpu().numpy()


def test_noalloc_matches_batch_decode_twice(mixed):
    codes, batch, frozens = mixed
    code_idx, offs, flat, _ = make_mixed(frozens, 77, 1200, MIXED["ebn0_db"])
    bo, rb, total = layout(codes, code_idx)
    llr = torch.from_numpy(flat).cuda()
    out = torch.full((total,), SENTINEL, dtype=torch.uint8, device="cuda")
    for n in (1200, 300):  # second call smaller: its rows only
        ci, lo, b = code_idx[:n], offs[:n], bo[:n]
        sub_total = int(b[-1] + rb[n - 1])
        print("noalloc call: %d frames" % n, flush=True)
        ref = reference(batch, ci, lo, b, llr, sub_total)
        out.fill_(SENTINEL)
        torch.cuda.synchronize()
        batch.decode_frames_noalloc(torch.from_numpy(ci).cuda(), torch.from_numpy(lo).cuda(),
                                    torch.from_numpy(b).cuda(), llr, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got[:sub_total], ref), "rows differ from polar_batch_decode (%d frames)" % n
        assert (got[sub_total:] == SENTINEL).all(), "rows beyond this call's frames were written"


def test_noalloc_skips_bad_frames(mixed):
    codes, batch, frozens = mixed
    code_idx, offs, flat, _ = make_mixed(frozens, 78, 64, MIXED["ebn0_db"])
    bo, rb, total = layout(codes, code_idx)
    llr = torch.from_numpy(flat).cuda()
    ref = reference(batch, code_idx, offs, bo, llr, total)
    bad_ci = code_idx.copy()
    bad_lo = offs.copy()
    bad_ci[3] = len(codes)      # code index out of range
    bad_ci[5] = -1
    bad_lo[9] = -4              # negative LLR offset
    out = torch.full((total,), SENTINEL, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    batch.decode_frames_noalloc(torch.from_numpy(bad_ci).cuda(), torch.from_numpy(bad_lo).cuda(),
                                torch.from_numpy(bo).cuda(), llr, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i in range(64):
        row, want = got[bo[i]:bo[i] + rb[i]], ref[bo[i]:bo[i] + rb[i]]
        if i in (3, 5, 9):
            assert (row == SENTINEL).all(), "skipped frame %d was written" % i
        else:
            assert np.array_equal(row, want), "frame %d differs" % i


def test_noalloc_rejects_oversize(mixed):
    _, batch, _ = mixed
    L = binding.lib()
    p = ctypes.c_void_p(256)
    rc = L.polar_batch_decode_frames_noalloc(batch._h, 262145, p, p, p, p, p, None)
    assert rc == binding.EINVAL
    assert b"262144" in L.polar_last_message()
    assert L.polar_batch_decode_frames_noalloc(batch._h, 0, None, None, None, None, None, None) == binding.OK
    assert L.polar_batch_decode_frames_noalloc(batch._h, -1, None, None, None, None, None, None) == binding.EINVAL
