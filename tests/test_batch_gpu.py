"""Mixed-code batches (one persistent launch over frames of several codes):
every frame against the oracle, the full 65,536-frame workload, HIP graph
replays, the autotuner and caller-owned descriptors."""
import numpy as np
import pytest

import oracle
from frames import make_mixed
from paper_1504_00353_amd import Batch, Code, synth, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIXED = workloads.MIXED


@pytest.fixture(scope="module")
def mixed():
    codes = [Code(n, k, d, llr="i8", prepare=False) for n, k, d in MIXED["codes"]]
    batch = Batch(codes)
    frozens = [c.frozen() for c in codes]
    return codes, batch, frozens


def expected_rows(frozens, code_idx, llr_flat, offs):
    """Oracle decode of every frame, grouped by code; packed info rows."""
    rows = [None] * len(code_idx)
    for c, fr in enumerate(frozens):
        sel = np.flatnonzero(code_idx == c)
        if sel.size == 0:
            continue
        n = fr.shape[0]
        l = np.stack([llr_flat[offs[f]:offs[f] + n] for f in sel])
        u, _, _ = oracle.decode(fr, l, "fastssc", nthreads=8)
        packed = synth.pack_bits(u[:, fr == 0])
        for j, f in enumerate(sel):
            rows[f] = packed[j]
    return rows


def bits_layout(codes, code_idx):
    rb = np.array([codes[c].row_bytes for c in code_idx], np.int64)
    return np.concatenate([[0], np.cumsum(rb)[:-1]]).astype(np.int64), rb, int(rb.sum())


def run(batch, codes, code_idx, offs, flat, tune=False):
    bo, rb, total = bits_layout(codes, code_idx)
    batch.set_frames(code_idx, offs, bo)
    llr = torch.from_numpy(flat).cuda()
    bits = torch.zeros(total, dtype=torch.uint8, device="cuda")
    if tune:
        batch.tune(llr, bits)
        bits.zero_()
    batch.decode(llr, bits)
    torch.cuda.synchronize()
    out = bits.cpu().numpy()
    return [out[bo[i]:bo[i] + rb[i]] for i in range(len(code_idx))], llr, bits


def test_mixed_batch_every_frame(mixed):
    """1,500 frames, code uniform over the 15 (N, R) pairs, Eb/N0 uniform
    2-5 dB: every frame equals the oracle."""
    codes, batch, frozens = mixed
    code_idx, offs, flat, _ = make_mixed(frozens, MIXED["seed"], 1500, MIXED["ebn0_db"])
    rows, _, _ = run(batch, codes, code_idx, offs, flat)
    exp = expected_rows(frozens, code_idx, flat, offs)
    bad = [i for i in range(len(rows)) if not np.array_equal(rows[i], exp[i])]
    assert not bad, "%d frames differ, first %s" % (len(bad), bad[:5])


def test_mixed_batch_65536_frames(mixed):
    """The full workload size in one launch: 65,536 descriptors over a pool
    of 960 distinct frames (64 per code); every output row checked."""
    codes, batch, frozens = mixed
    pool_idx = np.repeat(np.arange(len(codes), dtype=np.int32), 64)
    # pool frames: seeded per code, placed back to back
    sizes = np.array([codes[c].n for c in pool_idx], np.int64)
    poffs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = np.zeros(int(sizes.sum()), np.int8)
    for c, fr in enumerate(frozens):
        sel = np.flatnonzero(pool_idx == c)
        from frames import make_frames
        _, _, l = make_frames(fr, 300 + c, 64, 3.5, "i8")
        for j, f in enumerate(sel):
            flat[poffs[f]:poffs[f] + codes[c].n] = l[j]
    exp = expected_rows(frozens, pool_idx, flat, poffs)
    rng = np.random.default_rng(0)
    pick = rng.integers(0, pool_idx.shape[0], size=65536)
    code_idx = pool_idx[pick]
    rows, _, _ = run(batch, codes, code_idx, poffs[pick], flat)
    bad = [i for i in range(len(rows)) if not np.array_equal(rows[i], exp[pick[i]])]
    assert not bad, "%d of 65536 frames differ" % len(bad)


def test_mixed_batch_graph_replays(mixed):
    """A captured batch decode, replayed several times with eager work and
    synchronisation in between, matches the eager decode every time."""
    codes, batch, frozens = mixed
    code_idx, offs, flat, _ = make_mixed(frozens, 31, 700, MIXED["ebn0_db"])
    rows, llr, bits = run(batch, codes, code_idx, offs, flat)
    eager = bits.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bits.zero_()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            batch.decode(llr, bits, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        bits.fill_(0xA5)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bits, eager), "replay %d differs" % rep
        del junk


def test_mixed_batch_autotune_keeps_results(mixed):
    codes, batch, frozens = mixed
    code_idx, offs, flat, _ = make_mixed(frozens, 32, 900, MIXED["ebn0_db"])
    rows0, _, _ = run(batch, codes, code_idx, offs, flat)
    rows1, _, _ = run(batch, codes, code_idx, offs, flat, tune=True)
    shape = batch.launch_shape()
    assert shape["waves_per_block"] in (1, 2, 4) and shape["blocks"] >= 1
    assert all(np.array_equal(a, b) for a, b in zip(rows0, rows1))


def test_batch_caller_descriptors(mixed):
    """polar_batch_decode_desc with descriptors built by the caller equals
    polar_batch_decode."""
    codes, batch, frozens = mixed
    code_idx, offs, flat, _ = make_mixed(frozens, 33, 400, MIXED["ebn0_db"])
    rows, llr, bits = run(batch, codes, code_idx, offs, flat)
    bo, rb, total = bits_layout(codes, code_idx)
    desc = np.empty(2 * len(code_idx), np.uint64)
    desc[0::2] = code_idx.astype(np.uint64) | (bo.astype(np.uint64) << np.uint64(8))
    desc[1::2] = offs.astype(np.uint64)
    d = torch.from_numpy(desc.view(np.int64)).cuda()
    out = torch.zeros(total, dtype=torch.uint8, device="cuda")
    batch.decode_desc(d, len(code_idx), llr, out)
    torch.cuda.synchronize()
    assert torch.equal(out, bits)


def test_batch_zero_frames(mixed):
    codes, batch, frozens = mixed
    batch.set_frames(np.zeros(0, np.int32), np.zeros(0, np.int64), np.zeros(0, np.int64))
    llr = torch.zeros(16, dtype=torch.int8, device="cuda")
    bits = torch.zeros(16, dtype=torch.uint8, device="cuda")
    batch.decode(llr, bits)
    torch.cuda.synchronize()
    assert int(bits.sum()) == 0


def test_batch_of_codes_with_layouts():
    """Codes prepared with non-default register/LDS layouts carry them into
    a batch: every frame still equals the oracle."""
    codes = [Code(n, k, d, llr="i8", prepare=False, layout=lay) for n, k, d, lay in workloads.BATCH_LAYOUTS]
    batch = Batch(codes)
    frozens = [c.frozen() for c in codes]
    code_idx, offs, flat, _ = make_mixed(frozens, 77, 300, (3.0, 5.0))
    rows, _, _ = run(batch, codes, code_idx, offs, flat)
    exp = expected_rows(frozens, code_idx, flat, offs)
    bad = [i for i in range(len(rows)) if not np.array_equal(rows[i], exp[i])]
    assert not bad, "%d frames differ, first %s" % (len(bad), bad[:5])
    batch.close()


def test_float_batch_with_virtual_stage():
    """A float batch whose (32768,29492) code runs with stage 12 recomputed
    from its register stage (and stage 14 from the channel) beside smaller
    codes: every frame equals the float32 oracle."""
    codes = [Code(n, k, d, llr="f32", prepare=False) for n, k, d in workloads.BATCH_F32]
    assert codes[0].layouts()[0]["virtual_mid"] == 1
    batch = Batch(codes)
    frozens = [c.frozen() for c in codes]
    code_idx, offs, flat, _ = make_mixed(frozens, 78, 200, (3.0, 5.0), llr="f32")
    assert (code_idx == 0).sum() > 10
    rows, _, _ = run(batch, codes, code_idx, offs, flat)
    exp = expected_rows(frozens, code_idx, flat, offs)
    bad = [i for i in range(len(rows)) if not np.array_equal(rows[i], exp[i])]
    assert not bad, "%d frames differ, first %s" % (len(bad), bad[:5])
    batch.close()

