"""Continuous-batching request server: every result equals the oracle and
equals the same request decoded alone; requests wait for device slots when
memory is short; staging back-pressure; LLRs read in place from device
memory."""
import numpy as np
import pytest

import oracle
from frames import make_frames
from paper_1504_00353_amd import Batch, Code, Server, synth, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SERVING = workloads.SERVING


@pytest.fixture(scope="module")
def serving():
    codes = [Code(n, k, d, llr="i8", prepare=False) for n, k, d in SERVING["codes"]]
    batch = Batch(codes)
    frozens = [c.frozen() for c in codes]
    return codes, batch, frozens


def make_requests(codes, frozens, seed, count, max_frames=64):
    """Seeded requests: code uniform, 1..max_frames frames, Eb/N0 uniform 2-5 dB."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        c = int(rng.integers(0, len(codes)))
        nf = int(rng.integers(1, max_frames + 1))
        eb = float(rng.uniform(*SERVING["ebn0_db"]))
        _, _, l = make_frames(frozens[c], seed * 1000 + r, nf, eb, "i8")
        reqs.append((c, l))
    return reqs


def oracle_rows(frozen, llr):
    u, _, _ = oracle.decode(frozen, llr, "fastssc", nthreads=8)
    return synth.pack_bits(u[:, np.asarray(frozen) == 0])


def serve(server, codes, reqs, on_device=False, polls_between=1):
    outs = {}
    ids = {}
    pending = list(range(len(reqs)))
    while pending:
        i = pending[0]
        c, l = reqs[i]
        bits = np.zeros((l.shape[0], codes[c].row_bytes), np.uint8)
        src = torch.from_numpy(l).cuda() if on_device else l
        rid = server.submit(c, src, bits)
        if rid is None:  # staging full: make progress first
            server.poll()
            continue
        ids[rid] = i
        outs[i] = bits
        pending.pop(0)
        for _ in range(polls_between):
            server.poll()
    server.drain()
    return [outs[i] for i in range(len(reqs))]


def test_server_mix_equals_alone_and_oracle(serving):
    codes, batch, frozens = serving
    reqs = make_requests(codes, frozens, 41, 90)
    srv = Server(batch, slots_per_class=1024, streams=2)
    mixed = serve(srv, codes, reqs)
    for i, (c, l) in enumerate(reqs):
        assert np.array_equal(mixed[i], oracle_rows(frozens[c], l)), "request %d differs from the oracle" % i
    for i in range(0, len(reqs), 9):  # a sample decoded alone
        alone = serve(srv, codes, [reqs[i]])[0]
        assert np.array_equal(alone, mixed[i]), "request %d: alone != in the mix" % i
    srv.close()


def test_server_device_resident_llrs(serving):
    codes, batch, frozens = serving
    reqs = make_requests(codes, frozens, 42, 40)
    srv = Server(batch, slots_per_class=1024, streams=3)
    dev = serve(srv, codes, reqs, on_device=True)
    host = serve(srv, codes, reqs, on_device=False)
    for i in range(len(reqs)):
        assert np.array_equal(dev[i], host[i])
        assert np.array_equal(dev[i], oracle_rows(frozens[reqs[i][0]], reqs[i][1]))
    srv.close()


def test_server_admission_waits_for_slots(serving):
    """64 slots per frame length: requests queue until earlier ones retire."""
    codes, batch, frozens = serving
    reqs = make_requests(codes, frozens, 43, 40)
    srv = Server(batch, slots_per_class=64, streams=2)
    outs = []
    waited = 0
    for c, l in reqs:
        bits = np.zeros((l.shape[0], codes[c].row_bytes), np.uint8)
        assert srv.submit(c, l, bits) is not None
        outs.append(bits)
        srv.poll()
        waited = max(waited, srv.pending()[0])
    srv.drain()
    assert waited > 0
    for (c, l), o in zip(reqs, outs):
        assert np.array_equal(o, oracle_rows(frozens[c], l))
    srv.close()


def test_server_staging_back_pressure(serving):
    """A small pinned staging area: submit reports 'no room' until a poll
    retires earlier requests; every request still completes correctly."""
    codes, batch, frozens = serving
    reqs = make_requests(codes, frozens, 44, 30)
    srv = Server(batch, slots_per_class=512, streams=2, staging_bytes=2 << 20)
    refused = 0
    outs = []
    for c, l in reqs:
        bits = np.zeros((l.shape[0], codes[c].row_bytes), np.uint8)
        while srv.submit(c, l, bits) is None:
            refused += 1
            srv.poll()
        outs.append(bits)
    srv.drain()
    assert refused > 0
    for (c, l), o in zip(reqs, outs):
        assert np.array_equal(o, oracle_rows(frozens[c], l))
    srv.close()


def test_server_device_outputs_and_trace_replay(serving):
    """Device-resident results, and the native load generator replaying a
    timed trace: every request equals the oracle."""
    codes, batch, frozens = serving
    reqs = make_requests(codes, frozens, 45, 60)
    srv = Server(batch, slots_per_class=1024, streams=2)
    llrs = [torch.from_numpy(l).cuda() for _, l in reqs]
    outs = [torch.zeros((l.shape[0], codes[c].row_bytes), dtype=torch.uint8, device="cuda") for c, l in reqs]
    arrival = np.cumsum(np.full(len(reqs), 2e-4))
    done = srv.run_trace(arrival, [c for c, _ in reqs], [l.shape[0] for _, l in reqs],
                         [t.data_ptr() for t in llrs], [o.data_ptr() for o in outs])
    torch.cuda.synchronize()
    assert (done >= arrival).all()
    for (c, l), o in zip(reqs, outs):
        assert np.array_equal(o.cpu().numpy(), oracle_rows(frozens[c], l))
    # device outputs through submit/poll as well
    outs2 = [torch.zeros_like(o) for o in outs]
    for (c, _), t, o in zip(reqs, llrs, outs2):
        assert srv.submit(c, t, o) is not None
        srv.poll()
    srv.drain()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(outs, outs2))
    srv.close()


def test_server_short_code_not_behind_long(serving):
    """Steps are per frame length: a one-frame request of the shortest code,
    submitted right after a 64-frame request of the longest, is reported
    done no later than it (and both equal the oracle)."""
    codes, batch, frozens = serving
    ns = [c.n for c in codes]
    big, small = int(np.argmax(ns)), int(np.argmin(ns))
    _, _, lb = make_frames(frozens[big], 71, 64, 4.0, "i8")
    _, _, ls = make_frames(frozens[small], 72, 1, 4.0, "i8")
    srv = Server(batch, slots_per_class=256, streams=3)
    bb = np.zeros((64, codes[big].row_bytes), np.uint8)
    bs = np.zeros((1, codes[small].row_bytes), np.uint8)
    ib = srv.submit(big, lb, bb)
    isml = srv.submit(small, ls, bs)
    seen = {}
    polls = 0
    while len(seen) < 2:
        for rid in srv.poll():
            seen[rid] = polls
        polls += 1
        assert polls < 5_000_000, "requests not completed"
    srv.drain()
    srv.close()
    assert seen[isml] <= seen[ib]
    assert np.array_equal(bb, oracle_rows(frozens[big], lb))
    assert np.array_equal(bs, oracle_rows(frozens[small], ls))
