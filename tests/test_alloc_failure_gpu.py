"""Failure handling on the device: an allocation failure forced from the
host (polar_debug_fail_allocations) at each allocation of polar_prepare,
polar_batch_set_frames and polar_server_create comes back as POLAR_ENOMEM,
keeps no device memory, and the same call succeeds afterwards with results
equal to the oracle."""
import numpy as np
import pytest

import oracle
from frames import make_frames
from paper_1504_00353_amd import Batch, Code, Server, binding, synth, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def disarm():
    yield
    binding.lib().polar_debug_fail_allocations(-1)


def free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_prepare_enomem_then_ok():
    L = binding.lib()
    c = Code(1024, 512, 2.5, llr="i8", kernel="schedule", prepare=False)
    L.polar_debug_fail_allocations(0)
    assert L.polar_prepare(c.handle) == binding.ENOMEM
    c.prepare()
    fr = c.frozen()
    _, _, llr = make_frames(fr, 5, 32, 2.5)
    out = c.decode(torch.from_numpy(llr).cuda())
    torch.cuda.synchronize()
    u, _, _ = oracle.decode(fr, llr, "fastssc")
    assert np.array_equal(out.cpu().numpy(), synth.pack_bits(u[:, fr == 0]))


def test_set_frames_enomem_then_ok():
    L = binding.lib()
    codes = [Code(n, k, d, llr="i8", prepare=False) for n, k, d in workloads.MIXED["codes"][:3]]
    b = Batch(codes)
    n = codes[0].n
    L.polar_debug_fail_allocations(0)
    with pytest.raises(binding.PolarError) as e:
        b.set_frames(np.zeros(4, np.int32), np.arange(4, dtype=np.int64) * n, np.arange(4, dtype=np.int64) * 64)
    assert e.value.status == binding.ENOMEM
    b.set_frames(np.zeros(4, np.int32), np.arange(4, dtype=np.int64) * n, np.arange(4, dtype=np.int64) * 64)
    b.close()


def test_server_create_enomem_at_each_allocation():
    """polar_server_create makes 7 allocations (the object, three device
    pools, three pinned buffers): failing each in turn gives ENOMEM and
    leaks no device memory; with the hook disarmed the server works."""
    L = binding.lib()
    codes = [Code(n, k, d, llr="i8", prepare=False) for n, k, d in workloads.SERVING["codes"]]
    batch = Batch(codes)
    free0 = free_bytes()
    for k in range(7):
        L.polar_debug_fail_allocations(k)
        with pytest.raises(binding.PolarError) as e:
            Server(batch, slots_per_class=256, streams=2, staging_bytes=8 << 20, device_bytes=64 << 20)
        assert e.value.status == binding.ENOMEM, k
    L.polar_debug_fail_allocations(-1)
    assert abs(free_bytes() - free0) < (16 << 20)
    srv = Server(batch, slots_per_class=256, streams=2, staging_bytes=8 << 20, device_bytes=64 << 20)
    fr = codes[0].frozen()
    _, _, llr = make_frames(fr, 9, 8, 3.0)
    out = np.zeros((8, codes[0].row_bytes), np.uint8)
    rid = srv.submit(0, llr, out)
    assert rid is not None
    srv.drain()
    u, _, _ = oracle.decode(fr, llr, "fastssc")
    assert np.array_equal(out, synth.pack_bits(u[:, fr == 0]))
    srv.close()
