"""Host-side logic of libpolar (no GPU needed): exported symbols, argument
validation, construction, schedule and encoder against the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1504_00353_amd import binding, synth, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polar.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(polar_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(binding.EXPORTS)


def test_invalid_arguments_are_rejected():
    L = binding.lib()
    for n, k in [(0, 0), (3, 1), (6, 3), (65536, 100), (8, 0), (8, 9), (-8, 4)]:
        assert not L.polar_construct(n, k, 2.0)
        assert L.polar_last_status() == binding.EINVAL
    assert not L.polar_construct_mask(8, None)
    assert L.polar_last_status() == binding.EINVAL
    allfrozen = np.ones(8, np.uint8)
    assert not L.polar_construct_mask(8, allfrozen.ctypes.data_as(ctypes.c_void_p))
    bad = np.array([0, 2, 0, 0], np.uint8)
    assert not L.polar_construct_mask(4, bad.ctypes.data_as(ctypes.c_void_p))
    c = binding.Code(64, 32, 2.5, prepare=False)
    assert L.polar_configure(c.handle, 7, 0) == binding.EINVAL
    assert L.polar_configure(c.handle, 0, 9) == binding.EINVAL
    # decode before prepare
    assert L.polar_decode(c.handle, ctypes.c_void_p(16), 1, ctypes.c_void_p(16), None) == binding.ESTATE
    assert L.polar_decode(c.handle, None, -1, None, None) == binding.EINVAL
    assert L.polar_decode(None, None, 1, None, None) == binding.EINVAL
    assert L.polar_schedule(None, None, None, None, 0, None) == binding.EINVAL
    assert L.polar_encode(c.handle, None, 1, None) == binding.EINVAL
    assert L.polar_n(None) == 0 and L.polar_k(None) == 0
    assert L.polar_set_kernel(c.handle, 2) == binding.EINVAL
    assert L.polar_set_kernel(None, 0) == binding.EINVAL
    assert L.polar_build_kernel(None) == binding.EINVAL
    L.polar_destroy(None)
    assert binding.lib().polar_strerror(binding.ESTATE) == b"invalid state"
    assert binding.lib().polar_strerror(binding.ECOMPILE) == b"kernel compilation failed"


def test_unrolled_kernel_builds_into_cache(tmp_path, monkeypatch):
    """polar_build_kernel compiles a code's unrolled kernel on the host into
    the cache directory; a second build is a cache hit; another code or
    LLR type gets another code object."""
    import time
    monkeypatch.setenv("POLAR_KERNEL_CACHE", str(tmp_path))
    fr = np.array([1, 1, 0, 0, 1, 0, 0, 0], np.uint8)
    c = binding.Code(frozen=fr, prepare=False, kernel="unrolled")
    c.build_kernel()
    files = sorted(os.listdir(tmp_path))
    assert len(files) == 1 and files[0].endswith(".hsaco")
    blob = open(os.path.join(tmp_path, files[0]), "rb").read()
    assert blob[:4] == b"\x7fELF" and b"polar_unrolled_trace" in blob and b"polar_unrolled" in blob
    t0 = time.perf_counter()
    c.build_kernel()
    assert time.perf_counter() - t0 < 0.5
    assert sorted(os.listdir(tmp_path)) == files
    binding.Code(frozen=fr, llr="f32", prepare=False, kernel="unrolled").build_kernel()
    binding.Code(frozen=fr, algo="sc", prepare=False, kernel="unrolled").build_kernel()
    assert len(os.listdir(tmp_path)) == 3


CODES = sorted({(n, k, d) for w in workloads.ALL for (n, k, d) in w["codes"]} | {(8, 5, 2.0), (64, 32, 2.5)})


@pytest.mark.parametrize("n,k,d", CODES)
def test_construction_matches_oracle(n, k, d):
    c = binding.Code(n, k, d, prepare=False)
    assert c.n == n and c.k == k
    assert np.array_equal(c.frozen(), oracle.construct(n, k, d))


def random_mask(n, rng, p):
    m = (rng.random(n) < p).astype(np.uint8)
    if m.all():
        m[rng.integers(0, n)] = 0
    return m


@pytest.mark.parametrize("algo", ["fastssc", "sc"])
def test_schedule_matches_oracle_walk(algo):
    rng = np.random.default_rng(5)
    masks = [oracle.construct(n, k, d) for (n, k, d) in CODES if n <= 4096 or algo == "fastssc"]
    masks += [random_mask(n, rng, p) for n in (2, 4, 8, 16, 64, 256, 1024) for p in (0.2, 0.5, 0.8)]
    for fr in masks:
        c = binding.Code(frozen=fr, algo=algo, prepare=False)
        mine = [(name, size) for name, size, _ in c.schedule()]
        assert mine == oracle.schedule(fr, algo)


def test_listing1_schedule_offsets():
    fr = np.array([1, 1, 0, 0, 1, 0, 0, 0], np.uint8)
    c = binding.Code(frozen=fr, prepare=False)
    assert c.schedule() == [("F", 8, 0), ("G_0R", 4, 0), ("Info", 2, 2), ("Combine_0R", 4, 0),
                            ("G", 8, 0), ("SPC", 4, 4), ("Combine", 8, 0)]


@pytest.mark.parametrize("n,k,d", [(8, 5, 2.0), (64, 32, 2.5), (1024, 922, 4.0), (32768, 29492, 4.0)])
def test_encoder_matches_oracle(n, k, d):
    c = binding.Code(n, k, d, prepare=False)
    fr = c.frozen()
    bits = synth.info_bits(9, np.arange(6), k)
    x = c.encode(synth.pack_bits(bits))
    expect = oracle.encode(synth.scatter_info(bits, fr))
    assert np.array_equal(synth.unpack_bits(x, n), expect)


def test_unrolled_kernel_builds_with_torch_loaded(tmp_path):
    """In a process that imported torch first, the HIP run-time compiler
    runs on the compiler library torch brought along; the generated source
    must compile there too (the kernel cache may be filled from such a
    process)."""
    import subprocess
    import sys
    code = (
        "import torch, sys, numpy as np\n"
        "sys.path.insert(0, %r)\n"
        "from paper_1504_00353_amd import binding\n"
        "fr = np.array([1, 1, 0, 0, 1, 0, 0, 0], np.uint8)\n"
        "for llr in ('i8', 'f32'):\n"
        "    binding.Code(frozen=fr, llr=llr, prepare=False, kernel='unrolled').build_kernel()\n"
        "binding.Code(256, 128, 2.5, prepare=False, kernel='unrolled').build_kernel()\n"
        "print('built')\n" % ROOT)
    env = dict(os.environ, POLAR_KERNEL_CACHE=str(tmp_path))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "built" in r.stdout, r.stdout + r.stderr
    assert len(os.listdir(tmp_path)) == 3


def test_batch_arguments_and_build(tmp_path, monkeypatch):
    """Batch creation checks its codes; set_frames before prepare is out of
    order; the batch kernel of two small codes builds on the host."""
    L = binding.lib()
    monkeypatch.setenv("POLAR_KERNEL_CACHE", str(tmp_path))
    assert not L.polar_batch_create(None, 1)
    assert L.polar_last_status() == binding.EINVAL
    a = binding.Code(64, 32, 2.5, prepare=False)
    b = binding.Code(128, 100, 4.0, llr="f32", prepare=False)
    arr = (ctypes.c_void_p * 2)(a.handle.value, b.handle.value)
    assert not L.polar_batch_create(arr, 2)  # mixed LLR types
    assert L.polar_last_status() == binding.EINVAL
    c = binding.Code(128, 100, 4.0, prepare=False)
    bt = binding.Batch([a, c], prepare=False)
    with pytest.raises(binding.PolarError):
        bt.set_frames([0], [0], [0])  # not prepared
    bt.build_kernel()
    assert len(os.listdir(tmp_path)) == 1
    assert L.polar_batch_decode(None, None, None, None) == binding.EINVAL
    L.polar_batch_destroy(None)


def _leaf_kind(fr, o, size):
    f = fr[o:o + size]
    nf = int(f.sum())
    if nf == size:
        return "R0"
    if nf == 0:
        return "R1"
    if size >= 2 and nf == size - 1 and not f[-1]:
        return "REP"
    if size >= 4 and nf == 1 and f[0]:
        return "SPC"
    return None


def _expected_pairs(fr):
    """(op, stage, offset) of every internal node of size <= 64 whose
    children are Rate-0 / repetition (left) and Rate-1 / SPC (right), in
    depth-first order."""
    names = {("R0", "R1"): "P_01", ("R0", "SPC"): "0SPC", ("REP", "SPC"): "RepSPC", ("REP", "R1"): "Rep-R1"}
    out = []

    def walk(o, size):
        if _leaf_kind(fr, o, size) is not None:
            return
        h = size // 2
        key = (_leaf_kind(fr, o, h), _leaf_kind(fr, o + h, h))
        if size <= 64 and key in names:
            out.append((names[key], size.bit_length() - 1, o))
            return
        walk(o, h)
        walk(o + h, h)
    walk(0, len(fr))
    return out


def test_fused_leaf_pairs_in_device_schedule():
    """The device schedule holds one fused op per leaf-pair node of size
    <= 64 and none of the separate ops inside it; with the fusion off (or
    for plain SC) it holds no fused op."""
    from paper_1504_00353_amd import workloads
    rng = np.random.default_rng(9)
    masks = [np.asarray(workloads.UNROLLED_MASKS["m2k_leaf_pairs"][1], np.uint8), oracle.construct(32768, 29492, 4.0),
             oracle.construct(1024, 512, 2.5)]
    masks += [random_mask(n, rng, p) for n in (8, 64, 256, 1024) for p in (0.3, 0.5, 0.7)]
    fused_names = ("P_01", "0SPC", "RepSPC", "Rep-R1")
    for fr in masks:
        on = binding.Code(frozen=fr, prepare=False).device_schedule()
        off = binding.Code(frozen=fr, prepare=False, fused=False).device_schedule()
        assert [t for t in on if t[0] in fused_names] == _expected_pairs(fr)
        assert not [t for t in off if t[0] in fused_names]
        sc = binding.Code(frozen=fr, algo="sc", prepare=False).device_schedule()
        assert not [t for t in sc if t[0] in fused_names]
        # a fused node replaces 5 (repetition left) or 3 (Rate-0 left) ops,
        # 4 or 2 when its estimate is never read again (no combine)
        saved = len(off) - len(on)
        pairs = _expected_pairs(fr)
        lo = sum(3 if name.startswith("Rep") else 1 for name, _, _ in pairs)
        hi = sum(4 if name.startswith("Rep") else 2 for name, _, _ in pairs)
        assert lo <= saved <= hi
    pairs = _expected_pairs(np.asarray(workloads.UNROLLED_MASKS["m2k_leaf_pairs"][1], np.uint8))
    for name in fused_names:
        assert {st for nm, st, _ in pairs if nm == name} >= ({2, 3, 4, 5, 6} if name == "P_01" else {3, 4, 5, 6})


def test_set_fused_nodes_arguments():
    L = binding.lib()
    c = binding.Code(64, 32, 2.5, prepare=False)
    assert L.polar_set_fused_nodes(c.handle, 2) == binding.EINVAL
    assert L.polar_set_fused_nodes(None, 1) == binding.EINVAL
    assert L.polar_device_schedule(None, None, 0, None) == binding.EINVAL
    assert L.polar_set_fused_nodes(c.handle, 0) == binding.OK


def test_layout_candidates_and_arguments():
    """Layouts of the unrolled kernels: index 0 is the default rule, every
    candidate satisfies the decoder templates' constraints, and the LDS slot
    follows from the register stages."""
    L = binding.lib()
    c = binding.Code(32768, 29492, 4.0, prepare=False, kernel="unrolled")
    lay = c.layouts()
    assert lay[0] == {"reg_stages": 2, "virtual_top": 1, "virtual_mid": 0, "wave_lds_bytes": 8192}
    assert len(lay) == len({(x["reg_stages"], x["virtual_top"]) for x in lay})
    for x in lay:  # int8: register stages of >= 2^11 LLRs, at most 3
        assert 1 <= x["reg_stages"] <= 3 and 15 - x["virtual_top"] - x["reg_stages"] >= 11
        assert x["virtual_mid"] == 0
    f = binding.Code(32768, 29492, 4.0, llr="f32", prepare=False, kernel="unrolled")
    fl = f.layouts()
    # float N = 32768: stage 14 and stage 12 recomputed, stage 13 in registers,
    # stages 7..11 (15,872 B) + sign table + beta in LDS
    assert fl[0] == {"reg_stages": 1, "virtual_top": 1, "virtual_mid": 1, "wave_lds_bytes": 20096}
    assert fl[1] == {"reg_stages": 1, "virtual_top": 1, "virtual_mid": 0, "wave_lds_bytes": 36480}
    assert all(x["reg_stages"] <= x["virtual_top"] and x["virtual_mid"] <= x["reg_stages"] for x in fl)
    h = binding.Code(16384, 14746, 4.0, llr="f32", prepare=False, kernel="unrolled")
    assert all(x["virtual_mid"] == 0 for x in h.layouts())
    s = binding.Code(1024, 512, 2.5, prepare=False, kernel="unrolled")
    assert s.layouts() == [{"reg_stages": 0, "virtual_top": 0, "virtual_mid": 0, "wave_lds_bytes": 1152}]
    assert L.polar_layout_count(None) == 0
    assert L.polar_set_layout(c.handle, -1) == binding.EINVAL
    assert L.polar_set_layout(c.handle, len(lay)) == binding.EINVAL
    assert L.polar_layout_info(c.handle, len(lay), None, None, None, None) == binding.EINVAL
    assert L.polar_set_layout(c.handle, len(lay) - 1) == binding.OK
    assert L.polar_tune_layout(c.handle, None, 1, None, None, None) == binding.EINVAL
    assert L.polar_tune_layout(c.handle, ctypes.c_void_p(18), 1, ctypes.c_void_p(16), None, None) == binding.EINVAL
    assert L.polar_tune_layout(c.handle, ctypes.c_void_p(16), 0, ctypes.c_void_p(16), None, None) == binding.EINVAL
    sched = binding.Code(32768, 29492, 4.0, prepare=False, kernel="schedule")
    assert L.polar_tune_layout(sched.handle, ctypes.c_void_p(16), 1, ctypes.c_void_p(16), None, None) == binding.ESTATE


def test_virtual_top_only_without_top_decision_nodes():
    """A code whose root child is a decision node cannot use the virtual top
    stage: no candidate offers it."""
    fr = np.zeros(16384, np.uint8)
    fr[:8192] = 1  # left half Rate-0, right half Rate-1: decision node of size N/2
    c = binding.Code(frozen=fr, prepare=False, kernel="unrolled")
    assert all(x["virtual_top"] == 0 for x in c.layouts())


def test_configure_resets_layout():
    """The layout index refers to the candidates of the configuration it was
    chosen in; reconfiguring returns to the default."""
    L = binding.lib()
    c = binding.Code(32768, 29492, 4.0, prepare=False, kernel="unrolled", layout=3)
    assert L.polar_configure(c.handle, 0, 1) == binding.OK  # float LLRs: 4 candidates
    assert L.polar_layout_count(c.handle) == 4
    assert L.polar_set_layout(c.handle, 3) == binding.OK
    assert L.polar_set_fused_nodes(c.handle, 0) == binding.OK
    assert L.polar_set_layout(c.handle, 4) == binding.EINVAL


def test_allocation_failure_hook_objects():
    """Failure handling: an armed allocation failure makes the object
    allocation of polar_construct / polar_batch_create return NULL with
    POLAR_ENOMEM, once; the next call succeeds."""
    L = binding.lib()
    try:
        assert L.polar_debug_fail_allocations(0) == binding.OK
        assert not L.polar_construct(64, 32, 2.5)
        assert L.polar_last_status() == binding.ENOMEM
        h = L.polar_construct(64, 32, 2.5)
        assert h
        L.polar_destroy(h)
        c = binding.Code(64, 32, 2.5, prepare=False)
        arr = (ctypes.c_void_p * 1)(c.handle.value)
        L.polar_debug_fail_allocations(0)
        assert not L.polar_batch_create(arr, 1)
        assert L.polar_last_status() == binding.ENOMEM
        b = L.polar_batch_create(arr, 1)
        assert b
        L.polar_batch_destroy(b)
        # the countdown: the second allocation from now fails
        L.polar_debug_fail_allocations(1)
        h1 = L.polar_construct(64, 32, 2.5)
        assert h1
        assert not L.polar_construct(64, 32, 2.5)
        assert L.polar_last_status() == binding.ENOMEM
        L.polar_destroy(h1)
        L.polar_debug_fail_allocations(-1)
        h = L.polar_construct(64, 32, 2.5)
        assert h
        L.polar_destroy(h)
    finally:
        L.polar_debug_fail_allocations(-1)


@pytest.mark.parametrize("n,k,d", [(1024, 512, 2.5), (4096, 3686, 4.0)])
def test_benchmark_inputs_match_oracle_encoded_frames(n, k, d):
    """The benchmark's and the study's channel frames (library encoder,
    threaded) are the frames the tests build with the oracle's encoder."""
    from frames import make_frames
    from paper_1504_00353_amd import inputs
    c = binding.Code(n, k, d, prepare=False)
    ids = np.arange(37) * 3 + 5
    l32, info = inputs.channel_frames(c, 11, ids, d + 0.5, threads=4)
    u, _, ref = make_frames(c.frozen(), 11, ids, d + 0.5, llr="f32")
    assert np.array_equal(l32, ref)
    assert np.array_equal(info, u[:, c.frozen() == 0])
