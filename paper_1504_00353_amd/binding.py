"""ctypes binding over libpolar.so (include/polar.h).

Argument marshalling only: every step of decoding runs in the library's HIP
kernels.  Device buffers are torch tensors (memory and streams only).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# POLAR_LIBRARY: another build of the same library (the sanitizer test
# loads an ASan/UBSan build of the host code through it)
SO_PATH = os.environ.get("POLAR_LIBRARY") or os.path.join(_HERE, "libpolar.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ECOMPILE, EAGAIN = 0, 1, 2, 3, 4, 5, 6
ALGO = {"fastssc": 0, "sc": 1}
LLR = {"i8": 0, "f32": 1}
KERNEL = {"schedule": 0, "unrolled": 1}
OP_NAMES = ["F", "G", "G_0R", "Combine", "Combine_0R", "Info", "Repetition", "SPC"]
DEV_OP_NAMES = ["F", "G", "G_0R", "Combine", "Combine_0R", "Combine_R0", "Info", "Repetition", "SPC", "Flush",
                "End", "P_01", "0SPC", "RepSPC", "Rep-R1"]
EXPORTS = [
    "polar_construct", "polar_construct_mask", "polar_configure", "polar_prepare", "polar_destroy",
    "polar_last_status", "polar_strerror", "polar_n", "polar_k", "polar_frozen_mask", "polar_schedule",
    "polar_encode", "polar_decode", "polar_decode_trace", "polar_set_kernel", "polar_set_fused_nodes",
    "polar_device_schedule", "polar_layout_count", "polar_layout_info", "polar_set_layout", "polar_tune_layout",
    "polar_build_kernel",
    "polar_last_message", "polar_batch_create", "polar_batch_build_kernel", "polar_batch_prepare",
    "polar_batch_set_frames", "polar_batch_decode", "polar_batch_decode_desc", "polar_batch_tune",
    "polar_batch_decode_frames_noalloc", "polar_debug_fail_allocations",
    "polar_batch_launch_shape", "polar_batch_destroy", "polar_server_create", "polar_server_submit",
    "polar_server_poll", "polar_server_pending", "polar_server_destroy", "polar_server_run_trace",
    "polar_server_device_bytes",
]


class PolarError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        detail = _lib().polar_last_message().decode(errors="replace")
        super().__init__("%s: %s%s" % (what, _lib().polar_strerror(status).decode(),
                                       ("\n" + detail) if detail else ""))


_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError("libpolar.so is not built (run __graft_entry__.build()); "
                               "there is no fallback decoder")
        L = ctypes.CDLL(SO_PATH)
        P, I = ctypes.c_void_p, ctypes.c_int
        L.polar_construct.argtypes = [I, I, ctypes.c_double]
        L.polar_construct.restype = P
        L.polar_construct_mask.argtypes = [I, P]
        L.polar_construct_mask.restype = P
        L.polar_configure.argtypes = [P, I, I]
        L.polar_prepare.argtypes = [P]
        L.polar_set_kernel.argtypes = [P, I]
        L.polar_set_fused_nodes.argtypes = [P, I]
        L.polar_device_schedule.argtypes = [P, P, I, P]
        L.polar_layout_count.argtypes = [P]
        L.polar_layout_info.argtypes = [P, I, P, P, P, P]
        L.polar_set_layout.argtypes = [P, I]
        L.polar_tune_layout.argtypes = [P, P, I, P, P, P]
        L.polar_build_kernel.argtypes = [P]
        L.polar_destroy.argtypes = [P]
        L.polar_destroy.restype = None
        L.polar_last_status.argtypes = []
        L.polar_strerror.argtypes = [I]
        L.polar_strerror.restype = ctypes.c_char_p
        L.polar_last_message.argtypes = []
        L.polar_last_message.restype = ctypes.c_char_p
        L.polar_debug_fail_allocations.argtypes = [I]
        L.polar_n.argtypes = [P]
        L.polar_k.argtypes = [P]
        L.polar_frozen_mask.argtypes = [P, P]
        L.polar_schedule.argtypes = [P, P, P, P, I, P]
        L.polar_encode.argtypes = [P, P, I, P]
        L.polar_decode.argtypes = [P, P, I, P, P]
        L.polar_decode_trace.argtypes = [P, P, I, P, P, P]
        L.polar_batch_create.argtypes = [P, I]
        L.polar_batch_create.restype = P
        L.polar_batch_build_kernel.argtypes = [P]
        L.polar_batch_prepare.argtypes = [P]
        L.polar_batch_set_frames.argtypes = [P, I, P, P, P]
        L.polar_batch_decode.argtypes = [P, P, P, P]
        L.polar_batch_decode_desc.argtypes = [P, P, I, P, P, P]
        L.polar_batch_tune.argtypes = [P, P, P, P]
        L.polar_batch_decode_frames_noalloc.argtypes = [P, I, P, P, P, P, P, P]
        L.polar_batch_launch_shape.argtypes = [P, P, P, P]
        L.polar_batch_destroy.argtypes = [P]
        L.polar_batch_destroy.restype = None
        L.polar_server_create.argtypes = [P, P, I, I, I, ctypes.c_size_t, ctypes.c_size_t]
        L.polar_server_create.restype = P
        L.polar_server_submit.argtypes = [P, I, I, P, I, P, P]
        L.polar_server_poll.argtypes = [P, P, I, P]
        L.polar_server_pending.argtypes = [P, P, P, P]
        L.polar_server_device_bytes.argtypes = [P, P, P]
        L.polar_server_destroy.argtypes = [P]
        L.polar_server_destroy.restype = None
        L.polar_server_run_trace.argtypes = [P, I, P, P, P, P, P, P]
        _L = L
    return _L


def lib():
    return _lib()


def _check(rc, what):
    if rc != OK:
        raise PolarError(rc, what)


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Code:
    """A polar code plus its decoder schedule (host) and device tables."""

    def __init__(self, n=None, k=None, design_db=None, algo="fastssc", llr="i8", frozen=None, prepare=True,
                 kernel="schedule", fused=True, layout=0):
        L = _lib()
        if frozen is not None:
            frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
            h = L.polar_construct_mask(int(frozen.shape[0]), _np_ptr(frozen))
        else:
            h = L.polar_construct(int(n), int(k), float(design_db))
        if not h:
            raise PolarError(L.polar_last_status(), "polar_construct")
        self._h = ctypes.c_void_p(h)
        self.n = L.polar_n(self._h)
        self.k = L.polar_k(self._h)
        self.algo, self.llr = algo, llr
        _check(L.polar_configure(self._h, ALGO[algo], LLR[llr]), "polar_configure")
        self.kernel = kernel
        _check(L.polar_set_kernel(self._h, KERNEL[kernel]), "polar_set_kernel")
        self.fused = bool(fused)
        _check(L.polar_set_fused_nodes(self._h, 1 if fused else 0), "polar_set_fused_nodes")
        self.layout = int(layout)
        _check(L.polar_set_layout(self._h, self.layout), "polar_set_layout")
        self.prepared = False
        if prepare:
            self.prepare()

    def prepare(self):
        _check(_lib().polar_prepare(self._h), "polar_prepare")
        self.prepared = True

    def build_kernel(self):
        """Compile this code's unrolled kernel into the kernel cache (host only)."""
        _check(_lib().polar_build_kernel(self._h), "polar_build_kernel")

    def layouts(self):
        """The unrolled kernel's candidate layouts, the default first: dicts
        of reg_stages, virtual_top, virtual_mid and wave_lds_bytes."""
        L = _lib()
        out = []
        for i in range(L.polar_layout_count(self._h)):
            r, v, b, m = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
            _check(L.polar_layout_info(self._h, i, ctypes.byref(r), ctypes.byref(v), ctypes.byref(b), ctypes.byref(m)),
                   "polar_layout_info")
            out.append({"reg_stages": r.value, "virtual_top": v.value, "virtual_mid": m.value,
                        "wave_lds_bytes": b.value})
        return out

    def set_layout(self, index):
        _check(_lib().polar_set_layout(self._h, int(index)), "polar_set_layout")
        self.layout = int(index)

    def tune_layout(self, llr, out=None, stream=None):
        """Time every layout on these frames and prepare the code with the
        fastest (unrolled kernel, before prepare); returns its index."""
        import torch
        self._check_llr(llr)
        if out is None:
            out = torch.empty((llr.shape[0], self.row_bytes), dtype=torch.uint8, device=llr.device)
        chosen = ctypes.c_int(-1)
        _check(_lib().polar_tune_layout(self._h, ctypes.c_void_p(llr.data_ptr()), llr.shape[0],
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream),
                                        ctypes.byref(chosen)), "polar_tune_layout")
        self.layout = chosen.value
        self.prepared = True
        return chosen.value

    def close(self):
        if getattr(self, "_h", None):
            _lib().polar_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def row_bytes(self):
        return (self.k + 7) // 8

    def frozen(self):
        out = np.zeros(self.n, np.uint8)
        _check(_lib().polar_frozen_mask(self._h, _np_ptr(out)), "polar_frozen_mask")
        return out

    def device_schedule(self):
        """The device op words the kernels run: (op, stage, offset) with op a
        DEV_OP_NAMES entry."""
        L = _lib()
        cnt = ctypes.c_int(0)
        _check(L.polar_device_schedule(self._h, None, 0, ctypes.byref(cnt)), "polar_device_schedule")
        w = np.zeros(max(cnt.value, 1), np.uint32)
        _check(L.polar_device_schedule(self._h, _np_ptr(w), cnt.value, ctypes.byref(cnt)), "polar_device_schedule")
        return [(DEV_OP_NAMES[int(x) & 255], (int(x) >> 8) & 255, int(x) >> 16) for x in w[:cnt.value]]

    def schedule(self):
        cnt = ctypes.c_int(0)
        _check(_lib().polar_schedule(self._h, None, None, None, 0, ctypes.byref(cnt)), "polar_schedule")
        k = np.zeros(cnt.value, np.int32)
        s = np.zeros(cnt.value, np.int32)
        o = np.zeros(cnt.value, np.int32)
        _check(_lib().polar_schedule(self._h, _np_ptr(k), _np_ptr(s), _np_ptr(o), cnt.value, ctypes.byref(cnt)),
               "polar_schedule")
        return [(OP_NAMES[a], int(b), int(c)) for a, b, c in zip(k, s, o)]

    def encode(self, info_packed):
        """Host encoder: [frames, ceil(K/8)] packed info rows -> [frames, ceil(N/8)]."""
        info = np.ascontiguousarray(np.atleast_2d(info_packed), dtype=np.uint8)
        x = np.zeros((info.shape[0], (self.n + 7) // 8), np.uint8)
        _check(_lib().polar_encode(self._h, _np_ptr(info), info.shape[0], _np_ptr(x)), "polar_encode")
        return x

    def _check_llr(self, llr):
        import torch
        want = torch.int8 if self.llr == "i8" else torch.float32
        if llr.dtype != want or not llr.is_cuda or not llr.is_contiguous() or llr.dim() != 2 or llr.shape[1] != self.n:
            raise ValueError("llr must be a contiguous CUDA %s tensor [frames, %d]" % (want, self.n))

    def decode(self, llr, out=None, stream=None):
        """Decode [frames, N] LLRs on the GPU; returns [frames, ceil(K/8)] uint8."""
        import torch
        self._check_llr(llr)
        frames = llr.shape[0]
        if out is None:
            out = torch.empty((frames, self.row_bytes), dtype=torch.uint8, device=llr.device)
        _check(_lib().polar_decode(self._h, ctypes.c_void_p(llr.data_ptr()), frames,
                                   ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), "polar_decode")
        return out

    def decode_trace(self, llr, out=None, trace=None, stream=None):
        """decode() plus the leaf-LLR trace [frames, N] (LLR dtype)."""
        import torch
        self._check_llr(llr)
        frames = llr.shape[0]
        if out is None:
            out = torch.empty((frames, self.row_bytes), dtype=torch.uint8, device=llr.device)
        if trace is None:
            trace = torch.zeros_like(llr)
        _check(_lib().polar_decode_trace(self._h, ctypes.c_void_p(llr.data_ptr()), frames,
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(trace.data_ptr()),
                                         _stream_handle(stream)), "polar_decode_trace")
        return out, trace


class Batch:
    """Frames of several codes (one LLR type) decoded in one persistent
    launch; see polar_batch_* in include/polar.h."""

    def __init__(self, codes, prepare=True):
        L = _lib()
        self.codes = list(codes)
        arr = (ctypes.c_void_p * len(self.codes))(*[c.handle.value for c in self.codes])
        h = L.polar_batch_create(arr, len(self.codes))
        if not h:
            raise PolarError(L.polar_last_status(), "polar_batch_create")
        self._h = ctypes.c_void_p(h)
        self.llr = self.codes[0].llr
        self.nframes = 0
        if prepare:
            self.prepare()

    def build_kernel(self):
        _check(_lib().polar_batch_build_kernel(self._h), "polar_batch_build_kernel")

    def prepare(self):
        _check(_lib().polar_batch_prepare(self._h), "polar_batch_prepare")

    def set_frames(self, code_index, llr_offset, bits_offset):
        ci = np.ascontiguousarray(code_index, dtype=np.int32)
        lo = np.ascontiguousarray(llr_offset, dtype=np.int64)
        bo = np.ascontiguousarray(bits_offset, dtype=np.int64)
        if not (ci.shape == lo.shape == bo.shape) or ci.ndim != 1:
            raise ValueError("code_index, llr_offset and bits_offset must be 1-D of one length")
        _check(_lib().polar_batch_set_frames(self._h, ci.shape[0], _np_ptr(ci), _np_ptr(lo), _np_ptr(bo)),
               "polar_batch_set_frames")
        self.nframes = int(ci.shape[0])

    def decode(self, llr, bits, stream=None):
        """Decode the described frames: llr and bits are flat CUDA tensors
        (LLR dtype / uint8) that the descriptors' offsets index."""
        _check(_lib().polar_batch_decode(self._h, ctypes.c_void_p(llr.data_ptr()), ctypes.c_void_p(bits.data_ptr()),
                                         _stream_handle(stream)), "polar_batch_decode")
        return bits

    def decode_desc(self, desc, nframes, llr, bits, stream=None):
        _check(_lib().polar_batch_decode_desc(self._h, ctypes.c_void_p(desc.data_ptr()), int(nframes),
                                              ctypes.c_void_p(llr.data_ptr()), ctypes.c_void_p(bits.data_ptr()),
                                              _stream_handle(stream)), "polar_batch_decode_desc")
        return bits

    def decode_frames_noalloc(self, code_index, llr_offset, bits_offset, llr, bits, stream=None):
        """polar_batch_decode_frames_noalloc: the frames' code indices (int32)
        and LLR / bits offsets (int64) are 1-D CUDA tensors of one length;
        llr and bits as for decode."""
        import torch
        n = int(code_index.numel())
        if not (code_index.dtype == torch.int32 and llr_offset.dtype == torch.int64 == bits_offset.dtype and
                llr_offset.numel() == n == bits_offset.numel()):
            raise ValueError("code_index int32, llr_offset and bits_offset int64, all of one length")
        for t in (code_index, llr_offset, bits_offset):
            if not t.is_contiguous():
                raise ValueError("frame arrays must be contiguous")
        _check(_lib().polar_batch_decode_frames_noalloc(
            self._h, n, ctypes.c_void_p(code_index.data_ptr()), ctypes.c_void_p(llr_offset.data_ptr()),
            ctypes.c_void_p(bits_offset.data_ptr()), ctypes.c_void_p(llr.data_ptr()),
            ctypes.c_void_p(bits.data_ptr()), _stream_handle(stream)), "polar_batch_decode_frames_noalloc")
        return bits

    def tune(self, llr, bits, stream=None):
        _check(_lib().polar_batch_tune(self._h, ctypes.c_void_p(llr.data_ptr()), ctypes.c_void_p(bits.data_ptr()),
                                       _stream_handle(stream)), "polar_batch_tune")
        return self.launch_shape()

    def launch_shape(self):
        w, b, l = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _check(_lib().polar_batch_launch_shape(self._h, ctypes.byref(w), ctypes.byref(b), ctypes.byref(l)),
               "polar_batch_launch_shape")
        return {"waves_per_block": w.value, "blocks": b.value, "wave_lds_bytes": l.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib().polar_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server over a prepared Batch; see
    polar_server_* in include/polar.h.  One thread drives it."""

    def __init__(self, batch, slots_per_class=4096, streams=2, staging_bytes=256 << 20, device_bytes=1 << 30):
        L = _lib()
        self.batch = batch
        codes = batch.codes
        arr = (ctypes.c_void_p * len(codes))(*[c.handle.value for c in codes])
        h = L.polar_server_create(batch._h, arr, len(codes), int(slots_per_class), int(streams), int(staging_bytes),
                                  int(device_bytes))
        if not h:
            raise PolarError(L.polar_last_status(), "polar_server_create")
        self._h = ctypes.c_void_p(h)
        self._done = np.zeros(4096, np.int64)
        self._keep = {}

    def submit(self, code_index, llr, bits):
        """llr: numpy array (host) or CUDA tensor (device, read in place)
        [frames, N]; bits: numpy uint8 [frames, ceil(K/8)] (filled when the
        request completes) or a CUDA uint8 tensor (written in place).
        Returns the request id, or None if the staging memory is full
        (poll and retry)."""
        rid = ctypes.c_int64(0)
        where = 0
        if hasattr(llr, "data_ptr") or hasattr(bits, "data_ptr"):
            # the server's streams wait for no other stream: device buffers
            # must be ready at submit (include/polar.h, polar_server_submit)
            import torch
            torch.cuda.current_stream().synchronize()
        if hasattr(llr, "data_ptr"):
            ptr, frames = llr.data_ptr(), llr.shape[0]
            where |= 1
        else:
            llr = np.ascontiguousarray(llr)
            ptr, frames = llr.ctypes.data, llr.shape[0]
        if hasattr(bits, "data_ptr"):
            bptr = bits.data_ptr()
            where |= 2
        else:
            bptr = bits.ctypes.data
        rc = _lib().polar_server_submit(self._h, int(code_index), int(frames), ctypes.c_void_p(ptr), where,
                                        ctypes.c_void_p(bptr), ctypes.byref(rid))
        if rc == EAGAIN:
            return None
        _check(rc, "polar_server_submit")
        self._keep[rid.value] = (llr, bits)
        return rid.value

    def poll(self):
        """Progress; returns the ids of requests completed by this call."""
        n = ctypes.c_int(0)
        _check(_lib().polar_server_poll(self._h, _np_ptr(self._done), self._done.shape[0], ctypes.byref(n)),
               "polar_server_poll")
        ids = [int(x) for x in self._done[:min(n.value, self._done.shape[0])]]
        for i in ids:
            self._keep.pop(i, None)
        return ids

    def run_trace(self, arrival_s, code_index, nframes, llr_ptrs, bits_ptrs):
        """Native load generator: submits request i at arrival_s[i] seconds
        (device LLR / bits addresses), polls until all are done; returns
        the completion times (seconds, same clock)."""
        a = np.ascontiguousarray(arrival_s, np.float64)
        c = np.ascontiguousarray(code_index, np.int32)
        f = np.ascontiguousarray(nframes, np.int32)
        lp = np.ascontiguousarray(llr_ptrs, np.uint64)
        bp = np.ascontiguousarray(bits_ptrs, np.uint64)
        done = np.zeros(a.shape[0], np.float64)
        _check(_lib().polar_server_run_trace(self._h, a.shape[0], _np_ptr(a), _np_ptr(c), _np_ptr(f), _np_ptr(lp),
                                             _np_ptr(bp), _np_ptr(done)), "polar_server_run_trace")
        return done

    def device_bytes(self):
        """(caller device bytes referenced by admitted, unfinished requests,
        the budget)."""
        used, budget = ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(_lib().polar_server_device_bytes(self._h, ctypes.byref(used), ctypes.byref(budget)),
               "polar_server_device_bytes")
        return used.value, budget.value

    def pending(self):
        w, a, f = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _check(_lib().polar_server_pending(self._h, ctypes.byref(w), ctypes.byref(a), ctypes.byref(f)),
               "polar_server_pending")
        return w.value, a.value, f.value

    def drain(self):
        """Polls until nothing is waiting or in flight; returns completed ids."""
        done = []
        while True:
            done += self.poll()
            if self.pending() == (0, 0, 0) and not self._keep:
                return done

    def close(self):
        if getattr(self, "_h", None):
            _lib().polar_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
