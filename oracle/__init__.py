"""ctypes wrapper over the plain CPU oracle in ``oracle.cpp``.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark use this package.  The product library never
imports it, and it imports nothing from the product library.

Every function here takes and returns numpy arrays; bits are one per byte
(0/1) in natural index order.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
# POLAR_ORACLE_LIBRARY: another build of oracle.cpp (the sanitizer test)
_SO = os.environ.get("POLAR_ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")

ALGO = {"fastssc": 0, "sc": 1}
KIND = {"rate1": 1, "rep": 2, "spc": 3}
LOG_NAMES = ["F", "G", "G_0R", "Combine", "Combine_0R", "Info", "Repetition", "SPC"]


def build(force=True):
    """Compile oracle.cpp with g++ (no hand-written SIMD, no FP contraction)."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I = ctypes.c_int
        L.oracle_construct.argtypes = [I, I, ctypes.c_double, P]
        L.oracle_encode.argtypes = [I, I, P, P]
        L.oracle_bhattacharyya.argtypes = [I, ctypes.c_double, P]
        L.oracle_construct_lnz.argtypes = [I, I, ctypes.c_double, P, P]
        for name in ("oracle_decode_i8", "oracle_decode_f32", "oracle_decode_f64"):
            getattr(L, name).argtypes = [I, P, I, I, P, P, P, P, I]
        L.oracle_schedule.argtypes = [I, P, I, P, P, I]
        L.oracle_node_i8.argtypes = [I, I, P, P]
        L.oracle_node_f64.argtypes = [I, I, P, P]
        L.oracle_f_i8.argtypes = [I, I]
        L.oracle_g_i8.argtypes = [I, I, I]
        L.oracle_f_f64.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_f_f64.restype = ctypes.c_double
        L.oracle_g_f64.argtypes = [ctypes.c_double, ctypes.c_double, I]
        L.oracle_g_f64.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def construct(n, k, design_ebn0_db):
    """Frozen mask (1 = frozen) by the Bhattacharyya bound at the design Eb/N0."""
    frozen = np.zeros(n, np.uint8)
    rc = lib().oracle_construct(n, k, float(design_ebn0_db), _ptr(frozen))
    if rc:
        raise ValueError("oracle_construct(%d, %d) failed" % (n, k))
    return frozen


def construct_reliability(n, k, design_ebn0_db):
    """(ln z of every bit channel, ln z0 of the channel) that construct()
    ranks for an (n, k) code at the design Eb/N0."""
    out = np.zeros(n, np.float64)
    z0 = np.zeros(1, np.float64)
    if lib().oracle_construct_lnz(n, k, float(design_ebn0_db), _ptr(out), _ptr(z0)):
        raise ValueError("oracle_construct_lnz(%d, %d) failed" % (n, k))
    return out, float(z0[0])


def bhattacharyya(n, lnz0):
    """ln z of every bit channel for an initial ln z0 (exact for the BEC)."""
    out = np.zeros(n, np.float64)
    if lib().oracle_bhattacharyya(n, float(lnz0), _ptr(out)):
        raise ValueError("oracle_bhattacharyya failed")
    return out


def encode(u):
    """x = u G_N for a [frames, N] (or [N]) array of 0/1 bytes."""
    u = np.ascontiguousarray(u, dtype=np.uint8)
    squeeze = u.ndim == 1
    u2 = u.reshape(1, -1) if squeeze else u
    x = np.empty_like(u2)
    rc = lib().oracle_encode(u2.shape[1], u2.shape[0], _ptr(u2), _ptr(x))
    if rc:
        raise ValueError("oracle_encode failed")
    return x[0] if squeeze else x


def decode(frozen, llr, algo="fastssc", trace=False, nthreads=1):
    """Decode [frames, N] LLRs (int8, float32 or float64 selects the domain).

    Returns (u_hat, x_hat, trace_or_None); u_hat/x_hat are [frames, N] bytes.
    """
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    llr = np.ascontiguousarray(llr)
    if llr.ndim == 1:
        llr = llr.reshape(1, -1)
    frames, n = llr.shape
    if n != frozen.shape[0]:
        raise ValueError("LLR length %d != code length %d" % (n, frozen.shape[0]))
    fn = {np.dtype(np.int8): lib().oracle_decode_i8,
          np.dtype(np.float32): lib().oracle_decode_f32,
          np.dtype(np.float64): lib().oracle_decode_f64}[llr.dtype]
    u = np.empty((frames, n), np.uint8)
    x = np.empty((frames, n), np.uint8)
    t = np.empty((frames, n), llr.dtype) if trace else None
    rc = fn(n, _ptr(frozen), ALGO[algo], frames, _ptr(llr), _ptr(u), _ptr(x), _ptr(t), int(nthreads))
    if rc:
        raise ValueError("oracle decode failed")
    return u, x, t


def schedule(frozen, algo="fastssc"):
    """Node functions one decode runs, as [(name, size), ...] in order."""
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    n = frozen.shape[0]
    cap = 8 * n + 16
    kinds = np.zeros(cap, np.int32)
    sizes = np.zeros(cap, np.int32)
    cnt = lib().oracle_schedule(n, _ptr(frozen), ALGO[algo], _ptr(kinds), _ptr(sizes), cap)
    if cnt < 0 or cnt > cap:
        raise ValueError("oracle_schedule failed")
    return [(LOG_NAMES[kinds[i]], int(sizes[i])) for i in range(cnt)]


def node(kind, alpha):
    """Decode one constituent code ('rate1', 'rep', 'spc'); returns beta bytes."""
    alpha = np.ascontiguousarray(alpha)
    beta = np.zeros(alpha.shape[0], np.uint8)
    fn = lib().oracle_node_i8 if alpha.dtype == np.int8 else lib().oracle_node_f64
    if alpha.dtype not in (np.int8, np.float64):
        raise TypeError("node() takes int8 or float64 LLRs")
    rc = fn(KIND[kind], alpha.shape[0], _ptr(alpha), _ptr(beta))
    if rc:
        raise ValueError("oracle node decode failed")
    return beta


def f_i8(a, b):
    return lib().oracle_f_i8(int(a), int(b))


def g_i8(a, b, beta):
    return lib().oracle_g_i8(int(a), int(b), int(beta))


def f_f64(a, b):
    return lib().oracle_f_f64(float(a), float(b))


def g_f64(a, b, beta):
    return lib().oracle_g_f64(float(a), float(b), int(beta))
