"""Test helper: the forward-error scale of the float decoders.

Every message of the decoder tree at a position is the result of f (which
passes one operand's magnitude through) and g (which adds two), so running
the tree on absolute values with f -> max and g -> sum bounds the magnitude
of every intermediate value that reaches that position; rounding errors of
one binary32 operation are relative to that scale.  Independent of the bit
decisions, of the GPU library and of the oracle.
"""
import numpy as np


def forward_error_scale(llr64):
    """Per-position bound on the magnitude of every alpha computed at that
    position: f passes one operand through (scale max), g adds two (scale
    sum).  The maximum over all tree nodes covering a position bounds the
    leaf there."""
    acc = np.zeros_like(llr64)

    def walk(a, o):
        n = a.shape[-1]
        acc[..., o:o + n] = np.maximum(acc[..., o:o + n], a)
        if n == 1:
            return
        h = n // 2
        walk(np.maximum(a[..., :h], a[..., h:]), o)
        walk(a[..., :h] + a[..., h:], o + h)
    walk(np.abs(llr64), 0)
    return acc
