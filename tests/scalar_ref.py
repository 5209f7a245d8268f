"""Independent scalar evaluators used to pin the oracle by brute force.

Written directly from the tree definition (recursive descent over a prefix
array, one test case at a time) with numpy float32 scalar arithmetic, which is
IEEE binary32 with round-to-nearest-even.  They share nothing with the oracle
(C) or the GPU library; they are slow and only used on small trees.
"""
import numpy as np

ONE = np.float32(1.0)
TINY = np.float32(1e-6)


def eval_f32_case(tree, xs):
    """Value of a prefix tree on one case; xs = per-input float32 values."""
    pos = 0

    def rec():
        nonlocal pos
        b = int(tree[pos])
        pos += 1
        if b & 0x80 == 0:
            return np.float32(xs[b])
        a = rec()
        c = rec()
        f = b & 3
        with np.errstate(all="ignore"):
            if f == 0:
                return np.float32(a + c)
            if f == 1:
                return np.float32(a - c)
            if f == 2:
                return np.float32(a * c)
            if np.abs(c) < TINY:
                return ONE
            return np.float32(a / c)

    v = rec()
    assert pos == len(tree)
    return v


def eval_bool_case(tree, bits):
    pos = 0

    def rec():
        nonlocal pos
        b = int(tree[pos])
        pos += 1
        if b & 0x80 == 0:
            return bool(bits[b])
        a = rec()
        c = rec()
        f = b & 3
        return [a and c, a or c, not (a and c), not (a or c)][f]

    v = rec()
    assert pos == len(tree)
    return v


def same_f32(a, b):
    """Bit-equal, or both NaN."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return (a.view(np.uint32) == b.view(np.uint32)) | (np.isnan(a) & np.isnan(b))
