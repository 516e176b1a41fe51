"""Helpers of the GPU tests: column-major device buffers and decoding of the
library's slice layout (as documented in include/oz.h)."""
import numpy as np
import torch


def to_dev(X, ld=None):
    """Column-major device copy of the numpy matrix X with leading dimension ld."""
    rows, cols = X.shape
    ld = max(1, rows) if ld is None else ld
    buf = np.zeros((ld, cols), dtype=X.dtype, order="F")
    buf[:rows] = X
    return torch.from_numpy(buf.ravel(order="F").copy()).cuda(), ld


def from_dev(t, rows, cols, ld):
    a = t.cpu().numpy()
    return a.reshape((ld, cols), order="F")[:rows].copy(order="F")


def decode_slices(raw, s, rows_pad, kpad):
    """int8 bytes -> digits[p, vector, term] (p 0-based)."""
    a = np.asarray(raw, dtype=np.int8).reshape(kpad // 16, s, rows_pad, 16)
    return a.transpose(1, 2, 0, 3).reshape(s, rows_pad, kpad)


def complex_row_index(c):
    """Slice row of the real-part row of complex row c of a complex side-'A' operand;
    the imaginary-part row follows 8 rows later."""
    c = np.asarray(c)
    return 32 * (c // 16) + 16 * ((c // 8) % 2) + (c % 8)


def stored_shape(side, trans, nv, k):
    """Shape of the stored matrix whose op() gives nv vectors of k terms."""
    t = trans.upper() != "N"
    if side == "A":
        return (k, nv) if t else (nv, k)
    return (nv, k) if t else (k, nv)
