"""CPU oracle for the learned slice-count selector.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain definitions in
float64, written for a reader to check by eye, with no blocking or reordering.

The paper suggests choosing the number of splits per call (Sec. 4, the
outlook on a dynamic, accuracy-driven split count); the selector here is this
library's reading of that suggestion, so the definitions below are the
library's own, stated once in words:

* ``features``   16 numbers describing one product op(A) op(B) and a target
                 tolerance.  Per operand (rows of op(A), columns of op(B); a
                 complex operand contributes its real and imaginary parts as
                 separate entries, both scaled by the vector's shared exponent):
                   zero fraction, and over the non-zero entries x of vector v
                   with scale exponent E_v (frexp exponent of the vector max):
                   the gap g = E_v - frexp_exponent(x) and the width
                   w = g + bitlen(odd significand of x) -- the bit positions
                   from 2^E_v down to the lowest set bit, so x is exact with
                   ceil(w / 7) digits -- each capped at 127; features are mean
                   g, std g, 90th percentile of g, mean w, 90th percentile of w.
                 Globals: log2 of the term count (2k for complex: the stacked
                 real product), log2(m n) / 2, -log10(tol), and
                 log2 sqrt((1/M_A + 1/M_B) / 3) with M the mean over vectors
                 of the mean square of x 2^-E_v.
* ``eps_table``  eps_s = || W o (C_s - C_ref) ||_F / || W o C_ref ||_F for the
                 fixed-s emulations C_s (``emu_gemm``), C_ref the one at
                 s_ref, W_ij = 1 / (max|op(A)_i:| max|op(B)_:j|).
* ``label``      the smallest s in [smin, smax] with eps_s <= tol.

Parity: ``features`` is pinned by hand-built operands whose statistics are
known in closed form, ``eps_table`` and ``label`` by integer operands that are
exact at s = 1, by the per-slice decay, and by monotonicity (tests in
tests/test_oracle_select.py).
"""
import numpy as np

from . import emu_gemm

CAP = 127
NFEAT = 16


def _vectors(side, trans, X):
    """Entries as a [vectors, terms] real array (complex: parts side by side)."""
    t = trans.upper()
    if side == "A":
        V = X if t == "N" else X.T
    else:
        V = X.T if t == "N" else X
    V = np.asarray(V)
    if np.iscomplexobj(V):
        V = np.concatenate([V.real, V.imag], axis=1)
    return np.ascontiguousarray(V, dtype=np.float64)


def _scale_exponents(V):
    mx = np.max(np.abs(V), axis=1) if V.shape[1] else np.zeros(V.shape[0])
    _, E = np.frexp(mx)
    return mx, E.astype(np.int64)


def _quantile90(vals):
    """Smallest v with #(vals <= v) * 10 >= 9 * len(vals) (0 when empty)."""
    if vals.size == 0:
        return 0.0
    srt = np.sort(vals)
    need = -(-9 * vals.size // 10)  # ceil(0.9 n)
    return float(srt[need - 1])


def side_stats(side, trans, X):
    """(zero fraction, mean g, std g, p90 g, mean w, p90 w, M) of one operand."""
    V = _vectors(side, trans, X)
    nv, nt = V.shape
    mx, E = _scale_exponents(V)
    total = nv * nt
    nz = V != 0.0
    zero_frac = 1.0 - np.count_nonzero(nz) / total if total else 0.0
    f, e = np.frexp(V)
    g = np.minimum((E[:, None] - e)[nz], CAP)
    sig = np.abs(f[nz]) * 2.0 ** 53                      # integer in [2^52, 2^53)
    sig = sig.astype(np.uint64)
    tz = np.zeros(sig.shape, dtype=np.int64)
    rest = sig.copy()
    for _ in range(53):                                   # trailing zero count
        even = (rest & np.uint64(1)) == 0
        if not even.any():
            break
        tz += even
        rest = np.where(even, rest >> np.uint64(1), rest)
    w = np.minimum((E[:, None] - e)[nz] + (53 - tz), CAP)
    if g.size:
        gm, gs = float(np.mean(g)), float(np.std(g))
        wm = float(np.mean(w))
    else:
        gm = gs = wm = 0.0
    scaled = np.ldexp(V, -E[:, None])
    M = float(np.mean(np.mean(scaled * scaled, axis=1))) if nt and nv else 0.0
    return zero_frac, gm, gs, _quantile90(g), wm, _quantile90(w), M


def features(transa, transb, A, B, tol):
    """The 16 selector features (float64) of op(A) op(B) at tolerance tol."""
    cplx = np.iscomplexobj(A)
    ta, tb = transa.upper(), transb.upper()
    m = A.shape[0] if ta == "N" else A.shape[1]
    k = A.shape[1] if ta == "N" else A.shape[0]
    n = B.shape[1] if tb == "N" else B.shape[0]
    sa = side_stats("A", ta, A)
    sb = side_stats("B", tb, B)
    keff = 2 * k if cplx else k
    Ma, Mb = sa[6], sb[6]
    spread = 0.5 * np.log2((1.0 / Ma + 1.0 / Mb) / 3.0) if Ma > 0 and Mb > 0 else 0.0
    return np.array(list(sa[:6]) + list(sb[:6]) +
                    [np.log2(keff), 0.5 * np.log2(float(m) * float(n)), -np.log10(tol), spread])


def weights(transa, transb, A, B):
    """Row weights 1/max|op(A)_i:| and column weights 1/max|op(B)_:j| (0 for zero vectors)."""
    mxa, _ = _scale_exponents(_vectors("A", transa, A))
    mxb, _ = _scale_exponents(_vectors("B", transb, B))
    wa = np.where(mxa > 0, 1.0 / np.where(mxa > 0, mxa, 1.0), 0.0)
    wb = np.where(mxb > 0, 1.0 / np.where(mxb > 0, mxb, 1.0), 0.0)
    return wa, wb


def weighted_eps(C, Cref, wa, wb):
    W = wa[:, None] * wb[None, :]
    num = np.sum(np.abs(W * (C - Cref)) ** 2)
    den = np.sum(np.abs(W * Cref) ** 2)
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def eps_table(transa, transb, A, B, s_ref=12, s_lo=1):
    """{s: eps_s} for s = s_lo .. s_ref, against the fixed s_ref emulation."""
    Cref = emu_gemm(transa, transb, A, B, s_ref)
    wa, wb = weights(transa, transb, A, B)
    out = {s_ref: 0.0}
    for s in range(s_lo, s_ref):
        out[s] = weighted_eps(emu_gemm(transa, transb, A, B, s), Cref, wa, wb)
    return out


def label(eps, tol, smin=2, smax=12):
    """Smallest s in [smin, smax] with eps[s] <= tol (smax if none)."""
    for s in range(smin, smax + 1):
        if eps[s] <= tol:
            return s
    return smax
