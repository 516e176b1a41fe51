"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random matrices; it holds none of the method's
arithmetic.  Every generator uses numpy's PCG64 (``default_rng(seed)``) and
returns column-major (Fortran-order) arrays, the BLAS storage the library takes.

The paper measures on an application input (an LSMS case of MuST) that is not
available; these recipes stand in for it with the shapes and value
distributions of the workloads the emulated GEMM is benchmarked on:

* ``dgemm_uniform``   m x k and k x n, entries U(-1, 1) * 2^randint(-4, 4)
                      (both ends inclusive), independent per entry.
* ``zgemm_rowexp``    complex square operands; each stored row r of A and of B
                      gets one exponent e_r ~ randint(-20, 20) shared by the
                      real and imaginary parts: X = (N(0,1) + i N(0,1)) 2^e_r.
* ``zgemm_batch``     512 square complex problems, n_b = 32 * randint(1, 16),
                      entries N(0,1) + i N(0,1).
* ``dgemm_wide``      A m x k, B k x n, entries N(0,1); rows of A scaled by
                      10^U(-8, 8) and columns of B by 10^U(-8, 8).
* ``dgemm_spread``    general real operands whose per-entry exponents are
                      spread over sigma binades, for slice-count selection data.
"""
import numpy as np


def dgemm_uniform(m=256, n=256, k=256, seed=0):
    rng = np.random.default_rng(seed)

    def one(r, c):
        u = rng.uniform(-1.0, 1.0, size=(r, c))
        e = rng.integers(-4, 5, size=(r, c))
        return np.asfortranarray(np.ldexp(u, e))

    A = one(m, k)
    B = one(k, n)
    return A, B


def zgemm_rowexp(n=2048, seed=0, m=None, k=None):
    rng = np.random.default_rng(seed)
    m = n if m is None else m
    k = n if k is None else k

    def one(r, c):
        re = rng.standard_normal((r, c))
        im = rng.standard_normal((r, c))
        e = rng.integers(-20, 21, size=(r, 1))
        return np.asfortranarray(np.ldexp(re, e) + 1j * np.ldexp(im, e))

    A = one(m, k)
    B = one(k, n)
    return A, B


def zgemm_batch_sizes(count=512, seed=0):
    rng = np.random.default_rng(seed)
    return [int(32 * v) for v in rng.integers(1, 17, size=count)]


def zgemm_batch(count=512, seed=0):
    """Yield (A, B) pairs of the batched workload (generated lazily)."""
    sizes = zgemm_batch_sizes(count, seed)
    rng = np.random.default_rng(seed + 1)
    out = []
    for nb in sizes:
        A = np.asfortranarray(rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb)))
        B = np.asfortranarray(rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb)))
        out.append((A, B))
    return out


def dgemm_wide(m=4096, n=4096, k=8192, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((k, n))
    A *= 10.0 ** rng.uniform(-8.0, 8.0, size=(m, 1))
    B *= 10.0 ** rng.uniform(-8.0, 8.0, size=(1, n))
    return np.asfortranarray(A), np.asfortranarray(B)


def dgemm_spread(m, n, k, sigma, seed=0, per_row_frac=0.5):
    """Real operands with exponent spread sigma: entries N(0,1) * 2^e with
    e ~ randint(-floor(sigma/2), ceil(sigma/2)); a fraction per_row_frac of
    the spread is drawn once per row (A) / column (B), the rest per entry."""
    rng = np.random.default_rng(seed)
    lo, hi = -(sigma // 2), (sigma + 1) // 2

    def one(r, c, axis):
        x = rng.standard_normal((r, c))
        ent = rng.integers(lo, hi + 1, size=(r, c))
        vec_shape = (r, 1) if axis == 0 else (1, c)
        vec = rng.integers(lo, hi + 1, size=vec_shape)
        e = np.where(rng.random((r, c)) < per_row_frac, np.broadcast_to(vec, (r, c)), ent)
        return np.asfortranarray(np.ldexp(x, e))

    return one(m, k, 0), one(k, n, 1)
