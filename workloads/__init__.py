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
* ``zgemm_batch_mixed`` the batched workload's sizes with operands drawn per
                      problem from the selector's instance distribution
                      (exponent spread, kept significand bits, zeros, value
                      family), complex, and one tolerance per problem.
* ``zgemm_batch_lowprec`` the same with significands of bfloat16 / float16 /
                      float32 / float64 width (operands of lower-precision origin).
* ``zinv_gauss``      one n x n complex matrix to invert, entries
                      N(0,1) + i N(0,1) (condition number of order n), the
                      stand-in for the application's complex LU-inverted matrix.
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


def zinv_gauss(n=4096, seed=0):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))


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


# ---------------------------------------------------------------------------
# Counter-based instances for the slice-count selector.  The GPU library has
# its own implementation of the same generator (splitmix64, Steele, Lea and
# Flood, OOPSLA 2014): output number c (0-based) of the stream seeded with key
# is mix64(key + (c + 1) * GAMMA).  Both sides draw bit-identical operands
# from the parameter table below, so neither ships the other its inputs.
# ---------------------------------------------------------------------------
GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_U64 = (1 << 64) - 1

# fields of one instance (the C struct oz_gen_t has the same order)
GEN_FIELDS = ("m", "n", "k", "sig_el", "sig_vec", "bits", "family", "zero_q", "key")


def mix64(z):
    """splitmix64 output function on a numpy uint64 array (wrapping)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def draw(key, ctr):
    """Output number ctr of the splitmix64 stream seeded with key."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(key) + (ctr + np.uint64(1)) * np.uint64(GAMMA))


def _draw_scalar(key, ctr):
    z = (key + (ctr + 1) * GAMMA) & _U64
    z = ((z ^ (z >> 30)) * _M1) & _U64
    z = ((z ^ (z >> 27)) * _M2) & _U64
    return z ^ (z >> 31)


def gen_keys(key):
    """Sub-stream keys: A entries, B entries, A row exponents, B column exponents."""
    return tuple(_draw_scalar(int(key), c) for c in range(4))


def _gen_side(p, rows, cols, ekey, vkey, vec_axis):
    """One operand (rows x cols, column-major).  Five draws per entry, at
    counters 5*idx .. 5*idx + 4 with idx = i + j*rows:
      family 0: sign and 53-bit significand from draw 0, value in [1/2, 1);
      family 1: Irwin-Hall bell, ((u0 + u1) + u2) + u3 - 2 with u = (d >> 11) 2^-53;
      draw 4:   zero if (d4 >> 40) < zero_q, element exponent (d4 & 0xffffffff) mod (sig_el + 1) - sig_el // 2.
    Then the low 53 - bits significand bits are cleared, and the value is
    scaled by 2^(element exponent + vector exponent), the vector exponent of row
    i (A) / column j (B) being draw(vkey, i or j) mod (sig_vec + 1) - sig_vec // 2."""
    idx = np.arange(rows * cols, dtype=np.uint64)
    base = idx * np.uint64(5)
    d = [draw(ekey, base + np.uint64(c)) for c in range(5)]
    if p["family"] == 0:
        mant = (d[0] >> np.uint64(11)) | np.uint64(1 << 52)
        x = np.ldexp(mant.astype(np.float64), -53)
        x = np.where((d[0] & np.uint64(1)) == 1, -x, x)
    else:
        u = [(dd >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 for dd in d[:4]]
        x = (((u[0] + u[1]) + u[2]) + u[3]) - 2.0
    bits = int(p["bits"])
    if bits < 53:
        xb = x.view(np.uint64) & np.uint64(_U64 ^ ((1 << (53 - bits)) - 1))
        x = xb.view(np.float64)
    zero = (d[4] >> np.uint64(40)) < np.uint64(int(p["zero_q"]))
    sig_el, sig_vec = int(p["sig_el"]), int(p["sig_vec"])
    e_el = ((d[4] & np.uint64(0xFFFFFFFF)) % np.uint64(sig_el + 1)).astype(np.int64) - sig_el // 2
    nvec = rows if vec_axis == 0 else cols
    e_vec = (draw(vkey, np.arange(nvec, dtype=np.uint64)) % np.uint64(sig_vec + 1)).astype(np.int64) - sig_vec // 2
    i = (idx % np.uint64(rows)).astype(np.int64)
    j = (idx // np.uint64(rows)).astype(np.int64)
    e = e_el + (e_vec[i] if vec_axis == 0 else e_vec[j])
    x = np.where(zero, 0.0, np.ldexp(x, e))
    return np.asfortranarray(x.reshape(cols, rows).T)


def gen_operands(p):
    """A (m x k) and B (k x n) of one selector instance, column-major float64."""
    ka, kb, kva, kvb = gen_keys(p["key"])
    A = _gen_side(p, int(p["m"]), int(p["k"]), ka, kva, 0)
    B = _gen_side(p, int(p["k"]), int(p["n"]), kb, kvb, 1)
    return A, B


def selector_instances(count, seed=0, lo=64, hi=2048, tols_per=4, tol_lo=1e-15, tol_hi=1e-4):
    """Parameter table of the selector's training / test instances.

    m, n, k log-uniform in [lo, hi] rounded to a multiple of 16; spread
    sigma ~ randint(0, 40) dealt per entry, per vector, or half and half (one
    third each); 70% full 53-bit significands, else randint(4, 52) bits; 70%
    without zeros, else a zero fraction U(0, 0.8); family 0 or 1 with equal
    odds; tols_per tolerances log-uniform in [tol_lo, tol_hi] per instance.
    Returns (list of dicts, tols array [count, tols_per])."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        dims = [int(max(16, round(np.exp(rng.uniform(np.log(lo), np.log(hi))) / 16) * 16)) for _ in range(3)]
        sigma = int(rng.integers(0, 41))
        mode = int(rng.integers(0, 3))
        sig_el = sigma if mode == 0 else (0 if mode == 1 else sigma // 2)
        sig_vec = sigma - sig_el
        bits = 53 if rng.random() < 0.7 else int(rng.integers(4, 53))
        zero_q = 0 if rng.random() < 0.7 else int(rng.uniform(0.0, 0.8) * (1 << 24))
        out.append(dict(m=dims[0], n=dims[1], k=dims[2], sig_el=sig_el, sig_vec=sig_vec, bits=bits,
                        family=int(rng.integers(0, 2)), zero_q=zero_q,
                        key=int(rng.integers(0, 1 << 63, dtype=np.int64))))
    tols = np.exp(rng.uniform(np.log(tol_lo), np.log(tol_hi), size=(count, tols_per)))
    return out, tols


def zgemm_batch_spread(count=512, seed=0, sig_max=40):
    """The batched workload with a per-problem exponent spread: n_b =
    32 * randint(1, 16), Re, Im ~ N(0,1) scaled by 2^e, e per entry
    ~ randint(-sigma//2, sigma - sigma//2), sigma ~ randint(0, sig_max)."""
    sizes = zgemm_batch_sizes(count, seed)
    rng = np.random.default_rng(seed + 2)
    out = []
    for nb in sizes:
        sigma = int(rng.integers(0, sig_max + 1))
        lo, hi = -(sigma // 2), sigma - sigma // 2

        def one():
            re = np.ldexp(rng.standard_normal((nb, nb)), rng.integers(lo, hi + 1, size=(nb, nb)))
            im = np.ldexp(rng.standard_normal((nb, nb)), rng.integers(lo, hi + 1, size=(nb, nb)))
            return np.asfortranarray(re + 1j * im)

        out.append((one(), one()))
    return out


def zgemm_batch_mixed(count=512, seed=0, tol_lo=1e-15, tol_hi=1e-4):
    """Heterogeneous batch: the square sizes of ``zgemm_batch`` (n_b =
    32 * randint(1, 16)), each problem's structure drawn as one selector
    instance (spread sigma ~ randint(0, 40) per entry / per vector / half and
    half, 70% full significands else randint(4, 52) kept bits, 30% with a zero
    fraction U(0, 0.8), family 0 or 1), and one tolerance per problem,
    log-uniform in [tol_lo, tol_hi].  Returns (list of parameter dicts, tols);
    ``mixed_operands(p)`` draws a problem's complex operands."""
    sizes = zgemm_batch_sizes(count, seed)
    rng = np.random.default_rng(seed + 3)
    params = []
    for nb in sizes:
        sigma = int(rng.integers(0, 41))
        mode = int(rng.integers(0, 3))
        sig_el = sigma if mode == 0 else (0 if mode == 1 else sigma // 2)
        bits = 53 if rng.random() < 0.7 else int(rng.integers(4, 53))
        zero_q = 0 if rng.random() < 0.7 else int(rng.uniform(0.0, 0.8) * (1 << 24))
        params.append(dict(m=nb, n=nb, k=nb, sig_el=sig_el, sig_vec=sigma - sig_el, bits=bits,
                           family=int(rng.integers(0, 2)), zero_q=zero_q,
                           key=int(rng.integers(0, 1 << 63, dtype=np.int64))))
    tols = np.exp(rng.uniform(np.log(tol_lo), np.log(tol_hi), size=count))
    return params, tols


def zgemm_batch_lowprec(count=512, seed=0, tol_lo=1e-15, tol_hi=1e-4):
    """The heterogeneous batch with operands of lower-precision origin: as
    ``zgemm_batch_mixed`` (sizes, exponent spread, zeros, family, one
    tolerance per problem), but every problem's significands keep 8, 11, 24 or
    53 bits (those of bfloat16, float16, float32 and float64 values), one of
    the four with equal odds.  Returns (list of parameter dicts, tols)."""
    sizes = zgemm_batch_sizes(count, seed)
    rng = np.random.default_rng(seed + 4)
    params = []
    for nb in sizes:
        sigma = int(rng.integers(0, 41))
        mode = int(rng.integers(0, 3))
        sig_el = sigma if mode == 0 else (0 if mode == 1 else sigma // 2)
        bits = (8, 11, 24, 53)[int(rng.integers(0, 4))]
        zero_q = 0 if rng.random() < 0.7 else int(rng.uniform(0.0, 0.8) * (1 << 24))
        params.append(dict(m=nb, n=nb, k=nb, sig_el=sig_el, sig_vec=sigma - sig_el, bits=bits,
                           family=int(rng.integers(0, 2)), zero_q=zero_q,
                           key=int(rng.integers(0, 1 << 63, dtype=np.int64))))
    tols = np.exp(rng.uniform(np.log(tol_lo), np.log(tol_hi), size=count))
    return params, tols


def mixed_parts(p):
    """The two real instances whose operands give the real and imaginary parts
    of a ``zgemm_batch_mixed`` problem: p itself, and p with the key replaced
    by draw 4 of p's key stream and no per-vector spread.  The imaginary part
    is the second instance's operand scaled by the first one's per-vector
    powers of two (``vector_exponents``), so both parts of a row of A (column
    of B) share its scale, as the parts of one complex entry do."""
    q = dict(p)
    q["key"] = int(_draw_scalar(int(p["key"]), 4) & 0x7FFFFFFFFFFFFFFF)
    q["sig_vec"] = 0
    return p, q


def vector_exponents(p):
    """Per-vector exponents e_vec of an instance: rows of A, columns of B
    (the generator's draw(vkey, i) mod (sig_vec + 1) - sig_vec // 2)."""
    _, _, kva, kvb = gen_keys(p["key"])
    sv = int(p["sig_vec"])
    ea = (draw(kva, np.arange(int(p["m"]), dtype=np.uint64)) % np.uint64(sv + 1)).astype(np.int64) - sv // 2
    eb = (draw(kvb, np.arange(int(p["n"]), dtype=np.uint64)) % np.uint64(sv + 1)).astype(np.int64) - sv // 2
    return ea, eb


def mixed_operands(p):
    """Complex operands (A, B) of one ``zgemm_batch_mixed`` problem, column-major."""
    pr, pi = mixed_parts(p)
    Ar, Br = gen_operands(pr)
    Ai, Bi = gen_operands(pi)
    ea, eb = vector_exponents(pr)
    Ai = np.ldexp(Ai, ea[:, None])
    Bi = np.ldexp(Bi, eb[None, :])
    return np.asfortranarray(Ar + 1j * Ai), np.asfortranarray(Br + 1j * Bi)
