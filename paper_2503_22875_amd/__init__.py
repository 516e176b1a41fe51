"""Python binding of liboz.so, the Ozaki-scheme FP64 / complex-FP64 GEMM
emulation on MI355X INT8 matrix cores (C ABI: include/oz.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of liboz.so.  Functions keep the C names; pointer arguments accept a
torch tensor (its data_ptr), a plain integer address, or None.  There is no
CPU fallback: importing this module without the built library raises.
"""
import ctypes
import os

try:
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7)
    # as the one liboz.so links; whichever is loaded first serves the whole
    # process.  Loading torch first makes the library share torch's runtime, so
    # torch device pointers and streams passed in are valid for it.
    import torch  # noqa: F401
except ImportError:  # the library itself does not need torch
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboz.so")

OZ_OK = 0
OZ_ERR_HIP = -1
OZ_ERR_ALLOC = -2
OZ_ERR_NONFINITE = -3
OZ_ERR_HANDLE = -4
OZ_ERR_UNSUPPORTED = -5
OZ_ERR_ARG = -6
OZ_MAX_SLICES = 18
OZ_NOALLOC_SCRATCH_BYTES = 64 << 20

# Every symbol include/oz.h declares (checked by the CPU test-suite).
EXPORTS = ["oz_create", "oz_destroy", "oz_set_stream", "oz_status_string", "oz_workspace_size",
           "oz_set_workspace", "oz_dgemm", "oz_zgemm", "oz_split_layout", "oz_split", "oz_diag_sums",
           "oz_timing_enable", "oz_timing_read", "oz_select_slices", "oz_gemm_batched_plan", "oz_batch_execute",
           "oz_batch_graph_launch", "oz_batch_destroy", "oz_batch_info", "oz_zgemm_batched", "oz_dgemm_batched",
           "oz_load_tuning", "oz_gen_operands", "oz_features", "oz_selector_dataset", "oz_mlp_create",
           "oz_mlp_destroy", "oz_mlp_set_params", "oz_mlp_get_params", "oz_mlp_fit_norm", "oz_mlp_forward",
           "oz_mlp_grad", "oz_mlp_train_step", "oz_mlp_train", "oz_mlp_save", "oz_mlp_load", "oz_set_selector",
           "oz_predict_slices", "oz_batch_report", "oz_dgemm_x2", "oz_zgemm_x2", "oz_zgetrf", "oz_zgetri",
           "oz_gemm_noalloc", "oz_peak"]

OZ_NUM_FEATURES = 16
OZ_MLP_NPARAM = 5313


class OzError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__("%s failed: status %d (%s)" % (fn, status, oz_status_string(status)))
        self.status = status


class oz_prec_t(ctypes.Structure):
    _fields_ = [("slices", ctypes.c_int32), ("smax", ctypes.c_int32), ("kchunk", ctypes.c_int32),
                ("zmode", ctypes.c_int32), ("kernel", ctypes.c_int32), ("sstart", ctypes.c_int32),
                ("selector", ctypes.c_int32), ("digits", ctypes.c_int32), ("tol", ctypes.c_double)]


class oz_report_t(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slices_used", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("kchunks", ctypes.c_int32), ("zmode_used", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("resid_est", ctypes.c_double)]


class oz_gen_t(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64), ("sig_el", ctypes.c_int32),
                ("sig_vec", ctypes.c_int32), ("bits", ctypes.c_int32), ("family", ctypes.c_int32),
                ("zero_q", ctypes.c_int64), ("key", ctypes.c_uint64)]


def gen_params(d):
    """oz_gen_t from a dict with the fields of oz_gen_t."""
    return oz_gen_t(*[int(d[name]) for name, _ in oz_gen_t._fields_])


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liboz.so is not built (%s); run __graft_entry__.build() first" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, C, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_char, ctypes.c_double
    PP = ctypes.POINTER
    sig = {
        "oz_create": [PP(P), ctypes.c_int],
        "oz_destroy": [P],
        "oz_set_stream": [P, P],
        "oz_status_string": [ctypes.c_int],
        "oz_workspace_size": [P, C, C, I64, I64, I64, ctypes.c_int, PP(oz_prec_t), PP(ctypes.c_size_t)],
        "oz_set_workspace": [P, P, ctypes.c_size_t],
        "oz_dgemm": [P, C, C, I64, I64, I64, PP(D), P, I64, P, I64, PP(D), P, I64, PP(oz_prec_t),
                     PP(oz_report_t)],
        "oz_zgemm": [P, C, C, I64, I64, I64, PP(D), P, I64, P, I64, PP(D), P, I64, PP(oz_prec_t),
                     PP(oz_report_t)],
        "oz_gemm_noalloc": [P, ctypes.c_int, C, C, I64, I64, I64, PP(D), P, I64, P, I64, PP(D), P, I64,
                            PP(oz_prec_t)],
        "oz_dgemm_x2": [P, C, C, I64, I64, I64, P, I64, P, I64, P, P, I64, PP(oz_prec_t), PP(oz_report_t)],
        "oz_zgemm_x2": [P, C, C, I64, I64, I64, P, I64, P, I64, P, P, I64, PP(oz_prec_t), PP(oz_report_t)],
        "oz_zgetrf": [P, I64, P, I64, P, I32, PP(oz_prec_t), PP(I32)],
        "oz_zgetri": [P, I64, P, I64, P, P, I64, I32, PP(oz_prec_t)],
        "oz_split_layout": [C, ctypes.c_int, I64, I64, I32, PP(I64), PP(I64), PP(ctypes.c_size_t)],
        "oz_split": [P, C, C, ctypes.c_int, I64, I64, P, I64, I32, P, P],
        "oz_diag_sums": [P, I32, I64, I32, I64, I64, I64, P, P, P],
        "oz_timing_enable": [P, ctypes.c_int],
        "oz_timing_read": [P, PP(D), PP(D), PP(I64)],
        "oz_select_slices": [P, C, C, I64, I64, I64, ctypes.c_int, P, I64, P, I64, D, I32, PP(I32)],
        "oz_gemm_batched_plan": [P, ctypes.c_int, I32, P, P, P, P, P, P, P, P, P, P, P, P, P, PP(oz_prec_t), P,
                                 P, PP(P)],
        "oz_batch_execute": [P],
        "oz_batch_graph_launch": [P],
        "oz_batch_destroy": [P],
        "oz_batch_info": [P, PP(I32), PP(I64), PP(ctypes.c_size_t), P],
        "oz_batch_report": [P, P],
        "oz_zgemm_batched": [P, I32, P, P, P, P, P, P, P, P, P, P, P, P, P, PP(oz_prec_t), P],
        "oz_dgemm_batched": [P, I32, P, P, P, P, P, P, P, P, P, P, P, P, P, PP(oz_prec_t), P],
        "oz_load_tuning": [P, ctypes.c_char_p],
        "oz_gen_operands": [P, PP(oz_gen_t), P, I64, P, I64],
        "oz_features": [P, C, C, I64, I64, I64, ctypes.c_int, P, I64, P, I64, I32, P, I32, P, P],
        "oz_selector_dataset": [P, I32, P, I32, P, I32, I32, P, P, P, P],
        "oz_mlp_create": [P, ctypes.c_uint64, PP(P)],
        "oz_mlp_destroy": [P],
        "oz_mlp_set_params": [P, P, P, P],
        "oz_mlp_get_params": [P, P, P, P],
        "oz_mlp_fit_norm": [P, I64, P],
        "oz_mlp_forward": [P, I64, P, P],
        "oz_mlp_grad": [P, I64, P, P, ctypes.c_float, P, P],
        "oz_mlp_train_step": [P, I64, P, P, ctypes.c_float, ctypes.c_float, P],
        "oz_mlp_train": [P, I64, P, P, I32, I32, ctypes.c_float, ctypes.c_float, ctypes.c_uint64, P],
        "oz_mlp_save": [P, ctypes.c_char_p],
        "oz_mlp_load": [P, ctypes.c_char_p, PP(P)],
        "oz_set_selector": [P, P],
        "oz_predict_slices": [P, C, C, I64, I64, I64, ctypes.c_int, P, I64, P, I64, D, I32, PP(I32)],
        "oz_peak": [P, ctypes.c_int, I64, P, P, ctypes.c_size_t, PP(D)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "oz_status_string" else ctypes.c_int
    return lib


_lib = _load()

# Tuning table written by the autotuner for this device (see autotune.py)
TUNE_PATH = os.path.join(_HERE, "tune", "gfx950.json")


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _ch(c):
    return c.encode() if isinstance(c, str) else c


def _check(fn, status, allow=()):
    if status != OZ_OK and status not in allow:
        raise OzError(fn, status)
    return status


def oz_status_string(status):
    return _lib.oz_status_string(status).decode()


def oz_create(device=0):
    h = ctypes.c_void_p()
    _check("oz_create", _lib.oz_create(ctypes.byref(h), device))
    return h


def oz_destroy(handle):
    return _check("oz_destroy", _lib.oz_destroy(handle))


def oz_set_stream(handle, stream):
    """stream: a hipStream_t address (e.g. torch.cuda.current_stream().cuda_stream) or None."""
    return _check("oz_set_stream", _lib.oz_set_stream(handle, stream))


def prec(slices=7, tol=0.0, smax=0, kchunk=0, zmode=0, kernel=0, sstart=0, selector=0, digits=0):
    """Precision record; prec(0, tol=...) asks for a tolerance-driven call;
    digits=1 selects balanced (round-to-nearest) digits."""
    return oz_prec_t(slices, smax, kchunk, zmode, kernel, sstart, selector, digits, tol)


def oz_workspace_size(handle, transa, transb, m, n, k, is_complex, p=None):
    out = ctypes.c_size_t()
    _check("oz_workspace_size", _lib.oz_workspace_size(handle, _ch(transa), _ch(transb), m, n, k, int(is_complex),
                                                        ctypes.byref(p) if p is not None else None,
                                                        ctypes.byref(out)))
    return out.value


def oz_set_workspace(handle, dptr, nbytes):
    return _check("oz_set_workspace", _lib.oz_set_workspace(handle, _ptr(dptr), nbytes))


def _gemm(fn, cplx, handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p, report, check):
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    rep = oz_report_t() if report else None
    st = getattr(_lib, fn)(handle, _ch(transa), _ch(transb), m, n, k, al, _ptr(A), lda, _ptr(B), ldb, be, _ptr(C),
                           ldc, ctypes.byref(p) if p is not None else None,
                           ctypes.byref(rep) if rep is not None else None)
    if check:
        _check(fn, st)
    return (st, rep) if report else st


def oz_dgemm(handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p=None, report=False, check=True):
    """C = alpha*op(A)*op(B) + beta*C (column-major device buffers)."""
    return _gemm("oz_dgemm", False, handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p,
                 report, check)


def oz_zgemm(handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p=None, report=False, check=True):
    """Complex version; A, B, C hold interleaved (re, im) doubles."""
    return _gemm("oz_zgemm", True, handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p,
                 report, check)


def oz_gemm_noalloc(handle, is_complex, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p=None,
                    check=True):
    """oz_dgemm (is_complex 0) / oz_zgemm (1) on the library's fixed device
    scratch: allocates nothing, fixed slice counts only, no report."""
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    st = _lib.oz_gemm_noalloc(handle, int(is_complex), _ch(transa), _ch(transb), m, n, k, al, _ptr(A), lda, _ptr(B),
                              ldb, be, _ptr(C), ldc, ctypes.byref(p) if p is not None else None)
    if check:
        _check("oz_gemm_noalloc", st)
    return st


def _gemm_x2(fn, handle, transa, transb, m, n, k, A, lda, B, ldb, C_hi, C_lo, ldc, p, report, check):
    rep = oz_report_t() if report else None
    st = getattr(_lib, fn)(handle, _ch(transa), _ch(transb), m, n, k, _ptr(A), lda, _ptr(B), ldb, _ptr(C_hi),
                           _ptr(C_lo), ldc, ctypes.byref(p) if p is not None else None,
                           ctypes.byref(rep) if rep is not None else None)
    if check:
        _check(fn, st)
    return (st, rep) if report else st


def oz_dgemm_x2(handle, transa, transb, m, n, k, A, lda, B, ldb, C_hi, C_lo, ldc, p, report=False, check=True):
    """C_hi + C_lo = op(A)*op(B) as a double-double (fixed slice count p.slices)."""
    return _gemm_x2("oz_dgemm_x2", handle, transa, transb, m, n, k, A, lda, B, ldb, C_hi, C_lo, ldc, p, report,
                    check)


def oz_zgemm_x2(handle, transa, transb, m, n, k, A, lda, B, ldb, C_hi, C_lo, ldc, p, report=False, check=True):
    """Complex version of oz_dgemm_x2 (interleaved (re, im) doubles)."""
    return _gemm_x2("oz_zgemm_x2", handle, transa, transb, m, n, k, A, lda, B, ldb, C_hi, C_lo, ldc, p, report,
                    check)


def oz_zgetrf(handle, n, A, lda, ipiv, nb=0, p=None, check=True):
    """LU with partial pivoting in place (device A, device int32 ipiv); returns info."""
    info = ctypes.c_int32()
    st = _lib.oz_zgetrf(handle, n, _ptr(A), lda, _ptr(ipiv), nb, ctypes.byref(p) if p is not None else None,
                        ctypes.byref(info))
    if check:
        _check("oz_zgetrf", st)
        return info.value
    return st, info.value


def oz_zgetri(handle, n, LU, lda, ipiv, X, ldx, nb=0, p=None, check=True):
    """X = A^-1 from the factorisation oz_zgetrf left in LU and ipiv."""
    st = _lib.oz_zgetri(handle, n, _ptr(LU), lda, _ptr(ipiv), _ptr(X), ldx, nb,
                        ctypes.byref(p) if p is not None else None)
    if check:
        _check("oz_zgetri", st)
    return st


def oz_split_layout(side, is_complex, nv, k, slices):
    rp, kp, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    _check("oz_split_layout", _lib.oz_split_layout(_ch(side), int(is_complex), nv, k, slices, ctypes.byref(rp),
                                                    ctypes.byref(kp), ctypes.byref(nb)))
    return rp.value, kp.value, nb.value


def oz_split(handle, side, trans, is_complex, nv, k, X, ldx, slices, E, slices_out):
    return _check("oz_split", _lib.oz_split(handle, _ch(side), _ch(trans), int(is_complex), nv, k, _ptr(X), ldx,
                                            slices, _ptr(E), _ptr(slices_out)))


def oz_diag_sums(handle, slices, kchunk, rows_pad_a, rows_pad_b, kpad, slices_a, slices_b, out, kernel=0):
    return _check("oz_diag_sums", _lib.oz_diag_sums(handle, slices, kchunk, kernel, rows_pad_a, rows_pad_b, kpad,
                                                    _ptr(slices_a), _ptr(slices_b), _ptr(out)))


def oz_timing_enable(handle, enable=True):
    return _check("oz_timing_enable", _lib.oz_timing_enable(handle, int(enable)))


def oz_timing_read(handle):
    """-> (split_ms, gemm_ms, calls) summed since the previous read."""
    a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check("oz_timing_read", _lib.oz_timing_read(handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)))
    return a.value, b.value, n.value


def oz_select_slices(handle, transa, transb, m, n, k, is_complex, A, lda, B, ldb, tol, smax=0):
    """Starting slice count of a tolerance-driven call (the rule)."""
    out = ctypes.c_int32()
    _check("oz_select_slices", _lib.oz_select_slices(handle, _ch(transa), _ch(transb), m, n, k, int(is_complex),
                                                      _ptr(A), lda, _ptr(B), ldb, float(tol), smax,
                                                      ctypes.byref(out)))
    return out.value


def _batch_args(is_complex, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, slices):
    nb = len(m)
    I64A = ctypes.c_int64 * nb
    PA = ctypes.c_void_p * nb
    w = 2 if is_complex else 1
    DA = ctypes.c_double * (w * nb)

    def scal(vals):
        out = []
        for v in vals:
            z = complex(v)
            out += [z.real, z.imag] if is_complex else [z.real]
        return DA(*out)
    ta = ctypes.create_string_buffer(("".join(transa) if not isinstance(transa, str) else transa).encode(), nb + 1)
    tb = ctypes.create_string_buffer(("".join(transb) if not isinstance(transb, str) else transb).encode(), nb + 1)
    keep = dict(ta=ta, tb=tb, m=I64A(*m), n=I64A(*n), k=I64A(*k), alpha=scal(alpha), beta=scal(beta),
                A=PA(*[_ptr(x) for x in A]), lda=I64A(*lda), B=PA(*[_ptr(x) for x in B]), ldb=I64A(*ldb),
                C=PA(*[_ptr(x) for x in C]), ldc=I64A(*ldc),
                slices=(ctypes.c_int32 * nb)(*slices) if slices is not None else None)
    return nb, keep


def oz_gemm_batched_plan(handle, is_complex, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p=None,
                         slices=None, tols=None):
    """Plan a batch (host lists of per-problem arguments); returns the plan handle.
    transa / transb: strings or lists of one character per problem; tols: one
    tolerance per problem (tolerance-driven plans)."""
    nb, a = _batch_args(is_complex, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, slices)
    tl = (ctypes.c_double * nb)(*[float(t) for t in tols]) if tols is not None else None
    plan = ctypes.c_void_p()
    _check("oz_gemm_batched_plan", _lib.oz_gemm_batched_plan(
        handle, int(is_complex), nb, ctypes.cast(a["ta"], ctypes.c_void_p), ctypes.cast(a["tb"], ctypes.c_void_p),
        ctypes.cast(a["m"], ctypes.c_void_p), ctypes.cast(a["n"], ctypes.c_void_p),
        ctypes.cast(a["k"], ctypes.c_void_p), ctypes.cast(a["alpha"], ctypes.c_void_p),
        ctypes.cast(a["A"], ctypes.c_void_p), ctypes.cast(a["lda"], ctypes.c_void_p),
        ctypes.cast(a["B"], ctypes.c_void_p), ctypes.cast(a["ldb"], ctypes.c_void_p),
        ctypes.cast(a["beta"], ctypes.c_void_p), ctypes.cast(a["C"], ctypes.c_void_p),
        ctypes.cast(a["ldc"], ctypes.c_void_p), ctypes.byref(p) if p is not None else None,
        ctypes.cast(a["slices"], ctypes.c_void_p) if a["slices"] is not None else None,
        ctypes.cast(tl, ctypes.c_void_p) if tl is not None else None, ctypes.byref(plan)))
    return plan


def oz_batch_execute(plan):
    return _check("oz_batch_execute", _lib.oz_batch_execute(plan))


def oz_batch_graph_launch(plan):
    return _check("oz_batch_graph_launch", _lib.oz_batch_graph_launch(plan))


def oz_batch_destroy(plan):
    return _check("oz_batch_destroy", _lib.oz_batch_destroy(plan))


def oz_batch_info(plan, batch):
    """-> (gemm launches, tiles, device bytes, slices per problem)."""
    la, ti, by = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_size_t()
    sl = (ctypes.c_int32 * max(1, batch))()
    _check("oz_batch_info", _lib.oz_batch_info(plan, ctypes.byref(la), ctypes.byref(ti), ctypes.byref(by),
                                                ctypes.cast(sl, ctypes.c_void_p)))
    return la.value, ti.value, by.value, list(sl)[:batch]


def oz_batch_report(plan, batch):
    """Per-problem reports (oz_report_t) of the plan's last execution."""
    reps = (oz_report_t * max(1, batch))()
    _check("oz_batch_report", _lib.oz_batch_report(plan, ctypes.cast(reps, ctypes.c_void_p)))
    return list(reps)[:batch]


def _gemm_batched(fn, is_complex, handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p, slices,
                  check):
    nb, a = _batch_args(is_complex, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, slices)
    cv = lambda x: ctypes.cast(x, ctypes.c_void_p) if x is not None else None  # noqa: E731
    st = getattr(_lib, fn)(handle, nb, cv(a["ta"]), cv(a["tb"]), cv(a["m"]), cv(a["n"]), cv(a["k"]), cv(a["alpha"]),
                           cv(a["A"]), cv(a["lda"]), cv(a["B"]), cv(a["ldb"]), cv(a["beta"]), cv(a["C"]),
                           cv(a["ldc"]), ctypes.byref(p) if p is not None else None, cv(a["slices"]))
    if check:
        _check(fn, st)
    return st


def oz_zgemm_batched(handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p=None, slices=None,
                     check=True):
    return _gemm_batched("oz_zgemm_batched", True, handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C,
                         ldc, p, slices, check)


def oz_dgemm_batched(handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, p=None, slices=None,
                     check=True):
    return _gemm_batched("oz_dgemm_batched", False, handle, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C,
                         ldc, p, slices, check)


def oz_load_tuning(handle, path=None):
    """Load an autotuner table (default: the package's table for gfx950, if present)."""
    path = TUNE_PATH if path is None else path
    if path == "" or not os.path.exists(path):
        return _check("oz_load_tuning", _lib.oz_load_tuning(handle, None))
    return _check("oz_load_tuning", _lib.oz_load_tuning(handle, path.encode()))


# ---- learned slice-count selection -------------------------------------------

# Trained selector network for this device (see train_selector.py)
SELECTOR_PATH = os.path.join(_HERE, "tune", "selector_gfx950.bin")


def _host_array(ctype, n, values=None):
    arr = (ctype * max(1, n))()
    if values is not None:
        for i, v in enumerate(values):
            arr[i] = v
    return arr


def oz_gen_operands(handle, params, A, lda, B, ldb):
    """Draw the operands of one selector instance (dict or oz_gen_t) into device buffers."""
    g = params if isinstance(params, oz_gen_t) else gen_params(params)
    return _check("oz_gen_operands", _lib.oz_gen_operands(handle, ctypes.byref(g), _ptr(A), lda, _ptr(B), ldb))


def oz_features(handle, transa, transb, m, n, k, is_complex, A, lda, B, ldb, tols, feat, smax=0):
    """Feature rows (device float32 [len(tols), 16]) of op(A) op(B); returns the rule's s per tolerance."""
    nt = len(tols)
    th = _host_array(ctypes.c_double, nt, [float(t) for t in tols])
    sr = _host_array(ctypes.c_int32, nt)
    _check("oz_features", _lib.oz_features(handle, _ch(transa), _ch(transb), m, n, k, int(is_complex), _ptr(A), lda,
                                            _ptr(B), ldb, nt, ctypes.cast(th, ctypes.c_void_p), smax, _ptr(feat),
                                            ctypes.cast(sr, ctypes.c_void_p)))
    return list(sr)[:nt]


def oz_selector_dataset(handle, params, tols, X, y, s_ref=12, smax_rule=0):
    """Generate and label instances on the GPU.  params: list of dicts / oz_gen_t;
    tols: [count][ntol] tolerances; X, y: device float32 buffers of count*ntol rows.
    Returns (rule s per row, eps table [count][s_ref]) as lists."""
    count = len(params)
    ntol = len(tols[0]) if count else 1
    ga = (oz_gen_t * max(1, count))(*[p if isinstance(p, oz_gen_t) else gen_params(p) for p in params])
    flat = [float(t) for row in tols for t in row]
    th = _host_array(ctypes.c_double, len(flat), flat)
    sr = _host_array(ctypes.c_int32, count * ntol)
    ep = _host_array(ctypes.c_double, count * s_ref)
    _check("oz_selector_dataset", _lib.oz_selector_dataset(
        handle, count, ctypes.cast(ga, ctypes.c_void_p), ntol, ctypes.cast(th, ctypes.c_void_p), s_ref, smax_rule,
        _ptr(X), _ptr(y), ctypes.cast(sr, ctypes.c_void_p), ctypes.cast(ep, ctypes.c_void_p)))
    eps = list(ep)[:count * s_ref]
    return list(sr)[:count * ntol], [eps[b * s_ref:(b + 1) * s_ref] for b in range(count)]


def oz_mlp_create(handle, seed=0):
    out = ctypes.c_void_p()
    _check("oz_mlp_create", _lib.oz_mlp_create(handle, seed, ctypes.byref(out)))
    return out


def oz_mlp_destroy(mlp):
    return _check("oz_mlp_destroy", _lib.oz_mlp_destroy(mlp))


def oz_mlp_set_params(mlp, params=None, mu=None, sd=None):
    """Host sequences of floats (any may be None)."""
    def arr(v, n):
        return ctypes.cast(_host_array(ctypes.c_float, n, [float(x) for x in v]), ctypes.c_void_p) \
            if v is not None else None
    keep = [arr(params, OZ_MLP_NPARAM), arr(mu, 16), arr(sd, 16)]
    return _check("oz_mlp_set_params", _lib.oz_mlp_set_params(mlp, *keep))


def oz_mlp_get_params(mlp):
    """-> (params, mu, sd) as lists of floats."""
    p = _host_array(ctypes.c_float, OZ_MLP_NPARAM)
    mu = _host_array(ctypes.c_float, 16)
    sd = _host_array(ctypes.c_float, 16)
    _check("oz_mlp_get_params", _lib.oz_mlp_get_params(mlp, ctypes.cast(p, ctypes.c_void_p),
                                                        ctypes.cast(mu, ctypes.c_void_p),
                                                        ctypes.cast(sd, ctypes.c_void_p)))
    return list(p), list(mu), list(sd)


def oz_mlp_fit_norm(mlp, rows, X):
    return _check("oz_mlp_fit_norm", _lib.oz_mlp_fit_norm(mlp, rows, _ptr(X)))


def oz_mlp_forward(mlp, rows, X, y):
    return _check("oz_mlp_forward", _lib.oz_mlp_forward(mlp, rows, _ptr(X), _ptr(y)))


def oz_mlp_grad(mlp, rows, X, t, tau):
    """-> (gradient list, loss)."""
    g = _host_array(ctypes.c_float, OZ_MLP_NPARAM)
    loss = ctypes.c_float()
    _check("oz_mlp_grad", _lib.oz_mlp_grad(mlp, rows, _ptr(X), _ptr(t), tau, ctypes.cast(g, ctypes.c_void_p),
                                            ctypes.byref(loss)))
    return list(g), loss.value


def oz_mlp_train_step(mlp, rows, X, t, tau, lr):
    loss = ctypes.c_float()
    _check("oz_mlp_train_step", _lib.oz_mlp_train_step(mlp, rows, _ptr(X), _ptr(t), tau, lr, ctypes.byref(loss)))
    return loss.value


def oz_mlp_train(mlp, rows, X, t, epochs, batch=256, tau=0.9, lr=1e-3, seed=0):
    """-> mean loss of every epoch."""
    el = _host_array(ctypes.c_float, epochs)
    _check("oz_mlp_train", _lib.oz_mlp_train(mlp, rows, _ptr(X), _ptr(t), epochs, batch, tau, lr, seed,
                                              ctypes.cast(el, ctypes.c_void_p)))
    return list(el)[:epochs]


def oz_mlp_save(mlp, path):
    return _check("oz_mlp_save", _lib.oz_mlp_save(mlp, path.encode()))


def oz_mlp_load(handle, path=None):
    out = ctypes.c_void_p()
    _check("oz_mlp_load", _lib.oz_mlp_load(handle, (SELECTOR_PATH if path is None else path).encode(),
                                            ctypes.byref(out)))
    return out


def oz_set_selector(handle, mlp):
    return _check("oz_set_selector", _lib.oz_set_selector(handle, mlp))


def oz_predict_slices(handle, transa, transb, m, n, k, is_complex, A, lda, B, ldb, tol, smax=0):
    out = ctypes.c_int32()
    _check("oz_predict_slices", _lib.oz_predict_slices(handle, _ch(transa), _ch(transb), m, n, k, int(is_complex),
                                                        _ptr(A), lda, _ptr(B), ldb, float(tol), smax,
                                                        ctypes.byref(out)))
    return out.value


def oz_peak(handle, kind, iters, src=None, dst=None, nbytes=0):
    """Measured rate: kind 0 INT8 MFMA ops/s (32 x 32 x 32 shape), 1 FP64 MFMA
    flop/s, 2 device copy bytes/s (read + written) from src to dst, 3 INT8
    MFMA ops/s (16 x 16 x 64 shape), 4 INT8 MFMA ops/s (32 x 32 x 32 shape,
    full-range operands that change between instructions)."""
    out = ctypes.c_double()
    _check("oz_peak", _lib.oz_peak(handle, int(kind), int(iters), _ptr(src), _ptr(dst), int(nbytes),
                                   ctypes.byref(out)))
    return out.value
