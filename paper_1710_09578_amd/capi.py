"""ctypes binding of the C ABI in ``include/fm.h``, one Python function per C
entry point and with the same name.

Arguments are marshalled only: device pointers are passed as integers (or
torch tensors, whose ``data_ptr()`` is taken), streams as integers holding a
``hipStream_t``. A non-zero status raises ``FmError`` with the library's own
error text. The shared library must have been built (``build()``); loading
fails loudly otherwise -- there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfm.so")

FM_C64, FM_C128, FM_I32, FM_I64 = 1, 2, 3, 4
FM_FWD, FM_ADJ = 0, 1
FM_PRODUCT, FM_SUM, FM_KRON, FM_BLKDIAG = 0, 1, 2, 3

STATUS = {
    0: "FM_OK",
    1: "FM_E_INVALID",
    2: "FM_E_SHAPE",
    3: "FM_E_DTYPE",
    4: "FM_E_ALIAS",
    5: "FM_E_UNSUPPORTED",
    6: "FM_E_WORKSPACE",
    7: "FM_E_NOMEM",
    8: "FM_E_DEVICE",
    9: "FM_E_RELEASED",
}


class FmError(RuntimeError):
    """A library call returned a non-zero fm_status."""

    def __init__(self, func: str, status: int, text: str):
        self.status = status
        self.code = STATUS.get(status, str(status))
        super().__init__(f"{func}: {self.code}: {text}")


class fm_fista_opts(C.Structure):
    _fields_ = [
        ("max_iters", C.c_int32),
        ("momentum", C.c_int32),
        ("x0_given", C.c_int32),
        ("power_max_iters", C.c_int32),
        ("lambda_abs", C.c_double),
        ("lambda_rel", C.c_double),
        ("L", C.c_double),
        ("stop_tol", C.c_double),
        ("power_tol", C.c_double),
        ("seed", C.c_uint64),
    ]


class fm_fista_stat(C.Structure):
    _fields_ = [
        ("iters_done", C.c_int32),
        ("status", C.c_int32),
        ("L_used", C.c_double),
        ("lambda_used", C.c_double),
    ]


class fm_omp_stat(C.Structure):
    _fields_ = [("atoms", C.c_int32), ("status", C.c_int32), ("res_norm", C.c_double)]


class fm_calib_entry(C.Structure):
    _fields_ = [
        ("cls", C.c_int32),
        ("dt", C.c_int32),
        ("n", C.c_int32),
        ("reserved", C.c_int32),
        ("ncols", C.c_int64),
        ("ms_fast", C.c_double),
        ("ms_dense", C.c_double),
    ]


class fm_batch_schedule(C.Structure):
    _fields_ = [
        ("max_fuse", C.c_int32),
        ("region_mib", C.c_int32),
        ("graphs", C.c_int32),
        ("stages", C.c_int32),
        ("ms", C.c_double),
    ]


P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int32
ST = C.c_int

# name: (restype, argtypes)
SIGNATURES = {
    "fm_op_create_fourier": (ST, [C.POINTER(P), I64, C.c_int]),
    "fm_op_create_hadamard": (ST, [C.POINTER(P), I64, C.c_int]),
    "fm_op_create_diag": (ST, [C.POINTER(P), I64, P, C.c_int, P]),
    "fm_op_create_dense": (ST, [C.POINTER(P), I64, I64, P, I64, C.c_int, P]),
    "fm_op_create_circulant": (ST, [C.POINTER(P), I64, P, C.c_int, P]),
    "fm_op_create_lfsr_circulant": (ST, [C.POINTER(P), I32, C.c_uint64, C.c_uint64, C.c_int, P]),
    "fm_op_create_toeplitz": (ST, [C.POINTER(P), I64, I64, P, P, C.c_int, P]),
    "fm_op_create_mltoeplitz": (ST, [C.POINTER(P), I32, C.POINTER(I64), P, C.c_int, P]),
    "fm_op_create_select_rows": (ST, [C.POINTER(P), I64, I64, P, C.c_int, P]),
    "fm_op_compose": (ST, [C.POINTER(P), C.c_int, I32, C.POINTER(P)]),
    "fm_op_create_blocks": (ST, [C.POINTER(P), I32, I32, C.POINTER(P)]),
    "fm_omp": (ST, [P, I64, P, I64, I32, C.c_double, P, I64, P, C.POINTER(fm_omp_stat), P, C.c_size_t, P]),
    "fm_omp_workspace_size": (ST, [P, I64, I32, C.POINTER(C.c_size_t)]),
    "fm_op_adjoint": (ST, [C.POINTER(P), P]),
    "fm_op_conj": (ST, [C.POINTER(P), P]),
    "fm_op_gram": (ST, [C.POINTER(P), P]),
    "fm_op_inverse": (ST, [C.POINTER(P), P]),
    "fm_op_calibrate": (ST, [P, I64, C.POINTER(I32), C.POINTER(C.c_double), C.POINTER(C.c_double), P]),
    "fm_op_set_path": (ST, [P, I32]),
    "fm_calibration_build": (ST, [P]),
    "fm_calibration_entries": (ST, [C.POINTER(fm_calib_entry), I32, C.POINTER(I32)]),
    "fm_calibration_load": (ST, [C.POINTER(fm_calib_entry), I32]),
    "fm_op_choose_path": (ST, [P, I64, C.POINTER(I32)]),
    "fm_op_shape": (ST, [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(C.c_int)]),
    "fm_op_transform_length": (ST, [P, C.POINTER(I64)]),
    "fm_op_release": (ST, [P]),
    "fm_workspace_size": (ST, [P, C.c_int, I64, C.POINTER(C.c_size_t)]),
    "fm_apply": (ST, [P, C.c_int, I64, P, I64, P, I64, P, C.c_size_t, P]),
    "fm_apply_noalloc": (ST, [P, C.c_int, I64, P, I64, P, I64, P]),
    "fm_fista": (ST, [P, I64, P, I64, P, I64, C.POINTER(fm_fista_opts), C.POINTER(fm_fista_stat),
                      P, C.c_size_t, P]),
    "fm_fista_workspace_size": (ST, [P, I64, C.POINTER(fm_fista_opts), C.POINTER(C.c_size_t)]),
    "fm_power_iteration": (ST, [P, P, C.c_uint64, I32, C.c_double, C.POINTER(C.c_double),
                                C.POINTER(I32), P]),
    "fm_batch_create": (ST, [C.POINTER(P), I32, C.POINTER(P), C.POINTER(I64)]),
    "fm_batch_apply": (ST, [P, C.c_int, C.POINTER(P), C.POINTER(I64), C.POINTER(P), C.POINTER(I64), P]),
    "fm_batch_fista": (ST, [P, C.POINTER(P), C.POINTER(I64), C.POINTER(P), C.POINTER(I64),
                            C.POINTER(fm_fista_opts), C.POINTER(fm_fista_stat), P]),
    "fm_batch_release": (ST, [P]),
    "fm_batch_tune": (ST, [P, C.c_int, C.POINTER(P), C.POINTER(I64), C.POINTER(P), C.POINTER(I64), I32,
                           C.POINTER(fm_batch_schedule), P]),
    "fm_batch_get_schedule": (ST, [P, C.POINTER(fm_batch_schedule)]),
    "fm_batch_set_schedule": (ST, [P, C.POINTER(fm_batch_schedule)]),
    "fm_circulant_grad_generator": (ST, [I64, I64, C.c_int, P, I64, P, I64, P, I32, C.c_int, P]),
    "fm_fista_momentum": (ST, [I32, I32, C.POINTER(C.c_double)]),
    "fm_fista_step": (ST, [I64, I64, P, P, P, P, P, P, I64, P, C.c_double, I32, I32, C.c_int, P]),
    "fm_fista_step_vjp": (ST, [I64, I64, P, P, P, P, P, P, I64, P, C.c_double, I32, I32, C.c_int, P]),
    "fm_axpby": (ST, [I64, I64, C.c_double, P, I64, C.c_double, P, I64, P, I64, C.c_int, P]),
    "fm_op_norm_bound": (ST, [P, C.POINTER(C.c_double), P]),
    "fm_last_error": (C.c_char_p, []),
    "fm_version": (C.c_char_p, []),
}

_lib = None


def load(path: str | None = None):
    """Loads libfm.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime of torch first)

    path = path or os.environ.get("FM_LIB", LIB_PATH)
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library {path} is missing: build it with "
            "`python -m paper_1710_09578_amd.build` (there is no fallback path)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(v):
    """Device/host pointer of a tensor, an int, or None."""
    if v is None:
        return None
    if hasattr(v, "data_ptr"):
        return v.data_ptr()
    return int(v)


def _call(name, *args):
    lib = load()
    st = getattr(lib, name)(*args)
    if st != 0:
        raise FmError(name, st, lib.fm_last_error().decode(errors="replace"))
    return st


def fm_last_error() -> str:
    return load().fm_last_error().decode(errors="replace")


def fm_version() -> str:
    return load().fm_version().decode()


def fm_op_create_fourier(n, dt):
    h = P()
    _call("fm_op_create_fourier", C.byref(h), n, dt)
    return h


def fm_op_create_hadamard(n, dt):
    h = P()
    _call("fm_op_create_hadamard", C.byref(h), n, dt)
    return h


def fm_op_create_diag(n, d, dt, stream):
    h = P()
    _call("fm_op_create_diag", C.byref(h), n, _ptr(d), dt, _ptr(stream))
    return h


def fm_op_create_dense(m, n, a, lda, dt, stream):
    h = P()
    _call("fm_op_create_dense", C.byref(h), m, n, _ptr(a), lda, dt, _ptr(stream))
    return h


def fm_op_create_circulant(n, c, dt, stream):
    h = P()
    _call("fm_op_create_circulant", C.byref(h), n, _ptr(c), dt, _ptr(stream))
    return h


def fm_op_create_lfsr_circulant(order, taps, state, dt, stream):
    h = P()
    _call("fm_op_create_lfsr_circulant", C.byref(h), order, taps, state, dt, _ptr(stream))
    return h


def fm_op_create_toeplitz(m, n, col, row, dt, stream):
    h = P()
    _call("fm_op_create_toeplitz", C.byref(h), m, n, _ptr(col), _ptr(row), dt, _ptr(stream))
    return h


def fm_op_create_mltoeplitz(levels, n_per_level, t, dt, stream):
    h = P()
    arr = (I64 * len(n_per_level))(*n_per_level)
    _call("fm_op_create_mltoeplitz", C.byref(h), levels, arr, _ptr(t), dt, _ptr(stream))
    return h


def fm_op_create_select_rows(n_in, m, idx, dt, stream):
    h = P()
    _call("fm_op_create_select_rows", C.byref(h), n_in, m, _ptr(idx), dt, _ptr(stream))
    return h


def fm_op_compose(kind, terms):
    h = P()
    arr = (P * len(terms))(*[t.value if isinstance(t, P) else t for t in terms])
    _call("fm_op_compose", C.byref(h), kind, len(terms), arr)
    return h


def fm_op_create_blocks(nbr, nbc, terms):
    """terms: nbr * nbc handles, row-major."""
    h = P()
    arr = (P * len(terms))(*[t.value if isinstance(t, P) else t for t in terms])
    _call("fm_op_create_blocks", C.byref(h), nbr, nbc, arr)
    return h


def fm_omp(a, ncols, b, ldb, k, tol, x, ldx, support, stats, ws, ws_bytes, stream):
    _call("fm_omp", a, ncols, _ptr(b), ldb, k, tol, _ptr(x), ldx, _ptr(support),
          C.cast(stats, C.POINTER(fm_omp_stat)) if stats is not None else None, _ptr(ws), ws_bytes, _ptr(stream))


def fm_omp_workspace_size(a, ncols, k):
    v = C.c_size_t()
    _call("fm_omp_workspace_size", a, ncols, k, C.byref(v))
    return v.value


def fm_op_adjoint(a):
    h = P()
    _call("fm_op_adjoint", C.byref(h), a)
    return h


def fm_op_conj(a):
    h = P()
    _call("fm_op_conj", C.byref(h), a)
    return h


def fm_op_gram(a):
    h = P()
    _call("fm_op_gram", C.byref(h), a)
    return h


def fm_op_inverse(a):
    h = P()
    _call("fm_op_inverse", C.byref(h), a)
    return h


def fm_op_calibrate(a, ncols, stream):
    choice, tf, td = I32(), C.c_double(), C.c_double()
    _call("fm_op_calibrate", a, ncols, C.byref(choice), C.byref(tf), C.byref(td), _ptr(stream))
    return choice.value, tf.value, td.value


def fm_op_set_path(a, path):
    _call("fm_op_set_path", a, path)


CAL_CLASSES = {0: "circulant", 1: "toeplitz", 2: "fourier"}


def fm_calibration_build(stream):
    _call("fm_calibration_build", _ptr(stream))


def fm_calibration_entries():
    n = I32()
    _call("fm_calibration_entries", None, 0, C.byref(n))
    arr = (fm_calib_entry * max(n.value, 1))()
    _call("fm_calibration_entries", arr, n.value, C.byref(n))
    return [{"cls": arr[i].cls, "dt": arr[i].dt, "n": arr[i].n, "ncols": arr[i].ncols,
             "ms_fast": arr[i].ms_fast, "ms_dense": arr[i].ms_dense} for i in range(n.value)]


def fm_calibration_load(entries):
    arr = (fm_calib_entry * max(len(entries), 1))()
    for i, e in enumerate(entries):
        arr[i] = fm_calib_entry(int(e["cls"]), int(e["dt"]), int(e["n"]), 0, int(e["ncols"]), float(e["ms_fast"]),
                                float(e["ms_dense"]))
    _call("fm_calibration_load", arr, len(entries))


def fm_op_choose_path(a, ncols):
    choice = I32()
    _call("fm_op_choose_path", a, ncols, C.byref(choice))
    return choice.value


def fm_op_shape(a):
    m, n, dt = I64(), I64(), C.c_int()
    _call("fm_op_shape", a, C.byref(m), C.byref(n), C.byref(dt))
    return m.value, n.value, dt.value


def fm_op_transform_length(a):
    L = I64()
    _call("fm_op_transform_length", a, C.byref(L))
    return L.value


def fm_op_release(a):
    _call("fm_op_release", a)


def fm_workspace_size(a, direction, ncols):
    b = C.c_size_t()
    _call("fm_workspace_size", a, direction, ncols, C.byref(b))
    return b.value


def fm_apply(a, direction, ncols, x, ldx, y, ldy, ws, ws_bytes, stream):
    _call("fm_apply", a, direction, ncols, _ptr(x), ldx, _ptr(y), ldy, _ptr(ws), ws_bytes, _ptr(stream))


NOALLOC_SCRATCH_BYTES = 64 << 20


def fm_apply_noalloc(a, direction, ncols, x, ldx, y, ldy, stream):
    _call("fm_apply_noalloc", a, direction, ncols, _ptr(x), ldx, _ptr(y), ldy, _ptr(stream))


def fm_fista_workspace_size(a, ncols, opts):
    b = C.c_size_t()
    _call("fm_fista_workspace_size", a, ncols, C.byref(opts), C.byref(b))
    return b.value


def fm_fista(a, ncols, b, ldb, x, ldx, opts, stats, ws, ws_bytes, stream):
    _call("fm_fista", a, ncols, _ptr(b), ldb, _ptr(x), ldx, C.byref(opts),
          C.cast(stats, C.POINTER(fm_fista_stat)) if stats is not None else None, _ptr(ws), ws_bytes,
          _ptr(stream))


def fm_power_iteration(a, v0, seed, max_iters, tol, stream):
    L = C.c_double()
    its = I32()
    _call("fm_power_iteration", a, _ptr(v0), seed, max_iters, tol, C.byref(L), C.byref(its), _ptr(stream))
    return L.value, its.value


def fm_batch_create(ops, ncols):
    h = P()
    oa = (P * len(ops))(*[o.value if isinstance(o, P) else o for o in ops])
    na = (I64 * len(ncols))(*ncols)
    _call("fm_batch_create", C.byref(h), len(ops), oa, na)
    return h


def _parr(vals):
    return (P * len(vals))(*[_ptr(v) for v in vals])


def _iarr(vals):
    return (I64 * len(vals))(*vals)


def fm_batch_apply(b, direction, xs, ldx, ys, ldy, stream):
    _call("fm_batch_apply", b, direction, _parr(xs), _iarr(ldx), _parr(ys), _iarr(ldy), _ptr(stream))


def fm_batch_fista(b, bvecs, ldb, xs, ldx, opts, stats, stream):
    _call("fm_batch_fista", b, _parr(bvecs), _iarr(ldb), _parr(xs), _iarr(ldx), C.byref(opts),
          C.cast(stats, C.POINTER(fm_fista_stat)) if stats is not None else None, _ptr(stream))


def fm_batch_tune(b, direction, xs, ldx, ys, ldy, reps, stream):
    sc = fm_batch_schedule()
    _call("fm_batch_tune", b, direction, _parr(xs), _iarr(ldx), _parr(ys), _iarr(ldy), reps, C.byref(sc),
          _ptr(stream))
    return _sched_dict(sc)


def _sched_dict(sc):
    return {"max_fuse": sc.max_fuse, "region_mib": sc.region_mib, "graphs": sc.graphs, "stages": sc.stages,
            "ms": sc.ms}


def fm_batch_get_schedule(b):
    sc = fm_batch_schedule()
    _call("fm_batch_get_schedule", b, C.byref(sc))
    return _sched_dict(sc)


def fm_batch_set_schedule(b, max_fuse, region_mib):
    sc = fm_batch_schedule()
    sc.max_fuse = int(max_fuse)
    sc.region_mib = int(region_mib)
    _call("fm_batch_set_schedule", b, C.byref(sc))


def fm_batch_release(b):
    _call("fm_batch_release", b)


def fm_circulant_grad_generator(n, ncols, use, inp, ld_in, g, ld_g, grad_c, accumulate, dt, stream):
    _call("fm_circulant_grad_generator", n, ncols, use, _ptr(inp), ld_in, _ptr(g), ld_g, _ptr(grad_c),
          accumulate, dt, _ptr(stream))


def fm_fista_momentum(it, momentum=1):
    v = C.c_double()
    _call("fm_fista_momentum", it, momentum, C.byref(v))
    return v.value


def fm_fista_step(n, ncols, y, g, x_old, x_new, y_new, z_out, ld, lam, L, it, momentum, dt, stream):
    _call("fm_fista_step", n, ncols, _ptr(y), _ptr(g), _ptr(x_old), _ptr(x_new), _ptr(y_new), _ptr(z_out),
          ld, _ptr(lam), L, it, momentum, dt, _ptr(stream))


def fm_fista_step_vjp(n, ncols, z, gx_new, gy_new, gz, gg, gx_old, ld, lam, L, it, momentum, dt, stream):
    _call("fm_fista_step_vjp", n, ncols, _ptr(z), _ptr(gx_new), _ptr(gy_new), _ptr(gz), _ptr(gg), _ptr(gx_old),
          ld, _ptr(lam), L, it, momentum, dt, _ptr(stream))


def fm_axpby(n, ncols, alpha, x, ldx, beta, y, ldy, out, ldo, dt, stream):
    _call("fm_axpby", n, ncols, alpha, _ptr(x), ldx, beta, _ptr(y), ldy, _ptr(out), ldo, dt, _ptr(stream))


def fm_op_norm_bound(a, stream):
    v = C.c_double()
    _call("fm_op_norm_bound", a, C.byref(v), _ptr(stream))
    return v.value
