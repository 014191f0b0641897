"""ctypes binding of the rsilu C ABI (include/rsilu.h).

Argument marshalling only: numpy arrays for host data, torch tensors for
device memory and streams. Every step of the solve runs in the HIP library;
this module raises if the library has not been built.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "librsilu.so")

# status codes
OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
EINVAL, ENOMEM, EHIP, ESTATE, EINTERNAL = -1, -2, -3, -4, -5
S_AUTO, S_IDENTITY, S_DENSE, S_NONE, S_CG, S_CHEB = -1, 0, 1, 2, 3, 4
FORM_ALG3, FORM_ALG2 = 0, 1
PREC_FP64, PREC_FP32 = 0, 1
KRYLOV_PCGLS, KRYLOV_LSQR = 0, 1
TRSV_SYNCFREE, TRSV_LEVELS, TRSV_HYBRID = 0, 1, 2
SWEEP_AUTO, SWEEP_TWO_PHASE, SWEEP_SEGMENTED, SWEEP_ROWS = 0, 1, 2, 3
Y_IMPLICIT, Y_EXPLICIT = 0, 1
CG_NONE, CG_JACOBI = 0, 1
# factor / level selectors
L1, L2, U, AHAT, UDIAG, YEXP = 0, 1, 2, 3, 4, 5
LEV_L1, LEV_L1T, LEV_U, LEV_UT = 0, 1, 2, 3
# triangular-solve selectors of rsilu_trsv
T_L1, T_L1T, T_U, T_UT = 0, 1, 2, 3

EXPORTS = [
    "rsilu_params_default", "rsilu_factor", "rsilu_device_bytes", "rsilu_upload", "rsilu_add_rows", "rsilu_remove_rows",
    "rsilu_get_stats",
    "rsilu_get_perm", "rsilu_get_colnorm", "rsilu_factor_nnz", "rsilu_get_factor", "rsilu_get_levels",
    "rsilu_solve", "rsilu_spmv", "rsilu_trsv", "rsilu_apply", "rsilu_apply_z", "rsilu_set_profiling",
    "rsilu_set_profiling_mask", "rsilu_get_profile",
    "rsilu_destroy", "rsilu_status_string",
    "rsilu_server_create", "rsilu_server_submit", "rsilu_server_poll", "rsilu_server_drain", "rsilu_server_destroy",
    "rsilu_batch_tiles", "rsilu_batch_accepts", "rsilu_batch_create", "rsilu_batch_solve", "rsilu_batch_solve_auto", "rsilu_batch_destroy",
    "rsilu_tuner_create",
    "rsilu_tune", "rsilu_tuner_size", "rsilu_tuner_destroy", "rsilu_batch_solve_static", "rsilu_batch_static_max",
]
PROF_NAMES = ["spmv_A", "spmv_AT", "trsv_L1", "trsv_L1T", "trsv_U", "spmv_L2", "spmv_L2T", "dense_S", "trsv_UT",
              "k_trsv_sweep", "k_trsv_level", "k_gather_lo", "k_spmv_y"]
# classes that time whole steps (the rest time single kernels)
PROF_STEPS = PROF_NAMES[:9]


class rsilu_params_t(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("tau", ctypes.c_double), ("mu", ctypes.c_double),
                ("small", ctypes.c_double), ("colscale", ctypes.c_int32), ("smode", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("trsv", ctypes.c_int32), ("poll", ctypes.c_int32),
                ("form", ctypes.c_int32), ("precision", ctypes.c_int32), ("cg_steps", ctypes.c_int32),
                ("krylov", ctypes.c_int32), ("graph", ctypes.c_int32), ("sweep", ctypes.c_int32),
                ("ystore", ctypes.c_int32), ("ytau", ctypes.c_double), ("poly_degree", ctypes.c_int32),
                ("poly_delta", ctypes.c_double), ("cg_precond", ctypes.c_int32), ("reserved3", ctypes.c_int32)]


class rsilu_stats_t(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz_a", ctypes.c_int64),
                ("nnz_l1", ctypes.c_int64), ("nnz_l2", ctypes.c_int64), ("nnz_u", ctypes.c_int64),
                ("psize", ctypes.c_int64), ("nmod", ctypes.c_int64), ("levels_l1", ctypes.c_int32),
                ("levels_l1t", ctypes.c_int32), ("levels_u", ctypes.c_int32), ("levels_ut", ctypes.c_int32),
                ("smode", ctypes.c_int32), ("sweep_schemes", ctypes.c_int32), ("device_bytes", ctypes.c_size_t),
                ("nnz_y", ctypes.c_int64), ("cheb_b", ctypes.c_double), ("cheb_degree", ctypes.c_int32),
                ("reserved2", ctypes.c_int32), ("cheb_scale", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("reserved")}


class rsilu_profile_t(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 13), ("ms", ctypes.c_double * 13), ("bytes", ctypes.c_double * 13)]


class rsilu_tile_t(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("spmv_lanes", ctypes.c_int32), ("tri_lanes", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_tuple(self):
        return (self.threads, self.spmv_lanes, self.tri_lanes)


class rsilu_server_opts_t(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("slots", ctypes.c_int32), ("setup_threads", ctypes.c_int32),
                ("batch_max", ctypes.c_int32), ("hbm_bytes", ctypes.c_size_t), ("tune_slack", ctypes.c_double),
                ("batch_wait_ms", ctypes.c_double)]


class rsilu_request_t(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("tol", ctypes.c_double), ("params", rsilu_params_t),
                ("user", ctypes.c_void_p)]


class rsilu_result_t(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("user", ctypes.c_void_p), ("status", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("atr_norm", ctypes.c_double), ("atr_rel", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("wait_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("device_bytes", ctypes.c_size_t), ("path", ctypes.c_int32),
                ("launch_size", ctypes.c_int32), ("tile", rsilu_tile_t)]


class rsilu_batch_result_t(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("atr_norm", ctypes.c_double),
                ("atr_rel", ctypes.c_double)]


class rsilu_tune_result_t(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("tile", rsilu_tile_t),
                ("batched_ms_per_iter", ctypes.c_double), ("plain_ms_per_iter", ctypes.c_double)]


class RsiluError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s: %s (status %d)" % (what, status_string(code), code))
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librsilu.so is not built (run __graft_entry__.build() or "
                               "python paper_2603_28642_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.rsilu_params_default.argtypes = [ctypes.POINTER(rsilu_params_t)]
        L.rsilu_params_default.restype = None
        L.rsilu_factor.argtypes = [I64, I64, P, P, P, ctypes.POINTER(rsilu_params_t), ctypes.POINTER(P)]
        L.rsilu_factor.restype = ctypes.c_int
        L.rsilu_device_bytes.argtypes = [P]
        L.rsilu_device_bytes.restype = ctypes.c_size_t
        L.rsilu_upload.argtypes = [P, P, ctypes.c_size_t, P]
        L.rsilu_upload.restype = ctypes.c_int
        L.rsilu_add_rows.argtypes = [P, I64, P, P, P]
        L.rsilu_add_rows.restype = ctypes.c_int
        L.rsilu_remove_rows.argtypes = [P, I64, P]
        L.rsilu_remove_rows.restype = ctypes.c_int
        L.rsilu_get_stats.argtypes = [P, ctypes.POINTER(rsilu_stats_t)]
        L.rsilu_get_stats.restype = ctypes.c_int
        L.rsilu_get_perm.argtypes = [P, P]
        L.rsilu_get_perm.restype = ctypes.c_int
        L.rsilu_get_colnorm.argtypes = [P, P]
        L.rsilu_get_colnorm.restype = ctypes.c_int
        L.rsilu_factor_nnz.argtypes = [P, I32]
        L.rsilu_factor_nnz.restype = I64
        L.rsilu_get_factor.argtypes = [P, I32, P, P, P]
        L.rsilu_get_factor.restype = ctypes.c_int
        L.rsilu_get_levels.argtypes = [P, I32, P, P]
        L.rsilu_get_levels.restype = ctypes.c_int
        L.rsilu_solve.argtypes = [P, P, D, P, ctypes.POINTER(I32), ctypes.POINTER(D), ctypes.POINTER(D), P]
        L.rsilu_solve.restype = ctypes.c_int
        L.rsilu_spmv.argtypes = [P, I32, P, P, P]
        L.rsilu_spmv.restype = ctypes.c_int
        L.rsilu_trsv.argtypes = [P, I32, P, P, P]
        L.rsilu_trsv.restype = ctypes.c_int
        L.rsilu_apply.argtypes = [P, P, P, P]
        L.rsilu_apply.restype = ctypes.c_int
        L.rsilu_apply_z.argtypes = [P, P, P, P]
        L.rsilu_apply_z.restype = ctypes.c_int
        L.rsilu_set_profiling.argtypes = [P, I32]
        L.rsilu_set_profiling.restype = ctypes.c_int
        L.rsilu_set_profiling_mask.argtypes = [P, ctypes.c_uint32]
        L.rsilu_set_profiling_mask.restype = ctypes.c_int
        L.rsilu_get_profile.argtypes = [P, ctypes.POINTER(rsilu_profile_t)]
        L.rsilu_get_profile.restype = ctypes.c_int
        L.rsilu_destroy.argtypes = [P]
        L.rsilu_destroy.restype = None
        L.rsilu_status_string.argtypes = [ctypes.c_int]
        L.rsilu_status_string.restype = ctypes.c_char_p
        L.rsilu_server_create.argtypes = [ctypes.POINTER(rsilu_server_opts_t), ctypes.POINTER(P)]
        L.rsilu_server_create.restype = ctypes.c_int
        L.rsilu_server_submit.argtypes = [P, ctypes.POINTER(rsilu_request_t), ctypes.POINTER(I64)]
        L.rsilu_server_submit.restype = ctypes.c_int
        L.rsilu_server_poll.argtypes = [P, ctypes.POINTER(rsilu_result_t), I32, I32]
        L.rsilu_server_poll.restype = I32
        L.rsilu_server_drain.argtypes = [P]
        L.rsilu_server_drain.restype = ctypes.c_int
        L.rsilu_server_destroy.argtypes = [P]
        L.rsilu_server_destroy.restype = None
        L.rsilu_batch_tiles.argtypes = [ctypes.POINTER(rsilu_tile_t), I32]
        L.rsilu_batch_tiles.restype = I32
        L.rsilu_batch_accepts.argtypes = [P]
        L.rsilu_batch_accepts.restype = I32
        L.rsilu_batch_create.argtypes = [I32, ctypes.POINTER(P)]
        L.rsilu_batch_create.restype = ctypes.c_int
        L.rsilu_batch_solve.argtypes = [P, I32, P, P, P, P, ctypes.POINTER(rsilu_tile_t),
                                        ctypes.POINTER(rsilu_batch_result_t), P]
        L.rsilu_batch_solve.restype = ctypes.c_int
        L.rsilu_batch_solve_auto.argtypes = [P, P, I32, P, P, P, P, ctypes.POINTER(rsilu_batch_result_t),
                                             ctypes.POINTER(I32), ctypes.POINTER(rsilu_tile_t), P]
        L.rsilu_batch_solve_auto.restype = ctypes.c_int
        L.rsilu_batch_solve_static.argtypes = [I32, P, P, P, P, ctypes.POINTER(rsilu_tile_t),
                                               ctypes.POINTER(rsilu_batch_result_t), P]
        L.rsilu_batch_solve_static.restype = ctypes.c_int
        L.rsilu_batch_static_max.argtypes = []
        L.rsilu_batch_static_max.restype = I32
        L.rsilu_batch_destroy.argtypes = [P]
        L.rsilu_batch_destroy.restype = None
        L.rsilu_tuner_create.argtypes = [D, I32, ctypes.POINTER(P)]
        L.rsilu_tuner_create.restype = ctypes.c_int
        L.rsilu_tune.argtypes = [P, P, P, P, ctypes.POINTER(rsilu_tune_result_t), P]
        L.rsilu_tune.restype = ctypes.c_int
        L.rsilu_tuner_size.argtypes = [P]
        L.rsilu_tuner_size.restype = I32
        L.rsilu_tuner_destroy.argtypes = [P]
        L.rsilu_tuner_destroy.restype = None
        _lib = L
    return _lib


def status_string(code):
    return lib().rsilu_status_string(int(code)).decode()


def _check(code, what):
    if code < 0:
        raise RsiluError(code, what)
    return code


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _dev(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- the C calls


def rsilu_params_default(**overrides):
    p = rsilu_params_t()
    lib().rsilu_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def rsilu_factor(m, n, rowptr, colind, val, params=None):
    rp, prp = _host(rowptr, np.int64)
    ci, pci = _host(colind, np.int32)
    vv, pvv = _host(val, np.float64)
    if rp.shape != (m + 1,):
        raise ValueError("rowptr must have m + 1 entries")
    nnz = int(rp[-1]) if rp.size else 0
    if ci.size < nnz or vv.size < nnz:
        raise ValueError("colind/val shorter than rowptr[m]")
    h = ctypes.c_void_p()
    code = lib().rsilu_factor(int(m), int(n), prp, pci, pvv,
                              ctypes.byref(params) if params is not None else None, ctypes.byref(h))
    return code, (h if code == OK else None)


def rsilu_device_bytes(h):
    return int(lib().rsilu_device_bytes(h))


def rsilu_upload(h, dev_buf, stream=None):
    nbytes = dev_buf.numel() * dev_buf.element_size()
    return lib().rsilu_upload(h, _dev(dev_buf), nbytes, _stream(stream))


def rsilu_add_rows(h, rowptr, colind, val):
    """Append rows (host CSR) to the handle's A; the handle must be uploaded again."""
    rp, prp = _host(rowptr, np.int64)
    ci, pci = _host(colind, np.int32)
    vv, pvv = _host(val, np.float64)
    return lib().rsilu_add_rows(h, len(rp) - 1, prp, pci, pvv)


def rsilu_remove_rows(h, rows):
    """Remove rows (current numbering) from the handle's A; the handle must be uploaded again."""
    rr, prr = _host(rows, np.int64)
    return lib().rsilu_remove_rows(h, len(rr), prr)


def rsilu_get_stats(h):
    s = rsilu_stats_t()
    _check(lib().rsilu_get_stats(h, ctypes.byref(s)), "rsilu_get_stats")
    return s


def rsilu_get_perm(h, m):
    out = np.empty(m, dtype=np.int32)
    _check(lib().rsilu_get_perm(h, out.ctypes.data_as(ctypes.c_void_p)), "rsilu_get_perm")
    return out


def rsilu_get_colnorm(h, n):
    out = np.empty(n, dtype=np.float64)
    _check(lib().rsilu_get_colnorm(h, out.ctypes.data_as(ctypes.c_void_p)), "rsilu_get_colnorm")
    return out


def rsilu_factor_nnz(h, which):
    return int(lib().rsilu_factor_nnz(h, int(which)))


def rsilu_get_factor(h, which, nrows):
    """(rowptr int64, col int32, val float64) of factor `which`, or val only for UDIAG."""
    nnz = rsilu_factor_nnz(h, which)
    if nnz < 0:
        raise ValueError("bad factor selector")
    val = np.empty(nnz, dtype=np.float64)
    if which == UDIAG:
        _check(lib().rsilu_get_factor(h, which, None, None, val.ctypes.data_as(ctypes.c_void_p)), "get_factor")
        return val
    rowptr = np.empty(nrows + 1, dtype=np.int64)
    col = np.empty(nnz, dtype=np.int32)
    _check(lib().rsilu_get_factor(h, which, rowptr.ctypes.data_as(ctypes.c_void_p),
                                  col.ctypes.data_as(ctypes.c_void_p), val.ctypes.data_as(ctypes.c_void_p)),
           "get_factor")
    return rowptr, col, val


def rsilu_get_levels(h, which, n, nlev):
    ptr = np.empty(nlev + 1, dtype=np.int32)
    rows = np.empty(n, dtype=np.int32)
    _check(lib().rsilu_get_levels(h, int(which), ptr.ctypes.data_as(ctypes.c_void_p),
                                  rows.ctypes.data_as(ctypes.c_void_p)), "get_levels")
    return ptr, rows


def rsilu_solve(h, b_dev, tol, x_dev, stream=None):
    it = ctypes.c_int32(0)
    atr = ctypes.c_double(0.0)
    rel = ctypes.c_double(0.0)
    code = lib().rsilu_solve(h, _dev(b_dev), float(tol), _dev(x_dev), ctypes.byref(it), ctypes.byref(atr),
                             ctypes.byref(rel), _stream(stream))
    return code, int(it.value), float(atr.value), float(rel.value)


def rsilu_spmv(h, op, x_dev, y_dev, stream=None):
    return lib().rsilu_spmv(h, int(op), _dev(x_dev), _dev(y_dev), _stream(stream))


def rsilu_trsv(h, which, rhs_dev, x_dev, stream=None):
    return lib().rsilu_trsv(h, int(which), _dev(rhs_dev), _dev(x_dev), _stream(stream))


def rsilu_apply(h, r_dev, h_dev, stream=None):
    return lib().rsilu_apply(h, _dev(r_dev), _dev(h_dev), _stream(stream))


def rsilu_apply_z(h, z_dev, h_dev, stream=None):
    return lib().rsilu_apply_z(h, _dev(z_dev), _dev(h_dev), _stream(stream))


def rsilu_set_profiling(h, enable):
    return lib().rsilu_set_profiling(h, 1 if enable else 0)


def rsilu_set_profiling_mask(h, names):
    """Time only the named classes (names from PROF_NAMES; empty: profiling off)."""
    mask = 0
    for name in names:
        mask |= 1 << PROF_NAMES.index(name)
    return lib().rsilu_set_profiling_mask(h, mask)


def rsilu_get_profile(h):
    """{class: (launches, total ms, algorithmic bytes)} from the HIP events recorded during solves
    (bytes are reported for the single-kernel classes only)."""
    p = rsilu_profile_t()
    _check(lib().rsilu_get_profile(h, ctypes.byref(p)), "rsilu_get_profile")
    return {name: (int(p.launches[i]), float(p.ms[i]), float(p.bytes[i])) for i, name in enumerate(PROF_NAMES)}


def rsilu_destroy(h):
    if h is not None:
        lib().rsilu_destroy(h)


# ---------------------------------------------------------------- convenience


class Solver:
    """Owns a handle and the device buffer it was uploaded to."""

    def __init__(self, m, n, rowptr, colind, val, device="cuda", **params):
        self.m, self.n = int(m), int(n)
        self.params = rsilu_params_default(**params)
        code, h = rsilu_factor(m, n, rowptr, colind, val, self.params)
        _check(code, "rsilu_factor")
        if code != OK:
            raise RsiluError(code, "rsilu_factor")
        self.h = h
        self.stats = rsilu_get_stats(h)
        self.buf = None
        self.device = device

    @classmethod
    def from_problem(cls, prob, **params):
        return cls(prob.m, prob.n, prob.rowptr, prob.col, prob.val, **params)

    def upload(self, stream=None):
        import torch

        nbytes = rsilu_device_bytes(self.h)
        # over-allocate so the buffer can start on a 256-byte boundary
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self.buf = raw[off:off + nbytes]
        self._raw = raw
        _check(rsilu_upload(self.h, self.buf, stream), "rsilu_upload")
        return self

    def solve(self, b_dev, tol=1e-8, x_dev=None, stream=None):
        import torch

        if x_dev is None:
            x_dev = torch.empty(self.n, dtype=torch.float64, device=b_dev.device)
        code, it, atr, rel = rsilu_solve(self.h, b_dev, tol, x_dev, stream)
        _check(code, "rsilu_solve")
        return x_dev, code, it, atr, rel

    def add_rows(self, rowptr, colind, val, stream=None):
        """Append rows (Section 3.4) and upload the grown layout to a new buffer."""
        _check(rsilu_add_rows(self.h, rowptr, colind, val), "rsilu_add_rows")
        self.m += len(rowptr) - 1
        self.stats = rsilu_get_stats(self.h)
        return self.upload(stream)

    def remove_rows(self, rows, stream=None):
        """Remove rows (Section 3.4) and upload the changed layout to a new buffer."""
        _check(rsilu_remove_rows(self.h, rows), "rsilu_remove_rows")
        self.m -= len(rows)
        self.stats = rsilu_get_stats(self.h)
        return self.upload(stream)

    def perm(self):
        return rsilu_get_perm(self.h, self.m)

    def close(self):
        if self.h is not None:
            rsilu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The serving runtime (include/rsilu_serve.h): submit host problems, poll results.
    Host inputs are copied at submit; each request's x buffer is kept alive here until
    its result has been polled."""

    def __init__(self, hbm_bytes, slots=4, setup_threads=4, device=0, batch_max=0, tune_slack=0.0, batch_wait_ms=0.0):
        opts = rsilu_server_opts_t(device=device, slots=slots, setup_threads=setup_threads, batch_max=int(batch_max),
                                   hbm_bytes=int(hbm_bytes), tune_slack=float(tune_slack),
                                   batch_wait_ms=float(batch_wait_ms))
        h = ctypes.c_void_p()
        _check(lib().rsilu_server_create(ctypes.byref(opts), ctypes.byref(h)), "rsilu_server_create")
        self.h = h
        self.pending = {}  # id -> x array (and the problem, for the caller)

    def submit(self, m, n, rowptr, colind, val, b, tol=1e-8, **params):
        rp, prp = _host(rowptr, np.int64)
        ci, pci = _host(colind, np.int32)
        vv, pvv = _host(val, np.float64)
        bb, pbb = _host(b, np.float64)
        x = np.zeros(n, dtype=np.float64)
        req = rsilu_request_t(m=int(m), n=int(n), rowptr=prp, colind=pci, val=pvv, b=pbb,
                              x=x.ctypes.data_as(ctypes.c_void_p), tol=float(tol),
                              params=rsilu_params_default(**params), user=None)
        rid = ctypes.c_int64(-1)
        _check(lib().rsilu_server_submit(self.h, ctypes.byref(req), ctypes.byref(rid)), "rsilu_server_submit")
        self.pending[rid.value] = x
        return rid.value

    def poll(self, max_results=64, wait_ms=0):
        """[(result dict, x)] of completed requests."""
        buf = (rsilu_result_t * max_results)()
        k = lib().rsilu_server_poll(self.h, buf, max_results, int(wait_ms))
        out = []
        for i in range(k):
            r = buf[i]
            d = {f: getattr(r, f) for f, _ in r._fields_ if f not in ("user", "tile")}
            d["tile"] = r.tile.as_tuple()
            out.append((d, self.pending.pop(r.id)))
        return out

    def drain(self):
        _check(lib().rsilu_server_drain(self.h), "rsilu_server_drain")

    def close(self):
        if self.h is not None:
            lib().rsilu_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- batched persistent solves


def rsilu_batch_accepts(h):
    """Whether the batched kernel takes the handle's configuration."""
    return bool(lib().rsilu_batch_accepts(h))


def rsilu_batch_tiles():
    """The compiled tiles of the persistent kernel, as (threads, spmv_lanes, tri_lanes)."""
    k = lib().rsilu_batch_tiles(None, 0)
    buf = (rsilu_tile_t * k)()
    lib().rsilu_batch_tiles(buf, k)
    return [buf[i].as_tuple() for i in range(k)]


def make_tile(tile):
    if tile is None:
        return None
    t, s_, r = tile
    return rsilu_tile_t(threads=t, spmv_lanes=s_, tri_lanes=r, reserved=0)


def rsilu_batch_solve_static(handles, b_devs, tols, x_devs, tile=None, stream=None):
    """The batched solve without a batch object (fixed device descriptor table, no
    allocation). Returns (status code of the call, [result dicts])."""
    k = len(handles)
    hs = (ctypes.c_void_p * max(k, 1))(*[h if isinstance(h, int) else h.value for h in handles])
    bs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in b_devs])
    xs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in x_devs])
    ts = (ctypes.c_double * max(k, 1))(*[float(t) for t in tols])
    res = (rsilu_batch_result_t * max(k, 1))()
    tl = make_tile(tile)
    code = lib().rsilu_batch_solve_static(k, hs, bs, ts, xs, ctypes.byref(tl) if tl is not None else None, res,
                                          _stream(stream))
    return code, [{f: getattr(res[i], f) for f, _ in res[i]._fields_} for i in range(k)]


class Batch:
    """A batch object (include/rsilu_batch.h): solves many uploaded handles in one launch."""

    def __init__(self, capacity):
        h = ctypes.c_void_p()
        _check(lib().rsilu_batch_create(int(capacity), ctypes.byref(h)), "rsilu_batch_create")
        self.h = h
        self.capacity = int(capacity)

    def solve_raw(self, handles, b_devs, tols, x_devs, tile=None, stream=None):
        """Returns (status code of the call, [result dicts])."""
        k = len(handles)
        hs = (ctypes.c_void_p * max(k, 1))(*[h if isinstance(h, int) else h.value for h in handles])
        bs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in b_devs])
        xs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in x_devs])
        ts = (ctypes.c_double * max(k, 1))(*[float(t) for t in tols])
        res = (rsilu_batch_result_t * max(k, 1))()
        tl = make_tile(tile)
        code = lib().rsilu_batch_solve(self.h, k, hs, bs, ts, xs, ctypes.byref(tl) if tl is not None else None,
                                       res, _stream(stream))
        out = [{f: getattr(res[i], f) for f, _ in res[i]._fields_} for i in range(k)]
        return code, out

    def solve(self, solvers, b_devs, tols, x_devs=None, tile=None, stream=None):
        """Solve the problems of `solvers` (uploaded Solver objects); returns (xs, results)."""
        import torch

        if x_devs is None:
            x_devs = [torch.empty(S.n, dtype=torch.float64, device=b.device) for S, b in zip(solvers, b_devs)]
        if not isinstance(tols, (list, tuple)):
            tols = [tols] * len(solvers)
        code, res = self.solve_raw([S.h for S in solvers], b_devs, tols, x_devs, tile, stream)
        _check(code, "rsilu_batch_solve")
        return x_devs, res

    def solve_auto(self, tuner, solvers, b_devs, tols, x_devs=None, stream=None):
        """The autotuner's split between one batched launch and the plain path
        (rsilu_batch_solve_auto); returns (xs, results, paths, tile)."""
        import torch

        k = len(solvers)
        if x_devs is None:
            x_devs = [torch.empty(S.n, dtype=torch.float64, device=b.device) for S, b in zip(solvers, b_devs)]
        if not isinstance(tols, (list, tuple)):
            tols = [tols] * k
        hs = (ctypes.c_void_p * max(k, 1))(*[S.h.value for S in solvers])
        bs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in b_devs])
        xs = (ctypes.c_void_p * max(k, 1))(*[t.data_ptr() for t in x_devs])
        ts = (ctypes.c_double * max(k, 1))(*[float(t) for t in tols])
        res = (rsilu_batch_result_t * max(k, 1))()
        paths = (ctypes.c_int32 * max(k, 1))()
        tile = rsilu_tile_t()
        _check(lib().rsilu_batch_solve_auto(self.h, tuner.h, k, hs, bs, ts, xs, res, paths, ctypes.byref(tile),
                                            _stream(stream)), "rsilu_batch_solve_auto")
        out = [{f: getattr(res[i], f) for f, _ in res[i]._fields_} for i in range(k)]
        return x_devs, out, [paths[i] for i in range(k)], tile.as_tuple()

    def close(self):
        if self.h is not None:
            lib().rsilu_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tuner:
    """The autotuner (include/rsilu_batch.h): per problem signature, the batched tile or the plain path."""

    def __init__(self, slack=1.0, iters=8):
        h = ctypes.c_void_p()
        _check(lib().rsilu_tuner_create(float(slack), int(iters), ctypes.byref(h)), "rsilu_tuner_create")
        self.h = h

    def tune(self, solver, b_dev, x_dev=None, stream=None):
        import torch

        if x_dev is None:
            x_dev = torch.empty(solver.n, dtype=torch.float64, device=b_dev.device)
        r = rsilu_tune_result_t()
        _check(lib().rsilu_tune(self.h, solver.h, _dev(b_dev), _dev(x_dev), ctypes.byref(r), _stream(stream)),
               "rsilu_tune")
        return {"path": r.path, "from_cache": r.from_cache, "tile": r.tile.as_tuple(),
                "batched_ms_per_iter": r.batched_ms_per_iter, "plain_ms_per_iter": r.plain_ms_per_iter}

    def size(self):
        return lib().rsilu_tuner_size(self.h)

    def close(self):
        if self.h is not None:
            lib().rsilu_tuner_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
