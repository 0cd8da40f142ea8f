"""ctypes binding of ``libfth.so`` (the C ABI declared in include/fth.h).

Argument marshalling only: every step of the time integration runs in the
library's HIP kernels.  The functions keep the C names; ``Solver`` is a thin
convenience wrapper.  Importing this module does not touch the GPU; loading
the library raises ``FthError`` if it has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# FTH_LIB_PATH selects another build of the library (e.g. the host-sanitizer build)
LIB_PATH = os.environ.get("FTH_LIB_PATH", os.path.join(_PKG, "libfth.so"))

FTH_OK, FTH_EINVAL, FTH_ENOMEM, FTH_EDEVICE, FTH_ESTATE, FTH_ENONFINITE, FTH_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FTH_DENSE, FTH_CSR = 0, 1
FTH_FP64, FTH_FP32, FTH_FP32_BF16X3 = 0, 1, 2
_STATUS = {0: "FTH_OK", -1: "FTH_EINVAL", -2: "FTH_ENOMEM", -3: "FTH_EDEVICE", -4: "FTH_ESTATE",
           -5: "FTH_ENONFINITE", -6: "FTH_EUNSUPPORTED"}

# Every function the header declares (checked by the CPU tests).
EXPORTS = [
    "fth_default_options", "fth_create", "fth_run", "fth_num_outputs", "fth_read",
    "fth_get_accumulators", "fth_get_state", "fth_set_state", "fth_last_run_ms",
    "fth_launches_per_step", "fth_kernel_name", "fth_propagator", "fth_footprint_bytes",
    "fth_destroy", "fth_last_error", "fth_version", "fth_noise_sample", "fth_force",
    "fth_server_create", "fth_server_submit", "fth_server_tick", "fth_server_poll", "fth_server_result",
    "fth_server_cancel", "fth_server_clock", "fth_server_stats", "fth_server_destroy",
    "fth_spectral_map", "fth_gershgorin", "fth_unscale", "fth_device_bytes", "fth_save", "fth_load",
    "fth_force_noalloc", "fth_set_steps_per_graph",
]
FTH_TARGET_INVSQRT, FTH_TARGET_LN, FTH_TARGET_EXPNEG = 0, 1, 2
FTH_REQ_QUEUED, FTH_REQ_RUNNING, FTH_REQ_DONE, FTH_REQ_FAILED, FTH_REQ_CANCELLED = 0, 1, 2, 3, 4


class FthError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class fth_matrix(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int32), ("value_is_f64", ctypes.c_int32), ("n", ctypes.c_int64),
                ("dense", ctypes.c_void_p), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class fth_gle(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int32), ("A_p", ctypes.c_void_p), ("C_p", ctypes.c_void_p)]


class fth_options(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("burn_in", ctypes.c_int64), ("block_len", ctypes.c_int64), ("acc_diag", ctypes.c_int32),
                ("replicas", ctypes.c_int32), ("hip_stream", ctypes.c_void_p),
                ("steps_per_graph", ctypes.c_int32), ("tune", ctypes.c_int32),
                ("temporal_steps", ctypes.c_int32), ("temporal_threads", ctypes.c_int32),
                ("coded_matrix", ctypes.c_int32), ("acc_pp", ctypes.c_int32),
                ("temporal_persistent", ctypes.c_int32), ("acc_trace", ctypes.c_int32),
                ("scale_r", ctypes.c_double), ("scale_m", ctypes.c_double), ("gle_alpha", ctypes.c_double),
                ("gle_gamma", ctypes.c_double), ("allocator", ctypes.c_void_p)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class fth_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("user", ctypes.c_void_p)]


def torch_allocator():
    """An fth_allocator that takes device memory from PyTorch's caching
    allocator (the struct and its callbacks must be kept alive while a
    context uses them)."""
    import torch

    def _alloc(nbytes, _user):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes)))
        except RuntimeError:
            return None

    def _release(ptr, _user):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = fth_allocator(ALLOC_FN(_alloc), RELEASE_FN(_release), None)
    return a


class fth_server_options(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("steps_per_tick", ctypes.c_int32),
                ("max_active", ctypes.c_int32), ("min_blocks", ctypes.c_int32), ("quantum_ms", ctypes.c_double)]


class fth_request(ctypes.Structure):
    _fields_ = [("M", fth_matrix), ("gle", fth_gle), ("dt", ctypes.c_double), ("pairs", ctypes.c_void_p),
                ("npairs", ctypes.c_int64), ("replicas", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32), ("burn_in", ctypes.c_int64),
                ("block_len", ctypes.c_int64), ("target_rel_stderr", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("scale_r", ctypes.c_double), ("scale_m", ctypes.c_double), ("gle_alpha", ctypes.c_double),
                ("gle_gamma", ctypes.c_double), ("unscale_target", ctypes.c_int32),
                ("momentum_form", ctypes.c_int32)]


class fth_request_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("steps", ctypes.c_int64),
                ("nblocks", ctypes.c_int64), ("max_rel_stderr", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_finish", ctypes.c_double), ("n_out", ctypes.c_int64),
                ("replicas", ctypes.c_int32), ("packed", ctypes.c_int32), ("footprint", ctypes.c_size_t),
                ("device_ms", ctypes.c_double), ("chunks", ctypes.c_int64), ("device_first_ms", ctypes.c_double),
                ("device_last_ms", ctypes.c_double)]


_lib = None


def lib():
    """Load libfth.so (raises FthError if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FthError(FTH_EDEVICE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        sig = {
            "fth_default_options": (None, [P]),
            "fth_create": (i32, [P, P, dbl, P, i64, P, P]),
            "fth_run": (i32, [P, i64, i32]),
            "fth_num_outputs": (i64, [P]),
            "fth_read": (i32, [P, P, P, i64, P]),
            "fth_get_accumulators": (i32, [P, P, P, P, P, P]),
            "fth_get_state": (i32, [P, P, P, P]),
            "fth_set_state": (i32, [P, P, P, P]),
            "fth_last_run_ms": (dbl, [P]),
            "fth_launches_per_step": (i32, [P]),
            "fth_kernel_name": (i32, [P, ctypes.c_char_p, ctypes.c_size_t]),
            "fth_propagator": (i32, [P, dbl, P, P]),
            "fth_footprint_bytes": (ctypes.c_size_t, [P, i32, i32, i64, i32, i32]),
            "fth_destroy": (i32, [P]),
            "fth_last_error": (ctypes.c_char_p, []),
            "fth_version": (ctypes.c_char_p, []),
            "fth_noise_sample": (i32, [u64, ctypes.c_uint32, i64, P, P, P, P, i32, P, P]),
            "fth_force": (i32, [P, P, P]),
            "fth_force_noalloc": (i32, [P, P, P, P]),
            "fth_set_steps_per_graph": (i32, [P, i32]),
            "fth_server_create": (i32, [P, P]),
            "fth_server_submit": (i32, [P, P, P]),
            "fth_server_tick": (i32, [P]),
            "fth_server_poll": (i32, [P, u64, P]),
            "fth_server_result": (i32, [P, u64, P, P, i64]),
            "fth_server_cancel": (i32, [P, u64]),
            "fth_server_clock": (dbl, [P]),
            "fth_server_stats": (i32, [P, P, P, P]),
            "fth_server_destroy": (i32, [P]),
            "fth_spectral_map": (i32, [dbl, dbl, dbl, dbl, P, P]),
            "fth_gershgorin": (i32, [P, P, P]),
            "fth_unscale": (i32, [i32, dbl, dbl, dbl, dbl, i64, P, P, P]),
            "fth_device_bytes": (ctypes.c_size_t, [P]),
            "fth_save": (i32, [P, P, P]),
            "fth_load": (i32, [P, P, ctypes.c_size_t]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != FTH_OK:
        raise FthError(st, lib().fth_last_error().decode())


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def fth_last_error() -> str:
    return lib().fth_last_error().decode()


def fth_version() -> str:
    return lib().fth_version().decode()


def fth_default_options(**kw) -> fth_options:
    o = fth_options()
    lib().fth_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class _Matrix:
    """Keeps the numpy arrays alive while the struct points at them."""

    def __init__(self, M, value_dtype=None):
        self.keep = []
        s = fth_matrix()
        if isinstance(M, np.ndarray):
            d = np.ascontiguousarray(M, dtype=value_dtype or (np.float64 if M.dtype == np.float64 else np.float32))
            self.keep.append(d)
            s.format, s.n, s.dense = FTH_DENSE, d.shape[0], d.ctypes.data
            s.value_is_f64 = int(d.dtype == np.float64)
        else:
            rp = np.ascontiguousarray(M.row_ptr, dtype=np.int64)
            col = np.ascontiguousarray(M.col, dtype=np.int32)
            vd = value_dtype or (np.float64 if M.val.dtype == np.float64 else np.float32)
            val = np.ascontiguousarray(M.val, dtype=vd)
            self.keep += [rp, col, val]
            s.format, s.n, s.nnz = FTH_CSR, int(M.n), int(rp[-1])
            s.row_ptr, s.col, s.val = rp.ctypes.data, col.ctypes.data, val.ctypes.data
            s.value_is_f64 = int(val.dtype == np.float64)
        self.struct = s


def _gle_struct(A_p, C_p):
    A = np.ascontiguousarray(A_p, dtype=np.float64)
    C = np.ascontiguousarray(C_p, dtype=np.float64)
    g = fth_gle()
    g.ns, g.A_p, g.C_p = A.shape[0] - 1, A.ctypes.data, C.ctypes.data
    return g, (A, C)


def fth_propagator(A_p, C_p, dt: float):
    g, keep = _gle_struct(A_p, C_p)
    d = g.ns + 1
    T = np.zeros((d, d))
    S = np.zeros((d, d))
    _check(lib().fth_propagator(ctypes.byref(g), float(dt), _p(T), _p(S)))
    return T, S


def fth_footprint_bytes(M, ns: int, replicas: int, npairs: int, acc_diag: bool, precision: int) -> int:
    m = _Matrix(M)
    return int(lib().fth_footprint_bytes(ctypes.byref(m.struct), ns, replicas, npairs, int(acc_diag), precision))


def fth_create(M, A_p, C_p, dt: float, pairs=None, options: fth_options | None = None):
    """Returns an opaque context handle (ctypes.c_void_p)."""
    opt = options or fth_default_options()
    vd = np.float64 if opt.precision == FTH_FP64 else None
    m = _Matrix(M, vd)
    g, keep = _gle_struct(A_p, C_p)
    pr = np.ascontiguousarray(np.zeros((0, 2)) if pairs is None else pairs, dtype=np.int32).reshape(-1, 2)
    ctx = ctypes.c_void_p()
    _check(lib().fth_create(ctypes.byref(m.struct), ctypes.byref(g), float(dt), _p(pr), len(pr),
                            ctypes.byref(opt), ctypes.byref(ctx)))
    return ctx


def fth_run(ctx, nsteps: int, replicas: int = 0):
    _check(lib().fth_run(ctx, int(nsteps), int(replicas)))


def fth_num_outputs(ctx) -> int:
    return int(lib().fth_num_outputs(ctx))


def fth_read(ctx):
    n = fth_num_outputs(ctx)
    est = np.zeros(n)
    se = np.zeros(n)
    ns = ctypes.c_int64()
    _check(lib().fth_read(ctx, _p(est), _p(se), n, ctypes.byref(ns)))
    return est, se, int(ns.value)


def fth_get_accumulators(ctx):
    n = fth_num_outputs(ctx)
    blk, s1, s2 = np.zeros(n), np.zeros(n), np.zeros(n)
    nb, st = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().fth_get_accumulators(ctx, _p(blk), _p(s1), _p(s2), ctypes.byref(nb), ctypes.byref(st)))
    return blk, s1, s2, int(nb.value), int(st.value)


def fth_get_state(ctx, n: int, R: int, ns: int):
    q, p, s = np.zeros((n, R)), np.zeros((n, R)), np.zeros((ns, n, R))
    _check(lib().fth_get_state(ctx, _p(q), _p(p), _p(s) if ns > 0 else None))
    return q, p, s


def fth_set_state(ctx, q=None, p=None, s=None):
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (q, p, s)]
    _check(lib().fth_set_state(ctx, *[_p(a) for a in arrs]))


def fth_force(ctx, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    F = np.zeros_like(q)
    _check(lib().fth_force(ctx, _p(q), _p(F)))
    return F


def fth_force_noalloc(ctx, q_ptr: int, F_ptr: int, stream_ptr=None):
    """F = -M q on device arrays (raw device addresses in the state
    precision); enqueued on the stream, nothing allocated."""
    _check(lib().fth_force_noalloc(ctx, ctypes.c_void_p(q_ptr), ctypes.c_void_p(F_ptr),
                                   ctypes.c_void_p(stream_ptr) if stream_ptr else None))


def fth_last_run_ms(ctx) -> float:
    return float(lib().fth_last_run_ms(ctx))


def fth_launches_per_step(ctx) -> int:
    return int(lib().fth_launches_per_step(ctx))


def fth_kernel_name(ctx) -> str:
    buf = ctypes.create_string_buffer(128)
    _check(lib().fth_kernel_name(ctx, buf, 128))
    return buf.value.decode()


def fth_noise_sample(seed: int, stream: int, i, r, n, j, precision=FTH_FP64, raw=False):
    shape = np.broadcast(np.asarray(i), np.asarray(r), np.asarray(n), np.asarray(j)).shape
    arrs = [np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.uint32).ravel() for a in (i, r, n, j)]
    cnt = len(arrs[0])
    out = np.zeros(cnt)
    words = np.zeros((cnt, 4), dtype=np.uint32) if raw else None
    _check_plain(lib().fth_noise_sample(seed, stream, cnt, *[_p(a) for a in arrs], precision, _p(out), _p(words)))
    return (out, words) if raw else out


def _check_plain(st: int):
    if st != FTH_OK:
        raise FthError(st, "fth_noise_sample failed")


def fth_spectral_map(e_min: float, e_max: float, w_min: float, w_max: float):
    r, m = ctypes.c_double(), ctypes.c_double()
    _check(lib().fth_spectral_map(e_min, e_max, w_min, w_max, ctypes.byref(r), ctypes.byref(m)))
    return r.value, m.value


def fth_gershgorin(M):
    mat = _Matrix(M)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().fth_gershgorin(ctypes.byref(mat.struct), ctypes.byref(lo), ctypes.byref(hi)))
    return lo.value, hi.value


def fth_unscale(target: int, r: float, m: float, alpha: float, gamma: float, kind_weight, est, se=None):
    """In-place map of position-form estimates of the transformed problem back
    to f(M); returns (est, se) as new float64 arrays."""
    w = np.ascontiguousarray(kind_weight, dtype=np.float64)
    e = np.array(est, dtype=np.float64)
    s = None if se is None else np.array(se, dtype=np.float64)
    _check(lib().fth_unscale(int(target), float(r), float(m), float(alpha), float(gamma), len(e), _p(w), _p(e),
                             _p(s) if s is not None else None))
    return e, s


def fth_device_bytes(ctx) -> int:
    return int(lib().fth_device_bytes(ctx))


def fth_save(ctx) -> bytes:
    n = ctypes.c_size_t()
    _check(lib().fth_save(ctx, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().fth_save(ctx, buf, ctypes.byref(n)))
    return buf.raw[:n.value]


def fth_load(ctx, image: bytes):
    buf = ctypes.create_string_buffer(image, len(image))
    _check(lib().fth_load(ctx, buf, len(image)))


def fth_destroy(ctx):
    if ctx:
        _check(lib().fth_destroy(ctx))


class Solver:
    """One FTH solve: matrix, GLE, time step, selected pairs, options."""

    def __init__(self, M, A_p, C_p, dt, pairs=None, replicas=0, precision=FTH_FP32, seed=0, stream_id=0,
                 burn_in=0, block_len=100, acc_diag=False, steps_per_graph=0, hip_stream=None, tune=False,
                 temporal_steps=0, temporal_threads=0, temporal_persistent=0, coded_matrix=0, acc_pp=False,
                 acc_trace=False,
                 scale_r=1.0, scale_m=0.0, gle_alpha=1.0, gle_gamma=1.0, allocator=None):
        self.n = int(M.shape[0] if isinstance(M, np.ndarray) else M.n)
        self.ns = int(np.asarray(A_p).shape[0] - 1)
        self.R = int(replicas)
        opt = fth_default_options(seed=seed, stream_id=stream_id, precision=precision, burn_in=burn_in,
                                  block_len=block_len, acc_diag=int(acc_diag), replicas=int(replicas),
                                  steps_per_graph=steps_per_graph, tune=int(tune),
                                  temporal_steps=int(temporal_steps), temporal_threads=int(temporal_threads),
                                  temporal_persistent=int(temporal_persistent),
                                  coded_matrix=int(coded_matrix), acc_pp=int(acc_pp), acc_trace=int(acc_trace),
                                  scale_r=float(scale_r), scale_m=float(scale_m), gle_alpha=float(gle_alpha),
                                  gle_gamma=float(gle_gamma))
        if hip_stream is not None:
            opt.hip_stream = hip_stream
        self._allocator = allocator   # the library keeps calling it: hold a reference
        if allocator is not None:
            opt.allocator = ctypes.cast(ctypes.pointer(allocator), ctypes.c_void_p)
        self.ctx = fth_create(M, A_p, C_p, dt, pairs, opt)

    def run(self, nsteps, replicas=0):
        fth_run(self.ctx, nsteps, replicas)
        if replicas:
            self.R = replicas
        return self

    def read(self):
        return fth_read(self.ctx)

    def set_steps_per_graph(self, steps: int):
        _check(lib().fth_set_steps_per_graph(self.ctx, int(steps)))
        return self

    def accumulators(self):
        return fth_get_accumulators(self.ctx)

    def state(self):
        return fth_get_state(self.ctx, self.n, self.R, self.ns)

    def set_state(self, q=None, p=None, s=None):
        fth_set_state(self.ctx, q, p, s)

    def force(self, q):
        return fth_force(self.ctx, q)

    def save(self) -> bytes:
        return fth_save(self.ctx)

    def load(self, image: bytes):
        fth_load(self.ctx, image)
        return self

    @property
    def device_bytes(self) -> int:
        return fth_device_bytes(self.ctx)

    @property
    def last_run_ms(self):
        return fth_last_run_ms(self.ctx)

    @property
    def kernel_name(self):
        return fth_kernel_name(self.ctx)

    def close(self):
        if self.ctx:
            fth_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop over many solves on one GPU (fth_server_*)."""

    def __init__(self, hbm_budget=0, steps_per_tick=0, max_active=0, min_blocks=0, quantum_ms=0.0):
        o = fth_server_options(hbm_budget, steps_per_tick, max_active, min_blocks, float(quantum_ms))
        h = ctypes.c_void_p()
        _check(lib().fth_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.h = h

    def submit(self, M, A_p, C_p, dt, pairs, replicas=0, precision=FTH_FP32, seed=0, stream_id=0, burn_in=0,
               block_len=0, target=1e-2, max_steps=0, scale_r=1.0, scale_m=0.0, gle_alpha=1.0, gle_gamma=1.0,
               unscale_target=-1, momentum_form=False) -> int:
        m = _Matrix(M)
        g, keep = _gle_struct(A_p, C_p)
        pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        q = fth_request(m.struct, g, float(dt), pr.ctypes.data, len(pr), int(replicas), int(precision), int(seed),
                        int(stream_id), int(burn_in), int(block_len), float(target), int(max_steps),
                        float(scale_r), float(scale_m), float(gle_alpha), float(gle_gamma), int(unscale_target),
                        int(bool(momentum_form)))
        rid = ctypes.c_uint64()
        _check(lib().fth_server_submit(self.h, ctypes.byref(q), ctypes.byref(rid)))
        return int(rid.value)

    def tick(self):
        _check(lib().fth_server_tick(self.h))

    def poll(self, rid: int) -> dict:
        info = fth_request_info()
        _check(lib().fth_server_poll(self.h, rid, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in fth_request_info._fields_}

    def result(self, rid: int):
        n = self.poll(rid)["n_out"]
        est, se = np.zeros(n), np.zeros(n)
        _check(lib().fth_server_result(self.h, rid, _p(est), _p(se), n))
        return est, se

    def cancel(self, rid: int):
        _check(lib().fth_server_cancel(self.h, rid))

    def clock(self) -> float:
        return float(lib().fth_server_clock(self.h))

    def stats(self):
        q, r, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        _check(lib().fth_server_stats(self.h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b)))
        return int(q.value), int(r.value), int(b.value)

    def close(self):
        if self.h:
            lib().fth_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
