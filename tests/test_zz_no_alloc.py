"""The allocation-free dense force (fth_force_noalloc): its work buffers
live in one fixed device array per GPU, for callers that cannot allocate.
It must agree with fth_force (which allocates its scratch per call) bit for
bit, on consecutive calls that reuse the array with a smaller system second,
in both precisions, and reject a system whose work space exceeds the array."""
import ctypes

import numpy as np
import pytest

import fth_inputs as fi
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu


class DeviceArray:
    """Caller-side device buffer from the HIP runtime the library already
    loaded (the caller allocates; the entry point under test must not)."""
    _hip = None

    @classmethod
    def hip(cls):
        if cls._hip is None:
            fth.lib()
            L = ctypes.CDLL("libamdhip64.so.7")
            L.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
            L.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
            L.hipFree.argtypes = [ctypes.c_void_p]
            cls._hip = L
        return cls._hip

    def __init__(self, host: np.ndarray):
        self.shape, self.dtype, self.nbytes = host.shape, host.dtype, host.nbytes
        self.ptr = ctypes.c_void_p()
        assert self.hip().hipMalloc(ctypes.byref(self.ptr), self.nbytes) == 0
        self.put(host)

    def put(self, host):
        h = np.ascontiguousarray(host, dtype=self.dtype)
        assert self.hip().hipMemcpy(self.ptr, h.ctypes.data, self.nbytes, 1) == 0   # host to device

    def get(self):
        out = np.empty(self.shape, dtype=self.dtype)
        assert self.hip().hipMemcpy(out.ctypes.data, self.ptr, self.nbytes, 2) == 0   # device to host (synchronous)
        return out

    def free(self):
        self.hip().hipFree(self.ptr)


def dense_solver(n, R, prec, seed):
    M = fi.dense_ggt(n, seed)
    g = fi.load_gle("invsqrt_ns4")
    sol = fth.Solver(M, g.A_p, g.C_p, fi.dt_rule(fi.power_lambda_max(M.astype(np.float64))), replicas=R,
                     precision=prec, seed=seed)
    sol.run(0)   # fixes R: the context holds M and its state, the force needs no more allocations
    return sol


def force_both(sol, n, R, prec, seed):
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((n, R))
    if prec == fth.FTH_FP32_BF16X3:
        q = q.astype(np.float32).astype(np.float64)   # the state precision
    ref = sol.force(q)
    dt = np.float64 if prec == fth.FTH_FP64 else np.float32
    qd = DeviceArray(q.astype(dt))
    Fd = DeviceArray(np.full((n, R), np.nan, dtype=dt))
    fth.fth_force_noalloc(sol.ctx, qd.ptr.value, Fd.ptr.value)   # the context's stream
    sol.read()            # waits for the context's stream
    got = Fd.get().astype(np.float64)
    qd.free()
    Fd.free()
    return got, ref


@pytest.mark.parametrize("prec", [fth.FTH_FP32_BF16X3, fth.FTH_FP64], ids=["bf16x3", "fp64"])
def test_noalloc_force_matches_fth_force(prec):
    print(f"[noalloc] prec={prec}", flush=True)
    big = dense_solver(1800, 64, prec, 11)     # first call: padded to 2048 rows
    small = dense_solver(700, 16, prec, 12)    # second call, smaller: 768 rows
    for sol, n, R, seed in ((big, 1800, 64, 21), (small, 700, 16, 22)):
        got, ref = force_both(sol, n, R, prec, seed)
        print(f"  n={n} R={R} max|F|={np.max(np.abs(ref)):.3e}", flush=True)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))
    big.close()
    small.close()


def test_noalloc_force_rejects_oversized_system():
    print("[noalloc] oversized", flush=True)
    n, R = 8192, 128   # FP64: (1 + 8 slices) x 8192 x 128 x 8 bytes = 72 MiB of work space > 64 MiB
    M = np.eye(n) * 2.0
    g = fi.load_gle("invsqrt_ns4")
    sol = fth.Solver(M, g.A_p, g.C_p, 0.05, replicas=R, precision=fth.FTH_FP64)
    sol.run(0)
    q = DeviceArray(np.zeros((n, R)))
    F = DeviceArray(np.zeros((n, R)))
    with pytest.raises(fth.FthError) as e:
        fth.fth_force_noalloc(sol.ctx, q.ptr.value, F.ptr.value)
    assert e.value.status == fth.FTH_EINVAL and "work space" in str(e.value)
    q.free()
    F.free()
    sol.close()
