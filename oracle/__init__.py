"""FP64 CPU oracle for the f-thermostat (FTH) hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the library and its binding
never do.  It shares no code with the HIP path (its own Philox, its own
propagator, its own step loop); the only common dependency is the seeded
input module ``fth_inputs``.

Layout:
  fth_oracle.c  step loop and noise (plain C, FP64, OpenMP over rows)
  __init__.py   loader, GLE checks, propagator T/S, run wrapper, estimators
  exact.py      exact stationary responses g0(lambda), g_h(lambda), g_h(M)
  fit_gle.py    offline GLE fitter that writes the parameter files

Citations refer to the paper's sections and equations (Nava, Ceriotti,
Dryzun, Parrinello, "Evaluating functions of positive-definite matrices using
colored noise thermostats").
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.linalg

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fth_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True, sanitize: bool = False, out: str | None = None) -> str:
    """Compile the C step loop with gcc (FP64, -O2, OpenMP); with sanitize,
    a copy instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
    (to be loaded with gcc's libasan preloaded)."""
    path = out or _LIB
    if force or not os.path.exists(path):
        tmp = path + ".tmp"
        flags = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                 "-fno-omit-frame-pointer"] if sanitize else []
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", *flags, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, path)
    return path


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("FTH_ORACLE_LIB", _LIB)   # another build of the same source (sanitizer runs)
        if path == _LIB and not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, u64, u32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_philox_batch.argtypes = [i64, P, P, P]
        L.orc_u01.argtypes = [u32]
        L.orc_u01.restype = ctypes.c_double
        L.orc_noise_block.argtypes = [u64, u32, u64, u64, u32, u32, P]
        L.orc_normal.argtypes = [u64, u32, u64, u32, u64, u32]
        L.orc_normal.restype = ctypes.c_double
        L.orc_normals.argtypes = [u64, u32, i64, P, P, P, P, P]
        L.orc_run.argtypes = [i64, ctypes.c_int, P, P, P, P, ctypes.c_int, P, P, ctypes.c_double,
                              i64, u64, u32, i64, i64, i64, i64, P, P, P, i64, P, P, P, P, P, P,
                              ctypes.c_int]
        L.orc_run.restype = ctypes.c_int
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


# --------------------------------------------------------------------------
# Noise
# --------------------------------------------------------------------------
def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Raw Philox4x32-10 blocks: ctr uint32 [count, 4], key (k0, k1)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(len(ctr), _ptr(ctr), _ptr(k), _ptr(out))
    return out


def u01(x: int) -> float:
    return lib().orc_u01(int(x) & 0xFFFFFFFF)


def normals(seed: int, stream: int, i, r, n, j) -> np.ndarray:
    """xi_j for dof i, replica r, step n (vectorised over equal-length arrays)."""
    shape = np.broadcast(np.asarray(i), np.asarray(r), np.asarray(n), np.asarray(j)).shape
    i = np.ascontiguousarray(np.broadcast_to(i, shape), dtype=np.uint64).ravel()
    r = np.ascontiguousarray(np.broadcast_to(r, shape), dtype=np.uint32).ravel()
    n = np.ascontiguousarray(np.broadcast_to(n, shape), dtype=np.uint64).ravel()
    j = np.ascontiguousarray(np.broadcast_to(j, shape), dtype=np.uint32).ravel()
    out = np.empty(len(i), dtype=np.float64)
    lib().orc_normals(seed, stream, len(i), _ptr(i), _ptr(r), _ptr(n), _ptr(j), _ptr(out))
    return out


# --------------------------------------------------------------------------
# GLE checks and the exact OU propagator (Sec. I, Eqs. for A_p, B_p, C_p)
# --------------------------------------------------------------------------
class GLEError(ValueError):
    pass


def diffusion(A_p: np.ndarray, C_p: np.ndarray) -> np.ndarray:
    """B_p B_p^T = A_p C_p + C_p A_p^T (the Lyapunov relation of Sec. I)."""
    return A_p @ C_p + C_p @ A_p.T


def check_gle(A_p: np.ndarray, C_p: np.ndarray, tol: float = 1e-10) -> None:
    """Drift must be stable (all eigenvalues with positive real part), C_p
    symmetric positive definite, and the implied B_p B_p^T positive
    semi-definite."""
    A_p = np.asarray(A_p, dtype=np.float64)
    C_p = np.asarray(C_p, dtype=np.float64)
    d = A_p.shape[0]
    if A_p.shape != (d, d) or C_p.shape != (d, d):
        raise GLEError("A_p and C_p must be square and of equal size")
    if not np.all(np.isfinite(A_p)) or not np.all(np.isfinite(C_p)):
        raise GLEError("non-finite GLE parameters")
    if np.max(np.abs(C_p - C_p.T)) > tol * max(1.0, np.max(np.abs(C_p))):
        raise GLEError("C_p is not symmetric")
    if np.min(np.linalg.eigvals(A_p).real) <= 0:
        raise GLEError("A_p is not stable")
    if np.min(np.linalg.eigvalsh(0.5 * (C_p + C_p.T))) <= 0:
        raise GLEError("C_p is not positive definite")
    bb = diffusion(A_p, C_p)
    bb = 0.5 * (bb + bb.T)
    if np.min(np.linalg.eigvalsh(bb)) < -tol * max(1.0, np.max(np.abs(bb))):
        raise GLEError("A_p C_p + C_p A_p^T is not positive semi-definite")


def propagator(A_p: np.ndarray, C_p: np.ndarray, h: float):
    """Exact one-step Ornstein-Uhlenbeck propagator of the free (p, s) part of
    the Markovian GLE (Sec. I): with drift -A_p and stationary covariance C_p,
    (p, s)(t+h) = T (p, s)(t) + S xi,  T = exp(-A_p h),  S S^T = C_p - T C_p T^T.
    S is the lower Cholesky factor (unique, so trajectories are reproducible).
    """
    check_gle(A_p, C_p)
    T = scipy.linalg.expm(-np.asarray(A_p, dtype=np.float64) * h)
    sig = C_p - T @ C_p @ T.T
    sig = 0.5 * (sig + sig.T)
    try:
        S = np.linalg.cholesky(sig)
    except np.linalg.LinAlgError as e:
        raise GLEError("C_p - T C_p T^T is not positive definite") from e
    return T, S


# --------------------------------------------------------------------------
# Run wrapper
# --------------------------------------------------------------------------
class OracleRun:
    """State and accumulators of one oracle integration.

    ``M`` is either a dense ndarray [N, N] or an object with ``n``,
    ``row_ptr``, ``col``, ``val`` (CSR).  Values are used in float64.
    ``pairs`` is int32 [A, 2]; diagonal entries are pairs (i, i).  With
    ``pp=True`` every pair is accumulated twice: first as <q_i q_j>, then (in
    a second block of the same order) as the momentum form <p_i p_j> of Eq. 7.
    With ``traces=True`` three trace estimators follow (Sec. I): sum_i
    <q_i^2>, <q^T M q> and, with pp, sum_i <p_i^2>.
    """

    def __init__(self, M, A_p, C_p, h, R, pairs, seed=0, stream=0, burn_in=0,
                 block_len=100, T=None, S=None, nthreads=0, pp=False, traces=False):
        if isinstance(M, np.ndarray):
            self.fmt = 0
            self.N = M.shape[0]
            self.dense = np.ascontiguousarray(M, dtype=np.float64)
            self.row_ptr = self.col = self.val = None
        else:
            self.fmt = 1
            self.N = int(M.n)
            self.dense = None
            self.row_ptr = np.ascontiguousarray(M.row_ptr, dtype=np.int64)
            self.col = np.ascontiguousarray(M.col, dtype=np.int32)
            self.val = np.ascontiguousarray(M.val, dtype=np.float64)
        if T is None or S is None:
            T, S = propagator(np.asarray(A_p), np.asarray(C_p), h)
        self.T = np.ascontiguousarray(T, dtype=np.float64)
        self.S = np.ascontiguousarray(S, dtype=np.float64)
        self.ns = self.T.shape[0] - 1
        if self.ns > 63:
            raise ValueError("oracle supports ns <= 63")
        self.h = float(h)
        self.R = int(R)
        self.seed = int(seed)
        self.stream = int(stream)
        self.burn_in = int(burn_in)
        self.L = int(block_len)
        self.nthreads = int(nthreads)
        N, R, ns = self.N, self.R, self.ns
        self.q = np.zeros((N, R))
        self.p = np.zeros((N, R))
        self.s = np.zeros((ns, N, R))
        base = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
        kinds = np.repeat(np.array([0, 1] if pp else [0], dtype=np.int32), len(base))
        allp = np.concatenate([base, base]) if pp else base
        if traces:
            tk = np.array([2, 3, 4] if pp else [2, 3], dtype=np.int32)
            kinds = np.concatenate([kinds, tk])
            allp = np.concatenate([allp, np.zeros((len(tk), 2), dtype=np.int32)])
        self.pairs = np.ascontiguousarray(allp, dtype=np.int32)
        self.kinds = np.ascontiguousarray(kinds, dtype=np.int32)
        A = len(self.pairs)
        self.blk = np.zeros(A)
        self.s1 = np.zeros(A)
        self.s2 = np.zeros(A)
        self.nblocks = np.zeros(1, dtype=np.int64)
        self.step = 0

    def set_state(self, q=None, p=None, s=None):
        if q is not None:
            self.q[...] = q
        if p is not None:
            self.p[...] = p
        if s is not None:
            self.s[...] = s

    def run(self, nsteps: int):
        rc = lib().orc_run(self.N, self.fmt, _ptr(self.dense), _ptr(self.row_ptr), _ptr(self.col),
                           _ptr(self.val), self.ns, _ptr(self.T), _ptr(self.S), self.h, self.R,
                           self.seed, self.stream, self.step, int(nsteps), self.burn_in, self.L,
                           _ptr(self.q), _ptr(self.p), _ptr(self.s), len(self.pairs),
                           _ptr(self.pairs), _ptr(self.kinds), _ptr(self.blk), _ptr(self.s1), _ptr(self.s2),
                           _ptr(self.nblocks), self.nthreads)
        if rc != 0:
            raise MemoryError("oracle allocation failed")
        self.step += int(nsteps)
        return self

    @property
    def n_acc(self) -> int:
        return max(0, self.step - self.burn_in)

    def estimates(self):
        """Mean <q_i q_j> over all accumulated steps and replicas, and the
        standard error from the complete blocks (inf with fewer than 2)."""
        return estimates(self.s1, self.s2, self.blk, int(self.nblocks[0]), self.R, self.n_acc, self.L)


def estimates(s1, s2, blk, nblocks, R, n_acc, L):
    """mean = (s1 + blk) / (R n_acc); block means b = blocksum / (R L);
    stderr = sqrt(sum (b - mean_b)^2 / (B (B - 1)))."""
    s1 = np.asarray(s1, dtype=np.float64)
    s2 = np.asarray(s2, dtype=np.float64)
    blk = np.asarray(blk, dtype=np.float64)
    mean = (s1 + blk) / (R * n_acc) if n_acc > 0 else np.full_like(s1, np.nan)
    B = int(nblocks)
    if B < 2:
        return mean, np.full_like(s1, np.inf)
    scale = 1.0 / (R * L)
    sb = s1 * scale
    sbb = s2 * scale * scale
    var = (sbb - sb * sb / B) / (B - 1)
    return mean, np.sqrt(np.maximum(var, 0.0) / B)


def max_threads() -> int:
    return lib().orc_max_threads()
