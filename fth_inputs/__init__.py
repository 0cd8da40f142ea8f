"""Seeded synthetic inputs for the f-thermostat (FTH) hot path.

This module is shared by the FP64 CPU oracle and the HIP library's tests and
benchmark.  It holds only input construction: matrices, index pairs, time
steps, the serving-mix arrival schedule and the reader of the GLE parameter
files.  None of the thermostat arithmetic (propagators, noise, integration,
estimators) lives here.

Matrix shapes follow the workloads the paper uses and the configurations this
project measures:

* dense SPD with a prescribed spectrum (Haar-random eigenvectors),
* the 3-D periodic 7-point Laplacian plus a shift (a cubic-lattice
  tight-binding-like sparse matrix, cf. the appendix's M1 family),
* a random banded SPD matrix (7 nonzeros per row),
* a dense Wishart-like matrix G G^T / N + 0.1 I,
* the appendix's M1 (cubic lattice, random hopping up to the 6th neighbour
  shell) and M2 (dense, Gerschgorin-bounded spectrum) generators.

CSR matrices are returned as ``(row_ptr int64[N+1], col int32[nnz],
val float32|float64[nnz])`` with sorted, unique column indices per row.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

GLE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gle")


# --------------------------------------------------------------------------
# CSR helpers
# --------------------------------------------------------------------------
@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float32 or float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n), dtype=np.float64)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        np.add.at(d, (rows, self.col.astype(np.int64)), self.val.astype(np.float64))
        return d


def _coo_to_csr(n, rows, cols, vals, dtype) -> CSR:
    """Sort (row, col), merge duplicates by summation, return CSR."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if len(vals) else vals
    r = uniq // n
    c = uniq % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return CSR(n, row_ptr, c.astype(np.int32), summed.astype(dtype))


# --------------------------------------------------------------------------
# Dense SPD with prescribed spectrum (Haar eigenvectors)
# --------------------------------------------------------------------------
def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    sign of diag(R) folded into Q (Mezzadri's correction)."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def haar_spd(n: int, seed: int, lam_lo: float = 1.0, lam_hi: float = 100.0):
    """M = Q diag(lam) Q^T with lam log-uniform in [lam_lo, lam_hi].

    Returns (M float64 [n,n] symmetric, lam float64 [n])."""
    rng = np.random.default_rng(seed)
    q = haar_orthogonal(n, rng)
    lam = 10.0 ** rng.uniform(math.log10(lam_lo), math.log10(lam_hi), size=n)
    m = (q * lam[None, :]) @ q.T
    m = 0.5 * (m + m.T)
    return m, lam


# --------------------------------------------------------------------------
# 3-D periodic Laplacian + shift
# --------------------------------------------------------------------------
def lattice_index(x, y, z, n):
    """Site (x, y, z) of an n^3 lattice -> row index, x slowest (the
    appendix's i -> (i / n^2, (i % n^2) / n, i % n) convention)."""
    return (x * n + y) * n + z


def laplacian3d_csr(n: int, sigma: float = 0.1, dtype=np.float32) -> CSR:
    """M = -Delta_h + sigma I on an n^3 periodic grid, unit spacing.

    Diagonal 6 + sigma; the six nearest neighbours carry -1 (merged when the
    grid is so small that two neighbours coincide).  Spectrum is
    sigma + sum_d (2 - 2 cos(2 pi k_d / n)), so it lies in [sigma, sigma + 12]."""
    N = n ** 3
    idx = np.arange(N, dtype=np.int64)
    x, rem = np.divmod(idx, n * n)
    y, z = np.divmod(rem, n)
    rows = [idx]
    cols = [idx]
    vals = [np.full(N, 6.0 + sigma)]
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        j = lattice_index((x + dx) % n, (y + dy) % n, (z + dz) % n, n)
        rows.append(idx)
        cols.append(j)
        vals.append(np.full(N, -1.0))
    return _coo_to_csr(N, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), dtype)


def laplacian3d_lambda_max(n: int, sigma: float) -> float:
    """Largest eigenvalue of laplacian3d_csr(n, sigma) (closed form)."""
    k = np.arange(n)
    mx = np.max(2.0 - 2.0 * np.cos(2.0 * np.pi * k / n))
    return sigma + 3.0 * float(mx)


def insulator3d_csr(n: int, delta: float = 1.2, hop: float = 0.9797958971132712, shift: float = 6.1,
                    dtype=np.float32) -> CSR:
    """A gapped stand-in for a tight-binding insulator (the setting of the
    Fermi-function example, Sec. II): an n^3 periodic cubic lattice (n even),
    on-site shift + delta on sites with x + y + z even and shift - delta on
    the others, hopping -hop to the six nearest neighbours.  Its spectrum is
    shift -/+ sqrt(delta^2 + hop^2 gamma_k^2), gamma_k = sum_d 2 cos(2 pi k_d / n):
    a lower and an upper band of N/2 states each, separated by a gap of
    2 delta around shift (exactly, when 4 divides n).  The defaults give
    [0.1, 4.9] and [7.3, 12.1]."""
    if n % 2:
        raise ValueError("the two sublattices need an even n")
    N = n ** 3
    idx = np.arange(N, dtype=np.int64)
    x, rem = np.divmod(idx, n * n)
    y, z = np.divmod(rem, n)
    par = (x + y + z) % 2
    rows, cols, vals = [idx], [idx], [np.where(par == 0, shift + delta, shift - delta)]
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        rows.append(idx)
        cols.append(lattice_index((x + dx) % n, (y + dy) % n, (z + dz) % n, n))
        vals.append(np.full(N, -hop))
    return _coo_to_csr(N, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), dtype)


# --------------------------------------------------------------------------
# Random banded SPD (7 nonzeros per row)
# --------------------------------------------------------------------------
def banded_spd_csr(n: int, seed: int, half_bw: int = 3, dtype=np.float32) -> CSR:
    """Symmetric banded matrix with offsets -half_bw..half_bw, open ends.

    Off-diagonals are U[-1, 0], drawn once per (i, i+k); the diagonal is
    |sum of the row's off-diagonals| + U[0.05, 1], which makes the matrix
    strictly diagonally dominant (lambda_min >= 0.05)."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    offd = {}
    rowsum = np.zeros(n, dtype=np.float64)
    for k in range(1, half_bw + 1):
        m = n - k
        if m <= 0:
            continue
        v = rng.uniform(-1.0, 0.0, size=m).astype(dtype).astype(np.float64)
        i = np.arange(m, dtype=np.int64)
        offd[k] = v
        rowsum[:m] += np.abs(v)
        rowsum[k:] += np.abs(v)
        rows += [i, i + k]
        cols += [i + k, i]
        vals += [v, v]
    diag = rowsum + rng.uniform(0.05, 1.0, size=n)
    idx = np.arange(n, dtype=np.int64)
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    return _coo_to_csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), dtype)


def gershgorin_max(csr: CSR) -> float:
    """Upper bound of the spectrum from Gerschgorin discs."""
    rows = np.repeat(np.arange(csr.n), np.diff(csr.row_ptr))
    v = csr.val.astype(np.float64)
    diag = np.zeros(csr.n)
    rad = np.zeros(csr.n)
    on = rows == csr.col
    np.add.at(diag, rows[on], v[on])
    np.add.at(rad, rows[~on], np.abs(v[~on]))
    return float(np.max(diag + rad))


# --------------------------------------------------------------------------
# Dense Wishart-like SPD: G G^T / N + 0.1 I
# --------------------------------------------------------------------------
def dense_ggt(n: int, seed: int, shift: float = 0.1, dtype=np.float32) -> np.ndarray:
    """M = G G^T / n + shift*I, G standard normal (drawn in float32, product
    formed in float64, stored as ``dtype``).  Spectrum ~ [shift, shift + 4]
    (Marchenko-Pastur with aspect ratio 1)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n), dtype=np.float32).astype(np.float64)
    try:
        from scipy.linalg.blas import dsyrk
        m = dsyrk(1.0 / n, g, lower=1)
        m = np.tril(m) + np.tril(m, -1).T
    except Exception:  # pragma: no cover - scipy always present here
        m = (g @ g.T) / n
    del g
    m[np.diag_indices(n)] += shift
    return m.astype(dtype)


def power_lambda_max(m: np.ndarray, iters: int = 60, seed: int = 0) -> float:
    """Power-iteration estimate of the largest eigenvalue of a dense SPD
    matrix, inflated by 1 % so that a time step chosen from it is safe."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(m.shape[0])
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = m @ v
        lam = float(np.linalg.norm(w))
        v = w / lam
    return 1.01 * lam


# --------------------------------------------------------------------------
# The appendix's M1 and M2 families
# --------------------------------------------------------------------------
def m1_lattice_csr(n: int, seed: int, onsite: float = 100.0, shells: int = 6,
                   hop_max: float = 2.0, dtype=np.float64) -> CSR:
    """Cubic periodic lattice, n sites per direction, on-site ``onsite`` and
    symmetric random hopping U[0, hop_max] to every site within the first
    ``shells`` distinct neighbour distances (periodic minimum image)."""
    rng = np.random.default_rng(seed)
    N = n ** 3
    half = n // 2
    offs = []
    for dx in range(-half, half + 1):
        for dy in range(-half, half + 1):
            for dz in range(-half, half + 1):
                if (dx, dy, dz) == (0, 0, 0):
                    continue
                offs.append((dx, dy, dz))
    d2 = sorted({dx * dx + dy * dy + dz * dz for dx, dy, dz in offs})
    keep = set(d2[:shells])
    # one representative per +/- pair so that each bond is drawn once
    bonds = sorted({tuple(o) for o in offs if (o[0] * o[0] + o[1] * o[1] + o[2] * o[2]) in keep
                    and o > tuple(-c for c in o)})
    idx = np.arange(N, dtype=np.int64)
    x, rem = np.divmod(idx, n * n)
    y, z = np.divmod(rem, n)
    rows, cols, vals = [idx], [idx], [np.full(N, onsite)]
    for dx, dy, dz in bonds:
        j = lattice_index((x + dx) % n, (y + dy) % n, (z + dz) % n, n)
        v = rng.uniform(0.0, hop_max, size=N)
        rows += [idx, j]
        cols += [j, idx]
        vals += [v, v]
    return _coo_to_csr(N, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), dtype)


def m2_gerschgorin(m: int, seed: int, a: float = -300.0, b: float = 300.0) -> np.ndarray:
    """Dense symmetric matrix whose Gerschgorin discs lie inside (a, b).

    Diagonal U[a + (b-a)/4, b - (b-a)/4]; lower-triangle element (i, j) is
    U[-r/(i-j), r/(i-j)] with r the smallest remaining disc margin of rows i
    and j, and both rows' radii grow by its magnitude."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(a + (b - a) / 4, b - (b - a) / 4, size=m)
    rad = np.zeros(m)
    out = np.diag(d).astype(np.float64)
    for i in range(m):
        for j in range(i):
            r = min(d[i] - rad[i] - a, b - d[i] - rad[i], d[j] - rad[j] - a, b - d[j] - rad[j])
            r = max(r, 0.0)
            x = rng.uniform(-r / (i - j), r / (i - j)) if r > 0 else 0.0
            out[i, j] = out[j, i] = x
            rad[i] += abs(x)
            rad[j] += abs(x)
    return out


# --------------------------------------------------------------------------
# Pairs, time steps
# --------------------------------------------------------------------------
def random_pairs(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` uniformly random off-diagonal pairs (i != j), int32 [count, 2]."""
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n, size=count)
    j = rng.integers(0, n - 1, size=count)
    j = j + (j >= i)
    return np.stack([i, j], axis=1).astype(np.int32)


def row_pairs(n: int, row: int = 0) -> np.ndarray:
    """All (row, j), j != row."""
    j = np.array([k for k in range(n) if k != row], dtype=np.int32)
    return np.stack([np.full_like(j, row), j], axis=1).astype(np.int32)


def diag_pairs(n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.int32)
    return np.stack([i, i], axis=1)


def dt_rule(lambda_max: float, c: float = 0.1) -> float:
    """Time step h = c / sqrt(lambda_max)."""
    return c / math.sqrt(lambda_max)


# --------------------------------------------------------------------------
# GLE parameter files
# --------------------------------------------------------------------------
@dataclass
class GLE:
    ns: int
    A_p: np.ndarray  # (ns+1, ns+1) float64
    C_p: np.ndarray  # (ns+1, ns+1) float64
    meta: dict = field(default_factory=dict)


def white_noise_gle(gamma: float = 1.0, kT: float = 1.0) -> GLE:
    """Markovian Langevin thermostat: no extra momenta."""
    return GLE(0, np.array([[gamma]]), np.array([[kT]]), {"name": "white", "gamma": gamma, "kT": kT})


def load_gle(name_or_path: str) -> GLE:
    path = name_or_path
    if not os.path.exists(path):
        path = os.path.join(GLE_DIR, name_or_path if name_or_path.endswith(".json") else name_or_path + ".json")
    with open(path) as f:
        d = json.load(f)
    ns = int(d["ns"])
    A = np.array(d["A_p"], dtype=np.float64).reshape(ns + 1, ns + 1)
    C = np.array(d["C_p"], dtype=np.float64).reshape(ns + 1, ns + 1)
    return GLE(ns, A, C, d)


# --------------------------------------------------------------------------
# Serving mix
# --------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival: float      # seconds after start
    kind: str           # "laplacian" | "banded" | "dense"
    n: int
    target: str         # "fermi" | "invsqrt"
    seed: int


def serving_mix(count: int, rate: float, seed: int, n_sparse=(10_000, 2_000_000),
                n_dense=(512, 8192), frac_dense: float = 0.3) -> list:
    """Poisson arrivals at ``rate`` per second; 70 % sparse (Laplacian and
    banded, 50:50, N uniform in n_sparse), 30 % dense (N uniform in n_dense);
    targets Fermi / x^-1/2 50:50."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < frac_dense:
            kind = "dense"
            n = int(rng.integers(n_dense[0], n_dense[1] + 1))
        else:
            kind = "laplacian" if rng.uniform() < 0.5 else "banded"
            n = int(rng.integers(n_sparse[0], n_sparse[1] + 1))
            if kind == "laplacian":
                side = max(3, int(round(n ** (1.0 / 3.0))))
                n = side ** 3
        target = "fermi" if rng.uniform() < 0.5 else "invsqrt"
        out.append(Request(k, t, kind, n, target, int(rng.integers(0, 2 ** 31))))
    return out
