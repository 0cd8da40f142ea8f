"""Host-side checks of the C-ABI library that need no GPU: it loads, it
exports every function include/fth.h declares, its FP64 propagator matches
the oracle's, and argument validation rejects malformed inputs before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import fth_inputs as fi
import oracle
from paper_1402_2095_amd import fth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "fth.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fth_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = fth.lib()
    names = header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(fth.EXPORTS)
    assert "gfx950" in fth.fth_version()


@pytest.mark.parametrize("name,dt", [("invsqrt_ns4", 0.0287), ("fermi_b20_ns4", 0.05)])
def test_host_propagator_matches_oracle(name, dt):
    g = fi.load_gle(name)
    T, S = fth.fth_propagator(g.A_p, g.C_p, dt)
    To, So = oracle.propagator(g.A_p, g.C_p, dt)
    assert np.allclose(T, To, rtol=0, atol=1e-14)
    # S is compared through its backward error: Cholesky factors of an
    # ill-conditioned C_p - T C_p T^T may differ by cond * eps between
    # correct implementations, S S^T may not.
    assert np.allclose(np.triu(S, 1), 0.0)
    assert np.max(np.abs(S @ S.T - So @ So.T)) <= 1e-13 * np.max(np.abs(g.C_p))


def test_host_propagator_large_argument_and_white_noise():
    # a stiff drift exercises the scaling-and-squaring branch
    A = np.array([[3.0, 40.0, 0.0], [-40.0, 5.0, 2.0], [0.0, -2.0, 80.0]])
    C = 1.5 * np.eye(3)
    T, S = fth.fth_propagator(A, C, 0.2)
    To, So = oracle.propagator(A, C, 0.2)
    assert np.allclose(T, To, atol=1e-13)
    assert np.allclose(S, So, atol=1e-12)
    T, S = fth.fth_propagator([[0.7]], [[2.0]], 0.1)
    assert T[0, 0] == pytest.approx(np.exp(-0.07), rel=1e-15)
    assert S[0, 0] == pytest.approx(np.sqrt(2.0 * (1 - np.exp(-0.14))), rel=1e-14)


def test_host_propagator_rejects_invalid_gles():
    with pytest.raises(fth.FthError) as e:
        fth.fth_propagator([[1.0]], [[-1.0]], 0.1)
    assert e.value.status == fth.FTH_EINVAL
    with pytest.raises(fth.FthError):
        fth.fth_propagator(np.array([[1.0, 10.0], [0.0, 1.0]]), np.eye(2), 0.1)
    with pytest.raises(fth.FthError):
        fth.fth_propagator([[1.0]], [[1.0]], -0.1)
    with pytest.raises(fth.FthError):
        fth.fth_propagator([[1.0]], [[1.0]], float("nan"))


def _create_status(M, A, C, dt, pairs=None, **opt):
    try:
        fth.fth_create(M, A, C, dt, pairs, fth.fth_default_options(**opt))
    except fth.FthError as e:
        return e.status, str(e)
    return fth.FTH_OK, ""


def test_validation_before_device():
    csr = fi.banded_spd_csr(50, 1)
    A, C = [[1.0]], [[1.0]]
    bad = fi.CSR(csr.n, csr.row_ptr.copy(), csr.col.copy(), csr.val.copy())
    bad.val[1] += 0.5  # breaks value symmetry
    st, msg = _create_status(bad, A, C, 0.05)
    assert st == fth.FTH_EINVAL and "symmetric" in msg
    bad = fi.CSR(csr.n, csr.row_ptr.copy(), csr.col.copy(), csr.val.copy())
    bad.col[0], bad.col[1] = bad.col[1], bad.col[0]
    st, msg = _create_status(bad, A, C, 0.05)
    assert st == fth.FTH_EINVAL
    st, msg = _create_status(csr, A, C, 0.05, pairs=np.array([[0, 50]]))
    assert st == fth.FTH_EINVAL and "pair" in msg
    st, msg = _create_status(csr, A, [[-1.0]], 0.05)
    assert st == fth.FTH_EINVAL
    st, msg = _create_status(csr, A, C, 0.05, block_len=0)
    assert st == fth.FTH_EINVAL
    dense = csr.to_dense()
    dense[0, 1] += 1.0
    st, msg = _create_status(dense, A, C, 0.05)
    assert st == fth.FTH_EINVAL and "symmetric" in msg
    st, msg = _create_status(csr, A, C, 0.05, precision=fth.FTH_FP32_BF16X3)
    assert st == fth.FTH_EUNSUPPORTED


def test_footprint_accounting():
    csr = fi.laplacian3d_csr(8)
    b = fth.fth_footprint_bytes(csr, 4, 8, 10, True, fth.FTH_FP32)
    n, nnz = csr.n, csr.nnz
    # q and (p, s) are both double-buffered: 2 + 2 (ns + 1) vectors of R reals per row
    expect = (n + 1) * 8 + nnz * 8 + n * 8 * 4 * 12 + (10 + n) * 24 + 10 * 8 + 2 * 25 * 4 + 64
    assert b == expect
    # the paper's count: M + (3 + S) N + 2 A reals; state bytes dominate and scale with R
    assert fth.fth_footprint_bytes(csr, 4, 16, 10, True, fth.FTH_FP32) - b == n * 8 * 4 * 12


def test_spectral_map_sends_the_spectrum_onto_the_window():
    """Sec. I scaling: M' = r M + m I with r e_min + m = w_min and
    r e_max + m = w_max (the affine map is fixed by its two end points)."""
    for e_lo, e_hi, w_lo, w_hi in ((85.0, 180.0, 1.2, 600.0), (-3.0, 3.0, 0.1, 6.1), (0.4, 199.6, 0.1, 12.1)):
        r, m = fth.fth_spectral_map(e_lo, e_hi, w_lo, w_hi)
        assert abs(r * e_lo + m - w_lo) < 1e-12 * max(1, abs(w_lo)) * 100
        assert abs(r * e_hi + m - w_hi) < 1e-12 * max(1, abs(w_hi)) * 100
    with pytest.raises(fth.FthError):
        fth.fth_spectral_map(1.0, 1.0, 0.1, 2.0)


def test_gershgorin_interval():
    M = fi.banded_spd_csr(400, 3, dtype=np.float64)
    lo, hi = fth.fth_gershgorin(M)
    A = np.zeros((400, 400))
    for i in range(400):
        for k in range(M.row_ptr[i], M.row_ptr[i + 1]):
            A[i, M.col[k]] = M.val[k]
    off = np.sum(np.abs(A), axis=1) - np.abs(np.diag(A))
    assert lo == pytest.approx(np.min(np.diag(A) - off), rel=1e-12)
    assert hi == pytest.approx(np.max(np.diag(A) + off), rel=1e-12)
    w = np.linalg.eigvalsh(A)
    assert lo <= w.min() and w.max() <= hi
    D = fi.m2_gerschgorin(50, 2)
    lo2, hi2 = fth.fth_gershgorin(D.astype(np.float64))
    w2 = np.linalg.eigvalsh(D)
    assert lo2 <= w2.min() and w2.max() <= hi2


def test_unscale_against_matrix_functions():
    """The undo identities, checked on eigendecompositions: ln(M) =
    ln(r M) - ln(r) I, M^-1/2 = sqrt(r) (r M)^-1/2, exp(-r M) = e^m exp(-(r M + m I));
    with (alpha, gamma) the q-response is (gamma/alpha^2) g(M'/alpha^2)."""
    from oracle.exact import matrix_function
    M, _ = fi.haar_spd(7, 5, 2.0, 40.0)
    n = 7
    iu = np.triu_indices(n)
    w = (iu[0] == iu[1]).astype(float)
    for target, r, m, f in ((fth.FTH_TARGET_LN, 3.0, 0.0, np.log), (fth.FTH_TARGET_INVSQRT, 0.25, 0.0, lambda x: x ** -0.5),
                            (fth.FTH_TARGET_EXPNEG, 0.05, 1.5, lambda x: np.exp(-x))):
        for alpha, gamma in ((1.0, 1.0), (2.0, 0.5)):
            Mp = r * M + m * np.eye(n)
            # what the transformed run estimates: (gamma / alpha^2) f(M' / alpha^2)
            run = (gamma / alpha ** 2) * matrix_function(Mp / alpha ** 2, f)[iu]
            est, se = fth.fth_unscale(target, r, m, alpha, gamma, w, run, np.ones(len(w)))
            rr = r / alpha ** 2
            if target == fth.FTH_TARGET_EXPNEG:   # recovers exp(-r' M), r' = r / alpha^2
                want = matrix_function(rr * M, lambda x: np.exp(-x))[iu]
            else:
                want = matrix_function(M, f)[iu]
            assert np.allclose(est, want, rtol=1e-10, atol=1e-12), (target, alpha, gamma)
            assert np.all(se > 0)
    with pytest.raises(fth.FthError):   # ln needs m = 0
        fth.fth_unscale(fth.FTH_TARGET_LN, 2.0, 1.0, 1.0, 1.0, w, np.ones(len(w)))
