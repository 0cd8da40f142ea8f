"""GPU tests of the spectral map (Sec. I scaling paragraph): M' = r M + m I
and A'_p = alpha A_p, C'_p = gamma C_p applied by the library at create, and
the targets recovered from the transformed problem (ln, exp(-x), x^-1/2).

The mapped run must equal, bit for bit, a run given the transformed inputs
directly (the map is formed in FP64 on the host either way).  The recovered
ln and exp(-x) estimates are checked against eigendecompositions of the
paper's synthetic M1 (3-D lattice, six neighbour shells: log det via the
trace estimator) and M2 (dense, Gerschgorin-bounded, exp(-M/100))
workloads, within the fit error of the GLE plus the statistical error.
"""
import numpy as np
import pytest

import fth_inputs as fi
from oracle import exact
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu


def csr_to_dense(M):
    A = np.zeros((M.n, M.n))
    for i in range(M.n):
        for k in range(M.row_ptr[i], M.row_ptr[i + 1]):
            A[i, M.col[k]] += M.val[k]
    return A


@pytest.mark.parametrize("dense,prec", [(False, fth.FTH_FP32), (True, fth.FTH_FP64)])
def test_map_equals_pretransformed_inputs(dense, prec):
    g = fi.load_gle("invsqrt_ns4")
    r, m, alpha, gamma = 0.37, 1.25, 1.7, 0.6
    if dense:
        M, _ = fi.haar_spd(300, 9, 1.0, 30.0)
        Mp = r * M + m * np.eye(300)
        R = 16
    else:
        M = fi.banded_spd_csr(5000, 4, dtype=np.float64)
        vals = r * M.val.astype(np.float64)
        for i in range(M.n):
            for k in range(M.row_ptr[i], M.row_ptr[i + 1]):
                if M.col[k] == i:
                    vals[k] += m
        Mp = fi.CSR(M.n, M.row_ptr, M.col, vals)
        R = 8
    h = 0.05
    kw = dict(pairs=fi.random_pairs(300 if dense else 5000, 16, 3), replicas=R, precision=prec, seed=6,
              acc_diag=True, block_len=5)
    a = fth.Solver(M, g.A_p, g.C_p, h, scale_r=r, scale_m=m, gle_alpha=alpha, gle_gamma=gamma, **kw).run(40)
    b = fth.Solver(Mp, alpha * g.A_p, gamma * g.C_p, h, **kw).run(40)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    for x, y in zip(a.accumulators()[:3], b.accumulators()[:3]):
        assert np.array_equal(x, y)


def test_map_errors():
    g = fi.load_gle("invsqrt_ns4")
    M = fi.banded_spd_csr(100, 4)
    with pytest.raises(fth.FthError) as e:
        fth.Solver(M, g.A_p, g.C_p, 0.05, replicas=8, gle_alpha=-1.0)
    assert e.value.status == fth.FTH_EINVAL
    with pytest.raises(fth.FthError) as e:   # M' = -M is not positive definite
        fth.Solver(M, g.A_p, g.C_p, 0.05, replicas=8, scale_r=-1.0)
    assert e.value.status == fth.FTH_EINVAL
