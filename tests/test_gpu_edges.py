"""Degenerate and edge cases of the step path, through the C ABI:

* a one-row system (N = 1), sparse and dense, one and several replicas,
  against the oracle step by step;
* a solve that keeps no estimates at all (no pairs, no diagonal);
* zero steps leave state and accumulators untouched;
* a pair and its mirror give bit-identical estimates (the product is
  commutative and both are summed in the same order), and a pair (i, i)
  agrees with the fused diagonal entry i;
* replica counts the library does not serve are rejected, not rounded.
"""
import numpy as np
import pytest

import fth_inputs as fi
import oracle
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu


def normwise(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


def one_row_csr(v=2.0):
    return fi.CSR(1, np.array([0, 1], dtype=np.int64), np.array([0], dtype=np.int32), np.array([v]))


@pytest.mark.parametrize("dense", [False, True], ids=["csr", "dense"])
@pytest.mark.parametrize("R,prec", [(1, fth.FTH_FP64), (8, fth.FTH_FP32), (32, fth.FTH_FP64)])
def test_one_row_system_matches_oracle(dense, R, prec):
    g = fi.load_gle("invsqrt_ns4")
    M = np.array([[2.0]]) if dense else one_row_csr(2.0)
    h = fi.dt_rule(2.0)
    sol = fth.Solver(M, g.A_p, g.C_p, h, replicas=R, precision=prec, seed=77, stream_id=2, burn_in=3,
                     block_len=5, acc_diag=True, steps_per_graph=8)
    orc = oracle.OracleRun(M if dense else M, g.A_p, g.C_p, h, R, fi.diag_pairs(1), seed=77, stream=2, burn_in=3,
                           block_len=5)
    tol = 1e-10 if prec == fth.FTH_FP64 else 1e-4
    done = 0
    for target in (1, 9, 100, 700):
        sol.run(target - done)
        orc.run(target - done)
        done = target
        q, p, s = sol.state()
        blk, s1, s2, nb, step = sol.accumulators()
        errs = {"q": normwise(q, orc.q), "p": normwise(p, orc.p), "s": normwise(s, orc.s),
                "acc": normwise(s1 + blk, orc.s1 + orc.blk)}
        print(f"[edge] N=1 {'dense' if dense else 'csr'} R={R} step {done}: "
              + " ".join(f"{k}={v:.1e}" for k, v in errs.items()) + f" ({sol.kernel_name})", flush=True)
        assert step == done
        for k, v in errs.items():
            assert v <= tol, (k, v)
    sol.close()


def test_no_estimates_kept():
    g = fi.load_gle("invsqrt_ns4")
    M = fi.banded_spd_csr(1000, 12)
    sol = fth.Solver(M, g.A_p, g.C_p, fi.dt_rule(fi.gershgorin_max(M)), replicas=8, seed=1, acc_diag=False)
    assert fth.fth_num_outputs(sol.ctx) == 0
    sol.run(25)
    est, se, nsamp = sol.read()
    assert est.size == 0 and se.size == 0 and nsamp == 25
    q, _, _ = sol.state()
    assert np.all(np.isfinite(q)) and np.any(q != 0)
    sol.close()


def test_zero_steps_is_a_no_op():
    g = fi.load_gle("invsqrt_ns4")
    M = fi.laplacian3d_csr(6, 0.1)
    sol = fth.Solver(M, g.A_p, g.C_p, fi.dt_rule(fi.laplacian3d_lambda_max(6, 0.1)), replicas=8, seed=3,
                     acc_diag=True, pairs=fi.random_pairs(M.n, 8, 2))
    sol.run(13)
    before = sol.state(), sol.accumulators()
    sol.run(0)
    after = sol.state(), sol.accumulators()
    for x, y in zip(before[0], after[0]):
        assert np.array_equal(x, y)
    for x, y in zip(before[1], after[1]):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    sol.close()


@pytest.mark.parametrize("prec", [fth.FTH_FP64, fth.FTH_FP32], ids=["fp64", "fp32"])
def test_mirrored_and_self_pairs(prec):
    g = fi.load_gle("invsqrt_ns4")
    M = fi.banded_spd_csr(3001, 21)
    pairs = np.array([[3, 7], [7, 3], [5, 5], [2999, 0], [0, 2999]], dtype=np.int32)
    sol = fth.Solver(M, g.A_p, g.C_p, fi.dt_rule(fi.gershgorin_max(M)), pairs=pairs, replicas=16, precision=prec,
                     seed=8, acc_diag=True, block_len=10)
    sol.run(200)
    est, se, _ = sol.read()
    assert est[0] == est[1] and se[0] == se[1]
    assert est[3] == est[4] and se[3] == se[4]
    diag5 = est[len(pairs) + 5]
    assert abs(est[2] - diag5) <= 1e-12 * abs(diag5)
    sol.close()


@pytest.mark.parametrize("R", [3, 6, 1024])
def test_unsupported_replica_counts_rejected(R):
    g = fi.load_gle("invsqrt_ns4")
    M = fi.banded_spd_csr(500, 1)
    sol = fth.Solver(M, g.A_p, g.C_p, 0.05, seed=1)
    with pytest.raises(fth.FthError) as e:
        sol.run(1, replicas=R)
    assert e.value.status == fth.FTH_EUNSUPPORTED
    sol.run(1, replicas=4)   # the context is still usable
    sol.close()
