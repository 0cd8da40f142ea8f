"""GPU parity of the persistent small-system path (one workgroup runs many
steps per launch) against the FP64 oracle, and the white-noise closed form
on the dense N = 64, R = 1, 2e5-step configuration."""
import numpy as np
import pytest

import fth_inputs as fi
import oracle
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu


def normwise(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


def random_gle(ns, seed):
    rng = np.random.default_rng(seed)
    d = ns + 1
    K = rng.normal(size=(d, d))
    return (K - K.T) + np.diag(rng.uniform(0.3, 2.0, d)), 0.9 * np.eye(d)


CASES = [
    # id, n, R, precision, gle
    ("haar64-white-R1-fp64", 64, 1, fth.FTH_FP64, "white"),
    ("haar100-ns4-R16-fp64", 100, 16, fth.FTH_FP64, "invsqrt"),
    ("haar200-ns4-R8-fp32-mglobal", 200, 8, fth.FTH_FP32, "invsqrt"),
    ("haar33-ns3-R2-fp32", 33, 2, fth.FTH_FP32, "rand3"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_small_trajectory_parity(case):
    cid, n, R, prec, gname = case
    print(f"[small] {cid}", flush=True)
    M, lam = fi.haar_spd(n, 1001 + n, 1.0, 100.0)
    h = fi.dt_rule(lam.max())
    if gname == "white":
        g = fi.white_noise_gle(1.0, 1.0)
        A, C = g.A_p, g.C_p
    elif gname == "invsqrt":
        g = fi.load_gle("invsqrt_ns4")
        A, C = g.A_p * 3.0, g.C_p * 3.0  # alpha = gamma = 3: window moves to lambda in [0.9, 109]
    else:
        A, C = random_gle(int(gname[4:]), 3)
    pairs = np.concatenate([fi.row_pairs(n, 0), fi.random_pairs(n, 9, 4)])
    sol = fth.Solver(M, A, C, h, pairs=pairs, replicas=R, precision=prec, seed=1, stream_id=9, burn_in=4,
                     block_len=11, acc_diag=True)
    assert "small_dense_kernel" in sol.kernel_name
    orc = oracle.OracleRun(M, A, C, h, R, np.concatenate([pairs, fi.diag_pairs(n)]), seed=1, stream=9,
                           burn_in=4, block_len=11)
    tol = 1e-10 if prec == fth.FTH_FP64 else 1e-4
    done = 0
    for target in (1, 10, 100, 1000, 5000):
        sol.run(target - done)
        orc.run(target - done)
        done = target
        q, p, s = sol.state()
        blk, s1, s2, nb, step = sol.accumulators()
        errs = {"q": normwise(q, orc.q), "p": normwise(p, orc.p), "acc": normwise(s1 + blk, orc.s1 + orc.blk)}
        if orc.ns:
            errs["s"] = normwise(s, orc.s)
        if nb:
            errs["s2"] = normwise(s2, orc.s2)
        print(f"  step {done}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v <= tol, (cid, done, k, v)
    sol.close()


def test_white_noise_n64_two_hundred_thousand_steps():
    """Dense SPD N = 64, Haar eigenvectors, eigenvalues log-uniform in
    [1, 100], white-noise Langevin (gamma = 1, kT = 1), h = 0.1 /
    sqrt(lambda_max), R = 1, 2e5 steps: diagonal and row 0 of kT M^-1 (exactly
    kT (M - h^2 M^2 / 4)^-1 for the integrated step) within 4.5 standard
    errors, in FP64."""
    n = 64
    M, lam = fi.haar_spd(n, 1001, 1.0, 100.0)
    h = fi.dt_rule(lam.max())
    pairs = fi.row_pairs(n, 0)
    sol = fth.Solver(M, [[1.0]], [[1.0]], h, pairs=pairs, replicas=1, precision=fth.FTH_FP64, seed=1,
                     burn_in=5000, block_len=3900, acc_diag=True)
    sol.run(200000)
    est, se, nsamp = sol.read()
    print(f"[n64] {sol.last_run_ms:.1f} ms for 2e5 steps", flush=True)
    allp = np.concatenate([pairs, fi.diag_pairs(n)])
    exact_h = np.linalg.inv(M - h * h * M @ M / 4)
    ref = exact_h[allp[:, 0], allp[:, 1]]
    z = (est - ref) / se
    print(f"[n64] max|z| {np.max(np.abs(z)):.2f}; max |M^-1 - exact_h| / se "
          f"{np.max(np.abs(np.linalg.inv(M)[allp[:, 0], allp[:, 1]] - ref) / se):.3f}", flush=True)
    assert np.max(np.abs(z)) < 4.5
