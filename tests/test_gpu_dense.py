"""GPU parity of the dense hot path (force as a GEMM on the matrix cores).

FP64 form: trajectories agree with the FP64 oracle to <= 1e-10 normwise over
1000 steps.  Split-BF16x3 form: the force itself is compared with an FP64
GEMM (its error is reported and bounded separately from the statistical
error), and trajectories with the oracle at the FP32 tolerance.
"""
import numpy as np
import pytest

import fth_inputs as fi
import oracle
from oracle import exact
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu


def normwise(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


def dense_case(n, seed=4004):
    M = fi.dense_ggt(n, seed)
    lam_max = fi.power_lambda_max(M.astype(np.float64))
    return M, fi.dt_rule(lam_max)


@pytest.mark.parametrize("prec", [fth.FTH_FP64, fth.FTH_FP32_BF16X3], ids=["fp64", "bf16x3"])
# 2195 pads to 2560: eight K slices of 320 (whole 64-wide k-steps); 9000 pads to 9216, where the
# split form takes four K slices of 2304 (72 row blocks x 4 = 288 workgroups, one round)
@pytest.mark.parametrize("n,R", [(300, 16), (1000, 32), (520, 128), (2195, 64), (9000, 16)])
def test_force_against_fp64_gemm(prec, n, R):
    M, h = dense_case(n)
    g = fi.load_gle("invsqrt_ns4")
    sol = fth.Solver(M, g.A_p, g.C_p, h, replicas=R, precision=prec)
    rng = np.random.default_rng(3)
    q = rng.normal(size=(n, R))
    if prec == fth.FTH_FP32_BF16X3:
        q = q.astype(np.float32).astype(np.float64)
    F = sol.force(q)
    ref = -(M.astype(np.float64) @ q)
    err = normwise(F, ref)
    rel_rows = np.max(np.abs(F - ref), axis=0) / np.max(np.abs(ref), axis=0)
    print(f"[force] n={n} R={R} prec={prec}: normwise {err:.2e}, worst column {rel_rows.max():.2e} "
          f"({sol.kernel_name})", flush=True)
    assert err <= (1e-13 if prec == fth.FTH_FP64 else 3e-5)
    if n == 9000:
        assert ("ksplit=4" if prec == fth.FTH_FP32_BF16X3 else "ksplit=8") in sol.kernel_name
    sol.close()


@pytest.mark.parametrize("prec", [fth.FTH_FP64, fth.FTH_FP32_BF16X3], ids=["fp64", "bf16x3"])
def test_dense_trajectory_parity(prec):
    n, R = 700, 32
    M, h = dense_case(n, 77)
    M64 = M.astype(np.float64)
    g = fi.load_gle("invsqrt_ns4")
    pairs = fi.random_pairs(n, 40, 9)
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=R, precision=prec, seed=21, stream_id=5,
                     burn_in=3, block_len=9, acc_diag=True, steps_per_graph=16)
    orc = oracle.OracleRun(M64, g.A_p, g.C_p, h, R, np.concatenate([pairs, fi.diag_pairs(n)]), seed=21, stream=5,
                           burn_in=3, block_len=9)
    tol = 1e-10 if prec == fth.FTH_FP64 else 1e-4
    done = 0
    for target in (1, 10, 100, 1000):
        sol.run(target - done)
        orc.run(target - done)
        done = target
        q, p, s = sol.state()
        blk, s1, s2, nb, step = sol.accumulators()
        errs = {"q": normwise(q, orc.q), "p": normwise(p, orc.p), "s": normwise(s, orc.s),
                "acc": normwise(s1 + blk, orc.s1 + orc.blk)}
        print(f"  [{prec}] step {done}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v <= tol, (prec, done, k, v)
    sol.close()


@pytest.mark.parametrize("n,R,prec,steps", [(4200, 1, fth.FTH_FP64, (1, 10, 100, 1000)),
                                             (4200, 2, fth.FTH_FP32_BF16X3, (1, 10, 100, 1000)),
                                             (2100, 4, fth.FTH_FP32, (1, 10, 100, 1000)),
                                             (4500, 1, fth.FTH_FP32, (1, 10, 100, 1000)),
                                             (1100, 8, fth.FTH_FP64, (1, 10, 100, 1000)),
                                             (5003, 8, fth.FTH_FP32_BF16X3, (1, 10, 100)),
                                             (4097, 1, fth.FTH_FP64, (1, 10, 100)),
                                             (2049, 2, fth.FTH_FP32, (1, 10, 100))],
                         ids=["4200-R1-fp64", "4200-R2-split", "2100-R4-fp32", "4500-R1-fp32", "1100-R8-fp64",
                              "5003-R8-split", "4097-R1-fp64", "2049-R2-fp32"])
def test_few_replica_dense_against_oracle(n, R, prec, steps):
    """Dense systems beyond one workgroup with R <= 8 (the paper's own runs
    use a single trajectory): the force as R matrix-vector products in the
    state precision, against an FP64 GEMV, and the trajectory and
    accumulators against the oracle."""
    print(f"[few-replica dense] n={n} R={R} prec={prec}", flush=True)
    M, h = dense_case(n, 91)
    M64 = M.astype(np.float64)
    g = fi.load_gle("invsqrt_ns4")
    pairs = fi.random_pairs(n, 32, 8)
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=R, precision=prec, seed=3, stream_id=2, burn_in=3,
                     block_len=9, acc_diag=True, steps_per_graph=16)
    rng = np.random.default_rng(n + R)
    q = rng.normal(size=(n, R))
    if prec != fth.FTH_FP64:
        q = q.astype(np.float32).astype(np.float64)
    err = normwise(sol.force(q), -(M64 @ q))
    print(f"  force normwise error {err:.2e} ({sol.kernel_name})", flush=True)
    assert "dense_gemv_kernel" in sol.kernel_name
    assert err <= (1e-13 if prec == fth.FTH_FP64 else 2e-5)
    orc = oracle.OracleRun(M64, g.A_p, g.C_p, h, R, np.concatenate([pairs, fi.diag_pairs(n)]), seed=3, stream=2,
                           burn_in=3, block_len=9)
    tol = 1e-10 if prec == fth.FTH_FP64 else 1e-4
    done = 0
    for target in steps:
        sol.run(target - done)
        orc.run(target - done)
        done = target
        q, p, s = sol.state()
        blk, s1, s2, nb, step = sol.accumulators()
        errs = {"q": normwise(q, orc.q), "p": normwise(p, orc.p), "s": normwise(s, orc.s),
                "acc": normwise(s1 + blk, orc.s1 + orc.blk)}
        print(f"  step {done}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v <= tol, (n, R, prec, done, k, v)
    sol.close()


def test_dense_full_size_two_steps():
    """N = 16384, R = 128, split-BF16x3 (the configuration the benchmark
    times): force against an FP64 GEMM on the full state, then two steps of
    the whole path against the oracle, and two more from the GPU's own state
    at step 1000."""
    n, R = 16384, 128
    print("[fullsize] dense 16384 generating matrix", flush=True)
    M = fi.dense_ggt(n, 4004)
    h = fi.dt_rule(fi.power_lambda_max(M.astype(np.float64), iters=30))
    g = fi.load_gle("invsqrt_ns4")
    pairs = fi.random_pairs(n, 1024, 4005)
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=R, precision=fth.FTH_FP32_BF16X3, seed=5,
                     acc_diag=True, steps_per_graph=2)
    rng = np.random.default_rng(1)
    q = rng.normal(size=(n, R)).astype(np.float32).astype(np.float64)
    M64 = M.astype(np.float64)
    F = sol.force(q)
    err = normwise(F, -(M64 @ q))
    print(f"[fullsize] force normwise error {err:.2e}", flush=True)
    assert err <= 3e-5
    sol.run(2)
    orc = oracle.OracleRun(M64, g.A_p, g.C_p, h, R, np.concatenate([pairs, fi.diag_pairs(n)]), seed=5).run(2)
    qg, pg, sg = sol.state()
    for name, a, b in (("q", qg, orc.q), ("p", pg, orc.p), ("s", sg, orc.s)):
        e = normwise(a, b)
        print(f"[fullsize] {name}: {e:.2e}", flush=True)
        assert e <= 1e-4
    # late steps: the oracle restarts from the GPU's state at step 1000 (noise counters and block
    # bookkeeping from the global step index); both take two more steps
    del orc
    sol.run(998)
    q0, p0, s0 = sol.state()
    blk0, s1_0, s2_0, nb0, step0 = sol.accumulators()
    assert step0 == 1000
    late = oracle.OracleRun(M64, g.A_p, g.C_p, h, R, np.concatenate([pairs, fi.diag_pairs(n)]), seed=5)
    late.step = 1000
    late.set_state(q0, p0, s0)
    sol.run(2)
    late.run(2)
    qg, pg, sg = sol.state()
    blk, s1, s2, nb, step = sol.accumulators()
    assert step == late.step == 1002
    for name, a, b in (("q", qg, late.q), ("p", pg, late.p), ("s", sg, late.s),
                       ("acc", (s1 - s1_0) + (blk - blk0), late.s1 + late.blk)):
        e = normwise(a, b)
        print(f"[fullsize] late steps 1000..1002 {name}: {e:.2e}", flush=True)
        assert e <= 1e-4
    sol.close()


@pytest.mark.parametrize("prec", [fth.FTH_FP64, fth.FTH_FP32_BF16X3], ids=["fp64", "bf16x3"])
def test_dense_estimates_match_gh(prec):
    """Statistics: <q_i q_j> from the dense path against g_h(M) by eigh."""
    n, R = 256, 64
    M, h = dense_case(n, 11)
    g = fi.load_gle("invsqrt_ns4")
    pairs = fi.random_pairs(n, 64, 3)
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=R, precision=prec, seed=8, burn_in=2000,
                     block_len=2000, acc_diag=True)
    sol.run(42000)
    est, se, _ = sol.read()
    ref_m = exact.gh_matrix(M.astype(np.float64), g.A_p, g.C_p, h)
    allp = np.concatenate([pairs, fi.diag_pairs(n)])
    ref = ref_m[allp[:, 0], allp[:, 1]]
    z = (est - ref) / se
    print(f"[stats {prec}] max|z| {np.max(np.abs(z)):.2f}, mean rel diag err "
          f"{np.mean(np.abs(est[64:] / ref[64:] - 1)):.2e}", flush=True)
    assert np.max(np.abs(z)) < 5.5


def test_dense_repeatable_and_resume():
    M, h = dense_case(400, 5)
    g = fi.load_gle("invsqrt_ns4")
    a = fth.Solver(M, g.A_p, g.C_p, h, replicas=16, precision=fth.FTH_FP32_BF16X3, seed=3, acc_diag=True).run(30).run(20)
    b = fth.Solver(M, g.A_p, g.C_p, h, replicas=16, precision=fth.FTH_FP32_BF16X3, seed=3, acc_diag=True,
                   steps_per_graph=1).run(50)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    for x, y in zip(a.accumulators()[:3], b.accumulators()[:3]):
        assert np.array_equal(x, y)


def test_dense_path_selection_and_unsupported_shapes():
    g = fi.load_gle("invsqrt_ns4")
    M, h = dense_case(64, 1)
    small = fth.Solver(M, g.A_p, g.C_p, h, replicas=8, precision=fth.FTH_FP32_BF16X3).run(1)
    assert "small_dense_kernel" in small.kernel_name     # N R <= 4096: one persistent workgroup
    M, h = dense_case(4200, 1)
    few = fth.Solver(M, g.A_p, g.C_p, h, replicas=8, precision=fth.FTH_FP32_BF16X3).run(1)
    assert "dense_gemv_kernel" in few.kernel_name        # R <= 8: matrix-vector products
    with pytest.raises(fth.FthError) as e:
        fth.Solver(M, g.A_p, g.C_p, h, replicas=256, precision=fth.FTH_FP32_BF16X3).run(1)
    assert e.value.status == fth.FTH_EUNSUPPORTED         # matrix-core path needs R in {16..128}
    with pytest.raises(fth.FthError) as e:
        fth.Solver(M, g.A_p, g.C_p, h, replicas=16, precision=fth.FTH_FP32)
    assert e.value.status == fth.FTH_EUNSUPPORTED          # plain FP32 beyond one workgroup: R <= 8 only
    with pytest.raises(fth.FthError) as e:
        fth.Solver(M, g.A_p, g.C_p, h, precision=fth.FTH_FP32)
    assert e.value.status == fth.FTH_EUNSUPPORTED          # ... given at create
    # a context set up for few replicas keeps that form
    with pytest.raises(fth.FthError) as e:
        fth.Solver(M, g.A_p, g.C_p, h, replicas=4, precision=fth.FTH_FP64).run(1, replicas=16)
    assert e.value.status == fth.FTH_ESTATE
