"""The largest thermostat the kernels take, ns = 10 extra momenta (Sec. I: 4 to
10 of them reach a 1 % fit), on every step form, and the blocked forms at
the odd sizes between.

- CSR one-step (FP32 and FP64), split-BF16x3 and FP64 dense, and the small
  dense persistent kernel: trajectories and accumulators against the FP64
  oracle over 1000 steps, at 1e-10 normwise for FP64 and 1e-4 for the FP32
  forms (the tolerances of the other parity tests).
- Blocked sparse step at ns = 1, 7 and 10, persistent and per tile: bit for
  bit the one-step kernel (every row's arithmetic is the one-step kernel's).

The GLE is a random stable drift with C_p = 0.9 I (an equilibrium
thermostat), the same construction as the other random-GLE parity cases."""
import types

import numpy as np
import pytest

import fth_inputs as fi
import oracle
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu

TOL = {fth.FTH_FP64: 1e-10, fth.FTH_FP32: 1e-4, fth.FTH_FP32_BF16X3: 1e-4}


def random_gle(ns, seed):
    rng = np.random.default_rng(seed)
    d = ns + 1
    K = rng.normal(size=(d, d))
    A = (K - K.T) + np.diag(rng.uniform(0.3, 2.0, d))
    return types.SimpleNamespace(A_p=A, C_p=0.9 * np.eye(d))


def normwise(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


def compare(sol, orc, tol, label, steps=(1, 10, 100, 1000)):
    done = 0
    for target in steps:
        sol.run(target - done)
        orc.run(target - done)
        done = target
        q, p, s = sol.state()
        blk, s1, _, _, step = sol.accumulators()
        assert step == done
        errs = {"q": normwise(q, orc.q), "p": normwise(p, orc.p), "s": normwise(s, orc.s),
                "acc": normwise(s1 + blk, orc.s1 + orc.blk)}
        print(f"  [{label}] step {done}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v <= tol, (label, done, k, v)


@pytest.mark.parametrize("prec", [fth.FTH_FP32, fth.FTH_FP64], ids=["fp32", "fp64"])
def test_csr_ns10_against_oracle(prec):
    print(f"[max ns] csr ns10 prec {prec}", flush=True)
    g = random_gle(10, 31)
    M = fi.banded_spd_csr(777, 4321, dtype=np.float64)
    h = fi.dt_rule(fi.gershgorin_max(M))
    R = 16
    pairs = fi.random_pairs(M.n, 48, 12)
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=R, precision=prec, seed=99, stream_id=4,
                     burn_in=5, block_len=7, acc_diag=True, temporal_steps=-1, steps_per_graph=16)
    orc = oracle.OracleRun(M, g.A_p, g.C_p, h, R, np.concatenate([pairs, fi.diag_pairs(M.n)]), seed=99, stream=4,
                           burn_in=5, block_len=7)
    compare(sol, orc, TOL[prec], f"csr ns10 {prec}")
    sol.close()


@pytest.mark.parametrize("prec,n,R", [(fth.FTH_FP64, 520, 32), (fth.FTH_FP32_BF16X3, 520, 32),
                                      (fth.FTH_FP64, 40, 16), (fth.FTH_FP32, 40, 16)],
                         ids=["fp64-gemm", "bf16x3-gemm", "fp64-small", "fp32-small"])
def test_dense_ns10_against_oracle(prec, n, R):
    print(f"[max ns] dense ns10 prec {prec} n {n} R {R}", flush=True)
    g = random_gle(10, 32)
    M = fi.dense_ggt(n, 5005)
    M64 = M.astype(np.float64)
    h = fi.dt_rule(fi.power_lambda_max(M64))
    pairs = fi.random_pairs(n, 24, 13)
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=R, precision=prec, seed=7, stream_id=6,
                     burn_in=3, block_len=9, acc_diag=True, steps_per_graph=16)
    orc = oracle.OracleRun(M64, g.A_p, g.C_p, h, R, np.concatenate([pairs, fi.diag_pairs(n)]), seed=7, stream=6,
                           burn_in=3, block_len=9)
    compare(sol, orc, TOL[prec], f"dense ns10 {prec} n {n}")
    print(f"  kernel: {sol.kernel_name}", flush=True)
    assert ("small_dense_kernel" in sol.kernel_name) == (n == 40), sol.kernel_name
    sol.close()


def assert_identical(a, b, label):
    for name, x, y in zip("qps", a.state(), b.state()):
        assert np.array_equal(x, y), (label, name, float(np.max(np.abs(x - y))))
    for name, x, y in zip(("blk", "s1", "s2"), a.accumulators()[:3], b.accumulators()[:3]):
        assert np.array_equal(x, y), (label, name)
    assert a.accumulators()[3:] == b.accumulators()[3:]


# (ns, precision, threads): the largest workgroup the blocked forms allow for that ns
@pytest.mark.parametrize("ns,prec,threads", [(1, fth.FTH_FP32, 1024), (7, fth.FTH_FP32, 512),
                                             (10, fth.FTH_FP32, 256), (7, fth.FTH_FP64, 256),
                                             (10, fth.FTH_FP64, 256)],
                         ids=["ns1-fp32", "ns7-fp32", "ns10-fp32", "ns7-fp64", "ns10-fp64"])
@pytest.mark.parametrize("persistent", [0, -1], ids=["persistent", "per-tile"])
def test_blocked_odd_and_max_ns_bit_identical(ns, prec, threads, persistent):
    print(f"[max ns] blocked ns {ns} prec {prec} threads {threads} persistent {persistent}", flush=True)
    g = random_gle(ns, 40 + ns)
    M = fi.banded_spd_csr(5003, 17, dtype=np.float64 if prec == fth.FTH_FP64 else np.float32)
    h = fi.dt_rule(fi.gershgorin_max(M))
    kw = dict(pairs=fi.random_pairs(M.n, 64, 5), replicas=8, precision=prec, seed=11, stream_id=2, burn_in=4,
              block_len=7, acc_diag=True, steps_per_graph=20)
    a = fth.Solver(M, g.A_p, g.C_p, h, temporal_steps=5, temporal_threads=threads, temporal_persistent=persistent,
                   **kw)
    b = fth.Solver(M, g.A_p, g.C_p, h, temporal_steps=-1, **kw)
    for k in (23, 40):
        a.run(k)
        b.run(k)
    print(f"  kernel: {a.kernel_name}", flush=True)
    assert "KT=5" in a.kernel_name and f"block={threads}" in a.kernel_name, a.kernel_name
    assert a.kernel_name.startswith("tbp_step_kernel" if persistent == 0 else "tb_step_kernel"), a.kernel_name
    assert_identical(a, b, f"ns {ns}")
    a.close()
    b.close()
