"""GPU tests of the temporally blocked sparse step (several steps per launch
for narrow-band CSR matrices).

Each row's arithmetic is the one-step kernel's (same gather order, noise
counters and update), and the diagonal and pair accumulators are formed in
the same order, so the blocked form must reproduce the one-step form bit for
bit: state, accumulators and step counter.  It is also compared with the FP64
oracle directly at the FP64 tolerance.
"""
import numpy as np
import pytest

import fth_inputs as fi
import oracle
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu


def banded(n, seed, prec):
    M = fi.banded_spd_csr(n, seed, dtype=np.float64 if prec == fth.FTH_FP64 else np.float32)
    return M, fi.dt_rule(fi.gershgorin_max(M))


def run_pair(M, h, g, kt, threads, R, prec, chunks, steps_per_graph, npairs=64, persistent=0):
    kw = dict(pairs=fi.random_pairs(M.n, npairs, 5) if npairs else None, replicas=R, precision=prec, seed=11,
              stream_id=2, burn_in=4, block_len=7, acc_diag=True, steps_per_graph=steps_per_graph)
    a = fth.Solver(M, g.A_p, g.C_p, h, temporal_steps=kt, temporal_threads=threads, temporal_persistent=persistent,
                   **kw)
    b = fth.Solver(M, g.A_p, g.C_p, h, temporal_steps=-1, **kw)
    for k in chunks:
        a.run(k)
        b.run(k)
    return a, b


def assert_identical(a, b, label):
    for name, x, y in zip("qps", a.state(), b.state()):
        assert np.array_equal(x, y), (label, name, float(np.max(np.abs(x - y))))
    for name, x, y in zip(("blk", "s1", "s2"), a.accumulators()[:3], b.accumulators()[:3]):
        assert np.array_equal(x, y), (label, name)
    assert a.accumulators()[3:] == b.accumulators()[3:]


# (KT, threads, R): every combination keeps at least half of a workgroup's rows as output
@pytest.mark.parametrize("kt,threads,R", [(3, 256, 16), (3, 512, 32), (3, 1024, 32), (5, 1024, 32), (5, 512, 8)])
@pytest.mark.parametrize("prec", [fth.FTH_FP32, fth.FTH_FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("persistent", [0, -1], ids=["persistent", "per-tile"])
def test_blocked_bit_identical_to_one_step(kt, threads, R, prec, persistent):
    """Both blocked forms (the persistent one, which stages the next tile in
    LDS, and one workgroup per tile) reproduce the one-step kernel bit for
    bit."""
    if prec == fth.FTH_FP64 and threads > 512:
        threads = 512   # FP64 with ns = 4 keeps (p, s) in the registers of at most 512 threads
    g = fi.load_gle("fermi_b20_ns4")
    M, h = banded(30011, 7, prec)   # ragged: no tile size divides n
    # chunks: shorter than a launch pair, a graph length that is not a multiple of 2 KT, a long run
    a, b = run_pair(M, h, g, kt, threads, R, prec, chunks=(1, 2 * kt - 1, 37, 100), steps_per_graph=16,
                    persistent=persistent)
    print(f"[tb] {a.kernel_name}", flush=True)
    assert ("tbp_step_kernel" if persistent == 0 else "tb_step_kernel") in a.kernel_name
    assert_identical(a, b, (kt, threads, prec, persistent))


@pytest.mark.parametrize("R", [4, 8, 64])
def test_blocked_replica_counts_and_tiny_systems(R):
    g = fi.load_gle("invsqrt_ns4")
    for n in (5, 1000, 4099):
        M, h = banded(n, 100 + n, fth.FTH_FP32)
        a, b = run_pair(M, h, g, 3, 0, R, fth.FTH_FP32, chunks=(13, 50), steps_per_graph=12,
                        npairs=min(16, n))
        assert_identical(a, b, (R, n))


def test_blocked_white_noise_and_no_pairs():
    """ns = 0 (white-noise Langevin) and no selected pairs: only the diagonal."""
    M, h = banded(20000, 3, fth.FTH_FP32)
    a, b = run_pair(M, h, fi.white_noise_gle(1.0, 1.0), 5, 1024, 16, fth.FTH_FP32, chunks=(60,),
                    steps_per_graph=20, npairs=0)
    assert_identical(a, b, "ns0")


def test_blocked_against_oracle_fp64():
    g = fi.load_gle("fermi_b20_ns4")
    M, h = banded(3000, 21, fth.FTH_FP64)
    pairs = fi.random_pairs(M.n, 32, 8)
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=16, precision=fth.FTH_FP64, seed=4, stream_id=1,
                     burn_in=3, block_len=9, acc_diag=True, temporal_steps=3, steps_per_graph=24)
    orc = oracle.OracleRun(M, g.A_p, g.C_p, h, 16, np.concatenate([pairs, fi.diag_pairs(M.n)]), seed=4, stream=1,
                           burn_in=3, block_len=9)
    sol.run(1000)
    orc.run(1000)
    q, p, s = sol.state()
    blk, s1, s2, nb, step = sol.accumulators()
    for name, x, y in (("q", q, orc.q), ("p", p, orc.p), ("s", s, orc.s), ("acc", s1 + blk, orc.s1 + orc.blk)):
        err = float(np.max(np.abs(x - y)) / np.max(np.abs(y)))
        print(f"[tb oracle] {name}: {err:.2e}", flush=True)
        assert err <= 1e-10


def test_blocking_rejected_where_it_does_not_apply():
    g = fi.load_gle("invsqrt_ns4")
    lap = fi.laplacian3d_csr(16, 0.1)   # half-bandwidth 16^2 * 15: far too wide
    sol = fth.Solver(lap, g.A_p, g.C_p, 0.1, replicas=8, temporal_steps=3)
    with pytest.raises(fth.FthError) as e:
        sol.run(1)
    assert e.value.status == fth.FTH_EUNSUPPORTED
    M, h = banded(5000, 1, fth.FTH_FP32)
    sol = fth.Solver(M, g.A_p, g.C_p, h, replicas=128, temporal_steps=3)   # 32 rows per workgroup: too few
    with pytest.raises(fth.FthError) as e:
        sol.run(1)
    assert e.value.status == fth.FTH_EUNSUPPORTED
    with pytest.raises(fth.FthError) as e:
        fth.Solver(M, g.A_p, g.C_p, h, replicas=8, temporal_steps=4)
    assert e.value.status == fth.FTH_EINVAL


def test_autotuner_may_block_and_keeps_trajectory():
    g = fi.load_gle("fermi_b20_ns4")
    M, h = banded(400_000, 77, fth.FTH_FP32)
    kw = dict(pairs=fi.random_pairs(M.n, 64, 1), replicas=32, seed=3, acc_diag=True, block_len=10)
    a = fth.Solver(M, g.A_p, g.C_p, h, tune=True, **kw).run(66)
    b = fth.Solver(M, g.A_p, g.C_p, h, temporal_steps=-1, **kw).run(66)
    print(f"[tune] {a.kernel_name}", flush=True)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    for x, y in zip(a.accumulators()[:3], b.accumulators()[:3]):
        assert np.allclose(x, y, rtol=1e-12, atol=0)


def test_autotuner_cache_distinguishes_estimators():
    """Two tuned contexts of the same shape in one process, the first with
    position-form accumulators only and the second also with the momentum
    form and traces (which change the eligible blocked shapes): the second
    must not reuse a shape it cannot launch, and both reproduce the one-step
    kernel."""
    g = fi.load_gle("fermi_b20_ns4")
    M, h = banded(200_003, 78, fth.FTH_FP32)
    base = dict(pairs=fi.random_pairs(M.n, 64, 2), replicas=32, seed=5, acc_diag=True, block_len=10)
    for extra in (dict(), dict(acc_pp=True, acc_trace=True), dict()):
        kw = dict(base, **extra)
        a = fth.Solver(M, g.A_p, g.C_p, h, tune=True, **kw).run(40)
        b = fth.Solver(M, g.A_p, g.C_p, h, temporal_steps=-1, **kw).run(40)
        print(f"[tune {sorted(extra)}] {a.kernel_name}", flush=True)
        for x, y in zip(a.state(), b.state()):
            assert np.array_equal(x, y)
        for x, y in zip(a.accumulators()[:3], b.accumulators()[:3]):
            assert np.allclose(x, y, rtol=1e-12, atol=0)   # traces: FP64 sums tiled differently
        a.close()
        b.close()


@pytest.mark.parametrize("persistent", [0, -1], ids=["persistent", "per-tile"])
def test_blocked_full_size_bit_identical(persistent):
    """Banded N = 1e6, R = 32 in the launch shape the benchmark's autotuner
    picks (KT = 5, 1024 threads): bit-identical to the one-step kernel."""
    g = fi.load_gle("fermi_b20_ns4")
    M = fi.banded_spd_csr(1_000_000, 3003)
    h = fi.dt_rule(fi.gershgorin_max(M))
    kw = dict(pairs=fi.random_pairs(M.n, 1024, 3004), replicas=32, seed=2, acc_diag=True, block_len=4,
              steps_per_graph=10)
    a = fth.Solver(M, g.A_p, g.C_p, h, temporal_steps=5, temporal_threads=1024, temporal_persistent=persistent,
                   **kw).run(20)
    b = fth.Solver(M, g.A_p, g.C_p, h, temporal_steps=-1, **kw).run(20)
    print(f"[tb] {a.kernel_name}", flush=True)
    assert "KT=5" in a.kernel_name and "block=1024" in a.kernel_name
    assert ("tbp_step_kernel" if persistent == 0 else "tb_step_kernel") in a.kernel_name
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    for x, y in zip(a.accumulators()[:3], b.accumulators()[:3]):
        assert np.array_equal(x, y)
