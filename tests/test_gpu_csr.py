"""GPU parity of the sparse (CSR) hot path against the FP64 oracle.

Tolerances: trajectories and accumulators are compared normwise,
max|x_gpu - x_oracle| / max|x_oracle| per array, at <= 1e-10 for the FP64
form and <= 1e-4 for the FP32 form over 1000 steps.  The noise is integer
work first: Philox words must agree bit for bit; the normals then agree to
the rounding of the transcendental functions used on each side.
"""
import numpy as np
import pytest

import fth_inputs as fi
import oracle
from oracle import exact
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu

TOL = {fth.FTH_FP64: 1e-10, fth.FTH_FP32: 1e-4}


def normwise(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


def random_gle(ns, seed):
    rng = np.random.default_rng(seed)
    d = ns + 1
    K = rng.normal(size=(d, d))
    A = (K - K.T) + np.diag(rng.uniform(0.3, 2.0, d))
    return A, 0.9 * np.eye(d)


# ------------------------------------------------------------------ noise
def test_noise_words_bit_exact_and_normals():
    rng = np.random.default_rng(17)
    m = 1 << 16
    i = rng.integers(0, 2 ** 32, size=m, dtype=np.uint64)
    r = rng.integers(0, 2 ** 18, size=m, dtype=np.uint64)
    n = rng.integers(0, 2 ** 32, size=m, dtype=np.uint64)
    j = rng.integers(0, 16, size=m, dtype=np.uint64)
    seed, stream = 0x0123456789ABCDEF, 0xA5A5A5A5
    z64, words = fth.fth_noise_sample(seed, stream, i, r, n, j, fth.FTH_FP64, raw=True)
    ctr = np.stack([i, n, (j << 16) | (r >> 2), np.full(m, stream, dtype=np.uint64)], axis=1)
    ref_words = oracle.philox4x32_10(ctr.astype(np.uint32), [seed & 0xFFFFFFFF, seed >> 32])
    assert np.array_equal(words, ref_words)
    ref = oracle.normals(seed, stream, i, r, n, j)
    assert np.max(np.abs(z64 - ref) / np.maximum(1.0, np.abs(ref))) < 1e-14
    z32 = fth.fth_noise_sample(seed, stream, i, r, n, j, fth.FTH_FP32)
    assert np.max(np.abs(z32 - ref) / np.maximum(1.0, np.abs(ref))) < 5e-6


# ----------------------------------------------------------- trajectories
def make_case(kind, n):
    if kind == "lap":
        return fi.laplacian3d_csr(n, 0.1, dtype=np.float64)
    if kind == "m1":   # the paper's M1 lattice: 81 entries per row (long-row gather batches)
        return fi.m1_lattice_csr(n, 3, dtype=np.float64)
    return fi.banded_spd_csr(n, 3003 + n, dtype=np.float64)


CASES = [
    # id, matrix kind, size, gle, R, precision, random start
    ("lap8-invsqrt-R8-fp64", "lap", 8, "invsqrt_ns4", 8, fth.FTH_FP64, False),
    ("lap8-invsqrt-R8-fp32", "lap", 8, "invsqrt_ns4", 8, fth.FTH_FP32, False),
    ("band1001-fermi-R32-fp32", "band", 1001, "fermi_b20_ns4", 32, fth.FTH_FP32, True),
    ("band1001-invsqrt-R4-fp64", "band", 1001, "invsqrt_ns4", 4, fth.FTH_FP64, True),
    ("band301-white-R1-fp64", "band", 301, "white", 1, fth.FTH_FP64, False),
    ("band301-ns1-R2-fp32", "band", 301, "rand1", 2, fth.FTH_FP32, True),
    ("band257-ns7-R16-fp64", "band", 257, "rand7", 16, fth.FTH_FP64, True),
    ("lap4-invsqrt-R512-fp32", "lap", 4, "invsqrt_ns4", 512, fth.FTH_FP32, False),
    ("m1-6-invsqrt-R8-fp32", "m1", 6, "invsqrt_ns4", 8, fth.FTH_FP32, True),
    ("m1-6-rand3-R32-fp64", "m1", 6, "rand3", 32, fth.FTH_FP64, True),
]


def gle_for(name):
    if name == "white":
        g = fi.white_noise_gle(1.0, 1.0)
        return g.A_p, g.C_p
    if name.startswith("rand"):
        return random_gle(int(name[4:]), 7)
    g = fi.load_gle(name)
    return g.A_p, g.C_p


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_trajectory_parity(case):
    cid, kind, size, gname, R, prec, rand_start = case
    print(f"[parity] {cid}", flush=True)
    M = make_case(kind, size)
    A, C = gle_for(gname)
    lam_max = fi.laplacian3d_lambda_max(size, 0.1) if kind == "lap" else fi.gershgorin_max(M)
    if kind == "m1":
        assert int(np.max(np.diff(M.row_ptr))) == 81
    h = fi.dt_rule(lam_max)
    pairs = fi.random_pairs(M.n, 64, 11)
    seed, stream, burn, L = 123456789, 3, 5, 7
    sol = fth.Solver(M, A, C, h, pairs=pairs, replicas=R, precision=prec, seed=seed, stream_id=stream,
                     burn_in=burn, block_len=L, acc_diag=True, steps_per_graph=16)
    diag = fi.diag_pairs(M.n)
    orc = oracle.OracleRun(M, A, C, h, R, np.concatenate([pairs, diag]), seed=seed, stream=stream,
                           burn_in=burn, block_len=L)
    ns = orc.ns
    if rand_start:
        rng = np.random.default_rng(5)
        q0, p0, s0 = rng.normal(size=(M.n, R)), rng.normal(size=(M.n, R)), rng.normal(size=(ns, M.n, R))
        if prec == fth.FTH_FP32:  # both sides start from the same (FP32-representable) state
            q0, p0, s0 = (x.astype(np.float32).astype(np.float64) for x in (q0, p0, s0))
        sol.set_state(q0, p0, s0)
        orc.set_state(q0, p0, s0)
    done = 0
    for target in (1, 10, 100, 1000):
        sol.run(target - done)
        orc.run(target - done)
        done = target
        q, p, s = sol.state()
        blk, s1, s2, nb, step = sol.accumulators()
        assert step == done and nb == int(orc.nblocks[0])
        errs = {"q": normwise(q, orc.q), "p": normwise(p, orc.p),
                "acc": normwise(s1 + blk, orc.s1 + orc.blk)}
        if ns:
            errs["s"] = normwise(s, orc.s)
        if nb:
            errs["s2"] = normwise(s2, orc.s2)
        print(f"  step {done}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
        for k, v in errs.items():
            assert v <= TOL[prec], (cid, done, k, v)
    est, se, nsamp = sol.read()
    m_o, se_o = orc.estimates()
    assert nsamp == orc.n_acc
    assert normwise(est, m_o) <= 10 * TOL[prec]
    finite = np.isfinite(se_o)
    assert normwise(se[finite], se_o[finite]) <= (1e-2 if prec == fth.FTH_FP32 else 1e-6)
    if kind == "m1":
        print(f"  kernel: {sol.kernel_name}", flush=True)
        assert "long-row batches" in sol.kernel_name
    sol.close()


# ------------------------------------------------ full-size configurations
def compare_full_state(sol, orc, tol, label):
    q, p, s = sol.state()
    blk, s1, s2, nb, step = sol.accumulators()
    assert step == orc.step
    for name, a, b in (("q", q, orc.q), ("p", p, orc.p), ("s", s, orc.s), ("acc", s1 + blk, orc.s1 + orc.blk),
                       ("s2", s2, orc.s2)):
        if not np.any(b):
            assert not np.any(a), name
            continue
        e = normwise(a, b)
        print(f"  {label} step {step} {name}: {e:.2e}", flush=True)
        assert e <= tol, (label, step, name)


@pytest.mark.parametrize("prec", [fth.FTH_FP32, fth.FTH_FP64], ids=["fp32", "fp64"])
def test_laplacian_64cubed_full_size(prec):
    """64^3 periodic Laplacian + 0.1, R = 8, diagonal + 1024 pairs, in the
    benchmark's launch configuration (autotuned shape, 64-step graphs and
    direct tails): the whole state and the accumulators against the oracle
    after 1, 10, 100 and (FP32) 1000 steps."""
    print(f"[fullsize] laplacian 64^3 prec={prec}", flush=True)
    M = fi.laplacian3d_csr(64, 0.1)
    g = fi.load_gle("invsqrt_ns4")
    h = fi.dt_rule(fi.laplacian3d_lambda_max(64, 0.1))
    pairs = fi.random_pairs(M.n, 1024, 2002)
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=8, precision=prec, seed=2, acc_diag=True,
                     steps_per_graph=64, block_len=100, tune=True)
    M64 = fi.CSR(M.n, M.row_ptr, M.col, M.val.astype(np.float64))
    orc = oracle.OracleRun(M64, g.A_p, g.C_p, h, 8, np.concatenate([pairs, fi.diag_pairs(M.n)]), seed=2,
                           block_len=100)
    checkpoints = (1, 10, 100, 1000) if prec == fth.FTH_FP32 else (1, 10, 100)
    done = 0
    for c in checkpoints:
        sol.run(c - done)
        orc.run(c - done)
        done = c
        compare_full_state(sol, orc, TOL[prec], "lap64")
    print(f"  kernel: {sol.kernel_name}", flush=True)
    est, se, nsamp = sol.read()
    m_o, se_o = orc.estimates()
    assert normwise(est, m_o) <= 10 * TOL[prec]
    sol.close()


def test_banded_1e6_full_size_blocked():
    """Banded SPD N = 1e6, R = 32, Fermi GLE, FP32, diagonal + 1024 pairs, in
    the benchmark's blocked launch shape (5 steps per launch, 1024-thread
    workgroups, 20-step graphs): the whole state and the accumulators against
    the oracle after 5 and 100 steps, and over steps 1000 to 1010 from the
    GPU's own state at step 1000."""
    print("[fullsize] banded 1e6 R=32 blocked KT=5", flush=True)
    M = fi.banded_spd_csr(1_000_000, 3003)
    g = fi.load_gle("fermi_b20_ns4")
    h = fi.dt_rule(fi.gershgorin_max(M))
    pairs = fi.random_pairs(M.n, 1024, 3004)
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=32, precision=fth.FTH_FP32, seed=4,
                     acc_diag=True, steps_per_graph=20, block_len=10, temporal_steps=5, temporal_threads=1024)
    M64 = fi.CSR(M.n, M.row_ptr, M.col, M.val.astype(np.float64))
    orc = oracle.OracleRun(M64, g.A_p, g.C_p, h, 32, np.concatenate([pairs, fi.diag_pairs(M.n)]), seed=4,
                           block_len=10)
    done = 0
    for c in (5, 100):
        sol.run(c - done)
        orc.run(c - done)
        done = c
        compare_full_state(sol, orc, 1e-4, "band1e6")
    print(f"  kernel: {sol.kernel_name}", flush=True)
    assert "KT=5" in sol.kernel_name and "block=1024" in sol.kernel_name
    est, se, nsamp = sol.read()
    m_o, se_o = orc.estimates()
    assert normwise(est, m_o) <= 1e-3
    # late steps: the oracle restarts from the GPU's state at step 1000 (noise counters and block
    # bookkeeping from the global step index) and both take one pair of blocked launches
    del orc
    sol.run(900)
    late = oracle.OracleRun(M64, g.A_p, g.C_p, h, 32, np.concatenate([pairs, fi.diag_pairs(M.n)]), seed=4,
                            block_len=10)
    late_step_check(sol, late, 1000, 10, 1e-4, "band1e6")
    sol.close()


def late_step_check(sol, orc, at, more, tol, label):
    """Continue sol (already at step `at`) and a fresh oracle started from
    sol's state at that step by `more` steps; compare the state and what the
    accumulators gained over those steps."""
    q, p, s = sol.state()
    blk0, s1_0, s2_0, nb0, step0 = sol.accumulators()
    assert step0 == at
    orc.step = at
    orc.set_state(q, p, s)
    sol.run(more)
    orc.run(more)
    q, p, s = sol.state()
    blk, s1, s2, nb, step = sol.accumulators()
    assert step == orc.step == at + more and nb - nb0 == int(orc.nblocks[0])
    for name, a, b in (("q", q, orc.q), ("p", p, orc.p), ("s", s, orc.s),
                       ("acc", (s1 - s1_0) + (blk - blk0), orc.s1 + orc.blk), ("s2", s2 - s2_0, orc.s2)):
        if not np.any(b):
            assert not np.any(a), name
            continue
        e = normwise(a, b)
        print(f"  {label} late steps {at}..{at + more} {name}: {e:.2e}", flush=True)
        assert e <= tol, (label, name, e)


# ---------------------------------------------------------- invariances
def _lap_solver(R, spg=16, prec=fth.FTH_FP32, n=12, seed=9):
    M = fi.laplacian3d_csr(n, 0.1)
    g = fi.load_gle("invsqrt_ns4")
    h = fi.dt_rule(fi.laplacian3d_lambda_max(n, 0.1))
    return fth.Solver(M, g.A_p, g.C_p, h, pairs=fi.random_pairs(M.n, 100, 1), replicas=R, precision=prec,
                      seed=seed, acc_diag=True, steps_per_graph=spg, block_len=10)


def test_graph_direct_resume_and_repeat_bit_identical():
    a = _lap_solver(8, spg=16).run(37).run(63)   # graph chunks + direct tails
    b = _lap_solver(8, spg=1).run(100)           # one-step graphs
    c = _lap_solver(8, spg=1000).run(100)        # direct launches only
    d = _lap_solver(8, spg=16).run(100)
    ref_state = d.state()
    ref_acc = d.accumulators()
    for o in (a, b, c):
        for x, y in zip(o.state(), ref_state):
            assert np.array_equal(x, y)
        for x, y in zip(o.accumulators()[:3], ref_acc[:3]):
            assert np.array_equal(x, y)


def test_replica_count_independence():
    a = _lap_solver(8).run(50)
    b = _lap_solver(32).run(50)
    qa, pa, sa = a.state()
    qb, pb, sb = b.state()
    assert np.array_equal(qa, qb[:, :8]) and np.array_equal(pa, pb[:, :8]) and np.array_equal(sa, sb[:, :, :8])


def test_state_roundtrip_and_errors():
    s = _lap_solver(8)
    with pytest.raises(fth.FthError) as e:
        s.run(1, replicas=16)
    assert e.value.status == fth.FTH_ESTATE
    rng = np.random.default_rng(1)
    q = rng.normal(size=(s.n, 8)).astype(np.float32).astype(np.float64)
    s.set_state(q=q)
    q2, _, _ = s.state()
    assert np.array_equal(q, q2)


def test_nonfinite_detection_poisons_context():
    M = fi.laplacian3d_csr(6, 0.1)
    g = fi.load_gle("invsqrt_ns4")
    sol = fth.Solver(M, g.A_p, g.C_p, 1.5, replicas=8, precision=fth.FTH_FP32)  # omega_max h ~ 5 > 2
    with pytest.raises(fth.FthError) as e:
        sol.run(3000)
    assert e.value.status == fth.FTH_ENONFINITE
    with pytest.raises(fth.FthError) as e:
        sol.run(1)
    assert e.value.status == fth.FTH_ESTATE


# ---------------------------------------------------------- statistics
def test_fp32_estimates_match_closed_form_gh():
    """Time averages from the FP32 path approach g_h(M) (normal-mode
    invariance, Sec. I); for the periodic Laplacian every diagonal element
    equals mean_k g_h(lambda_k) and pairs follow from the FFT closed form."""
    n = 16
    M = fi.laplacian3d_csr(n, 0.1)
    g = fi.load_gle("invsqrt_ns4")
    h = fi.dt_rule(fi.laplacian3d_lambda_max(n, 0.1))
    pairs = np.concatenate([fi.random_pairs(M.n, 64, 5),
                            np.array([[0, 1], [0, n], [0, n * n], [5, 6], [100, 100 + n]], dtype=np.int32)])
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=8, precision=fth.FTH_FP32, seed=77,
                     burn_in=3000, block_len=2500, acc_diag=True)
    sol.run(53000)
    est, se, nsamp = sol.read()
    T, S = oracle.propagator(g.A_p, g.C_p, h)
    K = exact.laplacian_function(n, 0.1, lambda l: exact.gh(l, g.A_p, g.C_p, h, T, S))
    all_pairs = np.concatenate([pairs, fi.diag_pairs(M.n)])
    ref = exact.laplacian_element(K, all_pairs[:, 0], all_pairs[:, 1])
    z = (est - ref) / se
    print(f"max|z|={np.max(np.abs(z)):.2f} mean z={np.mean(z):.3f}", flush=True)
    assert np.max(np.abs(z)) < 5.5
    rel = np.abs(est[len(pairs):] / ref[len(pairs):] - 1.0)
    assert np.mean(rel) < 0.01


def test_autotuner_keeps_trajectory():
    """The autotuner picks a launch shape by timing candidates on a saved copy
    of the state; trajectories are unchanged (replicas per thread only changes
    the FP64 summation order of the diagonal accumulators)."""
    M = fi.banded_spd_csr(200_000, 77)
    g = fi.load_gle("invsqrt_ns4")
    h = fi.dt_rule(fi.gershgorin_max(M))
    kw = dict(pairs=fi.random_pairs(M.n, 64, 1), replicas=32, seed=3, acc_diag=True, block_len=10)
    a = fth.Solver(M, g.A_p, g.C_p, h, tune=True, **kw).run(60)
    b = fth.Solver(M, g.A_p, g.C_p, h, tune=False, **kw).run(60)
    print(f"[tune] {a.kernel_name}", flush=True)
    assert "autotuned" in a.kernel_name
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    for x, y in zip(a.accumulators()[:3], b.accumulators()[:3]):
        assert np.allclose(x, y, rtol=1e-12, atol=0)
    assert a.accumulators()[4] == b.accumulators()[4] == 60


def random_symmetric_csr(n, per_row, seed):
    """Symmetric sparse SPD matrix with random far-apart off-diagonals (many
    distinct column offsets)."""
    rng = np.random.default_rng(seed)
    i = np.repeat(np.arange(n), per_row)
    j = rng.integers(0, n, size=n * per_row)
    keep = i != j
    i, j = i[keep], j[keep]
    v = -rng.uniform(0.1, 1.0, size=i.size)
    rows = np.concatenate([i, j])
    cols = np.concatenate([j, i])
    vals = np.concatenate([v, v])
    key = rows * n + cols
    uniq, inv = np.unique(key, return_inverse=True)
    acc = np.zeros(uniq.size)
    np.add.at(acc, inv, vals)
    r, c = uniq // n, uniq % n
    diag = np.zeros(n)
    np.add.at(diag, r, -acc)
    r = np.concatenate([r, np.arange(n)])
    c = np.concatenate([c, np.arange(n)])
    v = np.concatenate([acc, diag + rng.uniform(0.5, 1.0, n)])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    return fi.CSR(n, np.cumsum(row_ptr), c.astype(np.int32), v.astype(np.float32))


@pytest.mark.parametrize("kind,R,prec", [("lap", 8, fth.FTH_FP32), ("lap", 32, fth.FTH_FP64),
                                         ("band", 32, fth.FTH_FP32), ("band", 8, fth.FTH_FP64)])
def test_coded_matrix_bit_identical_to_plain_csr(kind, R, prec):
    """The coded form (one-byte column and value codes into tables, slots in
    CSR order) sums the same products in the same order: bit-identical."""
    M = fi.laplacian3d_csr(20, 0.1) if kind == "lap" else fi.banded_spd_csr(40_000, 9)
    h = fi.dt_rule(fi.laplacian3d_lambda_max(20, 0.1) if kind == "lap" else fi.gershgorin_max(M))
    g = fi.load_gle("invsqrt_ns4")
    kw = dict(pairs=fi.random_pairs(M.n, 64, 2), replicas=R, precision=prec, seed=5, acc_diag=True, block_len=7,
              temporal_steps=-1, steps_per_graph=16)
    a = fth.Solver(M, g.A_p, g.C_p, h, **kw).run(3).run(70)
    b = fth.Solver(M, g.A_p, g.C_p, h, coded_matrix=-1, **kw).run(3).run(70)
    print(f"[coded] {a.kernel_name} | {b.kernel_name}", flush=True)
    assert "CODED=1" in a.kernel_name and "CODED=0" in b.kernel_name
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    for x, y in zip(a.accumulators()[:3], b.accumulators()[:3]):
        assert np.array_equal(x, y)


def test_coded_matrix_not_built_for_scattered_patterns():
    M = random_symmetric_csr(3000, 1, 4)
    assert np.diff(M.row_ptr).max() <= 8
    g = fi.load_gle("invsqrt_ns4")
    h = fi.dt_rule(fi.gershgorin_max(M))
    a = fth.Solver(M, g.A_p, g.C_p, h, replicas=8, seed=1).run(20)
    assert "CODED=0" in a.kernel_name   # far more than 255 distinct offsets j - i
    b = fth.Solver(M, g.A_p, g.C_p, h, replicas=8, seed=1, coded_matrix=-1).run(20)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
