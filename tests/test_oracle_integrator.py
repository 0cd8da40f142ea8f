"""Pins of the oracle's step loop and estimators.

* A deterministic pin against a different formulation: the whole state of a
  tiny system advanced by explicit block matrices (Kronecker products of M,
  T, S with identities) fed with the same normals.
* Textbook leapfrog: with T = I and S = 0 the positions obey Stormer's
  three-term recurrence.
* Closed forms: the white-noise Langevin limit of Sec. I (<q q^T> = kT M^-1,
  exactly kT (M - h^2 M^2 / 4)^-1 for the integrated step), g_h(M) of a
  fitted GLE, and the exact finite-time covariance from the zero state.
* Bookkeeping: block sums against a recorded history; resume and replica
  independence; standard-error calibration over independent seeds.
"""
import numpy as np
import pytest

import fth_inputs
import oracle
from oracle import exact


def random_spd(n, seed, lo=1.0, hi=10.0):
    m, lam = fth_inputs.haar_spd(n, seed, lo, hi)
    return m, lam


def random_gle(ns, seed):
    rng = np.random.default_rng(seed)
    d = ns + 1
    K = rng.normal(size=(d, d))
    A = (K - K.T) + np.diag(rng.uniform(0.3, 2.0, d))
    return A, 0.9 * np.eye(d)


def full_state_step(M, T, S, h, x, xi):
    """x = [q; p; s_1..s_ns] (blocks of N) for one replica, xi = [xi_0..xi_ns]."""
    N = M.shape[0]
    d = T.shape[0]
    n = (d + 1) * N
    I = np.eye(N)
    KB = np.eye(n)
    KB[N:2 * N, 0:N] = -0.5 * h * M
    KA = np.eye(n)
    KA[0:N, N:2 * N] = h * I
    O = np.eye(n)
    O[N:, N:] = np.kron(T, I)
    WO = np.zeros((n, d * N))
    WO[N:, :] = np.kron(S, I)
    return KA @ KB @ (O @ (KB @ x) + WO @ xi)


def test_step_matches_full_state_linear_map(orc):
    N, ns, R, steps, h = 3, 2, 5, 7, 0.17
    M, _ = random_spd(N, 1, 1.0, 6.0)
    A, C = random_gle(ns, 2)
    T, S = oracle.propagator(A, C, h)
    rng = np.random.default_rng(3)
    q0, p0, s0 = rng.normal(size=(N, R)), rng.normal(size=(N, R)), rng.normal(size=(ns, N, R))
    run = oracle.OracleRun(M, A, C, h, R, np.zeros((0, 2)), seed=77, stream=5)
    run.set_state(q0, p0, s0)
    run.run(steps)
    for r in range(R):
        x = np.concatenate([q0[:, r], p0[:, r]] + [s0[k, :, r] for k in range(ns)])
        for n in range(steps):
            xi = np.concatenate([orc.normals(77, 5, np.arange(N), r, n, j) for j in range(ns + 1)])
            x = full_state_step(M, T, S, h, x, xi)
        assert np.allclose(run.q[:, r], x[:N], rtol=1e-12, atol=1e-12)
        assert np.allclose(run.p[:, r], x[N:2 * N], rtol=1e-12, atol=1e-12)
        for k in range(ns):
            assert np.allclose(run.s[k, :, r], x[(2 + k) * N:(3 + k) * N], rtol=1e-12, atol=1e-12)


def test_csr_and_dense_forms_agree(orc):
    csr = fth_inputs.banded_spd_csr(40, 8, dtype=np.float64)
    A, C = random_gle(3, 4)
    pairs = np.array([[0, 1], [5, 5], [39, 2]], dtype=np.int32)
    a = oracle.OracleRun(csr, A, C, 0.05, 6, pairs, seed=1, block_len=5).run(23)
    b = oracle.OracleRun(csr.to_dense(), A, C, 0.05, 6, pairs, seed=1, block_len=5).run(23)
    assert np.allclose(a.q, b.q, rtol=1e-12, atol=1e-14)
    assert np.allclose(a.s1, b.s1, rtol=1e-12, atol=1e-14)


def test_leapfrog_recurrence_without_thermostat(orc):
    N, R, h = 5, 3, 0.11
    M, _ = random_spd(N, 7, 1.0, 20.0)
    rng = np.random.default_rng(8)
    q0, p0 = rng.normal(size=(N, R)), rng.normal(size=(N, R))
    run = oracle.OracleRun(M, None, None, h, R, np.zeros((0, 2)), T=np.eye(1), S=np.zeros((1, 1)))
    run.set_state(q0, p0)
    qs = [q0.copy()]
    for _ in range(40):
        run.run(1)
        qs.append(run.q.copy())
    # first step of leapfrog with the stored p as the half-step momentum
    assert np.allclose(qs[1], q0 + h * p0 - h * h * (M @ q0), atol=1e-13)
    for n in range(1, 40):
        assert np.allclose(qs[n + 1], 2 * qs[n] - qs[n - 1] - h * h * (M @ qs[n]), atol=1e-11)


def test_accumulator_bookkeeping(orc):
    N, R, burn, L, steps = 4, 3, 3, 4, 23
    M, _ = random_spd(N, 9)
    A, C = random_gle(1, 10)
    pairs = np.array([[0, 0], [1, 3], [2, 1]], dtype=np.int32)
    run = oracle.OracleRun(M, A, C, 0.1, R, pairs, seed=4, burn_in=burn, block_len=L)
    hist = []
    for _ in range(steps):
        hist.append(run.q.copy())
        run.run(1)
    x = np.array([[np.sum(q[a] * q[b]) for a, b in pairs] for q in hist[burn:]])
    nb = (steps - burn) // L
    blocks = x[:nb * L].reshape(nb, L, -1).sum(axis=1)
    assert int(run.nblocks[0]) == nb
    assert np.allclose(run.s1, blocks.sum(axis=0), rtol=1e-13)
    assert np.allclose(run.s2, (blocks ** 2).sum(axis=0), rtol=1e-13)
    assert np.allclose(run.blk, x[nb * L:].sum(axis=0), rtol=1e-13)
    mean, se = run.estimates()
    assert np.allclose(mean, x.mean(axis=0) / R, rtol=1e-13)
    bm = blocks / (R * L)
    assert np.allclose(se, bm.std(axis=0, ddof=1) / np.sqrt(nb), rtol=1e-10)


def test_resume_and_replica_independence(orc):
    csr = fth_inputs.laplacian3d_csr(4, 0.1, dtype=np.float64)
    A, C = random_gle(4, 12)
    pairs = fth_inputs.random_pairs(csr.n, 10, 1)
    a = oracle.OracleRun(csr, A, C, 0.03, 8, pairs, seed=5, stream=2, block_len=7).run(13).run(17)
    b = oracle.OracleRun(csr, A, C, 0.03, 8, pairs, seed=5, stream=2, block_len=7).run(30)
    assert np.array_equal(a.q, b.q) and np.array_equal(a.s, b.s) and np.array_equal(a.s1, b.s1)
    c = oracle.OracleRun(csr, A, C, 0.03, 4, pairs, seed=5, stream=2, block_len=7).run(30)
    assert np.array_equal(c.q, b.q[:, :4]) and np.array_equal(c.p, b.p[:, :4])


def test_white_noise_closed_form(orc):
    """Sec. I canonical limit: <q q^T> = kT M^-1 in continuous time; the
    integrated step samples kT (M - h^2 M^2 / 4)^-1 exactly.  h is chosen so
    the two differ by ~6 % on the stiffest mode and the test tells them apart."""
    N, R = 6, 256
    M, lam = random_spd(N, 21, 1.0, 10.0)
    h = 0.5 / np.sqrt(lam.max())
    kT, gamma = 1.0, 1.0
    pairs = np.array([(i, j) for i in range(N) for j in range(i, N)], dtype=np.int32)
    run = oracle.OracleRun(M, [[gamma]], [[kT]], h, R, pairs, seed=31, burn_in=400, block_len=100)
    run.run(6400)
    mean, se = run.estimates()
    exact_h = kT * np.linalg.inv(M - h * h * M @ M / 4)
    exact_0 = kT * np.linalg.inv(M)
    ref_h = exact_h[pairs[:, 0], pairs[:, 1]]
    ref_0 = exact_0[pairs[:, 0], pairs[:, 1]]
    z = (mean - ref_h) / se
    assert np.max(np.abs(z)) < 4.5, z
    z0 = (mean - ref_0) / se
    assert np.max(np.abs(z0)) > 6.0


def test_fitted_gle_matches_gh_matrix(orc):
    """Normal-mode invariance (Sec. I): time averages of q_i q_j approach
    g_h(M)_ij = (U g_h(Lambda) U^T)_ij."""
    try:
        g = fth_inputs.load_gle("invsqrt_ns4")
    except FileNotFoundError:
        pytest.skip("GLE file not fitted yet")
    N, R = 6, 128
    M, lam = random_spd(N, 41, 0.2, 10.0)
    h = 0.1 / np.sqrt(lam.max())
    pairs = np.array([(i, j) for i in range(N) for j in range(i, N)], dtype=np.int32)
    run = oracle.OracleRun(M, g.A_p, g.C_p, h, R, pairs, seed=32, burn_in=2000, block_len=400)
    run.run(12000)
    mean, se = run.estimates()
    ref = exact.gh_matrix(M, g.A_p, g.C_p, h)[pairs[:, 0], pairs[:, 1]]
    z = (mean - ref) / se
    assert np.max(np.abs(z)) < 4.5, z


def test_finite_time_covariance_from_zero(orc):
    """Brute force on a tiny system: the replica covariance of q after n steps
    from the all-zero state equals U diag(X_qq(lambda_k, n)) U^T, with X the
    exact per-mode covariance recursion X <- G X G^T + W W^T."""
    N, ns, R, n = 3, 2, 40000, 25
    M, lam = random_spd(N, 51, 0.5, 4.0)
    A, C = random_gle(ns, 52)
    h = 0.2
    T, S = oracle.propagator(A, C, h)
    run = oracle.OracleRun(M, A, C, h, R, np.zeros((0, 2)), seed=53).run(n)
    lam_, U = np.linalg.eigh(M)
    xq = np.array([exact.finite_cov(l, T, S, h, n)[0, 0] for l in lam_])
    ref = (U * xq) @ U.T
    q = run.q
    emp = q @ q.T / R
    # sampling error of E[q_i q_j]: sqrt((S_ii S_jj + S_ij^2) / R)
    sd = np.sqrt((np.outer(np.diag(ref), np.diag(ref)) + ref ** 2) / R)
    assert np.max(np.abs(emp - ref) / sd) < 4.5


def test_stderr_calibration_over_seeds(orc):
    N, R, L = 4, 4, 50
    M, lam = random_spd(N, 61, 1.0, 5.0)
    h = 0.1 / np.sqrt(lam.max())
    pairs = np.array([[0, 0], [1, 1], [0, 2]], dtype=np.int32)
    means, ses = [], []
    for seed in range(48):
        run = oracle.OracleRun(M, [[1.0]], [[1.0]], h, R, pairs, seed=1000 + seed, burn_in=300, block_len=L)
        run.run(300 + 40 * L)
        m, s = run.estimates()
        means.append(m)
        ses.append(s)
    ratio = np.std(means, axis=0, ddof=1) / np.mean(ses, axis=0)
    assert np.all((ratio > 0.65) & (ratio < 1.5)), ratio


def test_momentum_form_white_noise_closed_form(orc):
    """Momentum form of the estimator (Eq. 7, p_n sampled with q_n): with a
    white-noise thermostat the integrated step samples <p p^T> =
    kT (I - h^2 M / 4)^-1 exactly; the continuous-time kT I is excluded at
    this h.  The q-q block of the same run is unchanged by keeping p-p."""
    N, R = 6, 256
    M, lam = random_spd(N, 22, 1.0, 10.0)
    h = 0.9 / np.sqrt(lam.max())
    kT = 1.3
    pairs = np.array([(i, j) for i in range(N) for j in range(i, N)], dtype=np.int32)
    run = oracle.OracleRun(M, [[1.0]], [[kT]], h, R, pairs, seed=35, burn_in=400, block_len=100, pp=True)
    run.run(6400)
    mean, se = run.estimates()
    A = len(pairs)
    ref_h = (kT * np.linalg.inv(np.eye(N) - h * h * M / 4))[pairs[:, 0], pairs[:, 1]]
    ref_0 = (kT * np.eye(N))[pairs[:, 0], pairs[:, 1]]
    z = (mean[A:] - ref_h) / se[A:]
    assert np.max(np.abs(z)) < 4.5, z
    assert np.max(np.abs((mean[A:] - ref_0) / se[A:])) > 6.0
    q_only = oracle.OracleRun(M, [[1.0]], [[kT]], h, R, pairs, seed=35, burn_in=400, block_len=100).run(6400)
    assert np.array_equal(q_only.s1, run.s1[:A]) and np.array_equal(q_only.blk, run.blk[:A])


def test_momentum_form_fitted_gle_matches_exact(orc):
    """Colored noise: time averages of p_i p_j approach U gh_p(Lambda) U^T,
    the exact stationary momentum response of the integrated step."""
    g = fth_inputs.load_gle("invsqrt_ns4")
    N, R = 5, 128
    M, lam = random_spd(N, 43, 0.2, 10.0)
    h = 0.1 / np.sqrt(lam.max())
    pairs = np.array([(i, j) for i in range(N) for j in range(i, N)], dtype=np.int32)
    run = oracle.OracleRun(M, g.A_p, g.C_p, h, R, pairs, seed=36, burn_in=2000, block_len=400, pp=True)
    run.run(12000)
    mean, se = run.estimates()
    A = len(pairs)
    ref = exact.gh_p_matrix(M, g.A_p, g.C_p, h)[pairs[:, 0], pairs[:, 1]]
    z = (mean[A:] - ref) / se[A:]
    assert np.max(np.abs(z)) < 4.5, z


def test_trace_estimators(orc):
    """Traces of Sec. I: sum_i <q_i^2> = Tr g_h(M), <q^T M q> = Tr[M g_h(M)]
    (= -<q . F>) and sum_i <p_i^2> = Tr gh_p(M), from the eigenvalues; with
    white noise <q^T M q> = kT Tr (I - h^2 M / 4)^-1 in closed form.  The
    trace of the positions also equals the sum of the diagonal estimates of
    the same run up to rounding (every row is in the trace)."""
    N, R = 7, 64
    M, lam = random_spd(N, 44, 0.3, 8.0)
    g = fth_inputs.load_gle("invsqrt_ns4")
    h = 0.1 / np.sqrt(lam.max())
    diag = fth_inputs.diag_pairs(N)
    run = oracle.OracleRun(M, g.A_p, g.C_p, h, R, diag, seed=37, burn_in=2000, block_len=400, pp=True,
                           traces=True)
    run.run(14000)
    mean, se = run.estimates()
    tr_q, tr_qmq, tr_p = mean[2 * N:]
    assert abs(tr_q - mean[:N].sum()) <= 1e-12 * abs(tr_q)
    assert abs(tr_p - mean[N:2 * N].sum()) <= 1e-12 * abs(tr_p)
    T, S = oracle.propagator(g.A_p, g.C_p, h)
    ref = np.array([exact.gh(lam, g.A_p, g.C_p, h, T, S).sum(),
                    (lam * exact.gh(lam, g.A_p, g.C_p, h, T, S)).sum(),
                    exact.gh_p(lam, g.A_p, g.C_p, h, T, S).sum()])
    z = (mean[2 * N:] - ref) / se[2 * N:]
    assert np.max(np.abs(z)) < 4.5, z

    kT = 0.8
    hw = 0.9 / np.sqrt(lam.max())
    w = oracle.OracleRun(M, [[1.0]], [[kT]], hw, R, np.zeros((0, 2)), seed=38, burn_in=400, block_len=100,
                         traces=True).run(8000)
    mw, sw = w.estimates()
    closed = kT * np.trace(np.linalg.inv(np.eye(N) - hw * hw * M / 4))
    assert abs(mw[1] - closed) / sw[1] < 4.5
    assert abs(mw[1] - kT * N) / sw[1] > 6.0   # the continuous-time kT N is excluded
