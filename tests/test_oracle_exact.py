"""Pins of the exact stationary responses g0 and g_h used as statistical
references: closed forms, the paper's scaling relation, independent library
routes (scipy's Lyapunov solvers, eigh, dense inverse), h -> 0 convergence,
and the FFT / Lanczos routes against dense eigendecomposition."""
import numpy as np
import pytest
import scipy.linalg

import fth_inputs
import oracle
from oracle import exact


def gle(ns, seed):
    rng = np.random.default_rng(seed)
    d = ns + 1
    K = rng.normal(size=(d, d))
    A = (K - K.T) + np.diag(rng.uniform(0.3, 2.0, d))
    return A, 1.1 * np.eye(d)


def test_g0_canonical_limit():
    """Sec. I: with a white-noise thermostat at temperature kT a mode of
    frequency omega has <q^2> = kT / omega^2 and <p^2> = kT."""
    lam = np.geomspace(0.01, 100, 17)
    for gamma in (0.1, 1.0, 7.0):
        assert np.allclose(exact.g0(lam, [[gamma]], [[2.5]]), 2.5 / lam, rtol=1e-12)
        assert np.allclose(exact.g0_p(lam, [[gamma]], [[2.5]]), 2.5, rtol=1e-12)


def test_g0_matches_scipy_lyapunov():
    A, C = gle(4, 3)
    lam = np.geomspace(0.1, 12, 9)
    ref = [exact.g0_cov(l, A, C) for l in lam]
    got = exact.g0_cov_batch(lam, A, C)
    for r, g in zip(ref, got):
        assert np.allclose(r, g, rtol=1e-10, atol=1e-12)


def test_g0_scaling_relation():
    """Sec. I scaling: A' = alpha A, C' = gamma C gives
    <p p^T> = gamma f(M' / alpha^2); for positions <q^2>'(alpha^2 lam) =
    (gamma / alpha^2) <q^2>(lam)."""
    A, C = gle(4, 5)
    lam = np.geomspace(0.1, 12, 11)
    for alpha, gam in ((2.0, 0.5), (0.3, 3.0)):
        gp = exact.g0_p(alpha ** 2 * lam, alpha * A, gam * C)
        assert np.allclose(gp, gam * exact.g0_p(lam, A, C), rtol=1e-10)
        gq = exact.g0(alpha ** 2 * lam, alpha * A, gam * C)
        assert np.allclose(gq, gam / alpha ** 2 * exact.g0(lam, A, C), rtol=1e-10)


def test_gh_white_noise_closed_form():
    """Velocity Verlet conserves p^2/2 + omega^2 (1 - h^2 omega^2 / 4) q^2 / 2
    and the exact OU step preserves p ~ N(0, kT), so the integrated step
    samples <q^2> = kT / (omega^2 (1 - h^2 omega^2 / 4))."""
    h = 0.3
    lam = np.geomspace(0.05, 30.0, 13)
    for gamma in (0.2, 1.0, 5.0):
        got = exact.gh(lam, [[gamma]], [[1.7]], h)
        assert np.allclose(got, 1.7 / (lam * (1 - h * h * lam / 4)), rtol=1e-10)


def test_gh_converges_to_g0_second_order():
    A, C = gle(4, 7)
    lam = np.array([0.3, 2.0, 9.0])
    e1 = np.abs(exact.gh(lam, A, C, 0.02) - exact.g0(lam, A, C))
    e2 = np.abs(exact.gh(lam, A, C, 0.01) - exact.g0(lam, A, C))
    ratio = e1 / e2
    assert np.all((ratio > 3.5) & (ratio < 4.5)), ratio


def test_gh_matches_long_time_limit_of_finite_cov():
    A, C = gle(2, 9)
    h = 0.1
    T, S = oracle.propagator(A, C, h)
    for lam in (0.5, 3.0):
        X = exact.finite_cov(lam, T, S, h, 20000)
        assert np.allclose(X, exact.gh_cov(lam, T, S, h), rtol=1e-8, atol=1e-12)


def test_matrix_function_reduces_to_inverse():
    m, _ = fth_inputs.haar_spd(12, 3, 0.5, 20.0)
    assert np.allclose(exact.matrix_function(m, lambda l: 1.0 / l), np.linalg.inv(m), atol=1e-12)
    assert np.allclose(exact.g0_matrix(m, [[1.0]], [[1.0]]), np.linalg.inv(m), atol=1e-11)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_laplacian_fft_route_matches_eigh(n):
    A, C = gle(2, 11)
    h = 0.05
    csr = fth_inputs.laplacian3d_csr(n, 0.1, dtype=np.float64)
    M = csr.to_dense()
    T, S = oracle.propagator(A, C, h)
    g = lambda l: exact.gh(l, A, C, h, T, S)
    dense = exact.matrix_function(M, g)
    K = exact.laplacian_function(n, 0.1, g)
    i, j = np.meshgrid(np.arange(n ** 3), np.arange(n ** 3), indexing="ij")
    assert np.allclose(exact.laplacian_element(K, i, j), dense, atol=1e-11)


def test_lanczos_quadratic_form_matches_eigh():
    csr = fth_inputs.banded_spd_csr(300, 4, dtype=np.float64)
    M = csr.to_dense()
    g = lambda l: l ** -0.5
    ref = exact.matrix_function(M, g)
    for i, j in ((5, 5), (100, 102), (7, 40)):
        e_i = np.zeros(300); e_i[i] = 1
        e_j = np.zeros(300); e_j[j] = 1
        mv = lambda v: M @ v
        if i == j:
            val = exact.lanczos_quadratic_form(mv, 300, e_i, g, 120)
        else:
            val = 0.25 * (exact.lanczos_quadratic_form(mv, 300, e_i + e_j, g, 120)
                          - exact.lanczos_quadratic_form(mv, 300, e_i - e_j, g, 120))
        assert val == pytest.approx(ref[i, j], abs=1e-10)


def test_gh_p_white_noise_closed_form():
    """The step boundary lies between the drift and the first kick of a
    velocity-Verlet block.  Before that block (p, q) follow the Gibbs law of
    the conserved p^2/2 + omega^2 (1 - h^2 omega^2/4) q^2/2 (p ~ N(0, kT)); the
    half kick p - (h/2) omega^2 q then has variance kT / (1 - h^2 omega^2 / 4)."""
    h = 0.3
    lam = np.geomspace(0.05, 30.0, 13)
    for gamma in (0.2, 1.0, 5.0):
        got = exact.gh_p(lam, [[gamma]], [[1.7]], h)
        assert np.allclose(got, 1.7 / (1 - h * h * lam / 4), rtol=1e-10)


def test_g0_momentum_position_relation():
    """Stationarity of <q p> for a harmonic mode under the GLE (continuous
    time): q' = p, p' = -omega^2 q - A_pp p - sum_k A_{p s_k} s_k + noise, and
    <q p> = 0 (from d<q^2>/dt = 0), give
        <p^2> = omega^2 <q^2> + sum_k A_{p s_k} <q s_k>.
    For an equilibrium GLE (C_p = kT I) both sides reduce to equipartition,
    <p^2> = kT = omega^2 <q^2>; a colored-noise GLE fitted to a target has
    <q s_k> != 0, so its momentum and position responses differ."""
    lam = np.geomspace(0.1, 12, 9)
    A, C = gle(4, 9)      # C = 1.1 I: equipartition
    assert np.allclose(exact.g0_p(lam, A, C), 1.1, rtol=1e-9)
    assert np.allclose(exact.g0(lam, A, C), 1.1 / lam, rtol=1e-9)
    g = fth_inputs.load_gle("invsqrt_ns4")
    for Ap, Cp in ((g.A_p, g.C_p), (A, C)):
        for l in lam:
            X = exact.g0_cov(float(l), Ap, Cp)     # order (q, p, s_1..s_ns)
            assert abs(X[0, 1]) <= 1e-9 * np.sqrt(X[0, 0] * X[1, 1])
            rhs = l * X[0, 0] + float(np.dot(Ap[0, 1:], X[0, 2:]))
            assert X[1, 1] == pytest.approx(rhs, rel=1e-9)
    # the fitted thermostat is far from equipartition at the low end of its window
    assert exact.g0_p(np.array([0.1]), g.A_p, g.C_p)[0] > 2 * 0.1 * exact.g0(np.array([0.1]), g.A_p, g.C_p)[0]


def test_gh_p_converges_to_g0_p_second_order():
    A, C = gle(4, 11)
    lam = np.array([0.3, 2.0, 9.0])
    e1 = np.abs(exact.gh_p(lam, A, C, 0.02) - exact.g0_p(lam, A, C))
    e2 = np.abs(exact.gh_p(lam, A, C, 0.01) - exact.g0_p(lam, A, C))
    ratio = e1 / e2
    assert np.all((ratio > 3.5) & (ratio < 4.5)), ratio


def test_tau_slowest_white_noise_closed_form():
    """Langevin thermostat (ns = 0, friction gamma): a mode's relaxation
    rates are the roots of mu^2 - gamma mu + lambda = 0, so the slowest time
    is 2 / gamma when underdamped (gamma^2 < 4 lambda) and
    2 / (gamma - sqrt(gamma^2 - 4 lambda)) when overdamped."""
    for gamma in (0.3, 1.0, 4.0):
        lam = np.geomspace(0.01, 50, 23)
        disc = gamma * gamma - 4 * lam
        want = np.where(disc < 0, 2.0 / gamma, 2.0 / (gamma - np.sqrt(np.maximum(disc, 0.0))))
        assert np.allclose(exact.tau_slowest(lam, np.array([[gamma]])), want, rtol=1e-10)


@pytest.mark.parametrize("name", ["invsqrt_ns4", "fermi_b20_ns4", "ln_ns4"])
def test_tau_slowest_from_discrete_step_map(name):
    """Independent route: the one-step map G of the integrated dynamics
    (kick, exact OU step exp(-A_p h), kick, drift) has spectral radius
    exp(-h / tau) + O(h^2), so -h / ln rho(G) tends to the slowest
    relaxation time as h -> 0 (first order in h)."""
    g = fth_inputs.load_gle(name)
    lo, hi = g.meta["window_lambda"]
    for lam in np.geomspace(lo, hi, 5):
        want = float(exact.tau_slowest(lam, g.A_p)[0])
        errs = []
        for h in (2e-3 / np.sqrt(hi), 1e-3 / np.sqrt(hi)):
            T, S = oracle.propagator(g.A_p, g.C_p, h)
            rho = exact.spectral_radius(lam, T, S, h)
            errs.append(abs(-h / np.log(rho) / want - 1.0))
        assert errs[1] < 2e-3, (lam, errs)
        assert errs[1] < 0.75 * errs[0] + 1e-9  # shrinks with h


@pytest.mark.parametrize("n", [4, 6, 8])
def test_insulator_closed_form_spectrum(n):
    """The two-sublattice lattice's closed-form spectrum against a dense
    eigensolver: half the states below the gap, none inside (4.9, 7.3) with
    the default parameters, bands exactly [0.1, 4.9] and [7.3, 12.1]."""
    M = fth_inputs.insulator3d_csr(n, dtype=np.float64)
    A = np.zeros((M.n, M.n))
    for i in range(M.n):
        for k in range(M.row_ptr[i], M.row_ptr[i + 1]):
            A[i, M.col[k]] += M.val[k]
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    cf = exact.insulator_eigs(n, 1.2, 0.9797958971132712, 6.1)
    assert np.allclose(ev, cf, rtol=0, atol=1e-12)
    assert np.sum(ev < 6.1) == M.n // 2
    assert np.max(ev[ev < 6.1]) <= 4.9 + 1e-12 and np.min(ev[ev > 6.1]) >= 7.3 - 1e-12
    assert ev.min() == pytest.approx(0.1, abs=1e-12) and ev.max() == pytest.approx(12.1, abs=1e-12)


def test_insulator_sublattice_diagonal_against_eigh():
    """Sublattice-resolved diagonal of g(M) from the 2 x 2 Bloch blocks
    against U g(Lambda) U^T from a dense eigensolver, for g = exp(-x / 4) and
    g = 1 / x; every site of a sublattice takes the same value."""
    n = 6
    M = fth_inputs.insulator3d_csr(n, dtype=np.float64)
    A = np.zeros((M.n, M.n))
    for i in range(M.n):
        for k in range(M.row_ptr[i], M.row_ptr[i + 1]):
            A[i, M.col[k]] += M.val[k]
    lam, U = np.linalg.eigh(A)
    idx = np.arange(M.n)
    x, rem = np.divmod(idx, n * n)
    y, z = np.divmod(rem, n)
    even = (x + y + z) % 2 == 0
    for fn in (lambda v: np.exp(-v / 4), lambda v: 1.0 / v):
        d = np.einsum("ik,k,ik->i", U, fn(lam), U)
        e, o = exact.insulator_sublattice_diagonal(n, 1.2, 0.9797958971132712, 6.1, fn)
        assert np.allclose(d[even], e, rtol=1e-12, atol=1e-14)
        assert np.allclose(d[~even], o, rtol=1e-12, atol=1e-14)
        assert not np.isclose(e, o)
