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
import oracle
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


def eig_sum(lam, fn):
    return float(np.sum(fn(lam)))


def test_m1_log_det_via_ln_target_and_trace():
    """The paper's M1 (3-D periodic lattice, on-site 100, hopping U[0, 2] to
    six neighbour shells: 81 entries per row).  log det M = Tr ln M from the
    position trace of a run on M' = r M with the ln GLE (m = 0), undone by
    subtracting N ln r.  Statistical parity is against the exact response of
    the integrated step, sum_k g_h(r lambda_k); the fit and time-step error
    (against slogdet) are reported separately and bounded by the fit report."""
    g = fi.load_gle("ln_ns4")
    lo_w, hi_w = g.meta["window_lambda"]
    M = fi.m1_lattice_csr(6, 3)
    n = M.n
    lo, hi = fth.fth_gershgorin(M)
    r = hi_w / hi
    lam = np.linalg.eigvalsh(csr_to_dense(M))
    assert r * lam.min() >= lo_w      # the spectrum lands inside the fitted window
    h = 0.1 / np.sqrt(hi_w)
    sol = fth.Solver(M, g.A_p, g.C_p, h, replicas=32, precision=fth.FTH_FP32, seed=12, burn_in=2000,
                     block_len=2000, acc_diag=True, acc_trace=True, scale_r=r)
    sol.run(60000)
    est, se, _ = sol.read()
    weights = np.concatenate([np.ones(n), [n, 0.0]])   # diagonal, Tr ln, q^T M q (not undone)
    est_u, se_u = fth.fth_unscale(fth.FTH_TARGET_LN, r, 0.0, 1.0, 1.0, weights, est, se)
    logdet = est_u[n]
    ref_h = eig_sum(r * lam, lambda x: exact.gh(x, g.A_p, g.C_p, h)) - n * np.log(r)
    exact_ld = float(np.linalg.slogdet(csr_to_dense(M))[1])
    z = (logdet - ref_h) / se_u[n]
    print(f"[M1 logdet] est {logdet:.3f} +- {se_u[n]:.3f}, exact response {ref_h:.3f}, slogdet {exact_ld:.3f}, "
          f"z {z:.2f}", flush=True)
    assert abs(z) < 5.0
    # the model error (fit + time step) stays within what the fit report states
    bound = g.meta["fit_report"]["max_rel_err"] * np.sum(np.abs(np.log(r * lam))) + \
        g.meta["fit_report"]["max_rel_dt_err_gh_vs_g0"] * np.sum(np.abs(np.log(r * lam))) * 2
    assert abs(ref_h - exact_ld) <= bound


@pytest.mark.parametrize("n_side,gle", [(6, "ln_p_ns8"), (10, "ln_p_ns8"), (10, "ln_p_ns10")])
def test_m1_log_det_via_momentum_form(n_side, gle):
    """log det M1 the way the paper estimates it (Eq. 7 and the Sec. II
    examples, which compare lattices of several sizes): a GLE fitted so that
    <p^2>(omega) = ln omega^2 over omega in [e, 100 e], eight or ten extra
    momenta, no rescaling needed since M1's spectrum (about [80, 190]) sits
    inside the window.  log det M = Tr ln M is the kinetic trace
    sum_i <p_i^2>.  Statistical parity against the exact momentum response
    of the integrated step, sum_k gh_p(lambda_k); the model error (fit +
    step) against slogdet stays within the fit report."""
    g = fi.load_gle(gle)
    assert g.meta["form"] == "p"
    lo_w, hi_w = g.meta["window_lambda"]
    M = fi.m1_lattice_csr(n_side, 3)
    n = M.n
    lam = np.linalg.eigvalsh(csr_to_dense(M))
    assert lo_w <= lam.min() and lam.max() <= hi_w
    _, hi = fth.fth_gershgorin(M)
    h = 0.1 / np.sqrt(hi)
    sol = fth.Solver(M, g.A_p, g.C_p, h, replicas=128, precision=fth.FTH_FP32, seed=31, burn_in=5000,
                     block_len=5000, acc_diag=True, acc_pp=True, acc_trace=True)
    sol.run(100000)
    est, se, _ = sol.read()
    assert est.shape == (2 * n + 3,)       # q diagonal, p diagonal, Tr q^2, q^T M q, Tr p^2
    logdet, se_ld = est[-1], se[-1]
    T, S = oracle.propagator(g.A_p, g.C_p, h)
    ref_h = float(np.sum(exact.gh_p(lam, g.A_p, g.C_p, h, T, S)))
    exact_ld = float(np.sum(np.log(lam)))
    assert exact_ld == pytest.approx(float(np.linalg.slogdet(csr_to_dense(M))[1]), rel=1e-12)
    z = (logdet - ref_h) / se_ld
    print(f"[M1 logdet p-form {n_side}^3 {gle}] est {logdet:.3f} +- {se_ld:.3f}, exact response {ref_h:.3f}, "
          f"slogdet {exact_ld:.3f}, z {z:.2f}", flush=True)
    assert abs(z) < 5.0
    # the per-row diagonal <p_i^2> sums to the trace output
    assert np.sum(est[n:2 * n]) == pytest.approx(logdet, rel=1e-5)
    rep = g.meta["fit_report"]
    bound = (rep["max_rel_err"] + 2 * rep["max_rel_dt_err_gh_vs_g0"]) * np.sum(np.abs(np.log(lam)))
    assert abs(ref_h - exact_ld) <= bound
    assert abs(logdet - exact_ld) <= bound + 5 * se_ld


def test_m2_trace_of_exponential():
    """The paper's M2 (dense, eigenvalues in (-300, 300) by Gerschgorin):
    Tr exp(-M2 / 100) from the exp(-x) GLE on M' = M2 / 100 + 3.1 I, undone by
    e^3.1.  Parity against the exact response; model error against eigh."""
    g = fi.load_gle("expneg_ns4")
    lo_w, hi_w = g.meta["window_lambda"]
    M = fi.m2_gerschgorin(96, 4)
    lo, hi = fth.fth_gershgorin(M.astype(np.float64))
    assert lo > -300 and hi < 300
    r, m = fth.fth_spectral_map(-300.0, 300.0, lo_w, hi_w)
    n = 96
    lam = np.linalg.eigvalsh(M.astype(np.float64))
    h = 0.1 / np.sqrt(hi_w)
    sol = fth.Solver(M.astype(np.float64), g.A_p, g.C_p, h, replicas=32, precision=fth.FTH_FP64, seed=14,
                     burn_in=2000, block_len=2000, acc_diag=True, acc_trace=True, scale_r=r, scale_m=m)
    sol.run(100000)
    assert "small_dense_kernel" in sol.kernel_name   # N R = 3072: one persistent workgroup
    est, se, _ = sol.read()
    weights = np.concatenate([np.ones(n), [n, 0.0]])
    est_u, se_u = fth.fth_unscale(fth.FTH_TARGET_EXPNEG, r, m, 1.0, 1.0, weights, est, se)
    tr = est_u[n]
    ref_h = eig_sum(r * lam + m, lambda x: exact.gh(x, g.A_p, g.C_p, h)) * np.exp(m)
    exact_tr = float(np.sum(np.exp(-r * lam)))
    z = (tr - ref_h) / se_u[n]
    print(f"[M2 Tr exp] est {tr:.4f} +- {se_u[n]:.4f}, exact response {ref_h:.4f}, eigh {exact_tr:.4f}, z {z:.2f}",
          flush=True)
    assert abs(z) < 5.0
    assert abs(ref_h - exact_tr) <= (g.meta["fit_report"]["max_rel_err"] + 0.01) * exact_tr


def test_time_step_aware_fit_corrects_the_step_error():
    """A GLE fitted for the integrated step at h5 = 0.5 / sqrt(lambda_max) (five
    times the standard step: the paper's suggestion of fitting for a specific
    time step) reproduces f = x^-1/2 at that step, while the GLE fitted in
    continuous time carries the time-step bias (about 4 % on the diagonal of
    the 12^3 Laplacian).  Both agree with their own exact responses."""
    n_side = 12
    M = fi.laplacian3d_csr(n_side, 0.1)
    h5 = 0.5 / np.sqrt(fi.laplacian3d_lambda_max(n_side, 0.1))
    f_diag = float(np.mean(exact.laplacian_eigs(n_side, 0.1) ** -0.5))
    bias = {}
    for name in ("invsqrt_ns4_h05", "invsqrt_ns4"):
        g = fi.load_gle(name)
        sol = fth.Solver(M, g.A_p, g.C_p, h5, replicas=32, seed=31, burn_in=500, block_len=500, acc_diag=True)
        sol.run(20000)
        est, se, _ = sol.read()
        T, S = oracle.propagator(g.A_p, g.C_p, h5)
        C = exact.laplacian_function(n_side, 0.1, lambda lam: exact.gh(lam, g.A_p, g.C_p, h5, T, S))
        z = (est - C[0, 0, 0]) / se
        bias[name] = float(np.mean(est)) / f_diag - 1
        print(f"[dt-aware] {name}: diagonal bias against f {bias[name]:+.4f}, max|z| vs exact {np.max(np.abs(z)):.2f}",
              flush=True)
        assert np.max(np.abs(z)) < 5.5
    assert abs(bias["invsqrt_ns4_h05"]) < 0.01
    assert bias["invsqrt_ns4"] > 0.025
