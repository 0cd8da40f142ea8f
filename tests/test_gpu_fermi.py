"""Zero-temperature occupation of an insulator (Sec. II, Fermi function
paragraph) on the GPU: a gapped two-sublattice lattice, the momentum-form
GLE fitted to a step across its gap, and the estimator of Eq. 7 (<p_i p_j>,
acc_pp) with the kinetic trace.

Parity is statistical, against the exact momentum response of the
integrated step evaluated on the lattice's closed-form spectrum: the trace
(electrons per site per spin times N) and the diagonal, which takes one
value on each sublattice.  The model error (fit + step) against the ideal
step, whose trace is exactly N / 2, stays within the fit report."""
import numpy as np
import pytest

import fth_inputs as fi
import oracle
from oracle import exact
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu

DELTA, HOP, SHIFT = 1.2, 0.9797958971132712, 6.1


@pytest.mark.parametrize("name,prec", [("fermi_gap_p_ns4", fth.FTH_FP32), ("fermi_gap_p_ns6", fth.FTH_FP64)],
                         ids=["ns4-fp32", "ns6-fp64"])
def test_insulator_occupation_and_sublattice_densities(name, prec):
    g = fi.load_gle(name)
    t = g.meta["target"]
    assert t["kind"] == "fermi_gap" and t["mu"] == SHIFT and t["gap"] == pytest.approx(2 * DELTA)
    n_side = 16
    M = fi.insulator3d_csr(n_side, DELTA, HOP, SHIFT, dtype=np.float64 if prec == fth.FTH_FP64 else np.float32)
    n = M.n
    lam = exact.insulator_eigs(n_side, DELTA, HOP, SHIFT)
    lo_w, hi_w = g.meta["window_lambda"]
    assert lam.min() >= lo_w - 1e-9 and lam.max() <= hi_w + 1e-9
    h = fi.dt_rule(hi_w)
    # 58 blocks of 10^4 steps (about four of the slowest relaxation times each), so that the
    # per-site standard errors are well determined and max |z| over 4096 sites stays moderate
    sol = fth.Solver(M, g.A_p, g.C_p, h, replicas=32, precision=prec, seed=41, burn_in=20000,
                     block_len=10000, acc_diag=True, acc_pp=True, acc_trace=True)
    sol.run(600000)
    est, se, _ = sol.read()
    assert est.shape == (2 * n + 3,)
    T, S = oracle.propagator(g.A_p, g.C_p, h)
    gh = lambda x: exact.gh_p(x, g.A_p, g.C_p, h, T, S)   # noqa: E731
    uniq, inv = np.unique(np.round(lam, 12), return_inverse=True)
    ref_tr = float(np.sum(gh(uniq)[inv]))
    z_tr = (est[-1] - ref_tr) / se[-1]
    occ = est[-1] / n
    print(f"[insulator {name}] occupation {occ:.5f} +- {se[-1] / n:.5f}, exact response {ref_tr / n:.5f}, "
          f"ideal 0.5, z {z_tr:.2f}", flush=True)
    assert abs(z_tr) < 5.0
    # sublattice densities: every site against the closed form of its sublattice
    even_ref, odd_ref = exact.insulator_sublattice_diagonal(n_side, DELTA, HOP, SHIFT, gh)
    idx = np.arange(n)
    x, rem = np.divmod(idx, n_side * n_side)
    y, zc = np.divmod(rem, n_side)
    even = (x + y + zc) % 2 == 0
    ref_d = np.where(even, even_ref, odd_ref)
    z = (est[n:2 * n] - ref_d) / se[n:2 * n]
    print(f"[insulator {name}] sublattice densities even {np.mean(est[n:2 * n][even]):.5f} (exact {even_ref:.5f}), "
          f"odd {np.mean(est[n:2 * n][~even]):.5f} (exact {odd_ref:.5f}), max|z| {np.max(np.abs(z)):.2f}", flush=True)
    assert np.max(np.abs(z)) < 5.5
    # the model error: the exact response against the ideal step (N / 2 states below the gap)
    rep = g.meta["fit_report"]
    bound = rep["max_abs_err_outside_gap_gh"] + 1e-12
    assert abs(ref_tr / n - 0.5) <= bound
    assert abs(occ - 0.5) <= bound + 5 * se[-1] / n
