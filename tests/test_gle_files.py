"""The GLE parameter files are valid thermostats and their recorded fit
reports (fit error g0 - f, time-step error g_h / g0 - 1, slowest relaxation
time) are what the oracle's exact responses give for them."""
import math

import numpy as np
import pytest

import fth_inputs as fi
import oracle
from oracle import exact


LIBRARY = ["invsqrt_ns4", "fermi_b20_ns4", "fermi_b5_ns4", "ln_ns4", "expneg_ns4", "invsqrt_ns4_h05"]
SMOOTH = {"invsqrt": lambda x: x ** -0.5, "ln": np.log, "expneg": lambda x: np.exp(-x)}


@pytest.mark.parametrize("name", LIBRARY)
def test_fit_report_is_reproduced(name):
    g = fi.load_gle(name)
    oracle.check_gle(g.A_p, g.C_p)
    lo, hi = g.meta["window_lambda"]
    lam = np.geomspace(lo, hi, 400)
    g0 = exact.g0(lam, g.A_p, g.C_p)
    rep = g.meta["fit_report"]
    t = g.meta["target"]
    if t["kind"] in SMOOTH:
        f = SMOOTH[t["kind"]](lam)
        assert np.max(np.abs(g0 / f - 1)) == pytest.approx(rep["max_rel_err"], rel=1e-6)
        if rep.get("h_fit") is None:
            assert rep["max_rel_err"] < 0.05
    else:
        f = 0.5 * (1 - np.tanh(0.5 * t["beta"] * (lam - t["mu"])))
        live = f >= t["delta"] * f.max()
        assert np.max(np.abs(g0 - f)[live]) / f.max() == pytest.approx(rep["max_abs_err_rel_to_max"], rel=1e-6)
    if rep.get("h_fit") is not None:
        # fitted for the integrated step: its exact response at that step follows f
        gfit = exact.gh(lam, g.A_p, g.C_p, rep["h_fit"])
        assert np.max(np.abs(gfit / f - 1)) == pytest.approx(rep["max_rel_err_gh_at_h_fit"], rel=1e-5)
        assert rep["max_rel_err_gh_at_h_fit"] < 0.05
        assert g.meta["fitted_time_step"] == rep["h_fit"]
    h = rep["dt_used_for_report"]
    gh = exact.gh(lam, g.A_p, g.C_p, h)
    assert np.max(np.abs(gh / g0 - 1)) == pytest.approx(rep["max_rel_dt_err_gh_vs_g0"], rel=1e-5)
    assert np.max(exact.tau_slowest(lam, g.A_p)) == pytest.approx(rep["max_tau_slowest"], rel=1e-6)
    assert rep["max_tau_slowest"] < 40  # no nearly undamped mode
