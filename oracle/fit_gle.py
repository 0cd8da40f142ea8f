"""Offline GLE fitter: (A_p, C_p) whose stationary <q^2>(omega) (position
form) or <p^2>(omega) (momentum form, Eq. 7) follows a target f(omega^2) over
a spectral window.

TEST INFRASTRUCTURE / INPUT PREPARATION (part of the oracle).  It writes the
parameter files under ``fth_inputs/gle/``; both the oracle and the HIP library
read those files as plain input, so the file is the contract and neither
side re-fits.

Parametrisation (the "delta-like memory kernel" form the paper starts from,
Sec. I, fitting paragraph):
    A_p = [[a_pp, a^T], [-a, A]],  A = blockdiag of 2x2 [[g_k, w_k], [-w_k, g_k]]
    (a trailing 1x1 block [g] when ns is odd),
with a_pp, g_k > 0.  The symmetric part of A_p is then diag(a_pp, g_k, ...),
positive definite, so A_p is stable by construction.  The diffusion B_p is
a lower-triangular matrix with positive diagonal, and C_p follows from the
Lyapunov relation A_p C_p + C_p A_p^T = B_p B_p^T (Sec. I), which keeps C_p
positive definite and B_p B_p^T positive semi-definite by construction.

Objective (the three requirements of Sec. II):
  (1) agreement of g0(lambda) = <q^2>(sqrt(lambda)) or <p^2>(sqrt(lambda))
      (or, for a fit at a given time step h, of the exact response g_h of
      the integrated step, which corrects the time-step error exactly: Sec. II,
      error paragraph) with f(lambda) on a log-spaced grid over the window:
      log residuals; for targets with an exponentially decaying tail (Fermi,
      or exp(-x) with a threshold) residuals relative to max f where f is
      not negligible plus a hinge penalty that only asks for
      g0 < delta * max g0 where f < delta (the paper's threshold delta); for
      a step across a spectral gap (zero-temperature Fermi occupation of an
      insulator, Sec. II) absolute residuals outside the gap, none inside;
  (2) stability for the time step: a_pp, the omega -> infinity limit of the
      friction kernel, kept below omega_max;
  (3) statistical efficiency: a mild penalty on the slowest relaxation time
      of each mode measured in units of its period.

Usage:  python -m oracle.fit_gle          (writes the standard files)
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np
import scipy.optimize

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    __package__ = "oracle"

from . import check_gle, propagator  # noqa: E402
from .exact import g0, g0_cov, g0_p, gh, gh_cov, gh_p, tau_slowest  # noqa: E402


def n_params(ns: int) -> int:
    d = ns + 1
    nblk2 = ns // 2
    return 1 + ns + 2 * nblk2 + (ns % 2) + d * (d + 1) // 2


def unpack(theta: np.ndarray, ns: int):
    d = ns + 1
    k = 0
    a_pp = math.exp(theta[k]); k += 1
    a = theta[k:k + ns]; k += ns
    A = np.zeros((ns, ns))
    for b in range(ns // 2):
        g = math.exp(theta[k]); w = theta[k + 1]; k += 2
        A[2 * b:2 * b + 2, 2 * b:2 * b + 2] = [[g, w], [-w, g]]
    if ns % 2:
        A[ns - 1, ns - 1] = math.exp(theta[k]); k += 1
    Ap = np.zeros((d, d))
    Ap[0, 0] = a_pp
    Ap[0, 1:] = a
    Ap[1:, 0] = -a
    Ap[1:, 1:] = A
    B = np.zeros((d, d))
    for i in range(d):
        for j in range(i + 1):
            B[i, j] = math.exp(theta[k]) if i == j else theta[k]
            k += 1
    import scipy.linalg
    BB = B @ B.T
    Cp = scipy.linalg.solve_continuous_lyapunov(Ap, BB)
    Cp = 0.5 * (Cp + Cp.T)
    return Ap, Cp


def make_target(kind: str, **kw):
    if kind == "invsqrt":
        return (lambda x: x ** -0.5), None
    if kind == "fermi":
        beta, mu = kw["beta"], kw["mu"]
        return (lambda x: 0.5 * (1.0 - np.tanh(0.5 * beta * (x - mu)))), kw.get("delta", 1e-3)
    if kind == "ln":        # positive on a window above 1 (the method needs f > 0, Sec. I)
        return (lambda x: np.log(x)), None
    if kind == "expneg":    # exp(-x); with delta, followed only down to delta * max (Sec. I, tails)
        return (lambda x: np.exp(-x)), kw.get("delta")
    if kind == "fermi_gap":
        # zero-temperature occupation with the Fermi level mid-gap (Sec. II, Fermi function
        # paragraph): 1 below the gap, 0 above it, and free (NaN) inside it, where a smooth
        # transition changes nothing for a matrix with no eigenvalues there
        mu, half = kw["mu"], 0.5 * kw["gap"]
        return (lambda x: np.where(np.abs(np.asarray(x, dtype=np.float64) - mu) < half, np.nan,
                                   np.where(np.asarray(x) < mu, 1.0, 0.0))), -1.0   # -1: absolute residuals
    raise ValueError(kind)


def response(Ap, Cp, lam, h_fit=None, form="q"):
    """The fitted response at omega^2 = lam: <q^2> (form "q") or <p^2> (form
    "p", the paper's T*(omega) of Eq. 7), in continuous time (g0) or, with a
    time step, the exact response of the integrated step."""
    k = 0 if form == "q" else 1
    if h_fit is None:
        if Ap.shape[0] <= 5:   # small: one batched dense solve
            return g0(lam, Ap, Cp) if form == "q" else g0_p(lam, Ap, Cp)
        return np.array([g0_cov(float(l), Ap, Cp)[k, k] for l in lam])   # Bartels-Stewart per mode
    T, S = propagator(Ap, Cp, h_fit)
    return np.array([gh_cov(float(l), T, S, h_fit)[k, k] for l in lam])


def residuals(theta, ns, lam, f_lam, delta, w_max, w_tau=0.005, tail=None, h_fit=None, form="q"):
    try:
        Ap, Cp = unpack(theta, ns)
        g = response(Ap, Cp, lam, h_fit, form)
    except Exception:
        return np.full(len(lam) + len(lam) + 1, 1e3)
    if not np.all(np.isfinite(g)) or np.any(g <= 0):
        return np.full(len(lam) + len(lam) + 1, 1e3)
    if delta is not None and delta < 0:     # a target with a free gap: absolute error where it is set
        r_fit = np.where(np.isnan(f_lam), 0.0, g - np.nan_to_num(f_lam))
    elif delta is None:
        r_fit = np.log(g) - np.log(f_lam)
    else:
        fmax = np.max(f_lam)
        live = f_lam >= delta * fmax
        r_fit = np.where(live, (g - f_lam) / fmax, 0.0)
        gmax = np.max(g)
        over = np.maximum(0.0, np.log(np.maximum(g, 1e-300)) - np.log(delta * gmax))
        r_fit = r_fit + np.where(live, 0.0, 0.3 * over)
    tau = tau_slowest(lam, Ap)
    r_tau = w_tau * np.log(np.maximum(tau * np.sqrt(lam), 1e-12))
    r_stab = np.array([10.0 * max(0.0, math.log(Ap[0, 0] / w_max))])
    return np.concatenate([r_fit, r_tau, r_stab])


def structured_start(ns: int, lam_lo: float, lam_hi: float, f, rng, jitter: float) -> np.ndarray:
    """Starting point for a momentum-form fit of a smooth target: one
    memory block per log-spaced frequency omega_b of the window, each coupled
    to p and driven at the target's value there (an isolated block with
    friction g and noise b^2 holds variance b^2 / (2 g)), so <p^2>(omega)
    starts as a staircase through f(omega^2)."""
    nb = ns // 2
    th = np.zeros(n_params(ns))
    k = 0
    a_pp = 0.3 * math.sqrt(lam_lo)
    th[k] = math.log(a_pp)
    k += 1
    wb = np.exp(np.linspace(math.log(math.sqrt(lam_lo)), math.log(math.sqrt(lam_hi)), max(nb, 1)))[:nb]
    wb = wb * np.exp(jitter * rng.normal(size=nb))
    gam = 0.5 * wb
    for b in range(nb):
        th[k + 2 * b] = 0.7 * math.sqrt(gam[b] * wb[b])
    k += ns
    for b in range(nb):
        th[k] = math.log(gam[b])
        th[k + 1] = wb[b]
        k += 2
    rates, temps = [a_pp], [float(f(lam_lo))]
    for b in range(nb):
        rates += [gam[b], gam[b]]
        temps += [float(f(wb[b] ** 2))] * 2
    if ns % 2:
        th[k] = math.log(math.sqrt(lam_lo * lam_hi))
        k += 1
        rates.append(math.sqrt(lam_lo * lam_hi))
        temps.append(float(f(lam_hi)))
    d = ns + 1
    for i in range(d):
        for j in range(i + 1):
            th[k] = math.log(math.sqrt(2 * rates[i] * max(temps[i], 1e-12))) if i == j else 0.0
            k += 1
    return th


def gap_start(ns: int, lam_lo: float, lam_hi: float, mu: float, gap: float, rng, jitter: float) -> np.ndarray:
    """Starting point for a momentum-form step across a spectral gap: weak
    coupling, where a mode at omega takes the temperature of the memory
    blocks resonant with it.  ns/2 - 1 hot (kT = 1) blocks at log-spaced
    frequencies across the lower band, one cold block over the upper band,
    and a weak cold Markovian friction; each block's friction peak is 0.1."""
    if ns % 2 or ns < 4:
        raise ValueError("the gap start pairs the extra momenta into at least two blocks")
    nb = ns // 2
    w_lo, w_hi = math.sqrt(lam_lo), math.sqrt(lam_hi)
    w_v, w_c = math.sqrt(mu - 0.5 * gap), math.sqrt(mu + 0.5 * gap)
    hot = np.exp(np.linspace(math.log(1.5 * w_lo), math.log(0.95 * w_v), nb - 1)) * np.exp(jitter * rng.normal(size=nb - 1))
    spacing = (math.log(w_v) - math.log(w_lo)) / max(nb - 1, 1)
    wb = list(hot) + [0.5 * (w_c + w_hi)]
    gam = [0.5 * w * spacing for w in hot] + [0.5 * (w_hi - w_c)]
    kt = [1.0] * (nb - 1) + [1e-3]
    a_pp, peak = 0.005, 0.1
    th = np.zeros(n_params(ns))
    k = 0
    th[k] = math.log(a_pp)
    k += 1
    for b in range(nb):
        th[k + 2 * b] = math.sqrt(peak * gam[b])
    k += ns
    for b in range(nb):
        th[k], th[k + 1] = math.log(gam[b]), wb[b]
        k += 2
    rates, temps = [a_pp], [1e-3]
    for b in range(nb):
        rates += [gam[b], gam[b]]
        temps += [kt[b], kt[b]]
    for i in range(ns + 1):
        for j in range(i + 1):
            th[k] = math.log(math.sqrt(2 * rates[i] * temps[i])) if i == j else 0.0
            k += 1
    return th


def fit(kind: str, ns: int, lam_lo: float, lam_hi: float, starts: int = 8, seed: int = 0,
        npts: int = 48, w_tau: float = 0.005, max_nfev: int = 600, h_fit=None, form="q", **kw):
    f, delta = make_target(kind, **kw)
    lam = np.geomspace(lam_lo, lam_hi, npts)
    if kind == "fermi":  # denser near the step
        lam = np.unique(np.concatenate([lam, np.linspace(kw["mu"] - 6 / kw["beta"], kw["mu"] + 6 / kw["beta"], 24)]))
    if kind == "fermi_gap":   # no points inside the gap, denser at its edges
        lo_e, hi_e = kw["mu"] - 0.5 * kw["gap"], kw["mu"] + 0.5 * kw["gap"]
        lam = lam[np.abs(lam - kw["mu"]) >= 0.5 * kw["gap"]]
        lam = np.unique(np.concatenate([lam, np.linspace(max(lam_lo, lo_e - 1.0), lo_e, 12),
                                        np.linspace(hi_e, min(lam_hi, hi_e + 1.0), 12)]))
    f_lam = f(lam)
    w_max = math.sqrt(lam_hi)
    rng = np.random.default_rng(seed)
    best = None
    for s in range(starts):
        if form == "p" and kind != "fermi":
            if kind == "fermi_gap":
                th = gap_start(ns, lam_lo, lam_hi, kw["mu"], kw["gap"], rng, 0.3)
            else:
                th = structured_start(ns, lam_lo, lam_hi, f, rng, 0.0 if s == 0 else 0.15)
            try:
                res = scipy.optimize.least_squares(residuals, th,
                                                   args=(ns, lam, f_lam, delta, w_max, w_tau, None, h_fit, form),
                                                   method="trf", max_nfev=max_nfev, x_scale="jac")
            except Exception:
                continue
            cost = float(np.sum(res.fun ** 2))
            if best is None or cost < best[0]:
                best = (cost, res.x)
            print(f"  start {s}: cost {cost:.4e}", flush=True)
            continue
        th = np.zeros(n_params(ns))
        k = 0
        th[k] = math.log(math.sqrt(lam_lo * lam_hi) * rng.uniform(0.2, 1.0)); k += 1
        th[k:k + ns] = rng.normal(0, 1.0, ns) * math.sqrt(lam_hi) ** 0.5; k += ns
        for b in range(ns // 2):
            if kind == "fermi":
                # band-pass start: oscillating memory near the step frequency
                w0 = math.sqrt(kw["mu"])
                th[k] = math.log(rng.uniform(0.05, 0.5) * w0)
                th[k + 1] = w0 * rng.uniform(0.7, 1.4)
            else:
                th[k] = rng.uniform(math.log(math.sqrt(lam_lo)), math.log(math.sqrt(lam_hi)))
                th[k + 1] = rng.uniform(0, 2 * math.sqrt(lam_hi))
            k += 2
        if ns % 2:
            th[k] = math.log(math.sqrt(lam_lo * lam_hi)); k += 1
        d = ns + 1
        for i in range(d):
            for j in range(i + 1):
                th[k] = rng.normal(0, 0.3) if i == j else rng.normal(0, 0.5)
                k += 1
        try:
            res = scipy.optimize.least_squares(residuals, th,
                                               args=(ns, lam, f_lam, delta, w_max, w_tau, None, h_fit, form),
                                               method="trf", max_nfev=max_nfev, x_scale="jac")
        except Exception:
            continue
        cost = float(np.sum(res.fun ** 2))
        if best is None or cost < best[0]:
            best = (cost, res.x)
        print(f"  start {s}: cost {cost:.4e}", flush=True)
    Ap, Cp = unpack(best[1], ns)
    check_gle(Ap, Cp)
    return Ap, Cp, lam, f


def report(kind, Ap, Cp, lam_lo, lam_hi, f, h, h_fit=None, form="q", **kw):
    lam = np.geomspace(lam_lo, lam_hi, 400)
    g = g0(lam, Ap, Cp) if form == "q" else g0_p(lam, Ap, Cp)
    fl = f(lam)
    T, S = propagator(Ap, Cp, h)
    g_h = gh(lam, Ap, Cp, h, T, S) if form == "q" else gh_p(lam, Ap, Cp, h, T, S)
    out = {"form": form}
    if h_fit is not None:  # fitted at a time step: the integrated response is what counts
        gfit = response(Ap, Cp, lam, h_fit, form)
        out["h_fit"] = h_fit
        out["max_rel_err_gh_at_h_fit"] = float(np.max(np.abs(gfit / fl - 1.0)))
        out["max_rel_err_g0"] = float(np.max(np.abs(g / fl - 1.0)))
    if kind == "fermi_gap":
        free = np.isnan(fl)
        out["max_abs_err_outside_gap"] = float(np.max(np.abs(g - np.nan_to_num(fl))[~free]))
        out["max_abs_err_outside_gap_gh"] = float(np.max(np.abs(g_h - np.nan_to_num(fl))[~free]))
        out["response_range_in_gap"] = [float(np.min(g[free])), float(np.max(g[free]))] if np.any(free) else None
    elif kind == "fermi" or kw.get("delta") is not None:
        fmax = float(np.max(fl))
        live = fl >= kw.get("delta", 1e-3) * fmax
        out["max_abs_err_rel_to_max"] = float(np.max(np.abs(g - fl)[live]) / fmax)
        if kind == "fermi":
            away = np.abs(lam - kw["mu"]) > 5.0 / kw["beta"]
            out["max_abs_err_rel_to_max_outside_step"] = float(np.max(np.abs(g - fl)[away]) / fmax)
        else:   # an exponential tail: relative error where f is within two decades of its maximum
            top = fl >= 1e-2 * fmax
            out["max_rel_err_top_two_decades"] = float(np.max(np.abs(g / fl - 1.0)[top]))
        out["max_tail_over_delta"] = float(np.max(g[~live]) / (kw.get("delta", 1e-3) * np.max(g))) if np.any(~live) else 0.0
    else:
        out["max_rel_err"] = float(np.max(np.abs(g / fl - 1.0)))
        out["rms_log_err"] = float(np.sqrt(np.mean(np.log(g / fl) ** 2)))
    out["max_rel_dt_err_gh_vs_g0"] = float(np.max(np.abs(g_h / g - 1.0)))
    out["max_tau_slowest"] = float(np.max(tau_slowest(lam, Ap)))
    out["dt_used_for_report"] = h
    return out


def write(path, name, kind, ns, Ap, Cp, lam_lo, lam_hi, rep, form="q", **kw):
    d = {
        "name": name,
        "ns": ns,
        "A_p": Ap.ravel().tolist(),
        "C_p": Cp.ravel().tolist(),
        "target": dict(kind=kind, **kw),
        "form": form,
        "estimator": ("<q_i q_j>: the fit targets the stationary <q^2>(omega) = f(omega^2)" if form == "q" else
                      "<p_i p_j> (Eq. 7): the fit targets the stationary <p^2>(omega) = f(omega^2)"),
        "window_lambda": [lam_lo, lam_hi],
        "fitted_time_step": rep.get("h_fit"),   # null: fitted in continuous time (g0)
        "fit_report": rep,
        "written_by": "oracle/fit_gle.py",
    }
    with open(path, "w") as fh:
        json.dump(d, fh, indent=1)


def main():
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out_dir = os.path.join(here, "fth_inputs", "gle")
    os.makedirs(out_dir, exist_ok=True)
    lap = (0.1, 12.1)                   # spectrum of the 64^3 periodic Laplacian + 0.1
    # name, target, ns, target parameters, window, fit settings (those that produced the files)
    fermi_opts = dict(starts=12, seed=10, w_tau=0.1, max_nfev=300)
    smooth_opts = dict(starts=8, seed=0, w_tau=0.005, max_nfev=4000)
    h5 = 0.5 / math.sqrt(lap[1])        # five times the standard step of the Laplacian window
    jobs = [
        ("invsqrt_ns4", "invsqrt", 4, {}, lap, smooth_opts),
        # fitted for the integrated step at h5: g_h(h5) follows f, the time-step error is corrected
        ("invsqrt_ns4_h05", "invsqrt", 4, {}, lap, dict(smooth_opts, h_fit=h5)),
        ("fermi_b20_ns4", "fermi", 4, {"beta": 20.0, "mu": 6.1, "delta": 1e-2}, lap, fermi_opts),
        ("fermi_b5_ns4", "fermi", 4, {"beta": 5.0, "mu": 6.1, "delta": 1e-2}, lap, fermi_opts),
        # ln on a window well above 1 (relative errors of ln blow up near x = 1) and of ratio 4,
        # like the paper's lattice spectra (ratio ~2): a stationary <q^2> decays as 1/omega^2
        # above the thermostat's reach, so a rising ln can only be followed over a short
        # window.  A spectrum [e_lo, e_hi] with e_hi / e_lo <= 4 maps into it with M' = r M
        # (the undo is ln M = ln M' - ln r)
        ("ln_ns4", "ln", 4, {}, (10.0, 40.0), dict(smooth_opts, w_tau=0.05)),
        # exp(-x): a Gershgorin interval of width <= 6 maps into it with M' = M + m I
        ("expneg_ns4", "expneg", 4, {}, (0.1, 6.1), smooth_opts),
    ]
    # The paper's own standard (Sec. I fitting paragraph, Sec. II examples): the momentum form
    # <p^2>(omega) = f(omega^2) of Eq. 7, ln over omega in [e, 100 e], exp(-x) down to about 1e-4,
    # 4 to 10 extra momenta.  The momentum response can rise with omega (a position response
    # decays as 1/omega^2 above the thermostat's reach), so ln follows over four decades of lambda.
    e2 = math.e ** 2
    p_opts = dict(starts=3, seed=1, w_tau=0.001, max_nfev=3000, npts=60, form="p")
    for ns in (4, 6, 8, 10):
        jobs.append((f"ln_p_ns{ns}", "ln", ns, {}, (e2, 1e4 * e2), p_opts))
        jobs.append((f"expneg_p_ns{ns}", "expneg", ns, {"delta": 1e-4}, (0.1, 9.3), p_opts))
        # zero-temperature Fermi occupation for an insulator (Sec. II, Fermi function paragraph): the
        # Laplacian window with a gap of 2.4 (a fifth of the band, like a wide-gap crystal) around mu = 6.1
        jobs.append((f"fermi_gap_p_ns{ns}", "fermi_gap", ns, {"mu": 6.1, "gap": 2.4}, lap,
                     dict(p_opts, starts=3, w_tau=0.003)))
    only = sys.argv[1:]
    for name, kind, ns, kw, (lam_lo, lam_hi), opts in jobs:
        if only and name not in only:
            continue
        h = opts.get("h_fit") or 0.1 / math.sqrt(lam_hi)
        t0 = time.time()
        print(f"fitting {name}", flush=True)
        Ap, Cp, _, f = fit(kind, ns, lam_lo, lam_hi, **opts, **kw)
        rep = report(kind, Ap, Cp, lam_lo, lam_hi, f, h, h_fit=opts.get("h_fit"), form=opts.get("form", "q"), **kw)
        print(f"  {name}: {rep}  ({time.time() - t0:.1f}s)", flush=True)
        write(os.path.join(out_dir, name + ".json"), name, kind, ns, Ap, Cp, lam_lo, lam_hi, rep,
              form=opts.get("form", "q"), **kw)


if __name__ == "__main__":
    main()
