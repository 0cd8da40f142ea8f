"""Exact stationary responses of the GLE-thermostatted harmonic system.

TEST INFRASTRUCTURE ONLY (part of the oracle).

The paper's Sec. I argues that, because the GLE is linear with Gaussian
noise and is applied identically to every Cartesian degree of freedom, each
normal mode of M (eigenvalue lambda = omega^2) responds as an independent 1-D
GLE oscillator.  Hence any stationary second moment of the dynamical
variables is U g(Lambda) U^T (the covariance identity of Sec. I), with g the
1-D response.  This module computes g in two forms:

* g0(lambda): continuous-time stationary <q^2>(omega) of the Markovian SDE of
  Sec. I with V = omega^2 q^2 / 2, from the Lyapunov equation
      Acal X + X Acal^T = blkdiag(0, B_p B_p^T),
      Acal = [[0, -1, 0], [omega^2, a_pp, a_p^T], [0, abar_p, A]].
  This is the curve the GLE fit targets.
* g_h(lambda): the exact stationary <q^2> of the discrete step actually
  integrated (kick, exact OU step, kick, drift), from the discrete Lyapunov
  equation X = G X G^T + W W^T for the per-mode one-step map.  Statistical
  parity of time averages is against g_h(M); g_h - g0 is the time-step
  error and g0 - f the fit error (the error budget of Sec. I).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import diffusion, propagator


def _as_arr(x):
    return np.atleast_1d(np.asarray(x, dtype=np.float64))


def g0_cov(lam: float, A_p: np.ndarray, C_p: np.ndarray) -> np.ndarray:
    """Full stationary covariance of (q, p, s) for one mode, continuous time."""
    d = A_p.shape[0]
    acal = np.zeros((d + 1, d + 1))
    acal[0, 1] = -1.0
    acal[1, 0] = lam
    acal[1:, 1:] = A_p
    D = np.zeros((d + 1, d + 1))
    D[1:, 1:] = diffusion(A_p, C_p)
    # solve_continuous_lyapunov solves a X + X a^H = q
    X = scipy.linalg.solve_continuous_lyapunov(-acal, -D)
    return 0.5 * (X + X.T)


def g0_cov_batch(lam, A_p: np.ndarray, C_p: np.ndarray) -> np.ndarray:
    """Stationary covariances for many modes at once: the Lyapunov equation
    written as (I kron Acal + Acal kron I) vec X = vec D and solved densely
    per mode.  Returns [len(lam), d+1, d+1]."""
    lam = _as_arr(lam)
    d = A_p.shape[0]
    n = d + 1
    acal = np.zeros((len(lam), n, n))
    acal[:, 0, 1] = -1.0
    acal[:, 1, 0] = lam
    acal[:, 1:, 1:] = A_p
    D = np.zeros((n, n))
    D[1:, 1:] = diffusion(A_p, C_p)
    eye = np.eye(n)
    K = (np.einsum("ij,bkl->bikjl", eye, acal) + np.einsum("bij,kl->bikjl", acal, eye)).reshape(len(lam), n * n, n * n)
    X = np.linalg.solve(K, np.broadcast_to(D.reshape(n * n), (len(lam), n * n))[..., None])[..., 0]
    X = X.reshape(len(lam), n, n)
    return 0.5 * (X + np.swapaxes(X, 1, 2))


def g0(lam, A_p, C_p) -> np.ndarray:
    """Continuous-time stationary <q^2> at omega^2 = lam (vectorised)."""
    return g0_cov_batch(lam, np.asarray(A_p, dtype=np.float64), np.asarray(C_p, dtype=np.float64))[:, 0, 0]


def g0_p(lam, A_p, C_p) -> np.ndarray:
    """Continuous-time stationary <p^2> (the paper's T*(omega))."""
    return g0_cov_batch(lam, np.asarray(A_p, dtype=np.float64), np.asarray(C_p, dtype=np.float64))[:, 1, 1]


def tau_slowest(lam, A_p) -> np.ndarray:
    """1 / (smallest real part of the eigenvalues of Acal(omega)): the slowest
    relaxation time of a mode, a proxy for the correlation time that sets
    the statistical error (Sec. II, third fit requirement)."""
    lam = _as_arr(lam)
    d = A_p.shape[0]
    n = d + 1
    acal = np.zeros((len(lam), n, n))
    acal[:, 0, 1] = -1.0
    acal[:, 1, 0] = lam
    acal[:, 1:, 1:] = A_p
    ev = np.linalg.eigvals(acal)
    return 1.0 / np.min(ev.real, axis=1)


def step_map(lam: float, T: np.ndarray, S: np.ndarray, h: float):
    """One-step linear map x' = G x + W xi of a single mode, x = (q, p, s).

    Kick K_B: p <- p - (h/2) lam q;  OU: (p, s) <- T (p, s) + S xi;
    kick K_B again; drift K_A: q <- q + h p."""
    d = T.shape[0]
    n = d + 1
    KB = np.eye(n)
    KB[1, 0] = -0.5 * h * lam
    KA = np.eye(n)
    KA[0, 1] = h
    O = np.eye(n)
    O[1:, 1:] = T
    WO = np.zeros((n, d))
    WO[1:, :] = S
    G = KA @ KB @ O @ KB
    W = KA @ KB @ WO
    return G, W


def gh_cov(lam: float, T: np.ndarray, S: np.ndarray, h: float) -> np.ndarray:
    G, W = step_map(lam, T, S, h)
    X = scipy.linalg.solve_discrete_lyapunov(G, W @ W.T)
    return 0.5 * (X + X.T)


def gh(lam, A_p, C_p, h, T=None, S=None) -> np.ndarray:
    """Exact stationary <q^2> of the integrated discrete dynamics at
    omega^2 = lam (vectorised)."""
    if T is None or S is None:
        T, S = propagator(A_p, C_p, h)
    lam = _as_arr(lam)
    return np.array([gh_cov(float(l), T, S, h)[0, 0] for l in lam])


def gh_p(lam, A_p, C_p, h, T=None, S=None) -> np.ndarray:
    """Exact stationary <p^2> of the integrated discrete dynamics at the
    step boundary (p_n, the instant q_n is sampled), at omega^2 = lam: the
    response behind the momentum form of the estimator (Eq. 7)."""
    if T is None or S is None:
        T, S = propagator(A_p, C_p, h)
    lam = _as_arr(lam)
    return np.array([gh_cov(float(l), T, S, h)[1, 1] for l in lam])


def spectral_radius(lam: float, T: np.ndarray, S: np.ndarray, h: float) -> float:
    G, _ = step_map(lam, T, S, h)
    return float(np.max(np.abs(np.linalg.eigvals(G))))


def finite_cov(lam: float, T, S, h, nsteps: int, x0cov=None) -> np.ndarray:
    """Exact E[x_n x_n^T] after nsteps steps from a deterministic start with
    covariance x0cov (zeros: the all-zero initial state)."""
    G, W = step_map(lam, T, S, h)
    X = np.zeros((G.shape[0],) * 2) if x0cov is None else np.array(x0cov, dtype=np.float64)
    WW = W @ W.T
    for _ in range(nsteps):
        X = G @ X @ G.T + WW
    return X


def matrix_function(M: np.ndarray, g_of_lam) -> np.ndarray:
    """U g(Lambda) U^T for a symmetric M (the paper's Eq. 1 route)."""
    lam, U = np.linalg.eigh(np.asarray(M, dtype=np.float64))
    return (U * g_of_lam(lam)[None, :]) @ U.T


def gh_matrix(M, A_p, C_p, h) -> np.ndarray:
    T, S = propagator(A_p, C_p, h)
    return matrix_function(M, lambda lam: gh(lam, A_p, C_p, h, T, S))


def gh_p_matrix(M, A_p, C_p, h) -> np.ndarray:
    T, S = propagator(A_p, C_p, h)
    return matrix_function(M, lambda lam: gh_p(lam, A_p, C_p, h, T, S))


def g0_matrix(M, A_p, C_p) -> np.ndarray:
    return matrix_function(M, lambda lam: g0(lam, A_p, C_p))


def laplacian_eigs(n: int, sigma: float) -> np.ndarray:
    """lambda(k) = sigma + sum_d (2 - 2 cos(2 pi k_d / n)), shape (n, n, n)."""
    c = 2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n)
    return sigma + c[:, None, None] + c[None, :, None] + c[None, None, :]


def insulator_eigs(n: int, delta: float, hop: float, shift: float) -> np.ndarray:
    """Spectrum of the two-sublattice cubic lattice (on-site shift +/- delta
    by the parity of x + y + z, nearest-neighbour hopping -hop, periodic, n
    even), all N = n^3 values.  The staggered potential couples the Bloch
    waves k and k + (pi, pi, pi), whose hopping energies are -hop gamma_k and
    +hop gamma_k; each such pair is a 2 x 2 block [[-hop g, delta], [delta,
    hop g]] with eigenvalues +/- sqrt(delta^2 + hop^2 g^2).  Summed over the
    whole grid every pair is met twice, so the spectrum is shift +/- E_k over
    the grid, each sign taken once per pair: the multiset {shift - E_k} over
    half the grid and {shift + E_k} over the other half, which for sums is
    half of each over the whole grid."""
    c = 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n)
    gam = (c[:, None, None] + c[None, :, None] + c[None, None, :]).ravel()
    E = np.sqrt(delta * delta + hop * hop * gam * gam)
    # k and k + Q give the same E: keep the half of the grid with k_x < n/2 (one of each pair)
    kx = np.repeat(np.arange(n), n * n)
    Eh = E[kx < n // 2]
    return np.sort(np.concatenate([shift - Eh, shift + Eh]))


def insulator_sublattice_diagonal(n: int, delta: float, hop: float, shift: float, g_of_lam):
    """Diagonal of g(M) for the two-sublattice lattice, which takes one value
    on each sublattice (translation invariance within it): (even, odd) for
    sites with x + y + z even (on-site shift + delta) and odd.  In the basis
    of the two sublattice Bloch sums at k (one k per pair k, k + Q), M is
    [[shift + delta, -hop g], [-hop g, shift - delta]]; its eigenvector of
    shift + E puts weight (1 + delta / E) / 2 on the even sublattice and that
    of shift - E weight (1 - delta / E) / 2, so the even diagonal is the
    average over the N/2 values of k of those weights times g."""
    c = 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n)
    gam = (c[:, None, None] + c[None, :, None] + c[None, None, :])[: n // 2].ravel()
    E = np.sqrt(delta * delta + hop * hop * gam * gam)
    gp, gm = g_of_lam(shift + E), g_of_lam(shift - E)
    w = delta / E
    even = np.mean(0.5 * (1 + w) * gp + 0.5 * (1 - w) * gm)
    odd = np.mean(0.5 * (1 - w) * gp + 0.5 * (1 + w) * gm)
    return float(even), float(odd)


def laplacian_function(n: int, sigma: float, g_of_lam) -> np.ndarray:
    """g(M) for the periodic n^3 Laplacian + sigma, as the translation
    invariant kernel C(dx, dy, dz) = ifftn(g(lambda(k))) (the DFT diagonalises
    every circulant).  Element (i, j) is C[(xi-xj)%n, (yi-yj)%n, (zi-zj)%n]."""
    lam = laplacian_eigs(n, sigma)
    uniq, inv = np.unique(np.round(lam, 12), return_inverse=True)
    vals = g_of_lam(uniq)[inv].reshape(lam.shape)
    c = np.fft.ifftn(vals)
    return c.real


def laplacian_element(C: np.ndarray, i, j) -> np.ndarray:
    n = C.shape[0]
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    xi, ri = np.divmod(i, n * n)
    yi, zi = np.divmod(ri, n)
    xj, rj = np.divmod(j, n * n)
    yj, zj = np.divmod(rj, n)
    return C[(xi - xj) % n, (yi - yj) % n, (zi - zj) % n]


def lanczos_quadratic_form(matvec, n: int, u: np.ndarray, g_of_lam, iters: int = 200) -> float:
    """u^T g(M) u by Gauss quadrature on the Lanczos tridiagonalisation from
    u (Golub-Meurant), with full reorthogonalisation, FP64."""
    u = np.asarray(u, dtype=np.float64)
    nrm = np.linalg.norm(u)
    if nrm == 0:
        return 0.0
    V = np.zeros((iters + 1, n))
    V[0] = u / nrm
    alpha = np.zeros(iters)
    beta = np.zeros(iters)
    k_used = iters
    for k in range(iters):
        w = matvec(V[k])
        alpha[k] = V[k] @ w
        w = w - alpha[k] * V[k] - (beta[k - 1] * V[k - 1] if k > 0 else 0.0)
        w -= V[:k + 1].T @ (V[:k + 1] @ w)
        b = np.linalg.norm(w)
        if b < 1e-14:
            k_used = k + 1
            break
        beta[k] = b
        V[k + 1] = w / b
    a = alpha[:k_used]
    b = beta[:k_used - 1]
    theta, Y = scipy.linalg.eigh_tridiagonal(a, b)
    return float(nrm * nrm * np.sum(Y[0, :] ** 2 * g_of_lam(theta)))
