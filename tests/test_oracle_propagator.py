"""Pins of the oracle's exact Ornstein-Uhlenbeck propagator (T, S) and of
the GLE validity checks (the Markovian GLE and its A_p, B_p, C_p relation,
Sec. I)."""
import math

import numpy as np
import pytest

import oracle


def random_gle(ns, seed):
    """A valid GLE: skew coupling + positive diagonal drift, C_p from a
    random SPD matrix scaled until B B^T is PSD is awkward, so instead take
    C_p = c I, for which A_p C_p + C_p A_p^T = 2c sym(A_p) is PSD."""
    rng = np.random.default_rng(seed)
    d = ns + 1
    K = rng.normal(size=(d, d))
    A = (K - K.T) + np.diag(rng.uniform(0.2, 2.0, d))
    C = 1.3 * np.eye(d)
    return A, C


def test_white_noise_closed_form():
    gamma, kT, h = 0.7, 1.9, 0.13
    T, S = oracle.propagator(np.array([[gamma]]), np.array([[kT]]), h)
    assert T.shape == (1, 1) and S.shape == (1, 1)
    assert T[0, 0] == pytest.approx(math.exp(-gamma * h), rel=1e-14)
    assert S[0, 0] == pytest.approx(math.sqrt(kT * (1.0 - math.exp(-2 * gamma * h))), rel=1e-13)


def test_rotation_block_closed_form():
    g, w, h, c = 0.4, 2.3, 0.21, 0.8
    A = np.array([[g, w], [-w, g]])
    T, S = oracle.propagator(A, c * np.eye(2), h)
    e = math.exp(-g * h)
    ref = e * np.array([[math.cos(w * h), -math.sin(w * h)], [math.sin(w * h), math.cos(w * h)]])
    assert np.allclose(T, ref, atol=1e-14)
    # C = cI is preserved by a rotation, so Sigma = c (1 - e^{-2gh}) I
    assert np.allclose(S, math.sqrt(c * (1 - e * e)) * np.eye(2), atol=1e-13)


@pytest.mark.parametrize("ns", [1, 2, 4, 7])
def test_semigroup_and_stationarity(ns):
    A, C = random_gle(ns, 100 + ns)
    T1, S1 = oracle.propagator(A, C, 0.05)
    T2, _ = oracle.propagator(A, C, 0.08)
    T3, _ = oracle.propagator(A, C, 0.13)
    assert np.allclose(T1 @ T2, T3, atol=1e-13)
    # S lower triangular with positive diagonal; C is stationary under one step
    assert np.allclose(np.triu(S1, 1), 0.0)
    assert np.all(np.diag(S1) > 0)
    assert np.allclose(T1 @ C @ T1.T + S1 @ S1.T, C, atol=1e-13)
    # small-h limit: S S^T / h -> B B^T
    _, Ss = oracle.propagator(A, C, 1e-6)
    assert np.allclose(Ss @ Ss.T / 1e-6, oracle.diffusion(A, C), rtol=1e-4, atol=1e-5)


def test_fitted_files_are_valid_gles():
    import fth_inputs
    import glob
    files = glob.glob(fth_inputs.GLE_DIR + "/*.json")
    if not files:
        pytest.skip("no fitted GLE files yet")
    for f in files:
        g = fth_inputs.load_gle(f)
        oracle.check_gle(g.A_p, g.C_p)
        oracle.propagator(g.A_p, g.C_p, 0.03)


def test_rejects_invalid_gles():
    with pytest.raises(oracle.GLEError):
        oracle.check_gle(np.array([[-1.0]]), np.array([[1.0]]))           # unstable drift
    with pytest.raises(oracle.GLEError):
        oracle.check_gle(np.array([[1.0]]), np.array([[-1.0]]))           # C_p not PD
    with pytest.raises(oracle.GLEError):
        oracle.check_gle(np.eye(2), np.array([[1.0, 0.5], [0.2, 1.0]]))   # C_p asymmetric
    # stable drift but A C + C A^T indefinite
    A = np.array([[1.0, 10.0], [0.0, 1.0]])
    with pytest.raises(oracle.GLEError):
        oracle.check_gle(A, np.eye(2))
