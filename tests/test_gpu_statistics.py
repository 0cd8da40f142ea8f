"""Statistical properties the paper states (Sec. II and the conclusions):

* the statistical error falls as the square root of the simulated time:
  four times the steps halve the standard error;
* the relative statistical error of an element does not depend on the size
  of the matrix (it is set by the correlation time of the mode, and every
  element is an average over the same dynamics): periodic Laplacians of
  different sizes give the same relative standard error of the diagonal at a
  fixed number of steps.
"""
import numpy as np
import pytest

import fth_inputs as fi
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu


def lap_solver(n_side, seed, **kw):
    M = fi.laplacian3d_csr(n_side, 0.1)
    g = fi.load_gle("invsqrt_ns4")
    h = fi.dt_rule(fi.laplacian3d_lambda_max(n_side, 0.1))
    return fth.Solver(M, g.A_p, g.C_p, h, replicas=8, seed=seed, burn_in=1000, block_len=1000, acc_diag=True, **kw)


def test_stderr_halves_with_four_times_the_steps():
    sol = lap_solver(16, 3)
    sol.run(1000 + 16000)
    _, se1, _ = sol.read()
    sol.run(3 * 16000)
    _, se4, _ = sol.read()
    ratio = float(np.median(se4 / se1))
    print(f"[stats] stderr(4t) / stderr(t) = {ratio:.3f}", flush=True)
    assert 0.4 < ratio < 0.6


def test_relative_stderr_independent_of_size():
    rel = {}
    for n_side in (12, 20, 32):
        sol = lap_solver(n_side, 5)
        sol.run(1000 + 20000)
        est, se, _ = sol.read()
        rel[n_side] = float(np.median(se / est))
        sol.close()
    print(f"[stats] median relative stderr of the diagonal by size: {rel}", flush=True)
    vals = np.array(list(rel.values()))
    assert vals.max() / vals.min() < 1.25
