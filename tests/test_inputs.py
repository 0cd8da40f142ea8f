"""Properties of the seeded synthetic inputs."""
import numpy as np
import pytest

import fth_inputs as fi


def test_laplacian_structure_and_spectrum():
    for n in (3, 4, 6):
        csr = fi.laplacian3d_csr(n, 0.1, dtype=np.float64)
        M = csr.to_dense()
        assert csr.nnz == 7 * n ** 3
        assert np.allclose(M, M.T)
        assert np.allclose(M.sum(axis=1), 0.1)
        ev = np.linalg.eigvalsh(M)
        assert ev.min() == pytest.approx(0.1, abs=1e-10)
        assert ev.max() == pytest.approx(fi.laplacian3d_lambda_max(n, 0.1), abs=1e-10)
        assert ev.max() <= 12.1 + 1e-12
    assert fi.laplacian3d_lambda_max(64, 0.1) == pytest.approx(12.1)
    # index convention: x slowest, z fastest
    assert fi.lattice_index(1, 2, 3, 64) == (1 * 64 + 2) * 64 + 3


def test_laplacian_tiny_grid_merges_duplicates():
    csr = fi.laplacian3d_csr(2, 0.1, dtype=np.float64)
    M = csr.to_dense()
    assert np.allclose(M.sum(axis=1), 0.1)
    assert np.all(np.diff(csr.row_ptr) == 4)


def test_banded_spd():
    csr = fi.banded_spd_csr(500, 3)
    M = csr.to_dense()
    assert np.allclose(M, M.T)
    counts = np.diff(csr.row_ptr)
    assert counts.max() == 7 and counts.min() == 4
    off = M - np.diag(np.diag(M))
    assert np.all(off <= 0) and np.all(off >= -1)
    assert np.all(np.diag(M) - np.abs(off).sum(axis=1) >= 0.05 - 1e-6)
    ev = np.linalg.eigvalsh(M)
    assert ev.min() >= 0.05 - 1e-6
    assert ev.max() <= fi.gershgorin_max(csr) + 1e-9 <= 13.0 + 1e-6
    for r in range(500):
        cols = csr.col[csr.row_ptr[r]:csr.row_ptr[r + 1]]
        assert np.all(np.diff(cols) > 0)


def test_dense_ggt_and_haar():
    M = fi.dense_ggt(200, 4004)
    assert M.dtype == np.float32
    assert np.allclose(M, M.T)
    ev = np.linalg.eigvalsh(M.astype(np.float64))
    assert ev.min() > 0.09 and ev.max() < 4.5
    assert fi.power_lambda_max(M.astype(np.float64)) >= ev.max()
    m, lam = fi.haar_spd(30, 1001)
    assert np.allclose(np.sort(np.linalg.eigvalsh(m)), np.sort(lam), rtol=1e-10)
    assert lam.min() >= 1.0 and lam.max() <= 100.0


def test_m2_spectrum_inside_interval():
    """Appendix: the M2 construction keeps every Gerschgorin disc, hence the
    spectrum, inside (a, b)."""
    M = fi.m2_gerschgorin(120, 7, -300.0, 300.0)
    ev = np.linalg.eigvalsh(M)
    assert np.allclose(M, M.T)
    assert ev.min() > -300 and ev.max() < 300
    assert np.count_nonzero(M) > 0.9 * 120 * 120


def test_m1_lattice_neighbour_shells():
    """Appendix: cubic periodic lattice with hopping up to the 6th neighbour
    shell; squared distances 1..6 hold 6+12+8+6+24+24 = 80 sites."""
    csr = fi.m1_lattice_csr(8, 1)
    counts = np.diff(csr.row_ptr)
    assert np.all(counts == 81)
    M = csr.to_dense()
    assert np.allclose(M, M.T)
    assert np.allclose(np.diag(M), 100.0)
    assert np.linalg.eigvalsh(M).min() > 0


def test_pairs():
    p = fi.random_pairs(1000, 1024, 2002)
    assert p.shape == (1024, 2) and p.dtype == np.int32
    assert np.all(p[:, 0] != p[:, 1]) and p.min() >= 0 and p.max() < 1000
    assert np.array_equal(fi.row_pairs(5)[:, 1], [1, 2, 3, 4])


def test_serving_mix_shape():
    reqs = fi.serving_mix(400, 2.0, 5005)
    kinds = [r.kind for r in reqs]
    assert 0.2 < kinds.count("dense") / 400 < 0.4
    assert all(np.diff([r.arrival for r in reqs]) > 0)
    for r in reqs:
        if r.kind == "dense":
            assert 512 <= r.n <= 8192
