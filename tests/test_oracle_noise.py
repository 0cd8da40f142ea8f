"""Pins of the oracle's noise: Philox4x32-10 against an independent library
implementation (rocRAND's host-callable engine), the uniform mapping, and the
distribution of the Box-Muller normals."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND pin")
    out = str(tmp_path_factory.mktemp("pin") / "philox_pin")
    src = os.path.join(HERE, "golden", "philox_rocrand_pin.cpp")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", out],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out


def test_philox_matches_rocrand(orc, rocrand_pin):
    rng = np.random.default_rng(11)
    count = 3000
    ctr = rng.integers(0, 2 ** 32, size=(count, 4), dtype=np.uint64)
    ctr[:, 1] %= 2 ** 30  # the pin maps c1:c0 to an offset of 4*(c1:c0) < 2^64
    ctr[:8] = [[0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1],
               [2 ** 32 - 1, 2 ** 30 - 1, 2 ** 32 - 1, 2 ** 32 - 1], [7, 9, 65536 * 3 + 5, 42], [5, 5, 5, 5]]
    keys = [(0, 0), (0xDEADBEEF, 0x12345678), (2 ** 32 - 1, 2 ** 32 - 1)]
    for k0, k1 in keys:
        lines = "\n".join(f"{a} {b} {c} {d} {k0} {k1}" for a, b, c, d in ctr) + "\n"
        res = subprocess.run([rocrand_pin], input=lines, capture_output=True, text=True, check=True)
        ref = np.array([list(map(int, l.split())) for l in res.stdout.strip().splitlines()], dtype=np.uint64)
        got = orc.philox4x32_10(ctr.astype(np.uint32), [k0, k1]).astype(np.uint64)
        assert ref.shape == got.shape
        assert np.array_equal(ref, got)


def test_uniform_mapping_endpoints_and_exactness(orc):
    assert orc.u01(0) == 2.0 ** -24
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert orc.u01(0x1FF) == 2.0 ** -24          # low 9 bits are dropped
    assert orc.u01(0x200) == 3.0 * 2.0 ** -24
    rng = np.random.default_rng(3)
    for x in rng.integers(0, 2 ** 32, size=2000):
        u = orc.u01(int(x))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u        # exact in FP32 as well as FP64


def test_normals_distribution(orc):
    n = 1 << 20
    rng = np.random.default_rng(5)
    i = rng.integers(0, 1 << 31, size=n)
    r = rng.integers(0, 1 << 12, size=n)
    st = rng.integers(0, 1 << 31, size=n)
    j = rng.integers(0, 8, size=n)
    z = orc.normals(1234, 7, i, r, st, j)
    se = 1.0 / np.sqrt(n)
    assert abs(z.mean()) < 5 * se
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0) * se
    kurt = np.mean(z ** 4) / np.mean(z ** 2) ** 2
    assert abs(kurt - 3.0) < 5 * np.sqrt(24.0) * se
    assert np.max(np.abs(z)) <= np.sqrt(-2.0 * np.log(2.0 ** -24)) + 1e-12
    assert scipy.stats.kstest(z[:200000], "norm").pvalue > 1e-4


def test_normals_uncorrelated_across_counter_fields(orc):
    """Neighbouring values of each counter field, and the two members of a
    Box-Muller pair, must be uncorrelated."""
    n = 200000
    rng = np.random.default_rng(9)
    i = rng.integers(0, 1 << 20, size=n)
    r = 4 * rng.integers(0, 1 << 10, size=n)
    st = rng.integers(0, 1 << 20, size=n)
    j = rng.integers(0, 6, size=n)
    base = orc.normals(99, 3, i, r, st, j)
    variants = {
        "pair partner": orc.normals(99, 3, i, r + 1, st, j),
        "other pair": orc.normals(99, 3, i, r + 2, st, j),
        "next quad": orc.normals(99, 3, i, r + 4, st, j),
        "next dof": orc.normals(99, 3, i + 1, r, st, j),
        "next step": orc.normals(99, 3, i, r, st + 1, j),
        "next component": orc.normals(99, 3, i, r, st, j + 1),
        "other stream": orc.normals(99, 4, i, r, st, j),
        "other seed": orc.normals(100, 3, i, r, st, j),
    }
    for name, v in variants.items():
        c = np.corrcoef(base, v)[0, 1]
        assert abs(c) < 5.0 / np.sqrt(n), name
        assert not np.array_equal(base, v), name
    # a Box-Muller pair is also independent in its squares (radius shared)
    c2 = np.corrcoef(base ** 2, variants["pair partner"] ** 2)[0, 1]
    assert abs(c2) < 5.0 / np.sqrt(n)
