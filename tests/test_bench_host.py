"""Host logic of the benchmark (CPU): the algorithmic byte model of a step,
the parsing of the library's kernel descriptions into the kernels of a timed
unit, and the committed rocprofv3 summaries it reads counters from.

The byte model is the roofline's numerator: per step the state q, p and
s_1..s_ns are read and written once, and the matrix is read once (CSR with
32-bit row pointers and column indices; dense M as bf16 hi + lo).  The
figures for the 64^3 Laplacian (120.6 MB) and the banded 1e6 system
(1.612 GB) are worked out here from the sizes, not from the function."""
import os
import types

import numpy as np
import pytest

import bench
import fth_inputs as fi
from paper_1402_2095_amd import fth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_step_bytes_laplacian_and_banded():
    # 64^3 Laplacian, R = 8, ns = 4, FP32: state 2 * 6 * 4 B * N R, CSR (N + 1) * 4 + nnz * 8,
    # FP64 diagonal block sums read and written (16 B per row)
    n, R = 64 ** 3, 8
    nnz = 7 * n
    expect = 2 * 6 * 4 * n * R + (n + 1) * 4 + nnz * 8 + 16 * n
    w = bench.workload("laplacian64")
    assert w["n"] == n and w["M"].nnz == nnz
    assert bench.step_bytes(w) == pytest.approx(expect, rel=1e-12)
    assert expect == pytest.approx(120.6e6, rel=1e-3)
    # banded 1e6, R = 32: 7 entries per row except at the two ends (open band)
    n, R = 10 ** 6, 32
    w = bench.workload("banded1e6")
    nnz = w["M"].nnz
    assert nnz == 7 * n - 12
    expect = 2 * 6 * 4 * n * R + (n + 1) * 4 + nnz * 8 + 16 * n
    assert bench.step_bytes(w) == pytest.approx(expect, rel=1e-12)
    assert expect == pytest.approx(1.612e9, rel=1e-3)


def test_step_bytes_dense():
    g = types.SimpleNamespace(ns=4)
    for prec, mb in ((fth.FTH_FP32_BF16X3, 4), (fth.FTH_FP64, 8)):
        rb = 8 if prec == fth.FTH_FP64 else 4
        w = dict(dense=True, prec=prec, n=16384, R=128, g=g, extra={}, M=np.zeros((1, 1)))
        expect = 2 * 6 * rb * 16384 * 128 + 16384 * 16384 * mb
        assert bench.step_bytes(w) == pytest.approx(expect, rel=1e-12)


@pytest.mark.parametrize("name,kind,kernels,unit", [
    ("tbp_step_kernel<float,NS=4,KT=5> block=1024 grid=256 (persistent; + csr_step_kernel block=256 tail)",
     "tbp", ["tbp_step_kernel<float, 4, 5,", "tb_pairs_kernel<float, 4, 5>"], 5),
    ("tb_step_kernel<float,NS=4,RPT=4,KT=3> block=512 (+ csr_step_kernel block=256 tail)",
     "tb", ["tb_step_kernel<float, 4, 4, 3,", "tb_pairs_kernel<float, 4, 3>"], 3),
    ("csr_step_kernel<float,NS=4,RPT=4,NT=0,CODED=1> block=128 (autotuned)",
     "csr", ["csr_step_kernel<float, 4, 4, false, true,"], 1),
    ("gemm_bf16x3_kernel<RT=8,ksplit=4> + dense_epilogue_kernel<float,NS=4,RPT=4,NT=0>",
     "dense", ["gemm_bf16x3_kernel<8>", "dense_epilogue_kernel<float, 4, 4, false,"], 1),
    ("dense_gemv_kernel<double,R=8> + dense_epilogue_kernel<double,NS=4,RPT=4,NT=1>",
     "gemv", ["dense_gemv_kernel<double, 8>", "dense_epilogue_kernel<double, 4, 4, true,"], 1),
    ("small_dense_kernel<double,NS=0,RPT=1> (persistent, M in LDS)", None, [], 1),
])
def test_unit_of_kernel_descriptions(name, kind, kernels, unit):
    assert bench.unit_of(name) == (kind, kernels, unit)


def test_committed_profiles_are_complete():
    d = os.path.join(ROOT, "profiles")
    files = [f for f in sorted(os.listdir(d)) if f.endswith(".txt") and not f.endswith("_stalls.txt")]
    assert len(files) >= 4
    for f in files:
        fields = {}
        with open(os.path.join(d, f)) as fh:
            head = fh.readline()
            for line in fh:
                if ": " in line and not line.startswith(" "):
                    k, v = line.rstrip("\n").split(": ", 1)
                    fields[k] = v
        assert head.startswith("rocprofv3 summary: "), f
        kind, names, _ = bench.unit_of(head[len("rocprofv3 summary: "):])
        assert kind in bench.KERNEL_SOURCES, f
        assert fields["unit_kernels"] == " + ".join(names), f
        assert len(fields["source_sha256"]) == 64, f
        assert float(fields["traffic_bytes_per_unit"]) > 0, f
        assert "rocprofv3 --kernel-trace --stats" in open(os.path.join(d, f)).read(), f
