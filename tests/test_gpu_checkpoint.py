"""Checkpoint and resume (fth_save / fth_load), the caller's allocator and
the footprint model.

The noise is counter-based, so (q, p, s, accumulators, step counter) is the
complete state of a solve: a run saved at step k and resumed in a fresh
context must continue bit for bit like the uninterrupted run, for every step
form.  Device memory can come from PyTorch's caching allocator without
changing any result; the footprint the library predicts for admission
matches what a context really holds.
"""
import numpy as np
import pytest

import fth_inputs as fi
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu


def cases():
    g = fi.load_gle("invsqrt_ns4")
    lap = fi.laplacian3d_csr(10, 0.1)
    band = fi.banded_spd_csr(20011, 5)
    dense, lam = fi.haar_spd(600, 3, 1.0, 50.0)
    small, lam_s = fi.haar_spd(80, 4, 1.0, 50.0)
    few, lam_f = fi.haar_spd(1100, 6, 1.0, 50.0)
    return [
        ("coded", lap, g, fi.dt_rule(fi.laplacian3d_lambda_max(10, 0.1)),
         dict(replicas=8, acc_pp=True, acc_trace=True)),
        ("blocked", band, fi.load_gle("fermi_b20_ns4"), fi.dt_rule(fi.gershgorin_max(band)),
         dict(replicas=32, temporal_steps=5, acc_pp=True)),
        ("dense", dense.astype(np.float32), g, fi.dt_rule(lam.max()),
         dict(replicas=32, precision=fth.FTH_FP32_BF16X3, acc_trace=True)),
        ("small", small, fi.GLE(4, 3.0 * g.A_p, 3.0 * g.C_p), fi.dt_rule(lam_s.max()),
         dict(replicas=16, precision=fth.FTH_FP64, acc_pp=True, acc_trace=True)),
        ("dense-few", few, fi.GLE(4, 3.0 * g.A_p, 3.0 * g.C_p), fi.dt_rule(lam_f.max()),
         dict(replicas=8, precision=fth.FTH_FP64, acc_pp=True, acc_trace=True)),
    ]


@pytest.mark.parametrize("case", cases(), ids=lambda c: c[0])
def test_save_and_resume_bit_identical(case):
    name, M, g, h, kw = case
    n = M.shape[0] if isinstance(M, np.ndarray) else M.n
    common = dict(pairs=fi.random_pairs(n, 32, 9), seed=17, stream_id=3, burn_in=5, block_len=7, acc_diag=True,
                  steps_per_graph=10, **kw)
    ref = fth.Solver(M, g.A_p, g.C_p, h, **common).run(37).run(50)
    a = fth.Solver(M, g.A_p, g.C_p, h, **common).run(37)
    image = a.save()
    a.close()
    b = fth.Solver(M, g.A_p, g.C_p, h, **common).load(image).run(50)
    print(f"[checkpoint] {name}: image {len(image)} bytes, {b.kernel_name}", flush=True)
    for x, y in zip(ref.state(), b.state()):
        assert np.array_equal(x, y)
    for x, y in zip(ref.accumulators(), b.accumulators()):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    e1, s1, n1 = ref.read()
    e2, s2, n2 = b.read()
    assert np.array_equal(e1, e2) and np.array_equal(s1, s2) and n1 == n2


def test_load_rejects_other_streams_and_damage():
    g = fi.load_gle("invsqrt_ns4")
    M = fi.banded_spd_csr(3000, 2)
    h = fi.dt_rule(fi.gershgorin_max(M))
    a = fth.Solver(M, g.A_p, g.C_p, h, replicas=8, seed=1).run(10)
    image = a.save()
    with pytest.raises(fth.FthError) as e:
        fth.Solver(M, g.A_p, g.C_p, h, replicas=8, seed=2).load(image)
    assert e.value.status == fth.FTH_EINVAL
    with pytest.raises(fth.FthError) as e:
        fth.Solver(M, g.A_p, g.C_p, h, replicas=16, seed=1).load(image)
    assert e.value.status in (fth.FTH_EINVAL, fth.FTH_ESTATE)
    bad = bytearray(image)
    bad[len(bad) // 2] ^= 0xFF
    with pytest.raises(fth.FthError) as e:
        fth.Solver(M, g.A_p, g.C_p, h, replicas=8, seed=1).load(bytes(bad))
    assert e.value.status == fth.FTH_EINVAL


def test_load_rejects_other_parameters():
    """The image records every parameter a continuation depends on: block
    length, burn-in, time step, GLE, accumulators, matrix values and pairs.
    A context that differs in any of them rejects it (the estimates would
    otherwise be formed from blocks of another length, or the trajectory
    would continue under other dynamics)."""
    g = fi.load_gle("invsqrt_ns4")
    g2 = fi.load_gle("fermi_b20_ns4")
    M = fi.banded_spd_csr(3000, 2)
    h = fi.dt_rule(fi.gershgorin_max(M))
    pairs = fi.random_pairs(M.n, 8, 3)
    base = dict(replicas=8, seed=1, pairs=pairs, block_len=10, acc_diag=True)
    image = fth.Solver(M, g.A_p, g.C_p, h, **base).run(25).save()
    fth.Solver(M, g.A_p, g.C_p, h, **base).load(image).close()   # same parameters: accepted
    M2 = fi.CSR(M.n, M.row_ptr, M.col, M.val * np.float32(1.0001))
    variants = [
        ((M, g.A_p, g.C_p, h), dict(base, block_len=20)),
        ((M, g.A_p, g.C_p, h), dict(base, burn_in=5)),
        ((M, g.A_p, g.C_p, 0.9 * h), base),
        ((M, g2.A_p, g2.C_p, h), base),
        ((M, g.A_p, g.C_p, h), dict(base, acc_pp=True, acc_diag=False)),
        ((M2, g.A_p, g.C_p, h), base),
        ((M, g.A_p, g.C_p, h), dict(base, pairs=pairs[::-1].copy())),
    ]
    for args, kw in variants:
        s = fth.Solver(*args, **kw)
        with pytest.raises(fth.FthError) as e:
            s.load(image)
        assert e.value.status == fth.FTH_EINVAL, kw
        s.close()


def test_footprint_matches_held_memory():
    g = fi.load_gle("invsqrt_ns4")
    M = fi.banded_spd_csr(50000, 6)
    h = fi.dt_rule(fi.gershgorin_max(M))
    pairs = fi.random_pairs(M.n, 100, 1)
    kw = dict(pairs=pairs, replicas=16, seed=4, acc_diag=True, coded_matrix=-1, temporal_steps=-1)
    plain = fth.Solver(M, g.A_p, g.C_p, h, **kw).run(30)
    fp = fth.fth_footprint_bytes(M, 4, 16, len(pairs), True, fth.FTH_FP32)
    held = plain.device_bytes
    print(f"[footprint] predicted {fp} bytes, held {held} bytes", flush=True)
    assert abs(fp - held) <= 1024
    # the few-replica dense form (matrix-vector force)
    D = fi.dense_ggt(5001, 7)
    dpairs = fi.random_pairs(5001, 64, 2)
    few = fth.Solver(D, g.A_p, g.C_p, fi.dt_rule(fi.power_lambda_max(D.astype(np.float64))), pairs=dpairs, replicas=4,
                     precision=fth.FTH_FP32, seed=4, acc_diag=True).run(3)
    fp = fth.fth_footprint_bytes(D, 4, 4, len(dpairs), True, fth.FTH_FP32)
    held = few.device_bytes
    print(f"[footprint] dense 5001, R = 4: predicted {fp} bytes, held {held} bytes ({few.kernel_name})", flush=True)
    assert "dense_gemv_kernel" in few.kernel_name
    assert abs(fp - held) <= 4096


# PyTorch brings its own HIP runtime; it must be initialised before the
# library is loaded in a process, so this part runs in a child process.
TORCH_CHILD = r"""
import sys, numpy as np, torch
torch.cuda.init()
sys.path.insert(0, sys.argv[1])
import fth_inputs as fi
from paper_1402_2095_amd import fth
g = fi.load_gle("invsqrt_ns4")
M = fi.banded_spd_csr(50000, 6)
h = fi.dt_rule(fi.gershgorin_max(M))
kw = dict(pairs=fi.random_pairs(M.n, 100, 1), replicas=16, seed=4, acc_diag=True)
plain = fth.Solver(M, g.A_p, g.C_p, h, **kw).run(30)
torch.cuda.synchronize()
before = torch.cuda.memory_allocated()
alloc = fth.torch_allocator()
t = fth.Solver(M, g.A_p, g.C_p, h, allocator=alloc, **kw).run(30)
during = torch.cuda.memory_allocated()
assert during - before >= t.device_bytes > 0, (before, during, t.device_bytes)
for x, y in zip(plain.state(), t.state()):
    assert np.array_equal(x, y)
for x, y in zip(plain.accumulators()[:3], t.accumulators()[:3]):
    assert np.array_equal(x, y)
t.close()
torch.cuda.synchronize()
assert torch.cuda.memory_allocated() == before
print("torch allocator: identical results,", during - before, "bytes from the caching allocator", flush=True)
"""


def test_torch_caching_allocator():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", TORCH_CHILD, root], capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
