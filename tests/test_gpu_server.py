"""GPU tests of the serving layer: continuous batching with the packed
multi-request kernel, admission by device footprint, stopping at a target
standard error, cancellation, spectral maps and the momentum estimator; and
a request's result is the same alone and in the mix (bit for bit: the packed
kernel runs the same per-row arithmetic, with the request's own noise stream
and step counter)."""
import numpy as np
import pytest

import fth_inputs as fi
from paper_1402_2095_amd import fth

pytestmark = pytest.mark.gpu


def request_pairs(n, seed, nd=16, no=16):
    rng = np.random.default_rng(seed)
    d = rng.choice(n, size=nd, replace=False)
    diag = np.stack([d, d], axis=1)
    a = rng.integers(0, nd, size=no)
    b = (a + 1 + rng.integers(0, nd - 1, size=no)) % nd
    off = np.stack([d[a], d[b]], axis=1)
    return np.concatenate([diag, off]).astype(np.int32)


def lap_request(n_side, seed, stream):
    M = fi.laplacian3d_csr(n_side, 0.1)
    g = fi.load_gle("invsqrt_ns4")
    h = fi.dt_rule(fi.laplacian3d_lambda_max(n_side, 0.1))
    return dict(M=M, A_p=g.A_p, C_p=g.C_p, dt=h, pairs=request_pairs(M.n, seed), seed=seed, stream_id=stream)


def band_request(n, seed, stream):
    M = fi.banded_spd_csr(n, seed)
    g = fi.load_gle("invsqrt_ns4")
    return dict(M=M, A_p=g.A_p, C_p=g.C_p, dt=fi.dt_rule(fi.gershgorin_max(M)), pairs=request_pairs(n, seed),
                seed=seed, stream_id=stream)


def dense_request(n, seed, stream):
    M = fi.dense_ggt(n, seed)
    g = fi.load_gle("invsqrt_ns4")
    return dict(M=M, A_p=g.A_p, C_p=g.C_p, dt=fi.dt_rule(fi.power_lambda_max(M.astype(np.float64))),
                pairs=request_pairs(n, seed), seed=seed, stream_id=stream, precision=fth.FTH_FP32_BF16X3)


def run_to_done(srv, ids, max_ticks=10000):
    for _ in range(max_ticks):
        if all(srv.poll(i)["state"] >= fth.FTH_REQ_DONE for i in ids):
            return
        srv.tick()
    raise AssertionError("requests did not finish")


def test_alone_and_in_mix_identical():
    x = lap_request(12, 7, 3)
    y = dense_request(600, 9, 4)
    common = dict(block_len=50, max_steps=1000, target=0.0)
    alone = fth.Server(steps_per_tick=100)
    ax = alone.submit(**x, **common)
    ay = alone.submit(**y, **common, replicas=64)
    run_to_done(alone, [ax, ay])
    ex_alone, sx_alone = alone.result(ax)
    ey_alone, sy_alone = alone.result(ay)
    assert alone.poll(ax)["packed"] == 1 and alone.poll(ay)["packed"] == 0

    mix = fth.Server(steps_per_tick=100)
    ids = [mix.submit(**band_request(5000, 11, 21), **common),
           mix.submit(**lap_request(10, 12, 22), **common)]
    mx = mix.submit(**x, **common)
    ids.append(mix.submit(**band_request(20000, 13, 23), **common))
    my = mix.submit(**y, **common, replicas=64)
    run_to_done(mix, ids + [mx, my])
    ex, sx = mix.result(mx)
    ey, sy = mix.result(my)
    assert np.array_equal(ex, ex_alone) and np.array_equal(sx, sx_alone)
    assert np.array_equal(ey, ey_alone) and np.array_equal(sy, sy_alone)
    assert mix.poll(mx)["steps"] == 1000

    # and equal to a standalone context with the same inputs (the per-request kernel)
    sol = fth.Solver(x["M"], x["A_p"], x["C_p"], x["dt"], pairs=x["pairs"], replicas=32, seed=7, stream_id=3,
                     block_len=50)
    sol.run(1000)
    est, se, _ = sol.read()
    assert np.array_equal(est, ex) and np.array_equal(se, sx)


def test_admission_by_footprint_and_order():
    a = band_request(40000, 31, 1)
    b = band_request(40000, 32, 2)
    fp = fth.fth_footprint_bytes(a["M"], 4, 32, len(a["pairs"]), False, fth.FTH_FP32)
    srv = fth.Server(hbm_budget=int(1.5 * fp), steps_per_tick=100)
    ia = srv.submit(**a, block_len=50, max_steps=500, target=0.0)
    ib = srv.submit(**b, block_len=50, max_steps=500, target=0.0)
    srv.tick()
    assert srv.poll(ia)["state"] == fth.FTH_REQ_RUNNING
    assert srv.poll(ib)["state"] == fth.FTH_REQ_QUEUED   # waits for memory
    q, r, reserved = srv.stats()
    assert (q, r) == (1, 1) and reserved == srv.poll(ia)["footprint"] <= int(1.5 * fp)
    run_to_done(srv, [ia, ib])
    pa, pb = srv.poll(ia), srv.poll(ib)
    assert pb["t_start"] >= pa["t_finish"] - 1e-9
    assert pa["state"] == pb["state"] == fth.FTH_REQ_DONE
    with pytest.raises(fth.FthError) as e:
        fth.Server(hbm_budget=fp // 2).submit(**a)
    assert e.value.status == fth.FTH_ENOMEM


def test_stops_at_target_stderr():
    x = lap_request(10, 41, 5)
    srv = fth.Server(steps_per_tick=200, min_blocks=8)
    rid = srv.submit(**x, block_len=100, burn_in=200, target=0.05, max_steps=400000)
    run_to_done(srv, [rid])
    info = srv.poll(rid)
    est, se = srv.result(rid)
    print(f"[serve] steps {info['steps']}, max rel stderr {info['max_rel_stderr']:.4f}", flush=True)
    assert info["state"] == fth.FTH_REQ_DONE
    assert info["max_rel_stderr"] <= 0.05 and info["steps"] < 400000
    assert np.all(np.isfinite(est[:16])) and np.all(est[:16] > 0)


def test_cancel_releases_memory():
    srv = fth.Server(steps_per_tick=50)
    rid = srv.submit(**band_request(30000, 51, 6), target=0.0, max_steps=10 ** 6)
    srv.tick()
    assert srv.stats()[2] > 0
    srv.cancel(rid)
    assert srv.poll(rid)["state"] == fth.FTH_REQ_CANCELLED
    assert srv.stats() == (0, 0, 0)
    srv.tick()  # an empty tick is fine


def normwise(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


def test_mix_against_oracle():
    """One server running sparse FP32 requests of uneven size (packed), a
    dense split-BF16x3 request, a dense request of 8 replicas (matrix-vector
    force) and a sparse FP64 request side by side for
    1000 steps: each request's estimates and block stderrs equal the FP64
    oracle's for the same inputs, seed and noise stream, to the FP32 (1e-4)
    or FP64 (1e-10) trajectory tolerance."""
    import oracle
    common = dict(block_len=50, max_steps=1000, target=0.0)
    reqs = [("band2000", band_request(2000, 61, 31), fth.FTH_FP32, 32),
            ("lap12", lap_request(12, 62, 32), fth.FTH_FP32, 32),
            ("band5003", band_request(5003, 63, 33), fth.FTH_FP32, 32),
            ("dense600", dense_request(600, 64, 34), fth.FTH_FP32_BF16X3, 64),
            ("dense1100-r8", dense_request(1100, 66, 36), fth.FTH_FP32_BF16X3, 8),   # matrix-vector form
            ("band3001-fp64", dict(band_request(3001, 65, 35), precision=fth.FTH_FP64), fth.FTH_FP64, 8)]
    srv = fth.Server(steps_per_tick=100)
    ids = []
    for name, kw, prec, R in reqs:
        kw = dict(kw)
        kw.pop("precision", None)
        ids.append(srv.submit(**kw, precision=prec, replicas=R, **common))
    run_to_done(srv, ids)
    for (name, kw, prec, R), rid in zip(reqs, ids):
        info = srv.poll(rid)
        assert info["state"] == fth.FTH_REQ_DONE and info["steps"] == 1000, (name, info)
        est, se = srv.result(rid)
        M = kw["M"]
        M64 = M.astype(np.float64) if isinstance(M, np.ndarray) else fi.CSR(M.n, M.row_ptr, M.col,
                                                                                M.val.astype(np.float64))
        orc = oracle.OracleRun(M64, kw["A_p"], kw["C_p"], kw["dt"], R, kw["pairs"], seed=kw["seed"],
                               stream=kw["stream_id"], block_len=50).run(1000)
        m_o, se_o = orc.estimates()
        tol = 1e-10 if prec == fth.FTH_FP64 else 1e-4
        e_est, e_se = normwise(est, m_o), normwise(se, se_o)
        print(f"  {name}: packed={info['packed']} est {e_est:.2e} stderr {e_se:.2e}", flush=True)
        assert e_est <= 10 * tol, name
        assert e_se <= (1e-6 if prec == fth.FTH_FP64 else 1e-2), name
        assert info["packed"] == (1 if prec == fth.FTH_FP32 else 0), name


def test_admission_does_not_wait_for_slow_request():
    """A long request's work is issued in chunks of about the quantum, so a
    request that arrives while it runs starts within a few chunks and finishes
    long before it, instead of waiting for a whole check interval of the slow
    request."""
    slow = dict(band_request(200_000, 71, 41), precision=fth.FTH_FP64)
    srv = fth.Server(steps_per_tick=2000, quantum_ms=10)
    a = srv.submit(**slow, replicas=32, block_len=100, max_steps=4000, target=0.0)
    for _ in range(3):
        srv.tick()
    b = srv.submit(**lap_request(8, 72, 42), block_len=20, max_steps=200, target=0.0)
    run_to_done(srv, [a, b])
    pa, pb = srv.poll(a), srv.poll(b)
    wait = pb["t_start"] - pb["t_submit"]
    print(f"[serve] slow request {pa['t_finish'] - pa['t_start']:.3f} s in {pa['chunks']} chunks; "
          f"arrival waited {wait * 1e3:.1f} ms, finished after {pb['t_finish'] - pb['t_submit']:.3f} s", flush=True)
    assert pa["chunks"] > 2 * 4000 // 2000   # cut below the check interval
    assert pb["t_finish"] < pa["t_finish"]
    assert wait < 0.25 * (pa["t_finish"] - pa["t_start"])


# The overlap is a property of one serving process: it is measured in a child
# process of its own, so that it does not depend on what the test process ran
# before.  (In the full suite's process the two requests' chunks were seen
# serialized in two runs, while a fresh process overlapped them in every run,
# also with up to 64 other HIP streams held and after every other GPU test
# file had run in it; the cause was not found.)
OVERLAP_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
from paper_1402_2095_amd import fth
import test_gpu_server as T
d = T.dense_request(8192, 81, 51)
srv = fth.Server(steps_per_tick=200, quantum_ms=-1)
ids = [srv.submit(**d, replicas=128, block_len=100, max_steps=1000, target=0.0),
       srv.submit(**T.band_request(100_000, 82, 52), block_len=100, max_steps=1000, target=0.0)]
T.run_to_done(srv, ids)
dn, sp = (srv.poll(i) for i in ids)
assert dn["packed"] == 0 and sp["packed"] == 1
span = max(dn["device_last_ms"], sp["device_last_ms"]) - min(dn["device_first_ms"], sp["device_first_ms"])
busy = dn["device_ms"] + sp["device_ms"]
print(f"[serve] dense {dn['device_ms']:.1f} ms in {dn['chunks']} chunks, sparse {sp['device_ms']:.1f} ms "
      f"in {sp['chunks']} chunks, together {span:.1f} ms on the device clock", flush=True)
print(f"OVERLAP {busy / span:.4f}", flush=True)
"""


def test_dense_and_packed_chunks_overlap():
    """A dense GEMM request and a packed sparse request run on their own
    streams: on the device clock (HIP events around every chunk), the two
    requests' chunk time adds up to more than the span they occupied
    together, so their kernels ran at the same time."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", OVERLAP_CHILD, root], capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    ratio = float(r.stdout.split("OVERLAP")[1].split()[0])
    assert ratio > 1.25


def test_spectral_map_and_unscale_in_serving():
    """A request with a spectral map (Sec. I) is run on M' = r M with the GLE
    scaled by (alpha, gamma) and its x^-1/2 estimates are mapped back: equal
    to a standalone context with the same options, unscaled by fth_unscale."""
    x = lap_request(10, 91, 61)
    g = fi.load_gle("invsqrt_ns4")
    lo, hi = g.meta["window_lambda"]
    r = hi / (fi.laplacian3d_lambda_max(10, 0.1) * 1.5)
    opts = dict(scale_r=r, gle_alpha=1.3, gle_gamma=0.8)
    srv = fth.Server(steps_per_tick=100)
    rid = srv.submit(**x, block_len=50, max_steps=500, target=0.0, unscale_target=fth.FTH_TARGET_INVSQRT, **opts)
    run_to_done(srv, [rid])
    est, se = srv.result(rid)
    sol = fth.Solver(x["M"], x["A_p"], x["C_p"], x["dt"], pairs=x["pairs"], replicas=32, seed=x["seed"],
                     stream_id=x["stream_id"], block_len=50, **opts).run(500)
    e0, s0, _ = sol.read()
    w = (x["pairs"][:, 0] == x["pairs"][:, 1]).astype(np.float64)
    e1, s1 = fth.fth_unscale(fth.FTH_TARGET_INVSQRT, r, 0.0, 1.3, 0.8, w, e0, s0)
    assert np.array_equal(est, e1) and np.array_equal(se, s1)


def test_failed_admission_does_not_stop_the_others():
    bad = dense_request(700, 101, 71)   # R = 48 is not a dense matrix-core width
    good = lap_request(8, 102, 72)
    srv = fth.Server(steps_per_tick=50)
    ib = srv.submit(**bad, replicas=48, max_steps=100, target=0.0)
    ig = srv.submit(**good, block_len=10, max_steps=100, target=0.0)
    run_to_done(srv, [ib, ig])
    assert srv.poll(ib)["state"] == fth.FTH_REQ_FAILED and srv.poll(ib)["status"] == fth.FTH_EUNSUPPORTED
    assert srv.poll(ig)["state"] == fth.FTH_REQ_DONE and srv.poll(ig)["steps"] == 100


def test_momentum_form_requests():
    """Requests for the paper's momentum estimator (Eq. 7): results are the
    <p p> block of a standalone context with acc_pp, bit for bit, packed beside
    a position-form request; with a spectral map (r, alpha, gamma) and the ln
    target, the momentum prefactor (gamma, not gamma / alpha^2) is undone."""
    g = fi.load_gle("ln_p_ns8")
    M = fi.m1_lattice_csr(8, 95)
    _, hi = fth.fth_gershgorin(M)
    h = 0.1 / np.sqrt(hi)
    pairs = request_pairs(M.n, 96)
    x = dict(M=M, A_p=g.A_p, C_p=g.C_p, dt=h, pairs=pairs, seed=96, stream_id=11)
    y = lap_request(10, 97, 12)      # a position-form request packed with it
    r, alpha, gamma = 2.0, 1.3, 0.8
    srv = fth.Server(steps_per_tick=100)
    common = dict(block_len=50, max_steps=600, target=0.0)
    ids = [srv.submit(**x, **common, momentum_form=True),
           srv.submit(**x, **common, momentum_form=True, scale_r=r, gle_alpha=alpha, gle_gamma=gamma,
                      unscale_target=fth.FTH_TARGET_LN),
           srv.submit(**y, **common)]
    run_to_done(srv, ids)
    infos = [srv.poll(i) for i in ids]
    assert all(i["state"] == fth.FTH_REQ_DONE and i["steps"] == 600 for i in infos)
    assert infos[0]["packed"] == 1 and infos[2]["packed"] == 1
    n_out = len(pairs)
    # plain momentum request
    est, se = srv.result(ids[0])
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=32, seed=96, stream_id=11, block_len=50,
                     acc_pp=True).run(600)
    e0, s0, _ = sol.read()
    assert np.array_equal(est, e0[n_out:]) and np.array_equal(se, s0[n_out:])
    # mapped momentum request: p block times alpha^-2, then the ln identity
    est, se = srv.result(ids[1])
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=32, seed=96, stream_id=11, block_len=50, acc_pp=True,
                     scale_r=r, gle_alpha=alpha, gle_gamma=gamma).run(600)
    e1, s1, _ = sol.read()
    w = (pairs[:, 0] == pairs[:, 1]).astype(np.float64)
    a2 = 1.0 / (alpha * alpha)
    ep, sp = e1[n_out:] * a2, s1[n_out:] * a2
    eu, su = fth.fth_unscale(fth.FTH_TARGET_LN, r, 0.0, alpha, gamma, w, ep, sp)
    assert np.array_equal(est, eu) and np.array_equal(se, su)
    # both estimate ln M: the diagonal agrees between the two within their errors and the model error
    d = w > 0
    e_plain, s_plain = srv.result(ids[0])
    z = (est[d] - e_plain[d]) / np.sqrt(se[d] ** 2 + s_plain[d] ** 2)
    print(f"[serve p-form] mapped vs plain diagonal of ln M: max|z| {np.max(np.abs(z)):.2f}", flush=True)
    assert np.max(np.abs(z)) < 6.0 or np.max(np.abs(est[d] / e_plain[d] - 1)) < 0.03
