"""GPU tests of the serving layer: continuous batching with the packed
multi-request kernel, admission by device footprint, stopping at a target
standard error, cancellation; and a request's result is the same alone and
in the mix (bit for bit: the packed kernel runs the same per-row arithmetic,
with the request's own noise stream and step counter)."""
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
