"""Throughput benchmark of the f-thermostat hot path on one MI355X.

A benchmark "step" is one time step of the whole hot path over the
workload: force -M q, diagonal and pair accumulation, kicks, the exact GLE
Ornstein-Uhlenbeck update with fresh Philox noise, drift, and block folding
when due.  The default workload is the 64^3 periodic Laplacian + 0.1
(N = 262144, CSR, FP32 values) with an ns = 4 GLE (x^-1/2 target), R = 8
replicas, estimating the diagonal plus 1024 random pairs, 1e4 steps.

Prints one JSON line: throughput in replica*dof*steps/s (inputs resident in
HBM, timed between stream synchronisations), the step kernel's roofline
(algorithmic bytes per launch over its HIP-event-measured average duration)
and, at N = 1 on rank 0, the FP64 CPU oracle timed on a bounded sample of
the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import fth_inputs as fi  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Full-rate 32-bit VALU lane operations per second: 256 CUs x 4 SIMDs x 32
# lanes x 2.4 GHz (the FP32 vector peak of 157.3 TFLOP/s counts an FMA as 2).
ALU_PEAK_GOPS = 256 * 4 * 32 * 2.4
PROFILE_DIR = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1402_2095_amd", "csrc")
# Device sources of each step form; a committed traffic figure is used only
# while their hash is unchanged.
KERNEL_SOURCES = {
    "csr": ["csr_step.hpp", "csr_step_f32.hip", "csr_step_f64.hip", "row_update.hpp", "noise.hpp"],
    "tb": ["tb_step.hpp", "tb_step.hip", "row_update.hpp", "noise.hpp"],
    "tbp": ["tbp_step.hpp", "tbp_step.hip", "tb_step.hpp", "row_update.hpp", "noise.hpp"],
    "dense": ["dense.hpp", "dense_f32.hip", "dense_f64.hip", "row_update.hpp", "noise.hpp"],
}


# Extra solver options of a workload (spectral map, estimators), set by workload().
EXTRA = {}


def workload(name: str):
    """Returns (description dict, matrix CSR, GLE, dt, R, pairs, precision, default steps)."""
    from paper_1402_2095_amd import fth
    if name in ("laplacian64", "laplacian64-fp64"):
        M = fi.laplacian3d_csr(64, 0.1)
        g = fi.load_gle("invsqrt_ns4")
        h = fi.dt_rule(fi.laplacian3d_lambda_max(64, 0.1))
        pairs = fi.random_pairs(M.n, 1024, 2002)
        prec = fth.FTH_FP64 if name.endswith("fp64") else fth.FTH_FP32
        desc = {"workload": "3-D periodic 7-point Laplacian 64^3 + 0.1 I (N=262144, CSR)",
                "gle": "ns=4, x^-1/2 target", "replicas": 8, "estimates": "diagonal + 1024 pairs",
                "steps_in_config": 10000}
        return desc, M, g, h, 8, pairs, prec, 10000
    if name in ("banded1e6", "banded1e6-fp64"):
        M = fi.banded_spd_csr(1_000_000, 3003)
        g = fi.load_gle("fermi_b20_ns4")
        h = fi.dt_rule(fi.gershgorin_max(M))
        pairs = fi.random_pairs(M.n, 1024, 3004)
        prec = fth.FTH_FP64 if name.endswith("fp64") else fth.FTH_FP32
        desc = {"workload": "random banded SPD N=1e6, 7 nonzeros/row (CSR)",
                "gle": "ns=4, Fermi target", "replicas": 32, "estimates": "diagonal + 1024 pairs",
                "steps_in_config": 5000}
        return desc, M, g, h, 32, pairs, prec, 5000
    if name in ("dense16384", "dense16384-fp64"):
        n = 16384
        M = fi.dense_ggt(n, 4004)
        g = fi.load_gle("invsqrt_ns4")
        h = fi.dt_rule(fi.power_lambda_max(M.astype(np.float64), iters=30))
        pairs = fi.random_pairs(n, 1024, 4005)
        prec = fth.FTH_FP64 if name.endswith("fp64") else fth.FTH_FP32_BF16X3
        desc = {"workload": "dense SPD N=16384, M = G G^T / N + 0.1 I (FP32 values)",
                "gle": "ns=4, x^-1/2 target", "replicas": 128, "estimates": "diagonal + 1024 pairs",
                "steps_in_config": 2000}
        return desc, M, g, h, 128, pairs, prec, 2000
    if name == "m1-logdet":
        # the paper's M1 (logarithm example): periodic 24^3 lattice, on-site 100, hopping U[0, 2]
        # to the first six neighbour shells (81 entries per row); log det M = Tr ln M from the
        # position trace with the ln GLE, run on M' = r M (the spectral map of Sec. I)
        M = fi.m1_lattice_csr(24, 6006, dtype=np.float32)
        g = fi.load_gle("ln_ns4")
        lo_w, hi_w = g.meta["window_lambda"]
        _, hi = fth.fth_gershgorin(M)
        EXTRA.update(scale_r=hi_w / hi, acc_trace=True)
        desc = {"workload": "M1 lattice 24^3 (N=13824, 81 nonzeros/row, CSR), log det via Tr ln",
                "gle": "ns=4, ln target, M' = r M", "replicas": 32, "estimates": "diagonal + 1024 pairs + traces",
                "steps_in_config": 20000}
        return desc, M, g, 0.1 / np.sqrt(hi_w), 32, fi.random_pairs(M.n, 1024, 6007), fth.FTH_FP32, 20000
    if name == "m2-exp":
        # the paper's M2 (exponential example): dense, eigenvalues in (-300, 300) by Gerschgorin;
        # Tr exp(-M / 100) with the exp(-x) GLE on M' = M / 100 + 3.1 I
        n = 2048
        M = fi.m2_gerschgorin(n, 7007).astype(np.float32)
        g = fi.load_gle("expneg_ns4")
        lo_w, hi_w = g.meta["window_lambda"]
        r, m = fth.fth_spectral_map(-300.0, 300.0, lo_w, hi_w)
        EXTRA.update(scale_r=r, scale_m=m, acc_trace=True)
        desc = {"workload": "M2 dense N=2048, eigenvalues in (-300, 300), Tr exp(-M/100)",
                "gle": "ns=4, exp(-x) target, M' = M/100 + 3.1 I", "replicas": 128,
                "estimates": "diagonal + 1024 pairs + traces", "steps_in_config": 5000}
        return desc, M, g, 0.1 / np.sqrt(hi_w), 128, fi.random_pairs(n, 1024, 7008), fth.FTH_FP32_BF16X3, 5000
    raise SystemExit(f"unknown workload {name}")


def dense_roofline(M, ns: int, R: int, npairs: int, prec: int, per_step_s: float):
    """Dense step = GEMM + epilogue.  Bytes: M once (split form: hi + lo
    bf16 = 4 B per entry; FP64: 8 B), the state as in the sparse step, the
    split-K partials written and read back.  Flops: 2 N^2 R (algorithmic;
    the split form issues three bf16 products)."""
    from paper_1402_2095_amd import fth
    n = M.shape[0]
    P = (n + 255) // 256 * 256
    if P >= 2048:   # the library pads to whole 64-wide k-steps in each of its 8 K slices
        P = (n + 511) // 512 * 512
    ks = 8 if P >= 2048 else P // 256
    b = 8 if prec == fth.FTH_FP64 else 4
    mbytes = P * P * (8 if prec == fth.FTH_FP64 else 4)
    state = 2 * (ns + 2) * b * n * R + 16 * n + npairs * (2 * R * b + 24)
    part = 2 * ks * P * R * b
    flops = 2.0 * n * n * R
    return float(mbytes + state + part), flops


def coded_matrix_bytes(M, b: int) -> float:
    """Bytes of the coded sparse form: 8 one-byte column codes per row, and 8
    one-byte value codes (values in a table when there are at most 256
    distinct ones at state precision) or 8 raw values per row."""
    vals = M.val.astype(np.float64 if b == 8 else np.float32)
    table = np.unique(vals).size <= 256
    return float(M.n * (8 + (8 if table else 8 * b)))


def algorithmic_bytes(M, ns: int, R: int, npairs: int, prec: int, steps_per_launch: int = 1,
                      coded: bool = False) -> float:
    """Bytes one launch must move at minimum: state q (read q_n, write
    q_{n+k}), p and s_1..s_ns read and written; the matrix once (CSR: row_ptr
    8 B, col 4 B and a value per nonzero; or the coded form); the diagonal
    block accumulator read and written (FP64); per step, each pair's two q
    rows and its accumulator.  A blocked launch advancing k steps moves the
    state and the matrix once."""
    from paper_1402_2095_amd import fth
    b = 8 if prec == fth.FTH_FP64 else 4
    n = M.n
    state = 2 * (ns + 2) * b * n * R
    csr = coded_matrix_bytes(M, b) if coded else (n + 1) * 8 + M.nnz * (4 + b)
    diag = 16 * n
    pairs = steps_per_launch * npairs * (2 * R * b + 16 + 8)
    return float(state + csr + diag + pairs)


def alu_ops_per_row_step(ns: int, nnz_row: float) -> float:
    """Full-rate-equivalent VALU lane operations one replica of one row needs
    per step (half-rate operations count 2, quarter-rate 4):
      Philox4x32-10, per component, shared by 4 replicas: 10 rounds of two
        32x32->64 multiplies (2 each) and four XORs            -> 20 / replica
      uniform from a word: shift, convert (2), FMA               -> 4
      Box-Muller, per pair of normals: log2, sqrt, sin, cos (4 each) and
        three multiplies                                         -> 9.5 / normal
      force: one FMA per nonzero; OU update: (ns+1)^2 + (ns+1)(ns+2)/2 FMAs,
      two kicks and the drift; diagonal accumulator: convert and FP64 FMA (2 each)."""
    d = ns + 1
    noise = d * (20.0 + 4.0 + 9.5)
    return noise + nnz_row + d * d + d * (d + 1) / 2 + 3 + 4


def source_hash(kind: str) -> str:
    import hashlib
    hsh = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def unit_of(kernel_name: str):
    """The kernels of one timed unit, its kind and the steps it covers, from
    the library's description of the step.  Kernel names are prefixes of
    rocprofv3's names up to the last template argument the description fixes
    (the trailing flags select optional estimators)."""
    import re
    m = re.search(r"tbp_step_kernel<(\w+),NS=(\d+),KT=(\d+)>", kernel_name)
    if m:
        real, ns, kt = m.group(1), m.group(2), int(m.group(3))
        return "tbp", [f"tbp_step_kernel<{real}, {ns}, {kt},", f"tb_pairs_kernel<{real}, 4, {kt}>"], kt
    m = re.search(r"tb_step_kernel<(\w+),NS=(\d+),RPT=4,KT=(\d+)>", kernel_name)
    if m:
        real, ns, kt = m.group(1), m.group(2), int(m.group(3))
        return "tb", [f"tb_step_kernel<{real}, {ns}, 4, {kt},", f"tb_pairs_kernel<{real}, 4, {kt}>"], kt
    m = re.search(r"csr_step_kernel<(\w+),NS=(\d+),RPT=(\d+),NT=(\d),CODED=(\d)>", kernel_name)
    if m:
        real, ns, rpt, nt, coded = m.groups()
        tf = {"0": "false", "1": "true"}
        return "csr", [f"csr_step_kernel<{real}, {ns}, {rpt}, {tf[nt]}, {tf[coded]},"], 1
    m = re.search(r"(gemm_bf16x3_kernel|gemm_f64_kernel)<RT=(\d+),ksplit=\d+> \+ "
                  r"dense_epilogue_kernel<(\w+),NS=(\d+),RPT=(\d+),NT=(\d)>", kernel_name)
    if m:
        gemm, rt, real, ns, rpt, nt = m.groups()
        return "dense", [f"{gemm}<{rt}>", f"dense_epilogue_kernel<{real}, {ns}, {rpt}, "
                                          f"{'true' if nt == '1' else 'false'},"], 1
    return None, [], 1


def committed_traffic(workload_name: str, kernel_name: str):
    """HBM bytes per unit from the committed rocprofv3 summary of this
    workload, if it covers the kernels now selected and their sources are
    unchanged since the counters were taken; else None."""
    kind, names, _ = unit_of(kernel_name)
    if kind is None or not os.path.isdir(PROFILE_DIR):
        return None
    for f in sorted(os.listdir(PROFILE_DIR)):
        if not f.endswith(f"_{workload_name}.txt"):
            continue
        fields = {}
        with open(os.path.join(PROFILE_DIR, f)) as fh:
            for line in fh:
                if ": " in line and not line.startswith(" "):
                    k, v = line.rstrip("\n").split(": ", 1)
                    fields[k] = v
        if fields.get("unit_kernels") == " + ".join(names) and fields.get("source_sha256") == source_hash(kind):
            try:
                return float(fields["traffic_bytes_per_unit"])
            except (KeyError, ValueError):
                return None
    return None


def profile_summary(d: str, workload_name: str) -> str:
    """Condense one rocprofv3 profiling pass of a workload (kernel trace with
    --stats, a FETCH_SIZE and a WRITE_SIZE counter run, and the same two
    counters on a plain 1 GiB float32 copy for scale) into the text kept
    under profiles/.  Layout of d: kt/ (kernel trace, -o kt), kt.log (the
    bench line printed under the trace), fetch/ and write/ (-o pmc),
    fetch_copy/ and write_copy/ (-o pmc), commands.txt."""
    import csv
    import statistics
    from collections import defaultdict

    def pmc(sub):
        vals = defaultdict(list)
        with open(os.path.join(d, sub, "pmc_counter_collection.csv")) as fh:
            for row in csv.DictReader(fh):
                vals[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        return vals

    with open(os.path.join(d, "kt.log")) as fh:
        bench_line = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    kname = bench_line["config"]["kernel"]
    kind, names, unit_steps = unit_of(kname)
    with open(os.path.join(d, "kt", "kt_kernel_stats.csv")) as fh:
        stats = list(csv.DictReader(fh))
    cf, cw = pmc("fetch_copy"), pmc("write_copy")
    copy_key = max((k for k in cf if "elementwise" in k), key=lambda k: len(cf[k]))
    copy_bytes = float(1 << 30)
    fscale = copy_bytes / 1024.0 / statistics.median(cf[copy_key])
    wscale = copy_bytes / 1024.0 / statistics.median(cw[copy_key])
    fe, wr = pmc("fetch"), pmc("write")
    lines = [f"rocprofv3 summary: {kname}",
             f"workload: {workload_name} ({bench_line['config']['workload']}, R={bench_line['config']['replicas']})",
             f"unit of work: {bench_line['roofline']['unit_of_work']}", "",
             "commands (from the repository root on one MI355X, after cd /tmp && export TMPDIR=/tmp;",
             "           REPO is the repository root, OUT the output directory):"]
    with open(os.path.join(d, "commands.txt")) as fh:
        lines += ["  " + ln.rstrip() for ln in fh if ln.strip()]
    lines += ["", "kernel trace statistics (top 8 by total time):",
              f"  {'kernel':<72} {'calls':>6} {'avg us':>9} {'min us':>9} {'max us':>9} {'%':>6}"]
    for r in stats[:8]:
        lines.append(f"  {r['Name'].replace('void fth::dev::', '')[:72]:<72} {r['Calls']:>6} "
                     f"{float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:9.2f} "
                     f"{float(r['MaxNs']) / 1e3:9.2f} {float(r['Percentage']):6.2f}")
    lines += ["", f"counter scale from the copy kernel ({copy_key.split('(')[0][:60]}..., 1 GiB read + 1 GiB written):",
              f"  FETCH_SIZE x {fscale:.3f}, WRITE_SIZE x {wscale:.3f}", "",
              "per dispatch of the unit's kernels (median over dispatches):"]
    avg_ns, fetch_b, write_b = 0.0, 0.0, 0.0
    for nm in names:
        st = [r for r in stats if nm in r["Name"]]
        kf = [k for k in fe if nm in k]
        kw = [k for k in wr if nm in k]
        a = float(st[0]["AverageNs"]) if st else float("nan")
        f_raw = statistics.median(fe[kf[0]]) if kf else float("nan")
        w_raw = statistics.median(wr[kw[0]]) if kw else float("nan")
        avg_ns += a
        fetch_b += f_raw * 1024 * fscale
        write_b += w_raw * 1024 * wscale
        lines.append(f"  {nm}: avg {a / 1e3:.2f} us, FETCH_SIZE {f_raw:.0f} KiB -> {f_raw * 1024 * fscale / 1e6:.1f} MB, "
                     f"WRITE_SIZE {w_raw:.0f} KiB -> {w_raw * 1024 * wscale / 1e6:.1f} MB")
    roof = bench_line["roofline"]
    lines += ["", f"unit totals: avg {avg_ns / 1e3:.2f} us (bench, HIP events: {roof['avg_unit_us']:.2f} us), "
                  f"HBM traffic {(fetch_b + write_b) / 1e6:.1f} MB "
                  f"(algorithmic {roof['algorithmic_bytes_per_unit'] / 1e6:.1f} MB)",
              f"measured traffic rate {(fetch_b + write_b) / avg_ns:.0f} GB/s; roofline in the bench line: "
              f"bound {roof['bound']}, frac {roof['frac']:.3f}", "",
              "bench line printed under the trace:", "  " + json.dumps(bench_line), "",
              f"unit_kernels: {' + '.join(names)}",
              f"source_sha256: {source_hash(kind)}",
              f"avg_unit_ns: {avg_ns:.1f}",
              f"fetch_bytes_per_unit: {fetch_b:.6e}",
              f"write_bytes_per_unit: {write_b:.6e}",
              f"traffic_bytes_per_unit: {fetch_b + write_b:.6e}"]
    return "\n".join(lines) + "\n"


def cpu_baseline(M, g, h, R, pairs, budget_s: float):
    import oracle
    nthreads = oracle.max_threads()
    r, m = EXTRA.get("scale_r", 1.0), EXTRA.get("scale_m", 0.0)   # the same spectral map as the GPU run
    if isinstance(M, np.ndarray):
        M64 = r * M.astype(np.float64) + m * np.eye(M.shape[0])
        n = M.shape[0]
    else:
        val = r * M.val.astype(np.float64)
        rows = np.repeat(np.arange(M.n), np.diff(M.row_ptr))
        val[rows == M.col] += m
        M64 = fi.CSR(M.n, M.row_ptr, M.col, val)
        n = M.n
    run = oracle.OracleRun(M64, g.A_p, g.C_p, h, R, np.concatenate([pairs, fi.diag_pairs(n)]), seed=2)
    run.run(1)  # warm-up
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < 2000:
        run.run(1)
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": n * R * steps / dt, "unit": "replica*dof*steps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"full workload (N={n}, R={R}, diagonal + {len(pairs)} pairs), {steps} steps after 1 "
                      f"warm-up step, {dt:.1f} s, FP64, OpenMP over rows"}


def serving_pairs(n: int, seed: int, nd: int = 128, no: int = 128) -> np.ndarray:
    """128 diagonal elements and 128 off-diagonal pairs among them (so each
    off-diagonal stderr can be normalised by its two diagonals)."""
    rng = np.random.default_rng(seed)
    d = rng.choice(n, size=nd, replace=False)
    a = rng.integers(0, nd, size=no)
    b = (a + 1 + rng.integers(0, nd - 1, size=no)) % nd
    return np.concatenate([np.stack([d, d], 1), np.stack([d[a], d[b]], 1)]).astype(np.int32)


def serving(args):
    """Poisson arrivals of mixed sparse/dense solves, each run to a target
    relative stderr; reports p50/p99 latency and throughput."""
    from paper_1402_2095_amd import fth
    reqs = fi.serving_mix(args.serve_count, args.serve_rate, 5005, n_sparse=(10_000, args.serve_nmax),
                          n_dense=(512, args.serve_dense_nmax))
    gles = {"invsqrt": fi.load_gle("invsqrt_ns4"), "fermi": fi.load_gle("fermi_b20_ns4")}
    prepared = []
    for r in reqs:
        if r.kind == "laplacian":
            side = round(r.n ** (1 / 3))
            M = fi.laplacian3d_csr(side, 0.1)
            lmax, n, prec, R = fi.laplacian3d_lambda_max(side, 0.1), M.n, fth.FTH_FP32, 32
        elif r.kind == "banded":
            M = fi.banded_spd_csr(r.n, r.seed)
            lmax, n, prec, R = fi.gershgorin_max(M), M.n, fth.FTH_FP32, 32
        else:
            M = fi.dense_ggt(r.n, r.seed)
            lmax, n, prec, R = fi.power_lambda_max(M.astype(np.float64), iters=30), r.n, fth.FTH_FP32_BF16X3, 64
        g = gles[r.target]
        prepared.append(dict(arrival=r.arrival, kind=r.kind, n=n, R=R, target=r.target,
                             kw=dict(M=M, A_p=g.A_p, C_p=g.C_p, dt=fi.dt_rule(lmax), pairs=serving_pairs(n, r.seed),
                                     replicas=R, precision=prec, seed=r.seed, stream_id=r.rid + 1, burn_in=1000,
                                     block_len=200, target=args.serve_target, max_steps=args.serve_max_steps)))
    srv = fth.Server(steps_per_tick=args.serve_tick)
    t0 = srv.clock()
    pending = list(prepared)
    ids = {}
    print(f"[serve] {len(prepared)} requests prepared, rate {args.serve_rate}/s, target {args.serve_target}",
          file=sys.stderr, flush=True)
    last_report = 0.0
    while True:
        now = srv.clock() - t0
        while pending and pending[0]["arrival"] <= now:
            p = pending.pop(0)
            ids[srv.submit(**p["kw"])] = p
        infos = {i: srv.poll(i) for i in ids}
        live = [i for i, inf in infos.items() if inf["state"] < fth.FTH_REQ_DONE]
        if not pending and not live:
            break
        if now > args.serve_budget:
            for i in live:
                srv.cancel(i)
            break
        if not live:
            time.sleep(max(0.0, min(0.05, pending[0]["arrival"] - now)))
            continue
        srv.tick()
        if now - last_report > 10:
            last_report = now
            q, r, b = srv.stats()
            done = sum(1 for inf in infos.values() if inf["state"] == fth.FTH_REQ_DONE)
            print(f"[serve] t={now:.0f}s queued={q} running={r} done={done} reserved={b / 1e9:.2f} GB",
                  file=sys.stderr, flush=True)
    wall = srv.clock() - t0
    infos = {i: srv.poll(i) for i in ids}
    done = [(ids[i], inf) for i, inf in infos.items() if inf["state"] == fth.FTH_REQ_DONE]
    not_done = [{"kind": ids[i]["kind"], "n": ids[i]["n"], "state": inf["state"], "status": inf["status"],
                 "steps": inf["steps"]} for i, inf in infos.items() if inf["state"] != fth.FTH_REQ_DONE]
    for nd in not_done:
        print(f"[serve] not completed: {nd}", file=sys.stderr, flush=True)
    lat = np.array([inf["t_finish"] - inf["t_submit"] for _, inf in done])
    work = sum(p["n"] * inf["replicas"] * inf["steps"] for p, inf in done)
    at_target = sum(1 for _, inf in done if inf["max_rel_stderr"] <= args.serve_target)
    out = {
        "metric": "replica*dof*steps/s (serving mix) with p50/p99 latency at fixed stderr",
        "value": work / wall, "unit": "replica*dof*steps/s", "n_gpus": 1, "steps": None, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving mix: Poisson arrivals, 70% sparse (3-D Laplacian / banded SPD, "
                               f"N in [1e4, {args.serve_nmax:.0e}]), 30% dense (N in [512, {args.serve_dense_nmax}]), "
                               "Fermi / x^-1/2 50:50, 128 diagonal + 128 off-diagonal estimates each",
                   "requests": len(prepared), "rate_per_s": args.serve_rate,
                   "target_rel_stderr": args.serve_target, "steps_per_tick": args.serve_tick,
                   "scaled": "N ranges and stderr target scaled down from the full mix (see DESIGN)"},
        "serving": {"completed": len(done), "not_completed": not_done, "at_target": at_target, "wall_s": wall,
                    "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
                    "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
                    "mean_latency_s": float(lat.mean()) if len(lat) else None,
                    "requests_per_s": len(done) / wall},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="laplacian64")
    ap.add_argument("--steps-per-graph", type=int, default=64)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain elementwise copy (y = -x, float32) of this many MiB, 5 times, "
                         "to scale the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--serve-count", type=int, default=24)
    ap.add_argument("--serve-rate", type=float, default=0.5)
    ap.add_argument("--serve-target", type=float, default=2e-2)
    ap.add_argument("--serve-nmax", type=int, default=200_000)
    ap.add_argument("--serve-dense-nmax", type=int, default=4096)
    ap.add_argument("--serve-tick", type=int, default=200)
    ap.add_argument("--serve-max-steps", type=int, default=2_000_000)
    ap.add_argument("--serve-budget", type=float, default=150.0, help="seconds before the rest is cancelled")
    ap.add_argument("--profile-summary", default=None, metavar="DIR",
                    help="write profiles/<kernel>_<workload>.txt from a rocprofv3 pass stored in DIR and exit")
    args = ap.parse_args()
    if args.profile_summary:
        text = profile_summary(args.profile_summary, args.workload)
        kind, names, _ = unit_of(text.splitlines()[0])
        base = names[0].split("<")[0] if names else "kernel"
        os.makedirs(PROFILE_DIR, exist_ok=True)
        with open(os.path.join(PROFILE_DIR, f"{base}_{args.workload}.txt"), "w") as fh:
            fh.write(text)
        print(text)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "torch.neg float32", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "dispatches": 5}), flush=True)
        return

    if args.workload == "serving":
        serving(args)
        return

    import torch
    from paper_1402_2095_amd import fth

    desc, M, g, h, R, pairs, prec, default_steps = workload(args.workload)
    steps = args.steps or default_steps
    print(f"[bench] workload={args.workload} R={R} steps={steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    sol = fth.Solver(M, g.A_p, g.C_p, h, pairs=pairs, replicas=R, precision=prec, seed=2, acc_diag=True,
                     steps_per_graph=args.steps_per_graph, block_len=100, hip_stream=stream.cuda_stream,
                     tune=not args.no_tune, **EXTRA)
    if args.warmup:
        sol.run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = sol.last_run_ms
    est, se, nsamp = sol.read()
    assert np.all(np.isfinite(est)), "non-finite estimates"
    dense = isinstance(M, np.ndarray)
    n = M.shape[0] if dense else M.n
    result = None
    if args.workload in ("m1-logdet", "m2-exp"):  # the trace, mapped back to the original matrix
        tgt = fth.FTH_TARGET_LN if args.workload == "m1-logdet" else fth.FTH_TARGET_EXPNEG
        k = len(est) - 2          # position trace (then q^T M q)
        e_u, s_u = fth.fth_unscale(tgt, EXTRA.get("scale_r", 1.0), EXTRA.get("scale_m", 0.0), 1.0, 1.0,
                                   [float(n)], est[k:k + 1], se[k:k + 1])
        result = {"quantity": "log det M" if tgt == fth.FTH_TARGET_LN else "Tr exp(-M/100)",
                  "estimate": float(e_u[0]), "stderr": float(s_u[0]), "steps": steps + args.warmup}
    kind, unit_kernels, unit_steps = unit_of(sol.kernel_name)
    units = steps / unit_steps
    per_unit_s = gpu_ms * 1e-3 / units   # HIP events around the timed run, on the library's stream
    traffic = committed_traffic(args.workload, sol.kernel_name)
    alu_ops = n * R * unit_steps * alu_ops_per_row_step(g.ns, 0.0 if dense else M.nnz / M.n)
    alu = {"achieved": alu_ops / per_unit_s / 1e9, "peak": ALU_PEAK_GOPS, "unit": "Gop/s",
           "frac": alu_ops / per_unit_s / 1e9 / ALU_PEAK_GOPS}
    if dense:
        abytes, flops = dense_roofline(M, g.ns, R, len(pairs), prec, per_unit_s)
    elif kind in ("tb", "tbp"):
        abytes = algorithmic_bytes(M, g.ns, R, len(pairs), prec, steps_per_launch=unit_steps)
    else:
        abytes = algorithmic_bytes(M, g.ns, R, len(pairs), prec, coded="CODED=1" in sol.kernel_name)
    achieved = abytes / per_unit_s / 1e9
    hbm = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
    unit_desc = {"csr": "one step (one step-kernel launch)",
                 "tb": f"one blocked launch = {unit_steps} steps (step kernel + pair kernel)",
                 "tbp": f"one blocked launch = {unit_steps} steps (persistent step kernel + pair kernel)",
                 "dense": "one step (GEMM + epilogue launches)"}.get(kind, "one step")
    if kind in ("tb", "tbp"):
        # several steps per launch with the state in registers and LDS: VALU-limited
        roof = {"bound": "alu", **{k: alu[k] for k in ("achieved", "peak", "unit", "frac")}, "traffic": traffic,
                "hbm": {k: hbm[k] for k in ("achieved", "peak", "unit", "frac")}}
    else:
        roof = dict(hbm)
        roof["alu"] = alu
    roof.update({"unit_of_work": unit_desc, "kernels": unit_kernels, "algorithmic_bytes_per_unit": abytes,
                 "alu_ops_per_unit": alu_ops, "avg_unit_us": per_unit_s * 1e6})
    if dense:
        mfma_peak = 78.6 if prec == fth.FTH_FP64 else 2500.0
        tf = flops * (3 if prec == fth.FTH_FP32_BF16X3 else 1) / per_unit_s / 1e12
        roof["mfma"] = {"issued_tflops": tf, "peak_tflops": mfma_peak, "frac": tf / mfma_peak,
                        "algorithmic_tflops": flops / per_unit_s / 1e12}

    value = n * R * steps / wall
    out = {
        "metric": "replica*dof*steps/s",
        "value": value,
        "unit": "replica*dof*steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == fth.FTH_FP64 else "f32",
        "data": "synthetic",
        "config": dict(desc, precision="fp64" if prec == fth.FTH_FP64 else "fp32 state, fp64 accumulators",
                       steps_per_graph=args.steps_per_graph, kernel=sol.kernel_name),
        "roofline": roof,
        "cpu_baseline": None,
    }
    if result is not None:
        out["result"] = result
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(M, g, h, R, pairs, args.cpu_budget)
    sol.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
