"""Throughput benchmark of the f-thermostat hot path on one MI355X.

A benchmark "step" is one time step of the whole hot path over the
workload: force -M q, diagonal and pair accumulation, kicks, the exact GLE
Ornstein-Uhlenbeck update with fresh Philox noise, drift, and block folding
when due.  The default workload is the largest single-GPU configuration:
the random banded SPD system with N = 1e6 rows and 7 nonzeros per row
(CSR, FP32 values), R = 32 replicas, an ns = 4 GLE fitted to a Fermi
function, estimating the diagonal plus 1024 random pairs.

Prints one JSON line: throughput in replica*dof*steps/s (inputs resident in
HBM, K timed steps between stream synchronisations, replayed from a graph
built during the warm-up), the step kernel's roofline (algorithmic bytes per
launch over its HIP-event-measured average duration), with the committed
rocprofv3 counter figures beside it, secondary workloads (the 64^3
Laplacian, the dense 16384 system, and the plain FP64 forms), a short
serving measurement (p50/p99 latency at a scaled stderr target, with a
projection to 1e-3), and the FP64 CPU oracle timed on a bounded sample of
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
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp64": 78.6}
CACHE_BYTES = 256 << 20   # Infinity Cache (MALL)
PROFILE_DIR = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1402_2095_amd", "csrc")
# Device sources of each step form; a committed counter figure is used only
# while their hash is unchanged.
KERNEL_SOURCES = {
    "csr": ["csr_step.hpp", "csr_step_f32.hip", "csr_step_f64.hip", "row_update.hpp", "noise.hpp"],
    "tb": ["tb_step.hpp", "tb_step.hip", "row_update.hpp", "noise.hpp"],
    "tbp": ["tbp_step.hpp", "tbp_step.hip", "tb_step.hpp", "row_update.hpp", "noise.hpp"],
    "dense": ["dense.hpp", "dense_f32.hip", "dense_f64.hip", "row_update.hpp", "noise.hpp"],
    "gemv": ["dense_gemv.hip", "dense.hpp", "dense_f32.hip", "row_update.hpp", "noise.hpp"],
}


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------- workloads
def workload(name: str) -> dict:
    """Synthetic inputs of a named configuration (seeded)."""
    from paper_1402_2095_amd import fth
    w = dict(name=name, extra={})
    if name in ("laplacian64", "laplacian64-fp64"):
        M = fi.laplacian3d_csr(64, 0.1)
        w.update(desc={"workload": "3-D periodic 7-point Laplacian 64^3 + 0.1 I (N=262144, CSR, FP32 values)",
                       "gle": "ns=4, x^-1/2 target", "replicas": 8, "estimates": "diagonal + 1024 pairs",
                       "steps_in_config": 10000},
                 M=M, g=fi.load_gle("invsqrt_ns4"), h=fi.dt_rule(fi.laplacian3d_lambda_max(64, 0.1)), R=8,
                 pairs=fi.random_pairs(M.n, 1024, 2002),
                 prec=fth.FTH_FP64 if name.endswith("fp64") else fth.FTH_FP32, steps=10000)
    elif name in ("banded1e6", "banded1e6-fp64"):
        M = fi.banded_spd_csr(1_000_000, 3003)
        w.update(desc={"workload": "random banded SPD N=1e6, 7 nonzeros/row (CSR, FP32 values)",
                       "gle": "ns=4, Fermi target (beta=20, mu mid-spectrum)", "replicas": 32,
                       "estimates": "diagonal + 1024 pairs", "steps_in_config": 5000},
                 M=M, g=fi.load_gle("fermi_b20_ns4"), h=fi.dt_rule(fi.gershgorin_max(M)), R=32,
                 pairs=fi.random_pairs(M.n, 1024, 3004),
                 prec=fth.FTH_FP64 if name.endswith("fp64") else fth.FTH_FP32, steps=5000)
    elif name == "banded1e6-pp":
        # the same system with the paper's own estimator (Eq. 7): <p_i p_j> kept beside <q_i q_j>,
        # with the momentum-form GLE of a zero-temperature Fermi step (same ns, so the same state)
        M = fi.banded_spd_csr(1_000_000, 3003)
        w.update(desc={"workload": "random banded SPD N=1e6, 7 nonzeros/row (CSR, FP32 values), momentum estimator",
                       "gle": "ns=4, momentum-form Fermi step across a gap", "replicas": 32,
                       "estimates": "diagonal + 1024 pairs, position and momentum forms", "steps_in_config": 5000},
                 M=M, g=fi.load_gle("fermi_gap_p_ns4"), h=fi.dt_rule(fi.gershgorin_max(M)), R=32,
                 pairs=fi.random_pairs(M.n, 1024, 3004), prec=fth.FTH_FP32, steps=5000,
                 extra=dict(acc_pp=True))
    elif name in ("dense16384", "dense16384-fp64", "dense16384-r1"):
        # -r1: a single trajectory, as the paper runs its examples (the force as a matrix-vector
        # product in FP32)
        n = 16384
        R = 1 if name.endswith("r1") else 128
        M = fi.dense_ggt(n, 4004)
        w.update(desc={"workload": "dense SPD N=16384, M = G G^T / N + 0.1 I (FP32 values)",
                       "gle": "ns=4, x^-1/2 target", "replicas": R, "estimates": "diagonal + 1024 pairs",
                       "steps_in_config": 2000},
                 M=M, g=fi.load_gle("invsqrt_ns4"), h=fi.dt_rule(fi.power_lambda_max(M.astype(np.float64), iters=30)),
                 R=R, pairs=fi.random_pairs(n, 1024, 4005),
                 prec=(fth.FTH_FP64 if name.endswith("fp64") else fth.FTH_FP32 if name.endswith("r1")
                       else fth.FTH_FP32_BF16X3), steps=2000)
    elif name == "m1-logdet":
        # the paper's M1 (logarithm example): periodic 24^3 lattice, on-site 100, hopping U[0, 2]
        # to the first six neighbour shells (81 entries per row); log det M = Tr ln M as the
        # kinetic trace sum_i <p_i^2> with the momentum-form ln GLE (Eq. 7; omega in [e, 100 e],
        # which holds M1's spectrum without a map); the first 2000 steps (the warm-up of a
        # --warmup 2000 run) are burn-in, so the estimate leaves out the transient from q = p = 0
        M = fi.m1_lattice_csr(24, 6006, dtype=np.float32)
        g = fi.load_gle("ln_p_ns8")
        _, hi = fth.fth_gershgorin(M)
        w.update(desc={"workload": "M1 lattice 24^3 (N=13824, 81 nonzeros/row, CSR), log det via the kinetic trace",
                       "gle": "ns=8, ln target, momentum form (Eq. 7)", "replicas": 32,
                       "estimates": "diagonal + 1024 pairs, position and momentum forms, traces",
                       "steps_in_config": 20000},
                 M=M, g=g, h=0.1 / np.sqrt(hi), R=32, pairs=fi.random_pairs(M.n, 1024, 6007), prec=fth.FTH_FP32,
                 steps=20000, extra=dict(acc_pp=True, acc_trace=True, burn_in=2000))
    elif name == "m2-exp":
        # the paper's M2 (exponential example): dense, eigenvalues in (-300, 300) by Gerschgorin;
        # Tr exp(-M / 100) with the exp(-x) GLE on M' = M / 100 + 3.1 I
        n = 2048
        M = fi.m2_gerschgorin(n, 7007).astype(np.float32)
        g = fi.load_gle("expneg_ns4")
        lo_w, hi_w = g.meta["window_lambda"]
        r, m = fth.fth_spectral_map(-300.0, 300.0, lo_w, hi_w)
        w.update(desc={"workload": "M2 dense N=2048, eigenvalues in (-300, 300), Tr exp(-M/100)",
                       "gle": "ns=4, exp(-x) target, M' = M/100 + 3.1 I", "replicas": 128,
                       "estimates": "diagonal + 1024 pairs + traces", "steps_in_config": 5000},
                 M=M, g=g, h=0.1 / np.sqrt(hi_w), R=128, pairs=fi.random_pairs(n, 1024, 7008),
                 prec=fth.FTH_FP32_BF16X3, steps=5000, extra=dict(scale_r=r, scale_m=m, acc_trace=True))
    else:
        raise SystemExit(f"unknown workload {name}")
    w["dense"] = isinstance(w["M"], np.ndarray)
    w["n"] = w["M"].shape[0] if w["dense"] else w["M"].n
    return w


# --------------------------------------------------- algorithmic figures
def step_bytes(w: dict) -> float:
    """Bytes one time step must move at minimum (a per replica-dof figure
    times N R): the state q, p, s_1..s_ns read and written once; sparse: the
    CSR matrix once (32-bit row pointers, 32-bit column indices, one value
    per nonzero) and the FP64 diagonal block accumulator (and its
    momentum-form twin, when kept) read and written; dense: M once as bf16
    hi + lo (4 bytes per entry; FP64: 8).  Selected pairs are negligible and
    left out."""
    from paper_1402_2095_amd import fth
    b = 8 if w["prec"] == fth.FTH_FP64 else 4
    n, R, ns = w["n"], w["R"], w["g"].ns
    state = 2.0 * (ns + 2) * b * n * R
    if w["dense"]:
        return state + float(n) * n * (8 if w["prec"] == fth.FTH_FP64 else 4)
    M = w["M"]
    acc = 16.0 * n * (2 if w["extra"].get("acc_pp") else 1)   # FP64 block sums: q-q, and p-p when kept
    return state + (n + 1) * 4.0 + M.nnz * (4.0 + b) + acc


def alu_ops_per_row_step(ns: int, nnz_row: float) -> float:
    """Full-rate-equivalent VALU lane operations one replica of one row needs
    per step (half-rate operations count 2, quarter-rate 4):
      Philox4x32-10, per component, shared by 4 replicas: 10 rounds of two
        32x32->64 products (2 each) and two three-way XORs       -> 15 / replica
      uniform from a word: shift, or, subtract                   -> 3
      Box-Muller, per pair of normals: log2, sqrt, sin, cos (4 each) and
        three multiplies                                         -> 9.5 / normal
      force: one FMA per nonzero; OU update: (ns+1)^2 + (ns+1)(ns+2)/2 FMAs,
      two kicks and the drift; diagonal accumulator: convert and FP64 FMA (2 each)."""
    d = ns + 1
    noise = d * (15.0 + 3.0 + 9.5)
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
    m = re.search(r"dense_gemv_kernel<(\w+),R=(\d+)> \+ dense_epilogue_kernel<(\w+),NS=(\d+),RPT=(\d+),NT=(\d)>",
                  kernel_name)
    if m:
        real, r, _, ns, rpt, nt = m.groups()
        return "gemv", [f"dense_gemv_kernel<{real}, {r}>", f"dense_epilogue_kernel<{real}, {ns}, {rpt}, "
                                                          f"{'true' if nt == '1' else 'false'},"], 1
    return None, [], 1


def committed_counters(workload_name: str, kernel_name: str) -> dict:
    """Counter figures of the committed rocprofv3 summary of this workload,
    if it covers the kernels now selected and their sources are unchanged
    since the counters were taken; else {}."""
    kind, names, _ = unit_of(kernel_name)
    if kind is None or not os.path.isdir(PROFILE_DIR):
        return {}
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
            out = {}
            for k in ("traffic_bytes_per_unit", "valu_busy", "valu_insts_per_unit", "mfma_busy"):
                try:
                    out[k] = float(fields[k])
                except (KeyError, ValueError):
                    pass
            out["profile"] = f"profiles/{f}"
            return out
    return {}


# ------------------------------------------------------------ timed runs
def graph_length(steps: int, warmup: int, kt: int) -> int:
    """Steps per captured graph: a whole number of blocked launches that
    divides the timed steps, no longer than the warm-up (which then builds
    the graph, so the timed region only replays it) nor 64 steps."""
    cap = max(kt, min(64, warmup))
    best = None
    for d in range(kt, cap + 1, kt):
        if steps % d == 0:
            best = d
    return best or max(kt, cap // kt * kt)


def timed_run(w: dict, steps: int, warmup: int, tune: bool, stream) -> dict:
    import torch
    from paper_1402_2095_amd import fth
    sol = fth.Solver(w["M"], w["g"].A_p, w["g"].C_p, w["h"], pairs=w["pairs"], replicas=w["R"], precision=w["prec"],
                     seed=2, acc_diag=True, steps_per_graph=64, block_len=100, hip_stream=stream.cuda_stream,
                     tune=tune, **w["extra"])
    sol.run(0)   # fixes R and, when tuning, the launch shape
    kind, kernels, unit_steps = unit_of(sol.kernel_name)
    spg = graph_length(steps, warmup, unit_steps)
    sol.set_steps_per_graph(spg)
    if warmup:
        sol.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    est, se, nsamp = sol.read()
    assert np.all(np.isfinite(est)), "non-finite estimates"
    res = dict(wall=wall, gpu_ms=sol.last_run_ms, kernel=sol.kernel_name, kind=kind, kernels=kernels,
               unit_steps=unit_steps, steps_per_graph=spg, est=est, se=se)
    sol.close()
    return res


def roofline(w: dict, r: dict, steps: int) -> dict:
    """Roofline of the dominant kernel: algorithmic bytes of the launches
    over their average duration (HIP events on the library's stream)."""
    from paper_1402_2095_amd import fth
    units = steps / r["unit_steps"]
    per_unit_s = r["gpu_ms"] * 1e-3 / units
    sb = step_bytes(w)
    abytes = sb * r["unit_steps"]
    achieved = abytes / per_unit_s / 1e9
    cnt = committed_counters(w["name"], r["kernel"])
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": cnt.get("traffic_bytes_per_unit"),
            "unit_of_work": {"csr": "one step (one step-kernel launch)",
                             "tb": f"one blocked launch = {r['unit_steps']} steps (step kernel + pair kernel)",
                             "tbp": f"one blocked launch = {r['unit_steps']} steps (persistent step kernel "
                                    "+ pair kernel)",
                             "dense": "one step (GEMM + epilogue launches)",
                             "gemv": "one step (matrix-vector + epilogue launches)"}.get(r["kind"], "one step"),
            "kernels": r["kernels"], "algorithmic_bytes_per_unit": abytes,
            "algorithmic_bytes_per_replica_dof_step": sb / (w["n"] * w["R"]), "avg_unit_us": per_unit_s * 1e6}
    if cnt:
        roof["counters_from"] = cnt["profile"]
    if r["kind"] in ("tb", "tbp"):
        # several steps per launch: the state crosses HBM once per launch, so the
        # launch is limited by VALU work (noise generation) rather than by bytes
        alu_ops = w["n"] * w["R"] * r["unit_steps"] * alu_ops_per_row_step(w["g"].ns, w["M"].nnz / w["n"])
        roof["note"] = ("temporally blocked: achieved = bytes a one-step-per-launch schedule must move for "
                        f"these {r['unit_steps']} steps over the launch time; the launch itself moves `traffic` "
                        "bytes and is VALU-bound (valu_busy from SQ_ACTIVE_INST_VALU)")
        roof["valu"] = {"busy_frac_counter": cnt.get("valu_busy"), "insts_per_unit_counter": cnt.get("valu_insts_per_unit"),
                        "model_ops_per_unit": alu_ops, "model_frac": alu_ops / per_unit_s / 1e9 / ALU_PEAK_GOPS}
    elif cnt.get("valu_busy") is not None:
        roof["valu"] = {"busy_frac_counter": cnt["valu_busy"], "insts_per_unit_counter": cnt.get("valu_insts_per_unit")}
    if not w["dense"]:
        ws = 2 * (w["g"].ns + 2) * (8 if w["prec"] == fth.FTH_FP64 else 4) * w["n"] * w["R"]
        if ws < CACHE_BYTES:
            roof["cache_resident"] = "working set fits the 256 MB Infinity Cache: effective bandwidth"
    elif r["kind"] == "gemv":
        roof["note"] = "few replicas: the force as matrix-vector products with plain FMAs, one pass over M per step"
    else:
        flops = 2.0 * w["n"] * w["n"] * w["R"]
        issued = flops * (3 if w["prec"] == fth.FTH_FP32_BF16X3 else 1)
        peak = MFMA_PEAK_TFLOPS["fp64" if w["prec"] == fth.FTH_FP64 else "bf16"]
        roof["mfma"] = {"algorithmic_tflops": flops / per_unit_s / 1e12, "issued_tflops": issued / per_unit_s / 1e12,
                        "peak_tflops": peak, "issued_frac": issued / per_unit_s / 1e12 / peak,
                        "busy_frac_counter": cnt.get("mfma_busy")}
        if w["prec"] == fth.FTH_FP64:
            # 2 N^2 R flops at the FP64 matrix-core peak take longer than M's bytes at 8 TB/s: the
            # roofline is the MFMA one, with the byte figure kept beside it
            roof["bound_by"] = "FP64 MFMA (2 N^2 R flops at 78.6 TFLOP/s exceed M's bytes at 8 TB/s)"
            roof["hbm"] = {"achieved": roof["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": roof["frac"]}
            tf = flops / per_unit_s / 1e12
            roof.update(bound="mfma", achieved=tf, peak=peak, unit="TFLOP/s", frac=tf / peak)
    return roof


def secondary(name: str, steps: int, warmup: int, stream) -> dict:
    from paper_1402_2095_amd import fth
    log(f"secondary {name}: preparing")
    w = workload(name)
    r = timed_run(w, steps, warmup, True, stream)
    roof = roofline(w, r, steps)
    out = {"workload": w["desc"]["workload"], "replicas": w["R"],
           "dtype": "f64" if w["prec"] == fth.FTH_FP64 else "f32", "kernel": r["kernel"],
           "ms_per_step": r["wall"] * 1e3 / steps, "value": w["n"] * w["R"] * steps / r["wall"],
           "steps": steps, "warmup": warmup,
           "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "avg_unit_us", "traffic")
                        if k in roof}}
    for k in ("cache_resident", "mfma", "bound_by", "hbm", "note", "valu"):
        if k in roof:
            out["roofline"][k] = roof[k]
    log(f"secondary {name}: {out['ms_per_step'] * 1e3:.1f} us/step")
    return out


# ---------------------------------------------------------------- serving
def serving_pairs(n: int, seed: int, nd: int = 128, no: int = 128) -> np.ndarray:
    """128 diagonal elements and 128 off-diagonal pairs among them (so each
    off-diagonal stderr can be normalised by its two diagonals)."""
    rng = np.random.default_rng(seed)
    d = rng.choice(n, size=nd, replace=False)
    a = rng.integers(0, nd, size=no)
    b = (a + 1 + rng.integers(0, nd - 1, size=no)) % nd
    return np.concatenate([np.stack([d, d], 1), np.stack([d[a], d[b]], 1)]).astype(np.int32)


def serving_request(r, gles) -> tuple:
    """Inputs of one serving request, with the spectral map of Sec. I that
    places its spectrum in the fitted GLE's window: x^-1/2 with M' = r M
    (mapped back exactly), Fermi with M' = r M + m I (the result is the Fermi
    function of M with beta r and mu (mu' - m) / r)."""
    from paper_1402_2095_amd import fth
    if r.kind == "laplacian":
        side = round(r.n ** (1 / 3))
        M = fi.laplacian3d_csr(side, 0.1)
        lo, hi, n, prec, R = 0.1, fi.laplacian3d_lambda_max(side, 0.1), M.n, fth.FTH_FP32, 32
    elif r.kind == "banded":
        M = fi.banded_spd_csr(r.n, r.seed)
        lo, hi = fth.fth_gershgorin(M)
        lo = max(lo, 1e-3)
        n, prec, R = M.n, fth.FTH_FP32, 32
    else:
        M = fi.dense_ggt(r.n, r.seed)
        lo, hi, n, prec, R = 0.1, fi.power_lambda_max(M.astype(np.float64), iters=30), r.n, fth.FTH_FP32_BF16X3, 64
    g = gles[r.target]
    w_lo, w_hi = g.meta["window_lambda"]
    if r.target == "invsqrt":
        smap = dict(scale_r=w_hi / hi, scale_m=0.0, unscale_target=fth.FTH_TARGET_INVSQRT)
    else:
        sr, sm = fth.fth_spectral_map(lo, hi, w_lo, w_hi)
        smap = dict(scale_r=sr, scale_m=sm, unscale_target=-1)
    return dict(M=M, A_p=g.A_p, C_p=g.C_p, dt=fi.dt_rule(w_hi), pairs=serving_pairs(n, r.seed), replicas=R,
                precision=prec, seed=r.seed, stream_id=r.rid + 1, burn_in=1000, block_len=200, **smap), n


def run_serving(count: int, rate: float, target: float, nmax: int, dense_nmax: int, tick: int, max_steps: int,
                budget: float, seed: int = 5005) -> dict:
    """Poisson arrivals of mixed sparse/dense solves, each run to a target
    relative stderr; p50/p99 latency, throughput, and a projection of the
    latencies at the full mix's 1e-3 target from the measured rates."""
    from paper_1402_2095_amd import fth
    reqs = fi.serving_mix(count, rate, seed, n_sparse=(10_000, nmax), n_dense=(512, dense_nmax))
    gles = {"invsqrt": fi.load_gle("invsqrt_ns4"), "fermi": fi.load_gle("fermi_b20_ns4")}
    prepared = []
    for r in reqs:
        kw, n = serving_request(r, gles)
        prepared.append(dict(arrival=r.arrival, kind=r.kind, n=n, R=kw["replicas"], target=r.target,
                             kw=dict(kw, target=target, max_steps=max_steps)))
    srv = fth.Server(steps_per_tick=tick)
    t0 = srv.clock()
    pending = list(prepared)
    ids = {}
    log(f"serving: {len(prepared)} requests prepared, rate {rate}/s, target {target}")
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
        if now > budget:
            for i in live:
                srv.cancel(i)
            break
        if not live:
            time.sleep(max(0.0, min(0.05, pending[0]["arrival"] - now)))
            continue
        srv.tick()
        if now - last_report > 10:
            last_report = now
            q, rr, b = srv.stats()
            done = sum(1 for inf in infos.values() if inf["state"] == fth.FTH_REQ_DONE)
            log(f"serving: t={now:.0f}s queued={q} running={rr} done={done} reserved={b / 1e9:.2f} GB")
    wall = srv.clock() - t0
    infos = {i: srv.poll(i) for i in ids}
    done = [(ids[i], inf) for i, inf in infos.items() if inf["state"] == fth.FTH_REQ_DONE]
    not_done = [{"kind": ids[i]["kind"], "n": ids[i]["n"], "state": inf["state"], "status": inf["status"],
                 "steps": inf["steps"]} for i, inf in infos.items() if inf["state"] != fth.FTH_REQ_DONE]
    srv.close()
    lat = np.array([inf["t_finish"] - inf["t_submit"] for _, inf in done])
    work = sum(p["n"] * inf["replicas"] * inf["steps"] for p, inf in done)
    at_target = sum(1 for _, inf in done if inf["max_rel_stderr"] <= target)
    # projection to the full mix at 1e-3: steps scale as (stderr / 1e-3)^2; a request's
    # device time per replica-dof-step (measured in the mix) scales its time with N
    proj = {}
    rates = {}
    steps_1e3 = {}
    for p, inf in done:
        if inf["steps"] <= 0 or inf["device_ms"] <= 0 or not np.isfinite(inf["max_rel_stderr"]):
            continue
        s3 = inf["steps"] * (inf["max_rel_stderr"] / 1e-3) ** 2
        steps_1e3.setdefault(p["kind"], []).append(s3)
        rates.setdefault(p["kind"], []).append(p["n"] * inf["replicas"] * inf["steps"] / (inf["device_ms"] * 1e-3))
    if rates:
        full = fi.serving_mix(400, rate, seed + 1)
        tt = []
        for r in full:
            if r.kind not in rates:
                continue
            R = 64 if r.kind == "dense" else 32
            tt.append(float(np.median(steps_1e3[r.kind])) * r.n * R / float(np.median(rates[r.kind])))
        if tt:
            proj = {"p50_latency_s": float(np.percentile(tt, 50)), "p99_latency_s": float(np.percentile(tt, 99)),
                    "requests": len(tt),
                    "method": "full-size mix (sparse N in [1e4, 2e6], dense N in [512, 8192]), per kind: median "
                              "steps to 1e-3 = measured steps x (achieved stderr / 1e-3)^2, time = steps x N R / "
                              "measured replica*dof*steps/s of that kind in the mix; each request alone, no queueing"}
    return {"requests": len(prepared), "rate_per_s": rate, "target_rel_stderr": target, "steps_per_tick": tick,
            "completed": len(done), "at_target": at_target, "not_completed": not_done, "wall_s": wall,
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_latency_s": float(lat.mean()) if len(lat) else None,
            "requests_per_s": len(done) / wall if wall > 0 else None,
            "replica_dof_steps_per_s": work / wall if wall > 0 else None,
            "scaled": f"sparse N in [1e4, {nmax:.0e}], dense N in [512, {dense_nmax}], target {target} "
                      "(the full mix at 1e-3 takes hours per large request)",
            "projection_1e-3": proj}


# ---------------------------------------------------------------- CPU oracle
def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w: dict, budget_s: float) -> dict:
    """The FP64 oracle on the same workload, on all host threads for about
    budget_s seconds, and on one thread for one step."""
    import oracle
    nthreads = oracle.max_threads()
    r, m = w["extra"].get("scale_r", 1.0), w["extra"].get("scale_m", 0.0)   # the same spectral map
    M = w["M"]
    if w["dense"]:
        M64 = r * M.astype(np.float64) + m * np.eye(w["n"])
    else:
        val = r * M.val.astype(np.float64)
        rows = np.repeat(np.arange(M.n), np.diff(M.row_ptr))
        val[rows == M.col] += m
        M64 = fi.CSR(M.n, M.row_ptr, M.col, val)
    pairs = np.concatenate([w["pairs"], fi.diag_pairs(w["n"])])
    run = oracle.OracleRun(M64, w["g"].A_p, w["g"].C_p, w["h"], w["R"], pairs, seed=2)
    run.run(1)  # warm-up
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < 2000:
        run.run(1)
        steps += 1
    dt = time.perf_counter() - t0
    one = oracle.OracleRun(M64, w["g"].A_p, w["g"].C_p, w["h"], w["R"], pairs, seed=2, nthreads=1)
    t1 = time.perf_counter()
    one.run(1)
    dt1 = time.perf_counter() - t1
    n, R = w["n"], w["R"]
    return {"value": n * R * steps / dt, "unit": "replica*dof*steps/s", "cores": nthreads, "kind": "oracle",
            "cpu_model": cpu_model(), "value_1_core": n * R / dt1,
            "sample": f"full workload (N={n}, R={R}, diagonal + {len(w['pairs'])} pairs): {steps} steps after 1 "
                      f"warm-up step in {dt:.1f} s on {nthreads} threads (OpenMP over rows, FP64); one step on "
                      f"1 thread in {dt1:.1f} s"}


# ---------------------------------------------------------------- profiles
def profile_summary(d: str, workload_name: str) -> str:
    """Condense one rocprofv3 profiling pass of a workload into the text kept
    under profiles/.  Layout of d: kt/ (kernel trace with --stats, -o kt),
    kt.log (the bench line printed under the trace), fetch/ and write/
    (FETCH_SIZE, WRITE_SIZE runs, -o pmc), valu/ (optional: SQ_INSTS_VALU,
    SQ_ACTIVE_INST_VALU, GRBM_GUI_ACTIVE ...; -o pmc), mfma/ (optional:
    SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE), fetch_copy/ and write_copy/
    (the same two counters on a plain 1 GiB float32 copy, for scale),
    commands.txt."""
    import csv
    import statistics
    from collections import defaultdict

    def pmc(sub):
        vals = defaultdict(lambda: defaultdict(list))
        path = os.path.join(d, sub, "pmc_counter_collection.csv")
        if not os.path.exists(path):
            return None
        with open(path) as fh:
            for row in csv.DictReader(fh):
                vals[row["Kernel_Name"]][row["Counter_Name"]].append(float(row["Counter_Value"]))
        return vals

    def med(vals, names_sub, counter):
        ks = [k for k in vals if names_sub in k]
        if not ks or counter not in vals[ks[0]]:
            return float("nan")
        return statistics.median(vals[ks[0]][counter])

    with open(os.path.join(d, "kt.log")) as fh:
        bench_line = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    kname = bench_line["config"]["kernel"]
    kind, names, unit_steps = unit_of(kname)
    with open(os.path.join(d, "kt", "kt_kernel_stats.csv")) as fh:
        stats = list(csv.DictReader(fh))
    # per-dispatch durations; the timed region is the last steps / unit_steps launches (the
    # statistics' average also holds the autotuner's trial launches and the warm-up)
    with open(os.path.join(d, "kt", "kt_kernel_trace.csv")) as fh:
        trace = list(csv.DictReader(fh))
    n_timed = max(1, int(bench_line["steps"]) // unit_steps)

    def timed_avg_ns(nm):
        ds = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
                    for r in trace if nm in r["Kernel_Name"])
        ds = [x[1] for x in ds[-n_timed:]]
        return (sum(ds) / len(ds), len(ds)) if ds else (float("nan"), 0)
    cf, cw = pmc("fetch_copy"), pmc("write_copy")
    copy_key = max((k for k in cf if "elementwise" in k), key=lambda k: len(cf[k]["FETCH_SIZE"]))
    copy_bytes = float(1 << 30)
    fscale = copy_bytes / 1024.0 / statistics.median(cf[copy_key]["FETCH_SIZE"])
    wscale = copy_bytes / 1024.0 / statistics.median(cw[copy_key]["WRITE_SIZE"])
    fe, wr, va, mf = pmc("fetch"), pmc("write"), pmc("valu"), pmc("mfma")
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
              f"per dispatch of the unit's kernels (time: mean over the timed region's last {n_timed} dispatches "
              "in the kernel trace; counters: median over dispatches):"]
    avg_ns, fetch_b, write_b = 0.0, 0.0, 0.0
    valu_busy, valu_insts, mfma_busy = None, None, None
    for nm in names:
        a, cnt = timed_avg_ns(nm)
        f_raw = med(fe, nm, "FETCH_SIZE")
        w_raw = med(wr, nm, "WRITE_SIZE")
        avg_ns += a
        fetch_b += f_raw * 1024 * fscale
        write_b += w_raw * 1024 * wscale
        lines.append(f"  {nm}: avg {a / 1e3:.2f} us over {cnt}, FETCH_SIZE {f_raw:.0f} KiB -> "
                     f"{f_raw * 1024 * fscale / 1e6:.1f} MB, "
                     f"WRITE_SIZE {w_raw:.0f} KiB -> {w_raw * 1024 * wscale / 1e6:.1f} MB")
        if va is not None and nm == names[0]:
            act = med(va, nm, "SQ_ACTIVE_INST_VALU")
            ins = med(va, nm, "SQ_INSTS_VALU")
            gui = med(va, nm, "GRBM_GUI_ACTIVE")
            trans = med(va, nm, "SQ_INSTS_VALU_TRANS_F32")
            # VALUBusy as rocprofv3 derives it: 100 SQ_ACTIVE_INST_VALU / CU_NUM / GRBM_GUI_ACTIVE(max);
            # GRBM_GUI_ACTIVE is summed over the 8 XCDs here, so its max is the sum / 8
            valu_busy = act / 256.0 / (gui / 8.0)
            valu_insts = ins
            lines.append(f"    VALU: SQ_INSTS_VALU {ins:.4e} (transcendental F32 {trans:.3e}), SQ_ACTIVE_INST_VALU "
                         f"{act:.4e} quad-cycles, GRBM_GUI_ACTIVE {gui:.4e} (8 XCDs) -> VALU busy {valu_busy:.3f}")
        if mf is not None and nm == names[0]:
            busy = med(mf, nm, "SQ_VALU_MFMA_BUSY_CYCLES")
            gui = med(mf, nm, "GRBM_GUI_ACTIVE")
            mfma_busy = busy / (gui / 8.0) / 1024.0   # per SIMD (1024 SIMDs)
            lines.append(f"    MFMA: SQ_VALU_MFMA_BUSY_CYCLES {busy:.4e}, GRBM_GUI_ACTIVE {gui:.4e} -> MFMA busy "
                         f"{mfma_busy:.3f}")
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
    if valu_busy is not None:
        lines += [f"valu_busy: {valu_busy:.4f}", f"valu_insts_per_unit: {valu_insts:.6e}"]
    if mfma_busy is not None:
        lines += [f"mfma_busy: {mfma_busy:.4f}"]
    return "\n".join(lines) + "\n"


# -------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="banded1e6")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="budget of the short serving measurement (0: skip)")
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
        print("bench.py: the library runs on one GPU (it has no multi-GPU path); --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.init()   # before the library touches HIP in this process
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "torch.neg float32", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "dispatches": 5}), flush=True)
        return
    from paper_1402_2095_amd import fth

    if args.workload == "serving":
        s = run_serving(args.serve_count, args.serve_rate, args.serve_target, args.serve_nmax,
                        args.serve_dense_nmax, args.serve_tick, args.serve_max_steps, args.serve_budget)
        out = {"metric": "replica*dof*steps/s (serving mix) with p50/p99 latency at fixed stderr",
               "value": s["replica_dof_steps_per_s"], "unit": "replica*dof*steps/s", "n_gpus": 1, "steps": None,
               "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f32", "data": "synthetic",
               "config": {"workload": "serving mix: Poisson arrivals, 70% sparse (3-D Laplacian / banded SPD), "
                                      "30% dense, Fermi / x^-1/2 50:50, 128 diagonal + 128 off-diagonal estimates"},
               "serving": s, "roofline": None, "cpu_baseline": None}
        print(json.dumps(out), flush=True)
        return

    stream = torch.cuda.current_stream()
    log(f"workload={args.workload} steps={args.steps} warmup={args.warmup}")
    w = workload(args.workload)
    r = timed_run(w, args.steps, args.warmup, not args.no_tune, stream)
    roof = roofline(w, r, args.steps)
    log(f"{r['kernel']}: {r['wall'] * 1e6 / args.steps:.1f} us/step")
    out = {
        "metric": "replica*dof*steps/s",
        "value": w["n"] * w["R"] * args.steps / r["wall"],
        "unit": "replica*dof*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w["prec"] == fth.FTH_FP64 else "f32",
        "data": "synthetic",
        "config": dict(w["desc"], precision="fp64" if w["prec"] == fth.FTH_FP64 else "fp32 state, fp64 accumulators",
                       steps_per_graph=r["steps_per_graph"], kernel=r["kernel"]),
        "roofline": roof,
        "cpu_baseline": None,
    }
    if args.workload == "m1-logdet":   # the kinetic trace (the last output) is Tr ln M itself
        out["result"] = {"quantity": "log det M", "estimate": float(r["est"][-1]), "stderr": float(r["se"][-1]),
                         "steps": args.steps + args.warmup}
    if args.workload == "m2-exp":   # the position trace, mapped back to the original matrix
        k = len(r["est"]) - 2          # position trace (then q^T M q)
        e_u, s_u = fth.fth_unscale(fth.FTH_TARGET_EXPNEG, w["extra"]["scale_r"], w["extra"]["scale_m"], 1.0, 1.0,
                                   [float(w["n"])], r["est"][k:k + 1], r["se"][k:k + 1])
        out["result"] = {"quantity": "Tr exp(-M/100)", "estimate": float(e_u[0]), "stderr": float(s_u[0]),
                         "steps": args.steps + args.warmup}
    if args.workload == "banded1e6" and not args.no_secondary:
        sec = {}
        # warm-ups of about 0.2 s each: the inputs are generated on the host first, and a GPU left
        # idle meanwhile needs that long to return to full clocks
        for name, st, wu in (("banded1e6-fp64", 100, 300), ("banded1e6-pp", 100, 300), ("laplacian64", 1000, 10000),
                             ("dense16384", 100, 800), ("dense16384-fp64", 50, 200), ("dense16384-r1", 100, 800)):
            try:
                sec[name] = secondary(name, st, wu, stream)
            except Exception as e:  # a secondary workload never hides the headline line
                sec[name] = {"error": f"{type(e).__name__}: {e}"}
        if "ms_per_step" in sec.get("banded1e6-fp64", {}):
            sec["fp32_over_fp64_at_equal_stderr"] = sec["banded1e6-fp64"]["ms_per_step"] / out["ms_per_step"]
            sec["note"] = ("the FP32 and FP64 forms take the same number of steps to a given stderr (the stderr "
                           "depends on the samples only), so the step-time ratio is the time-to-stderr ratio")
        out["secondary"] = sec
    if args.serve_seconds > 0 and args.workload == "banded1e6":
        log("serving measurement")
        try:
            out["serving"] = run_serving(16, 1.0, args.serve_target, args.serve_nmax, args.serve_dense_nmax,
                                         args.serve_tick, args.serve_max_steps, args.serve_seconds)
        except Exception as e:
            out["serving"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
