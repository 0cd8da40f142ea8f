"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Two separate builds, each exercised in a child process with its compiler's
sanitizer runtime preloaded (the runtimes of gcc and clang cannot share a
process):
  - the oracle's C step loop (gcc): dense and CSR runs with every
    accumulator kind, the noise functions;
  - the library's host code (hipcc, host side only): validation of every
    input kind (each failure path), the propagator, the spectral map
    helpers, the footprint model, and a create that reaches the device
    query (FTH_EDEVICE without a GPU).
A report from either sanitizer fails the child and the test."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_child(code: str, env_extra: dict) -> subprocess.CompletedProcess:
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"   # the interpreter itself leaks by design
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = ROOT
    return subprocess.run([sys.executable, "-c", textwrap.dedent(code)], env=env, capture_output=True, text=True,
                          timeout=600, cwd=ROOT)


def test_oracle_under_asan_ubsan(tmp_path):
    import oracle
    lib = oracle.build(force=True, sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ub = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    code = """
        import numpy as np
        import fth_inputs as fi
        import oracle
        g = fi.load_gle("invsqrt_ns4")
        M = fi.banded_spd_csr(301, 5, dtype=np.float64)
        pairs = np.concatenate([fi.random_pairs(M.n, 7, 1), fi.diag_pairs(M.n)])
        r = oracle.OracleRun(M, g.A_p, g.C_p, 0.05, 8, pairs, seed=3, stream=2, burn_in=3, block_len=5,
                             pp=True, traces=True).run(23)
        e, s = r.estimates()
        assert np.all(np.isfinite(e))
        D = fi.haar_spd(24, 7, 1.0, 10.0)[0]
        w = fi.white_noise_gle(1.0, 1.0)
        r2 = oracle.OracleRun(D, w.A_p, w.C_p, 0.05, 1, fi.diag_pairs(24), seed=1, block_len=4).run(17)
        z = oracle.normals(5, 6, np.arange(100), np.arange(100) % 7, 3, np.arange(100) % 5)
        assert np.all(np.isfinite(z))
        print("oracle ok")
    """
    res = run_child(code, {"LD_PRELOAD": f"{rt}:{ub}", "FTH_ORACLE_LIB": lib})
    assert res.returncode == 0 and "oracle ok" in res.stdout, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_1402_2095_amd import build
    rt = build.asan_runtime()
    if not rt:
        pytest.skip("no shared ASan runtime for the HIP compiler in this image")
    lib = build.build_sanitized(str(tmp_path / "libfth_san.so"))
    code = """
        import numpy as np
        import fth_inputs as fi
        from paper_1402_2095_amd import fth
        g = fi.load_gle("fermi_b20_ns4")
        T, S = np.zeros((5, 5)), np.zeros((5, 5))
        import ctypes
        gs, keep = fth._gle_struct(g.A_p, g.C_p)
        assert fth.lib().fth_propagator(ctypes.byref(gs), 0.03, fth._p(T), fth._p(S)) == fth.FTH_OK
        assert np.all(np.isfinite(T)) and np.allclose(np.tril(S), S)
        assert fth.lib().fth_propagator(ctypes.byref(gs), -1.0, fth._p(T), fth._p(S)) == fth.FTH_EINVAL
        r, m = fth.fth_spectral_map(0.1, 12.1, 1.0, 5.0)
        M = fi.banded_spd_csr(500, 3)
        lo, hi = fth.fth_gershgorin(M)
        w = np.array([1.0, 0.0, 500.0])
        e, s = fth.fth_unscale(fth.FTH_TARGET_LN, 0.5, 0.0, 1.2, 0.9, w, np.ones(3), np.ones(3))
        for prec in (fth.FTH_FP32, fth.FTH_FP64):
            assert fth.fth_footprint_bytes(M, 4, 32, 100, True, prec) > 0
        D = fi.dense_ggt(300, 2)
        assert fth.fth_footprint_bytes(D, 4, 64, 10, False, fth.FTH_FP32_BF16X3) > 0
        # every validation failure returns an error code (no device is touched before validation ends)
        bad = []
        Mb = fi.CSR(M.n, M.row_ptr, M.col.copy(), M.val.copy()); Mb.col[5] = M.n + 3; bad.append(Mb)
        Mb = fi.CSR(M.n, M.row_ptr, M.col, M.val.copy()); Mb.val[1] += 0.5; bad.append(Mb)   # not symmetric
        Mb = fi.CSR(M.n, M.row_ptr, M.col, M.val.copy()); Mb.val[0] = -1.0; bad.append(Mb)     # diagonal <= 0
        Db = D.copy(); Db[0, 1] += 1.0; bad.append(Db)
        for Mb in bad:
            try:
                fth.Solver(Mb, g.A_p, g.C_p, 0.05, replicas=8)
                raise AssertionError("accepted an invalid matrix")
            except fth.FthError as ex:
                assert ex.status == fth.FTH_EINVAL, ex
        for kw in (dict(dt=-1.0), dict(pairs=np.array([[0, 10**6]], dtype=np.int32)), dict(block_len=0),
                   dict(temporal_steps=4), dict(precision=7)):
            args = dict(dt=0.05, replicas=8); args.update(kw)
            dt = args.pop("dt")
            try:
                fth.Solver(M, g.A_p, g.C_p, dt, **args)
                raise AssertionError(f"accepted {kw}")
            except fth.FthError as ex:
                assert ex.status == fth.FTH_EINVAL, (kw, ex)
        try:   # valid inputs reach the device query
            fth.Solver(M, g.A_p, g.C_p, 0.05, replicas=8).close()
        except fth.FthError as ex:
            assert ex.status == fth.FTH_EDEVICE, ex
        print(fth.fth_version(), "library host ok")
    """
    res = run_child(code, {"LD_PRELOAD": rt, "FTH_LIB_PATH": lib})
    assert res.returncode == 0 and "library host ok" in res.stdout, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
