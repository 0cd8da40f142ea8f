// Host-side context of one FTH solve, shared by the C-ABI entry points
// (fth_api.cpp) and the serving layer (fth_server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fth.h"
#include "fth_internal.h"

struct fth_ctx {
    // problem
    int64_t n = 0;
    int fmt = FTH_CSR;
    int prec = FTH_FP32;
    int ns = 0;
    double h = 0.0;
    fth_options opt{};
    int64_t npairs = 0;
    int64_t nnz = 0;
    std::vector<double> T, S;
    // device buffers
    std::vector<void*> allocs;
    int64_t* d_row_ptr = nullptr;
    int32_t* d_col = nullptr;
    void* d_val = nullptr;
    void* d_TS = nullptr;
    int32_t* d_pairs = nullptr;
    // dense: M padded to rows_pad x rows_pad (bf16 hi/lo tiled, or double), split-K partials, bf16 q split
    int64_t rows_pad = 0;
    int ksplit = 1;
    void* d_m_hi = nullptr;
    void* d_part = nullptr;
    uint16_t* d_qt = nullptr;
    bool qt_dirty = true;
    // small dense systems: persistent single-workgroup kernel, M [n][n] in state precision
    bool small = false;
    bool gemv = false;  // dense, R < 16: the force as R matrix-vector products (dense_gemv.hip)
    void* d_msmall = nullptr;
    size_t small_lds = 0;
    int small_m_in_lds = 0;
    std::vector<double> m_host;  // dense M kept until R fixes the path (n <= 4096)
    bool m_uploaded = false;
    void* d_q[2] = {nullptr, nullptr};
    void* d_ps[2] = {nullptr, nullptr};  // p then s_1..s_ns, ping-pong by step parity,
                                         // rows grouped by 2^ps_lg (see ps_offset)
    int ps_lg = 0;         // log2 of rows per (p, s) group
    int64_t ps_rows = 0;   // n rounded up to whole groups
    double* d_acc = nullptr;  // [3][n_out]: blk, s1, s2 (pairs first, then diagonal)
    int64_t* d_step = nullptr;
    int32_t* d_flag = nullptr;
    // coded sparse form: per row 8 one-byte column / value codes into tables
    bool coded = false;
    uint64_t* d_ell_col = nullptr;    // [n]
    uint64_t* d_ell_vcode = nullptr;  // [n] or null
    void* d_ell_vraw = nullptr;       // [n][8] when the values do not fit a table
    int32_t* d_dict_off = nullptr;
    void* d_dict_val = nullptr;
    int32_t n_off = 0, n_val = 0;
    // trace estimators: per-step, per-tile partials [tpart_k][tpart_w][3] and per-step sums
    double* d_tpart = nullptr;
    double* d_tsum = nullptr;
    int32_t tpart_k = 0, tpart_w = 0;
    // temporal blocking of narrow-band CSR systems
    int64_t band_w = -1;   // half-bandwidth max |j - i| of the CSR pattern
    int max_row_nnz = 0;   // longest CSR row
    int tb_kt = 0;         // steps per blocked launch, 0: one-step kernels
    int tb_block = 1024;   // threads per blocked workgroup
    int32_t* d_pair_slot = nullptr;    // [n]: snapshot slot of a row in a pair, or -1
    int32_t* d_pair_slots = nullptr;   // [npairs][2]
    void* d_snap = nullptr;            // [kTbMaxSteps][2][nslots][R]
    int64_t tb_nslots = 0;
    void* d_tb_slots = nullptr;        // slot form of the rows (TbSlotRow) for the persistent form
    int tbp_grid = 0;                  // workgroups of the persistent blocked step, 0: one per tile
    // schedule
    int R = 0;
    int rpt = 0;
    bool nt = false;  // streaming state access (state larger than the Infinity Cache)
    int block = 256;
    bool tuned = false;     // launch shape chosen by the autotuner
    double tuned_us = 0.0;  // its measured step time
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipGraphExec_t gexec = nullptr;
    int gK = 0;
    int64_t step = 0;
    bool poisoned = false;
    uint64_t m_hash = 0;     // hash of the matrix as used (recorded in state images)
    uint64_t pair_hash = 0;  // hash of the selected pairs
    double last_ms = 0.0;
    int device = 0;

    fth_allocator hook{};      // caller's device allocator (alloc == NULL: hipMalloc / hipFree)
    std::vector<size_t> alloc_bytes;  // sizes of allocs, same order

    ~fth_ctx() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (stream) (void)hipStreamSynchronize(stream);
        for (void* p : allocs) raw_free(p);
        if (stream) (void)hipStreamDestroy(stream);
    }

    // Device memory through the caller's allocator when one is given.
    void* raw_alloc(size_t bytes) {
        if (hook.alloc) return hook.alloc(bytes, hook.user);
        void* p = nullptr;
        return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
    }
    void raw_free(void* p) {
        if (!p) return;
        if (hook.alloc) {
            if (hook.release) hook.release(p, hook.user);
        } else {
            (void)hipFree(p);
        }
    }
    size_t device_bytes() const {
        size_t s = 0;
        for (size_t b : alloc_bytes) s += b;
        return s;
    }

    size_t real_bytes() const { return prec == FTH_FP64 ? 8 : 4; }
    bool dense() const { return fmt == FTH_DENSE; }
    bool mfma() const { return dense() && !small; }
    int64_t q_rows() const { return mfma() ? rows_pad : n; }
    // accumulated estimates: q-q pairs, q-q diagonal, then the same for p-p if kept
    int64_t n_kind() const { return npairs + (opt.acc_diag ? n : 0); }
    int ntr() const { return opt.acc_trace ? (opt.acc_pp ? 3 : 2) : 0; }  // trace estimators
    int64_t n_out() const { return n_kind() * (opt.acc_pp ? 2 : 1) + ntr(); }
    size_t ps_bytes() const { return size_t(ps_rows) * size_t(R) * size_t(ns + 1) * real_bytes(); }
    // element offset of (row i, component c, replica r) in the (p, s) buffer:
    // groups of 2^ps_lg rows, each component of a group a contiguous [2^ps_lg][R] block
    size_t ps_offset(int64_t i, int c, int r) const {
        const int64_t g = i >> ps_lg, w = i & ((int64_t(1) << ps_lg) - 1);
        return size_t((((g * (ns + 1) + c) << ps_lg) + w) * R + r);
    }

    void dfree(void*& p) {
        for (size_t k = 0; k < allocs.size(); ++k)
            if (allocs[k] == p) {
                allocs.erase(allocs.begin() + long(k));
                alloc_bytes.erase(alloc_bytes.begin() + long(k));
                raw_free(p);
                break;
            }
        p = nullptr;
    }

    hipError_t dalloc(void** p, size_t bytes) {
        if (bytes == 0) bytes = 256;
        *p = raw_alloc(bytes);
        if (!*p) return hipErrorOutOfMemory;
        allocs.push_back(*p);
        alloc_bytes.push_back(bytes);
        return hipSuccess;
    }
};

// Scratch device memory for the duration of one call (freed on scope exit).
struct ctx_scratch {
    fth_ctx* c;
    std::vector<void*> p;
    explicit ctx_scratch(fth_ctx* ctx) : c(ctx) {}
    ~ctx_scratch() {
        for (void* x : p) c->raw_free(x);
    }
    void* get(size_t bytes) {
        void* x = c->raw_alloc(bytes);
        if (x) p.push_back(x);
        return x;
    }
};

namespace fth {
namespace host {

fth_status fail(fth_status st, const char* fmt, ...);
// 64-bit hash of a byte range (FNV-1a over 8-byte words, then the tail
// bytes), continuing from seed (0: a fresh hash).  Identifies inputs in
// state images; not a checksum against deliberate changes.
uint64_t hash_words(const void* p, size_t bytes, uint64_t seed);
extern thread_local std::string g_last_error;

fth_status check_csr(const fth_matrix* M);
// M' = r M + m I into store (FP64 values; the CSR pattern is shared with M).
fth_status spectral_transform(const fth_matrix* M, double r, double m, std::vector<double>& store, fth_matrix* out);
// A' = alpha A_p, C' = gamma C_p into A, C.
fth_status scaled_gle(const fth_gle* g, double alpha, double gamma, std::vector<double>& A, std::vector<double>& C,
                      fth_gle* out);
fth_status check_dense(const fth_matrix* M);
fth_status make_propagator(const fth_gle* g, double dt, std::vector<double>& T, std::vector<double>& S);
// Allocate (and zero) the state for R replicas; fixes R and the launch shape.
fth_status ensure_state(fth_ctx* c, int32_t R);
template <typename Real>
fth::StepArgs<Real> step_args(fth_ctx* c);
fth::StepLaunch step_launch(fth_ctx* c);
// Enqueue K steps (no graph) followed by the step-counter advance.
fth_status enqueue_chunk(fth_ctx* c, int K);
// Temporal blocking: whether the CSR system qualifies for KT steps per launch
// with the given workgroup size, and the device buffers it needs.
bool tb_eligible(const fth_ctx* c, int KT, int block);
fth_status tb_prepare(fth_ctx* c);
// Trace partial buffers large enough for chunks of K steps in the current
// launch shape (reallocated, and the graph dropped, when they must grow).
fth_status trace_prepare(fth_ctx* c, int K);
// Enqueue K steps of a small dense system (persistent kernel).
fth_status enqueue_small(fth_ctx* c, int64_t nsteps);
// Enqueue nsteps steps on the context's stream (graphs, tails, small path).
fth_status run_enqueue(fth_ctx* c, int64_t nsteps);
// Wait for the context's stream, count the steps, check the non-finite flag.
fth_status run_complete(fth_ctx* c, int64_t nsteps);

}  // namespace host
}  // namespace fth

// Return an fth_status (with a message) from a failed HIP runtime call.
#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? FTH_ENOMEM : FTH_EDEVICE, "%s: %s", #expr, \
                        hipGetErrorString(e_));                                               \
    } while (0)
