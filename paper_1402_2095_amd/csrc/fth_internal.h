// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>

namespace fth {

// Largest number of extra GLE momenta the kernels are instantiated for
// (the paper reports 4 to 10 extra momenta as sufficient, Sec. I).
constexpr int kNsMax = 10;

// Arguments of one step launch of one request (sparse step or dense
// epilogue); fields that a kernel does not use are ignored.
template <typename Real>
struct StepArgs {
    // force source, sparse: CSR rows
    const int64_t* row_ptr;
    const int32_t* col;
    const Real* val;
    // force source, sparse, coded form (rows of at most 8 entries, CSR order): per row
    // 8 one-byte column codes (255: empty slot) into the table of distinct offsets
    // j - i, and 8 one-byte value codes into the table of distinct values, or, when
    // the values do not fit a table, 8 raw values per row
    const uint64_t* ell_col;   // [N], null: plain CSR
    const uint64_t* ell_vcode; // [N], null: raw values in ell_vraw
    const Real* ell_vraw;      // [N][8]
    const int32_t* dict_off;   // [n_off]
    const Real* dict_val;      // [n_val]
    int32_t n_off, n_val;
    // force source, dense: split-K partial sums [ksplit][rows_pad][R] of M q_n
    const Real* part;
    int32_t ksplit;
    int64_t rows_pad;
    // dense split-BF16x3 only: q_{n+1} split into bf16 hi/lo, tiled [rows_pad/8][R][2][8]
    uint16_t* qt;
    // small dense systems: M column-major (element (i, j) at j * N + i) in state precision;
    // kept in LDS if m_in_lds
    const Real* mdense;
    int32_t m_in_lds;
    // state: q ping-pong [rows][R]; (p, s) ping-pong as well (step n reads buffer
    // n & 1 and writes the other), each in groups of 2^ps_lg rows, component-major
    // inside a group: ps[row >> ps_lg][ns+1][row & (2^ps_lg - 1)][R] (p is component 0)
    Real* q0;
    Real* q1;
    Real* ps;    // buffer 0
    Real* ps_b;  // buffer 1
    int32_t ps_lg;
    // propagator T then S, each (ns+1)^2 row-major, state precision
    const Real* TS;
    Real h;
    Real hh;  // h / 2
    int64_t N;
    int32_t R;
    int32_t lg_tpr;  // log2(threads per row) = log2(R / replicas per thread)
    // noise
    uint32_t key0, key1, stream;
    // step bookkeeping: global step n = *step_base + k (k: launch argument)
    const int64_t* step_base;
    int64_t burn_in;
    int64_t block_len;
    // accumulators (FP64): diagonal (length N, or null) and pairs
    double* dblk;
    double* ds1;
    double* ds2;
    const int32_t* pairs;  // [npairs][2]
    int64_t npairs;
    double* pblk;
    double* ps1;
    double* ps2;
    // p-p accumulators (p_n, sampled with q_n) for the same pairs and diagonal; null if not kept
    double* pp_blk;
    double* pp_s1;
    double* pp_s2;
    double* dp_blk;
    double* dp_s1;
    double* dp_s2;
    // trace partials (null if traces are not kept): for in-chunk step k and row
    // tile t, tpart[(k * tpart_w + t) * 3 + c] = sum over the tile's rows and
    // replicas of q^2 (c = 0), q (M q) (c = 1) and p^2 (c = 2)
    double* tpart;
    int32_t tpart_w;
    int32_t* flag;  // set to 1 when a non-finite state value appears
    int32_t ns;     // extra GLE momenta
    // launch geometry
    int64_t row_tiles;         // tiles of rows
    int64_t row_tiles_padded;  // rounded up to a multiple of 8 (XCD remap)

    __host__ __device__ int D() const { return ns + 1; }
};

// Launch shape of a step kernel.
constexpr int kCodedSlots = 8;       // entries per row of the coded sparse form
constexpr int kCodedMaxOffsets = 255;  // distinct column offsets (code 255 marks an empty slot)
constexpr int kCodedMaxValues = 256;   // distinct values held in a table

struct StepLaunch {
    int ns;              // extra GLE momenta (template)
    int rpt;             // replicas per thread (template: 1, 2, 4, 8)
    bool nt;             // streaming (non-temporal) state loads/stores (template)
    bool coded;          // coded sparse form (template; replicas per thread 4 or 8)
    bool long_rows;      // plain CSR with long-row gather batches (template; replicas per thread 4 or 8)
    int block;           // threads per workgroup
    int64_t pair_tiles;  // extra workgroups for the selected pairs
};

// Arguments of the dense split-K force GEMM  part[ks] = M[:, kslice] q_n[kslice, :].
struct DenseGemmArgs {
    const void* m_hi;     // split form: bf16 hi and lo parts of M, tiled (see dense.hpp);
                          // FP64 form: double [rows_pad][rows_pad]
    const uint16_t* qt;   // split form: q_n as bf16 hi/lo, tiled [rows_pad/8][R][2][8]
    const void* q0;       // FP64 form: q ping-pong buffers [rows_pad][R] (double)
    const void* q1;
    const int64_t* step_base;
    int32_t k;            // in-chunk step offset
    void* part;           // [ksplit][rows_pad][R] float (split form) or double
    int64_t rows_pad;
    int32_t R;
    int32_t ksplit;
    int64_t kslice;       // rows_pad / ksplit
};

// Largest workgroup of the temporally blocked step: a row's (p, s) and CSR
// entries stay in registers for the whole launch, so larger NS (and FP64)
// need the register file of fewer threads.
// Momentum-form and trace accumulators (xtra) need more registers: with
// them, 1024 threads only for FP32 at ns <= 4, where the compiler spills
// some of the row's data and reloads it each step (correct, but slower than
// the one-step kernel on the banded shapes measured).
constexpr int tb_max_block(bool f64, int ns, bool xtra = false) {
    const int b = f64 ? (ns == 0 ? 1024 : ns <= 4 ? 512 : 256) : (ns <= 4 ? 1024 : ns <= 9 ? 512 : 256);
    return xtra && b > 512 && (f64 || ns > 4) ? 512 : b;
}

// Extra arguments of the temporally blocked sparse step.
template <typename Real>
struct TbArgs {
    int32_t E;                 // extended rows per workgroup
    int32_t T;                 // output rows per workgroup
    int32_t w;                 // half-bandwidth of M
    const int32_t* pair_slot;  // [N]: snapshot slot of a row used by a pair, or -1
    Real* snap;                // [KT][2][nslots][R]: q (and p, if kept) of pair rows at each step
    int64_t nslots;
    const int32_t* pair_slots; // [npairs][2]: snapshot slots of each pair's rows
    // persistent form: the slot form of the rows (TbSlotRow<Real>[N], null: the
    // one-launch-per-tile form) and the workgroups of the persistent grid
    const void* slots;
    int32_t grid;
};

// Slot form of a CSR row of at most 8 entries for the persistent blocked
// step: values in stored order (unused slots 0), column offsets j - i as
// signed bytes, the entry count; a whole number of 16-byte chunks, so a wave
// stages its rows with 16-byte direct-to-LDS loads.
template <typename Real>
struct TbSlotRow {
    Real val[8];
    int8_t off[8];
    int32_t nz;
    int32_t pad;
};
static_assert(sizeof(TbSlotRow<float>) % 16 == 0 && sizeof(TbSlotRow<double>) % 16 == 0, "slot rows are 16-byte chunks");

// Bookkeeping words a wave stages per tile with 4-byte direct-to-LDS loads
// (256 bytes each): the diagonal block sum (two words) and the pair snapshot
// slot.  (The momentum-form block sum is prefetched into a register.)
constexpr int kTbpAuxWords = 3;

// LDS bytes of the persistent blocked step for a workgroup of `block`
// threads (4 replicas per thread): q of the extended rows twice, the trace
// row sums (if kept), each wave's staging area (state, slot rows and
// bookkeeping of the next tile) and, with the momentum or trace
// accumulators (xtra), the extended rows' matrix values.
constexpr size_t tbp_lds_bytes(bool f64, int ns, int block, int R, int T, bool traces, bool xtra) {
    const size_t rb = f64 ? 8 : 4;
    const size_t E = size_t(block) * 4 / size_t(R);
    const size_t q = 2 * E * size_t(R) * rb;
    const size_t tr = traces ? 2 * size_t(T) * 3 * 8 : 0;
    const size_t vi = 4 * rb / 16;                       // 16-byte loads per 4-replica vector
    const size_t rows_per_wave = 64 / (size_t(R) / 4);
    const size_t sb = f64 ? sizeof(TbSlotRow<double>) : sizeof(TbSlotRow<float>);
    const size_t ci = (rows_per_wave * sb + 1023) / 1024;  // slot-row loads per wave
    const size_t stage = (size_t(block) / 64) * ((size_t(ns + 2) * vi + ci) * 1024 + size_t(kTbpAuxWords) * 256);
    const size_t vals = xtra ? E * 8 * rb : 0;
    return q + tr + stage + vals;
}

// One entry of the packed multi-request work list.
struct PackedTile {
    int32_t slot;   // request slot in the table
    int32_t pairs;  // 0: row tile, 1: pair tile
    int64_t index;  // tile index within the request
};

// Launch wrappers (defined in the .hip files).
template <typename Real>
int launch_csr_step(const StepArgs<Real>& a, const StepLaunch& L, int k, void* stream);
template <typename Real>  // the instantiations with trace partials
int launch_csr_step_traced(const StepArgs<Real>& a, const StepLaunch& L, int k, void* stream);
template <typename Real>
int launch_dense_epilogue(const StepArgs<Real>& a, const StepLaunch& L, int k, void* stream);
int launch_gemm_bf16x3(const DenseGemmArgs& g, void* stream);
int launch_gemm_f64(const DenseGemmArgs& g, void* stream);
// Dense force for R in {1, 2, 4, 8}: part[i][r] = (M q_n)_ir with M row-major [N][ld]
// (ld a multiple of 4, >= N, <= g.rows_pad) in the state precision.
template <typename Real>
int launch_dense_gemv(const DenseGemmArgs& g, const Real* M, int64_t N, int64_t ld, void* stream);
// M [P][P] FP32 -> bf16 hi/lo parts in the split GEMM's tiled layout (4 P^2 bytes at mt).
int launch_split_bf16_tiled(const float* m, void* mt, int64_t P, void* stream);
int launch_qt_from_q(const float* q, uint16_t* qt, int64_t N, int64_t rows_pad, int32_t R, void* stream);
int launch_advance(int64_t* step_base, int64_t k, void* stream);
// Trace estimators: sum the per-tile partials of K steps (fixed order), fold
// them into the trace accumulators in step order and clear the partials.
// Step k of the chunk is global step *step_base + shift + k.
int launch_trace_fold(double* tpart, double* tsum, int K, int W, int ntr, double* blk, double* s1, double* s2,
                      const int64_t* step_base, int64_t shift, int64_t burn_in, int64_t block_len, void* stream);
// Temporally blocked step: one launch advances KT steps (KT odd); pairs follow.
template <typename Real>
int launch_tb_step(const StepArgs<Real>& a, const TbArgs<Real>& tb, const StepLaunch& L, int KT, int k, void* stream);
template <typename Real>
int launch_tb_pairs(const StepArgs<Real>& a, const TbArgs<Real>& tb, const StepLaunch& L, int KT, int k, void* stream);
// Persistent form of the blocked step (tb.slots and tb.grid set): one
// workgroup per slot of the grid walks a contiguous range of row tiles.
template <typename Real>
int launch_tbp_step(const StepArgs<Real>& a, const TbArgs<Real>& tb, const StepLaunch& L, int KT, int k, void* stream);
// Workgroups of the persistent blocked step that fit on the device at once
// (0 if the shape does not fit); lds = tbp_lds_bytes of the shape.
template <typename Real>
int tbp_resident_grid(int ns, int KT, bool xtra, int block, size_t lds);
// Slot form of CSR rows (at most 8 entries each) for the persistent blocked step.
template <typename Real>
int launch_tb_slots(const int64_t* row_ptr, const int32_t* col, const Real* val, int64_t N, void* out, void* stream);
int launch_packed_csr(const StepArgs<float>* table, const PackedTile* tiles, const int32_t* ntiles, int ns, bool nt,
                      int grid, int k, void* stream);
int launch_advance_all(const StepArgs<float>* table, const int32_t* nslots, int64_t K, void* stream);
// One workgroup advances a small dense system by K steps (and the step counter).
template <typename Real>
int launch_small_dense(const StepArgs<Real>& a, const StepLaunch& L, int K, size_t lds_bytes, void* stream);

// Host FP64 linear algebra (fth_linalg.cpp).
namespace la {
// exp(A) for an n x n row-major matrix (scaling and squaring with a
// diagonal Pade approximant).  Returns false on non-finite input.
bool expm(const double* A, int n, double* out);
// Lower Cholesky factor L of a symmetric matrix; false if not positive
// definite (pivot <= tol * max diagonal).
bool cholesky(const double* A, int n, double* L, double rel_tol);
// Eigenvalues of a symmetric matrix (cyclic Jacobi).
void sym_eigvals(const double* A, int n, double* ev);
}  // namespace la

}  // namespace fth
