// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>

namespace fth {

// Largest number of extra GLE momenta the kernels are instantiated for
// (the paper reports 4 to 10 extra momenta as sufficient, Sec. I).
constexpr int kNsMax = 10;

// Arguments of one fused sparse step launch (one request).
template <typename Real>
struct CsrStepArgs {
    // matrix (CSR)
    const int64_t* row_ptr;
    const int32_t* col;
    const Real* val;
    // state: q ping-pong [N][R]; p and s interleaved per row, ps[N][ns+1][R]
    Real* q0;
    Real* q1;
    Real* ps;
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
    int32_t* flag;  // set to 1 when a non-finite state value appears
    // launch geometry
    int64_t row_tiles;         // tiles of rows
    int64_t row_tiles_padded;  // rounded up to a multiple of 8 (XCD remap)
};

// Launch shape of the sparse step.
struct CsrLaunch {
    int ns;              // extra GLE momenta (template)
    int rpt;             // replicas per thread (template: 1, 2, 4, 8)
    bool nt;             // streaming (non-temporal) state loads/stores (template)
    int block;           // threads per workgroup
    int64_t pair_tiles;  // extra workgroups for the selected pairs
};

// Launch wrappers (defined in the .hip files).
template <typename Real>
int launch_csr_step(const CsrStepArgs<Real>& a, const CsrLaunch& L, int k, void* stream);

int launch_advance(int64_t* step_base, int64_t k, void* stream);

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
