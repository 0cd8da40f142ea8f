// C ABI of the f-thermostat library: validation, per-solve setup (T, S in
// FP64), device memory, the captured step schedule, and result readout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <map>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "fth_ctx.hpp"

namespace fth {
namespace host {

thread_local std::string g_last_error;

fth_status fail(fth_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}


uint64_t hash_words(const void* p, size_t bytes, uint64_t seed) {
    uint64_t h = seed ? seed : 1469598103934665603ull;
    const unsigned char* b = static_cast<const unsigned char*>(p);
    size_t k = 0;
    for (; k + 8 <= bytes; k += 8) {
        uint64_t w;
        std::memcpy(&w, b + k, 8);
        h = (h ^ w) * 1099511628211ull;
    }
    for (; k < bytes; ++k) h = (h ^ b[k]) * 1099511628211ull;
    return h;
}

constexpr int kDefaultGraphSteps = 64;
constexpr int kTbMaxSteps = 5;   // longest temporally blocked launch (snapshot depth)
constexpr int64_t kTbMaxW = 16;  // widest half-bandwidth blocked

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int64_t x) {
    int r = 0;
    while ((int64_t(1) << r) < x) ++r;
    return r;
}


// ------------------------------------------------------------------ checks
fth_status check_csr(const fth_matrix* M) {
    const int64_t n = M->n, nnz = M->nnz;
    if (!M->row_ptr || !M->col || !M->val) return fail(FTH_EINVAL, "CSR arrays must not be NULL");
    if (M->row_ptr[0] != 0 || M->row_ptr[n] != nnz) return fail(FTH_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] == nnz");
    auto val = [&](int64_t k) {
        return M->value_is_f64 ? static_cast<const double*>(M->val)[k] : double(static_cast<const float*>(M->val)[k]);
    };
    double vmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t b = M->row_ptr[i], e = M->row_ptr[i + 1];
        if (e < b) return fail(FTH_EINVAL, "row_ptr decreases at row %lld", (long long)i);
        bool diag = false;
        for (int64_t k = b; k < e; ++k) {
            const int32_t c = M->col[k];
            if (c < 0 || c >= n) return fail(FTH_EINVAL, "column index out of range in row %lld", (long long)i);
            if (k > b && c <= M->col[k - 1]) return fail(FTH_EINVAL, "columns not strictly increasing in row %lld", (long long)i);
            const double v = val(k);
            if (!std::isfinite(v)) return fail(FTH_EINVAL, "non-finite value in row %lld", (long long)i);
            vmax = std::max(vmax, std::fabs(v));
            if (c == i) {
                if (!(v > 0)) return fail(FTH_EINVAL, "diagonal entry of row %lld is not positive", (long long)i);
                diag = true;
            }
        }
        if (!diag) return fail(FTH_EINVAL, "missing diagonal entry in row %lld", (long long)i);
    }
    const double tol = (M->value_is_f64 ? 1e-12 : 1e-6) * vmax;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = M->row_ptr[i]; k < M->row_ptr[i + 1]; ++k) {
            const int32_t j = M->col[k];
            if (j == i) continue;
            const int32_t* b = M->col + M->row_ptr[j];
            const int32_t* e = M->col + M->row_ptr[j + 1];
            const int32_t* f = std::lower_bound(b, e, int32_t(i));
            if (f == e || *f != i) return fail(FTH_EINVAL, "CSR pattern not symmetric at (%lld, %d)", (long long)i, j);
            if (std::fabs(val(f - M->col) - val(k)) > tol)
                return fail(FTH_EINVAL, "CSR values not symmetric at (%lld, %d)", (long long)i, j);
        }
    }
    return FTH_OK;
}

fth_status check_dense(const fth_matrix* M) {
    const int64_t n = M->n;
    if (!M->dense) return fail(FTH_EINVAL, "dense pointer must not be NULL");
    auto at = [&](int64_t i, int64_t j) {
        return M->value_is_f64 ? static_cast<const double*>(M->dense)[i * n + j]
                               : double(static_cast<const float*>(M->dense)[i * n + j]);
    };
    double vmax = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            const double v = at(i, j);
            if (!std::isfinite(v)) return fail(FTH_EINVAL, "non-finite matrix entry (%lld, %lld)", (long long)i, (long long)j);
            vmax = std::max(vmax, std::fabs(v));
        }
    const double tol = (M->value_is_f64 ? 1e-12 : 1e-6) * vmax;
    for (int64_t i = 0; i < n; ++i) {
        if (!(at(i, i) > 0)) return fail(FTH_EINVAL, "diagonal entry %lld is not positive", (long long)i);
        for (int64_t j = 0; j < i; ++j)
            if (std::fabs(at(i, j) - at(j, i)) > tol)
                return fail(FTH_EINVAL, "dense matrix not symmetric at (%lld, %lld)", (long long)i, (long long)j);
    }
    return FTH_OK;
}

// GLE validity and the exact OU propagator (T = exp(-A_p h), S S^T = C_p - T C_p T^T).
fth_status make_propagator(const fth_gle* g, double dt, std::vector<double>& T, std::vector<double>& S) {
    if (!g || !g->A_p || !g->C_p) return fail(FTH_EINVAL, "GLE parameters must not be NULL");
    if (g->ns < 0 || g->ns > 64) return fail(FTH_EINVAL, "ns must be in [0, 64]");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(FTH_EINVAL, "dt must be positive and finite");
    const int d = g->ns + 1;
    const double* A = g->A_p;
    const double* C = g->C_p;
    double cmax = 0.0;
    for (int i = 0; i < d * d; ++i) {
        if (!std::isfinite(A[i]) || !std::isfinite(C[i])) return fail(FTH_EINVAL, "non-finite GLE parameter");
        cmax = std::max(cmax, std::fabs(C[i]));
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < i; ++j)
            if (std::fabs(C[i * d + j] - C[j * d + i]) > 1e-10 * std::max(1.0, cmax))
                return fail(FTH_EINVAL, "C_p is not symmetric");
    std::vector<double> L(d * d), BB(d * d), ev(d);
    if (!fth::la::cholesky(C, d, L.data(), 0.0)) return fail(FTH_EINVAL, "C_p is not positive definite");
    double bbmax = 0.0;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double v = 0.0;
            for (int k = 0; k < d; ++k) v += A[i * d + k] * C[k * d + j] + C[i * d + k] * A[j * d + k];
            BB[i * d + j] = v;
        }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < i; ++j) BB[i * d + j] = BB[j * d + i] = 0.5 * (BB[i * d + j] + BB[j * d + i]);
    fth::la::sym_eigvals(BB.data(), d, ev.data());
    for (double e : ev) bbmax = std::max(bbmax, std::fabs(e));
    for (double e : ev)
        if (e < -1e-10 * std::max(1.0, bbmax)) return fail(FTH_EINVAL, "A_p C_p + C_p A_p^T is not positive semi-definite");

    std::vector<double> mA(d * d);
    for (int i = 0; i < d * d; ++i) mA[i] = -A[i] * dt;
    T.assign(d * d, 0.0);
    S.assign(d * d, 0.0);
    if (!fth::la::expm(mA.data(), d, T.data())) return fail(FTH_EINVAL, "exp(-A_p dt) failed");
    std::vector<double> TC(d * d), sig(d * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double v = 0.0;
            for (int k = 0; k < d; ++k) v += T[i * d + k] * C[k * d + j];
            TC[i * d + j] = v;
        }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double v = 0.0;
            for (int k = 0; k < d; ++k) v += TC[i * d + k] * T[j * d + k];
            sig[i * d + j] = C[i * d + j] - v;
        }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < i; ++j) sig[i * d + j] = sig[j * d + i] = 0.5 * (sig[i * d + j] + sig[j * d + i]);
    if (!fth::la::cholesky(sig.data(), d, S.data(), 1e-13))
        return fail(FTH_EINVAL, "C_p - T C_p T^T is not positive definite for this dt");
    return FTH_OK;
}

template <typename Real>
fth_status upload_converted(fth_ctx* c, void** dst, const void* src, int64_t count, bool src_f64) {
    std::vector<Real> tmp(size_t(std::max<int64_t>(count, 1)));
    for (int64_t k = 0; k < count; ++k)
        tmp[k] = src_f64 ? Real(static_cast<const double*>(src)[k]) : Real(static_cast<const float*>(src)[k]);
    HIP_OK(c->dalloc(dst, sizeof(Real) * size_t(count)));
    HIP_OK(hipMemcpy(*dst, tmp.data(), sizeof(Real) * size_t(count), hipMemcpyHostToDevice));
    return FTH_OK;
}

// Coded copy of a CSR matrix with at most 8 entries per row: one-byte codes
// into the tables of distinct column offsets j - i and distinct values (at
// state precision), slots in CSR order.  Left out (plain CSR only) when there
// are more than 255 distinct offsets; values stay raw when there are more
// than 256 distinct ones.
template <typename Real>
fth_status build_coded(fth_ctx* c, const fth_matrix* M) {
    const int64_t n = M->n;
    std::map<int64_t, int32_t> offs;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = M->row_ptr[i]; k < M->row_ptr[i + 1]; ++k) {
            offs.emplace(int64_t(M->col[k]) - i, 0);
            if (int(offs.size()) > fth::kCodedMaxOffsets) return FTH_OK;
        }
    std::vector<int32_t> off_tab;
    for (auto& kv : offs) {
        kv.second = int32_t(off_tab.size());
        off_tab.push_back(int32_t(kv.first));
    }
    auto value = [&](int64_t k) -> Real {
        return M->value_is_f64 ? Real(static_cast<const double*>(M->val)[k]) : Real(static_cast<const float*>(M->val)[k]);
    };
    // distinct values by bit pattern (so -0 and +0 stay distinct, NaN cannot occur: M is validated)
    using Bits = typename std::conditional<sizeof(Real) == 8, uint64_t, uint32_t>::type;
    std::map<Bits, int32_t> vals;
    bool vtab = true;
    for (int64_t k = 0; k < M->nnz && vtab; ++k) {
        const Real v = value(k);
        Bits b;
        std::memcpy(&b, &v, sizeof(b));
        vals.emplace(b, 0);
        vtab = int(vals.size()) <= fth::kCodedMaxValues;
    }
    std::vector<Real> val_tab;
    if (vtab)
        for (auto& kv : vals) {
            kv.second = int32_t(val_tab.size());
            Real v;
            std::memcpy(&v, &kv.first, sizeof(v));
            val_tab.push_back(v);
        }
    std::vector<uint64_t> cc(static_cast<size_t>(n)), vc(vtab ? static_cast<size_t>(n) : 0);
    std::vector<Real> vraw(vtab ? 0 : size_t(n) * fth::kCodedSlots, Real(0));
    for (int64_t i = 0; i < n; ++i) {
        uint64_t ccode = ~uint64_t(0), vcode = 0;
        for (int64_t k = M->row_ptr[i], u = 0; k < M->row_ptr[i + 1]; ++k, ++u) {
            const uint64_t oc = uint64_t(offs[int64_t(M->col[k]) - i]);
            ccode = (ccode & ~(uint64_t(255) << (8 * u))) | (oc << (8 * u));
            const Real v = value(k);
            if (vtab) {
                Bits b;
                std::memcpy(&b, &v, sizeof(b));
                vcode |= uint64_t(vals[b]) << (8 * u);
            } else {
                vraw[size_t(i) * fth::kCodedSlots + size_t(u)] = v;
            }
        }
        cc[size_t(i)] = ccode;
        if (vtab) vc[size_t(i)] = vcode;
    }
    HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_ell_col), sizeof(uint64_t) * cc.size()));
    HIP_OK(hipMemcpy(c->d_ell_col, cc.data(), sizeof(uint64_t) * cc.size(), hipMemcpyHostToDevice));
    HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_dict_off), sizeof(int32_t) * off_tab.size()));
    HIP_OK(hipMemcpy(c->d_dict_off, off_tab.data(), sizeof(int32_t) * off_tab.size(), hipMemcpyHostToDevice));
    c->n_off = int32_t(off_tab.size());
    if (vtab) {
        HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_ell_vcode), sizeof(uint64_t) * vc.size()));
        HIP_OK(hipMemcpy(c->d_ell_vcode, vc.data(), sizeof(uint64_t) * vc.size(), hipMemcpyHostToDevice));
        HIP_OK(c->dalloc(&c->d_dict_val, sizeof(Real) * val_tab.size()));
        HIP_OK(hipMemcpy(c->d_dict_val, val_tab.data(), sizeof(Real) * val_tab.size(), hipMemcpyHostToDevice));
        c->n_val = int32_t(val_tab.size());
    } else {
        HIP_OK(c->dalloc(&c->d_ell_vraw, sizeof(Real) * vraw.size()));
        HIP_OK(hipMemcpy(c->d_ell_vraw, vraw.data(), sizeof(Real) * vraw.size(), hipMemcpyHostToDevice));
    }
    c->coded = true;
    return FTH_OK;
}

template <typename Real>
fth_status upload_TS(fth_ctx* c) {
    const int d = c->ns + 1;
    std::vector<Real> ts(2 * d * d);
    for (int i = 0; i < d * d; ++i) {
        ts[i] = Real(c->T[i]);
        ts[d * d + i] = Real(c->S[i]);
    }
    HIP_OK(c->dalloc(&c->d_TS, sizeof(Real) * ts.size()));
    HIP_OK(hipMemcpy(c->d_TS, ts.data(), sizeof(Real) * ts.size(), hipMemcpyHostToDevice));
    return FTH_OK;
}

// Padded size of a dense M: a multiple of 256, and of 512 from 2048 on, where
// the split-K GEMM cuts K into 8 slices that must each be whole 64-wide k-steps.
int64_t dense_rows_pad(int64_t n) {
    const int64_t p = (n + 255) / 256 * 256;
    return p >= 2048 ? (n + 511) / 512 * 512 : p;
}

// K slices of the dense force GEMM.  FP64: 8 from 2048 rows on.  Split form:
// the largest power of two <= 8 that keeps the grid at or under 512
// workgroups of 128 rows (two per CU, one round): fewer slices mean fewer
// partial sums for the epilogue to read (16384 rows: 4 slices).
int dense_ksplit(int64_t P, int prec) {
    if (P < 2048) return int(P / 256);
    int ks = 8;
    if (prec == FTH_FP32_BF16X3)
        while (ks > 1 && (P / 128) * ks > 512) ks /= 2;
    return ks;
}

// Dense M padded to rows_pad x rows_pad with zeros: bf16 hi/lo split on the
// device for the split form, FP64 as is.
fth_status upload_dense(fth_ctx* c, const std::vector<double>& M) {
    const int64_t n = c->n;
    c->rows_pad = dense_rows_pad(n);
    const int64_t P = c->rows_pad;
    c->ksplit = dense_ksplit(P, c->prec);
    const size_t cnt = size_t(P) * size_t(P);
    if (c->prec == FTH_FP64) {
        HIP_OK(c->dalloc(&c->d_m_hi, cnt * sizeof(double)));
        HIP_OK(hipMemset(c->d_m_hi, 0, cnt * sizeof(double)));
        HIP_OK(hipMemcpy2D(c->d_m_hi, size_t(P) * 8, M.data(), size_t(n) * 8, size_t(n) * 8, size_t(n),
                           hipMemcpyHostToDevice));
        return FTH_OK;
    }
    if (c->prec != FTH_FP32_BF16X3)
        return fail(FTH_EUNSUPPORTED,
                    "dense systems beyond one workgroup use FTH_FP32_BF16X3 or FTH_FP64 (FTH_FP32 needs replicas <= 8)");
    ctx_scratch scratch(c);
    float* tmp = static_cast<float*>(scratch.get(cnt * sizeof(float)));
    if (!tmp) return fail(FTH_ENOMEM, "scratch allocation for the bf16 split failed");
    HIP_OK(hipMemset(tmp, 0, cnt * sizeof(float)));
    {
        std::vector<float> mf(size_t(n) * size_t(n));
        for (size_t k = 0; k < mf.size(); ++k) mf[k] = float(M[k]);
        HIP_OK(hipMemcpy2D(tmp, size_t(P) * 4, mf.data(), size_t(n) * 4, size_t(n) * 4, size_t(n),
                           hipMemcpyHostToDevice));
    }
    HIP_OK(c->dalloc(&c->d_m_hi, cnt * 2 * sizeof(uint16_t)));  // hi and lo parts, tiled
    if (fth::launch_split_bf16_tiled(tmp, c->d_m_hi, P, c->stream) != 0)
        return fail(FTH_EDEVICE, "bf16 split launch failed");
    HIP_OK(hipStreamSynchronize(c->stream));
    return FTH_OK;
}

// Small dense systems: M [n][n] in the state precision for the persistent kernel,
// column-major, so that the threads of consecutive rows read consecutive words
// (M is only symmetric to the validation tolerance, so the copy is a transpose).
fth_status upload_small(fth_ctx* c, const std::vector<double>& M) {
    const size_t cnt = M.size();
    const size_t n = size_t(c->n);
    if (c->prec == FTH_FP64) {
        std::vector<double> mt(cnt);
        for (size_t i = 0; i < n; ++i)
            for (size_t j = 0; j < n; ++j) mt[j * n + i] = M[i * n + j];
        HIP_OK(c->dalloc(&c->d_msmall, cnt * sizeof(double)));
        HIP_OK(hipMemcpy(c->d_msmall, mt.data(), cnt * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> mf(cnt);
        for (size_t i = 0; i < n; ++i)
            for (size_t j = 0; j < n; ++j) mf[j * n + i] = float(M[i * n + j]);
        HIP_OK(c->dalloc(&c->d_msmall, cnt * sizeof(float)));
        HIP_OK(hipMemcpy(c->d_msmall, mf.data(), cnt * sizeof(float), hipMemcpyHostToDevice));
    }
    return FTH_OK;
}

// Dense M for the few-replica force (R < 16): row-major in the state precision
// (FP32 for both FP32 forms), ld = n rounded up to 4, zero columns past n.
fth_status upload_gemv(fth_ctx* c, const std::vector<double>& M) {
    const int64_t n = c->n, ld = (n + 3) / 4 * 4;
    c->rows_pad = ld;
    c->ksplit = 1;
    c->gemv = true;
    const size_t cnt = size_t(n) * size_t(ld);
    if (c->prec == FTH_FP64) {
        std::vector<double> m(cnt, 0.0);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) m[size_t(i * ld + j)] = M[size_t(i * n + j)];
        HIP_OK(c->dalloc(&c->d_m_hi, cnt * sizeof(double)));
        HIP_OK(hipMemcpy(c->d_m_hi, m.data(), cnt * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> m(cnt, 0.0f);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) m[size_t(i * ld + j)] = float(M[size_t(i * n + j)]);
        HIP_OK(c->dalloc(&c->d_m_hi, cnt * sizeof(float)));
        HIP_OK(hipMemcpy(c->d_m_hi, m.data(), cnt * sizeof(float), hipMemcpyHostToDevice));
    }
    return FTH_OK;
}

std::vector<double> dense_to_double(const fth_matrix* M) {
    const size_t cnt = size_t(M->n) * size_t(M->n);
    std::vector<double> out(cnt);
    if (M->value_is_f64)
        std::memcpy(out.data(), M->dense, cnt * sizeof(double));
    else
        for (size_t k = 0; k < cnt; ++k) out[k] = static_cast<const float*>(M->dense)[k];
    return out;
}

constexpr int64_t kSmallMaxNR = 4096;       // n * R handled by one workgroup
constexpr size_t kSmallMaxLds = 152 * 1024;  // LDS budget of the persistent kernel (160 KB per workgroup)

fth_status ensure_state(fth_ctx* c, int32_t R) {
    if (c->R != 0) {
        if (R != 0 && R != c->R) return fail(FTH_ESTATE, "replica count is fixed at %d", c->R);
        return FTH_OK;
    }
    if (R == 0) R = c->opt.replicas;
    if (R == 0) return fail(FTH_EINVAL, "replica count not given");
    if (!is_pow2(R) || R > 512) return fail(FTH_EUNSUPPORTED, "R must be a power of two <= 512 (got %d)", R);
    int rpt = R >= 4 ? (R > 256 ? 8 : 4) : R;
    if (c->dense() && !c->m_uploaded) {
        const int64_t threads = c->n * (R / std::min(R, 4));
        const size_t rb = c->real_bytes();
        const size_t lds_base = (size_t(c->n_out()) + 3) * 8 + 2 * size_t(c->n) * R * rb *
                                (c->opt.acc_pp && c->npairs > 0 ? 2 : 1) +
                                2 * size_t(c->ns + 1) * size_t(c->ns + 1) * rb;  // + T and S
        const bool small = c->n * R <= kSmallMaxNR && R <= 64 && threads <= 1024 && lds_base <= kSmallMaxLds;
        fth_status st2;
        if (small) {
            c->small = true;
            rpt = std::min(R, 4);
            c->small_m_in_lds = lds_base + size_t(c->n) * size_t(c->n) * rb <= kSmallMaxLds;
            c->small_lds = lds_base + (c->small_m_in_lds ? size_t(c->n) * size_t(c->n) * rb : 0);
            st2 = upload_small(c, c->m_host);
        } else if (R == 1 || R == 2 || R == 4 || R == 8) {
            st2 = upload_gemv(c, c->m_host);
        } else {
            if (R != 16 && R != 32 && R != 64 && R != 128)
                return fail(FTH_EUNSUPPORTED, "dense systems of this size need R in {1, 2, 4, 8, 16, 32, 64, 128} (got %d)",
                            R);
            st2 = upload_dense(c, c->m_host);
        }
        if (st2 != FTH_OK) return st2;
        c->m_host.clear();
        c->m_host.shrink_to_fit();
        c->m_uploaded = true;
    } else if (c->mfma()) {
        const bool few = R == 1 || R == 2 || R == 4 || R == 8;
        if (c->gemv ? !few : (R != 16 && R != 32 && R != 64 && R != 128))
            return fail(FTH_EUNSUPPORTED, "this dense context was set up for R in %s (got %d)",
                        c->gemv ? "{1, 2, 4, 8}" : "{16, 32, 64, 128}", R);
    }
    c->R = R;
    c->rpt = rpt;
    const size_t rb = c->real_bytes();
    // (p, s) row groups: one component of a group fills at least a 128-byte line
    c->ps_lg = R * int(rb) >= 128 ? 0 : ilog2(128 / (R * int(rb)));
    c->ps_rows = (c->n + (int64_t(1) << c->ps_lg) - 1) >> c->ps_lg << c->ps_lg;
    const size_t qst = size_t(c->q_rows()) * size_t(R) * rb;
    const size_t st = size_t(c->n) * size_t(R) * rb;
    // State streamed once per step: bypass L2/MALL when it cannot stay resident.
    c->nt = st * size_t(c->ns + 3) > (size_t(128) << 20);
    HIP_OK(c->dalloc(&c->d_q[0], qst));
    HIP_OK(c->dalloc(&c->d_q[1], qst));
    HIP_OK(c->dalloc(&c->d_ps[0], c->ps_bytes()));
    HIP_OK(c->dalloc(&c->d_ps[1], c->ps_bytes()));
    HIP_OK(hipMemsetAsync(c->d_q[0], 0, qst, c->stream));
    HIP_OK(hipMemsetAsync(c->d_q[1], 0, qst, c->stream));
    HIP_OK(hipMemsetAsync(c->d_ps[0], 0, c->ps_bytes(), c->stream));
    HIP_OK(hipMemsetAsync(c->d_ps[1], 0, c->ps_bytes(), c->stream));
    if (c->mfma()) {
        const size_t pb = size_t(c->ksplit) * size_t(c->rows_pad) * size_t(R) * rb;
        HIP_OK(c->dalloc(&c->d_part, pb));
        HIP_OK(hipMemsetAsync(c->d_part, 0, pb, c->stream));
        if (c->prec == FTH_FP32_BF16X3 && !c->gemv) {
            const size_t qtb = size_t(c->rows_pad) * size_t(R) * 2 * sizeof(uint16_t);
            HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_qt), qtb));
            HIP_OK(hipMemsetAsync(c->d_qt, 0, qtb, c->stream));
            c->qt_dirty = true;
        }
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    return FTH_OK;
}

template <typename Real>
fth::StepArgs<Real> step_args(fth_ctx* c) {
    fth::StepArgs<Real> a{};
    a.row_ptr = c->d_row_ptr;
    a.col = c->d_col;
    a.ell_col = c->d_ell_col;
    a.ell_vcode = c->d_ell_vcode;
    a.ell_vraw = static_cast<const Real*>(c->d_ell_vraw);
    a.dict_off = c->d_dict_off;
    a.dict_val = static_cast<const Real*>(c->d_dict_val);
    a.n_off = c->n_off;
    a.n_val = c->n_val;
    a.val = static_cast<const Real*>(c->d_val);
    a.part = static_cast<const Real*>(c->d_part);
    a.ksplit = c->ksplit;
    a.rows_pad = c->rows_pad;
    a.qt = c->d_qt;
    a.mdense = static_cast<const Real*>(c->d_msmall);
    a.m_in_lds = c->small_m_in_lds;
    a.q0 = static_cast<Real*>(c->d_q[0]);
    a.q1 = static_cast<Real*>(c->d_q[1]);
    a.ps = static_cast<Real*>(c->d_ps[0]);
    a.ps_b = static_cast<Real*>(c->d_ps[1]);
    a.ns = c->ns;
    a.ps_lg = c->ps_lg;
    a.TS = static_cast<const Real*>(c->d_TS);
    a.h = Real(c->h);
    a.hh = Real(0.5 * c->h);
    a.N = c->n;
    a.R = c->R;
    a.lg_tpr = ilog2(c->R / c->rpt);
    a.key0 = uint32_t(c->opt.seed);
    a.key1 = uint32_t(c->opt.seed >> 32);
    a.stream = c->opt.stream_id;
    a.step_base = c->d_step;
    a.burn_in = c->opt.burn_in;
    a.block_len = c->opt.block_len;
    const int64_t no = c->n_out();
    double* blk = c->d_acc;
    double* s1 = c->d_acc + no;
    double* s2 = c->d_acc + 2 * no;
    a.pairs = c->d_pairs;
    a.npairs = c->npairs;
    a.pblk = blk;
    a.ps1 = s1;
    a.ps2 = s2;
    if (c->opt.acc_diag) {
        a.dblk = blk + c->npairs;
        a.ds1 = s1 + c->npairs;
        a.ds2 = s2 + c->npairs;
    }
    if (c->opt.acc_pp) {  // the p-p block follows the q-q block
        const int64_t o = c->n_kind();
        a.pp_blk = blk + o;
        a.pp_s1 = s1 + o;
        a.pp_s2 = s2 + o;
        if (c->opt.acc_diag) {
            a.dp_blk = blk + o + c->npairs;
            a.dp_s1 = s1 + o + c->npairs;
            a.dp_s2 = s2 + o + c->npairs;
        }
    }
    a.flag = c->d_flag;
    a.tpart = c->opt.acc_trace ? c->d_tpart : nullptr;
    a.tpart_w = c->tpart_w;
    const int per_block = c->block / (c->R / c->rpt);
    a.row_tiles = (c->n + per_block - 1) / per_block;
    a.row_tiles_padded = (a.row_tiles + 7) / 8 * 8;
    return a;
}

// Plain CSR rows longer than 16 entries take the long-row gather batches.
bool long_rows(const fth_ctx* c) {
    return !c->dense() && !(c->coded && c->rpt >= 4) && c->rpt >= 4 && c->max_row_nnz > 16;
}

fth::StepLaunch step_launch(fth_ctx* c) {
    const int per_block = c->block / (c->R / c->rpt);
    return fth::StepLaunch{c->ns, c->rpt, c->nt, c->coded && c->rpt >= 4, long_rows(c), c->block,
                           (c->npairs + per_block - 1) / per_block};
}

fth::DenseGemmArgs gemm_args(fth_ctx* c, int k) {
    fth::DenseGemmArgs g{};
    g.m_hi = c->d_m_hi;
    g.qt = c->d_qt;
    g.q0 = c->d_q[0];
    g.q1 = c->d_q[1];
    g.step_base = c->d_step;
    g.k = k;
    g.part = c->d_part;
    g.rows_pad = c->rows_pad;
    g.R = c->R;
    g.ksplit = c->ksplit;
    g.kslice = c->rows_pad / c->ksplit;
    return g;
}

// The dense force partials of one step: the matrix-core GEMM, or for R < 16
// the matrix-vector form.
int launch_force(const fth_ctx* c, const fth::DenseGemmArgs& g) {
    if (c->gemv)
        return c->prec == FTH_FP64
                   ? fth::launch_dense_gemv<double>(g, static_cast<const double*>(c->d_m_hi), c->n, c->rows_pad, c->stream)
                   : fth::launch_dense_gemv<float>(g, static_cast<const float*>(c->d_m_hi), c->n, c->rows_pad, c->stream);
    return c->prec == FTH_FP64 ? fth::launch_gemm_f64(g, c->stream) : fth::launch_gemm_bf16x3(g, c->stream);
}

// Enqueue one step with in-chunk offset k (global step = *d_step + k).
fth_status enqueue_step(fth_ctx* c, int k) {
    int rc;
    if (c->dense()) {
        const fth::DenseGemmArgs g = gemm_args(c, k);
        rc = launch_force(c, g);
        if (rc != 0) return fail(FTH_EDEVICE, "dense force launch failed (%d)", rc);
        if (c->prec == FTH_FP64)
            rc = fth::launch_dense_epilogue<double>(step_args<double>(c), step_launch(c), k, c->stream);
        else
            rc = fth::launch_dense_epilogue<float>(step_args<float>(c), step_launch(c), k, c->stream);
    } else if (c->prec == FTH_FP64) {
        rc = fth::launch_csr_step<double>(step_args<double>(c), step_launch(c), k, c->stream);
    } else {
        rc = fth::launch_csr_step<float>(step_args<float>(c), step_launch(c), k, c->stream);
    }
    if (rc == -2) return fail(FTH_EUNSUPPORTED, "no kernel instantiated for ns=%d", c->ns);
    if (rc != 0) return fail(FTH_EDEVICE, "step kernel launch failed (%d): %s", rc, hipGetErrorString(hipGetLastError()));
    return FTH_OK;
}

// Rows of the widest tiling the current shape launches (one-step, blocked or small).
int64_t trace_tiles(const fth_ctx* c) {
    if (c->small) return 1;
    const int per_block = c->block / (c->R / c->rpt);
    int64_t w = (c->n + per_block - 1) / per_block;
    if (c->tb_kt > 0) {
        const int E = c->tb_block / (c->R / 4);
        const int64_t T = E - 2 * int64_t(c->tb_kt) * c->band_w;
        w = std::max(w, (c->n + T - 1) / T);
    }
    return w;
}

fth_status trace_prepare(fth_ctx* c, int K) {
    if (!c->opt.acc_trace) return FTH_OK;
    const int64_t w = trace_tiles(c);
    if (K <= c->tpart_k && w <= c->tpart_w) return FTH_OK;
    if (w > 0x7FFFFFFF) return fail(FTH_EUNSUPPORTED, "too many row tiles for trace partials");
    const int nk = std::max(K, c->tpart_k);
    const int nw = int(std::max<int64_t>(w, c->tpart_w));
    if (c->gexec) {  // the captured graph holds the old buffers
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    c->dfree(reinterpret_cast<void*&>(c->d_tpart));
    c->dfree(reinterpret_cast<void*&>(c->d_tsum));
    const size_t pb = sizeof(double) * 3 * size_t(nk) * size_t(nw);
    HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_tpart), pb));
    HIP_OK(hipMemset(c->d_tpart, 0, pb));
    HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_tsum), sizeof(double) * 3 * size_t(nk)));
    c->tpart_k = nk;
    c->tpart_w = nw;
    return FTH_OK;
}

// Sum and fold the trace partials of the K steps just enqueued; the chunk's
// first step is *d_step + shift.
fth_status enqueue_trace_fold(fth_ctx* c, int K, int64_t shift) {
    const int64_t o = c->n_out() - c->ntr();
    const int64_t no = c->n_out();
    if (fth::launch_trace_fold(c->d_tpart, c->d_tsum, K, c->tpart_w, c->ntr(), c->d_acc + o, c->d_acc + no + o,
                               c->d_acc + 2 * no + o, c->d_step, shift, c->opt.burn_in, c->opt.block_len,
                               c->stream) != 0)
        return fail(FTH_EDEVICE, "trace fold launch failed");
    return FTH_OK;
}

fth_status enqueue_small(fth_ctx* c, int64_t nsteps) {
    for (int64_t done = 0; done < nsteps;) {
        const int K = int(std::min<int64_t>(nsteps - done, 4096));
        const int rc = c->prec == FTH_FP64
                           ? fth::launch_small_dense<double>(step_args<double>(c), step_launch(c), K, c->small_lds, c->stream)
                           : fth::launch_small_dense<float>(step_args<float>(c), step_launch(c), K, c->small_lds, c->stream);
        if (rc == -2) return fail(FTH_EUNSUPPORTED, "no kernel instantiated for ns=%d", c->ns);
        if (rc != 0) return fail(FTH_EDEVICE, "small-system kernel launch failed (%d)", rc);
        if (c->opt.acc_trace) {  // the kernel has advanced the step counter by K already
            fth_status st = enqueue_trace_fold(c, K, -int64_t(K));
            if (st != FTH_OK) return st;
        }
        done += K;
    }
    return FTH_OK;
}

bool tb_eligible(const fth_ctx* c, int KT, int block) {
    if (c->dense() || c->band_w < 0 || c->band_w > kTbMaxW || c->max_row_nnz > 8) return false;
    if (c->R < 4 || c->R > 256) return false;
    if (KT != 3 && KT != 5) return false;
    if (block != 256 && block != 512 && block != 1024) return false;
    if (block > fth::tb_max_block(c->prec == FTH_FP64, c->ns, c->opt.acc_pp || c->opt.acc_trace)) return false;
    const int E = block / (c->R / 4);
    const int64_t T = E - 2 * int64_t(KT) * c->band_w;
    return T >= 1 && 2 * T >= E;
}

// Selects the blocked launch shape (KT steps, `block` threads) and, unless
// the caller asked for one workgroup per tile, the persistent form when its
// LDS staging fits the device (building the slot form of the rows once).
fth_status tb_select(fth_ctx* c, int KT, int block) {
    c->tb_kt = KT;
    c->tb_block = block;
    c->tbp_grid = 0;
    if (c->opt.temporal_persistent != 0) return FTH_OK;
    const bool f64 = c->prec == FTH_FP64;
    const bool xtra = c->opt.acc_pp || c->opt.acc_trace;
    const int E = block / (c->R / 4);
    const int T = E - 2 * KT * int(c->band_w);
    const size_t lds = fth::tbp_lds_bytes(f64, c->ns, block, c->R, T, c->opt.acc_trace != 0, xtra);
    const int grid = f64 ? fth::tbp_resident_grid<double>(c->ns, KT, xtra, block, lds)
                         : fth::tbp_resident_grid<float>(c->ns, KT, xtra, block, lds);
    (void)hipGetLastError();  // an unsupported shape query leaves no sticky error behind
    if (grid <= 0) return FTH_OK;
    if (!c->d_tb_slots) {
        const size_t sb = f64 ? sizeof(fth::TbSlotRow<double>) : sizeof(fth::TbSlotRow<float>);
        HIP_OK(c->dalloc(&c->d_tb_slots, sb * size_t(c->n)));
        const int rc = f64 ? fth::launch_tb_slots<double>(c->d_row_ptr, c->d_col, static_cast<const double*>(c->d_val),
                                                          c->n, c->d_tb_slots, c->stream)
                           : fth::launch_tb_slots<float>(c->d_row_ptr, c->d_col, static_cast<const float*>(c->d_val),
                                                         c->n, c->d_tb_slots, c->stream);
        if (rc != 0) return fail(FTH_EDEVICE, "slot-form build launch failed");
    }
    c->tbp_grid = grid;
    return FTH_OK;
}

fth_status tb_prepare(fth_ctx* c) {
    if (c->d_snap || c->d_pair_slot) return FTH_OK;
    const size_t rb = c->real_bytes();
    if (c->npairs > 0) {
        std::vector<int32_t> pairs(size_t(2 * c->npairs));
        HIP_OK(hipMemcpy(pairs.data(), c->d_pairs, sizeof(int32_t) * pairs.size(), hipMemcpyDeviceToHost));
        std::vector<int32_t> slot(size_t(c->n), -1);
        std::vector<int32_t> pslots(pairs.size());
        int32_t ns = 0;
        for (size_t k = 0; k < pairs.size(); ++k) {
            int32_t& sl = slot[size_t(pairs[k])];
            if (sl < 0) sl = ns++;
            pslots[k] = sl;
        }
        c->tb_nslots = ns;
        HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_pair_slot), sizeof(int32_t) * slot.size()));
        HIP_OK(hipMemcpy(c->d_pair_slot, slot.data(), sizeof(int32_t) * slot.size(), hipMemcpyHostToDevice));
        HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_pair_slots), sizeof(int32_t) * pslots.size()));
        HIP_OK(hipMemcpy(c->d_pair_slots, pslots.data(), sizeof(int32_t) * pslots.size(), hipMemcpyHostToDevice));
        HIP_OK(c->dalloc(&c->d_snap, size_t(kTbMaxSteps) * 2 * size_t(ns) * size_t(c->R) * rb));
    }
    return FTH_OK;
}

void tb_release(fth_ctx* c) {
    c->dfree(reinterpret_cast<void*&>(c->d_pair_slot));
    c->dfree(reinterpret_cast<void*&>(c->d_pair_slots));
    c->dfree(c->d_snap);
    c->dfree(c->d_tb_slots);
    c->tb_nslots = 0;
    c->tb_kt = 0;
    c->tbp_grid = 0;
}

// Blocked launch j of a chunk: steps [j KT, j KT + KT) of it.
template <typename Real>
fth_status enqueue_tb(fth_ctx* c, int j) {
    fth::StepArgs<Real> a = step_args<Real>(c);
    fth::TbArgs<Real> tb{};
    tb.E = c->tb_block / (c->R / 4);
    tb.w = int32_t(c->band_w);
    tb.T = tb.E - 2 * c->tb_kt * tb.w;
    tb.pair_slot = c->d_pair_slot;
    tb.snap = static_cast<Real*>(c->d_snap);
    tb.nslots = c->tb_nslots;
    tb.pair_slots = c->d_pair_slots;
    a.row_tiles = (c->n + tb.T - 1) / tb.T;
    a.row_tiles_padded = (a.row_tiles + 7) / 8 * 8;
    const fth::StepLaunch L = step_launch(c);
    int rc;
    if (c->tbp_grid > 0) {
        tb.slots = c->d_tb_slots;
        tb.grid = int32_t(std::min<int64_t>(c->tbp_grid, a.row_tiles));
        rc = fth::launch_tbp_step<Real>(a, tb, L, c->tb_kt, j * c->tb_kt, c->stream);
    } else {
        rc = fth::launch_tb_step<Real>(a, tb, L, c->tb_kt, j * c->tb_kt, c->stream);
    }
    if (rc == 0) rc = fth::launch_tb_pairs<Real>(a, tb, L, c->tb_kt, j * c->tb_kt, c->stream);
    if (rc == -2) return fail(FTH_EUNSUPPORTED, "no blocked kernel for ns=%d, KT=%d", c->ns, c->tb_kt);
    if (rc != 0) return fail(FTH_EDEVICE, "blocked step launch failed (%d): %s", rc, hipGetErrorString(hipGetLastError()));
    return FTH_OK;
}

fth_status enqueue_chunk(fth_ctx* c, int K) {
    int k0 = 0;
    if (c->tb_kt > 0) {
        const int nl = K / c->tb_kt;
        for (int j = 0; j < nl; ++j) {
            fth_status st = c->prec == FTH_FP64 ? enqueue_tb<double>(c, j) : enqueue_tb<float>(c, j);
            if (st != FTH_OK) return st;
        }
        k0 = nl * c->tb_kt;
    }
    for (int k = k0; k < K; ++k) {
        fth_status st = enqueue_step(c, k);
        if (st != FTH_OK) return st;
    }
    if (c->opt.acc_trace) {
        fth_status st = enqueue_trace_fold(c, K, 0);
        if (st != FTH_OK) return st;
    }
    if (fth::launch_advance(c->d_step, K, c->stream) != 0) return fail(FTH_EDEVICE, "advance launch failed");
    return FTH_OK;
}

fth_status build_graph(fth_ctx* c, int K) {
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    HIP_OK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    fth_status st = enqueue_chunk(c, K);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st != FTH_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(FTH_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(FTH_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    c->gK = K;
    return FTH_OK;
}

// ------------------------------------------------------------- autotuner
// Candidate launch shapes of the sparse step: threads per workgroup,
// replicas per thread, streaming state access.  Each candidate runs a few
// steps on the live state, which is saved before and restored after, so
// tuning leaves the trajectory untouched.  The winner is cached per shape
// key: precision, GLE size, R, n, nnz, half-bandwidth, longest row and
// whether momentum-form or trace accumulators are kept (they lower the
// largest blocked workgroup).
struct TuneKey {
    int prec, ns, R, xtra, max_row_nnz;
    int64_t n, nnz, band_w;
    bool operator<(const TuneKey& o) const {
        return std::tie(prec, ns, R, xtra, max_row_nnz, n, nnz, band_w) <
               std::tie(o.prec, o.ns, o.R, o.xtra, o.max_row_nnz, o.n, o.nnz, o.band_w);
    }
};
struct TuneChoice {
    int block, rpt;
    bool nt;
    double us;
    int tb_kt, tb_block;
};
std::map<TuneKey, TuneChoice>& tune_cache() {
    static std::map<TuneKey, TuneChoice> cache;
    return cache;
}

// Time K steps (enqueued without a graph) on the live state; us per step.
fth_status time_chunk(fth_ctx* c, int K, double* us) {
    fth_status st = trace_prepare(c, K);
    if (st != FTH_OK) return st;
    st = enqueue_chunk(c, K);  // warm-up
    if (st != FTH_OK) return st;
    HIP_OK(hipEventRecord(c->ev0, c->stream));
    st = enqueue_chunk(c, K);
    if (st != FTH_OK) return st;
    HIP_OK(hipEventRecord(c->ev1, c->stream));
    HIP_OK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    *us = 1e3 * double(ms) / double(K);
    return FTH_OK;
}

fth_status autotune(fth_ctx* c) {
    if (c->dense() || c->R < 4) return FTH_OK;  // dense GEMM tiles and tiny R have one shape
    if (c->tb_kt > 0) return FTH_OK;            // blocking fixed by the caller
    const bool try_tb = c->opt.temporal_steps == 0 && (tb_eligible(c, 3, 1024) || tb_eligible(c, 3, 512) ||
                                                       tb_eligible(c, 3, 256));
    // (KT = 5 is eligible only where KT = 3 is.)
    const TuneKey key{c->prec, c->ns, c->R, (c->opt.acc_pp || c->opt.acc_trace) ? 1 : 0, c->max_row_nnz,
                      c->n, c->nnz, c->band_w};
    auto hit = tune_cache().find(key);
    if (hit != tune_cache().end() &&
        (hit->second.tb_kt == 0 || (try_tb && tb_eligible(c, hit->second.tb_kt, hit->second.tb_block)))) {
        c->block = hit->second.block;
        c->rpt = hit->second.rpt;
        c->nt = hit->second.nt;
        c->tuned_us = hit->second.us;
        if (hit->second.tb_kt > 0) {
            fth_status st = tb_prepare(c);
            if (st != FTH_OK) return st;
            return tb_select(c, hit->second.tb_kt, hit->second.tb_block);
        }
        return FTH_OK;
    }
    // save the state (q pair, ps, accumulators, counter)
    const size_t rb = c->real_bytes();
    const size_t qb = size_t(c->q_rows()) * size_t(c->R) * rb;
    const size_t psb = c->ps_bytes();
    const size_t ab = sizeof(double) * size_t(3 * c->n_out());
    ctx_scratch sv(c);
    void* bufs[4] = {c->d_q[0], c->d_q[1], c->d_ps[c->step & 1], c->d_acc};
    const size_t sizes[4] = {qb, qb, psb, std::max<size_t>(ab, 8)};
    void* saved[4];
    for (int k = 0; k < 4; ++k) {
        saved[k] = sv.get(sizes[k]);
        if (!saved[k]) return fail(FTH_ENOMEM, "autotuner could not save the state");
        HIP_OK(hipMemcpyAsync(saved[k], bufs[k], sizes[k], hipMemcpyDeviceToDevice, c->stream));
    }
    int64_t step0 = 0;
    HIP_OK(hipMemcpy(&step0, c->d_step, sizeof(int64_t), hipMemcpyDeviceToHost));
    TuneChoice best{c->block, c->rpt, c->nt, 1e30, 0, 0};
    TuneChoice best4 = best;  // best one-step shape with 4 replicas per thread (tail of blocked chunks)
    const int blocks[3] = {64, 128, 256};
    const int rpts[2] = {4, 8};
    for (int b : blocks)
        for (int rp : rpts)
            for (int ntv = 0; ntv < 2; ++ntv) {
                if (rp > c->R || c->R / rp > 64 || c->R / rp > b) continue;
                c->block = b;
                c->rpt = rp;
                c->nt = ntv != 0;
                double us = 0.0;
                fth_status st = time_chunk(c, 8, &us);
                if (st != FTH_OK) return st;
                if (us < best.us) best = TuneChoice{b, rp, ntv != 0, us, 0, 0};
                if (rp == 4 && us < best4.us) best4 = TuneChoice{b, rp, ntv != 0, us, 0, 0};
            }
    if (try_tb && best4.us < 1e30) {
        fth_status st = tb_prepare(c);
        if (st != FTH_OK) return st;
        c->block = best4.block;
        c->rpt = 4;
        c->nt = best4.nt;
        const int kts[2] = {3, 5};
        const int tbs[3] = {256, 512, 1024};
        for (int kt : kts)
            for (int tbb : tbs) {
                if (!tb_eligible(c, kt, tbb)) continue;
                st = tb_select(c, kt, tbb);
                if (st != FTH_OK) return st;
                double us = 0.0;
                st = time_chunk(c, 2 * kt, &us);
                if (st != FTH_OK) return st;
                if (us < best.us) best = TuneChoice{best4.block, 4, best4.nt, us, kt, tbb};
            }
        c->tb_kt = 0;
    }
    // restore
    for (int k = 0; k < 4; ++k) HIP_OK(hipMemcpyAsync(bufs[k], saved[k], sizes[k], hipMemcpyDeviceToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(c->d_step, &step0, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemsetAsync(c->d_flag, 0, sizeof(int32_t), c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    c->block = best.block;
    c->rpt = best.rpt;
    c->nt = best.nt;
    c->tuned_us = best.us;
    if (best.tb_kt > 0) {
        fth_status st2 = tb_select(c, best.tb_kt, best.tb_block);
        if (st2 != FTH_OK) return st2;
    } else {
        tb_release(c);
        c->tb_block = 1024;
    }
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    tune_cache()[key] = best;
    return FTH_OK;
}

fth_status run_enqueue(fth_ctx* c, int64_t nsteps) {
    fth_status st;
    int K = c->opt.steps_per_graph > 0 ? c->opt.steps_per_graph : kDefaultGraphSteps;
    if (c->tb_kt > 0) K = std::max(1, K / c->tb_kt) * c->tb_kt;  // whole blocked launches
    st = trace_prepare(c, c->small ? 4096 : K);
    if (st != FTH_OK) return st;
    if (c->d_qt && c->qt_dirty) {
        if (fth::launch_qt_from_q(static_cast<const float*>(c->d_q[c->step & 1]), c->d_qt, c->n, c->rows_pad, c->R,
                                  c->stream) != 0)
            return fail(FTH_EDEVICE, "q split launch failed");
        c->qt_dirty = false;
    }
    if (c->small) return enqueue_small(c, nsteps);
    int64_t left = nsteps;
    if (left >= K) {
        if (!c->gexec || c->gK != K) {
            st = build_graph(c, K);
            if (st != FTH_OK) return st;
        }
        while (left >= K) {
            HIP_OK(hipGraphLaunch(c->gexec, c->stream));
            left -= K;
        }
    }
    if (left > 0) {
        st = enqueue_chunk(c, int(left));
        if (st != FTH_OK) return st;
    }
    return FTH_OK;
}

fth_status run_complete(fth_ctx* c, int64_t nsteps) {
    HIP_OK(hipStreamSynchronize(c->stream));
    c->step += nsteps;
    int32_t flag = 0;
    HIP_OK(hipMemcpy(&flag, c->d_flag, sizeof(flag), hipMemcpyDeviceToHost));
    if (flag) {
        c->poisoned = true;
        return fail(FTH_ENONFINITE, "non-finite state after step %lld (M not SPD or dt too large)", (long long)c->step);
    }
    return FTH_OK;
}

template fth::StepArgs<float> step_args<float>(fth_ctx* c);
template fth::StepArgs<double> step_args<double>(fth_ctx* c);

}  // namespace host
}  // namespace fth

using namespace fth::host;

extern "C" {

const char* fth_last_error(void) { return g_last_error.c_str(); }
const char* fth_version(void) { return "fth-mi355x 0.1 (gfx950)"; }

void fth_default_options(fth_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = FTH_FP32;
    opt->block_len = 100;
}

fth_status fth_propagator(const fth_gle* gle, double dt, double* T, double* S) {
    std::vector<double> t, s;
    fth_status st = make_propagator(gle, dt, t, s);
    if (st != FTH_OK) return st;
    if (T) std::memcpy(T, t.data(), sizeof(double) * t.size());
    if (S) std::memcpy(S, s.data(), sizeof(double) * s.size());
    return FTH_OK;
}

size_t fth_footprint_bytes(const fth_matrix* M, int32_t ns, int32_t R, int64_t npairs, int32_t acc_diag,
                           int32_t precision) {
    if (!M) return 0;
    const size_t rb = precision == FTH_FP64 ? 8 : 4;
    const size_t n = size_t(M->n);
    // (p, s) rows are padded to whole groups of 128 / (R rb) rows (when R rb < 128)
    const size_t grp = R > 0 && size_t(R) * rb < 128 ? 128 / (size_t(R) * rb) : 1;
    const size_t ps_rows = (n + grp - 1) / grp * grp;
    size_t bytes = 0;
    if (M->format == FTH_CSR) {
        bytes += (n + 1) * 8 + size_t(M->nnz) * (4 + rb);
        bytes += n * size_t(R) * rb * 2 + 2 * ps_rows * size_t(R) * rb * size_t(1 + ns);
    } else if ((R == 1 || R == 2 || R == 4 || R == 8) && int64_t(n) * R > kSmallMaxNR) {
        const size_t ld = (n + 3) / 4 * 4;                                    // matrix-vector form
        bytes += n * ld * rb;                                                  // M
        bytes += 2 * ld * size_t(R) * rb + 2 * ps_rows * size_t(R) * rb * size_t(1 + ns);
        bytes += ld * size_t(R) * rb;                                          // force partials
    } else {
        const size_t P = size_t(dense_rows_pad(int64_t(n)));
        const size_t ks = size_t(dense_ksplit(int64_t(P), precision));
        bytes += P * P * (precision == FTH_FP32_BF16X3 ? 4 : rb);           // M (hi + lo, or FP64)
        bytes += 2 * P * size_t(R) * rb + 2 * ps_rows * size_t(R) * rb * size_t(1 + ns);  // q, (p, s) pairs
        bytes += ks * P * size_t(R) * rb;                                      // split-K partials
        if (precision == FTH_FP32_BF16X3) bytes += P * size_t(R) * 4;          // bf16 q split
    }
    const size_t nout = size_t(npairs) + (acc_diag ? n : 0);
    bytes += nout * 24 + size_t(npairs) * 8;
    bytes += 2 * size_t(ns + 1) * size_t(ns + 1) * rb + 64;
    return bytes;
}

fth_status fth_create(const fth_matrix* M_in, const fth_gle* gle_in, double dt, const int32_t* pairs, int64_t npairs,
                      const fth_options* opt_in, fth_ctx** out) {
    g_last_error.clear();
    if (!out) return fail(FTH_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!M_in || !gle_in) return fail(FTH_EINVAL, "M and gle must not be NULL");
    fth_options opt;
    fth_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (M_in->n < 1 || M_in->n > 0xFFFFFFFFll) return fail(FTH_EINVAL, "n must be in [1, 2^32)");
    if (M_in->format != FTH_CSR && M_in->format != FTH_DENSE) return fail(FTH_EINVAL, "unknown matrix format");
    // spectral map: M' = r M + m I, A'_p = alpha A_p, C'_p = gamma C_p (identity by default)
    const double sr = opt.scale_r == 0.0 ? 1.0 : opt.scale_r, sm = opt.scale_m;
    const double ga = opt.gle_alpha == 0.0 ? 1.0 : opt.gle_alpha, gg = opt.gle_gamma == 0.0 ? 1.0 : opt.gle_gamma;
    fth_matrix M_map;
    std::vector<double> map_store;
    const fth_matrix* M = M_in;
    if (sr != 1.0 || sm != 0.0) {
        fth_status st0 = spectral_transform(M_in, sr, sm, map_store, &M_map);
        if (st0 != FTH_OK) return st0;
        M = &M_map;
    }
    fth_gle gle_map;
    std::vector<double> gle_a, gle_c;
    const fth_gle* gle = gle_in;
    if (ga != 1.0 || gg != 1.0) {
        fth_status st0 = scaled_gle(gle_in, ga, gg, gle_a, gle_c, &gle_map);
        if (st0 != FTH_OK) return st0;
        gle = &gle_map;
    }
    if (opt.precision < FTH_FP64 || opt.precision > FTH_FP32_BF16X3) return fail(FTH_EINVAL, "unknown precision");
    if (opt.block_len < 1) return fail(FTH_EINVAL, "block_len must be >= 1");
    if (opt.burn_in < 0) return fail(FTH_EINVAL, "burn_in must be >= 0");
    if (opt.temporal_steps != 0 && opt.temporal_steps != -1 && opt.temporal_steps != 3 && opt.temporal_steps != 5)
        return fail(FTH_EINVAL, "temporal_steps must be -1, 0, 3 or 5");
    if (opt.temporal_threads != 0 && opt.temporal_threads != 256 && opt.temporal_threads != 512 &&
        opt.temporal_threads != 1024)
        return fail(FTH_EINVAL, "temporal_threads must be 0, 256, 512 or 1024");
    if (opt.coded_matrix != 0 && opt.coded_matrix != -1) return fail(FTH_EINVAL, "coded_matrix must be 0 or -1");
    if (opt.temporal_persistent != 0 && opt.temporal_persistent != -1)
        return fail(FTH_EINVAL, "temporal_persistent must be 0 or -1");
    if (opt.acc_pp != 0 && opt.acc_pp != 1) return fail(FTH_EINVAL, "acc_pp must be 0 or 1");
    if (opt.acc_trace != 0 && opt.acc_trace != 1) return fail(FTH_EINVAL, "acc_trace must be 0 or 1");
    if (npairs < 0 || (npairs > 0 && !pairs)) return fail(FTH_EINVAL, "invalid pair list");
    for (int64_t k = 0; k < 2 * npairs; ++k)
        if (pairs[k] < 0 || pairs[k] >= M->n) return fail(FTH_EINVAL, "pair index out of range at %lld", (long long)k);
    fth_status st = M->format == FTH_CSR ? check_csr(M) : check_dense(M);
    if (st != FTH_OK) return st;
    if (M->format == FTH_CSR && opt.precision == FTH_FP32_BF16X3)
        return fail(FTH_EUNSUPPORTED, "split-BF16x3 applies to dense matrices only");
    if (M->format == FTH_DENSE && opt.precision == FTH_FP32 && M->n > kSmallMaxNR &&
        !(opt.replicas == 1 || opt.replicas == 2 || opt.replicas == 4 || opt.replicas == 8))
        return fail(FTH_EUNSUPPORTED,
                    "dense systems beyond one workgroup use FTH_FP32_BF16X3 or FTH_FP64 (FTH_FP32 needs replicas <= 8)");
    if (gle && (gle->ns > fth::kNsMax)) return fail(FTH_EUNSUPPORTED, "ns > %d not instantiated", fth::kNsMax);

    std::unique_ptr<fth_ctx> c(new fth_ctx());
    if (opt.allocator) {
        if (!opt.allocator->alloc || !opt.allocator->release)
            return fail(FTH_EINVAL, "an allocator needs both alloc and release");
        c->hook = *opt.allocator;
    }
    c->n = M->n;
    c->fmt = M->format;
    c->prec = opt.precision;
    c->ns = gle->ns;
    c->h = dt;
    c->opt = opt;
    c->npairs = npairs;
    c->nnz = M->nnz;
    {
        const size_t vb = M->value_is_f64 ? 8 : 4;
        uint64_t mh = hash_words(&M->n, sizeof(M->n), uint64_t(M->format) + 1);
        if (M->format == FTH_DENSE) {
            mh = hash_words(M->dense, size_t(M->n) * size_t(M->n) * vb, mh);
        } else {
            mh = hash_words(M->row_ptr, sizeof(int64_t) * size_t(M->n + 1), mh);
            mh = hash_words(M->col, sizeof(int32_t) * size_t(M->nnz), mh);
            mh = hash_words(M->val, vb * size_t(M->nnz), mh);
        }
        c->m_hash = hash_words(&M->value_is_f64, sizeof(M->value_is_f64), mh);
        c->pair_hash = npairs > 0 ? hash_words(pairs, sizeof(int32_t) * size_t(2 * npairs), 7) : 7;
    }
    st = make_propagator(gle, dt, c->T, c->S);
    if (st != FTH_OK) return st;

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(FTH_EDEVICE, "no HIP device available");
    HIP_OK(hipGetDevice(&c->device));
    HIP_OK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIP_OK(hipEventCreate(&c->ev0));
    HIP_OK(hipEventCreate(&c->ev1));

    // matrix
    if (c->dense()) {
        c->m_host = dense_to_double(M);
        if (M->n > kSmallMaxNR && opt.replicas != 0) {  // no single-workgroup path for any R
            const int32_t R0 = opt.replicas;
            st = (R0 == 1 || R0 == 2 || R0 == 4 || R0 == 8) ? upload_gemv(c.get(), c->m_host)
                                                             : upload_dense(c.get(), c->m_host);
            if (st != FTH_OK) return st;
            c->m_host.clear();
            c->m_host.shrink_to_fit();
            c->m_uploaded = true;
        }
    } else {
        int64_t w = 0, maxnz = 0;
        for (int64_t i = 0; i < M->n; ++i) {
            maxnz = std::max(maxnz, M->row_ptr[i + 1] - M->row_ptr[i]);
            for (int64_t k = M->row_ptr[i]; k < M->row_ptr[i + 1]; ++k)
                w = std::max(w, std::abs(int64_t(M->col[k]) - i));
        }
        c->band_w = w;
        c->max_row_nnz = int(std::min<int64_t>(maxnz, 1 << 30));
        HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_row_ptr), sizeof(int64_t) * size_t(M->n + 1)));
        HIP_OK(hipMemcpy(c->d_row_ptr, M->row_ptr, sizeof(int64_t) * size_t(M->n + 1), hipMemcpyHostToDevice));
        HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_col), sizeof(int32_t) * size_t(M->nnz)));
        HIP_OK(hipMemcpy(c->d_col, M->col, sizeof(int32_t) * size_t(M->nnz), hipMemcpyHostToDevice));
        st = c->prec == FTH_FP64 ? upload_converted<double>(c.get(), &c->d_val, M->val, M->nnz, M->value_is_f64)
                                 : upload_converted<float>(c.get(), &c->d_val, M->val, M->nnz, M->value_is_f64);
        if (st != FTH_OK) return st;
        if (opt.coded_matrix == 0 && c->max_row_nnz <= fth::kCodedSlots) {
            st = c->prec == FTH_FP64 ? build_coded<double>(c.get(), M) : build_coded<float>(c.get(), M);
            if (st != FTH_OK) return st;
        }
    }
    st = c->prec == FTH_FP64 ? upload_TS<double>(c.get()) : upload_TS<float>(c.get());
    if (st != FTH_OK) return st;

    // pairs and accumulators
    HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_pairs), sizeof(int32_t) * size_t(2 * npairs)));
    if (npairs > 0) HIP_OK(hipMemcpy(c->d_pairs, pairs, sizeof(int32_t) * size_t(2 * npairs), hipMemcpyHostToDevice));
    const size_t accb = sizeof(double) * size_t(3 * c->n_out());
    HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_acc), accb));
    HIP_OK(hipMemset(c->d_acc, 0, std::max<size_t>(accb, 8)));
    HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_step), sizeof(int64_t)));
    HIP_OK(hipMemset(c->d_step, 0, sizeof(int64_t)));
    HIP_OK(c->dalloc(reinterpret_cast<void**>(&c->d_flag), sizeof(int32_t)));
    HIP_OK(hipMemset(c->d_flag, 0, sizeof(int32_t)));
    if (opt.replicas != 0) {
        st = ensure_state(c.get(), opt.replicas);
        if (st != FTH_OK) return st;
    }
    *out = c.release();
    return FTH_OK;
}

fth_status fth_run(fth_ctx* c, int64_t nsteps, int32_t replicas) {
    g_last_error.clear();
    if (!c) return fail(FTH_EINVAL, "ctx must not be NULL");
    if (c->poisoned) return fail(FTH_ESTATE, "context is poisoned by a non-finite state");
    if (nsteps < 0) return fail(FTH_EINVAL, "nsteps must be >= 0");
    if (c->step + nsteps >= (int64_t(1) << 32)) return fail(FTH_EINVAL, "total steps must stay below 2^32");
    fth_status st = ensure_state(c, replicas);
    if (st != FTH_OK) return st;
    HIP_OK(hipSetDevice(c->device));
    if (c->opt.temporal_steps > 0 && c->tb_kt == 0) {
        const int tbb = c->opt.temporal_threads > 0
                            ? c->opt.temporal_threads
                            : fth::tb_max_block(c->prec == FTH_FP64, c->ns, c->opt.acc_pp || c->opt.acc_trace);
        if (!tb_eligible(c, c->opt.temporal_steps, tbb))
            return fail(FTH_EUNSUPPORTED,
                        "temporal blocking needs CSR with half-bandwidth <= %lld (%lld), <= 8 entries per row (%d), "
                        "4 <= R <= 256 and at least half of each workgroup's rows as output",
                        (long long)kTbMaxW, (long long)c->band_w, c->max_row_nnz);
        c->rpt = 4;
        st = tb_prepare(c);
        if (st != FTH_OK) return st;
        st = tb_select(c, c->opt.temporal_steps, tbb);
        if (st != FTH_OK) return st;
    }
    if (c->opt.tune && !c->tuned) {
        st = autotune(c);
        if (st != FTH_OK) return st;
        c->tuned = true;
    }
    if (nsteps == 0) return FTH_OK;  // shape fixed (and tuned): nothing to run
    if (c->opt.hip_stream) {
        // order after the caller's stream
        HIP_OK(hipEventRecord(c->ev0, static_cast<hipStream_t>(c->opt.hip_stream)));
        HIP_OK(hipStreamWaitEvent(c->stream, c->ev0, 0));
    }
    HIP_OK(hipEventRecord(c->ev0, c->stream));
    st = run_enqueue(c, nsteps);
    if (st != FTH_OK) return st;
    HIP_OK(hipEventRecord(c->ev1, c->stream));
    HIP_OK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms = ms;
    return run_complete(c, nsteps);
}

fth_status fth_set_steps_per_graph(fth_ctx* c, int32_t steps) {
    if (!c || steps < 0) return fail(FTH_EINVAL, "invalid arguments");
    if (c->gexec) {
        HIP_OK(hipStreamSynchronize(c->stream));
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    c->opt.steps_per_graph = steps;
    return FTH_OK;
}

int64_t fth_num_outputs(const fth_ctx* c) { return c ? c->n_out() : 0; }

fth_status fth_get_accumulators(fth_ctx* c, double* blk, double* s1, double* s2, int64_t* nblocks, int64_t* step) {
    if (!c) return fail(FTH_EINVAL, "ctx must not be NULL");
    const int64_t no = c->n_out();
    HIP_OK(hipStreamSynchronize(c->stream));
    double* dst[3] = {blk, s1, s2};
    for (int k = 0; k < 3; ++k)
        if (dst[k] && no > 0)
            HIP_OK(hipMemcpy(dst[k], c->d_acc + k * no, sizeof(double) * size_t(no), hipMemcpyDeviceToHost));
    const int64_t nacc = std::max<int64_t>(0, c->step - c->opt.burn_in);
    if (nblocks) *nblocks = nacc / c->opt.block_len;
    if (step) *step = c->step;
    return FTH_OK;
}

fth_status fth_read(fth_ctx* c, double* est, double* se, int64_t len, int64_t* nsamples) {
    if (!c) return fail(FTH_EINVAL, "ctx must not be NULL");
    const int64_t no = c->n_out();
    if (len < no) return fail(FTH_EINVAL, "output length %lld < %lld", (long long)len, (long long)no);
    std::vector<double> blk(no), s1(no), s2(no);
    int64_t nb = 0, step = 0;
    fth_status st = fth_get_accumulators(c, blk.data(), s1.data(), s2.data(), &nb, &step);
    if (st != FTH_OK) return st;
    const int64_t nacc = std::max<int64_t>(0, step - c->opt.burn_in);
    const double R = c->R > 0 ? double(c->R) : 1.0;
    const double L = double(c->opt.block_len);
    for (int64_t k = 0; k < no; ++k) {
        if (est) est[k] = nacc > 0 ? (s1[k] + blk[k]) / (R * double(nacc)) : std::numeric_limits<double>::quiet_NaN();
        if (se) {
            if (nb < 2) {
                se[k] = std::numeric_limits<double>::infinity();
            } else {
                const double sc = 1.0 / (R * L);
                const double sb = s1[k] * sc, sbb = s2[k] * sc * sc;
                const double var = (sbb - sb * sb / double(nb)) / double(nb - 1);
                se[k] = std::sqrt(std::max(var, 0.0) / double(nb));
            }
        }
    }
    if (nsamples) *nsamples = nacc;
    return FTH_OK;
}

fth_status fth_get_state(fth_ctx* c, double* q, double* p, double* s) {
    if (!c) return fail(FTH_EINVAL, "ctx must not be NULL");
    if (c->R == 0) return fail(FTH_ESTATE, "state not allocated (replica count not fixed)");
    HIP_OK(hipStreamSynchronize(c->stream));
    const size_t cnt = size_t(c->n) * size_t(c->R);
    const size_t D = size_t(c->ns + 1), R = size_t(c->R);
    const size_t pscnt = c->ps_bytes() / c->real_bytes();
    std::vector<double> qh(cnt), psh(pscnt);
    if (c->prec == FTH_FP64) {
        HIP_OK(hipMemcpy(qh.data(), c->d_q[c->step & 1], sizeof(double) * cnt, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(psh.data(), c->d_ps[c->step & 1], sizeof(double) * pscnt, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tq(cnt), tps(pscnt);
        HIP_OK(hipMemcpy(tq.data(), c->d_q[c->step & 1], sizeof(float) * cnt, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(tps.data(), c->d_ps[c->step & 1], sizeof(float) * pscnt, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < cnt; ++k) qh[k] = tq[k];
        for (size_t k = 0; k < pscnt; ++k) psh[k] = tps[k];
    }
    if (q) std::memcpy(q, qh.data(), sizeof(double) * cnt);
    for (size_t i = 0; i < size_t(c->n); ++i)
        for (size_t r = 0; r < R; ++r) {
            if (p) p[i * R + r] = psh[c->ps_offset(int64_t(i), 0, int(r))];
            if (s)
                for (size_t k = 0; k + 1 < D; ++k)
                    s[(k * size_t(c->n) + i) * R + r] = psh[c->ps_offset(int64_t(i), int(k + 1), int(r))];
        }
    return FTH_OK;
}

fth_status fth_set_state(fth_ctx* c, const double* q, const double* p, const double* s) {
    if (!c) return fail(FTH_EINVAL, "ctx must not be NULL");
    if (c->R == 0) return fail(FTH_ESTATE, "state not allocated (replica count not fixed)");
    HIP_OK(hipStreamSynchronize(c->stream));
    const size_t cnt = size_t(c->n) * size_t(c->R);
    const size_t D = size_t(c->ns + 1), R = size_t(c->R);
    const bool f64 = c->prec == FTH_FP64;
    const size_t rb = c->real_bytes();
    auto put = [&](void* dst, const std::vector<double>& src) -> hipError_t {
        if (f64) return hipMemcpy(dst, src.data(), sizeof(double) * src.size(), hipMemcpyHostToDevice);
        std::vector<float> t(src.size());
        for (size_t k = 0; k < src.size(); ++k) t[k] = float(src[k]);
        return hipMemcpy(dst, t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice);
    };
    if (q) {
        HIP_OK(put(c->d_q[c->step & 1], std::vector<double>(q, q + cnt)));
        c->qt_dirty = true;
    }
    if (p || s) {
        // read-modify-write of the interleaved (p, s) block
        const size_t pscnt = c->ps_bytes() / rb;
        std::vector<double> psh(pscnt);
        if (f64) {
            HIP_OK(hipMemcpy(psh.data(), c->d_ps[c->step & 1], sizeof(double) * pscnt, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> t(pscnt);
            HIP_OK(hipMemcpy(t.data(), c->d_ps[c->step & 1], rb * pscnt, hipMemcpyDeviceToHost));
            for (size_t k = 0; k < pscnt; ++k) psh[k] = t[k];
        }
        for (size_t i = 0; i < size_t(c->n); ++i)
            for (size_t r = 0; r < R; ++r) {
                if (p) psh[c->ps_offset(int64_t(i), 0, int(r))] = p[i * R + r];
                if (s)
                    for (size_t k = 0; k + 1 < D; ++k)
                        psh[c->ps_offset(int64_t(i), int(k + 1), int(r))] = s[(k * size_t(c->n) + i) * R + r];
            }
        HIP_OK(put(c->d_ps[c->step & 1], psh));
    }
    return FTH_OK;
}

fth_status fth_force(fth_ctx* c, const double* q, double* F) {
    if (!c || !q || !F) return fail(FTH_EINVAL, "invalid arguments");
    if (!c->mfma()) return fail(FTH_EUNSUPPORTED, "fth_force is provided for dense contexts on the matrix-core path");
    if (c->R == 0) return fail(FTH_ESTATE, "replica count not fixed");
    HIP_OK(hipStreamSynchronize(c->stream));
    const int64_t P = c->rows_pad, R = c->R, n = c->n;
    const size_t rb = c->real_bytes();
    ctx_scratch tmp(c);
    auto alloc = [&](size_t b) -> void* { return tmp.get(b); };
    void* dq = alloc(size_t(P * R) * rb);
    void* dpart = alloc(size_t(c->ksplit) * size_t(P * R) * rb);
    int64_t* dstep = static_cast<int64_t*>(alloc(sizeof(int64_t)));
    const bool split = c->prec == FTH_FP32_BF16X3 && !c->gemv;
    uint16_t* dqt = split ? static_cast<uint16_t*>(alloc(size_t(P * R) * 4)) : nullptr;
    if (!dq || !dpart || !dstep || (split && !dqt)) return fail(FTH_ENOMEM, "scratch allocation failed");
    HIP_OK(hipMemset(dq, 0, size_t(P * R) * rb));
    HIP_OK(hipMemset(dstep, 0, sizeof(int64_t)));
    if (c->prec == FTH_FP64) {
        HIP_OK(hipMemcpy(dq, q, sizeof(double) * size_t(n * R), hipMemcpyHostToDevice));
    } else {
        std::vector<float> t(size_t(n * R));
        for (size_t k = 0; k < t.size(); ++k) t[k] = float(q[k]);
        HIP_OK(hipMemcpy(dq, t.data(), sizeof(float) * t.size(), hipMemcpyHostToDevice));
        if (split) {
            HIP_OK(hipMemset(dqt, 0, size_t(P * R) * 4));
            if (fth::launch_qt_from_q(static_cast<const float*>(dq), dqt, n, P, int32_t(R), c->stream) != 0)
                return fail(FTH_EDEVICE, "q split launch failed");
        }
    }
    fth::DenseGemmArgs g = gemm_args(c, 0);
    g.qt = dqt;
    g.q0 = dq;
    g.q1 = dq;
    g.step_base = dstep;
    g.part = dpart;
    const int rc = launch_force(c, g);
    if (rc != 0) return fail(FTH_EDEVICE, "dense force launch failed (%d)", rc);
    HIP_OK(hipStreamSynchronize(c->stream));
    const size_t pc = size_t(c->ksplit) * size_t(P * R);
    if (c->prec == FTH_FP64) {
        std::vector<double> part(pc);
        HIP_OK(hipMemcpy(part.data(), dpart, sizeof(double) * pc, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i)
            for (int64_t r = 0; r < R; ++r) {
                double acc = 0.0;
                for (int s = 0; s < c->ksplit; ++s) acc = acc + part[(size_t(s) * P + i) * R + r];
                F[i * R + r] = -acc;
            }
    } else {
        std::vector<float> part(pc);
        HIP_OK(hipMemcpy(part.data(), dpart, sizeof(float) * pc, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i)
            for (int64_t r = 0; r < R; ++r) {
                float acc = 0.0f;
                for (int s = 0; s < c->ksplit; ++s) acc = acc + part[(size_t(s) * P + i) * R + r];
                F[i * R + r] = -double(acc);
            }
    }
    return FTH_OK;
}

double fth_last_run_ms(const fth_ctx* c) { return c ? c->last_ms : 0.0; }

int32_t fth_launches_per_step(const fth_ctx* c) { return c ? (c->mfma() ? 2 : 1) : 0; }

fth_status fth_kernel_name(const fth_ctx* c, char* name, size_t len) {
    if (!c || !name || len == 0) return fail(FTH_EINVAL, "invalid arguments");
    if (c->small)
        std::snprintf(name, len, "small_dense_kernel<%s,NS=%d,RPT=%d> (persistent, M in %s)",
                      c->prec == FTH_FP64 ? "double" : "float", c->ns, c->rpt, c->small_m_in_lds ? "LDS" : "global");
    else if (c->gemv)
        std::snprintf(name, len, "dense_gemv_kernel<%s,R=%d> + dense_epilogue_kernel<%s,NS=%d,RPT=%d,NT=%d>",
                      c->prec == FTH_FP64 ? "double" : "float", c->R, c->prec == FTH_FP64 ? "double" : "float", c->ns,
                      c->rpt, int(c->nt));
    else if (c->dense())
        std::snprintf(name, len, "%s<RT=%d,ksplit=%d> + dense_epilogue_kernel<%s,NS=%d,RPT=%d,NT=%d>",
                      c->prec == FTH_FP64 ? "gemm_f64_kernel" : "gemm_bf16x3_kernel", c->R / 16, c->ksplit,
                      c->prec == FTH_FP64 ? "double" : "float", c->ns, c->rpt, int(c->nt));
    else if (c->tb_kt > 0 && c->tbp_grid > 0)
        std::snprintf(name, len,
                      "tbp_step_kernel<%s,NS=%d,KT=%d> block=%d grid=%d (persistent; + csr_step_kernel block=%d tail)%s",
                      c->prec == FTH_FP64 ? "double" : "float", c->ns, c->tb_kt, c->tb_block, c->tbp_grid, c->block,
                      c->tuned ? " (autotuned)" : "");
    else if (c->tb_kt > 0)
        std::snprintf(name, len, "tb_step_kernel<%s,NS=%d,RPT=4,KT=%d> block=%d (+ csr_step_kernel block=%d tail)%s",
                      c->prec == FTH_FP64 ? "double" : "float", c->ns, c->tb_kt, c->tb_block, c->block,
                      c->tuned ? " (autotuned)" : "");
    else
        std::snprintf(name, len, "csr_step_kernel<%s,NS=%d,RPT=%d,NT=%d,CODED=%d> block=%d%s%s",
                      c->prec == FTH_FP64 ? "double" : "float", c->ns, c->rpt, int(c->nt),
                      int(c->coded && c->rpt >= 4), c->block, long_rows(c) ? " (long-row batches)" : "",
                      c->tuned ? " (autotuned)" : "");
    return FTH_OK;
}

size_t fth_device_bytes(const fth_ctx* c) { return c ? c->device_bytes() : 0; }

namespace {
// Image layout (version 2): this header, q_n, (p, s)_n, the accumulators,
// then an FNV-1a checksum of everything before it.  The header records every
// parameter a continuation depends on, so an image is only accepted by a
// context that would have produced the same trajectory and estimates.
struct SaveHeader {
    char magic[8];
    uint32_t version, prec;
    int64_t n, R, ns, n_out, step, q_bytes, ps_bytes;
    uint64_t seed;
    uint32_t stream_id, poisoned;
    int64_t burn_in, block_len;
    double h;
    uint32_t acc_diag, acc_pp, acc_trace, reserved;
    uint64_t ts_hash;    // propagator T and S as used (FP64)
    uint64_t m_hash;     // matrix as used (after the spectral map), pattern and values
    uint64_t pair_hash;  // selected pairs in input order
};
constexpr uint32_t kSaveVersion = 2;
constexpr char kSaveMagic[8] = {'F', 'T', 'H', 'S', 'T', 'A', 'T', 'E'};

uint64_t fnv1a(const unsigned char* p, size_t n) {
    uint64_t h = 1469598103934665603ull;
    for (size_t k = 0; k < n; ++k) h = (h ^ p[k]) * 1099511628211ull;
    return h;
}

uint64_t ts_hash(const fth_ctx* c) {
    uint64_t hsh = hash_words(c->T.data(), c->T.size() * sizeof(double), 0);
    return hash_words(c->S.data(), c->S.size() * sizeof(double), hsh);
}

size_t image_bytes(const fth_ctx* c) {
    return sizeof(SaveHeader) + size_t(c->q_rows()) * size_t(c->R) * c->real_bytes() + c->ps_bytes() +
           sizeof(double) * 3 * size_t(c->n_out()) + sizeof(uint64_t);
}
}  // namespace

fth_status fth_save(fth_ctx* c, void* buf, size_t* len) {
    if (!c || !len) return fail(FTH_EINVAL, "invalid arguments");
    if (c->R == 0) return fail(FTH_ESTATE, "state not allocated (replica count not fixed)");
    const size_t need = image_bytes(c);
    if (!buf) {
        *len = need;
        return FTH_OK;
    }
    if (*len < need) return fail(FTH_EINVAL, "buffer too small (%zu < %zu bytes)", *len, need);
    HIP_OK(hipStreamSynchronize(c->stream));
    SaveHeader hd{};
    std::memcpy(hd.magic, kSaveMagic, 8);
    hd.version = kSaveVersion;
    hd.prec = uint32_t(c->prec);
    hd.n = c->n;
    hd.R = c->R;
    hd.ns = c->ns;
    hd.n_out = c->n_out();
    hd.step = c->step;
    hd.q_bytes = int64_t(size_t(c->q_rows()) * size_t(c->R) * c->real_bytes());
    hd.ps_bytes = int64_t(c->ps_bytes());
    hd.seed = c->opt.seed;
    hd.stream_id = c->opt.stream_id;
    hd.poisoned = c->poisoned ? 1u : 0u;
    hd.burn_in = c->opt.burn_in;
    hd.block_len = c->opt.block_len;
    hd.h = c->h;
    hd.acc_diag = c->opt.acc_diag ? 1u : 0u;
    hd.acc_pp = c->opt.acc_pp ? 1u : 0u;
    hd.acc_trace = c->opt.acc_trace ? 1u : 0u;
    hd.ts_hash = ts_hash(c);
    hd.m_hash = c->m_hash;
    hd.pair_hash = c->pair_hash;
    unsigned char* out = static_cast<unsigned char*>(buf);
    std::memcpy(out, &hd, sizeof(hd));
    size_t off = sizeof(hd);
    HIP_OK(hipMemcpy(out + off, c->d_q[c->step & 1], size_t(hd.q_bytes), hipMemcpyDeviceToHost));
    off += size_t(hd.q_bytes);
    HIP_OK(hipMemcpy(out + off, c->d_ps[c->step & 1], size_t(hd.ps_bytes), hipMemcpyDeviceToHost));
    off += size_t(hd.ps_bytes);
    const size_t ab = sizeof(double) * 3 * size_t(hd.n_out);
    if (ab) HIP_OK(hipMemcpy(out + off, c->d_acc, ab, hipMemcpyDeviceToHost));
    off += ab;
    const uint64_t sum = fnv1a(out, off);
    std::memcpy(out + off, &sum, sizeof(sum));
    *len = need;
    return FTH_OK;
}

fth_status fth_load(fth_ctx* c, const void* buf, size_t len) {
    if (!c || !buf) return fail(FTH_EINVAL, "invalid arguments");
    if (len < sizeof(SaveHeader) + sizeof(uint64_t)) return fail(FTH_EINVAL, "image too short");
    SaveHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (std::memcmp(hd.magic, kSaveMagic, 8) != 0) return fail(FTH_EINVAL, "not a state image");
    if (hd.version != kSaveVersion)
        return fail(FTH_EINVAL, "state image version %u is not supported (expected %u)", hd.version, kSaveVersion);
    if (hd.R < 1 || hd.R > 512) return fail(FTH_EINVAL, "damaged image (replicas)");
    fth_status st = ensure_state(c, int32_t(hd.R));
    if (st != FTH_OK) return st;
    if (image_bytes(c) != len) return fail(FTH_EINVAL, "image size %zu does not match this context (%zu)", len, image_bytes(c));
    if (hd.prec != uint32_t(c->prec) || hd.n != c->n || hd.ns != c->ns || hd.n_out != c->n_out() ||
        hd.q_bytes != int64_t(size_t(c->q_rows()) * size_t(c->R) * c->real_bytes()) ||
        hd.ps_bytes != int64_t(c->ps_bytes()))
        return fail(FTH_EINVAL, "image was saved from a context of another shape");
    if (hd.seed != c->opt.seed || hd.stream_id != c->opt.stream_id)
        return fail(FTH_EINVAL, "image was saved with another noise stream (seed or stream id)");
    if (hd.burn_in != c->opt.burn_in || hd.block_len != c->opt.block_len)
        return fail(FTH_EINVAL, "image was saved with another burn-in or block length");
    if (hd.h != c->h || hd.ts_hash != ts_hash(c))
        return fail(FTH_EINVAL, "image was saved with another time step or GLE");
    if (hd.acc_diag != (c->opt.acc_diag ? 1u : 0u) || hd.acc_pp != (c->opt.acc_pp ? 1u : 0u) ||
        hd.acc_trace != (c->opt.acc_trace ? 1u : 0u))
        return fail(FTH_EINVAL, "image was saved with other accumulators");
    if (hd.m_hash != c->m_hash) return fail(FTH_EINVAL, "image was saved for another matrix");
    if (hd.pair_hash != c->pair_hash) return fail(FTH_EINVAL, "image was saved for other pairs");
    if (hd.step < 0 || hd.step >= (int64_t(1) << 32)) return fail(FTH_EINVAL, "damaged image (step)");
    const unsigned char* in = static_cast<const unsigned char*>(buf);
    uint64_t sum;
    std::memcpy(&sum, in + len - sizeof(sum), sizeof(sum));
    if (fnv1a(in, len - sizeof(sum)) != sum) return fail(FTH_EINVAL, "image checksum mismatch");
    HIP_OK(hipStreamSynchronize(c->stream));
    c->step = hd.step;
    size_t off = sizeof(hd);
    HIP_OK(hipMemcpy(c->d_q[c->step & 1], in + off, size_t(hd.q_bytes), hipMemcpyHostToDevice));
    off += size_t(hd.q_bytes);
    HIP_OK(hipMemcpy(c->d_ps[c->step & 1], in + off, size_t(hd.ps_bytes), hipMemcpyHostToDevice));
    off += size_t(hd.ps_bytes);
    const size_t ab = sizeof(double) * 3 * size_t(hd.n_out);
    if (ab) HIP_OK(hipMemcpy(c->d_acc, in + off, ab, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->d_step, &c->step, sizeof(int64_t), hipMemcpyHostToDevice));
    const int32_t flag = hd.poisoned ? 1 : 0;
    HIP_OK(hipMemcpy(c->d_flag, &flag, sizeof(flag), hipMemcpyHostToDevice));
    c->poisoned = hd.poisoned != 0;
    c->qt_dirty = true;
    return FTH_OK;
}

fth_status fth_destroy(fth_ctx* c) {
    delete c;
    return FTH_OK;
}

}  // extern "C"
