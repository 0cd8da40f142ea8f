// Spectral map of the f-thermostat (Sec. I, scaling paragraph): run the
// dynamics on M' = r M + m I with A'_p = alpha A_p, C'_p = gamma C_p, so a GLE
// fitted on one spectral window serves any spectrum, and map the estimates
// back for targets with a suitable algebra (ln, exp, powers).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "fth_ctx.hpp"

namespace fth {
namespace host {

fth_status spectral_transform(const fth_matrix* M, double r, double m, std::vector<double>& store, fth_matrix* out) {
    if (!std::isfinite(r) || !std::isfinite(m) || r == 0.0) return fail(FTH_EINVAL, "scale_r must be finite and non-zero, scale_m finite");
    *out = *M;
    out->value_is_f64 = 1;
    auto value = [&](const void* v, int64_t k) {
        return M->value_is_f64 ? static_cast<const double*>(v)[k] : double(static_cast<const float*>(v)[k]);
    };
    if (M->format == FTH_CSR) {
        if (!M->row_ptr || !M->col || !M->val || M->nnz < 0) return fail(FTH_EINVAL, "incomplete CSR matrix");
        // structure first (the full validation runs on M' afterwards)
        if (M->row_ptr[0] != 0 || M->row_ptr[M->n] != M->nnz) return fail(FTH_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] == nnz");
        for (int64_t i = 0; i < M->n; ++i)
            if (M->row_ptr[i + 1] < M->row_ptr[i]) return fail(FTH_EINVAL, "row_ptr must be non-decreasing");
        store.resize(size_t(M->nnz));
        for (int64_t k = 0; k < M->nnz; ++k) store[size_t(k)] = r * value(M->val, k);
        if (m != 0.0)
            for (int64_t i = 0; i < M->n; ++i) {
                bool found = false;
                for (int64_t k = M->row_ptr[i]; k < M->row_ptr[i + 1]; ++k)
                    if (M->col[k] == i) {
                        store[size_t(k)] += m;
                        found = true;
                    }
                if (!found) return fail(FTH_EINVAL, "a diagonal shift needs a stored diagonal entry in row %lld", (long long)i);
            }
        out->val = store.data();
    } else {
        if (!M->dense) return fail(FTH_EINVAL, "dense matrix pointer is NULL");
        const size_t cnt = size_t(M->n) * size_t(M->n);
        store.resize(cnt);
        for (size_t k = 0; k < cnt; ++k) store[k] = r * value(M->dense, int64_t(k));
        for (int64_t i = 0; i < M->n; ++i) store[size_t(i) * size_t(M->n) + size_t(i)] += m;
        out->dense = store.data();
    }
    return FTH_OK;
}

fth_status scaled_gle(const fth_gle* g, double alpha, double gamma, std::vector<double>& A, std::vector<double>& C,
                      fth_gle* out) {
    if (!(alpha > 0) || !(gamma > 0) || !std::isfinite(alpha) || !std::isfinite(gamma))
        return fail(FTH_EINVAL, "gle_alpha and gle_gamma must be positive");
    if (g->ns < 0 || !g->A_p || !g->C_p) return fail(FTH_EINVAL, "invalid GLE");
    const size_t d2 = size_t(g->ns + 1) * size_t(g->ns + 1);
    A.assign(g->A_p, g->A_p + d2);
    C.assign(g->C_p, g->C_p + d2);
    for (double& x : A) x *= alpha;
    for (double& x : C) x *= gamma;
    *out = fth_gle{g->ns, A.data(), C.data()};
    return FTH_OK;
}

}  // namespace host
}  // namespace fth

using namespace fth::host;

extern "C" {

fth_status fth_spectral_map(double e_min, double e_max, double w_min, double w_max, double* r, double* m) {
    if (!r || !m) return fail(FTH_EINVAL, "r and m must not be NULL");
    if (!std::isfinite(e_min) || !std::isfinite(e_max) || !std::isfinite(w_min) || !std::isfinite(w_max) ||
        !(e_min < e_max) || !(w_min < w_max))
        return fail(FTH_EINVAL, "need finite e_min < e_max and w_min < w_max");
    *r = (w_min - w_max) / (e_min - e_max);
    *m = (e_min * w_max - e_max * w_min) / (e_min - e_max);  // r e_min + m = w_min, r e_max + m = w_max
    return FTH_OK;
}

fth_status fth_gershgorin(const fth_matrix* M, double* lo, double* hi) {
    if (!M || !lo || !hi) return fail(FTH_EINVAL, "invalid arguments");
    auto value = [&](const void* v, int64_t k) {
        return M->value_is_f64 ? static_cast<const double*>(v)[k] : double(static_cast<const float*>(v)[k]);
    };
    double l = INFINITY, h = -INFINITY;
    for (int64_t i = 0; i < M->n; ++i) {
        double d = 0.0, off = 0.0;
        if (M->format == FTH_CSR) {
            for (int64_t k = M->row_ptr[i]; k < M->row_ptr[i + 1]; ++k) {
                if (M->col[k] == i)
                    d += value(M->val, k);
                else
                    off += std::fabs(value(M->val, k));
            }
        } else {
            for (int64_t j = 0; j < M->n; ++j) {
                const double v = value(M->dense, i * M->n + j);
                if (j == i)
                    d = v;
                else
                    off += std::fabs(v);
            }
        }
        l = std::fmin(l, d - off);
        h = std::fmax(h, d + off);
    }
    *lo = l;
    *hi = h;
    return FTH_OK;
}

fth_status fth_unscale(int32_t target, double r, double m, double alpha, double gamma, int64_t count,
                       const double* kind_weight, double* est, double* se) {
    if (count < 0 || (count > 0 && !kind_weight)) return fail(FTH_EINVAL, "invalid output description");
    if (!(alpha > 0) || !(gamma > 0)) return fail(FTH_EINVAL, "alpha and gamma must be positive");
    const double a2 = alpha * alpha;
    const double rr = r / a2, mm = m / a2;  // the response is (gamma/alpha^2) g(M' / alpha^2)
    double factor = a2 / gamma, shift = 0.0;
    switch (target) {
        case FTH_TARGET_INVSQRT:
            if (mm != 0.0 || !(rr > 0)) return fail(FTH_EINVAL, "x^-1/2 is recovered from M' = r M with r > 0 only");
            factor *= std::sqrt(rr);
            break;
        case FTH_TARGET_LN:
            if (mm != 0.0 || !(rr > 0)) return fail(FTH_EINVAL, "ln is recovered from M' = r M with r > 0 only");
            shift = -std::log(rr);
            break;
        case FTH_TARGET_EXPNEG:  // e^-(r' M + m') = e^-m' e^-(r' M): recovers exp(-r' M)
            if (!(rr > 0)) return fail(FTH_EINVAL, "exp(-x) needs r > 0");
            factor *= std::exp(mm);
            break;
        default:
            return fail(FTH_EINVAL, "unknown target %d", int(target));
    }
    for (int64_t k = 0; k < count; ++k) {
        if (est) est[k] = est[k] * factor + shift * kind_weight[k];
        if (se) se[k] = se[k] * std::fabs(factor);
    }
    return FTH_OK;
}

}  // extern "C"
