// Host FP64 linear algebra for the per-solve setup of the GLE propagator:
// T = exp(-A_p h) and S = chol(C_p - T C_p T^T) on (ns+1) x (ns+1) blocks.
//
// exp: scaling and squaring with the diagonal [8/8] Pade approximant of e^x.
// The Pade coefficients follow from the classical recurrence
//   c_0 = 1,  c_{k+1} = c_k (m - k) / ((2m - k)(k + 1)),
// N(x) = sum c_k x^k, D(x) = N(-x).  The argument is scaled by 2^-s so that
// its 1-norm is at most 1/2, where the [8/8] truncation error is below
// 1e-23 relative, then the result is squared s times.
#include <cmath>
#include <cstring>
#include <vector>

#include "fth_internal.h"

namespace fth {
namespace la {

namespace {

void matmul(const double* A, const double* B, double* C, int n) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += A[i * n + k] * B[k * n + j];
            C[i * n + j] = acc;
        }
}

double norm1(const double* A, int n) {
    double best = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += std::fabs(A[i * n + j]);
        if (s > best) best = s;
    }
    return best;
}

// Solve D X = N for X (Gaussian elimination with partial pivoting).
bool solve(std::vector<double> D, std::vector<double> N, int n, double* X) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(D[r * n + c]) > std::fabs(D[piv * n + c])) piv = r;
        if (D[piv * n + c] == 0.0) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                std::swap(D[c * n + k], D[piv * n + k]);
                std::swap(N[c * n + k], N[piv * n + k]);
            }
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = D[r * n + c] / D[c * n + c];
            if (f == 0.0) continue;
            for (int k = c; k < n; ++k) D[r * n + k] -= f * D[c * n + k];
            for (int k = 0; k < n; ++k) N[r * n + k] -= f * N[c * n + k];
        }
    }
    for (int col = 0; col < n; ++col) {
        for (int r = n - 1; r >= 0; --r) {
            double v = N[r * n + col];
            for (int k = r + 1; k < n; ++k) v -= D[r * n + k] * X[k * n + col];
            X[r * n + col] = v / D[r * n + r];
        }
    }
    return true;
}

}  // namespace

bool expm(const double* A, int n, double* out) {
    for (int i = 0; i < n * n; ++i)
        if (!std::isfinite(A[i])) return false;
    const int m = 8;
    double c[m + 1];
    c[0] = 1.0;
    for (int k = 0; k < m; ++k) c[k + 1] = c[k] * double(m - k) / (double(2 * m - k) * double(k + 1));

    int s = 0;
    const double nrm = norm1(A, n);
    if (nrm > 0.5) s = int(std::ceil(std::log2(nrm / 0.5)));
    const double scale = std::ldexp(1.0, -s);
    std::vector<double> X(n * n), P(n * n), tmp(n * n), Nm(n * n, 0.0), Dm(n * n, 0.0);
    for (int i = 0; i < n * n; ++i) X[i] = A[i] * scale;
    // P = X^k, accumulate N = sum c_k X^k, D = sum (-1)^k c_k X^k
    for (int i = 0; i < n; ++i) {
        P[i * n + i] = 1.0;
        Nm[i * n + i] = c[0];
        Dm[i * n + i] = c[0];
    }
    for (int k = 1; k <= m; ++k) {
        matmul(P.data(), X.data(), tmp.data(), n);
        P = tmp;
        const double sg = (k % 2) ? -1.0 : 1.0;
        for (int i = 0; i < n * n; ++i) {
            Nm[i] += c[k] * P[i];
            Dm[i] += sg * c[k] * P[i];
        }
    }
    std::vector<double> R(n * n);
    if (!solve(Dm, Nm, n, R.data())) return false;
    for (int q = 0; q < s; ++q) {
        matmul(R.data(), R.data(), tmp.data(), n);
        R = tmp;
    }
    std::memcpy(out, R.data(), sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i)
        if (!std::isfinite(out[i])) return false;
    return true;
}

bool cholesky(const double* A, int n, double* L, double rel_tol) {
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) dmax = std::fmax(dmax, std::fabs(A[i * n + i]));
    std::memset(L, 0, sizeof(double) * n * n);
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > rel_tol * dmax) || !std::isfinite(d)) return false;
        const double ljj = std::sqrt(d);
        L[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = v / ljj;
        }
    }
    return true;
}

void sym_eigvals(const double* A0, int n, double* ev) {
    std::vector<double> A(A0, A0 + n * n);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        if (off < 1e-30) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
            }
    }
    for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
}

}  // namespace la
}  // namespace fth
