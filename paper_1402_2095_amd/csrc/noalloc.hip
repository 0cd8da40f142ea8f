// Dense force for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
// F = -M q with the same GEMM and partial-sum order as fth_force, its work
// buffers in one fixed device array per GPU instead of per-call allocations.
#include <mutex>

#include "dense.hpp"
#include "fth_ctx.hpp"

namespace {

// Work buffers of fth_force_noalloc: the padded (split-form: bf16 hi/lo
// tiled) copy of q, then the split-K partial sums.  Each GPU the library runs
// on holds its own copy until the process ends; every call on that GPU
// shares it.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (looked up once per device, with
// that device current; the host-side name is not a device address).
fth_status scratch_address(int dev, void** out) {
    using fth::host::fail;
    if (dev < 0 || dev >= kMaxDevices) return fail(FTH_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        HIP_OK(hipGetDevice(&cur));
        if (cur != dev) HIP_OK(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || p == nullptr)
            return fail(FTH_EDEVICE, "scratch symbol lookup failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FTH_OK;
}

}  // namespace

namespace fth {
namespace dev {

// q [n][R] FP32 -> the GEMM's bf16 hi/lo tiled split, rows n..P-1 zero.
__global__ void noalloc_qt_kernel(const float* __restrict__ q, uint16_t* __restrict__ qt, int64_t n, int64_t P,
                                  int32_t R) {
    const int64_t total = P * R;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t k = t / R, r = t % R;
        put_qt(qt, k, r, R, k < n ? q[t] : 0.0f);
    }
}

// q [n][R] FP64 -> [P][R], rows n..P-1 zero.
__global__ void noalloc_pad_kernel(const double* __restrict__ q, double* __restrict__ qp, int64_t n, int64_t P,
                                   int32_t R) {
    const int64_t total = P * R;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x)
        qp[t] = t < n * R ? q[t] : 0.0;
}

// F[i][r] = -(sum over K slices s = 0, 1, ... of part[s][i][r]), in slice order.
template <typename Real>
__global__ void noalloc_sum_kernel(const Real* __restrict__ part, Real* __restrict__ F, int64_t n, int64_t P,
                                   int32_t R, int32_t ks) {
    const int64_t total = n * R;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
        Real acc = Real(0);
        for (int s = 0; s < ks; ++s) acc = acc + part[int64_t(s) * P * R + t];
        F[t] = -acc;
    }
}

}  // namespace dev
}  // namespace fth

using namespace fth::host;

extern "C" fth_status fth_force_noalloc(fth_ctx* c, const void* q, void* F, void* hip_stream) {
    if (!c || !q || !F) return fail(FTH_EINVAL, "invalid arguments");
    if (!c->mfma() || c->gemv)
        return fail(FTH_EUNSUPPORTED, "fth_force_noalloc is provided for dense contexts on the matrix-core path");
    if (c->R == 0) return fail(FTH_ESTATE, "replica count not fixed");
    const int64_t P = c->rows_pad, R = c->R, n = c->n;
    const bool f64 = c->prec == FTH_FP64;
    const size_t rb = f64 ? 8 : 4;
    const size_t qbytes = size_t(P) * size_t(R) * (f64 ? 8 : 4);  // padded q, or its bf16 hi/lo split
    const size_t pbytes = size_t(c->ksplit) * size_t(P) * size_t(R) * rb;
    if (qbytes + pbytes > kScratchBytes)
        return fail(FTH_EINVAL, "this system needs %zu bytes of work space; the fixed scratch array holds %zu",
                    qbytes + pbytes, kScratchBytes);
    void* base = nullptr;
    fth_status st = scratch_address(c->device, &base);
    if (st != FTH_OK) return st;
    int cur = 0;
    HIP_OK(hipGetDevice(&cur));
    if (cur != c->device) HIP_OK(hipSetDevice(c->device));
    const hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream;
    unsigned char* qs = static_cast<unsigned char*>(base);
    void* part = qs + qbytes;  // qbytes is a multiple of 256 (P is)
    fth::DenseGemmArgs g{};
    g.m_hi = c->d_m_hi;
    g.step_base = c->d_step;  // read only: selects between q0 and q1, which are the same buffer here
    g.k = 0;
    g.part = part;
    g.rows_pad = P;
    g.R = int32_t(R);
    g.ksplit = c->ksplit;
    g.kslice = P / c->ksplit;
    int rc;
    if (f64) {
        hipLaunchKernelGGL(fth::dev::noalloc_pad_kernel, dim3(1024), dim3(256), 0, s, static_cast<const double*>(q),
                           reinterpret_cast<double*>(qs), n, P, int32_t(R));
        g.q0 = g.q1 = qs;
        rc = hipGetLastError() == hipSuccess ? fth::launch_gemm_f64(g, s) : -1;
        if (rc == 0)
            hipLaunchKernelGGL(fth::dev::noalloc_sum_kernel<double>, dim3(1024), dim3(256), 0, s,
                               static_cast<const double*>(part), static_cast<double*>(F), n, P, int32_t(R), c->ksplit);
    } else {
        hipLaunchKernelGGL(fth::dev::noalloc_qt_kernel, dim3(1024), dim3(256), 0, s, static_cast<const float*>(q),
                           reinterpret_cast<uint16_t*>(qs), n, P, int32_t(R));
        g.qt = reinterpret_cast<const uint16_t*>(qs);
        rc = hipGetLastError() == hipSuccess ? fth::launch_gemm_bf16x3(g, s) : -1;
        if (rc == 0)
            hipLaunchKernelGGL(fth::dev::noalloc_sum_kernel<float>, dim3(1024), dim3(256), 0, s,
                               static_cast<const float*>(part), static_cast<float*>(F), n, P, int32_t(R), c->ksplit);
    }
    const hipError_t e = hipGetLastError();
    if (cur != c->device) (void)hipSetDevice(cur);
    if (rc != 0 || e != hipSuccess) return fail(FTH_EDEVICE, "force launch failed (%d): %s", rc, hipGetErrorString(e));
    return FTH_OK;
}
