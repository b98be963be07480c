// probe.hip -- sustained device rates for the rooflines of the product kernels:
// streaming HBM read and copy bandwidth, FP64 fma, and three ways of forming a
// modular product of 50-bit residues on the vector unit (the FP64 one the
// library uses, 64-bit Barrett and 64-bit Shoup).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "pimm_probe.h"

namespace {

constexpr int kChains = 8;
constexpr int kThreads = 256;

// Streaming reads: every wave reads one contiguous span of the buffer, eight
// loads in flight per lane, each wave instruction over 64 consecutive elements
// (1 KiB with 16-byte loads, 512 bytes with 8-byte loads), non-temporal.  A
// grid-stride loop, whose consecutive loads of a wave lie a grid apart, reads
// about 10% slower on MI355X.
template <class T>
__device__ __forceinline__ double read_span(const T *__restrict__ a, size_t n)
{
    constexpr int U = 8;
    const size_t waves = (size_t)gridDim.x * (kThreads / 64);
    const size_t wave = (size_t)blockIdx.x * (kThreads / 64) + threadIdx.x / 64;
    const size_t lane = threadIdx.x % 64;
    const size_t per = (n + waves - 1) / waves;
    const size_t begin = wave * per, end = begin + per < n ? begin + per : n;
    double s0 = 0.0, s1 = 0.0;
    size_t i = begin + lane;
    for (; i + (U - 1) * 64 < end; i += U * 64) {
        T x[U];
#pragma unroll
        for (int k = 0; k < U; ++k) x[k] = __builtin_nontemporal_load(a + i + k * 64);
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if constexpr (sizeof(T) == 16) {
                s0 += x[k][0];
                s1 += x[k][1];
            } else {
                s0 += x[k];
            }
        }
    }
    for (; i < end; i += 64) {
        if constexpr (sizeof(T) == 16)
            s0 += a[i][0] + a[i][1];
        else
            s0 += a[i];
    }
    return s0 + s1;
}

__global__ __launch_bounds__(kThreads) void k_read(const double2 *__restrict__ a, size_t n2,
                                                   double *__restrict__ out)
{
    typedef double v2 __attribute__((ext_vector_type(2)));
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = read_span((const v2 *)a, n2);
}

__global__ __launch_bounds__(kThreads) void k_read8(const double *__restrict__ a, size_t n,
                                                    double *__restrict__ out)
{
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = read_span(a, n);
}

__global__ __launch_bounds__(kThreads) void k_copy(const double2 *__restrict__ a,
                                                   double2 *__restrict__ b, size_t n2)
{
    const size_t stride = (size_t)gridDim.x * kThreads;
    size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + 3 * stride < n2; i += 4 * stride) {
        const double2 x0 = a[i], x1 = a[i + stride], x2 = a[i + 2 * stride], x3 = a[i + 3 * stride];
        b[i] = x0;
        b[i + stride] = x1;
        b[i + 2 * stride] = x2;
        b[i + 3 * stride] = x3;
    }
    for (; i < n2; i += stride) b[i] = a[i];
}

__global__ __launch_bounds__(kThreads) void k_fma64(double *__restrict__ out, int iters, double y,
                                                    double z)
{
    double x[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = (double)(threadIdx.x + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) x[j] = __builtin_fma(x[j], y, z);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += x[j];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_modmul_f64(double *__restrict__ out, int iters,
                                                         double c, double p, double pinv)
{
    double x[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = (double)(blockIdx.x * kThreads + threadIdx.x + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) x[j] = pimm::mulmod(x[j], c, p, pinv);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += x[j];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// Barrett for p < 2^50 (Menezes et al., Handbook of Applied Cryptography, 14.42
// with base 2 and k = 50): q = ((ab >> 49) * floor(2^100 / p)) >> 51 is at most
// two below floor(ab / p).
__device__ __forceinline__ uint64_t barrett50(uint64_t a, uint64_t b, uint64_t p, uint64_t mu)
{
    const uint64_t lo = a * b, hi = __umul64hi(a, b);
    const uint64_t q1 = (hi << 15) | (lo >> 49);
    const uint64_t q3 = (__umul64hi(q1, mu) << 13) | ((q1 * mu) >> 51);
    uint64_t r = lo - q3 * p;
    r = r >= p ? r - p : r;
    return r >= p ? r - p : r;
}

__global__ __launch_bounds__(kThreads) void k_modmul_barrett(uint64_t *__restrict__ out, int iters,
                                                             uint64_t c, uint64_t p, uint64_t mu)
{
    uint64_t x[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = (uint64_t)(blockIdx.x * kThreads + threadIdx.x + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) x[j] = barrett50(x[j], c, p, mu);
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s ^= x[j];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

// Shoup's product by a fixed w with w' = floor(w 2^64 / p): x w - hi(x w') p lies in [0, 2p).
__global__ __launch_bounds__(kThreads) void k_modmul_shoup(uint64_t *__restrict__ out, int iters,
                                                           uint64_t w, uint64_t wq, uint64_t p)
{
    uint64_t x[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = (uint64_t)(blockIdx.x * kThreads + threadIdx.x + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            const uint64_t r = x[j] * w - __umul64hi(x[j], wq) * p;
            x[j] = r >= p ? r - p : r;
        }
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s ^= x[j];
    out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

struct Run {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *a = nullptr, *b = nullptr, *o = nullptr;
    ~Run()
    {
        if (s) (void)hipStreamSynchronize(s);
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        if (o) (void)hipFree(o);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    }
};

// Time `reps` launches of `launch` after one untimed one; seconds per launch.
template <typename F>
int timed(Run &r, int reps, F launch, double *sec)
{
    launch();
    if (hipEventRecord(r.e0, r.s) != hipSuccess) return PIMM_E_DEVICE;
    for (int i = 0; i < reps; ++i) launch();
    if (hipEventRecord(r.e1, r.s) != hipSuccess || hipEventSynchronize(r.e1) != hipSuccess ||
        hipGetLastError() != hipSuccess)
        return PIMM_E_DEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess || ms <= 0.f) return PIMM_E_DEVICE;
    *sec = (double)ms * 1e-3 / reps;
    return PIMM_OK;
}

}  // namespace

extern "C" int pimm_probe(int device, int kind, uint64_t size, int reps, double *rate)
{
    if (!rate || reps < 1 || kind < PIMM_PROBE_READ || kind > PIMM_PROBE_READ8) return PIMM_E_ARG;
    const bool mem = kind <= PIMM_PROBE_COPY || kind == PIMM_PROBE_READ8;
    if (mem ? (size < (16u << 20) || size % 16 != 0) : (size < 1024 || size > (1u << 30)))
        return PIMM_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return PIMM_E_DEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0)
        return PIMM_E_DEVICE;
    Run r;
    if (hipStreamCreate(&r.s) != hipSuccess || hipEventCreate(&r.e0) != hipSuccess ||
        hipEventCreate(&r.e1) != hipSuccess)
        return PIMM_E_DEVICE;
    const unsigned max_grid = (unsigned)cus * 16;
    if (hipMalloc(&r.o, (size_t)max_grid * kThreads * 8) != hipSuccess) return PIMM_E_OOM;

    if (mem) {
        if (hipMalloc(&r.a, size) != hipSuccess) return PIMM_E_OOM;
        if (kind == PIMM_PROBE_COPY && hipMalloc(&r.b, size) != hipSuccess) return PIMM_E_OOM;
        if (hipMemsetAsync(r.a, 0, size, r.s) != hipSuccess) return PIMM_E_DEVICE;
        const size_t n2 = size / 16;
        double best = 0.0;
        for (unsigned per_cu = 2; per_cu <= 16; per_cu *= 2) {
            const unsigned grid = (unsigned)cus * per_cu;
            double sec = 0.0;
            int rc;
            if (kind == PIMM_PROBE_READ)
                rc = timed(r, reps, [&] {
                    hipLaunchKernelGGL(k_read, dim3(grid), dim3(kThreads), 0, r.s,
                                       (const double2 *)r.a, n2, (double *)r.o);
                }, &sec);
            else if (kind == PIMM_PROBE_READ8)
                rc = timed(r, reps, [&] {
                    hipLaunchKernelGGL(k_read8, dim3(grid), dim3(kThreads), 0, r.s,
                                       (const double *)r.a, size / 8, (double *)r.o);
                }, &sec);
            else
                rc = timed(r, reps, [&] {
                    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kThreads), 0, r.s,
                                       (const double2 *)r.a, (double2 *)r.b, n2);
                }, &sec);
            if (rc != PIMM_OK) return rc;
            const double bytes = kind == PIMM_PROBE_COPY ? 2.0 * (double)size : (double)size;
            if (bytes / sec > best) best = bytes / sec;
        }
        *rate = best;
        return PIMM_OK;
    }

    // Arithmetic: a grid of 8 workgroups per CU, 8 independent chains per lane.
    const unsigned grid = (unsigned)cus * 8;
    const int iters = (int)size;
    const double lanes = (double)grid * kThreads * kChains * iters;
    const uint64_t p = 1125899906842597ull;  // 2^50 - 27
    const double pd = (double)p, pinv = 1.0 / pd;
    const uint64_t c = 0x2b7e151628aedull % p, w = 0x3243f6a8885a3ull % p;
    const uint64_t mu = (uint64_t)(((unsigned __int128)1 << 100) / p);
    const uint64_t wq = (uint64_t)(((unsigned __int128)w << 64) / p);
    double sec = 0.0;
    int rc = PIMM_OK;
    switch (kind) {
    case PIMM_PROBE_FMA64:
        rc = timed(r, reps, [&] {
            hipLaunchKernelGGL(k_fma64, dim3(grid), dim3(kThreads), 0, r.s, (double *)r.o, iters,
                               0.9990234375, 0.0009765625);
        }, &sec);
        *rate = 2.0 * lanes / sec;
        break;
    case PIMM_PROBE_MODMUL_F64:
        rc = timed(r, reps, [&] {
            hipLaunchKernelGGL(k_modmul_f64, dim3(grid), dim3(kThreads), 0, r.s, (double *)r.o,
                               iters, (double)c - pd * 0.5, pd, pinv);
        }, &sec);
        *rate = lanes / sec;
        break;
    case PIMM_PROBE_MODMUL_BARRETT:
        rc = timed(r, reps, [&] {
            hipLaunchKernelGGL(k_modmul_barrett, dim3(grid), dim3(kThreads), 0, r.s,
                               (uint64_t *)r.o, iters, c, p, mu);
        }, &sec);
        *rate = lanes / sec;
        break;
    default:
        rc = timed(r, reps, [&] {
            hipLaunchKernelGGL(k_modmul_shoup, dim3(grid), dim3(kThreads), 0, r.s, (uint64_t *)r.o,
                               iters, w, wq, p);
        }, &sec);
        *rate = lanes / sec;
        break;
    }
    return rc;
}
