// ntt.h -- negacyclic NTT kernels for gfx950 (one workgroup per polynomial).
//
// The polynomial products of the protocol go through the NTT and pointwise
// products (the paper's footnote in section 3.1.3).  The forward transform is
// the merged Cooley-Tukey form: stage s (s = 0 .. log N - 1) pairs elements
// j and j + t, t = N / 2^(s+1), and multiplies the upper one by
// psi^bitrev(2^s + i), i = j / (2t), which folds the negacyclic twist psi^j
// into the butterflies.  The inverse undoes the stages in reverse order with
// the inverse twiddles (Gentleman-Sande) and a final factor N^-1.
//
// Stages are grouped into passes of PS consecutive stages.  Within a pass the
// 2^PS elements a butterfly group touches sit in one thread's registers, so
// only passes exchange data through LDS (N doubles: 32 KiB at N = 4096,
// 64 KiB at N = 8192).  The transform's output order is free: nothing in NTT
// form crosses the ABI and every NTT-form operand uses the same order, so the
// last forward pass writes element c of set S to slot c * NSETS + S, which
// makes its global stores coalesced; the inverse's first pass reads the same.
//
// Loaders produce a double of magnitude <= p for (poly, prime, index);
// storers consume a balanced double.  Poly index p of a [..][L][N] buffer
// belongs to prime p % L.
#pragma once

#include "common.h"

namespace pimm {

constexpr int kNttThreads = 256;

template <int LOGN>
struct NttSched;
template <>
struct NttSched<12> {
    static constexpr int P0 = 4, P1 = 4, P2 = 4;
};
template <>
struct NttSched<13> {
    static constexpr int P0 = 5, P1 = 4, P2 = 4;
};

// LDS slot of element j, padded by one double every 32 to break bank aliasing
// of the strided pass patterns.
__device__ __forceinline__ int lds_idx(int j) { return j + (j >> 5); }

template <int LOGN, int S0, int PS>
struct Pass {
    static constexpr int N = 1 << LOGN;
    static constexpr int E = 1 << PS;
    static constexpr int STRIDE = N >> (S0 + PS);
    static constexpr int NSETS = N >> PS;
    static constexpr int PER_THREAD = NSETS / kNttThreads;
    static_assert(PER_THREAD >= 1 && NSETS % kNttThreads == 0, "pass shape");

    // Element index of member c of set S.
    __device__ static __forceinline__ int elem(int S, int c)
    {
        return (S / STRIDE) * (N >> S0) + (S % STRIDE) + c * STRIDE;
    }

    // Forward stages S0 .. S0+PS-1 on the registers of set S.
    __device__ static __forceinline__ void fwd(double *x, int S, const double *tw, double p,
                                               double pinv)
    {
        const int hi = S / STRIDE;
#pragma unroll
        for (int sp = 0; sp < PS; ++sp) {
            const int half = E >> (sp + 1);
#pragma unroll
            for (int c = 0; c < E; ++c) {
                if (c & half) continue;
                const double w = tw[(1 << (S0 + sp)) + (hi << sp) + (c >> (PS - sp))];
                const double u = x[c];
                const double v = mulmod(x[c + half], w, p, pinv);
                x[c] = u + v;
                x[c + half] = u - v;
            }
        }
    }

    // Inverse stages S0+PS-1 .. S0 on the registers of set S.
    __device__ static __forceinline__ void inv(double *x, int S, const double *tw, double p,
                                               double pinv)
    {
        const int hi = S / STRIDE;
#pragma unroll
        for (int sp = PS - 1; sp >= 0; --sp) {
            const int half = E >> (sp + 1);
#pragma unroll
            for (int c = 0; c < E; ++c) {
                if (c & half) continue;
                const double w = tw[(1 << (S0 + sp)) + (hi << sp) + (c >> (PS - sp))];
                const double u = x[c], v = x[c + half];
                x[c] = reduce(u + v, p, pinv);
                x[c + half] = mulmod(u - v, w, p, pinv);
            }
        }
    }
};

template <int LOGN>
struct NttPasses {
    using S = NttSched<LOGN>;
    using A = Pass<LOGN, 0, S::P0>;
    using B = Pass<LOGN, S::P0, S::P1>;
    using C = Pass<LOGN, S::P0 + S::P1, S::P2>;
    static_assert(S::P0 + S::P1 + S::P2 == LOGN, "schedule covers every stage");
    static constexpr int N = 1 << LOGN;
    static constexpr int LDS = N + (N >> 5);
};

// Forward negacyclic NTT of polynomial `poly` by the calling workgroup
// (kNttThreads threads), with `lds` holding NttPasses<LOGN>::LDS doubles.
template <int LOGN, class Load, class Store>
__device__ __forceinline__ void ntt_fwd_block(const Load &ld, const Store &st, const DevParams &dp,
                                              int poly, double *lds)
{
    using NP = NttPasses<LOGN>;
    using PA = typename NP::A;
    using PB = typename NP::B;
    using PC = typename NP::C;
    const int l = poly % dp.L;
    const double p = dp.p[l], pinv = dp.pinv[l];
    const double *tw = dp.tw_fwd + ((size_t)l << LOGN);
    const int tid = threadIdx.x;

#pragma unroll
    for (int k = 0; k < PA::PER_THREAD; ++k) {
        const int S = tid + k * kNttThreads;
        double x[PA::E];
#pragma unroll
        for (int c = 0; c < PA::E; ++c) x[c] = ld(poly, l, PA::elem(S, c), p, pinv);
        PA::fwd(x, S, tw, p, pinv);
#pragma unroll
        for (int c = 0; c < PA::E; ++c) lds[lds_idx(PA::elem(S, c))] = reduce(x[c], p, pinv);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PB::PER_THREAD; ++k) {
        const int S = tid + k * kNttThreads;
        double x[PB::E];
#pragma unroll
        for (int c = 0; c < PB::E; ++c) x[c] = lds[lds_idx(PB::elem(S, c))];
        PB::fwd(x, S, tw, p, pinv);
#pragma unroll
        for (int c = 0; c < PB::E; ++c) lds[lds_idx(PB::elem(S, c))] = reduce(x[c], p, pinv);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PC::PER_THREAD; ++k) {
        const int S = tid + k * kNttThreads;
        double x[PC::E];
#pragma unroll
        for (int c = 0; c < PC::E; ++c) x[c] = lds[lds_idx(PC::elem(S, c))];
        PC::fwd(x, S, tw, p, pinv);
#pragma unroll
        for (int c = 0; c < PC::E; ++c) st(poly, l, c * PC::NSETS + S, reduce(x[c], p, pinv), p, pinv);
    }
}

// Inverse negacyclic NTT (including the factor N^-1) of polynomial `poly`.
template <int LOGN, class Load, class Store>
__device__ __forceinline__ void ntt_inv_block(const Load &ld, const Store &st, const DevParams &dp,
                                              int poly, double *lds)
{
    using NP = NttPasses<LOGN>;
    using PA = typename NP::A;
    using PB = typename NP::B;
    using PC = typename NP::C;
    const int l = poly % dp.L;
    const double p = dp.p[l], pinv = dp.pinv[l];
    const double *tw = dp.tw_inv + ((size_t)l << LOGN);
    const int tid = threadIdx.x;

#pragma unroll
    for (int k = 0; k < PC::PER_THREAD; ++k) {
        const int S = tid + k * kNttThreads;
        double x[PC::E];
#pragma unroll
        for (int c = 0; c < PC::E; ++c) x[c] = ld(poly, l, c * PC::NSETS + S, p, pinv);
        PC::inv(x, S, tw, p, pinv);
#pragma unroll
        for (int c = 0; c < PC::E; ++c) lds[lds_idx(PC::elem(S, c))] = reduce(x[c], p, pinv);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PB::PER_THREAD; ++k) {
        const int S = tid + k * kNttThreads;
        double x[PB::E];
#pragma unroll
        for (int c = 0; c < PB::E; ++c) x[c] = lds[lds_idx(PB::elem(S, c))];
        PB::inv(x, S, tw, p, pinv);
#pragma unroll
        for (int c = 0; c < PB::E; ++c) lds[lds_idx(PB::elem(S, c))] = reduce(x[c], p, pinv);
    }
    __syncthreads();
    const double ninv = dp.n_inv[l];
#pragma unroll
    for (int k = 0; k < PA::PER_THREAD; ++k) {
        const int S = tid + k * kNttThreads;
        double x[PA::E];
#pragma unroll
        for (int c = 0; c < PA::E; ++c) x[c] = lds[lds_idx(PA::elem(S, c))];
        PA::inv(x, S, tw, p, pinv);
#pragma unroll
        for (int c = 0; c < PA::E; ++c)
            st(poly, l, PA::elem(S, c), mulmod(x[c], ninv, p, pinv), p, pinv);
    }
}

template <int LOGN, class Load, class Store>
__global__ __launch_bounds__(kNttThreads) void k_ntt_fwd(Load ld, Store st, DevParams dp)
{
    __shared__ double lds[NttPasses<LOGN>::LDS];
    ntt_fwd_block<LOGN>(ld, st, dp, (int)blockIdx.x, lds);
}

// Forward transform that also clears its share of another buffer (the
// product's accumulators), saving a launch: workgroup b zeroes
// zero[b * per, (b + 1) * per), per = ceil(zero_n / gridDim.x).
template <int LOGN, class Load, class Store>
__global__ __launch_bounds__(kNttThreads) void k_ntt_fwd_zero(Load ld, Store st, double *zero,
                                                              size_t zero_n, DevParams dp)
{
    __shared__ double lds[NttPasses<LOGN>::LDS];
    ntt_fwd_block<LOGN>(ld, st, dp, (int)blockIdx.x, lds);
    const size_t per = (zero_n + gridDim.x - 1) / gridDim.x;
    const size_t b = (size_t)blockIdx.x * per;
    const size_t e = b + per < zero_n ? b + per : zero_n;
    for (size_t i = b + threadIdx.x; i < e; i += kNttThreads) zero[i] = 0.0;
}

template <int LOGN, class Load, class Store>
__global__ __launch_bounds__(kNttThreads) void k_ntt_inv(Load ld, Store st, DevParams dp)
{
    __shared__ double lds[NttPasses<LOGN>::LDS];
    ntt_inv_block<LOGN>(ld, st, dp, (int)blockIdx.x, lds);
}

// Inverse transform whose result stays in the workgroup's LDS (natural order,
// lds_idx layout), followed by an epilogue that reads it with the whole
// workgroup: epi(poly, lds, dp).  The last pass's storer writes exactly the
// elements its thread has just read, so no barrier is needed before it.
struct StoreLds {
    double *lds;
    __device__ void operator()(int, int, int j, double v, double, double) const
    {
        lds[lds_idx(j)] = v;
    }
};

template <int LOGN, class Load, class Epi>
__global__ __launch_bounds__(kNttThreads) void k_ntt_inv_lds(Load ld, Epi epi, DevParams dp)
{
    __shared__ double lds[NttPasses<LOGN>::LDS];
    const int poly = (int)blockIdx.x;
    ntt_inv_block<LOGN>(ld, StoreLds{lds}, dp, poly, lds);
    __syncthreads();
    epi(poly, lds, dp);
}

// ---- loaders ----------------------------------------------------------------

// Canonical uint64 residues, [npoly][N].
struct LoadU64 {
    const uint64_t *in;
    int logn;
    __device__ double operator()(int poly, int, int j, double, double) const
    {
        return (double)in[((size_t)poly << logn) + j];
    }
};

// Small signed integers shared by the L primes: source poly = poly / L.
struct LoadI64Shared {
    const int64_t *in;
    int logn, L;
    __device__ double operator()(int poly, int, int j, double, double) const
    {
        return (double)in[((size_t)(poly / L) << logn) + j];
    }
};

// Pointwise product of two NTT-form operands: a[poly] * b[poly % bmod].
struct LoadSlotsMul {
    const double *a, *b;
    int logn, bmod;
    __device__ double operator()(int poly, int, int z, double p, double pinv) const
    {
        return mulmod(a[((size_t)poly << logn) + z], b[((size_t)(poly % bmod) << logn) + z], p,
                      pinv);
    }
};

// NTT-form operand as is.
struct LoadSlots {
    const double *a;
    int logn;
    __device__ double operator()(int poly, int, int z, double, double) const
    {
        return a[((size_t)poly << logn) + z];
    }
};

// ---- storers ----------------------------------------------------------------

struct StoreSlots {
    double *out;
    int logn;
    __device__ void operator()(int poly, int, int z, double v, double, double) const
    {
        out[((size_t)poly << logn) + z] = v;
    }
};

struct StoreU64 {
    uint64_t *out;
    int logn;
    __device__ void operator()(int poly, int, int j, double v, double p, double pinv) const
    {
        out[((size_t)poly << logn) + j] = to_canonical(v, p, pinv);
    }
};

// Instantiate and launch a transform for the context's ring degree.
template <class Load, class Store>
int launch_fwd(const Ctx &c, Load ld, Store st, int npoly, hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_fwd", s);
    if (c.dp.logN == 12)
        hipLaunchKernelGGL((k_ntt_fwd<12, Load, Store>), dim3(npoly), dim3(kNttThreads), 0, s, ld,
                           st, c.dp);
    else
        hipLaunchKernelGGL((k_ntt_fwd<13, Load, Store>), dim3(npoly), dim3(kNttThreads), 0, s, ld,
                           st, c.dp);
    return check_hip(hipGetLastError(), "ntt_fwd launch");
}

template <class Load, class Store>
int launch_fwd_zero(const Ctx &c, Load ld, Store st, int npoly, double *zero, size_t zero_n,
                    hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_fwd", s);
    if (c.dp.logN == 12)
        hipLaunchKernelGGL((k_ntt_fwd_zero<12, Load, Store>), dim3(npoly), dim3(kNttThreads), 0, s,
                           ld, st, zero, zero_n, c.dp);
    else
        hipLaunchKernelGGL((k_ntt_fwd_zero<13, Load, Store>), dim3(npoly), dim3(kNttThreads), 0, s,
                           ld, st, zero, zero_n, c.dp);
    return check_hip(hipGetLastError(), "ntt_fwd launch");
}

template <class Load, class Store>
int launch_inv(const Ctx &c, Load ld, Store st, int npoly, hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_inv", s);
    if (c.dp.logN == 12)
        hipLaunchKernelGGL((k_ntt_inv<12, Load, Store>), dim3(npoly), dim3(kNttThreads), 0, s, ld,
                           st, c.dp);
    else
        hipLaunchKernelGGL((k_ntt_inv<13, Load, Store>), dim3(npoly), dim3(kNttThreads), 0, s, ld,
                           st, c.dp);
    return check_hip(hipGetLastError(), "ntt_inv launch");
}

template <class Load, class Epi>
int launch_inv_lds(const Ctx &c, Load ld, Epi epi, int npoly, hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_inv", s);
    if (c.dp.logN == 12)
        hipLaunchKernelGGL((k_ntt_inv_lds<12, Load, Epi>), dim3(npoly), dim3(kNttThreads), 0, s, ld,
                           epi, c.dp);
    else
        hipLaunchKernelGGL((k_ntt_inv_lds<13, Load, Epi>), dim3(npoly), dim3(kNttThreads), 0, s, ld,
                           epi, c.dp);
    return check_hip(hipGetLastError(), "ntt_inv launch");
}

}  // namespace pimm
