// server.hip -- the server's side of Pi_MatMul (Algorithm 1 steps 1 and 3 and
// the sparse reply of section 3.1.3).
//
// The product [[c]] = a [[b]] of step 3, accumulated over the inner blocks, is
// for every NTT slot z and prime l a small modular matrix product
//     acc^[ib, kb](z) = sum_jb  W^[ib, jb](z) * c^[jb, kb](z),
// done for both ciphertext components.  The weight transforms W^ are computed
// once per weight matrix and kept in HBM (the weights are static), so the
// per-call work is: forward NTT of the I input ciphertexts, the slot-wise
// products (which stream W^ once: 8 bytes per two modular MACs when each
// weight block meets one input column block), and the inverse NTT of the O
// accumulators.
#include <string.h>

#include "common.h"
#include "mac.h"
#include "mfma.h"
#include "ntt.h"

namespace pimm {

// ---- weights (Algorithm 1 step 1, pi_A) ---------------------------------------------

// Coefficient j of block w = ib*R + jb of pi_A(W^T), read straight from W [r][m]:
// j = i*rb + rb - 1 - jj holds W[jb*rb + jj][ib*mb + i]; j >= mb*rb is zero.
// Largest weight magnitude the transform takes: the weights enter the NTT as
// balanced doubles, which must stay exact and below a few primes.
constexpr unsigned long long kMaxWeight = 1ull << 48;

// Weight block w = (g*M + ib)*R + jb of product g (W: [G][r][m]).
struct LoadWeights {
    const int64_t *W;
    uint32_t r, m, mb, rb, R, M;
    int L;
    __device__ double operator()(const PolyIx &pi, int j, double, double) const
    {
        const uint32_t uj = (uint32_t)j;
        if (uj >= mb * rb) return 0.0;
        const uint32_t w = (uint32_t)pi.x;
        const uint32_t rowblk = w / R, jb = w % R, g = rowblk / M, ib = rowblk % M;
        const int64_t *W = this->W + (size_t)g * r * m;
        const uint32_t i = uj / rb, jj = rb - 1 - uj % rb;
        const uint32_t row = jb * rb + jj, col = ib * mb + i;
        if (row >= r || col >= m) return 0.0;
        return (double)W[(size_t)row * m + col];
    }
};

__global__ void k_absmax(const int64_t *W, size_t n, unsigned long long *out)
{
    unsigned long long best = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int64_t v = W[i];
        const unsigned long long a = v < 0 ? (unsigned long long)(-(v + 1)) + 1 : (unsigned long long)v;
        best = a > best ? a : best;
    }
    atomicMax(out, best);
}

// (The slot-wise products of step 3 are in mac.h / mac.hip.)

// ---- re-randomisation, mask and extraction --------------------------------------

// The re-randomisation draws of every output ciphertext y in one launch: u_y
// (ternary, stream RR_U) into u [O][N], e1_y and e2_y (Gaussian, RR_E1 / RR_E2)
// into e [O][2][N], one signed byte each.
static SampleJobs rerand_jobs(uint32_t O, size_t N, int8_t *u, int8_t *e)
{
    SampleJobs js{};
    js.n = 3;
    js.job[0] = SampleJob{kSampleTernary8, kTagRrU, 0, (int)O, 0, 1, u, N, 0, 0};
    js.job[1] = SampleJob{kSampleGauss8, kTagRrE1, 0, (int)O, 0, 1, e, 2 * N, 0, 0};
    js.job[2] = SampleJob{kSampleGauss8, kTagRrE2, 0, (int)O, 0, 1, e + N, 2 * N, 0, 0};
    return js;
}

// Pointwise u^[o][l] * pk^[comp][l] for polynomials [O][2][L].
struct LoadRerand {
    const double *uh;   // [O][L][N]
    const double *pkh;  // [2][L][N]
    int logn, L;
    __device__ double operator()(const PolyIx &pi, int z, double p, double pinv) const
    {
        const size_t o = (size_t)(pi.x >> 1), comp = (size_t)(pi.x & 1), l = (size_t)pi.l;
        return mulmod(uh[((o * L + l) << logn) + z], pkh[((comp * L + l) << logn) + z], p, pinv);
    }
};

// Inputs of the re-randomisation transforms as one polynomial list: the 2L
// polynomials of pk (canonical residues, [2][L][N], LoadU64) then, for each output
// ciphertext, u shared by the L primes (one signed byte per coefficient, [O][N]):
// polynomial index poly keeps prime poly % L in both parts (2L is a multiple of L), and
// u's polynomial is poly / L - x0 with x0 = 2.
struct LoadI8Shared {
    const int8_t *u;
    int logn;
    uint32_t x0;
    __device__ double operator()(const PolyIx &pi, int j, double, double) const
    {
        return (double)u[((size_t)(pi.x - x0) << logn) + j];
    }
};

// acc[o][comp][l][j] += (u pk_comp)_j + e_comp[j]  (mod q_l); e: [O][2][N].  The
// accumulator and error words are read ahead of the transform's last pass (Pre).
struct StoreAddErr {
    uint64_t *acc;
    const int8_t *e;
    int logn, L;
    struct Pre {
        uint64_t a;
        int e;
    };
    __device__ Pre pre(const PolyIx &pi, int j) const
    {
        return Pre{acc[((size_t)pi.poly << logn) + j], (int)e[((size_t)pi.x << logn) + j]};
    }
    __device__ void operator()(const PolyIx &pi, int j, double v, double p, double pinv,
                               const Pre &pr) const
    {
        const uint64_t q = (uint64_t)p;
        const uint64_t up = to_canonical(v, p, pinv);
        const uint64_t ee = lift_small((int64_t)pr.e, q);
        acc[((size_t)pi.poly << logn) + j] = add_mod(add_mod(pr.a, up, q), ee, q);
    }
};

// One thread per decoded coefficient of each output ciphertext y:
// s = mask draw number pos of stream (MASK, 0, op, y);
// c0s[y][l][k*mb + i] = [acc0[pos] - Delta_l s]_{q_l}; server share = s.
__global__ void k_mask_extract(Key key, uint32_t op, const uint64_t *acc, uint64_t *c0s,
                               uint64_t *share, pimm_plan_info f, DevParams dp)
{
    const uint32_t per = f.mb * f.nb;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)f.O * per) return;
    const uint32_t y = (uint32_t)(gid / per), idx = (uint32_t)(gid % per);
    const uint32_t k = idx / f.mb, i = idx % f.mb;
    const uint32_t pos = k * f.mb * f.rb + i * f.rb + f.rb - 1;
    uint32_t w[16];
    chacha_block(key, pos / 8, nonce0(kTagMask, 0), op, y, w);
    const uint64_t sm = mask_of(word64(w, (int)(pos % 8)), dp.ell);
    const size_t N = (size_t)dp.N, L = (size_t)dp.L;
    uint64_t a0[kMaxL];  // every prime's word read before the first store
#pragma unroll
    for (int l = 0; l < kMaxL; ++l)
        if (l < dp.L) a0[l] = acc[(((size_t)y * 2 + 0) * L + l) * N + pos];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l)
        if (l < dp.L)
            c0s[((size_t)y * L + l) * per + idx] =
                sub_mod(a0[l], mul_mod(dp.delta[l], sm, dp.p[l], dp.pinv[l]), dp.q[l]);
    const OutPos yp = out_pos(y, f);
    const uint32_t row = yp.kb * f.nb + k, col = yp.ib * f.mb + i;
    if (row < f.n && col < f.m) share[(size_t)yp.g * f.n * f.m + (size_t)row * f.m + col] = sm;
}

// ---- fused server step: product, re-randomisation, mask and reply ----------------

// acc^ (reduced) plus, with re-randomisation (RR), u^ pk^ (NTT domain) for polynomials
// [O][2][L]; RUN: acc^ in the matrix-core product's layout (acc_run_index).  Both choices are
// compile-time, so the reads of a pass carry no branches and are issued together.
template <bool RR, bool RUN>
struct LoadAccRerand {
    const double *ah;   // [O][2][L][N], or the matrix-core layout with RUN
    const double *uh;   // [O][L][N]
    const double *pkh;  // [2][L][N]
    int logn, L;
    uint32_t O2, NR;  // 2 * O and N / kAccRun (RUN layout)
    __device__ double operator()(const PolyIx &pi, int z, double p, double pinv) const
    {
        const size_t at = RUN ? acc_run_index(pi, z, O2, NR) : ((size_t)pi.poly << logn) + z;
        double v = reduce(ah[at], p, pinv);
        if constexpr (RR) {
            const size_t o = (size_t)(pi.x >> 1), comp = (size_t)(pi.x & 1), l = (size_t)pi.l;
            v += mulmod(uh[((o * L + l) << logn) + z], pkh[((comp * L + l) << logn) + z], p, pinv);
        }
        return v;
    }
};

// The reply of output ciphertext y from its coefficient form in LDS: add the
// re-randomisation error (RR), then write c1 (component 1, every coefficient) or
// the unmasked c0 at the m_b n_b decoded positions k*mb*rb + i*rb + rb - 1
// (component 0).  The error bytes a thread needs (all 16 of a c1 polynomial, the first
// round of 4 decoded positions of a c0 one) are read before the transform (Pre).
template <bool RR>
struct ReplyOutBase {
    uint64_t *c1, *c0s;
    const int8_t *e;  // [O][2][N]
    FastDiv mb;
    uint32_t rb, nb;
    int logn, L;
    static constexpr int kPer = 16;  // coefficients per thread: N / T for both ring degrees
    static constexpr int kB = 4;     // decoded positions per round
    // Component 0 is read at the decoded positions only.
    __device__ bool sparse(const PolyIx &pi) const { return (pi.x & 1) == 0; }
    __device__ uint32_t pos_of(uint32_t idx) const
    {
        const uint32_t k = mb.div(idx), i = idx - k * mb.d;
        return (k * mb.d + i) * rb + rb - 1;
    }
    template <int LOGN, int T>
    __device__ void run_with(const PolyIx &pi, const double *lds, const DevParams &dp, const int *e16) const
    {
        static_assert((1 << LOGN) / T == kPer, "coefficients per thread");
        const int l = pi.l;
        const uint32_t y = (uint32_t)(pi.x >> 1), comp = (uint32_t)(pi.x & 1);
        const double p = dp.p[l], pinv = dp.pinv[l];
        const int8_t *ey = e + (((size_t)y * 2 + comp) << LOGN);
        // The transform's output (within 1.5 q_l) plus the error (|e| <= 19), reduced once.
        if (comp == 1) {
            uint64_t *dst = c1 + (((size_t)y * L + l) << LOGN);
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int j = (int)threadIdx.x + k * T;
                dst[j] = to_canonical(lds[lds_idx(j)] + (double)e16[k], p, pinv);
            }
            return;
        }
        const uint32_t per = mb.d * nb;
        uint64_t *dst = c0s + ((size_t)y * L + l) * per;
        for (uint32_t idx0 = threadIdx.x; idx0 < per; idx0 += kB * T) {
            uint32_t jj[kB];
            double ev[kB];
            const bool first = idx0 == threadIdx.x;
#pragma unroll
            for (int b = 0; b < kB; ++b) {
                const uint32_t idx = idx0 + b * T;
                jj[b] = pos_of(idx);
                ev[b] = first ? (double)e16[b] : ((RR && idx < per) ? (double)ey[jj[b]] : 0.0);
            }
#pragma unroll
            for (int b = 0; b < kB; ++b) {
                const uint32_t idx = idx0 + b * T;
                if (idx < per) dst[idx] = to_canonical(lds[lds_idx((int)jj[b])] + ev[b], p, pinv);
            }
        }
    }
};

template <bool RR>
struct ReplyOut;

// With re-randomisation: the error bytes come ahead of the transform.
template <>
struct ReplyOut<true> : ReplyOutBase<true> {
    struct Pre {
        int e[kPer];
    };
    template <int LOGN, int T>
    __device__ Pre pre(const PolyIx &pi) const
    {
        Pre pr;
        const uint32_t y = (uint32_t)(pi.x >> 1), comp = (uint32_t)(pi.x & 1);
        const int8_t *ey = e + (((size_t)y * 2 + comp) << LOGN);
        if (comp == 1) {
#pragma unroll
            for (int k = 0; k < kPer; ++k) pr.e[k] = ey[(int)threadIdx.x + k * T];
        } else {
            const uint32_t per = mb.d * nb;
            // Every lane reads (position 0 past the end) and selects: a read under a branch
            // would wait for every read issued before it.
#pragma unroll
            for (int b = 0; b < kB; ++b) {
                const uint32_t idx = threadIdx.x + b * T;
                const int v = ey[idx < per ? pos_of(idx) : 0u];
                pr.e[b] = idx < per ? v : 0;
            }
        }
        return pr;
    }
    template <int LOGN, int T>
    __device__ void run(const PolyIx &pi, const double *lds, const DevParams &dp, const Pre &pr) const
    {
        run_with<LOGN, T>(pi, lds, dp, pr.e);
    }
    // The bytes read after the transform instead (still all before the first store).
    template <int LOGN, int T>
    __device__ void run(const PolyIx &pi, const double *lds, const DevParams &dp) const
    {
        const Pre pr = pre<LOGN, T>(pi);
        run_with<LOGN, T>(pi, lds, dp, pr.e);
    }
};

template <>
struct ReplyOut<false> : ReplyOutBase<false> {
    template <int LOGN, int T>
    __device__ void run(const PolyIx &pi, const double *lds, const DevParams &dp) const
    {
        const int zero[kPer] = {};
        run_with<LOGN, T>(pi, lds, dp, zero);
    }
};

// The mask of output ciphertext y over Z_t at its decoded positions
// pos = k*mb*rb + i*rb + rb-1: s = mask draw number pos of stream (MASK, 0, op, y);
// c0s[y][l][k*mb + i] -= Delta_l s (every prime) and the server's share is s.
// Two thread layouts compute the same values: with rb >= 8 a ChaCha20 block holds at
// most one decoded position, so one thread per decoded position (no block computed for
// nothing); with rb < 8 one thread per block takes the block's 8 / rb positions.
__device__ __forceinline__ void mask_one(uint64_t *c0s, uint64_t *share, uint32_t y, uint32_t idx,
                                         uint64_t sm, const pimm_plan_info &f, const DevParams &dp)
{
    const uint32_t per = f.mb * f.nb;
    uint64_t *dst = c0s + (size_t)y * dp.L * per + idx;
    // Every prime's word is read (prime 0's again past L) before the first store, without a
    // branch around the reads.
    uint64_t cur[kMaxL];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l) cur[l] = dst[(size_t)(l < dp.L ? l : 0) * per];
#pragma unroll
    for (int l = 0; l < kMaxL; ++l)
        if (l < dp.L)
            dst[(size_t)l * per] = sub_mod(cur[l], mul_mod(dp.delta[l], sm, dp.p[l], dp.pinv[l]), dp.q[l]);
    const OutPos yp = out_pos(y, f);
    const uint32_t k = idx / f.mb, i = idx - k * f.mb;
    const uint32_t row = yp.kb * f.nb + k, col = yp.ib * f.mb + i;
    if (row < f.n && col < f.m) share[(size_t)yp.g * f.n * f.m + (size_t)row * f.m + col] = sm;
}

__global__ void k_mask_reply_pos(Key key, uint32_t op, uint64_t *c0s, uint64_t *share, pimm_plan_info f,
                                 DevParams dp)
{
    const uint32_t per = f.mb * f.nb;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)f.O * per) return;
    const uint32_t y = (uint32_t)(gid / per), idx = (uint32_t)(gid % per);
    const uint32_t k = idx / f.mb, i = idx - k * f.mb;
    const uint32_t pos = (k * f.mb + i) * f.rb + f.rb - 1;
    uint32_t w[16];
    chacha_block(key, pos / 8, nonce0(kTagMask, 0), op, y, w);
    mask_one(c0s, share, y, idx, mask_of(word64(w, (int)(pos % 8)), dp.ell), f, dp);
}

__global__ void k_mask_reply(Key key, uint32_t op, uint64_t *c0s, uint64_t *share, uint32_t blocks,
                             pimm_plan_info f, DevParams dp)
{
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)f.O * blocks) return;
    const uint32_t y = (uint32_t)(gid / blocks), b = (uint32_t)(gid % blocks);
    uint32_t w[16];
    chacha_block(key, b, nonce0(kTagMask, 0), op, y, w);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const uint32_t pos = b * 8 + t;
        if (pos % f.rb != f.rb - 1) continue;
        const uint32_t k = pos / (f.mb * f.rb), i = (pos / f.rb) % f.mb;
        if (k >= f.nb) continue;
        mask_one(c0s, share, y, k * f.mb + i, mask_of(word64(w, t), dp.ell), f, dp);
    }
}

// The reply transform of every output polynomial: acc^ (+ u^ pk^), inverse transform,
// + error, then c1 and the decoded positions of c0.
template <bool RR, bool RUN>
static int reply_transform(const Ctx &c, const pimm_plan_info &f, const double *ah, const double *uh,
                           const double *pkh, uint64_t *c1, uint64_t *c0s, const int8_t *e, hipStream_t s)
{
    const int lg = c.dp.logN;
    const int L = (int)c.params.L;
    return launch_inv_lds(c, LoadAccRerand<RR, RUN>{ah, uh, pkh, lg, L, 2 * f.O, (uint32_t)(c.params.N / kAccRun)},
                          ReplyOut<RR>{{c1, c0s, e, FastDiv::make(f.mb), f.rb, f.nb, lg, L}},
                          (int)(f.O * 2 * L), prune_factor(f.rb), s);
}

// The re-randomised reply of output ciphertext y at prime l by one workgroup (O L
// workgroups; ntt_poly() = y L + l keeps a ciphertext's primes on one XCD):
//  - the forward transform of u (one byte per coefficient, shared by the primes), whose
//    last pass leaves each thread's slots in LDS where the inverse's first pass (the same
//    sets on the same threads) reads them back;
//  - the first inverse pass of both components on acc^ + u^ pk^: component 0 pruned to the
//    few registers its decoded positions depend on, component 1 into LDS;
//  - the rest of component 1's inverse and its epilogue (c1), then component 0's.
// The same values as the forward transform of u to memory followed by the reply transform
// of each component, without u^ leaving the compute unit.  Four waves per SIMD (at most 128
// registers) keep two 512-thread workgroups on a compute unit, as their LDS allows; left to
// itself the compiler takes 130 registers and one workgroup.
template <int LOGN, int G, bool RUN>
__global__ __launch_bounds__(ntt_threads<LOGN>()) __attribute__((amdgpu_waves_per_eu(4))) void k_reply_rr(const int8_t *u, const double *ah,
                                                                    const double *pkh, ReplyOut<true> epi,
                                                                    uint32_t O2, uint32_t NR, DevParams dp)
{
    constexpr int T = ntt_threads<LOGN>();
    using NP = NttPasses<LOGN, T>;
    using P = typename NP::PFirst;
    static_assert(P::PER_THREAD == 1 && P::E == 16 && P::STRIDE == 1, "one set of 16 adjacent slots per thread");
    static_assert(G == 4 || G == 16, "pruned component 0");
    __shared__ double lds[NP::LDS];
    const int wg = ntt_poly();
    const int L = dp.L;
    const int y = wg / L, l = wg - y * L;
    ntt_fwd_block<LOGN, T>(LoadI8Shared{u, LOGN, 0u}, StoreKeepLds{}, dp, wg, lds);
    const PolyIx p0{(y * 2) * L + l, l, y * 2}, p1{(y * 2 + 1) * L + l, l, y * 2 + 1};
    const double p = dp.p[l], pinv = dp.pinv[l];
    const double *tw = dp.tw_inv + ((size_t)l << LOGN);
    const int S = (int)threadIdx.x;
    const int b0 = lds_idx(P::elem(S, 0));
    const double *pk0 = pkh + ((size_t)l << LOGN), *pk1 = pkh + ((size_t)(L + l) << LOGN);
    double s0[P::E / G];
    {
        double x[P::E];
#pragma unroll
        for (int c = 0; c < P::E; ++c) {
            const int z = c * P::NSETS + S;
            const size_t at = RUN ? acc_run_index(p0, z, O2, NR) : ((size_t)p0.poly << LOGN) + z;
            x[c] = reduce(ah[at], p, pinv) + mulmod(lds[b0 + P::lds_off(c)], pk0[z], p, pinv);
        }
        P::template inv_pruned<G>(x, S, tw, p, pinv);
#pragma unroll
        for (int c = G - 1; c < P::E; c += G) s0[c / G] = reduce(x[c], p, pinv);
    }
    // One component's reads at a time (both at once would not fit two workgroups per CU).
    __builtin_amdgcn_sched_barrier(0);
    {
        double x[P::E];
#pragma unroll
        for (int c = 0; c < P::E; ++c) {
            const int z = c * P::NSETS + S;
            const size_t at = RUN ? acc_run_index(p1, z, O2, NR) : ((size_t)p1.poly << LOGN) + z;
            x[c] = reduce(ah[at], p, pinv) + mulmod(lds[b0 + P::lds_off(c)], pk1[z], p, pinv);
        }
        P::inv(x, S, tw, p, pinv);
#pragma unroll
        for (int c = 0; c < P::E; ++c) lds[b0 + P::lds_off(c)] = reduce(x[c], p, pinv);
    }
    // Every wave is past the forward's passes that read the LDS twiddle table.
    __syncthreads();
    load_tw_table<LOGN, T>(tw, lds);
    // The error bytes of both epilogues, read ahead of component 1's other passes.
    const ReplyOut<true>::Pre e1 = epi.template pre<LOGN, T>(p1);
    const ReplyOut<true>::Pre e0 = epi.template pre<LOGN, T>(p0);
    __syncthreads();
    ntt_inv_rest<LOGN, T, 1>(StoreLds{lds}, dp, p1, lds);
    __syncthreads();
    epi.template run<LOGN, T>(p1, lds, dp, e1);
    __syncthreads();
#pragma unroll
    for (int c = G - 1; c < P::E; c += G) lds[b0 + P::lds_off(c)] = s0[c / G];
    __syncthreads();
    ntt_inv_rest<LOGN, T, G>(StoreLds{lds}, dp, p0, lds);
    __syncthreads();
    epi.template run<LOGN, T>(p0, lds, dp, e0);
}

template <int LOGN, bool RUN>
static void launch_reply_rr(int g, const int8_t *u, const double *ah, const double *pkh,
                            const ReplyOut<true> &epi, uint32_t O2, uint32_t NR, int nwg, const DevParams &dp,
                            hipStream_t s)
{
    if (g == 16)
        hipLaunchKernelGGL((k_reply_rr<LOGN, 16, RUN>), dim3(nwg), dim3(ntt_threads<LOGN>()), 0, s, u, ah, pkh,
                           epi, O2, NR, dp);
    else
        hipLaunchKernelGGL((k_reply_rr<LOGN, 4, RUN>), dim3(nwg), dim3(ntt_threads<LOGN>()), 0, s, u, ah, pkh,
                           epi, O2, NR, dp);
}

// The re-randomised reply from u (bytes) and pk^ in one launch (k_reply_rr); for plans
// whose reply needs every coefficient of c0 (no output pruning) the caller takes the
// separate transform of u and the reply transform instead.
template <bool RUN>
static int reply_rr(const Ctx &c, const pimm_plan_info &f, const int8_t *u, const double *ah, const double *pkh,
                    uint64_t *c1, uint64_t *c0s, const int8_t *e, hipStream_t s)
{
    const int lg = c.dp.logN;
    const int L = (int)c.params.L;
    const int g = prune_factor(f.rb);
    if (g < 4) return set_error(PIMM_E_ARG, "reply_rr: the plan's reply allows no output pruning");
    const ReplyOut<true> epi{{c1, c0s, e, FastDiv::make(f.mb), f.rb, f.nb, lg, L}};
    const uint32_t O2 = 2 * f.O, NR = (uint32_t)(c.params.N / kAccRun);
    ProfScope prof("ntt_inv", s);
    if (lg == 12)
        launch_reply_rr<12, RUN>(g, u, ah, pkh, epi, O2, NR, (int)(f.O * L), c.dp, s);
    else
        launch_reply_rr<13, RUN>(g, u, ah, pkh, epi, O2, NR, (int)(f.O * L), c.dp, s);
    return check_hip(hipGetLastError(), "reply_rr launch");
}

// The query ciphertexts (already in evaluation form) into the vector product's tiled layout
// as balanced doubles, and the accumulators zeroed, in one launch.
static int ct_to_tiled(const Ctx &c, const pimm_plan_info &f, const uint64_t *ct, double *ch, double *ah,
                       hipStream_t s)
{
    const int lg = c.dp.logN, L = (int)c.params.L;
    const size_t N = c.params.N;
    return launch_move(c, LoadSlotsBalanced{ct, lg}, StoreCtTiled{ch, lg, L, f.K, f.R, f.groups, -1},
                       (int)(f.I * 2 * L), ah, (size_t)f.O * 2 * L * N, s);
}

// The fused step after the product, on the workspace laid out as
// c^ [I][2][L][N], acc^ [O][2][L][N], pk^ [2][L][N], u^ [O][L][N] (doubles),
// u [O][N], e [O][2][N] (int64), acc^ already summed over the inner blocks:
// re-randomisation draws and transforms, the inverse transform with the reply
// epilogue, then the mask at the decoded positions and the server's share.
int fused_tail(const pimm_plan *plan, const uint64_t *pk, const Key &key, uint32_t op_id,
               double *ws, uint64_t *c1, uint64_t *c0s, uint64_t *server_share, bool mx_layout,
               hipStream_t s)
{
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    const size_t N = c.params.N, L = c.params.L;
    const int rr = c.params.rerandomize ? 1 : 0;
    const int lg = c.dp.logN;
    double *ah = ws + (size_t)f.I * 2 * L * N;
    double *pkh = ah + (size_t)f.O * 2 * L * N;
    double *uh = pkh + 2 * L * N;
    // u [O][N] and e [O][2][N], one byte each, at the start of their int64-sized regions.
    int8_t *u = (int8_t *)(uh + (size_t)f.O * L * N);
    int8_t *e = u + (size_t)f.O * N * 8;
    int rc = PIMM_OK;
    // With output pruning the transform of u runs inside the reply's workgroups (u^ stays on
    // chip); otherwise pk^ and u^ are transformed in one launch (adjacent in the workspace).
    const bool in_reply = rr && prune_factor(f.rb) >= 4;
    if (rr) {
        rc = launch_samples(c, key, op_id, rerand_jobs(f.O, N, u, e), s);
        if (!rc && in_reply)
            rc = launch_fwd(c, LoadU64{pk, lg}, StoreSlots{pkh, lg}, (int)(2 * L), s);
        else if (!rc)
            rc = launch_fwd2(c, LoadU64{pk, lg}, LoadI8Shared{u, lg, 2u}, (int)(2 * L), StoreSlots{pkh, lg},
                             (int)((2 + f.O) * L), s);
    }
    if (!rc) {
        if (in_reply)
            rc = mx_layout ? reply_rr<true>(c, f, u, ah, pkh, c1, c0s, e, s)
                           : reply_rr<false>(c, f, u, ah, pkh, c1, c0s, e, s);
        else if (rr)
            rc = mx_layout ? reply_transform<true, true>(c, f, ah, uh, pkh, c1, c0s, e, s)
                       : reply_transform<true, false>(c, f, ah, uh, pkh, c1, c0s, e, s);
        else
            rc = mx_layout ? reply_transform<false, true>(c, f, ah, uh, pkh, c1, c0s, e, s)
                       : reply_transform<false, false>(c, f, ah, uh, pkh, c1, c0s, e, s);
    }
    if (!rc) {
        ProfScope prof("mask_extract", s);
        if (f.rb >= 8) {
            const size_t total = (size_t)f.O * f.mb * f.nb;
            hipLaunchKernelGGL(k_mask_reply_pos, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, key,
                               op_id, c0s, server_share, f, c.dp);
        } else {
            const uint32_t blocks = (f.mb * f.rb * f.nb + 7) / 8;
            const size_t total = (size_t)f.O * blocks;
            hipLaunchKernelGGL(k_mask_reply, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, key,
                               op_id, c0s, server_share, blocks, f, c.dp);
        }
        rc = check_hip(hipGetLastError(), "mask_reply launch");
    }
    return rc;
}

}  // namespace pimm

using namespace pimm;

namespace pimm {
// A weight cache holds pi_A blocks in NTT form; it serves every plan with the
// same context, matrix shape (r, m) and block split (mb, rb), whatever n and nb.
bool weights_fit(const Weights *w, const Plan *plan)
{
    const pimm_plan_info &a = w->info, &b = plan->info;
    return w->ctx == plan->ctx && a.r == b.r && a.m == b.m && a.mb == b.mb && a.rb == b.rb &&
           a.groups == b.groups;
}

// The matrix-core product needs an eligible plan and the digit form of the weights.
int mfma_ready(const Plan *plan, const Weights *w, const char *who)
{
    if (!mfma_eligible(plan->info))
        return set_error(PIMM_E_UNSUPPORTED,
                         "%s: the matrix-core product needs at most 64 inner blocks and at least 8 "
                         "column blocks (plan: R = %u, K = %u)",
                         who, plan->info.R, plan->info.K);
    if (!w->d_w_dig)
        return set_error(PIMM_E_UNSUPPORTED,
                         "%s: the weight cache has no digit form (it is built when the cache is "
                         "made for a plan the matrix-core product serves)",
                         who);
    return PIMM_OK;
}
}  // namespace pimm

extern "C" {

int pimm_weights_create(const pimm_plan *plan, const int64_t *W, pimm_weights **out, void *stream)
{
    if (!plan || !W || !out) return set_error(PIMM_E_ARG, "pimm_weights_create: NULL argument");
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    hipStream_t s = (hipStream_t)stream;
    int rc = check_hip(hipSetDevice(c.device), "hipSetDevice");
    if (rc) return rc;
    unsigned long long *d_max = nullptr, h_max = 0;
    rc = check_hip(hipMalloc((void **)&d_max, sizeof *d_max), "hipMalloc absmax");
    if (rc) return rc;
    rc = check_hip(hipMemsetAsync(d_max, 0, sizeof *d_max, s), "memset absmax");
    if (!rc) {
        hipLaunchKernelGGL(k_absmax, dim3(1024), dim3(256), 0, s, W, (size_t)f.groups * f.r * f.m,
                           d_max);
        rc = check_hip(hipGetLastError(), "absmax launch");
    }
    if (!rc) rc = check_hip(hipMemcpyAsync(&h_max, d_max, sizeof h_max, hipMemcpyDeviceToHost, s),
                            "copy absmax");
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "absmax synchronize");
    (void)hipFree(d_max);
    if (rc) return rc;
    if (h_max > kMaxWeight)
        return set_error(PIMM_E_ARG, "max |W| = %llu exceeds 2^48", h_max);
    if (!noise_ok(c, f, h_max))
        return set_error(PIMM_E_NOISE,
                         "max |W| = %llu: worst-case noise of the reply breaks decryption for "
                         "these parameters and this plan",
                         h_max);
    pimm_weights *w = new pimm_weights();
    w->ctx = plan->ctx;
    w->info = plan->info;
    w->wmax = (int64_t)h_max;
    const uint64_t f64_bytes = (uint64_t)f.Wb * c.params.L * c.params.N * 8;
    rc = check_hip(hipMalloc((void **)&w->d_w_hat, f64_bytes), "hipMalloc weights");
    if (!rc && mfma_eligible(f))
        rc = check_hip(hipMalloc(&w->d_w_dig, digit_cache_bytes(c, f)), "hipMalloc weight digits");
    // The FC completion's copy of W as doubles (plans of one product only).
    if (!rc && f.groups == 1)
        rc = check_hip(hipMalloc((void **)&w->d_w_plain, (size_t)f.r * f.m * sizeof(double)),
                       "hipMalloc plain weights");
    if (!rc && w->d_w_plain) rc = weights_plain(W, w->d_w_plain, (size_t)f.r * f.m, s);
    if (!rc)
        rc = launch_fwd(c, LoadWeights{W, f.r, f.m, f.mb, f.rb, f.R, f.M, (int)c.params.L},
                        StoreWeightTiled{w->d_w_hat, c.dp.logN, (int)c.params.L, f.groups * f.M, f.R},
                        (int)(f.Wb * c.params.L), s);
    if (!rc && w->d_w_dig) rc = build_weight_digits(c, f, w->d_w_hat, w->d_w_dig, s);
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "weights synchronize");
    if (rc) {
        pimm_weights_destroy(w);
        return rc;
    }
    *out = w;
    return PIMM_OK;
}

int pimm_weights_update(pimm_weights *w, const int64_t *W, uint64_t wmax, void *stream)
{
    if (!w || !W) return set_error(PIMM_E_ARG, "pimm_weights_update: NULL argument");
    const Ctx &c = *w->ctx;
    const pimm_plan_info &f = w->info;
    if (wmax > kMaxWeight) return set_error(PIMM_E_ARG, "pimm_weights_update: wmax exceeds 2^48");
    if (!noise_ok(c, f, wmax))
        return set_error(PIMM_E_NOISE,
                         "pimm_weights_update: |W| <= %llu breaks decryption for these parameters "
                         "and this plan",
                         (unsigned long long)wmax);
    hipStream_t s = (hipStream_t)stream;
    int rc = check_hip(hipSetDevice(c.device), "hipSetDevice");
    if (!rc && w->d_w_plain) rc = weights_plain(W, w->d_w_plain, (size_t)f.r * f.m, s);
    if (!rc)
        rc = launch_fwd(c, LoadWeights{W, f.r, f.m, f.mb, f.rb, f.R, f.M, (int)c.params.L},
                        StoreWeightTiled{w->d_w_hat, c.dp.logN, (int)c.params.L, f.groups * f.M, f.R},
                        (int)(f.Wb * c.params.L), s);
    if (!rc && w->d_w_dig) rc = build_weight_digits(c, f, w->d_w_hat, w->d_w_dig, s);
    if (!rc) w->wmax = (int64_t)wmax;
    return rc;
}

int pimm_weights_destroy(pimm_weights *w)
{
    if (!w) return PIMM_OK;
    if (w->d_w_hat) (void)hipFree(w->d_w_hat);
    if (w->d_w_plain) (void)hipFree(w->d_w_plain);
    if (w->d_w_dig) (void)hipFree(w->d_w_dig);
    delete w;
    return PIMM_OK;
}

// Workspace: c^ [I][2][L][N] doubles, then acc^ [O][2][L][N] doubles.
int pimm_matmul(const pimm_plan *plan, const pimm_weights *w, const uint64_t *ct, uint64_t *acc,
                void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !w || !ct || !acc) return set_error(PIMM_E_ARG, "pimm_matmul: NULL argument");
    if (!weights_fit(w, plan))
        return set_error(PIMM_E_ARG, "pimm_matmul: weights were made for another shape or block split");
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    const size_t N = c.params.N, L = c.params.L;
    const size_t need = ((size_t)f.I + f.O) * 2 * L * N * 8;
    if (!ws || ws_bytes < need) return set_error(PIMM_E_WORKSPACE, "pimm_matmul: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int lg = c.dp.logN;
    double *ch = (double *)ws;
    double *ah = ch + (size_t)f.I * 2 * L * N;
    int rc = PIMM_OK;
    if (plan->mac_rows == 0) {
        rc = mfma_ready(plan, w, "pimm_matmul");
        // The product reads the query ciphertexts, already in evaluation form, in place.
        if (!rc) rc = launch_mac_mfma(c, f, w->d_w_dig, ct, ah, s);
        if (!rc)
            rc = launch_inv(c, LoadSlotsReduceRun{ah, 2 * f.O, (uint32_t)(N / kAccRun), (int)L},
                            StoreU64{acc, lg}, (int)(f.O * 2 * L), s);
        return rc;
    }
    rc = ct_to_tiled(c, f, ct, ch, ah, s);
    if (!rc)
        rc = launch_mac(c, f, plan->mac_rows, plan->mac_cols, plan->waves, w->d_w_hat, ch, ah, true, s);
    if (!rc) rc = launch_inv(c, LoadSlotsReduce{ah, lg}, StoreU64{acc, lg}, (int)(f.O * 2 * L), s);
    return rc;
}

// Workspace (re-randomisation on): pk^ [2][L][N] doubles, u^ [O][L][N] doubles,
// u [O][N] int64, e [O][2][N] int64.
int pimm_mask_share(const pimm_plan *plan, const uint64_t *pk, const uint8_t seed[32],
                    uint32_t op_id, uint64_t *acc, uint64_t *c1, uint64_t *c0s,
                    uint64_t *server_share, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !seed || !acc || !c1 || !c0s || !server_share)
        return set_error(PIMM_E_ARG, "pimm_mask_share: NULL argument");
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    const size_t N = c.params.N, L = c.params.L;
    hipStream_t s = (hipStream_t)stream;
    const int lg = c.dp.logN;
    const Key key = make_key(seed);
    int rc = PIMM_OK;
    if (c.params.rerandomize) {
        if (!pk) return set_error(PIMM_E_ARG, "pimm_mask_share: re-randomisation needs pk");
        const size_t need = 2 * L * N * 8 + (size_t)f.O * L * N * 8 + (size_t)f.O * 3 * N * 8;
        if (!ws || ws_bytes < need)
            return set_error(PIMM_E_WORKSPACE, "pimm_mask_share: workspace too small");
        double *pkh = (double *)ws;
        double *uh = pkh + 2 * L * N;
        int8_t *u = (int8_t *)(uh + (size_t)f.O * L * N);
        int8_t *e = u + (size_t)f.O * N * 8;
        rc = launch_samples(c, key, op_id, rerand_jobs(f.O, N, u, e), s);
        // pk^ and u^ in one launch: they are adjacent in the workspace.
        if (!rc)
            rc = launch_fwd2(c, LoadU64{pk, lg}, LoadI8Shared{u, lg, 2u}, (int)(2 * L), StoreSlots{pkh, lg},
                             (int)((2 + f.O) * L), s);
        if (!rc)
            rc = launch_inv(c, LoadRerand{uh, pkh, lg, (int)L}, StoreAddErr{acc, e, lg, (int)L},
                            (int)(f.O * 2 * L), s);
    }
    if (!rc) {
        const size_t total = (size_t)f.O * f.mb * f.nb;
        const int threads = 256;
        ProfScope prof("mask_extract", s);
        hipLaunchKernelGGL(k_mask_extract, dim3((unsigned)((total + threads - 1) / threads)),
                           dim3(threads), 0, s, key, op_id, acc, c0s, server_share, f, c.dp);
        rc = check_hip(hipGetLastError(), "mask_extract launch");
    }
    if (!rc)
        rc = check_hip(hipMemcpy2DAsync(c1, L * N * 8, acc + L * N, 2 * L * N * 8, L * N * 8, f.O,
                                        hipMemcpyDeviceToDevice, s),
                       "copy c1");
    return rc;
}

// Workspace: c^ [I][2][L][N], acc^ [O][2][L][N], pk^ [2][L][N], u^ [O][L][N] doubles,
// then u [O][N] and e [O][2][N] int64.
int pimm_matmul_share(const pimm_plan *plan, const pimm_weights *w, const uint64_t *pk,
                      const uint8_t seed[32], uint32_t op_id, const uint64_t *ct, uint64_t *c1,
                      uint64_t *c0s, uint64_t *server_share, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !w || !seed || !ct || !c1 || !c0s || !server_share)
        return set_error(PIMM_E_ARG, "pimm_matmul_share: NULL argument");
    if (!weights_fit(w, plan))
        return set_error(PIMM_E_ARG, "pimm_matmul_share: weights were made for another shape or block split");
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    const size_t N = c.params.N, L = c.params.L;
    const int rr = c.params.rerandomize ? 1 : 0;
    if (rr && !pk) return set_error(PIMM_E_ARG, "pimm_matmul_share: re-randomisation needs pk");
    const size_t need = fused_workspace_bytes(c, f);
    if (!ws || ws_bytes < need)
        return set_error(PIMM_E_WORKSPACE, "pimm_matmul_share: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int lg = c.dp.logN;
    double *ch = (double *)ws;
    double *ah = ch + (size_t)f.I * 2 * L * N;
    const bool mx = plan->mac_rows == 0;
    int rc = PIMM_OK;
    if (mx) {
        rc = mfma_ready(plan, w, "pimm_matmul_share");
        // The product reads the query ciphertexts, already in evaluation form, in place.
        if (!rc) rc = launch_mac_mfma(c, f, w->d_w_dig, ct, ah, s);
    } else {
        rc = ct_to_tiled(c, f, ct, ch, ah, s);
        if (!rc)
            rc = launch_mac(c, f, plan->mac_rows, plan->mac_cols, plan->waves, w->d_w_hat, ch, ah,
                            true, s);
    }
    if (!rc)
        rc = fused_tail(plan, pk, make_key(seed), op_id, (double *)ws, c1, c0s, server_share, mx, s);
    return rc;
}

int pimm_ct_expand(const pimm_plan *plan, const uint8_t a_seed[32], uint32_t op_id,
                   const uint64_t *c0, uint64_t *ct, void *stream)
{
    if (!plan || !a_seed || !c0 || !ct) return set_error(PIMM_E_ARG, "pimm_ct_expand: NULL argument");
    const Ctx &c = *plan->ctx;
    const pimm_plan_info &f = plan->info;
    const size_t N = c.params.N, L = c.params.L;
    hipStream_t s = (hipStream_t)stream;
    int rc = check_hip(hipSetDevice(c.device), "hipSetDevice");
    if (!rc)
        rc = check_hip(hipMemcpy2DAsync(ct, 2 * L * N * 8, c0, L * N * 8, L * N * 8, f.I,
                                        hipMemcpyDeviceToDevice, s),
                       "pimm_ct_expand: copy c0");
    if (!rc)
        rc = launch_sample(c, 0, make_key(a_seed), kTagEncA, op_id, 0, (int)f.I, 0, (int)L, ct + L * N,
                           2 * L * N, N, s);
    return rc;
}

}  // extern "C"
