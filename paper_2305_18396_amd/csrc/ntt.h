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
// Loaders produce a double of magnitude <= p for (polynomial, index); storers
// consume a balanced double.  Poly index p of a [..][L][N] buffer belongs to
// prime p % L; the workgroup works out the prime and the quotient p / L once
// (PolyIx) and hands them to its loader and storer.
#pragma once

#include <type_traits>

#include "common.h"

namespace pimm {


// Workgroup size of the batch kernels (and of every N = 4096 transform).
constexpr int kNttThreads = 256;

// Pass sizes (stages per register pass) for a transform of 2^LOGN points done
// by T threads.  Every pass gives each thread whole sets of 2^PS elements.  At
// N = 8192 with 512 threads the 13 stages are 1 + 4 + 4 + 4, so that every
// thread holds 16 elements and two workgroups (16 waves) fit in a CU's LDS;
// with 256 threads they are 5 + 4 + 4.
template <int LOGN, int T>
struct NttSched;
template <>
struct NttSched<12, 256> {
    static constexpr int P0 = 4, P1 = 4, P2 = 4, P3 = 0;
};
template <>
struct NttSched<13, 256> {
    static constexpr int P0 = 5, P1 = 4, P2 = 4, P3 = 0;
};
template <>
struct NttSched<13, 512> {
    static constexpr int P0 = 1, P1 = 4, P2 = 4, P3 = 4;
};

// Threads of a stand-alone transform kernel.
template <int LOGN>
constexpr int ntt_threads()
{
    return LOGN == 13 ? 512 : 256;
}

// LDS slot of element j, padded by one double every 32 to break bank aliasing
// of the strided pass patterns.
__host__ __device__ constexpr int lds_idx(int j) { return j + (j >> 5); }

// Output pruning of the inverse transform.  When only the coefficients j with
// j % G == G - 1 are read afterwards (G a power of two <= 16: the decoded
// positions of a reply, j = t * r_b + r_b - 1, with G dividing r_b), the first
// inverse pass -- the four stages that combine elements differing in the low four
// index bits -- computes only the butterfly outputs those coefficients depend on,
// and the later passes run only on the sets whose elements have those low bits.
// prune_mask<PS, G>(sp): bit c set when register c of a set is still needed after
// inverse stage sp (the stages run PS - 1 down to 0; stage sp pairs c with
// c + (2^PS >> (sp + 1))).
template <int PS, int G>
__host__ __device__ constexpr uint32_t prune_mask(int sp)
{
    uint32_t m = 0;
    for (int c = 0; c < (1 << PS); ++c)
        if (c % G == G - 1) m |= 1u << c;
    for (int st = 1; st <= sp; ++st) {
        const int h = (1 << PS) >> st;  // the pair distance of stage st - 1
        uint32_t n = m;
        for (int c = 0; c < (1 << PS); ++c)
            if ((m >> (c ^ h)) & 1u) n |= 1u << c;
        m = n;
    }
    return m;
}

template <int LOGN, int S0, int PS, int T>
struct Pass {
    static constexpr int N = 1 << LOGN;
    static constexpr int E = 1 << PS;
    static constexpr int STRIDE = N >> (S0 + PS);
    static constexpr int NSETS = N >> PS;
    static constexpr int PER_THREAD = NSETS / T;
    static_assert(PER_THREAD >= 1 && NSETS % T == 0, "pass shape");

    // Element index of member c of set S.
    __host__ __device__ static constexpr int elem(int S, int c)
    {
        return (S / STRIDE) * (N >> S0) + (S % STRIDE) + c * STRIDE;
    }

    // LDS slot of member c relative to member 0: the members of a set are STRIDE apart
    // and never cross a padding boundary differently from member 0's offset
    // (lds_split_ok), so a pass computes one address per set and the rest are
    // instruction offsets.
    __host__ __device__ static constexpr int lds_off(int c) { return lds_idx(c * STRIDE); }
    static constexpr bool lds_split_ok()
    {
        for (int S = 0; S < NSETS; ++S)
            for (int c = 0; c < E; ++c)
                if (lds_idx(elem(S, c)) != lds_idx(elem(S, 0)) + lds_off(c)) return false;
        return true;
    }

    // Twiddles set S uses, stage by stage: w[2^sp - 1 + j] is the factor of the
    // butterflies of stage S0 + sp whose lower index c has c >> (PS - sp) == j.
    static constexpr int NTW = E - 1;
    __device__ static __forceinline__ void load_tw(int S, const double *tw, double *w)
    {
        const int hi = S / STRIDE;
#pragma unroll
        for (int sp = 0; sp < PS; ++sp)
#pragma unroll
            for (int j = 0; j < (1 << sp); ++j) w[(1 << sp) - 1 + j] = tw[(1 << (S0 + sp)) + (hi << sp) + j];
    }

    // Set of element e (the inverse of elem).
    __host__ __device__ static constexpr int set_of(int e)
    {
        return (e / (N >> S0)) * STRIDE + (e % (N >> S0)) % STRIDE;
    }

    // Forward stages S0 .. S0+PS-1 on the registers of a set whose twiddles are w.
    __device__ static __forceinline__ void fwd_w(double *x, const double *w, double p, double pinv)
    {
#pragma unroll
        for (int sp = 0; sp < PS; ++sp) {
            const int half = E >> (sp + 1);
#pragma unroll
            for (int c = 0; c < E; ++c) {
                if (c & half) continue;
                const double u = x[c];
                const double v = mulmod(x[c + half], w[(1 << sp) - 1 + (c >> (PS - sp))], p, pinv);
                x[c] = u + v;
                x[c + half] = u - v;
            }
        }
    }

    // Forward stages S0 .. S0+PS-1 on the registers of set S.
    __device__ static __forceinline__ void fwd(double *x, int S, const double *tw, double p,
                                               double pinv)
    {
        double w[NTW];
        load_tw(S, tw, w);
        fwd_w(x, w, p, pinv);
    }

    // Inverse stages S0+PS-1 .. S0 of set S computing only the registers that
    // prune_mask<PS, G> keeps.
    template <int G>
    __device__ static __forceinline__ void inv_pruned(double *x, int S, const double *tw, double p,
                                                      double pinv)
    {
        const int hi = S / STRIDE;
#pragma unroll
        for (int sp = PS - 1; sp >= 0; --sp) {
            const int half = E >> (sp + 1);
            const uint32_t need = prune_mask<PS, G>(sp);
#pragma unroll
            for (int c = 0; c < E; ++c) {
                if (c & half) continue;
                const bool lo = (need >> c) & 1u, up = (need >> (c + half)) & 1u;
                if (!lo && !up) continue;
                const double u = x[c], v = x[c + half];
                if (lo) x[c] = (sp & 1) ? u + v : reduce(u + v, p, pinv);
                if (up) {
                    const double w = tw[(1 << (S0 + sp)) + (hi << sp) + (c >> (PS - sp))];
                    x[c + half] = mulmod(u - v, w, p, pinv);
                }
            }
        }
    }

    // Inverse stages S0+PS-1 .. S0 on the registers of set S.  The sums are
    // reduced after the even stages only: with inputs within 1.1 p (every
    // loader's bound) the registers stay within 2.7 p between reductions, so the
    // differences that enter mulmod stay within 5.3 p (its result within 1.5 p,
    // exact), and the pass ends with every register reduced.
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
                x[c] = (sp & 1) ? u + v : reduce(u + v, p, pinv);
                x[c + half] = mulmod(u - v, w, p, pinv);
            }
        }
    }
};

template <int LOGN, int T>
struct NttPasses {
    using S = NttSched<LOGN, T>;
    using A = Pass<LOGN, 0, S::P0, T>;
    using B = Pass<LOGN, S::P0, S::P1, T>;
    using C = Pass<LOGN, S::P0 + S::P1, S::P2, T>;
    // Fourth pass (only when P3 > 0; otherwise a placeholder that is never used).
    using D = Pass<LOGN, S::P0 + S::P1 + S::P2, (S::P3 > 0 ? S::P3 : 1), T>;
    static_assert(S::P0 + S::P1 + S::P2 + S::P3 == LOGN, "schedule covers every stage");
    static constexpr bool d_split_ok()
    {
        if constexpr (S::P3 > 0)
            return D::lds_split_ok();
        else
            return true;
    }
    static_assert(A::lds_split_ok() && B::lds_split_ok() && C::lds_split_ok() && d_split_ok(),
                  "per-set LDS addressing");
    static constexpr int N = 1 << LOGN;
    // The pass that touches global memory in slot order (the forward's last, the inverse's
    // first) and its size.
    static constexpr int PL = S::P3 > 0 ? S::P3 : S::P2;
    using PFirst = std::conditional_t<(S::P3 > 0), D, C>;
    // LDS: the N elements (padded, lds_idx), then the twiddles of every other pass
    // (factor indices below N >> PL), copied from global memory once per transform so that
    // those passes read them from LDS.
    static constexpr int DATA = N + (N >> 5);
    static constexpr int TWL = N >> PL;
    static constexpr int LDS = DATA + TWL;
};

// Copy of the twiddle factors with index below TWL into the LDS table (visible after the
// next barrier).
template <int LOGN, int T>
__device__ __forceinline__ void load_tw_table(const double *tw, double *lds)
{
    using NP = NttPasses<LOGN, T>;
#pragma unroll
    for (int i = (int)threadIdx.x; i < NP::TWL; i += T) lds[NP::DATA + i] = tw[i];
}

// True when every element written by pass P (thread of set S: S % T) is read in pass Q by
// a thread of the same wave: the exchange between the two passes then needs no workgroup
// barrier, only ordering within the wave.
template <class P, class Q, int T>
__host__ __device__ constexpr bool exchange_in_wave()
{
    for (int e = 0; e < P::N; ++e)
        if ((P::set_of(e) % T) / 64 != (Q::set_of(e) % T) / 64) return false;
    return true;
}

// Orders the LDS writes of the calling wave before its later LDS reads (the lanes of a
// wave see each other's writes in program order; this keeps the compiler from moving
// them).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Loader of the passes that read only LDS (never called).
struct NoLoad {
    __device__ double operator()(const PolyIx &, int, double, double) const { return 0.0; }
};

// Storer of a transform whose result stays in the workgroup's LDS (natural order,
// lds_idx layout).
struct StoreLds {
    double *lds;
    __device__ void operator()(const PolyIx &, int j, double v, double, double) const
    {
        lds[lds_idx(j)] = v;
    }
};

// Storer of a forward transform whose last pass leaves its result where it read it in
// LDS: each thread's sets stay with that thread, so an inverse transform's first pass
// (the mirror of that pass: the same sets on the same threads) can read them there
// without a barrier.  Slot c * NSETS + S is then at LDS element P::elem(S, c).
struct StoreKeepLds {};

// A storer whose value needs global inputs of its own (the plaintext and error words of
// an encryption) declares `Pre`, reads them in `pre(pi, j)` and takes them back as the
// last argument of its call operator.  The last pass reads every element's inputs before
// its butterflies, so the reads overlap each other and the arithmetic; without this the
// stores in between would order every read after the previous store.
template <class St, class = void>
struct has_pre : std::false_type {};
template <class St>
struct has_pre<St, std::void_t<typename St::Pre>> : std::true_type {};

// Pre-read inputs of a storer without any (keeps the call sites uniform).
struct NoPre {};

template <class St, bool = has_pre<St>::value>
struct pre_of {
    using type = NoPre;
};
template <class St>
struct pre_of<St, true> {
    using type = typename St::Pre;
};
template <class Store>
using pre_t = typename pre_of<Store>::type;

template <class Store>
__device__ __forceinline__ pre_t<Store> store_pre(const Store &st, const PolyIx &pi, int j)
{
    if constexpr (has_pre<Store>::value)
        return st.pre(pi, j);
    else
        return NoPre{};
}

template <class Store>
__device__ __forceinline__ void store_val(const Store &st, const PolyIx &pi, int j, double v, double p,
                                          double pinv, const pre_t<Store> &pr)
{
    if constexpr (has_pre<Store>::value)
        st(pi, j, v, p, pinv, pr);
    else
        st(pi, j, v, p, pinv);
}

// Forward stages of pass P on every set the thread owns: read from LDS (or the
// loader for the first pass), write to LDS (or the storer, in slot order, for
// the last pass).  With w given (one set per thread), the set's twiddles are
// those already loaded there; otherwise they come from tw.
template <class P, int T, bool FIRST, bool LAST, class Load, class Store>
__device__ __forceinline__ void fwd_pass(const Load &ld, const Store &st, const PolyIx &pi,
                                         const double *tw, double p, double pinv, double *lds,
                                         const double *w = nullptr)
{
    if constexpr (FIRST && !LAST && P::PER_THREAD > 1) {
        // The first pass with several sets per thread reads every element of all of them
        // before any butterfly, so the reads are in flight together whatever the loader's
        // arithmetic (the compiler does not always move a later set's reads ahead by itself).
        double xs[P::PER_THREAD][P::E];
#pragma unroll
        for (int k = 0; k < P::PER_THREAD; ++k)
#pragma unroll
            for (int c = 0; c < P::E; ++c) xs[k][c] = ld(pi, P::elem((int)threadIdx.x + k * T, c), p, pinv);
#pragma unroll
        for (int k = 0; k < P::PER_THREAD; ++k) {
            const int S = (int)threadIdx.x + k * T;
            const int b0 = lds_idx(P::elem(S, 0));
            P::fwd(xs[k], S, tw, p, pinv);
#pragma unroll
            for (int c = 0; c < P::E; ++c) lds[b0 + P::lds_off(c)] = reduce(xs[k][c], p, pinv);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < P::PER_THREAD; ++k) {
        const int S = (int)threadIdx.x + k * T;
        const int b0 = lds_idx(P::elem(S, 0));
        pre_t<Store> pr[P::E];
        if constexpr (LAST && has_pre<Store>::value) {
#pragma unroll
            for (int c = 0; c < P::E; ++c) pr[c] = store_pre(st, pi, c * P::NSETS + S);
        }
        double x[P::E];
#pragma unroll
        for (int c = 0; c < P::E; ++c)
            x[c] = FIRST ? ld(pi, P::elem(S, c), p, pinv) : lds[b0 + P::lds_off(c)];
        if (w)
            P::fwd_w(x, w, p, pinv);
        else
            P::fwd(x, S, tw, p, pinv);
#pragma unroll
        for (int c = 0; c < P::E; ++c) {
            if constexpr (LAST && !std::is_same<Store, StoreKeepLds>::value)
                store_val(st, pi, c * P::NSETS + S, reduce(x[c], p, pinv), p, pinv, pr[c]);
            else
                lds[b0 + P::lds_off(c)] = reduce(x[c], p, pinv);
        }
    }
}

// Inverse stages of pass P (the mirror of fwd_pass: the first inverse pass reads
// the loader in slot order, the last one multiplies by N^-1 and calls the storer
// in natural order).
//
// With G > 1 (output pruning, see prune_mask) the first pass loads every element
// but keeps only the registers the needed coefficients depend on, and the other
// passes run only on the sets S with S % G == G - 1 (their elements are the ones
// whose low four index bits are G - 1 mod G), packed onto the first threads.
template <class P, int T, bool FIRST, bool LAST, int G = 1, class Load, class Store>
__device__ __forceinline__ void inv_pass(const Load &ld, const Store &st, const PolyIx &pi,
                                         const double *tw, double p, double pinv, double ninv,
                                         double *lds)
{
    if constexpr (G > 1 && FIRST) {
        static_assert(P::STRIDE == 1 && P::E == 16 && !LAST, "pruned first pass: 16 adjacent elements");
#pragma unroll
        for (int k = 0; k < P::PER_THREAD; ++k) {
            const int S = (int)threadIdx.x + k * T;
            const int b0 = lds_idx(P::elem(S, 0));
            double x[P::E];
#pragma unroll
            for (int c = 0; c < P::E; ++c) x[c] = ld(pi, c * P::NSETS + S, p, pinv);
            P::template inv_pruned<G>(x, S, tw, p, pinv);
#pragma unroll
            for (int c = 0; c < P::E; ++c)
                if (c % G == G - 1) lds[b0 + P::lds_off(c)] = reduce(x[c], p, pinv);
        }
        return;
    }
    if constexpr (G > 1) {
        constexpr int NEED = P::NSETS / G;
#pragma unroll
        for (int k = 0; k < (NEED + T - 1) / T; ++k) {
            const int u = (int)threadIdx.x + k * T;
            if (u >= NEED) break;
            const int S = u * G + (G - 1);
            const int b0 = lds_idx(P::elem(S, 0));
            pre_t<Store> pr[P::E];
            if constexpr (LAST && has_pre<Store>::value) {
#pragma unroll
                for (int c = 0; c < P::E; ++c) pr[c] = store_pre(st, pi, P::elem(S, c));
            }
            double x[P::E];
#pragma unroll
            for (int c = 0; c < P::E; ++c) x[c] = lds[b0 + P::lds_off(c)];
            P::inv(x, S, tw, p, pinv);
#pragma unroll
            for (int c = 0; c < P::E; ++c) {
                if constexpr (LAST && std::is_same<Store, StoreLds>::value)
                    lds[b0 + P::lds_off(c)] = mulmod(x[c], ninv, p, pinv);
                else if (LAST)
                    store_val(st, pi, P::elem(S, c), mulmod(x[c], ninv, p, pinv), p, pinv, pr[c]);
                else
                    lds[b0 + P::lds_off(c)] = reduce(x[c], p, pinv);
            }
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < P::PER_THREAD; ++k) {
        const int S = (int)threadIdx.x + k * T;
        const int b0 = lds_idx(P::elem(S, 0));
        pre_t<Store> pr[P::E];
        if constexpr (LAST && has_pre<Store>::value) {
#pragma unroll
            for (int c = 0; c < P::E; ++c) pr[c] = store_pre(st, pi, P::elem(S, c));
        }
        double x[P::E];
#pragma unroll
        for (int c = 0; c < P::E; ++c)
            x[c] = FIRST ? ld(pi, c * P::NSETS + S, p, pinv) : lds[b0 + P::lds_off(c)];
        P::inv(x, S, tw, p, pinv);
#pragma unroll
        for (int c = 0; c < P::E; ++c) {
            if constexpr (LAST && std::is_same<Store, StoreLds>::value)
                lds[b0 + P::lds_off(c)] = mulmod(x[c], ninv, p, pinv);
            else if (LAST)
                store_val(st, pi, P::elem(S, c), mulmod(x[c], ninv, p, pinv), p, pinv, pr[c]);
            else
                lds[b0 + P::lds_off(c)] = reduce(x[c], p, pinv);
        }
    }
}

// Forward negacyclic NTT of polynomial `poly` by the calling workgroup of T
// threads, with `lds` holding NttPasses<LOGN, T>::LDS doubles.  The first pass
// reads its few twiddles from global memory, the middle ones from the LDS table;
// the last pass's twiddles (one set per thread) are requested before the pass
// ahead of it, so their latency hides behind that pass.
template <int LOGN, int T, class Load, class Store>
__device__ __forceinline__ void ntt_fwd_block(const Load &ld, const Store &st, const DevParams &dp,
                                              int poly, double *lds)
{
    using NP = NttPasses<LOGN, T>;
    constexpr bool FOUR = NP::S::P3 > 0;
    const PolyIx pi = poly_ix(poly, dp.L);
    const int l = pi.l;
    const double p = dp.p[l], pinv = dp.pinv[l];
    const double *tw = dp.tw_fwd + ((size_t)l << LOGN);
    const double *twl = lds + NP::DATA;
    load_tw_table<LOGN, T>(tw, lds);
    fwd_pass<typename NP::A, T, true, false>(ld, st, pi, tw, p, pinv, lds);
    __syncthreads();
    if constexpr (FOUR) {
        using PC = typename NP::C;
        using PD = typename NP::D;
        fwd_pass<typename NP::B, T, false, false>(ld, st, pi, twl, p, pinv, lds);
        __syncthreads();
        if constexpr (PD::PER_THREAD == 1) {
            double w[PD::NTW];
            PD::load_tw((int)threadIdx.x, tw, w);
            fwd_pass<PC, T, false, false>(ld, st, pi, twl, p, pinv, lds);
            if constexpr (exchange_in_wave<PC, PD, T>())
                wave_sync();
            else
                __syncthreads();
            fwd_pass<PD, T, false, true>(ld, st, pi, tw, p, pinv, lds, w);
        } else {
            fwd_pass<PC, T, false, false>(ld, st, pi, twl, p, pinv, lds);
            __syncthreads();
            fwd_pass<PD, T, false, true>(ld, st, pi, tw, p, pinv, lds);
        }
    } else {
        using PB = typename NP::B;
        using PC = typename NP::C;
        if constexpr (PC::PER_THREAD == 1) {
            double w[PC::NTW];
            PC::load_tw((int)threadIdx.x, tw, w);
            fwd_pass<PB, T, false, false>(ld, st, pi, twl, p, pinv, lds);
            if constexpr (exchange_in_wave<PB, PC, T>())
                wave_sync();
            else
                __syncthreads();
            fwd_pass<PC, T, false, true>(ld, st, pi, tw, p, pinv, lds, w);
        } else {
            fwd_pass<PB, T, false, false>(ld, st, pi, twl, p, pinv, lds);
            __syncthreads();
            fwd_pass<PC, T, false, true>(ld, st, pi, tw, p, pinv, lds);
        }
    }
}

// Inverse negacyclic NTT (including the factor N^-1) of polynomial `poly`; with
// G > 1 only the coefficients j with j % G == G - 1 are produced.  The first pass
// reads its twiddles from global memory (with its inputs), the others from the
// LDS table.
// The passes of an inverse transform after its first one, on the LDS data that pass
// left (visible after a barrier) with the LDS twiddle table loaded.
template <int LOGN, int T, int G = 1, class Store>
__device__ __forceinline__ void ntt_inv_rest(const Store &st, const DevParams &dp, const PolyIx &pi,
                                             double *lds)
{
    using NP = NttPasses<LOGN, T>;
    const int l = pi.l;
    const double p = dp.p[l], pinv = dp.pinv[l], ninv = dp.n_inv[l];
    const double *twl = lds + NP::DATA;
    const NoLoad nl;
    if constexpr (NP::S::P3 > 0) {
        inv_pass<typename NP::C, T, false, false, G>(nl, st, pi, twl, p, pinv, ninv, lds);
        __syncthreads();
    }
    inv_pass<typename NP::B, T, false, false, G>(nl, st, pi, twl, p, pinv, ninv, lds);
    __syncthreads();
    inv_pass<typename NP::A, T, false, true, G>(nl, st, pi, twl, p, pinv, ninv, lds);
}

template <int LOGN, int T, int G = 1, class Load, class Store>
__device__ __forceinline__ void ntt_inv_block(const Load &ld, const Store &st, const DevParams &dp,
                                              int poly, double *lds)
{
    using NP = NttPasses<LOGN, T>;
    const PolyIx pi = poly_ix(poly, dp.L);
    const int l = pi.l;
    const double p = dp.p[l], pinv = dp.pinv[l];
    const double *tw = dp.tw_inv + ((size_t)l << LOGN);
    load_tw_table<LOGN, T>(tw, lds);
    inv_pass<typename NP::PFirst, T, true, false, G>(ld, st, pi, tw, p, pinv, dp.n_inv[l], lds);
    __syncthreads();
    ntt_inv_rest<LOGN, T, G>(st, dp, pi, lds);
}

// Polynomial of a workgroup: workgroups are dispatched round-robin over the XCDs, so the
// transform kernels take xcd_local(blockIdx.x): neighbouring polynomials (the primes of one
// ciphertext, the two components of one output) run on one XCD and the operands they share
// (error and plaintext words, the re-randomisation term, the key) come from its L2.
__device__ __forceinline__ int ntt_poly() { return (int)xcd_local(blockIdx.x, gridDim.x); }

template <int LOGN, class Load, class Store>
__global__ __launch_bounds__(ntt_threads<LOGN>()) void k_ntt_fwd(Load ld, Store st, DevParams dp)
{
    constexpr int T = ntt_threads<LOGN>();
    __shared__ double lds[NttPasses<LOGN, T>::LDS];
    ntt_fwd_block<LOGN, T>(ld, st, dp, ntt_poly(), lds);
}

// Forward transform of two polynomial lists in one launch: polynomials below n1 read
// through ld1, the rest through ld2.  The choice is per workgroup, so each loader's
// reads stay free of branches (a branch between reads would make each wait for the last).
template <int LOGN, class Load1, class Load2, class Store>
__global__ __launch_bounds__(ntt_threads<LOGN>()) void k_ntt_fwd2(Load1 ld1, Load2 ld2, int n1, Store st,
                                                                   DevParams dp)
{
    constexpr int T = ntt_threads<LOGN>();
    __shared__ double lds[NttPasses<LOGN, T>::LDS];
    const int poly = ntt_poly();
    if (poly < n1)
        ntt_fwd_block<LOGN, T>(ld1, st, dp, poly, lds);
    else
        ntt_fwd_block<LOGN, T>(ld2, st, dp, poly, lds);
}

// Polynomial `poly`, already in evaluation form (a query ciphertext's component), moved into
// another layout through (ld, st), and, as in k_ntt_fwd_zero, the workgroup's share of another
// buffer zeroed.  Every read of a thread is issued before its first write.
template <int LOGN, class Load, class Store>
__global__ __launch_bounds__(ntt_threads<LOGN>()) void k_move(Load ld, Store st, double *zero, size_t zero_n,
                                                               DevParams dp)
{
    constexpr int T = ntt_threads<LOGN>();
    const PolyIx pi = poly_ix(ntt_poly(), dp.L);
    const double p = dp.p[pi.l], pinv = dp.pinv[pi.l];
    double v[(1 << LOGN) / T];
#pragma unroll
    for (int k = 0; k < (1 << LOGN) / T; ++k) v[k] = ld(pi, (int)threadIdx.x + k * T, p, pinv);
#pragma unroll
    for (int k = 0; k < (1 << LOGN) / T; ++k) st(pi, (int)threadIdx.x + k * T, v[k], p, pinv);
    if (zero_n) {
        const size_t per = (zero_n + gridDim.x - 1) / gridDim.x;
        const size_t b = (size_t)blockIdx.x * per;
        const size_t e = b + per < zero_n ? b + per : zero_n;
        for (size_t i = b + threadIdx.x; i < e; i += T) zero[i] = 0.0;
    }
}

// Forward transform that also clears its share of another buffer (the
// product's accumulators), saving a launch: workgroup b zeroes
// zero[b * per, (b + 1) * per), per = ceil(zero_n / gridDim.x).
template <int LOGN, class Load, class Store>
__global__ __launch_bounds__(ntt_threads<LOGN>()) void k_ntt_fwd_zero(Load ld, Store st, double *zero,
                                                                       size_t zero_n, DevParams dp)
{
    constexpr int T = ntt_threads<LOGN>();
    __shared__ double lds[NttPasses<LOGN, T>::LDS];
    ntt_fwd_block<LOGN, T>(ld, st, dp, ntt_poly(), lds);
    const size_t per = (zero_n + gridDim.x - 1) / gridDim.x;
    const size_t b = (size_t)blockIdx.x * per;
    const size_t e = b + per < zero_n ? b + per : zero_n;
    for (size_t i = b + threadIdx.x; i < e; i += T) zero[i] = 0.0;
}

template <int LOGN, class Load, class Store>
__global__ __launch_bounds__(ntt_threads<LOGN>()) void k_ntt_inv(Load ld, Store st, DevParams dp)
{
    constexpr int T = ntt_threads<LOGN>();
    __shared__ double lds[NttPasses<LOGN, T>::LDS];
    ntt_inv_block<LOGN, T>(ld, st, dp, ntt_poly(), lds);
}

// Inverse transform whose result stays in the workgroup's LDS (natural order,
// lds_idx layout), followed by an epilogue that reads it with the whole
// workgroup: epi.run<LOGN, T>(poly, lds, dp).  The last pass's storer writes exactly the
// elements its thread has just read, so no barrier is needed before it.  With
// G > 1, the polynomials for which epi.sparse(pi) holds are transformed with
// output pruning (only j % G == G - 1 is produced; the epilogue reads no other
// coefficient of them).
template <int LOGN, int G, class Load, class Epi>
__global__ __launch_bounds__(ntt_threads<LOGN>()) void k_ntt_inv_lds(Load ld, Epi epi, DevParams dp)
{
    constexpr int T = ntt_threads<LOGN>();
    __shared__ double lds[NttPasses<LOGN, T>::LDS];
    const int poly = ntt_poly();
    const PolyIx pi = poly_ix(poly, dp.L);
    // An epilogue with inputs of its own (Pre) reads them before the transform, so they
    // arrive behind its work instead of after it.  Not without pruning (G = 1): the
    // registers they take then make the compiler split the first pass's reads.
    constexpr bool PRE = has_pre<Epi>::value && G > 1;
    pre_t<Epi> epre;
    if constexpr (PRE) epre = epi.template pre<LOGN, T>(pi);
    if (G > 1 && epi.sparse(pi))
        ntt_inv_block<LOGN, T, G>(ld, StoreLds{lds}, dp, poly, lds);
    else
        ntt_inv_block<LOGN, T, 1>(ld, StoreLds{lds}, dp, poly, lds);
    __syncthreads();
    if constexpr (PRE)
        epi.template run<LOGN, T>(pi, lds, dp, epre);
    else
        epi.template run<LOGN, T>(pi, lds, dp);
}

// The output pruning an epilogue that reads the decoded positions t * rb + rb - 1
// allows: the largest of 16, 4 and 1 that divides rb.
inline int prune_factor(uint32_t rb) { return rb % 16 == 0 ? 16 : rb % 4 == 0 ? 4 : 1; }

// ---- loaders ----------------------------------------------------------------

// Canonical uint64 residues, [npoly][N].
struct LoadU64 {
    const uint64_t *in;
    int logn;
    __device__ double operator()(const PolyIx &pi, int j, double, double) const
    {
        return f64_of(in[((size_t)pi.poly << logn) + j]);
    }
};

// Canonical residues in slot order ([npoly][N], such as the query ciphertexts [I][2][L][N])
// as balanced doubles.
struct LoadSlotsBalanced {
    const uint64_t *in;
    int logn;
    __device__ double operator()(const PolyIx &pi, int z, double p, double) const
    {
        const double v = f64_of(in[((size_t)pi.poly << logn) + z]);
        return v > 0.5 * p ? v - p : v;
    }
};

// Small signed integers shared by the L primes: source poly = poly / L.
struct LoadI64Shared {
    const int64_t *in;
    int logn;
    __device__ double operator()(const PolyIx &pi, int j, double, double) const
    {
        return (double)in[((size_t)pi.x << logn) + j];
    }
};

// Pointwise product of two NTT-form operands: a[poly] times b[l] (an operand per
// prime, such as the key) or b[poly] (by_prime = 0).
struct LoadSlotsMul {
    const double *a, *b;
    int logn, by_prime;
    __device__ double operator()(const PolyIx &pi, int z, double p, double pinv) const
    {
        return mulmod(a[((size_t)pi.poly << logn) + z],
                      b[((size_t)(by_prime ? pi.l : pi.poly) << logn) + z], p, pinv);
    }
};

// NTT-form operand as is.
struct LoadSlots {
    const double *a;
    int logn;
    __device__ double operator()(const PolyIx &pi, int z, double, double) const
    {
        return a[((size_t)pi.poly << logn) + z];
    }
};

// ---- storers ----------------------------------------------------------------

struct StoreSlots {
    double *out;
    int logn;
    __device__ void operator()(const PolyIx &pi, int z, double v, double, double) const
    {
        out[((size_t)pi.poly << logn) + z] = v;
    }
};

struct StoreU64 {
    uint64_t *out;
    int logn;
    __device__ void operator()(const PolyIx &pi, int j, double v, double p, double pinv) const
    {
        out[((size_t)pi.poly << logn) + j] = to_canonical(v, p, pinv);
    }
};

// Instantiate and launch a transform for the context's ring degree.
template <class Load, class Store>
int launch_fwd(const Ctx &c, Load ld, Store st, int npoly, hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_fwd", s);
    if (c.dp.logN == 12)
        hipLaunchKernelGGL((k_ntt_fwd<12, Load, Store>), dim3(npoly), dim3(ntt_threads<12>()), 0, s, ld,
                           st, c.dp);
    else
        hipLaunchKernelGGL((k_ntt_fwd<13, Load, Store>), dim3(npoly), dim3(ntt_threads<13>()), 0, s, ld,
                           st, c.dp);
    return check_hip(hipGetLastError(), "ntt_fwd launch");
}

template <class Load1, class Load2, class Store>
int launch_fwd2(const Ctx &c, Load1 ld1, Load2 ld2, int n1, Store st, int npoly, hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_fwd", s);
    if (c.dp.logN == 12)
        hipLaunchKernelGGL((k_ntt_fwd2<12, Load1, Load2, Store>), dim3(npoly), dim3(ntt_threads<12>()), 0,
                           s, ld1, ld2, n1, st, c.dp);
    else
        hipLaunchKernelGGL((k_ntt_fwd2<13, Load1, Load2, Store>), dim3(npoly), dim3(ntt_threads<13>()), 0,
                           s, ld1, ld2, n1, st, c.dp);
    return check_hip(hipGetLastError(), "ntt_fwd launch");
}

template <class Load, class Store>
int launch_move(const Ctx &c, Load ld, Store st, int npoly, double *zero, size_t zero_n, hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_fwd", s);
    if (c.dp.logN == 12)
        hipLaunchKernelGGL((k_move<12, Load, Store>), dim3(npoly), dim3(ntt_threads<12>()), 0, s, ld, st, zero,
                           zero_n, c.dp);
    else
        hipLaunchKernelGGL((k_move<13, Load, Store>), dim3(npoly), dim3(ntt_threads<13>()), 0, s, ld, st, zero,
                           zero_n, c.dp);
    return check_hip(hipGetLastError(), "move launch");
}

template <class Load, class Store>
int launch_fwd_zero(const Ctx &c, Load ld, Store st, int npoly, double *zero, size_t zero_n,
                    hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_fwd", s);
    if (c.dp.logN == 12)
        hipLaunchKernelGGL((k_ntt_fwd_zero<12, Load, Store>), dim3(npoly), dim3(ntt_threads<12>()), 0, s,
                           ld, st, zero, zero_n, c.dp);
    else
        hipLaunchKernelGGL((k_ntt_fwd_zero<13, Load, Store>), dim3(npoly), dim3(ntt_threads<13>()), 0, s,
                           ld, st, zero, zero_n, c.dp);
    return check_hip(hipGetLastError(), "ntt_fwd launch");
}

template <class Load, class Store>
int launch_inv(const Ctx &c, Load ld, Store st, int npoly, hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_inv", s);
    if (c.dp.logN == 12)
        hipLaunchKernelGGL((k_ntt_inv<12, Load, Store>), dim3(npoly), dim3(ntt_threads<12>()), 0, s, ld,
                           st, c.dp);
    else
        hipLaunchKernelGGL((k_ntt_inv<13, Load, Store>), dim3(npoly), dim3(ntt_threads<13>()), 0, s, ld,
                           st, c.dp);
    return check_hip(hipGetLastError(), "ntt_inv launch");
}

template <int LOGN, class Load, class Epi>
void launch_inv_lds_g(int g, Load ld, Epi epi, int npoly, const DevParams &dp, hipStream_t s)
{
    if (g == 16)
        hipLaunchKernelGGL((k_ntt_inv_lds<LOGN, 16, Load, Epi>), dim3(npoly), dim3(ntt_threads<LOGN>()),
                           0, s, ld, epi, dp);
    else if (g == 4)
        hipLaunchKernelGGL((k_ntt_inv_lds<LOGN, 4, Load, Epi>), dim3(npoly), dim3(ntt_threads<LOGN>()),
                           0, s, ld, epi, dp);
    else
        hipLaunchKernelGGL((k_ntt_inv_lds<LOGN, 1, Load, Epi>), dim3(npoly), dim3(ntt_threads<LOGN>()),
                           0, s, ld, epi, dp);
}

// g: output pruning factor (prune_factor) for the polynomials epi.sparse marks.
template <class Load, class Epi>
int launch_inv_lds(const Ctx &c, Load ld, Epi epi, int npoly, int g, hipStream_t s)
{
    if (npoly <= 0) return PIMM_OK;
    ProfScope prof("ntt_inv", s);
    if (c.dp.logN == 12)
        launch_inv_lds_g<12>(g, ld, epi, npoly, c.dp, s);
    else
        launch_inv_lds_g<13>(g, ld, epi, npoly, c.dp, s);
    return check_hip(hipGetLastError(), "ntt_inv launch");
}

}  // namespace pimm
