// mac.h -- the slot-wise modular products of Algorithm 1 step 3.
//
// For NTT slot z and prime l the products of every inner block are summed:
//     acc^[(ib*K + kb)][comp][l][z] = sum_jb W^[ib, jb][l][z] * c^[jb, kb][comp][l][z]
// for both ciphertext components.
//
// Slots are grouped in chunks of 256 (one per thread of a workgroup) and the
// NTT-form operands are stored chunk-contiguous, so that a thread's stream over
// the inner blocks is sequential in memory:
//     W^   [L][chunks][M][R][256]        (weight cache)
//     c^   [L][chunks][K][R][2][256]     (the inputs, in evaluation form)
//     acc^ [O][2][L][N], O = M*K         (accumulators, read by the inverse NTT)
// A tile is (prime l, chunk zc, column block kb, rows ib0 .. ib0+G-1); a
// thread owns one slot of the tile and G output rows, streams G weight words
// and reuses the two input words per inner block.  Partial sums of balanced
// products (each below 0.6 p in magnitude) stay below 2^53 with a reduction
// every 8 inner blocks.
#pragma once

#include "common.h"

namespace pimm {

struct MacShape {
    int M, R, K, chunks;
};

__device__ __forceinline__ size_t w_tile_base(const MacShape &s, int l, int zc)
{
    return ((size_t)l * s.chunks + zc) * (size_t)s.M * s.R * 256;
}
__device__ __forceinline__ size_t c_tile_base(const MacShape &s, int l, int zc, int kb)
{
    return (((size_t)l * s.chunks + zc) * s.K + kb) * (size_t)s.R * 512;
}

// Column blocks of the product as seen by one tile: column `col` has its input
// words (the ciphertext in evaluation form, both components) and its accumulators.  For a
// single product the columns are its K column blocks; a batch may also line up
// the columns of several products that share one weight cache.
struct ColsOne {
    const double *Ct;  // c^ [L][chunks][K][R][2][256]
    double *Ah;        // acc^ [O][2][L][N], O = M*K
    MacShape s;
    int L, N;
    __device__ __forceinline__ int ncols() const { return s.K; }
    // c^ of column col at inner block 0, component 0, slot zz of chunk zc.
    __device__ __forceinline__ const double *c(int col, int l, int zc, int zz) const
    {
        return Ct + c_tile_base(s, l, zc, col) + zz;
    }
    // acc^ of column col, row 0, component 0, prime l, slot z; rows are arow() apart.
    __device__ __forceinline__ double *a(int col, int l, int z) const
    {
        return Ah + ((size_t)col * 2 * L + l) * N + z;
    }
    __device__ __forceinline__ size_t arow(int) const { return (size_t)s.K * 2 * L * N; }
    // One past the last weight row this tile may use.
    __device__ __forceinline__ int row_end(const MacShape &sh) const { return sh.M; }
};

// Columns of product g of a grouped plan (G products of one shape): the input layout
// holds the columns of all G products (g*K1 + kb), and the accumulators are
// [G*M1*K1][2][L][N] with weight rows g*M1 + ib.  The shape passed with it has M = G*M1
// rows and K = G*K1 columns (the strides of the weight and input layouts).
struct ColsGrouped {
    const double *Ct;  // c^ [L][chunks][G*K1][R][2][256]
    double *Ah;        // acc^ [G*M1*K1][2][L][N]
    MacShape s;
    int L, N, K1, g, M1;
    __device__ __forceinline__ int ncols() const { return K1; }
    __device__ __forceinline__ const double *c(int col, int l, int zc, int zz) const
    {
        return Ct + c_tile_base(s, l, zc, g * K1 + col) + zz;
    }
    __device__ __forceinline__ double *a(int col, int l, int z) const
    {
        return Ah + ((size_t)col * 2 * L + l) * N + z;
    }
    __device__ __forceinline__ size_t arow(int) const { return (size_t)K1 * 2 * L * N; }
    __device__ __forceinline__ int row_end(const MacShape &) const { return (g + 1) * M1; }
};

// Inner blocks [jb0, jb1) of one tile of G rows (ib0 ..) and KB columns (kb0 ..
// of `cs`): every weight word loaded is used for KB columns and every input
// word for G rows.  mode 0: store the reduced sums; mode 1: add them
// atomically (exact: every addend and every partial total is an integer below
// 2^53, so the order of the additions does not matter).
template <int G, int KB, class Cols>
__device__ __forceinline__ void mac_range(const double *__restrict__ Wt, const Cols &cs,
                                          const MacShape &s, const DevParams &dp, int l, int zc,
                                          int zz, int kb0, int ib0, int jb0, int jb1, int mode)
{
    const int L = dp.L, N = dp.N;
    const double p = dp.p[l], pinv = dp.pinv[l];
    const int re = cs.row_end(s);
    const int rows = re - ib0 < G ? re - ib0 : G;
    const int cols = cs.ncols() - kb0 < KB ? cs.ncols() - kb0 : KB;
    const double *wp = Wt + w_tile_base(s, l, zc) + ((size_t)ib0 * s.R + jb0) * 256 + zz;
    const size_t wrow = (size_t)s.R * 256;
    const double *cpk[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k)
        cpk[k] = k < cols ? cs.c(kb0 + k, l, zc, zz) + (size_t)jb0 * 512 : nullptr;

    double a0[G][KB], a1[G][KB];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < KB; ++k) a0[g][k] = a1[g][k] = 0.0;

    int jb = jb0;
    // Two inner blocks per iteration: all loads first, then the products.
    for (; jb + 1 < jb1; jb += 2) {
        double c00[KB], c01[KB], c10[KB], c11[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            if (k < cols) {
                const double *ck = cpk[k];
                c00[k] = ck[0];
                c01[k] = ck[256];
                c10[k] = ck[512];
                c11[k] = ck[768];
                cpk[k] = ck + 1024;
            } else {
                c00[k] = c01[k] = c10[k] = c11[k] = 0.0;
            }
        }
        double w0[G], w1[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g < rows) {
                // Weight words are used once per launch: stream them past the caches.
                w0[g] = __builtin_nontemporal_load(wp + g * wrow);
                w1[g] = __builtin_nontemporal_load(wp + g * wrow + 256);
            } else {
                w0[g] = w1[g] = 0.0;
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                a0[g][k] += mulmod(w0[g], c00[k], p, pinv);
                a1[g][k] += mulmod(w0[g], c01[k], p, pinv);
                a0[g][k] += mulmod(w1[g], c10[k], p, pinv);
                a1[g][k] += mulmod(w1[g], c11[k], p, pinv);
            }
        }
        if (((jb - jb0) & 7) == 6) {
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    a0[g][k] = reduce(a0[g][k], p, pinv);
                    a1[g][k] = reduce(a1[g][k], p, pinv);
                }
        }
        wp += 512;
    }
    if (jb < jb1) {
        double c0[KB], c1[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            if (k < cols) {
                c0[k] = cpk[k][0];
                c1[k] = cpk[k][256];
            } else {
                c0[k] = c1[k] = 0.0;
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double w = g < rows ? __builtin_nontemporal_load(wp + g * wrow) : 0.0;
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                a0[g][k] += mulmod(w, c0[k], p, pinv);
                a1[g][k] += mulmod(w, c1[k], p, pinv);
            }
        }
    }
    const int z = (zc << 8) + zz;
    const size_t comp = (size_t)L * N;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k >= cols) continue;
        double *ak = cs.a(kb0 + k, l, z);
        const size_t ar = cs.arow(kb0 + k);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g < rows) {
                double *d0 = ak + (size_t)(ib0 + g) * ar;
                const double v0 = reduce(a0[g][k], p, pinv), v1 = reduce(a1[g][k], p, pinv);
                if (mode == 0) {
                    d0[0] = v0;
                    d0[comp] = v1;
                } else {
                    atomicAdd(d0, v0);
                    atomicAdd(d0 + comp, v1);
                }
            }
        }
    }
}

// A tile whose last column tile is ragged (c < KB columns left) reads the
// weight words once either way: with c > KB/2 it runs at full width with the
// absent columns' input words taken as zero (the product is usually bound by
// HBM, not by those extra modular products); with c <= KB/2 it runs as
// narrower tiles (KB/2, KB/4, ...), each of which fits the columns left.
template <int G, int KB, class Cols>
__device__ __forceinline__ void mac_tile(const double *__restrict__ Wt, const Cols &cs,
                                         const MacShape &s, const DevParams &dp, int l, int zc,
                                         int zz, int kb0, int ib0, int jb0, int jb1, int mode)
{
    const int cols = cs.ncols() - kb0;
    if (KB == 1 || 2 * cols > KB) {
        mac_range<G, KB>(Wt, cs, s, dp, l, zc, zz, kb0, ib0, jb0, jb1, mode);
        return;
    }
    if constexpr (KB >= 2) mac_tile<G, KB / 2>(Wt, cs, s, dp, l, zc, zz, kb0, ib0, jb0, jb1, mode);
}

// Row tiles per workgroup of the stream-K product.  With RT > 1 a workgroup
// covers 256 / RT slots of a chunk for RT consecutive row tiles (one per group
// of 256 / RT lanes), so the input words of its column tile are fetched once
// into the CU's L1 and read by all RT row tiles; at RT = 1 it covers the whole
// chunk for one row tile.
__host__ __device__ constexpr int mac_rt(int G, int KB) { return KB > 1 ? 4 : 1; }

// Product tile shapes (G rows, KB column blocks per thread) the library instantiates.
#define PIMM_MAC_SHAPES(X) \
    X(4, 1) X(8, 1) X(16, 1) X(4, 2) X(8, 2) X(16, 2) X(2, 4) X(4, 4) X(8, 4) X(2, 8) X(4, 8)

__host__ __device__ constexpr bool mac_shape_ok(int G, int KB)
{
    return (KB == 1 && (G == 4 || G == 8 || G == 16)) ||
           (KB == 2 && (G == 4 || G == 8 || G == 16)) ||
           (KB == 4 && (G == 2 || G == 4 || G == 8)) || (KB == 8 && (G == 2 || G == 4));
}

// ---- stores into the chunk-contiguous layouts (NTT output slot z) --------------

// Weight block w = ib*R + jb, prime l: poly = w*L + l.
struct StoreWeightTiled {
    double *out;
    int logn, L;
    uint32_t M, R;
    __device__ void operator()(const PolyIx &pi, int z, double v, double, double) const
    {
        const uint32_t w = (uint32_t)pi.x, l = (uint32_t)pi.l;
        const uint32_t ib = w / R, jb = w % R;
        const size_t chunks = (size_t)1 << (logn - 8);
        const size_t zc = (size_t)(z >> 8), zz = (size_t)(z & 255);
        out[((((size_t)l * chunks + zc) * M + ib) * R + jb) * 256 + zz] = v;
    }
};

// Input ciphertext g*R*K + jb*K + kb (product g of G, inner block jb, column block kb),
// component c, prime l: poly = (x*2 + c)*L + l.  The layout has G*K columns, column
// g*K + kb for product g.
struct StoreCtTiled {
    double *out;
    int logn, L;
    uint32_t K, R, G;
    // comp < 0: polynomial (x*2 + c)*L + l of the ciphertexts; else polynomial x*L + l of
    // component comp alone.
    int comp;
    __device__ void operator()(const PolyIx &pi, int z, double v, double, double) const
    {
        const uint32_t xg = comp < 0 ? (uint32_t)(pi.x >> 1) : (uint32_t)pi.x;
        const uint32_t c = comp < 0 ? (uint32_t)(pi.x & 1) : (uint32_t)comp, l = (uint32_t)pi.l;
        const uint32_t g = xg / (K * R), x = xg - g * (K * R);
        const uint32_t jb = x / K, kb = g * K + x % K;
        const size_t chunks = (size_t)1 << (logn - 8);
        const size_t zc = (size_t)(z >> 8), zz = (size_t)(z & 255);
        out[(((((size_t)l * chunks + zc) * ((size_t)G * K) + kb) * R + jb) * 2 + c) * 256 + zz] = v;
    }
};

// Accumulator slots that may hold unreduced sums of a few partials.
struct LoadSlotsReduce {
    const double *a;
    int logn;
    __device__ double operator()(const PolyIx &pi, int z, double p, double pinv) const
    {
        return reduce(a[((size_t)pi.poly << logn) + z], p, pinv);
    }
};

}  // namespace pimm
