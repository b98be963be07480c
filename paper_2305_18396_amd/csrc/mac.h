// mac.h -- the slot-wise modular products of Algorithm 1 step 3.
//
// For NTT slot z and prime l the products of every inner block are summed:
//     acc^[(ib*K + kb)][comp][l][z] = sum_jb W^[(ib*R + jb)][l][z] * c^[(jb*K + kb)][comp][l][z]
// for both ciphertext components.  One thread owns one slot and G consecutive
// output rows ib0 .. ib0+G-1; per inner block it streams G weight words and
// reuses the two input words of that slot.  Partial sums of balanced products
// (each below 0.6 p in magnitude) stay below 2^53 with a reduction every 8
// inner blocks.
#pragma once

#include "common.h"

namespace pimm {

// Inner blocks jb0 .. jb1-1 only (a split of the inner dimension writes its own
// partial accumulator; the inverse NTT's loader adds the partials).
template <int G>
__device__ __forceinline__ void mac_tile(const double *__restrict__ Wh, const double *__restrict__ Ch,
                                         double *__restrict__ Ah, int M, int R, int K,
                                         const DevParams &dp, int l, int z, int ib0, int kb,
                                         int jb0 = 0, int jb1 = -1)
{
    if (jb1 < 0) jb1 = R;
    const int N = dp.N, L = dp.L;
    const double p = dp.p[l], pinv = dp.pinv[l];
    const int rows = M - ib0 < G ? M - ib0 : G;

    double a0[G], a1[G];
#pragma unroll
    for (int g = 0; g < G; ++g) a0[g] = a1[g] = 0.0;

    const size_t wstep = (size_t)L * N;          // next jb in W^
    const size_t cstep = (size_t)K * 2 * L * N;  // next jb in c^
    const size_t wrow = (size_t)R * L * N;       // next ib in W^
    const double *wp = Wh + (((size_t)ib0 * R + jb0) * L + l) * N + z;
    const double *cp = Ch + ((((size_t)jb0 * K + kb) * 2) * L + l) * N + z;

    for (int jb = jb0; jb < jb1; ++jb) {
        const double c0 = cp[0];
        const double c1 = cp[(size_t)L * N];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g < rows) {
                const double w = wp[g * wrow];
                a0[g] += mulmod(w, c0, p, pinv);
                a1[g] += mulmod(w, c1, p, pinv);
            }
        }
        if (((jb - jb0) & 7) == 7) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                a0[g] = reduce(a0[g], p, pinv);
                a1[g] = reduce(a1[g], p, pinv);
            }
        }
        wp += wstep;
        cp += cstep;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (g < rows) {
            const size_t y = (size_t)(ib0 + g) * K + kb;
            Ah[((y * 2 + 0) * L + l) * N + z] = reduce(a0[g], p, pinv);
            Ah[((y * 2 + 1) * L + l) * N + z] = reduce(a1[g], p, pinv);
        }
    }
}

}  // namespace pimm
