// mfma.h -- the matrix-core form of the slot-wise products (mfma.hip) and the
// 16-slot-chunk layouts its operands use.
#pragma once

#include "common.h"

namespace pimm {

// Plans the matrix-core product serves: at most 64 inner blocks (one 64-deep int8
// product per digit pair) and at least 8 column blocks (16 columns with both
// ciphertext components), where the product is bound by arithmetic.
bool mfma_eligible(const pimm_plan_info &f);
// Bytes of the digit form of a weight cache for plan f.
uint64_t digit_cache_bytes(const Ctx &c, const pimm_plan_info &f);
// Digit form [L][N][7][Mt][64][16 B] of the FP64 cache Wt [L][N/256][M][R][256].
int build_weight_digits(const Ctx &c, const pimm_plan_info &f, const double *Wt, void *Wd,
                        hipStream_t s);
// acc^ [L][N/kAccRun][O][2][kAccRun] = the slot-wise products of the query ciphertexts ct
// [I][2][L][N] (in evaluation form, read in place) with the digit weight cache Wd.  Every
// accumulator is written once (no zeroing needed).
int launch_mac_mfma(const Ctx &c, const pimm_plan_info &f, const void *Wd, const uint64_t *ct, double *Ah,
                    hipStream_t s);

// Accumulators of the matrix-core product in runs of the kAccRun slots one workgroup
// computes: polynomial (o*2 + comp)*L + l, slot z at [L][N/kAccRun][O][2][kAccRun] (a
// wave's stores then cover whole lines).  NR = N / kAccRun.
constexpr int kAccRun = 8;
__device__ __forceinline__ size_t acc_run_index(const PolyIx &pi, int z, uint32_t O2, uint32_t NR)
{
    const size_t base = ((size_t)pi.l * NR * O2 + (uint32_t)pi.x) * kAccRun + ((uint32_t)z % kAccRun);
    return (size_t)((uint32_t)z / kAccRun) * (O2 * (uint32_t)kAccRun) + base;
}

// Accumulators in that layout, reduced (the plain pimm_matmul's inverse transform).
struct LoadSlotsReduceRun {
    const double *a;
    uint32_t O2, NR;
    int L;
    __device__ double operator()(const PolyIx &pi, int z, double p, double pinv) const
    {
        return reduce(a[acc_run_index(pi, z, O2, NR)], p, pinv);
    }
};

}  // namespace pimm
