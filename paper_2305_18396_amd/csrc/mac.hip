// mac.hip -- launch of the slot-wise products (Algorithm 1 step 3) for one product.
#include "common.h"
#include "mac.h"

namespace pimm {

// Stream-K schedule: the flattened space of (tile, inner block) iterations is
// cut into equal contiguous ranges, one per workgroup of a grid sized to what
// the device holds at once (ranges placed XCD by XCD).  A tile is
// (prime l, chunk zc, slot group sub, column tile kbt, row-tile group ig) with
//     t = (((l * chunks + zc) * RT + sub) * ktiles + kbt) * mgroups + ig,
// row-tile groups fastest, so a workgroup's consecutive tiles share their input
// slice.  Lane group w of the workgroup takes row tile ig * RT + w.  A
// workgroup that covers a whole tile stores its sums; pieces of split tiles
// are added atomically into the zeroed accumulators.  At most 12 pieces meet
// in one accumulator, so the total stays below 8p < 2^53.
template <int G, int KB>
__global__ __launch_bounds__(256) void k_mac_sk(const double *__restrict__ Wt,
                                                const double *__restrict__ Ct,
                                                double *__restrict__ Ah, MacShape sh, int mtiles,
                                                int ktiles, uint64_t total, uint64_t per,
                                                DevParams dp)
{
    constexpr int RT = mac_rt(G, KB), SPW = 256 / RT;
    const int mgroups = (mtiles + RT - 1) / RT;
    const int lane = (int)threadIdx.x % SPW, w = (int)threadIdx.x / SPW;
    uint64_t u = (uint64_t)xcd_local(blockIdx.x, gridDim.x) * per;
    const uint64_t end = u + per < total ? u + per : total;
    const uint64_t R = (uint64_t)sh.R;
    while (u < end) {
        const uint64_t t = u / R;
        const int jb0 = (int)(u % R);
        const int jb1 = (int)(R - (uint64_t)jb0 < end - u ? R : (uint64_t)jb0 + (end - u));
        const int ig = (int)(t % mgroups);
        uint64_t r = t / mgroups;
        const int kbt = (int)(r % ktiles);
        r /= ktiles;
        const int sub = (int)(r % RT);
        r /= RT;
        const int zc = (int)(r % sh.chunks);
        const int l = (int)(r / sh.chunks);
        const int mode = (jb0 == 0 && jb1 == sh.R) ? 0 : 1;
        const int ibt = ig * RT + w;
        if (ibt < mtiles)
            mac_tile<G, KB>(Wt, ColsOne{Ct, Ah, sh, dp.L, dp.N}, sh, dp, l, zc, sub * SPW + lane,
                            kbt * KB, ibt * G, jb0, jb1, mode);
        u += (uint64_t)(jb1 - jb0);
    }
}

// Grouped plans (G products of one shape): one workgroup per (prime, chunk, product g,
// column block, row tile of GR rows within the product), the whole inner dimension,
// sums stored (no split tiles, no zeroing).  The 256 threads take the chunk's 256
// slots.  Logical index t = (((l * chunks + zc) * G + g) * K1 + kb) * mt1 + ibt.
template <int GR>
__global__ __launch_bounds__(256) void k_mac_grouped(const double *__restrict__ Wt,
                                                     const double *__restrict__ Ct,
                                                     double *__restrict__ Ah, MacShape sh, int M1,
                                                     int K1, int mt1, DevParams dp)
{
    uint32_t t = xcd_local(blockIdx.x, gridDim.x);
    const int ibt = (int)(t % (uint32_t)mt1);
    t /= (uint32_t)mt1;
    const int kb = (int)(t % (uint32_t)K1);
    t /= (uint32_t)K1;
    const uint32_t groups = (uint32_t)(sh.M / M1);
    const int g = (int)(t % groups);
    t /= groups;
    const int zc = (int)(t % (uint32_t)sh.chunks);
    const int l = (int)(t / (uint32_t)sh.chunks);
    mac_tile<GR, 1>(Wt, ColsGrouped{Ct, Ah, sh, dp.L, dp.N, K1, g, M1}, sh, dp, l, zc,
                    (int)threadIdx.x, kb, g * M1 + ibt * GR, 0, sh.R, 0);
}

__global__ void k_fill_zero(double *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

template <int G, int KB>
int launch_mac_gk(const Ctx &c, const pimm_plan_info &f, int waves, const double *Wt,
                  const double *Ct, double *Ah, bool zeroed, hipStream_t s)
{
    const MacShape sh{(int)f.M, (int)f.R, (int)f.K, (int)(c.params.N >> 8)};
    constexpr int RT = mac_rt(G, KB);
    const int mtiles = (int)((f.M + G - 1) / G), ktiles = (int)((f.K + KB - 1) / KB);
    const uint64_t mgroups = (uint64_t)((mtiles + RT - 1) / RT);
    const uint64_t total = (uint64_t)c.params.L * sh.chunks * RT * ktiles * mgroups * f.R;
    int per_cu = 0, cus = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mac_sk<G, KB>, 256, 0);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device);
    uint64_t grid = (uint64_t)(per_cu > 0 ? per_cu : 1) * (uint64_t)(cus > 0 ? cus : 1) * waves;
    uint64_t per = (total + grid - 1) / grid;
    const uint64_t min_per = (f.R + 10) / 11;  // at most 12 pieces per tile
    if (per < min_per) per = min_per;
    grid = (total + per - 1) / per;
    if (!zeroed) {
        const size_t acc_n = (size_t)f.O * 2 * c.params.L * c.params.N;
        hipLaunchKernelGGL(k_fill_zero, dim3(1024), dim3(256), 0, s, Ah, acc_n);
    }
    ProfScope prof("mac", s);
    hipLaunchKernelGGL((k_mac_sk<G, KB>), dim3((unsigned)grid), dim3(256), 0, s, Wt, Ct, Ah, sh,
                       mtiles, ktiles, total, per, c.dp);
    return check_hip(hipGetLastError(), "mac launch");
}

template <int GR>
int launch_mac_grouped(const Ctx &c, const pimm_plan_info &f, const double *Wt, const double *Ct,
                       double *Ah, hipStream_t s)
{
    const MacShape sh{(int)(f.groups * f.M), (int)f.R, (int)(f.groups * f.K), (int)(c.params.N >> 8)};
    const int mt1 = (int)((f.M + GR - 1) / GR);
    const uint64_t grid = (uint64_t)c.params.L * sh.chunks * f.groups * f.K * mt1;
    if (grid > 0x7fffffffull) return set_error(PIMM_E_SHAPE, "grouped product grid too large");
    ProfScope prof("mac", s);
    hipLaunchKernelGGL((k_mac_grouped<GR>), dim3((unsigned)grid), dim3(256), 0, s, Wt, Ct, Ah, sh,
                       (int)f.M, (int)f.K, mt1, c.dp);
    return check_hip(hipGetLastError(), "grouped mac launch");
}

int launch_mac(const Ctx &c, const pimm_plan_info &f, int G, int KB, int waves, const double *Wt,
               const double *Ct, double *Ah, bool zeroed, hipStream_t s)
{
    if (f.groups > 1) {
        // Every accumulator is stored by exactly one workgroup: no zeroing needed.
        if (KB == 1 && G == 4) return launch_mac_grouped<4>(c, f, Wt, Ct, Ah, s);
        if (KB == 1 && G == 8) return launch_mac_grouped<8>(c, f, Wt, Ct, Ah, s);
        if (KB == 1 && G == 16) return launch_mac_grouped<16>(c, f, Wt, Ct, Ah, s);
        return set_error(PIMM_E_UNSUPPORTED, "grouped plans take product tiles 4x1, 8x1 or 16x1");
    }
#define PIMM_LAUNCH_MAC(g, kb) \
    if (G == g && KB == kb) return launch_mac_gk<g, kb>(c, f, waves, Wt, Ct, Ah, zeroed, s);
    PIMM_MAC_SHAPES(PIMM_LAUNCH_MAC)
#undef PIMM_LAUNCH_MAC
    return set_error(PIMM_E_ARG, "product tile %dx%d is not built", G, KB);
}

}  // namespace pimm
