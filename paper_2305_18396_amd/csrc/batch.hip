// batch.hip -- many independent Pi_MatMul products in one pass over the device.
//
// A batch is a list of (plan, weight cache, input ciphertexts, accumulator)
// items of any shapes and sequence lengths on one context.  Its work is the
// union of three kinds of units:
//   in   one input polynomial (already in evaluation form) into the tiled layout (sum over items of I*2*L)
//   mac  one slot group x row-tile group x column tile (RT row tiles per group);
//        under the phased schedule the items that share a weight cache line up
//        their column blocks, and a column tile may span items, so every weight
//        word is read once per KB columns of the whole group
//        (sum over weight caches of (N/256)*L*RT*ceil(ceil(M/G)/RT)*ceil(sum K/KB));
//        the persistent schedule keeps one set per item (its dependency counters
//        are per item)
//   out  inverse NTT of one accumulator polynomial (sum of O*2*L)
// Two schedules run them:
//   PHASED      three launches (all in, all mac, all out), each over a flat
//               list of units of every item;
//   PERSISTENT  one launch of a resident grid that takes units from an atomic
//               counter in dependency order (in, then mac, then out).  A mac
//               unit waits until the 2R input moves of each column block of its
//               column tile and prime are done; an out unit waits until the
//               mac units of its (row-tile group, column tile, prime) are
//               done.  Every unit it waits for was taken
//               earlier by a running workgroup that itself only waits on
//               earlier units, so the waits always end; each wait is also
//               bounded (a spin limit sets an error flag and every later wait
//               returns at once), so every wave exits.
// The item table lives in device memory owned by the batch; the scratch (NTT
// forms, accumulators, dependency counters) is the caller's workspace.  Both
// schedules are plain kernel launches with no memset, so a stream capture of
// pimm_batch_matmul can be replayed as a hipGraph.
#include <string.h>

#include <algorithm>
#include <map>
#include <vector>

#include "batch.h"
#include "common.h"
#include "mac.h"
#include "ntt.h"

namespace pimm {

__device__ __forceinline__ int find_item(const BatchItemDev *items, int n, uint32_t u, int which)
{
    // last item whose first unit of this kind is <= u
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const uint32_t s = which == 0 ? items[mid].in0 : (which == 1 ? items[mid].mac0 : items[mid].out0);
        if (s <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Input polynomial `poly` of an item's ciphertexts [I][2][L][N], already in evaluation form,
// moved into the tiled layout as balanced doubles.
template <int LOGN>
__device__ __forceinline__ void run_in(const BatchItemDev &it, int poly, double *ws,
                                       const DevParams &dp, double *)
{
    const StoreCtTiled st{ws + it.chat_off, LOGN, dp.L, it.K, it.R, 1u, -1};
    const PolyIx pi = poly_ix(poly, dp.L);
    const double p = dp.p[pi.l];
    const uint64_t *src = it.ct + ((size_t)poly << LOGN);
    double v[(1 << LOGN) / kNttThreads];
#pragma unroll
    for (int k = 0; k < (1 << LOGN) / kNttThreads; ++k) v[k] = f64_of(src[(int)threadIdx.x + k * kNttThreads]);
#pragma unroll
    for (int k = 0; k < (1 << LOGN) / kNttThreads; ++k)
        st(pi, (int)threadIdx.x + k * kNttThreads, v[k] > 0.5 * p ? v[k] - p : v[k], p, 0.0);
}

template <int LOGN>
__device__ __forceinline__ void run_out(const BatchItemDev &it, int poly, double *ws,
                                        const DevParams &dp, double *lds)
{
    ntt_inv_block<LOGN, kNttThreads>(LoadSlotsReduce{ws + it.ahat_off, LOGN}, StoreU64{it.acc, LOGN}, dp,
                                     poly, lds);
}

// mac unit t of an item -> (l, slot chunk, slot group, column tile, row-tile group), row-tile
// groups fastest.  With RT = mac_rt(G, KB) row tiles per group, lane group w of the
// workgroup (256 / RT lanes) takes row tile ig * RT + w over slots sub * 256 / RT ...
struct MacCoord {
    int l, zc, sub, kbt, ig;
};
__device__ __forceinline__ MacCoord mac_coord(const BatchItemDev &it, uint32_t t, int chunks, int RT)
{
    MacCoord c;
    c.ig = (int)(t % it.mgroups);
    t /= it.mgroups;
    c.kbt = (int)(t % it.ktiles);
    t /= it.ktiles;
    c.sub = (int)(t % RT);
    t /= RT;
    c.zc = (int)(t % chunks);
    c.l = (int)(t / chunks);
    return c;
}

template <int G, int KB>
__device__ __forceinline__ void run_mac(const BatchItemDev &it, const MacCoord &c, double *ws,
                                        const DevParams &dp)
{
    constexpr int RT = mac_rt(G, KB), SPW = 256 / RT;
    const int lane = (int)threadIdx.x % SPW, w = (int)threadIdx.x / SPW;
    const int ibt = c.ig * RT + w;
    if (ibt >= (int)it.mtiles) return;
    const MacShape sh{(int)it.M, (int)it.R, (int)it.K, dp.N >> 8};
    mac_tile<G, KB>(it.wh, ColsOne{ws + it.chat_off, ws + it.ahat_off, sh, dp.L, dp.N}, sh, dp, c.l,
                    c.zc, c.sub * SPW + lane, c.kbt * KB, ibt * G, 0, (int)it.R, 0);
}

// ---- phased schedule ---------------------------------------------------------------

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_batch_in(const BatchItemDev *items, int n,
                                                          double *ws, DevParams dp)
{
    const uint32_t u = blockIdx.x;
    const BatchItemDev &it = items[find_item(items, n, u, 0)];
    run_in<LOGN>(it, (int)(u - it.in0), ws, dp, nullptr);
}

// The columns of one weight group (see BatchGroupDev): column j is block kb of
// item `item`, with that item's c^ and acc^ in the workspace.
struct ColsGroup {
    const BatchColDev *cols;  // the group's first column
    const BatchItemDev *items;
    double *ws;
    int n, chunks, L, N;
    __device__ __forceinline__ int ncols() const { return n; }
    __device__ __forceinline__ const double *c(int j, int l, int zc, int zz) const
    {
        const BatchColDev cd = cols[j];
        const BatchItemDev &it = items[cd.item];
        return ws + it.chat_off + ((((size_t)l * chunks + zc) * it.K + cd.kb) * it.R) * 512 + zz;
    }
    __device__ __forceinline__ double *a(int j, int l, int z) const
    {
        const BatchColDev cd = cols[j];
        return ws + items[cd.item].ahat_off + ((size_t)cd.kb * 2 * L + l) * N + z;
    }
    __device__ __forceinline__ size_t arow(int j) const
    {
        return (size_t)items[cols[j].item].K * 2 * L * N;
    }
    __device__ __forceinline__ int row_end(const MacShape &sh) const { return sh.M; }
};

// Phased product: one unit per (prime, slot chunk, slot group, column tile, row-tile
// group) of a weight group, whole inner dimension, row-tile groups fastest.
template <int G, int KB>
__global__ __launch_bounds__(256) void k_batch_mac(const BatchGroupDev *groups, int ng,
                                                   const BatchColDev *cols,
                                                   const BatchItemDev *items, double *ws,
                                                   int xcd_map, DevParams dp)
{
    constexpr int RT = mac_rt(G, KB), SPW = 256 / RT;
    const uint32_t u = xcd_map ? xcd_local(blockIdx.x, gridDim.x) : blockIdx.x;
    int lo = 0, hi = ng - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (groups[mid].mac0 <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchGroupDev &g = groups[lo];
    const int chunks = dp.N >> 8;
    uint32_t t = u - g.mac0;
    const int ig = (int)(t % g.mgroups);
    t /= g.mgroups;
    const int kbt = (int)(t % g.ktiles);
    t /= g.ktiles;
    const int sub = (int)(t % RT);
    t /= RT;
    const int zc = (int)(t % chunks);
    const int l = (int)(t / chunks);
    const int lane = (int)threadIdx.x % SPW, w = (int)threadIdx.x / SPW;
    const int ibt = ig * RT + w;
    if (ibt >= (int)g.mtiles) return;
    const MacShape sh{(int)g.M, (int)g.R, 0, chunks};
    mac_tile<G, KB>(g.wh, ColsGroup{cols + g.col0, items, ws, (int)g.ncols, chunks, dp.L, dp.N}, sh,
                    dp, l, zc, sub * SPW + lane, kbt * KB, ibt * G, 0, (int)g.R, 0);
}

template <int LOGN>
__global__ __launch_bounds__(kNttThreads) void k_batch_out(const BatchItemDev *items, int n,
                                                           double *ws, DevParams dp)
{
    __shared__ double lds[NttPasses<LOGN, kNttThreads>::LDS];
    const uint32_t u = blockIdx.x;
    const BatchItemDev &it = items[find_item(items, n, u, 2)];
    run_out<LOGN>(it, (int)(u - it.out0), ws, dp, lds);
}

// ---- persistent schedule -----------------------------------------------------------

__global__ void k_batch_reset(uint32_t *ctr, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        ctr[i] = 0;
}

// Thread 0 waits until ctr[idx] >= target (acquire, device scope) or the batch
// has failed; returns false on failure.  Bounded by spin_limit polls.
__device__ __forceinline__ bool wait_for(uint32_t *ctr, uint32_t idx, uint32_t target,
                                         uint32_t spin_limit)
{
    uint32_t spins = 0;
    while (__hip_atomic_load(&ctr[idx], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(&ctr[kCtrError], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return false;
        if (++spins > spin_limit) {
            __hip_atomic_store(&ctr[kCtrError], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

template <int LOGN, int G, int KB>
__global__ __launch_bounds__(kNttThreads) void k_batch_fused(const BatchItemDev *items, int n,
                                                             double *ws, uint32_t *ctr,
                                                             uint32_t n_in, uint32_t n_mac,
                                                             uint32_t n_out, uint32_t spin_limit,
                                                             DevParams dp)
{
    __shared__ double lds[NttPasses<LOGN, kNttThreads>::LDS];
    __shared__ uint32_t s_unit;
    __shared__ int s_ok;
    const uint32_t total = n_in + n_mac + n_out;
    const int chunks = dp.N >> 8, L = dp.L;
    for (;;) {
        if (threadIdx.x == 0)
            s_unit = __hip_atomic_fetch_add(&ctr[kCtrQueue], 1u, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t u = s_unit;
        __syncthreads();
        if (u >= total) break;
        uint32_t sig = 0xffffffffu;  // counter this unit bumps when done
        if (u < n_in) {
            const BatchItemDev &it = items[find_item(items, n, u, 0)];
            const int poly = (int)(u - it.in0);
            run_in<LOGN>(it, poly, ws, dp, lds);
            const int x = poly / (2 * L), l = poly % L;
            sig = it.dep_in0 + (uint32_t)(((x % (int)it.K) / KB) * L + l);
        } else if (u < n_in + n_mac) {
            const uint32_t v = u - n_in;
            const BatchItemDev &it = items[find_item(items, n, v, 1)];
            const MacCoord c = mac_coord(it, v - it.mac0, chunks, mac_rt(G, KB));
            // Every input move of the column tile's blocks for this prime.
            const int left = (int)it.K - c.kbt * KB;
            const uint32_t cols = (uint32_t)(left < KB ? left : KB);
            if (threadIdx.x == 0)
                s_ok = wait_for(ctr, it.dep_in0 + (uint32_t)(c.kbt * L + c.l), 2 * it.R * cols,
                                spin_limit);
            __syncthreads();
            __threadfence();
            if (s_ok) run_mac<G, KB>(it, c, ws, dp);
            sig = it.dep_mac0 + (uint32_t)(((c.ig * (int)it.ktiles) + c.kbt) * L + c.l);
        } else {
            const uint32_t v = u - n_in - n_mac;
            const BatchItemDev &it = items[find_item(items, n, v, 2)];
            const int poly = (int)(v - it.out0);
            const int y = poly / (2 * L), l = poly % L;
            // Every (slot chunk, slot group) unit of its row-tile group and column tile.
            constexpr int RT = mac_rt(G, KB);
            const int ig = (y / (int)it.K) / G / RT, kbt = (y % (int)it.K) / KB;
            if (threadIdx.x == 0)
                s_ok = wait_for(ctr, it.dep_mac0 + (uint32_t)((ig * (int)it.ktiles + kbt) * L + l),
                                (uint32_t)(chunks * RT), spin_limit);
            __syncthreads();
            __threadfence();
            if (s_ok) run_out<LOGN>(it, poly, ws, dp, lds);
        }
        if (sig != 0xffffffffu) {
            __threadfence();
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_fetch_add(&ctr[sig], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

}  // namespace pimm

using namespace pimm;

namespace {

int build_tables(pimm_batch *b, bool async, hipStream_t s)
{
    const Ctx &c = *b->ctx;
    const uint64_t N = c.params.N, L = c.params.L;
    const uint32_t chunks = (uint32_t)(N >> 8);
    const size_t n = b->items.size();
    std::vector<BatchItemDev> t(n);
    uint32_t in0 = 0, mac0 = 0, out0 = 0, dep = kCtrFirstDep;
    b->useful_macs = 0;
    for (size_t i = 0; i < n; ++i) {
        const pimm_batch_item &it = b->items[i];
        const pimm_plan_info &f = it.plan->info;
        BatchItemDev &d = t[i];
        d.ct = it.ct;
        d.acc = it.acc;
        d.wh = it.weights->d_w_hat;
        d.M = f.M;
        d.R = f.R;
        d.K = f.K;
        d.I = f.I;
        d.O = f.O;
        const uint32_t RT = (uint32_t)mac_rt(b->G, b->KB);
        d.mtiles = (f.M + b->G - 1) / b->G;
        d.mgroups = (d.mtiles + RT - 1) / RT;
        d.ktiles = (f.K + b->KB - 1) / b->KB;
        d.in0 = in0;
        d.mac0 = mac0;
        d.out0 = out0;
        d.dep_in0 = dep;
        dep += d.ktiles * (uint32_t)L;
        d.dep_mac0 = dep;
        dep += d.mgroups * d.ktiles * (uint32_t)L;
        in0 += f.I * 2 * (uint32_t)L;
        mac0 += chunks * (uint32_t)L * RT * d.mgroups * d.ktiles;
        out0 += f.O * 2 * (uint32_t)L;
        b->useful_macs += (uint64_t)f.n * f.r * f.m;
    }
    // Counters first (rounded to 256 bytes), then each item's c^ and acc^.
    uint64_t off = (((uint64_t)dep * 4 + 255) / 256) * 256 / 8;
    const bool fixed = b->fixed_chat.size() == n && b->fixed_ahat.size() == n;
    for (size_t i = 0; i < n; ++i) {
        if (fixed) {
            t[i].chat_off = b->fixed_chat[i];
            t[i].ahat_off = b->fixed_ahat[i];
            continue;
        }
        t[i].chat_off = off;
        off += (uint64_t)t[i].I * 2 * L * N;
        t[i].ahat_off = off;
        off += (uint64_t)t[i].O * 2 * L * N;
    }
    b->n_in = in0;
    b->n_mac = mac0;
    b->n_out = out0;
    b->n_dep = dep;
    b->ws_bytes = fixed ? (((uint64_t)dep * 4 + 255) / 256) * 256 : off * 8;

    // Weight groups (first-appearance order) and their columns.
    std::vector<BatchGroupDev> grp;
    std::vector<BatchColDev> cols;
    std::map<const double *, std::vector<uint32_t>> members;
    std::vector<const double *> order;
    for (size_t i = 0; i < n; ++i) {
        auto it = members.find(t[i].wh);
        if (it == members.end()) {
            order.push_back(t[i].wh);
            members[t[i].wh] = {(uint32_t)i};
        } else {
            it->second.push_back((uint32_t)i);
        }
    }
    const uint32_t RT = (uint32_t)mac_rt(b->G, b->KB);
    uint32_t gmac0 = 0;
    for (const double *wh : order) {
        const std::vector<uint32_t> &mem = members[wh];
        BatchGroupDev g;
        g.wh = wh;
        g.M = t[mem[0]].M;
        g.R = t[mem[0]].R;
        g.mtiles = (g.M + b->G - 1) / b->G;
        g.mgroups = (g.mtiles + RT - 1) / RT;
        g.col0 = (uint32_t)cols.size();
        for (uint32_t i : mem)
            for (uint32_t kb = 0; kb < t[i].K; ++kb) cols.push_back(BatchColDev{i, kb});
        g.ncols = (uint32_t)cols.size() - g.col0;
        g.ktiles = (g.ncols + b->KB - 1) / b->KB;
        g.mac0 = gmac0;
        gmac0 += chunks * (uint32_t)L * RT * g.mgroups * g.ktiles;
        grp.push_back(g);
    }
    b->n_groups = (uint32_t)grp.size();
    b->n_mac_grouped = gmac0;

    // One table allocation: items | groups | columns (each 256-byte aligned).
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_grp = a256(n * sizeof(BatchItemDev));
    const size_t o_col = o_grp + a256(grp.size() * sizeof(BatchGroupDev));
    const size_t bytes = o_col + a256(cols.size() * sizeof(BatchColDev));
    int rc = PIMM_OK;
    if (bytes > b->tab_cap) {
        if (b->d_tab) (void)hipFree(b->d_tab);
        b->d_tab = nullptr;
        b->tab_cap = 0;
        rc = check_hip(hipSetDevice(c.device), "hipSetDevice");
        if (!rc) rc = check_hip(hipMalloc((void **)&b->d_tab, bytes), "hipMalloc batch table");
        if (rc) return rc;
        b->tab_cap = bytes;
    }
    if (async && bytes > b->h_cap) {
        if (b->h_tab) (void)hipHostFree(b->h_tab);
        b->h_tab = nullptr;
        b->h_cap = 0;
        rc = check_hip(hipHostMalloc((void **)&b->h_tab, bytes, 0), "hipHostMalloc batch table");
        if (rc) return rc;
        b->h_cap = bytes;
    }
    b->d_items = (BatchItemDev *)b->d_tab;
    b->d_groups = (BatchGroupDev *)(b->d_tab + o_grp);
    b->d_cols = (BatchColDev *)(b->d_tab + o_col);
    std::vector<uint8_t> host(async ? 0 : bytes);
    uint8_t *h = async ? b->h_tab : host.data();
    memcpy(h, t.data(), n * sizeof(BatchItemDev));
    memcpy(h + o_grp, grp.data(), grp.size() * sizeof(BatchGroupDev));
    memcpy(h + o_col, cols.data(), cols.size() * sizeof(BatchColDev));
    if (async)
        return check_hip(hipMemcpyAsync(b->d_tab, h, bytes, hipMemcpyHostToDevice, s),
                         "upload batch table");
    return check_hip(hipMemcpy(b->d_tab, h, bytes, hipMemcpyHostToDevice), "copy batch table");
}

template <int LOGN, int G, int KB>
int run_batch(const pimm_batch *b, void *ws, bool with_out, hipStream_t s)
{
    const Ctx &c = *b->ctx;
    const int n = (int)b->items.size();
    double *wsd = (double *)ws;
    if (b->schedule == kPhased) {
        {
            ProfScope prof("ntt_fwd", s);
            hipLaunchKernelGGL(k_batch_in<LOGN>, dim3(b->n_in), dim3(kNttThreads), 0, s, b->d_items,
                               n, wsd, c.dp);
        }
        {
            ProfScope prof("mac", s);
            hipLaunchKernelGGL((k_batch_mac<G, KB>), dim3(b->n_mac_grouped), dim3(256), 0, s,
                               b->d_groups, (int)b->n_groups, b->d_cols, b->d_items, wsd, b->xcd_map,
                               c.dp);
        }
        if (with_out) {
            ProfScope prof("ntt_inv", s);
            hipLaunchKernelGGL(k_batch_out<LOGN>, dim3(b->n_out), dim3(kNttThreads), 0, s,
                               b->d_items, n, wsd, c.dp);
        }
        return check_hip(hipGetLastError(), "batch launch");
    }
    uint32_t *ctr = (uint32_t *)ws;
    hipLaunchKernelGGL(k_batch_reset, dim3((b->n_dep + 255) / 256), dim3(256), 0, s, ctr, b->n_dep);
    uint32_t grid = b->grid;
    if (!grid) {
        int per_cu = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_fused<LOGN, G, KB>,
                                                           kNttThreads, 0);
        int cus = 0;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device);
        grid = (uint32_t)std::max(1, per_cu) * (uint32_t)std::max(1, cus);
    }
    const uint32_t n_out = with_out ? b->n_out : 0;
    const uint32_t total = b->n_in + b->n_mac + n_out;
    if (grid > total) grid = total;
    {
        ProfScope prof("fused", s);
        hipLaunchKernelGGL((k_batch_fused<LOGN, G, KB>), dim3(grid), dim3(kNttThreads), 0, s, b->d_items,
                           n, wsd, ctr, b->n_in, b->n_mac, n_out, b->spin_limit, c.dp);
    }
    return check_hip(hipGetLastError(), "batch fused launch");
}

template <int LOGN>
int run_batch_g(const pimm_batch *b, void *ws, bool with_out, hipStream_t s)
{
#define PIMM_RUN_BATCH(g, kb) \
    if (b->G == g && b->KB == kb) return run_batch<LOGN, g, kb>(b, ws, with_out, s);
    PIMM_MAC_SHAPES(PIMM_RUN_BATCH)
#undef PIMM_RUN_BATCH
    return set_error(PIMM_E_ARG, "product tile %dx%d is not built", b->G, b->KB);
}

}  // namespace

namespace pimm {
int batch_rebuild(pimm_batch *b, bool async, hipStream_t s) { return build_tables(b, async, s); }
void batch_free_tables(pimm_batch *b)
{
    if (b->d_tab) (void)hipFree(b->d_tab);
    if (b->h_tab) (void)hipHostFree(b->h_tab);
    b->d_tab = b->h_tab = nullptr;
    b->d_items = nullptr;
    b->d_groups = nullptr;
    b->d_cols = nullptr;
    b->tab_cap = b->h_cap = 0;
}
int batch_run(const pimm_batch *b, void *ws, hipStream_t s, bool with_out)
{
    return b->ctx->dp.logN == 12 ? run_batch_g<12>(b, ws, with_out, s)
                                 : run_batch_g<13>(b, ws, with_out, s);
}
}  // namespace pimm

extern "C" {

int pimm_batch_create(const pimm_batch_item *items, uint32_t count, pimm_batch **out)
{
    if (!items || !count || !out) return set_error(PIMM_E_ARG, "pimm_batch_create: empty batch");
    Ctx *ctx = items[0].plan ? items[0].plan->ctx : nullptr;
    for (uint32_t i = 0; i < count; ++i) {
        const pimm_batch_item &it = items[i];
        if (!it.plan || !it.weights || !it.ct || !it.acc)
            return set_error(PIMM_E_ARG, "pimm_batch_create: item %u has a NULL field", i);
        if (it.plan->ctx != ctx)
            return set_error(PIMM_E_ARG, "pimm_batch_create: items on different contexts");
        if (!weights_fit(it.weights, it.plan))
            return set_error(PIMM_E_ARG, "pimm_batch_create: item %u weights do not fit its plan", i);
        if (it.plan->info.groups > 1)
            return set_error(PIMM_E_UNSUPPORTED, "pimm_batch_create: item %u has a grouped plan", i);
    }
    pimm_batch *b = new pimm_batch();
    b->ctx = ctx;
    b->items.assign(items, items + count);
    int rc = build_tables(b, false, nullptr);
    if (rc) {
        pimm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PIMM_OK;
}

int pimm_batch_destroy(pimm_batch *b)
{
    if (!b) return PIMM_OK;
    batch_free_tables(b);
    delete b;
    return PIMM_OK;
}

int pimm_batch_set_schedule(pimm_batch *b, int schedule, int mac_rows, int mac_cols, int xcd_map,
                            uint32_t grid)
{
    if (!b) return set_error(PIMM_E_ARG, "pimm_batch_set_schedule: NULL batch");
    if (schedule != kPhased && schedule != kPersistent)
        return set_error(PIMM_E_ARG, "schedule %d is not 0 (phased) or 1 (persistent)", schedule);
    if (!mac_shape_ok(mac_rows, mac_cols))
        return set_error(PIMM_E_ARG, "product tile %d rows x %d column blocks is not built",
                         mac_rows, mac_cols);
    b->schedule = schedule;
    b->xcd_map = xcd_map ? 1 : 0;
    b->grid = grid;
    if (mac_rows != b->G || mac_cols != b->KB) {
        b->G = mac_rows;
        b->KB = mac_cols;
        return build_tables(b, false, nullptr);
    }
    return PIMM_OK;
}

int pimm_batch_get_schedule(const pimm_batch *b, int *schedule, int *mac_rows, int *mac_cols,
                            int *xcd_map, uint32_t *grid)
{
    if (!b || !schedule || !mac_rows || !mac_cols || !xcd_map || !grid)
        return set_error(PIMM_E_ARG, "pimm_batch_get_schedule: NULL argument");
    *schedule = b->schedule;
    *mac_rows = b->G;
    *mac_cols = b->KB;
    *xcd_map = b->xcd_map;
    *grid = b->grid;
    return PIMM_OK;
}

int pimm_batch_query(const pimm_batch *b, uint64_t *workspace_bytes, uint64_t *useful_macs)
{
    if (!b) return set_error(PIMM_E_ARG, "pimm_batch_query: NULL batch");
    if (workspace_bytes) *workspace_bytes = b->ws_bytes;
    if (useful_macs) *useful_macs = b->useful_macs;
    return PIMM_OK;
}

int pimm_batch_matmul(const pimm_batch *b, void *ws, size_t ws_bytes, void *stream)
{
    if (!b) return set_error(PIMM_E_ARG, "pimm_batch_matmul: NULL batch");
    if (!ws || ws_bytes < b->ws_bytes)
        return set_error(PIMM_E_WORKSPACE, "pimm_batch_matmul: workspace too small");
    return batch_run(b, ws, (hipStream_t)stream);
}

int pimm_batch_status(const pimm_batch *b, const void *ws, void *stream)
{
    if (!b || !ws) return set_error(PIMM_E_ARG, "pimm_batch_status: NULL argument");
    if (b->schedule != kPersistent) return PIMM_OK;
    uint32_t flag = 0;
    hipStream_t s = (hipStream_t)stream;
    int rc = check_hip(hipMemcpyAsync(&flag, (const uint32_t *)ws + kCtrError, 4,
                                      hipMemcpyDeviceToHost, s), "copy batch status");
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "batch status synchronize");
    if (rc) return rc;
    return flag ? set_error(PIMM_E_DEVICE, "persistent batch: a dependency wait hit its bound")
                : PIMM_OK;
}

}  // extern "C"
