// serve.hip -- continuous-batching server for private-inference requests.
//
// A request is a stack of `layers` x `ops` private linear products (one
// Pi_MatMul per product, Algorithm 1) at the request's sequence length.  The
// non-linear layers between products are interactive protocols outside this
// library, so each product's client share X is drawn fresh from the request's
// client seed (stream tag 10, op id = product step, object = request id,
// draw j -> X[j / r][j % r], low l bits), and products run one after another
// as the interactive dependence requires.
//
// The server replays an arrival trace in real time.  At every tick it
//   1. admits waiting requests in arrival order while the HBM budget has room
//      for the request's buffers (key, ciphertexts, reply, shares and scratch,
//      sized for its largest product) and fewer than max_active run;
//   2. takes the step (layer, op) of the oldest admitted request and, when at least
//      min_batch admitted requests are at that step, runs it for all of them: client
//      share, encode, encrypt; one batched pass of forward transforms and slot-wise
//      products over them (pimm_batch machinery, stopping at acc^), whose products
//      share that step's weight cache and so read it once; then per request the fused
//      server tail (re-randomisation, inverse transform with the reply epilogue, mask)
//      and decryption.  With fewer, the oldest request runs alone through the plain
//      fused call, so light load is served in arrival order, one request at a time.
//      Requests at other steps wait: the oldest request never does, and requests
//      admitted behind it gather at step 0 and run as one cohort once it is done;
//   3. waits for the device, then retires requests whose last product is done.
// A request's key material and buffers stay in device memory from admission to
// completion.  Requests admitted while others are running are admitted at once
// (memory permitting) and share the batched launches of every tick at their step.
//
// Every product's two shares are folded into two order-independent checksums
// per request: one over the (client, server) share pairs and one over their
// sum mod 2^l (which must equal X W).
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "batch.h"
#include "common.h"
#include "mac.h"

namespace pimm {

int keygen_into(const Ctx &c, const Key &key, int64_t *s, double *s_hat, uint64_t *pk, double *tmp,
                int64_t *e, hipStream_t st);

constexpr uint32_t kTagX = 10;

// X[j / r][j % r] = low ell bits of draw j of stream (X, 0, op, obj).
__global__ void k_gen_x(Key key, uint32_t op, uint32_t obj, uint32_t count, int ell, uint64_t *X)
{
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;  // one ChaCha block = 8 draws
    if ((uint64_t)b * 8 >= count) return;
    uint32_t w[16];
    chacha_block(key, b, nonce0(kTagX, 0), op, obj, w);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint64_t j = (uint64_t)b * 8 + i;
        if (j < count) X[j] = mask_of(word64(w, i), ell);
    }
}

__global__ void k_zero_u64(unsigned long long *p, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// cs[0] += sum_i mix(y0_i, y1_i, i, step); cs[1] += sum_i mix((y0_i + y1_i) mod t, i, step).
__global__ void k_checksum(const uint64_t *y0, const uint64_t *y1, uint32_t count, uint32_t step,
                           int ell, unsigned long long *cs)
{
    unsigned long long a = 0, b = 0;
    const uint64_t t1 = (1ull << ell) - 1;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const uint64_t salt = ((uint64_t)step << 40) ^ i;
        a += mix64(y0[i] ^ mix64(y1[i] ^ salt));
        b += mix64(((y0[i] + y1[i]) & t1) ^ mix64(salt));
    }
    atomicAdd(&cs[0], a);
    atomicAdd(&cs[1], b);
}

// First-fit allocator over one device arena (offsets in bytes, 256-aligned).
class Arena {
  public:
    void init(uint64_t size) { free_[0] = size; }
    bool alloc(uint64_t n, uint64_t *off)
    {
        n = (n + 255) & ~255ull;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        n = (n + 255) & ~255ull;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<uint64_t, uint64_t> free_;
};

struct Active {
    pimm_request req;
    uint32_t step = 0;
    uint64_t off = 0, bytes = 0;
    std::vector<pimm_plan> plans;  // one per op of a layer
    pimm_sk sk;                    // views into the arena (never destroyed through the ABI)
    uint64_t *pk, *X, *pt, *ct, *c1, *c0s, *y0, *y1;
    double *ws;
    uint64_t ws_bytes;
    unsigned long long *cs;
    double admit_s = 0;
    uint64_t macs = 0;
};

}  // namespace pimm

using namespace pimm;

struct pimm_server {
    Ctx *ctx = nullptr;
    pimm_serve_config cfg;
    std::vector<uint32_t> d_in, d_out;
    std::vector<const pimm_weights *> weights;
    uint8_t *arena_base = nullptr;
    uint64_t arena_bytes = 0;
    uint64_t counters_bytes = 0;
    pimm_batch batch;
};

namespace {

uint64_t a256(uint64_t x) { return (x + 255) & ~255ull; }

// Buffer layout of one request (sizes for its largest product).
struct Layout {
    uint64_t s, s_hat, pk, X, pt, ct, c1, c0s, y0, y1, ws, cs, total;
};

Layout layout_for(const pimm_server &sv, const std::vector<pimm_plan> &plans)
{
    const uint64_t N = sv.ctx->params.N, L = sv.ctx->params.L;
    uint64_t X = 0, pt = 0, ct = 0, c1 = 0, c0s = 0, y = 0, ws = 0;
    for (const pimm_plan &p : plans) {
        const pimm_plan_info &f = p.info;
        X = std::max<uint64_t>(X, (uint64_t)f.n * f.r * 8);
        pt = std::max(pt, f.pt_bytes);
        ct = std::max(ct, f.ct_bytes);
        c1 = std::max(c1, f.c1_bytes);
        c0s = std::max(c0s, f.c0s_bytes);
        y = std::max(y, f.share_bytes);
        ws = std::max(ws, f.workspace_bytes);
    }
    Layout l;
    uint64_t o = 0;
    auto take = [&](uint64_t n) { uint64_t at = o; o += a256(n); return at; };
    l.s = take(N * 8);
    l.s_hat = take(L * N * 8);
    l.pk = take(2 * L * N * 8);
    l.X = take(X);
    l.pt = take(pt);
    l.ct = take(ct);
    l.c1 = take(c1);
    l.c0s = take(c0s);
    l.y0 = take(y);
    l.y1 = take(y);
    l.ws = take(ws);
    l.cs = take(16);
    l.total = o;
    return l;
}

double now_s(const std::chrono::steady_clock::time_point &t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

int pimm_serve_create(pimm_ctx *ctx, const pimm_serve_config *cfg, pimm_server **out)
{
    if (!ctx || !cfg || !out || !cfg->d_in || !cfg->d_out || !cfg->weights)
        return set_error(PIMM_E_ARG, "pimm_serve_create: NULL argument");
    if (!cfg->layers || !cfg->ops || !cfg->d_fix || !cfg->max_active)
        return set_error(PIMM_E_ARG, "pimm_serve_create: empty stack or zero limits");
    pimm_server *sv = new pimm_server();
    sv->ctx = ctx;
    sv->cfg = *cfg;
    sv->d_in.assign(cfg->d_in, cfg->d_in + cfg->ops);
    sv->d_out.assign(cfg->d_out, cfg->d_out + cfg->ops);
    sv->weights.assign(cfg->weights, cfg->weights + (size_t)cfg->layers * cfg->ops);
    sv->cfg.d_in = sv->d_in.data();
    sv->cfg.d_out = sv->d_out.data();
    sv->cfg.weights = sv->weights.data();
    for (size_t k = 0; k < sv->weights.size(); ++k) {
        const pimm_weights *w = sv->weights[k];
        const uint32_t o = (uint32_t)(k % cfg->ops);
        pimm_plan_info f;
        int rc = plan_rule(*ctx, 1, sv->d_in[o], sv->d_out[o], 0, 0, 0, cfg->d_fix, f);
        if (rc) {
            delete sv;
            return rc;
        }
        if (!w || w->ctx != ctx || w->info.r != f.r || w->info.m != f.m || w->info.mb != f.mb ||
            w->info.rb != f.rb) {
            delete sv;
            return set_error(PIMM_E_ARG, "pimm_serve_create: weights %zu do not fit op %u with "
                                         "block area %u", k, o, cfg->d_fix);
        }
    }
    sv->batch.ctx = ctx;
    sv->batch.schedule = cfg->schedule;
    sv->batch.G = cfg->mac_rows ? (int)cfg->mac_rows : 8;
    sv->batch.KB = cfg->mac_cols ? (int)cfg->mac_cols : 1;
    if (!mac_shape_ok(sv->batch.G, sv->batch.KB)) {
        delete sv;
        return set_error(PIMM_E_ARG, "pimm_serve_create: product tile %d rows x %d column blocks "
                                     "is not built", (int)cfg->mac_rows, (int)cfg->mac_cols);
    }
    // Dependency counters of the persistent schedule sit at the start of the arena.
    sv->counters_bytes = a256(4ull * (2 + (uint64_t)cfg->max_active * 4096));
    sv->arena_bytes = cfg->hbm_budget;
    int rc = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
    if (!rc) rc = check_hip(hipMalloc((void **)&sv->arena_base, sv->arena_bytes), "hipMalloc arena");
    if (rc) {
        delete sv;
        return rc;
    }
    *out = sv;
    return PIMM_OK;
}

int pimm_serve_destroy(pimm_server *sv)
{
    if (!sv) return PIMM_OK;
    if (sv->arena_base) (void)hipFree(sv->arena_base);
    batch_free_tables(&sv->batch);
    delete sv;
    return PIMM_OK;
}

int pimm_serve_footprint(const pimm_server *sv, uint32_t seq, uint64_t *bytes)
{
    if (!sv || !bytes || !seq) return set_error(PIMM_E_ARG, "pimm_serve_footprint: bad argument");
    std::vector<pimm_plan> plans(sv->cfg.ops);
    for (uint32_t o = 0; o < sv->cfg.ops; ++o) {
        plans[o].ctx = sv->ctx;
        int rc = plan_rule(*sv->ctx, seq, sv->d_in[o], sv->d_out[o], 0, 0, 0, sv->cfg.d_fix,
                           plans[o].info);
        if (rc) return rc;
    }
    *bytes = layout_for(*sv, plans).total;
    return PIMM_OK;
}

int pimm_serve_run(pimm_server *sv, const pimm_request *reqs, uint32_t count,
                   pimm_request_result *results, void *stream)
{
    if (!sv || (!reqs && count) || (!results && count))
        return set_error(PIMM_E_ARG, "pimm_serve_run: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const Ctx &c = *sv->ctx;
    const uint32_t steps = sv->cfg.layers * sv->cfg.ops;
    const uint64_t N = c.params.N, L = c.params.L;

    std::vector<uint32_t> order(count);
    for (uint32_t i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
    std::deque<uint32_t> waiting(order.begin(), order.end());
    std::vector<Active *> active;
    Arena arena;
    arena.init(sv->arena_bytes - sv->counters_bytes);
    const uint64_t base_off = sv->counters_bytes;
    unsigned long long *h_cs = nullptr;
    int rc = check_hip(hipHostMalloc((void **)&h_cs, 16ull * std::max(1u, count), 0), "hipHostMalloc");
    if (rc) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    uint32_t done = 0;

    auto fail = [&](int code) {
        (void)hipStreamSynchronize(s);
        for (Active *a : active) delete a;
        (void)hipHostFree(h_cs);
        return code;
    };

    while (done < count) {
        // 1. admission
        double now = now_s(t0);
        while (!waiting.empty() && active.size() < sv->cfg.max_active &&
               reqs[waiting.front()].arrival_s <= now) {
            const pimm_request &rq = reqs[waiting.front()];
            Active *a = new Active();
            a->req = rq;
            a->plans.resize(sv->cfg.ops);
            for (uint32_t o = 0; o < sv->cfg.ops; ++o) {
                a->plans[o].ctx = sv->ctx;
                rc = plan_rule(c, rq.seq, sv->d_in[o], sv->d_out[o], 0, 0, 0, sv->cfg.d_fix,
                               a->plans[o].info);
                if (rc) {
                    delete a;
                    return fail(rc);
                }
                // Schedule of the plain fused call a request outside a batch takes: one row per weight
                // word per column block when there are few column blocks.
                const uint32_t K = a->plans[o].info.K;
                a->plans[o].mac_rows = K <= 1 ? 16 : 8;
                a->plans[o].mac_cols = K <= 1 ? 1 : (K == 2 ? 2 : 4);
                a->plans[o].waves = 1;
            }
            const Layout lay = layout_for(*sv, a->plans);
            if (lay.total > sv->arena_bytes - sv->counters_bytes) {
                delete a;
                return fail(set_error(PIMM_E_OOM, "request %llu (seq %u) needs %llu bytes, more "
                                                  "than the whole budget",
                                      (unsigned long long)rq.id, rq.seq,
                                      (unsigned long long)lay.total));
            }
            uint64_t off = 0;
            if (!arena.alloc(lay.total, &off)) {
                delete a;
                break;  // no room now; retry after a retirement
            }
            a->off = base_off + off;
            a->bytes = lay.total;
            uint8_t *p = sv->arena_base + a->off;
            a->sk.ctx = sv->ctx;
            a->sk.d_s = (int64_t *)(p + lay.s);
            a->sk.d_s_hat = (double *)(p + lay.s_hat);
            a->pk = (uint64_t *)(p + lay.pk);
            a->X = (uint64_t *)(p + lay.X);
            a->pt = (uint64_t *)(p + lay.pt);
            a->ct = (uint64_t *)(p + lay.ct);
            a->c1 = (uint64_t *)(p + lay.c1);
            a->c0s = (uint64_t *)(p + lay.c0s);
            a->y0 = (uint64_t *)(p + lay.y0);
            a->y1 = (uint64_t *)(p + lay.y1);
            a->ws = (double *)(p + lay.ws);
            a->ws_bytes = lay.cs - lay.ws;
            a->cs = (unsigned long long *)(p + lay.cs);
            a->admit_s = now;
            const Key ck = make_key(rq.client_seed);
            // Key generation into the request's own buffers (scratch: its workspace).
            rc = keygen_into(c, ck, a->sk.d_s, a->sk.d_s_hat, a->pk, a->ws,
                             (int64_t *)(a->ws + L * N), s);
            if (!rc) {
                hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, a->cs, 2u);
                rc = check_hip(hipGetLastError(), "serve checksum reset");
            }
            if (rc) {
                arena.release(off, lay.total);
                delete a;
                return fail(rc);
            }
            active.push_back(a);
            waiting.pop_front();
        }
        if (active.empty()) {
            if (waiting.empty()) break;
            const double wait = reqs[waiting.front()].arrival_s - now_s(t0);
            if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
            continue;
        }
        // 2. one product for every active request at the oldest request's step: they
        // share that step's weight cache, so the batched pass reads it once for all of them.
        // Requests at other steps wait for a later tick (the oldest request never waits).
        const uint32_t step_now = active.front()->step;
        std::vector<Active *> tick;
        for (Active *a : active)
            if (a->step == step_now) tick.push_back(a);
        // Fewer than min_batch at that step: the oldest request runs alone (requests are
        // then served in arrival order, as one at a time would serve them); interleaving a
        // small cohort without the batched pass would only delay its first members.
        const size_t min_batch = sv->cfg.min_batch ? sv->cfg.min_batch : 8;
        if (tick.size() < min_batch) tick.resize(1);
        const uint32_t o_now = step_now % sv->cfg.ops;
        for (Active *a : tick) {
            const pimm_plan *plan = &a->plans[o_now];
            const pimm_plan_info &f = plan->info;
            const Key ck = make_key(a->req.client_seed);
            const uint32_t cnt = f.n * f.r;
            hipLaunchKernelGGL(k_gen_x, dim3((cnt / 8 + 255) / 256 + 1), dim3(256), 0, s, ck, a->step,
                               (uint32_t)a->req.id, cnt, c.dp.ell, a->X);
            rc = check_hip(hipGetLastError(), "serve gen_x");
            if (!rc) rc = pimm_encode_input(plan, a->X, a->pt, s);
            if (!rc) rc = pimm_encrypt(plan, &a->sk, a->req.client_seed, a->step, a->pt, a->ct, a->ws,
                                       a->ws_bytes, s);
            if (rc) return fail(rc);
        }
        const bool batched = tick.size() > 1;
        if (!batched) {
            // One request: the plain fused server call (stream-K product).
            Active *a = tick[0];
            rc = pimm_matmul_share(&a->plans[o_now], sv->weights[a->step], a->pk, a->req.server_seed,
                                   a->step, a->ct, a->c1, a->c0s, a->y1, a->ws, a->ws_bytes, s);
            if (rc) return fail(rc);
        } else {
            std::vector<pimm_batch_item> items(tick.size());
            sv->batch.fixed_chat.resize(tick.size());
            sv->batch.fixed_ahat.resize(tick.size());
            for (size_t i = 0; i < tick.size(); ++i) {
                Active *a = tick[i];
                const pimm_plan_info &f = a->plans[o_now].info;
                // No accumulator in coefficient form: the batched pass stops after the
                // products and each request's fused tail reads acc^ from its workspace.
                items[i] = pimm_batch_item{&a->plans[o_now], sv->weights[a->step], a->ct, nullptr};
                // The product's NTT forms live in the request's workspace (as pimm_matmul lays them).
                const uint64_t ws_off = (uint64_t)((uint8_t *)a->ws - sv->arena_base) / 8;
                sv->batch.fixed_chat[i] = ws_off;
                sv->batch.fixed_ahat[i] = ws_off + (uint64_t)f.I * 2 * L * N;
            }
            sv->batch.items = items;
            rc = batch_rebuild(&sv->batch, true, s);
            if (!rc && sv->batch.ws_bytes > sv->counters_bytes)
                rc = set_error(PIMM_E_ARG, "serve: too many dependency counters for the reserve");
            if (!rc) rc = batch_run(&sv->batch, sv->arena_base, s, false);
            if (rc) return fail(rc);
            for (Active *a : tick) {
                rc = fused_tail(&a->plans[o_now], a->pk, make_key(a->req.server_seed), a->step, a->ws,
                                a->c1, a->c0s, a->y1, false, s);
                if (rc) return fail(rc);
            }
        }
        for (Active *a : tick) {
            const pimm_plan *plan = &a->plans[o_now];
            const pimm_plan_info &f = plan->info;
            rc = pimm_decrypt(plan, &a->sk, a->c1, a->c0s, a->y0, a->ws, a->ws_bytes, s);
            if (!rc) {
                hipLaunchKernelGGL(k_checksum, dim3(64), dim3(256), 0, s, a->y0, a->y1, f.n * f.m,
                                   a->step, c.dp.ell, a->cs);
                rc = check_hip(hipGetLastError(), "serve checksum");
            }
            if (rc) return fail(rc);
            a->macs += (uint64_t)f.n * f.r * f.m;
        }
        // 3. wait, then retire finished requests
        rc = check_hip(hipStreamSynchronize(s), "serve tick synchronize");
        if (rc) return fail(rc);
        if (batched && sv->batch.schedule == kPersistent) {
            rc = pimm_batch_status(&sv->batch, sv->arena_base, s);
            if (rc) return fail(rc);
        }
        now = now_s(t0);
        for (Active *a : tick) a->step += 1;
        std::vector<Active *> still;
        for (Active *a : active) {
            if (a->step < steps) {
                still.push_back(a);
                continue;
            }
            const uint32_t idx = (uint32_t)(std::find_if(reqs, reqs + count, [&](const pimm_request &r) {
                                                 return r.id == a->req.id;
                                             }) - reqs);
            rc = check_hip(hipMemcpy(h_cs + 2 * idx, a->cs, 16, hipMemcpyDeviceToHost), "copy checksum");
            if (rc) return fail(rc);
            pimm_request_result &out = results[idx];
            out.id = a->req.id;
            out.arrival_s = a->req.arrival_s;
            out.admit_s = a->admit_s;
            out.done_s = now;
            out.pair_checksum = h_cs[2 * idx];
            out.sum_checksum = h_cs[2 * idx + 1];
            out.useful_macs = a->macs;
            out.steps = a->step;
            arena.release(a->off - base_off, a->bytes);
            delete a;
            ++done;
        }
        active.swap(still);
    }
    (void)hipHostFree(h_cs);
    return PIMM_OK;
}

}  // extern "C"
