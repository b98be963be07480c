// select.hip -- protocol-level choice of the block plan for a link speed.
//
// Section 3.1.1 splits matrices larger than one ciphertext into blocks and leaves
// the split open.  The split trades the server's GPU time against the bytes on the
// wire: larger blocks (mb * rb = D) shrink the weight cache and the product's
// bytes, but put more ciphertexts on the wire.  pimm_plan_select measures, on this
// device, the server's part of the protocol (input transforms, slot-wise products
// with an autotuned schedule, re-randomisation, mask and sparse reply:
// pimm_matmul_share) for each candidate plan on random inputs of the right shape,
// and picks the plan that minimises server time + wire bytes * 8 / link speed.
#include <float.h>

#include <vector>

#include "common.h"

using namespace pimm;

namespace {

template <class F>
int elapsed_ms(hipStream_t s, int reps, F &&run, double *ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    int rc = check_hip(hipEventCreate(&a), "event");
    if (!rc) rc = check_hip(hipEventCreate(&b), "event");
    if (!rc) rc = run();  // untimed first run
    if (!rc) rc = check_hip(hipEventRecord(a, s), "event record");
    for (int i = 0; !rc && i < reps; ++i) rc = run();
    if (!rc) rc = check_hip(hipEventRecord(b, s), "event record");
    if (!rc) rc = check_hip(hipEventSynchronize(b), "event synchronize");
    float t = 0.0f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&t, a, b), "event elapsed");
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    *ms = rc ? DBL_MAX : (double)t / (reps > 0 ? reps : 1);
    return rc;
}

// Device buffers of one candidate, freed on scope exit.
struct Buffers {
    std::vector<void *> p;
    ~Buffers()
    {
        for (void *q : p) (void)hipFree(q);
    }
    int alloc(void **out, size_t bytes, const char *what)
    {
        *out = nullptr;
        const int rc = check_hip(hipMalloc(out, bytes ? bytes : 8), what);
        if (!rc) p.push_back(*out);
        return rc;
    }
};

// Time the fused server step of one plan on random ciphertexts.
int time_candidate(pimm_ctx *ctx, uint32_t n, uint32_t r, uint32_t m, uint32_t d, const int64_t *W,
                   int reps, hipStream_t s, double *ms, uint64_t *wire)
{
    pimm_plan *plan = nullptr;
    int rc = pimm_plan_create(ctx, n, r, m, 0, 0, 0, d, &plan);
    if (rc) return rc;
    const pimm_plan_info &f = plan->info;
    *wire = f.ct_bytes + f.c1_bytes + f.c0s_bytes;
    const Ctx &c = *ctx;
    const size_t N = c.params.N, L = c.params.L;
    Buffers b;
    void *ct = nullptr, *acc = nullptr, *c1 = nullptr, *c0s = nullptr, *share = nullptr,
         *ws = nullptr, *pk = nullptr;
    rc = b.alloc(&ct, f.ct_bytes, "hipMalloc select ct");
    if (!rc) rc = b.alloc(&acc, f.acc_bytes, "hipMalloc select acc");
    if (!rc) rc = b.alloc(&c1, f.c1_bytes, "hipMalloc select c1");
    if (!rc) rc = b.alloc(&c0s, f.c0s_bytes, "hipMalloc select c0s");
    if (!rc) rc = b.alloc(&share, f.share_bytes, "hipMalloc select share");
    if (!rc) rc = b.alloc(&ws, f.workspace_bytes, "hipMalloc select workspace");
    if (!rc) rc = b.alloc(&pk, 2 * L * N * 8, "hipMalloc select pk");
    // Uniform residues stand for the ciphertexts and the public key (their values do not
    // change the work); the stream is keyed by a fixed seed.
    uint8_t seed[32] = {0};
    seed[0] = 0x5e;
    const Key key = make_key(seed);
    if (!rc)
        rc = launch_sample(c, 0, key, 0xf0, 0, 0, (int)(2 * f.I), 0, (int)L, ct, L * N, N, s);
    if (!rc) rc = launch_sample(c, 0, key, 0xf1, 0, 0, 2, 0, (int)L, pk, L * N, N, s);
    pimm_weights *w = nullptr;
    if (!rc) rc = pimm_weights_create(plan, W, &w, s);
    if (!rc)
        rc = pimm_plan_autotune(plan, w, (const uint64_t *)ct, (uint64_t *)acc, ws, f.workspace_bytes,
                                1, s, nullptr);
    if (!rc)
        rc = elapsed_ms(s, reps,
                        [&]() {
                            return pimm_matmul_share(plan, w, (const uint64_t *)pk, seed, 0,
                                                     (const uint64_t *)ct, (uint64_t *)c1,
                                                     (uint64_t *)c0s, (uint64_t *)share, ws,
                                                     f.workspace_bytes, s);
                        },
                        ms);
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "select synchronize");
    if (w) pimm_weights_destroy(w);
    pimm_plan_destroy(plan);
    return rc;
}

}  // namespace

extern "C" {

int pimm_plan_select(pimm_ctx *ctx, uint32_t n, uint32_t r, uint32_t m, const int64_t *W,
                     double link_bits_per_s, const uint32_t *d_candidates, uint32_t count, int reps,
                     void *stream, uint32_t *d_best, double *server_ms, uint64_t *wire_bytes)
{
    if (!ctx || !W || !d_candidates || !count || !d_best)
        return set_error(PIMM_E_ARG, "pimm_plan_select: NULL argument or no candidates");
    if (!(link_bits_per_s > 0.0)) return set_error(PIMM_E_ARG, "pimm_plan_select: link speed <= 0");
    hipStream_t s = (hipStream_t)stream;
    int rc = check_hip(hipSetDevice(ctx->device), "hipSetDevice");
    if (rc) return rc;
    double best = DBL_MAX;
    for (uint32_t i = 0; i < count; ++i) {
        double ms = 0.0;
        uint64_t wire = 0;
        rc = time_candidate(ctx, n, r, m, d_candidates[i], W, reps < 1 ? 1 : reps, s, &ms, &wire);
        if (rc) return rc;
        if (server_ms) server_ms[i] = ms;
        if (wire_bytes) wire_bytes[i] = wire;
        const double total = ms + (double)wire * 8.0 / link_bits_per_s * 1e3;
        if (total < best) {
            best = total;
            *d_best = d_candidates[i];
        }
    }
    return PIMM_OK;
}

}  // extern "C"
