// tune.hip -- a small native autotuner for the slot-wise product's schedule.
//
// Candidates are timed on the caller's real buffers with HIP events recorded on
// the caller's stream (one untimed run, then `reps` timed runs each), and the
// fastest is kept on the plan or batch.  The outputs of every candidate are the
// same bytes (the schedule only changes how the work is split), so tuning on
// live data is harmless.
#include <float.h>

#include "batch.h"
#include "common.h"
#include "mac.h"
#include "mfma.h"

using namespace pimm;

namespace {

template <class F>
int time_ms(hipStream_t s, int reps, F &&run, double *ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    int rc = check_hip(hipEventCreate(&a), "event");
    if (!rc) rc = check_hip(hipEventCreate(&b), "event");
    if (!rc) rc = run();
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

}  // namespace

extern "C" {

int pimm_plan_set_tuning(pimm_plan *plan, int mac_rows, int mac_cols, int waves)
{
    if (!plan) return set_error(PIMM_E_ARG, "pimm_plan_set_tuning: NULL plan");
    if (mac_rows == 0 && mac_cols == 0 && waves == 0) {  // the matrix-core product
        if (!mfma_eligible(plan->info))
            return set_error(PIMM_E_UNSUPPORTED,
                             "the matrix-core product needs at most 64 inner blocks and at least 8 "
                             "column blocks (plan: R = %u, K = %u)",
                             plan->info.R, plan->info.K);
        plan->mac_rows = plan->mac_cols = plan->waves = 0;
        return PIMM_OK;
    }
    if (!mac_shape_ok(mac_rows, mac_cols))
        return set_error(PIMM_E_ARG, "product tile %d rows x %d column blocks is not built",
                         mac_rows, mac_cols);
    if (plan->info.groups > 1 && mac_cols != 1)
        return set_error(PIMM_E_UNSUPPORTED, "grouped plans take product tiles 4x1, 8x1 or 16x1");
    if (waves != 1 && waves != 2 && waves != 4)
        return set_error(PIMM_E_ARG, "waves %d is not 1, 2 or 4", waves);
    plan->mac_rows = mac_rows;
    plan->mac_cols = mac_cols;
    plan->waves = waves;
    return PIMM_OK;
}

int pimm_plan_get_tuning(const pimm_plan *plan, int *mac_rows, int *mac_cols, int *waves)
{
    if (!plan || !mac_rows || !mac_cols || !waves)
        return set_error(PIMM_E_ARG, "pimm_plan_get_tuning: NULL argument");
    *mac_rows = plan->mac_rows;
    *mac_cols = plan->mac_cols;
    *waves = plan->waves;
    return PIMM_OK;
}

int pimm_plan_autotune(pimm_plan *plan, const pimm_weights *w, const uint64_t *ct, uint64_t *acc,
                       void *ws, size_t ws_bytes, int reps, void *stream, double *best_ms)
{
    if (!plan || !w || !ct || !acc) return set_error(PIMM_E_ARG, "pimm_plan_autotune: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    struct Shape {
        int g, kb;
    };
    const Shape shapes[] = {{4, 1}, {8, 1}, {16, 1}, {4, 2}, {8, 2}, {16, 2},
                            {2, 4}, {4, 4}, {8, 4}, {2, 8}, {4, 8}};
    const int waves[3] = {1, 2, 4};
    const int K = (int)plan->info.K;
    double best = DBL_MAX;
    int bg = plan->mac_rows, bk = plan->mac_cols, bw = plan->waves;
    const bool grouped = plan->info.groups > 1;
    for (const Shape &sh : shapes) {
        // Column blocking only pays when there are columns to share a weight word.
        if (sh.kb > 1 && sh.kb > 2 * K - 1) continue;
        if (grouped && sh.kb != 1) continue;  // the grouped product's tiles
        for (int wv : waves) {
            if (grouped && wv != 1) continue;  // one workgroup per tile: no grid to size
            plan->mac_rows = sh.g;
            plan->mac_cols = sh.kb;
            plan->waves = wv;
            double ms = 0;
            int rc = time_ms(s, reps,
                             [&]() { return pimm_matmul(plan, w, ct, acc, ws, ws_bytes, stream); }, &ms);
            if (rc) {
                plan->mac_rows = bg;
                plan->mac_cols = bk;
                plan->waves = bw;
                return rc;
            }
            if (ms < best) {
                best = ms;
                bg = sh.g;
                bk = sh.kb;
                bw = wv;
            }
        }
    }
    if (w->d_w_dig && mfma_eligible(plan->info)) {
        plan->mac_rows = plan->mac_cols = plan->waves = 0;
        double ms = 0;
        int rc = time_ms(s, reps,
                         [&]() { return pimm_matmul(plan, w, ct, acc, ws, ws_bytes, stream); }, &ms);
        if (rc) {
            plan->mac_rows = bg;
            plan->mac_cols = bk;
            plan->waves = bw;
            return rc;
        }
        if (ms < best) {
            best = ms;
            bg = bk = bw = 0;
        }
    }
    plan->mac_rows = bg;
    plan->mac_cols = bk;
    plan->waves = bw;
    if (best_ms) *best_ms = best;
    return PIMM_OK;
}

int pimm_batch_autotune(pimm_batch *b, void *ws, size_t ws_bytes, int reps, void *stream,
                        double *best_ms)
{
    if (!b) return set_error(PIMM_E_ARG, "pimm_batch_autotune: NULL batch");
    hipStream_t s = (hipStream_t)stream;
    struct Cand {
        int sched, g, kb, xcd;
    };
    const Cand cands[] = {{kPhased, 8, 1, 1},      {kPhased, 8, 1, 0},      {kPhased, 16, 1, 1},
                          {kPhased, 8, 2, 1},      {kPhased, 16, 2, 1},     {kPhased, 4, 4, 1},
                          {kPhased, 8, 4, 1},      {kPhased, 8, 4, 0},      {kPhased, 4, 8, 1},
                          {kPhased, 2, 8, 1},      {kPersistent, 8, 1, 1},
                          {kPersistent, 16, 2, 1}, {kPersistent, 4, 4, 1}, {kPersistent, 8, 4, 1}};
    double best = DBL_MAX;
    Cand bc = {b->schedule, b->G, b->KB, b->xcd_map};
    for (const Cand &c : cands) {
        int rc = pimm_batch_set_schedule(b, c.sched, c.g, c.kb, c.xcd, 0);
        if (rc) return rc;
        if (b->ws_bytes > ws_bytes) continue;
        double ms = 0;
        rc = time_ms(s, reps, [&]() { return pimm_batch_matmul(b, ws, ws_bytes, stream); }, &ms);
        if (!rc && c.sched == kPersistent) rc = pimm_batch_status(b, ws, stream);
        if (rc) return rc;
        if (ms < best) {
            best = ms;
            bc = c;
        }
    }
    if (best_ms) *best_ms = best;
    return pimm_batch_set_schedule(b, bc.sched, bc.g, bc.kb, bc.xcd, 0);
}

}  // extern "C"
