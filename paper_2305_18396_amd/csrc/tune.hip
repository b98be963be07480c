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

int pimm_plan_set_tuning(pimm_plan *plan, int mac_rows, int splits)
{
    if (!plan) return set_error(PIMM_E_ARG, "pimm_plan_set_tuning: NULL plan");
    if (mac_rows != 4 && mac_rows != 8 && mac_rows != 16)
        return set_error(PIMM_E_ARG, "mac_rows %d is not 4, 8 or 16", mac_rows);
    if (splits != 1 && splits != 2 && splits != 4)
        return set_error(PIMM_E_ARG, "splits %d is not 1, 2 or 4", splits);
    plan->mac_rows = mac_rows;
    plan->splits = splits;
    return PIMM_OK;
}

int pimm_plan_get_tuning(const pimm_plan *plan, int *mac_rows, int *splits)
{
    if (!plan || !mac_rows || !splits) return set_error(PIMM_E_ARG, "pimm_plan_get_tuning: NULL argument");
    *mac_rows = plan->mac_rows;
    *splits = plan->splits;
    return PIMM_OK;
}

int pimm_plan_autotune(pimm_plan *plan, const pimm_weights *w, const uint64_t *ct, uint64_t *acc,
                       void *ws, size_t ws_bytes, int reps, void *stream, double *best_ms)
{
    if (!plan || !w || !ct || !acc) return set_error(PIMM_E_ARG, "pimm_plan_autotune: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const int rows[3] = {4, 8, 16}, splits[3] = {1, 2, 4};
    double best = DBL_MAX;
    int bg = plan->mac_rows, bs = plan->splits;
    for (int g : rows)
        for (int sp : splits) {
            plan->mac_rows = g;
            plan->splits = sp;
            double ms = 0;
            int rc = time_ms(s, reps,
                             [&]() { return pimm_matmul(plan, w, ct, acc, ws, ws_bytes, stream); }, &ms);
            if (rc) {
                plan->mac_rows = bg;
                plan->splits = bs;
                return rc;
            }
            if (ms < best) {
                best = ms;
                bg = g;
                bs = sp;
            }
        }
    plan->mac_rows = bg;
    plan->splits = bs;
    if (best_ms) *best_ms = best;
    return PIMM_OK;
}

int pimm_batch_autotune(pimm_batch *b, void *ws, size_t ws_bytes, int reps, void *stream,
                        double *best_ms)
{
    if (!b) return set_error(PIMM_E_ARG, "pimm_batch_autotune: NULL batch");
    hipStream_t s = (hipStream_t)stream;
    struct Cand {
        int sched, g, xcd;
    };
    const Cand cands[] = {{kPhased, 8, 1}, {kPhased, 8, 0}, {kPhased, 4, 1}, {kPhased, 16, 1},
                          {kPersistent, 8, 1}, {kPersistent, 16, 1}};
    double best = DBL_MAX;
    Cand bc = {b->schedule, b->G, b->xcd_map};
    for (const Cand &c : cands) {
        int rc = pimm_batch_set_schedule(b, c.sched, c.g, c.xcd, 0);
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
    return pimm_batch_set_schedule(b, bc.sched, bc.g, bc.xcd, 0);
}

}  // extern "C"
