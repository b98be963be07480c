// profile.hip -- optional per-kernel timing with HIP events.
//
// When enabled, every kernel launch the library makes (or those of the
// selected classes) is bracketed by two events recorded on the launch's own
// stream, filed under the kernel's class name ("ntt_fwd", "ntt_inv", "mac",
// "sample", "encode", "decode", "mask_extract", "fused", "fc", "mod_switch").  pimm_profile_read
// waits for the recorded events, returns the number of launches and their
// summed duration, and forgets them.
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "common.h"

namespace pimm {

namespace {
struct ProfState {
    bool on = false;
    std::string select;  // ",a,b," or empty for every class
    std::mutex mu;
    std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> ev;
};
ProfState &prof()
{
    static ProfState s;
    return s;
}
}  // namespace

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), s_(s)
{
    if (!prof().on) return;
    {
        std::lock_guard<std::mutex> g(prof().mu);
        if (!prof().select.empty() &&
            prof().select.find("," + std::string(name) + ",") == std::string::npos)
            return;
    }
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) return;
    if (hipEventRecord(a_, s_) == hipSuccess) active_ = true;
}

ProfScope::~ProfScope()
{
    if (!active_) return;
    if (hipEventRecord(b_, s_) != hipSuccess) return;
    std::lock_guard<std::mutex> g(prof().mu);
    prof().ev[name_].emplace_back(a_, b_);
}

}  // namespace pimm

using namespace pimm;

extern "C" {

int pimm_profile_enable(int on)
{
    prof().on = on != 0;
    return PIMM_OK;
}

int pimm_profile_select(const char *classes)
{
    std::lock_guard<std::mutex> g(prof().mu);
    prof().select.clear();
    if (classes && *classes) {
        prof().select = ",";
        for (const char *c = classes; *c; ++c)
            if (*c != ' ') prof().select += *c;
        prof().select += ",";
    }
    return PIMM_OK;
}

int pimm_profile_read(const char *kernel, uint64_t *count, double *total_ms)
{
    if (!kernel || !count || !total_ms) return set_error(PIMM_E_ARG, "pimm_profile_read: NULL argument");
    std::vector<std::pair<hipEvent_t, hipEvent_t>> list;
    {
        std::lock_guard<std::mutex> g(prof().mu);
        auto it = prof().ev.find(kernel);
        if (it != prof().ev.end()) list.swap(it->second);
    }
    double total = 0.0;
    int rc = PIMM_OK;
    for (auto &pr : list) {
        float ms = 0.0f;
        if (!rc) rc = check_hip(hipEventSynchronize(pr.second), "profile event synchronize");
        if (!rc) rc = check_hip(hipEventElapsedTime(&ms, pr.first, pr.second), "profile elapsed");
        total += ms;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    *count = list.size();
    *total_ms = total;
    return rc;
}

}  // extern "C"
