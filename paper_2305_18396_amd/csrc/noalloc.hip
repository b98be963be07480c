// noalloc.hip -- the fused server step with library-held scratch, for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops that must not call the allocator, harnesses that forbid it).
//
// pimm_matmul_share needs a workspace of fused_workspace_bytes(plan) for the
// inputs in the product's layout, the accumulators in NTT form and the re-randomisation
// terms.  pimm_matmul_share_noalloc takes that workspace from `scratch`, an
// array in the code object's static device data: every device the library
// runs on holds one copy of it (kNoallocScratchBytes) from the loading of the
// code object until the process ends.  In host code the name `scratch` is a
// host-side stand-in, not a device address; the device address of each
// device's copy comes from hipGetSymbolAddress, taken once per device when
// the first context on that device is created (with that device current) and
// kept per device.  Host code uses only that address.
#include <mutex>

#include "common.h"

namespace pimm {

constexpr uint64_t kNoallocScratchBytes = PIMM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace pimm

static __device__ __align__(256) unsigned char scratch[pimm::kNoallocScratchBytes];

namespace pimm {

namespace {
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];
}  // namespace

// Called by pimm_ctx_create with `device` current.
int bind_noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return set_error(PIMM_E_ARG, "device %d is outside the %d the library tracks", device,
                         kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_addr[device]) return PIMM_OK;
    void *p = nullptr;
    const int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                             "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    if (!p) return set_error(PIMM_E_DEVICE, "hipGetSymbolAddress(scratch) gave no address");
    g_scratch_addr[device] = p;
    return PIMM_OK;
}

static void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_addr[device];
}

}  // namespace pimm

using namespace pimm;

extern "C" {

int pimm_matmul_share_noalloc(const pimm_plan *plan, const pimm_weights *w, const uint64_t *pk,
                              const uint8_t seed[32], uint32_t op_id, const uint64_t *ct,
                              uint64_t *c1, uint64_t *c0s, uint64_t *server_share, void *stream)
{
    if (!plan || !w || !seed || !ct || !c1 || !c0s || !server_share)
        return set_error(PIMM_E_ARG, "pimm_matmul_share_noalloc: NULL argument");
    const Ctx &c = *plan->ctx;
    const uint64_t need = fused_workspace_bytes(c, plan->info);
    if (need > kNoallocScratchBytes)
        return set_error(PIMM_E_WORKSPACE,
                         "pimm_matmul_share_noalloc: this plan needs %llu bytes of scratch, more "
                         "than the %llu bytes the library holds per device; call "
                         "pimm_matmul_share with a workspace instead",
                         (unsigned long long)need, (unsigned long long)kNoallocScratchBytes);
    void *ws = noalloc_scratch(c.device);
    if (!ws)
        return set_error(PIMM_E_DEVICE,
                         "pimm_matmul_share_noalloc: no scratch address for device %d", c.device);
    // Every kernel of the fused step writes the scratch words it reads (the input
    // transform also zeroes the accumulators), so the last call's contents do not matter.
    return pimm_matmul_share(plan, w, pk, seed, op_id, ct, c1, c0s, server_share, ws,
                             (size_t)kNoallocScratchBytes, stream);
}

}  // extern "C"
