// batch.h -- internal: the batch object shared by pimm_batch_* and the server.
#pragma once

#include <vector>

#include "common.h"

namespace pimm {

struct BatchItemDev {
    const uint64_t *ct;  // [I][2][L][N]
    uint64_t *acc;       // [O][2][L][N]
    const double *wh;    // [Wb][L][N]
    uint64_t chat_off;   // doubles into the workspace: c^ [I][2][L][N]
    uint64_t ahat_off;   // acc^ [O][2][L][N]
    uint32_t M, R, K, I, O;
    uint32_t mtiles, ktiles;    // ceil(M / G), ceil(K / KB)
    uint32_t mgroups;           // ceil(mtiles / RT), RT = mac_rt(G, KB) row tiles per unit
    uint32_t in0, mac0, out0;   // first unit of each kind
    uint32_t dep_in0, dep_mac0; // first dependency counter of each kind
};

// Counter words at the start of the workspace (uint32).
constexpr int kCtrQueue = 0;
constexpr int kCtrError = 1;
constexpr int kCtrFirstDep = 2;

enum Schedule : int { kPhased = 0, kPersistent = 1 };

}  // namespace pimm

struct pimm_batch {
    pimm::Ctx *ctx = nullptr;
    std::vector<pimm_batch_item> items;
    int G = 8;   // product rows per thread
    int KB = 1;  // product column blocks per thread
    int schedule = pimm::kPhased;
    int xcd_map = 1;
    uint32_t grid = 0;          // persistent grid size (0: from occupancy)
    uint32_t spin_limit = 1u << 22;
    pimm::BatchItemDev *d_items = nullptr;
    uint32_t n_in = 0, n_mac = 0, n_out = 0, n_dep = 0;
    uint64_t ws_bytes = 0;
    uint64_t useful_macs = 0;
    // Owner-supplied workspace offsets (doubles) of each item's c^ and acc^
    // (empty: the batch lays them out itself after the counters).
    std::vector<uint64_t> fixed_chat, fixed_ahat;
    size_t cap = 0;                          // capacity of d_items (items)
    pimm::BatchItemDev *h_items = nullptr;   // pinned staging for asynchronous uploads
};

namespace pimm {
// Rebuild the item table; async uploads use pinned staging on `s` (the caller
// must not have a run of this batch in flight).
int batch_rebuild(pimm_batch *b, bool async, hipStream_t s);
// with_out = false stops after the products: each item's acc^ stays in its
// workspace (summed over the inner blocks, in NTT form) and its acc is not written.
int batch_run(const pimm_batch *b, void *ws, hipStream_t s, bool with_out = true);
}  // namespace pimm


