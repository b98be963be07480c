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

// Items that share one weight cache line up their column blocks for the phased
// product, so that a weight word is read once per column tile of the whole
// group rather than once per item.  Column j of a group is block kb of item.
struct BatchColDev {
    uint32_t item, kb;
};
struct BatchGroupDev {
    const double *wh;  // the shared weight cache
    uint32_t M, R;
    uint32_t mtiles, mgroups;  // ceil(M / G), ceil(mtiles / RT)
    uint32_t ncols, ktiles;    // sum of the items' K, ceil(ncols / KB)
    uint32_t col0, mac0;       // first column, first phased product unit
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
    // Device tables, one allocation: items, then weight groups, then group columns.
    pimm::BatchItemDev *d_items = nullptr;
    pimm::BatchGroupDev *d_groups = nullptr;
    pimm::BatchColDev *d_cols = nullptr;
    uint32_t n_groups = 0;
    uint32_t n_in = 0, n_mac = 0, n_out = 0, n_dep = 0;
    uint32_t n_mac_grouped = 0;  // product units of the phased schedule
    uint64_t ws_bytes = 0;
    uint64_t useful_macs = 0;
    // Owner-supplied workspace offsets (doubles) of each item's c^ and acc^
    // (empty: the batch lays them out itself after the counters).
    std::vector<uint64_t> fixed_chat, fixed_ahat;
    uint8_t *d_tab = nullptr;  // the table allocation
    uint8_t *h_tab = nullptr;  // pinned staging for asynchronous uploads
    size_t tab_cap = 0, h_cap = 0;
};

namespace pimm {
// Rebuild the item table; async uploads use pinned staging on `s` (the caller
// must not have a run of this batch in flight).
int batch_rebuild(pimm_batch *b, bool async, hipStream_t s);
// with_out = false stops after the products: each item's acc^ stays in its
// workspace (summed over the inner blocks, in NTT form) and its acc is not written.
int batch_run(const pimm_batch *b, void *ws, hipStream_t s, bool with_out = true);
void batch_free_tables(pimm_batch *b);
}  // namespace pimm


