// hrr_ctx.hpp -- private state behind the C ABI (host side only).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hrr.h"
#include "hrr_build.hpp"
#include "hrr_types.hpp"

struct hrr_hierarchy {
    hrr_ctx* owner = nullptr;
    uint32_t n_lights = 0, leaf_size = 1, n_nodes = 0, depth = 0;
    uint32_t split = HRR_SPLIT_RADIX;
    float box[6] = {0, 0, 0, 0, 0, 0};
    hrr::Node* d_nodes = nullptr;
    float* d_frontier = nullptr;      // kFrontierMax entries of kFrontierFloats, then the entry count
    uint32_t n_frontier = 0;
    float* d_lights = nullptr;       // float4 per light
    uint32_t* d_perm = nullptr;
    // host copies (filled on demand for hierarchies built on the device)
    mutable std::vector<uint32_t> perm;
    mutable std::vector<float> sorted_xyz;
    mutable bool host_copies = true;
    uint64_t device_bytes = 0;
};

namespace hrr {

// Device buffer that only grows.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want);
    void release();
};

struct TuneKey {
    int log_lights, log_eyes;
    bool operator<(const TuneKey& o) const {
        return log_lights != o.log_lights ? log_lights < o.log_lights : log_eyes < o.log_eyes;
    }
};

struct TuneVal {
    uint32_t eyes_per_wave, stack_entries, leaf_size;
    float ms;
};

// Host description of one traversal item before it becomes an ItemDesc.
struct HostItem {
    const hrr_hierarchy* h;
    hrr_eyes eyes;
    float s;
    uint64_t out_offset, out_capacity;
};

// Host copy of one item's output layout in a launch.
struct ItemMeta {
    unsigned long long out_offset, capacity, slack, slack_off, partial_off, plan_off;
    uint32_t partial_cap, chunk_shift;
};

// Per-launch device scratch: one set per stream slot so that concurrent
// launches (the server) never share queue heads or counters.
struct LaunchScratch {
    DevBuf items, task_begin, counters, misc, spill, partials, plan, slack_pairs, slack_weights;
    DevBuf order_keys, order_idx, order_hist, order_items, order_vbegin, queues;
    std::vector<ItemDesc> h_items;
    std::vector<uint32_t> h_task_begin;
    std::vector<unsigned long long> h_partial_off;   // per item, first entry in `partials`
    unsigned long long* h_pinned = nullptr;          // pinned staging / readback area
    size_t h_pinned_n = 0;
    std::vector<ItemMeta> meta;
    size_t n_items = 0;
    bool with_weights = false;
    bool stats = false;
    // results of finish_items
    std::vector<unsigned long long> counts;    // true pairs per item
    std::vector<unsigned long long> stored;    // valid pairs stored at the front of each slice
    uint32_t error = 0;
    unsigned long long stat[ST_N] = {0};
    // optional events around the traversal kernel (created on first use)
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
    bool timed = false;
};

struct Server;

}  // namespace hrr

struct hrr_ctx {
    int device = 0;
    int n_cu = 256;
    uint32_t* d_tile = nullptr;
    uint32_t tile_tz = 32, tile_bits = 0;   // shared trailing zeros / significant bits of the tile values
    hrr::LaunchScratch scratch;   // scratch of the synchronous entry points
    hrr::LaunchScratch group_scratch[3];   // further launches of one batched call (items grouped by shape)
    std::mutex tune_mu;
    std::map<hrr::TuneKey, hrr::TuneVal> tune;
    std::map<int, uint32_t> tune_leaf;   // log2 lights -> leaf size
    hrr::Server* server = nullptr;
    std::mutex server_mu;
    void* noalloc_scratch = nullptr;   // this device's scratch of hrr_traverse_noalloc
};

namespace hrr {

void set_error(const char* fmt, ...);
hrr_status fail(hrr_status st, const char* fmt, ...);
hrr_status hip_fail(hipError_t e, const char* what);

int ilog2_floor(uint64_t x);

// Leaf size and split rule of a build's leaf_size argument; false if a bit
// outside the leaf size (1..8) and HRR_SPLIT_POW2 is set.
inline bool parse_leaf_arg(uint32_t arg, uint32_t* leaf, uint32_t* split) {
    *leaf = arg & 0xFFu;
    *split = arg & HRR_SPLIT_POW2;
    return (arg & ~(0xFFu | HRR_SPLIT_POW2)) == 0 && *leaf >= 1 && *leaf <= 8;
}

// Resolve launch parameters (eyes per wave, stack entries) from options, the
// tuner (an entry of the same or a neighbouring light class) and the built-in
// rule default_eyes_per_wave().
// With fixed_epw != 0 the eyes per wave are fixed and only the stack size is
// resolved (a tuned stack size applies only to the shape it was tuned with).
void resolve_shape(hrr_ctx* ctx, const hrr_traverse_opts* opts, uint32_t n_lights, uint64_t n_eyes,
                   uint32_t* epw, uint32_t* cap, uint32_t fixed_epw = 0);

// The launches of a call of several items.  With per_item, the items are
// grouped by the eyes per wave of their own shape (tuned or by hierarchy
// size; groups in the order 1, 2, 4, 8 eyes per wave, i.e. largest
// hierarchies first) and every group takes the stack size resolved for its
// own largest hierarchy and eye set; otherwise one group holds every item
// with the shape resolved for the largest of them.  Items without a
// hierarchy go to the one-eye-per-wave group (their launch rejects them).
struct LaunchGroup {
    std::vector<size_t> items;
    uint32_t epw = 1, cap = 512;
};
void group_by_shape(hrr_ctx* ctx, const hrr_traverse_opts* opts, const std::vector<HostItem>& items, bool per_item,
                    std::vector<LaunchGroup>& out);

// Enqueue one persistent launch of a set of items on `stream` with scratch
// `S`: the eye order, the traversal, the compaction that makes every item's
// stored pairs dense (on the device), and the readback of the counters.
// After the stream has been synchronised, finish_items() fills S.counts /
// S.stored / S.error / S.stat from that readback.
hrr_status launch_items(hrr_ctx* ctx, LaunchScratch& S, const std::vector<HostItem>& items, uint32_t epw,
                        uint32_t cap, uint32_t method, uint32_t n_samples, uint32_t psi_s0, bool stats,
                        bool reorder, uint32_t* pairs, float* weights, hipStream_t stream, bool timing = false);
// Duration of the last timed traversal kernel of S (after the stream has synchronised), ms.
double timed_kernel_ms(LaunchScratch& S);
hrr_status finish_items(hrr_ctx* ctx, LaunchScratch& S);

void release_scratch(LaunchScratch& S);

// Allocate h->d_frontier and enqueue the computation of the hierarchy's top
// (the entry count lands in the table's last word) on `stream`.
hrr_status attach_frontier(hrr_hierarchy* h, hipStream_t stream);

// The allocation-free traversal of one eye set (hrr_traverse_noalloc): every
// launch on `stream`, nothing allocated, nothing read back.
hrr_status launch_noalloc(hrr_ctx* ctx, const hrr_hierarchy* h, const hrr_eyes& eyes, float s,
                          const hrr_traverse_opts* opts, uint32_t* pairs, float* weights, uint64_t capacity,
                          unsigned long long* result_dev, hipStream_t stream);

}  // namespace hrr
