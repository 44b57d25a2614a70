// hrr_api.cpp -- C ABI: context, range minimum, hierarchy, traversal,
// batched traversal and autotuner.  The serving loop is in hrr_serve.cpp.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "hrr_ctx.hpp"
#include "hrr_layout.hpp"

extern "C" hipError_t hrr_noalloc_scratch(int device, void** out);   // hrr_kernels.hip
extern "C" hipError_t hrr_launch_frontier(const hrr::Node* nodes, uint32_t n_lights, uint32_t leaf_size, float* out,
                                          hipStream_t stream);   // hrr_kernels.hip

#define HRR_EXPORT extern "C" __attribute__((visibility("default")))

// kernels (hrr_kernels.hip)
extern "C" hipError_t hrr_launch_rmq(const uint32_t* a, const uint32_t* b, const uint32_t* r, uint64_t n,
                                     uint32_t method, uint32_t* k, uint32_t* v, unsigned long long* n_bad,
                                     int n_cu, hipStream_t stream);

namespace hrr {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

hrr_status fail(hrr_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

hrr_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? HRR_E_NOMEM : HRR_E_DEVICE;
}

int ilog2_floor(uint64_t x) { return x ? 63 - __builtin_clzll(x) : 0; }

hipError_t DevBuf::ensure(size_t want) {
    if (want <= bytes) return hipSuccess;
    if (p) {
        hipError_t e = hipFree(p);
        p = nullptr;
        bytes = 0;
        if (e != hipSuccess) return e;
    }
    size_t sz = std::max<size_t>(want, 256);
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    bytes = sz;
    return hipSuccess;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

void release_scratch(LaunchScratch& S) {
    S.items.release();
    S.task_begin.release();
    S.counters.release();
    S.misc.release();
    S.spill.release();
    S.partials.release();
    S.plan.release();
    S.slack_pairs.release();
    S.slack_weights.release();
    S.order_keys.release();
    S.order_idx.release();
    S.order_hist.release();
    S.order_items.release();
    S.order_vbegin.release();
    S.queues.release();
    if (S.h_pinned) (void)hipHostFree(S.h_pinned);
    S.h_pinned = nullptr;
    S.h_pinned_n = 0;
    if (S.ev_begin) (void)hipEventDestroy(S.ev_begin);
    if (S.ev_end) (void)hipEventDestroy(S.ev_end);
    S.ev_begin = S.ev_end = nullptr;
}

void resolve_shape(hrr_ctx* ctx, const hrr_traverse_opts* opts, uint32_t n_lights, uint64_t n_eyes, uint32_t* epw,
                   uint32_t* cap, uint32_t fixed_epw) {
    uint32_t e = fixed_epw ? fixed_epw : (opts ? opts->eyes_per_wave : 0);
    uint32_t c = opts ? opts->stack_entries : 0;
    if (e == 0 || c == 0) {
        TuneVal tv{0, 0, 0, 0.f};
        bool found = false;
        {
            std::lock_guard<std::mutex> g(ctx->tune_mu);
            const TuneKey key{ilog2_floor(n_lights), ilog2_floor(n_eyes)};
            auto it = ctx->tune.find(key);
            if (it == ctx->tune.end()) {
                // nearest tuned entry of the same or a neighbouring light class
                int best = 1 << 30;
                for (auto& kv : ctx->tune) {
                    if (abs(kv.first.log_lights - key.log_lights) > 1) continue;
                    const int d = abs(kv.first.log_lights - key.log_lights) * 4 + abs(kv.first.log_eyes - key.log_eyes);
                    if (d < best) {
                        best = d;
                        tv = kv.second;
                        found = true;
                    }
                }
            } else {
                tv = it->second;
                found = true;
            }
        }
        if (e == 0) e = found ? tv.eyes_per_wave : default_eyes_per_wave(n_lights);
        // a tuned stack size only for the shape it was tuned with
        if (c == 0) c = found && tv.eyes_per_wave == e ? tv.stack_entries : default_stack_entries(e);
    }
    *epw = e;
    *cap = c;
}

void group_by_shape(hrr_ctx* ctx, const hrr_traverse_opts* opts, const std::vector<HostItem>& items, bool per_item,
                    std::vector<LaunchGroup>& out) {
    out.clear();
    auto shape_of = [&](const std::vector<size_t>& members, uint32_t* epw, uint32_t* cap, uint32_t fixed_epw) {
        uint64_t max_eyes = 0;
        uint32_t max_lights = 0;
        for (size_t k : members) {
            max_eyes = std::max<uint64_t>(max_eyes, items[k].eyes.n);
            if (items[k].h) max_lights = std::max(max_lights, items[k].h->n_lights);
        }
        resolve_shape(ctx, opts, max_lights, max_eyes, epw, cap, fixed_epw);
    };
    if (!per_item) {
        LaunchGroup g;
        g.items.resize(items.size());
        for (size_t k = 0; k < items.size(); ++k) g.items[k] = k;
        shape_of(g.items, &g.epw, &g.cap, 0);
        out.push_back(std::move(g));
        return;
    }
    std::vector<uint32_t> item_epw(items.size(), 1u);
    for (size_t k = 0; k < items.size(); ++k) {
        uint32_t kc = 0;
        if (items[k].h) resolve_shape(ctx, opts, items[k].h->n_lights, items[k].eyes.n, &item_epw[k], &kc);
        const uint32_t ke = item_epw[k];
        if (!(ke == 1 || ke == 2 || ke == 4 || ke == 8)) item_epw[k] = 1;
    }
    for (uint32_t ge : {1u, 2u, 4u, 8u}) {
        LaunchGroup g;
        for (size_t k = 0; k < items.size(); ++k)
            if (item_epw[k] == ge) g.items.push_back(k);
        if (g.items.empty()) continue;
        shape_of(g.items, &g.epw, &g.cap, ge);
        out.push_back(std::move(g));
    }
}

static void fill_stats(const unsigned long long* st, hrr_stats* out) {
    out->eyes = st[ST_EYES];
    out->pairs = st[ST_PAIRS];
    out->node_visits = st[ST_VISITS];
    out->rmq_calls = st[ST_RMQ];
    out->leaf_tests = st[ST_LEAF];
    out->spills = st[ST_SPILLS];
    out->max_stack = st[ST_MAXSTACK];
}

}  // namespace hrr

using namespace hrr;

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

HRR_EXPORT int hrr_version(void) { return 10000 * 0 + 100 * 1 + 0; }

HRR_EXPORT const char* hrr_status_string(hrr_status s) {
    switch (s) {
        case HRR_OK: return "ok";
        case HRR_E_INVALID: return "invalid argument";
        case HRR_E_NOMEM: return "out of memory";
        case HRR_E_OVERFLOW: return "output capacity exceeded";
        case HRR_E_DEVICE: return "device error";
        case HRR_E_NOTREADY: return "not ready";
        case HRR_E_CANCELLED: return "cancelled";
        case HRR_E_BUSY: return "busy";
    }
    return "unknown status";
}

HRR_EXPORT const char* hrr_last_error(const hrr_ctx*) { return g_err.c_str(); }

HRR_EXPORT hrr_status hrr_create(int device, const uint32_t* tile, hrr_ctx** out) {
    if (!out || !tile) return fail(HRR_E_INVALID, "hrr_create: null argument");
    *out = nullptr;
    int n_dev = 0;
    hipError_t e = hipGetDeviceCount(&n_dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n_dev) return fail(HRR_E_INVALID, "device %d not present (%d devices)", device, n_dev);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    hrr_ctx* c = new hrr_ctx();
    c->device = device;
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if ((e = hipMalloc((void**)&c->d_tile, 4096 * sizeof(uint32_t))) != hipSuccess) {
        delete c;
        return hip_fail(e, "tile");
    }
    if ((e = hipMemcpy(c->d_tile, tile, 4096 * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(c->d_tile);
        delete c;
        return hip_fail(e, "tile upload");
    }
    // this device's scratch of the allocation-free traversal (its address is
    // looked up once per device, with the device current)
    if ((e = hrr_noalloc_scratch(device, &c->noalloc_scratch)) != hipSuccess) {
        (void)hipFree(c->d_tile);
        delete c;
        return hip_fail(e, "scratch address of the allocation-free traversal");
    }
    // Common trailing zeros and significant bits of the tile's values: the
    // eye ordering groups eyes by the low significant bits of their shift.
    uint32_t all = 0;
    for (int q = 0; q < 4096; ++q) all |= tile[q];
    if (all) {
        c->tile_tz = (uint32_t)__builtin_ctz(all);
        c->tile_bits = 32u - (uint32_t)__builtin_clz(all) - c->tile_tz;
    }
    *out = c;
    return HRR_OK;
}

extern void hrr_server_shutdown(hrr_ctx* ctx);   // hrr_serve.cpp

HRR_EXPORT void hrr_destroy(hrr_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    hrr_server_shutdown(ctx);
    release_scratch(ctx->scratch);
    for (auto& g : ctx->group_scratch) release_scratch(g);
    if (ctx->d_tile) (void)hipFree(ctx->d_tile);
    delete ctx;
}

// ---------------------------------------------------------------------------
// range minimum
// ---------------------------------------------------------------------------

HRR_EXPORT hrr_status hrr_range_min(hrr_ctx* ctx, const uint32_t* a, const uint32_t* b, const uint32_t* r, uint64_t n,
                                    uint32_t method, uint32_t* argmin_out, uint32_t* min_out,
                                    unsigned long long* n_invalid_dev, void* stream) {
    if (!ctx) return fail(HRR_E_INVALID, "hrr_range_min: null context");
    if (method > 4) return fail(HRR_E_INVALID, "hrr_range_min: unknown method %u", method);
    if (n == 0) return HRR_OK;
    if (!a || !b || !r || !argmin_out || !min_out) return fail(HRR_E_INVALID, "hrr_range_min: null array");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = hrr_launch_rmq(a, b, r, n, method, argmin_out, min_out, n_invalid_dev, ctx->n_cu, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "range-min launch");
    return HRR_OK;
}

// ---------------------------------------------------------------------------
// hierarchy
// ---------------------------------------------------------------------------

namespace hrr {

hrr_status attach_frontier(hrr_hierarchy* h, hipStream_t stream) {
    if (!h->n_nodes) return HRR_OK;
    const size_t fb = ((size_t)kFrontierMax * kFrontierFloats + 1) * sizeof(float);
    hipError_t e = hipMalloc((void**)&h->d_frontier, fb);
    if (e == hipSuccess) e = hrr_launch_frontier(h->d_nodes, h->n_lights, h->leaf_size, h->d_frontier, stream);
    if (e != hipSuccess) return hip_fail(e, "hierarchy top");
    h->device_bytes += fb;
    return HRR_OK;
}

}  // namespace hrr

HRR_EXPORT hrr_status hrr_build_hierarchy(hrr_ctx* ctx, const float* lights_xyz, uint32_t n_lights, uint32_t leaf_arg,
                                          const float* box, hrr_hierarchy** out) {
    if (!ctx || !out) return fail(HRR_E_INVALID, "hrr_build_hierarchy: null argument");
    *out = nullptr;
    if (n_lights > 0 && !lights_xyz) return fail(HRR_E_INVALID, "hrr_build_hierarchy: null lights");
    uint32_t leaf_size, split;
    if (!parse_leaf_arg(leaf_arg, &leaf_size, &split))
        return fail(HRR_E_INVALID, "leaf_size must be in [1, 8], optionally with HRR_SPLIT_POW2");
    if (n_lights >= kMaxLights) return fail(HRR_E_INVALID, "at most %u lights", kMaxLights - 1);
    if (box) {
        for (int k = 0; k < 3; ++k)
            if (!isfinite(box[k]) || !isfinite(box[3 + k]) || !(box[3 + k] > box[k]))
                return fail(HRR_E_INVALID, "box must be finite with hi > lo");
    }
    HostHierarchy H;
    if (!build_hierarchy(lights_xyz, n_lights, leaf_size, split == HRR_SPLIT_POW2, box, H))
        return fail(HRR_E_INVALID, "non-finite light coordinate");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hrr_hierarchy* h = new hrr_hierarchy();
    h->owner = ctx;
    h->n_lights = n_lights;
    h->leaf_size = leaf_size;
    h->split = split;
    h->n_nodes = (uint32_t)H.nodes.size();
    h->depth = H.depth;
    memcpy(h->box, H.box, sizeof h->box);
    const size_t nb = std::max<size_t>(H.nodes.size(), 1) * sizeof(Node);
    const size_t lb = std::max<size_t>(n_lights, 1) * 4 * sizeof(float);
    const size_t pb = std::max<size_t>(n_lights, 1) * sizeof(uint32_t);
    std::vector<float> l4(4 * (size_t)n_lights, 0.0f);
    for (size_t i = 0; i < n_lights; ++i)
        for (int k = 0; k < 3; ++k) l4[4 * i + k] = H.sorted_xyz[3 * i + k];
    if ((e = hipMalloc((void**)&h->d_nodes, nb)) != hipSuccess || (e = hipMalloc((void**)&h->d_lights, lb)) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_perm, pb)) != hipSuccess) {
        hrr_free_hierarchy(ctx, h);
        return hip_fail(e, "hierarchy allocation");
    }
    if ((H.nodes.size() && (e = hipMemcpy(h->d_nodes, H.nodes.data(), H.nodes.size() * sizeof(Node), hipMemcpyHostToDevice)) != hipSuccess) ||
        (n_lights && (e = hipMemcpy(h->d_lights, l4.data(), l4.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) ||
        (n_lights && (e = hipMemcpy(h->d_perm, H.perm.data(), H.perm.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess)) {
        hrr_free_hierarchy(ctx, h);
        return hip_fail(e, "hierarchy upload");
    }
    h->device_bytes = nb + lb + pb;
    hrr_status st = attach_frontier(h, nullptr);
    if (st == HRR_OK && h->d_frontier &&
        (e = hipMemcpy(&h->n_frontier, h->d_frontier + (size_t)kFrontierMax * kFrontierFloats, sizeof(uint32_t),
                       hipMemcpyDeviceToHost)) != hipSuccess)
        st = hip_fail(e, "hierarchy top");
    if (st != HRR_OK) {
        hrr_free_hierarchy(ctx, h);
        return st;
    }
    h->perm = std::move(H.perm);
    h->sorted_xyz = std::move(H.sorted_xyz);
    *out = h;
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_hierarchy_get_info(const hrr_hierarchy* h, hrr_hierarchy_info* out) {
    if (!h || !out) return fail(HRR_E_INVALID, "hrr_hierarchy_get_info: null argument");
    out->n_lights = h->n_lights;
    out->leaf_size = h->leaf_size;
    out->n_nodes = h->n_nodes;
    out->depth = h->depth;
    out->device_bytes = h->device_bytes;
    memcpy(out->box, h->box, sizeof out->box);
    out->split = h->split;
    return HRR_OK;
}

// Host copies of a device-built hierarchy's order and sorted positions.
static hrr_status ensure_host_copies(const hrr_hierarchy* h) {
    if (h->host_copies) return HRR_OK;
    hipError_t e = hipSetDevice(h->owner->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const size_t n = h->n_lights;
    std::vector<float> l4(4 * n);
    h->perm.resize(n);
    if (n && ((e = hipMemcpy(h->perm.data(), h->d_perm, n * sizeof(uint32_t), hipMemcpyDeviceToHost)) != hipSuccess ||
              (e = hipMemcpy(l4.data(), h->d_lights, 4 * n * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess))
        return hip_fail(e, "hierarchy download");
    h->sorted_xyz.resize(3 * n);
    for (size_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) h->sorted_xyz[3 * i + k] = l4[4 * i + k];
    h->host_copies = true;
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_hierarchy_permutation(const hrr_hierarchy* h, uint32_t* perm_out) {
    if (!h || (!perm_out && h->n_lights)) return fail(HRR_E_INVALID, "hrr_hierarchy_permutation: null argument");
    hrr_status st = ensure_host_copies(h);
    if (st != HRR_OK) return st;
    if (h->n_lights) memcpy(perm_out, h->perm.data(), h->n_lights * sizeof(uint32_t));
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_hierarchy_sorted_lights(const hrr_hierarchy* h, float* sorted_xyz_out) {
    if (!h || (!sorted_xyz_out && h->n_lights)) return fail(HRR_E_INVALID, "hrr_hierarchy_sorted_lights: null argument");
    hrr_status st = ensure_host_copies(h);
    if (st != HRR_OK) return st;
    if (h->n_lights) memcpy(sorted_xyz_out, h->sorted_xyz.data(), 3 * (size_t)h->n_lights * sizeof(float));
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_hierarchy_records(const hrr_hierarchy* h, void* nodes_out) {
    if (!h || (!nodes_out && h->n_nodes)) return fail(HRR_E_INVALID, "hrr_hierarchy_records: null argument");
    if (!h->n_nodes) return HRR_OK;
    hipError_t e = hipSetDevice(h->owner->device);
    if (e == hipSuccess) e = hipMemcpy(nodes_out, h->d_nodes, (size_t)h->n_nodes * sizeof(Node), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hierarchy records download");
    return HRR_OK;
}

HRR_EXPORT void hrr_free_hierarchy(hrr_ctx* ctx, hrr_hierarchy* h) {
    if (!h) return;
    if (ctx) (void)hipSetDevice(ctx->device);
    if (h->d_nodes) (void)hipFree(h->d_nodes);
    if (h->d_frontier) (void)hipFree(h->d_frontier);
    if (h->d_lights) (void)hipFree(h->d_lights);
    if (h->d_perm) (void)hipFree(h->d_perm);
    delete h;
}

// ---------------------------------------------------------------------------
// traversal
// ---------------------------------------------------------------------------

// One synchronous traversal call.  With the shape left to the library
// (eyes_per_wave = 0, no override) a call of several items groups them by
// their own shape -- hierarchies of different sizes want different numbers of
// eyes per wave -- and enqueues one launch per group on `stream` (largest
// hierarchies first), each with its own scratch; otherwise one launch.
static hrr_status run_sync(hrr_ctx* ctx, const std::vector<HostItem>& items, const hrr_traverse_opts* opts,
                           uint32_t* pairs, float* weights, uint64_t* counts, hrr_stats* stats, hipStream_t stream,
                           uint32_t epw_override = 0, uint32_t cap_override = 0) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const size_t n = items.size();
    // groups of items and their launch shapes
    constexpr int kMaxGroups = 4;
    const bool per_item = n > 1 && epw_override == 0 && !(opts && opts->eyes_per_wave);
    std::vector<LaunchGroup> groups;
    group_by_shape(ctx, opts, items, per_item, groups);
    for (auto& g : groups) {
        if (epw_override) g.epw = epw_override;
        if (cap_override) g.cap = cap_override;
    }
    const int n_groups = (int)groups.size();
    LaunchScratch* scr[kMaxGroups] = {&ctx->scratch, &ctx->group_scratch[0], &ctx->group_scratch[1],
                                      &ctx->group_scratch[2]};

    const uint32_t method = opts ? opts->rmq_method : HRR_RMQ_PAPER;
    const uint32_t ns = opts && opts->n_samples > 1 ? opts->n_samples : 1;
    const uint32_t s0 = opts ? opts->psi_s0 : 0;
    const bool want_stats = opts && (opts->flags & HRR_F_STATS);
    const bool reorder = !(opts && (opts->flags & HRR_F_NO_REORDER));
    const bool timing = opts && (opts->flags & HRR_F_TIMING);
    std::vector<HostItem> sub;
    for (int g = 0; g < n_groups; ++g) {
        sub.clear();
        for (size_t k : groups[g].items) sub.push_back(items[k]);
        const hrr_status st = launch_items(ctx, *scr[g], sub, groups[g].epw, groups[g].cap, method, ns, s0,
                                           want_stats, reorder, pairs, weights, stream, timing);
        if (st != HRR_OK) {
            // launches of earlier groups may be running: let them end before
            // the caller regains its buffers
            if (g > 0) (void)hipStreamSynchronize(stream);
            return st;
        }
    }
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "traverse");

    bool overflow = false;
    uint64_t total = 0;
    uint32_t error = 0;
    unsigned long long agg[ST_N] = {};
    double kernel_ms = 0.0;
    for (int g = 0; g < n_groups; ++g) {
        LaunchScratch& S = *scr[g];
        hrr_status st = finish_items(ctx, S);
        if (st != HRR_OK) return st;
        for (size_t q = 0; q < groups[g].items.size(); ++q) {
            const size_t k = groups[g].items[q];
            counts[k] = S.counts[q];
            total += counts[k];
            if (counts[k] > items[k].out_capacity) overflow = true;
        }
        error |= S.error;
        for (int q = 0; q < ST_N; ++q) agg[q] = q == ST_MAXSTACK ? std::max(agg[q], S.stat[q]) : agg[q] + S.stat[q];
        if (timing) kernel_ms += timed_kernel_ms(S);
    }
    if (stats) {
        memset(stats, 0, sizeof *stats);
        if (want_stats) fill_stats(agg, stats);
        stats->pairs = total;
        stats->kernel_ms = kernel_ms;
    }
    if (error & ERR_SPILL_OVERFLOW)
        return fail(HRR_E_DEVICE, "traversal kernel exhausted its stack spill region");
    if (error & ERR_PARTIALS_OVERFLOW)
        return fail(HRR_E_DEVICE, "traversal kernel exhausted its partial-chunk list");
    if (error & ERR_UNFILLED)
        return fail(HRR_E_DEVICE, "output compaction left positions below the count unfilled");
    if (error) return fail(HRR_E_DEVICE, "traversal kernel reported error %u", error);
    if (overflow) return fail(HRR_E_OVERFLOW, "output capacity exceeded");
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_traverse(hrr_ctx* ctx, const hrr_hierarchy* h, const hrr_eyes* eyes, float s,
                                   const hrr_traverse_opts* opts, uint32_t* pairs_out, float* weights_out,
                                   uint64_t capacity, uint64_t* n_pairs, hrr_stats* stats, void* stream) {
    if (!ctx || !h || !eyes || !n_pairs) return fail(HRR_E_INVALID, "hrr_traverse: null argument");
    *n_pairs = 0;
    std::vector<HostItem> items{HostItem{h, *eyes, s, 0, capacity}};
    uint64_t count = 0;
    hrr_status st = run_sync(ctx, items, opts, pairs_out, weights_out, &count, stats, (hipStream_t)stream);
    if (st == HRR_OK || st == HRR_E_OVERFLOW) *n_pairs = count;
    return st;
}

HRR_EXPORT hrr_status hrr_traverse_noalloc(hrr_ctx* ctx, const hrr_hierarchy* h, const hrr_eyes* eyes, float s,
                                           const hrr_traverse_opts* opts, uint32_t* pairs_out,
                                           float* weights_out, uint64_t capacity,
                                           unsigned long long* result_dev, void* stream) {
    if (!ctx || !h || !eyes || !result_dev) return fail(HRR_E_INVALID, "hrr_traverse_noalloc: null argument");
    return launch_noalloc(ctx, h, *eyes, s, opts, pairs_out, weights_out, capacity, result_dev,
                          (hipStream_t)stream);
}

HRR_EXPORT hrr_status hrr_traverse_batched(hrr_ctx* ctx, const hrr_work_item* items, uint32_t n_items,
                                           const hrr_traverse_opts* opts, uint32_t* pairs_out, float* weights_out,
                                           uint64_t* counts_out, hrr_stats* stats, void* stream) {
    if (!ctx || !items || !counts_out) return fail(HRR_E_INVALID, "hrr_traverse_batched: null argument");
    if (n_items == 0) return HRR_OK;
    std::vector<HostItem> v;
    v.reserve(n_items);
    for (uint32_t k = 0; k < n_items; ++k)
        v.push_back(HostItem{items[k].h, items[k].eyes, items[k].s, items[k].out_offset, items[k].out_capacity});
    return run_sync(ctx, v, opts, pairs_out, weights_out, counts_out, stats, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------

HRR_EXPORT hrr_status hrr_autotune(hrr_ctx* ctx, const hrr_hierarchy* const* hs, uint32_t n_h, const hrr_eyes* eyes,
                                   float s, uint32_t max_probe_eyes, hrr_tune_result* best, void* stream) {
    if (!ctx || !hs || n_h == 0 || !eyes) return fail(HRR_E_INVALID, "hrr_autotune: null argument");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    hrr_eyes probe = *eyes;
    if (max_probe_eyes && probe.n > max_probe_eyes) probe.n = max_probe_eyes;
    // candidates in order of preference: a later one must be more than 2 %
    // faster to win, so that probe noise does not trade resident waves for a
    // larger stack (1024 entries halve the waves per SIMD of a full launch)
    static const uint32_t epws[] = {1, 2, 4, 8};
    TuneVal bestv{0, 0, 0, 1e30f};
    DevBuf out;
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "event");
    }
    hrr_status result = HRR_OK;
    uint32_t n_lights_ref = hs[0]->n_lights;
    for (uint32_t q = 0; q < n_h && result == HRR_OK; ++q) {
        const hrr_hierarchy* h = hs[q];
        if (!h || h->owner != ctx) {
            result = fail(HRR_E_INVALID, "hrr_autotune: bad hierarchy %u", q);
            break;
        }
        // count pass, then size the scratch output
        uint64_t cnt = 0;
        std::vector<HostItem> items{HostItem{h, probe, s, 0, 0}};
        hrr_status r = run_sync(ctx, items, nullptr, nullptr, nullptr, &cnt, nullptr, st, 1, default_stack_entries(1));
        if (r != HRR_OK && r != HRR_E_OVERFLOW) {
            result = r;
            break;
        }
        if ((e = out.ensure(std::max<uint64_t>(cnt, 1) * 8)) != hipSuccess) {
            result = hip_fail(e, "tuner output");
            break;
        }
        items[0].out_capacity = cnt;
        for (uint32_t epw : epws) {
            uint32_t caps[3];
            tune_stack_candidates(epw, caps);
            for (uint32_t cap : caps) {
                float ms_best = 1e30f;
                for (int rep = 0; rep < 2; ++rep) {
                    uint64_t c2 = 0;
                    (void)hipEventRecord(e0, st);
                    r = run_sync(ctx, items, nullptr, static_cast<uint32_t*>(out.p), nullptr, &c2, nullptr, st, epw, cap);
                    (void)hipEventRecord(e1, st);
                    (void)hipEventSynchronize(e1);
                    if (r != HRR_OK) break;
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ms_best = std::min(ms_best, ms);
                }
                if (r != HRR_OK) {
                    result = r;
                    break;
                }
                if (ms_best < bestv.ms * 0.98f) bestv = TuneVal{epw, cap, h->leaf_size, ms_best};
            }
            if (result != HRR_OK) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    out.release();
    if (result != HRR_OK) return result;
    {
        std::lock_guard<std::mutex> g(ctx->tune_mu);
        ctx->tune[TuneKey{ilog2_floor(n_lights_ref), ilog2_floor(eyes->n)}] = bestv;
        ctx->tune_leaf[ilog2_floor(n_lights_ref)] = bestv.leaf_size;
    }
    if (best) {
        best->eyes_per_wave = bestv.eyes_per_wave;
        best->stack_entries = bestv.stack_entries;
        best->leaf_size = bestv.leaf_size;
        best->ms = bestv.ms;
    }
    return HRR_OK;
}

HRR_EXPORT hrr_status hrr_autotune_batched(hrr_ctx* ctx, const hrr_work_item* sets, uint32_t n_sets, uint32_t n_items,
                                           hrr_tune_result* best, void* stream) {
    if (!ctx || !sets || n_sets == 0 || n_items == 0) return fail(HRR_E_INVALID, "hrr_autotune_batched: null argument");
    for (uint32_t q = 0; q < n_sets; ++q)
        for (uint32_t k = 0; k < n_items; ++k) {
            const hrr_work_item& it = sets[(size_t)q * n_items + k];
            if (!it.h || it.h->owner != ctx) return fail(HRR_E_INVALID, "hrr_autotune_batched: bad hierarchy %u/%u", q, k);
            if (it.h->n_lights != sets[k].h->n_lights || it.eyes.n != sets[k].eyes.n)
                return fail(HRR_E_INVALID, "hrr_autotune_batched: set %u item %u differs from set 0", q, k);
        }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    static const uint32_t epws[] = {1, 2, 4, 8};
    TuneVal bestv{0, 0, 0, 1e30f};
    DevBuf out;
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "event");
    }
    hrr_status result = HRR_OK;
    std::vector<HostItem> items(n_items);
    std::vector<uint64_t> cnt(n_items), c2(n_items);
    for (uint32_t q = 0; q < n_sets && result == HRR_OK; ++q) {
        for (uint32_t k = 0; k < n_items; ++k) {
            const hrr_work_item& it = sets[(size_t)q * n_items + k];
            items[k] = HostItem{it.h, it.eyes, it.s, 0, 0};
        }
        // count pass, then every item gets its slice of the scratch output
        hrr_status r = run_sync(ctx, items, nullptr, nullptr, nullptr, cnt.data(), nullptr, st, 1,
                                default_stack_entries(1));
        if (r != HRR_OK && r != HRR_E_OVERFLOW) {
            result = r;
            break;
        }
        uint64_t total = 0;
        for (uint32_t k = 0; k < n_items; ++k) {
            items[k].out_offset = total;
            items[k].out_capacity = cnt[k];
            total += cnt[k];
        }
        if ((e = out.ensure(std::max<uint64_t>(total, 1) * 8)) != hipSuccess) {
            result = hip_fail(e, "tuner output");
            break;
        }
        for (uint32_t epw : epws) {
            uint32_t caps[3];
            tune_stack_candidates(epw, caps);
            for (uint32_t cap : caps) {
                float ms_best = 1e30f;
                for (int rep = 0; rep < 2; ++rep) {
                    (void)hipEventRecord(e0, st);
                    r = run_sync(ctx, items, nullptr, static_cast<uint32_t*>(out.p), nullptr, c2.data(), nullptr, st,
                                 epw, cap);
                    (void)hipEventRecord(e1, st);
                    (void)hipEventSynchronize(e1);
                    if (r != HRR_OK) break;
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ms_best = std::min(ms_best, ms);
                }
                if (r != HRR_OK) {
                    result = r;
                    break;
                }
                if (ms_best < bestv.ms * 0.98f) bestv = TuneVal{epw, cap, items[0].h->leaf_size, ms_best};
            }
            if (result != HRR_OK) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    out.release();
    if (result != HRR_OK) return result;
    {
        std::lock_guard<std::mutex> g(ctx->tune_mu);
        for (uint32_t k = 0; k < n_items; ++k) {
            const int ll = ilog2_floor(sets[k].h->n_lights);
            ctx->tune[TuneKey{ll, ilog2_floor(sets[k].eyes.n)}] = bestv;
            ctx->tune_leaf[ll] = bestv.leaf_size;
        }
    }
    if (best) {
        best->eyes_per_wave = bestv.eyes_per_wave;
        best->stack_entries = bestv.stack_entries;
        best->leaf_size = bestv.leaf_size;
        best->ms = bestv.ms;
    }
    return HRR_OK;
}

HRR_EXPORT uint32_t hrr_tuned_leaf_size(const hrr_ctx* ctx, uint32_t n_lights) {
    if (!ctx) return 0;
    hrr_ctx* c = const_cast<hrr_ctx*>(ctx);
    std::lock_guard<std::mutex> g(c->tune_mu);
    const int key = ilog2_floor(n_lights);
    auto it = c->tune_leaf.find(key);
    if (it != c->tune_leaf.end()) return it->second;
    int best = 1 << 30;
    uint32_t v = 0;
    for (auto& kv : c->tune_leaf)
        if (abs(kv.first - key) < best) {
            best = abs(kv.first - key);
            v = kv.second;
        }
    return v;
}
