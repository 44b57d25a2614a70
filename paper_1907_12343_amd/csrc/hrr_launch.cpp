// hrr_launch.cpp -- host side of one persistent traversal launch: work
// queue and item table set-up, output chunk sizing, and the hole filling that
// makes each item's pairs dense after the kernel.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "hrr_ctx.hpp"
#include "hrr_layout.hpp"

extern "C" hipError_t hrr_launch_traverse(const hrr::TravArgs* A, uint32_t eyes_per_wave, uint32_t method,
                                          int stats, int with_weights, uint32_t blocks, hipStream_t stream);
extern "C" size_t hrr_trav_lds_per_wave(uint32_t stack_cap, uint32_t eyes_per_wave);
extern "C" size_t hrr_trav_lds_per_block(uint32_t n_items, size_t lds_per_wave);
extern "C" hipError_t hrr_traverse_occupancy(uint32_t eyes_per_wave, uint32_t method, int stats, int with_weights,
                                             size_t lds_per_block, int* blocks_per_cu);
extern "C" hipError_t hrr_launch_order(const hrr::OrderItem* items, const uint32_t* vbegin, uint32_t n_items,
                                       uint32_t total, uint32_t bits, uint32_t rbits, const uint32_t* tile,
                                       uint32_t tile_tz, uint32_t* keys, uint32_t* hist, uint32_t* order, int n_cu,
                                       hipStream_t stream);
extern "C" hipError_t hrr_launch_compact(const hrr::ItemDesc* items, uint32_t n_items, uint32_t* error,
                                         hipStream_t stream);
extern "C" hipError_t hrr_launch_noalloc_setup(const hrr::ItemDesc* D, uint32_t n_tasks, void* base,
                                               hipStream_t stream);
extern "C" hipError_t hrr_launch_noalloc_finish(const void* base, unsigned long long* result, hipStream_t stream);

namespace hrr {

namespace {

// Bounds of the kernel's product-form keep test for one s (the derivation is
// beside rr_test in the kernels): t_cull >= s 2^32 (1 + 2^-18) and
// t_keep <= s 2^32 (1 - 2^-18), both rounded outward to binary32; the test is
// used for d2 <= d2_fast = s 2^60 (at most 2^80) only, and never for an s
// outside [2^-60, 2^60] (then d2_fast = 0 sends every test to the IEEE path).
void product_test_bounds(float s, float* t_cull, float* t_keep, float* d2_fast) {
    const double S = (double)s * 4294967296.0;
    float hi = (float)(S * (1.0 + 0x1p-18));
    if ((double)hi < S * (1.0 + 0x1p-18)) hi = nextafterf(hi, INFINITY);
    float lo = (float)(S * (1.0 - 0x1p-18));
    if ((double)lo > S * (1.0 - 0x1p-18)) lo = nextafterf(lo, 0.0f);
    *t_cull = hi;
    *t_keep = lo;
    *d2_fast = (s >= 0x1p-60f && s <= 0x1p60f) ? std::min((float)((double)s * 0x1p60), 0x1p80f) : 0.0f;
}

}  // namespace

hrr_status launch_items(hrr_ctx* ctx, LaunchScratch& S, const std::vector<HostItem>& items, uint32_t epw,
                        uint32_t cap, uint32_t method, uint32_t n_samples, uint32_t psi_s0, bool stats,
                        bool reorder, uint32_t* pairs, float* weights, hipStream_t stream, bool timing) {
    const size_t n = items.size();
    S.timed = false;
    if (n == 0 || n > kMaxItemsPerLaunch)
        return fail(HRR_E_INVALID, "items per launch must be in [1, %u]", kMaxItemsPerLaunch);
    if (!(epw == 1 || epw == 2 || epw == 4 || epw == 8))
        return fail(HRR_E_INVALID, "eyes_per_wave must be 1, 2, 4 or 8");
    if (cap % 64 != 0 || cap < 192 || cap > 4096)
        return fail(HRR_E_INVALID, "stack_entries must be a multiple of 64 in [192, 4096]");
    if (method > 5) return fail(HRR_E_INVALID, "unknown rmq method %u", method);
    if (n_samples == 0) n_samples = 1;
    const int with_w = weights != nullptr;

    // ---- grid: persistent waves, as many as stay resident ----
    const size_t lds_wave = hrr_trav_lds_per_wave(cap, epw);
    const size_t lds_block = hrr_trav_lds_per_block((uint32_t)n, lds_wave);
    int bpc = 0;
    hipError_t e;
    if ((e = hrr_traverse_occupancy(epw, method, stats, with_w, lds_block, &bpc)) != hipSuccess)
        return hip_fail(e, "occupancy");
    if (bpc <= 0) return fail(HRR_E_INVALID, "stack of %u entries does not fit in LDS", cap);

    std::vector<uint64_t> tasks_of(n);
    uint64_t tasks = 0;
    uint32_t dmax = 0;
    for (size_t k = 0; k < n; ++k) {
        const HostItem& it = items[k];
        const hrr_hierarchy* h = it.h;
        if (!h) return fail(HRR_E_INVALID, "item %zu: null hierarchy", k);
        if (h->owner != ctx) return fail(HRR_E_INVALID, "item %zu: hierarchy belongs to another context", k);
        if (!(it.s > 0.0f) || !isfinite(it.s)) return fail(HRR_E_INVALID, "item %zu: s must be finite and > 0", k);
        if (it.eyes.n > 0 && !it.eyes.xyz) return fail(HRR_E_INVALID, "item %zu: null eye positions", k);
        if (it.eyes.width == 0) return fail(HRR_E_INVALID, "item %zu: width must be >= 1", k);
        if (it.out_capacity > 0 && !pairs) return fail(HRR_E_INVALID, "item %zu: null pairs buffer", k);
        const uint64_t nv = (uint64_t)it.eyes.n * n_samples;
        if (nv > 0xFFFFFFFFull) return fail(HRR_E_INVALID, "item %zu: eyes x samples exceeds 2^32 - 1", k);
        tasks_of[k] = h->n_lights ? (nv + epw - 1) / epw : 0;
        tasks += tasks_of[k];
        if (tasks > 0xFFFFFFF0ull) return fail(HRR_E_INVALID, "too many tasks in one launch");
        dmax = std::max(dmax, h->depth);
    }
    const uint64_t need_blocks = (tasks + kWavesPerBlock - 1) / kWavesPerBlock;
    const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)ctx->n_cu * bpc, need_blocks));
    const uint64_t waves = (uint64_t)blocks * kWavesPerBlock;

    // ---- per-item output chunks, slack and partial lists ----
    std::vector<ItemMeta>& M = S.meta;
    M.assign(n, ItemMeta{});
    unsigned long long slack_total = 0, partial_total = 0, plan_total = 0;
    // Queue layout and the partial-chunk bound (hrr_layout.hpp).  Every
    // allocated chunk other than the partly filled ones is full, so the pairs
    // stored past the capacity (slack) and the holes below it are bounded by
    // partial_cap chunks each; a slack of twice that lets the compaction fill
    // every hole below min(count, capacity).
    const uint32_t il_shift = queue_interleave_shift(n, tasks);
    const uint64_t leaves_per_wave = departures_per_wave(n, il_shift);
    for (size_t k = 0; k < n; ++k) {
        const uint64_t wk = std::max<uint64_t>(1, std::min<uint64_t>(waves, tasks_of[k]));
        const uint64_t pk = std::max<uint64_t>(1, std::min<uint64_t>(leaves_per_wave * waves, tasks_of[k]));
        const unsigned long long capk = items[k].out_capacity;
        const uint32_t shift = chunk_shift_for(capk, wk);
        ItemMeta& m = M[k];
        m.out_offset = items[k].out_offset;
        m.capacity = capk;
        m.chunk_shift = shift;
        m.slack = capk ? 2ull * pk << shift : 0ull;
        m.slack_off = slack_total;
        slack_total += m.slack;
        m.partial_cap = (uint32_t)pk;
        m.partial_off = partial_total;
        partial_total += pk;
        m.plan_off = plan_total;
        plan_total += 3 * pk + 4;   // hole prefixes pk + 1, data prefixes 2 pk + 3
    }

    // ---- eye processing order: counting sort by (item, Morton cell) ----
    std::vector<uint32_t> vbegin(n + 1, 0);
    uint64_t vtotal = 0;
    for (size_t k = 0; k < n; ++k) {
        vbegin[k] = (uint32_t)std::min<uint64_t>(vtotal, 0xFFFFFFFFull);
        vtotal += items[k].h->n_lights ? (uint64_t)items[k].eyes.n * n_samples : 0ull;
    }
    vbegin[n] = (uint32_t)std::min<uint64_t>(vtotal, 0xFFFFFFFFull);
    // eye order key (hrr_layout.hpp), for launches with enough work to gain from it
    double order_cost = 0.0;
    for (size_t k = 0; k < n; ++k)
        order_cost += (double)tasks_of[k] * epw * pow((double)std::max<uint32_t>(items[k].h->n_lights, 1u), 0.6);
    uint32_t bits = 0, rbits = 0;
    if (reorder && order_pays(order_cost)) order_key_bits(n, vtotal, ctx->tile_bits, &bits, &rbits);
    const bool ordered = bits > 0;
    std::vector<OrderItem> oitems;
    if (ordered) {
        oitems.resize(n);
        for (size_t k = 0; k < n; ++k) {
            const hrr_hierarchy* h = items[k].h;
            OrderItem& o = oitems[k];
            o.eyes = items[k].eyes.xyz;
            o.n_samples = n_samples;
            o.width = items[k].eyes.width;
            o.pixel_base = items[k].eyes.pixel_base;
            o.pad = 0;
            for (int q = 0; q < 3; ++q) {
                const float ext = h->box[3 + q] - h->box[q];
                o.lo[q] = h->box[q];
                o.scale[q] = ext > 0.0f ? (float)(1u << bits) / ext : 0.0f;
            }
        }
        if ((e = S.order_keys.ensure(vtotal * sizeof(uint32_t))) != hipSuccess) return hip_fail(e, "order keys");
        if ((e = S.order_idx.ensure(vtotal * sizeof(uint32_t))) != hipSuccess) return hip_fail(e, "eye order");
        if ((e = S.order_hist.ensure((((size_t)n << (3 * bits + rbits)) + 1024) * sizeof(uint32_t))) != hipSuccess)
            return hip_fail(e, "order histogram");
        if ((e = S.order_items.ensure(n * sizeof(OrderItem))) != hipSuccess) return hip_fail(e, "order items");
        if ((e = S.order_vbegin.ensure((n + 1) * sizeof(uint32_t))) != hipSuccess) return hip_fail(e, "order offsets");
    }
    if ((e = S.queues.ensure(kQueues * kQueueStride * sizeof(uint32_t))) != hipSuccess) return hip_fail(e, "queues");

    S.n_items = n;
    S.with_weights = with_w;
    S.stats = stats;
    if ((e = S.counters.ensure(n * CNT_STRIDE * sizeof(unsigned long long))) != hipSuccess) return hip_fail(e, "counters");
    if ((e = S.misc.ensure(16 * sizeof(unsigned long long))) != hipSuccess) return hip_fail(e, "misc");
    if ((e = S.partials.ensure(std::max<unsigned long long>(partial_total, 1) * 2 * sizeof(unsigned long long))) != hipSuccess)
        return hip_fail(e, "partial-chunk list");
    if ((e = S.plan.ensure(std::max<unsigned long long>(plan_total, 1) * sizeof(unsigned long long))) != hipSuccess)
        return hip_fail(e, "compaction plan");
    if ((e = S.slack_pairs.ensure(std::max<unsigned long long>(slack_total, 1) * 2 * sizeof(uint32_t))) != hipSuccess)
        return hip_fail(e, "output slack");
    if (with_w && (e = S.slack_weights.ensure(std::max<unsigned long long>(slack_total, 1) * sizeof(float))) != hipSuccess)
        return hip_fail(e, "weight slack");
    unsigned long long* d_counters = static_cast<unsigned long long*>(S.counters.p);
    unsigned long long* d_misc = static_cast<unsigned long long*>(S.misc.p);
    unsigned long long* d_partials = static_cast<unsigned long long*>(S.partials.p);

    // ---- task order and work queues ----
    // Items are laid out in the task list by decreasing cost per task (light
    // count), and the eight queues get slices of roughly equal estimated cost
    // (cost of a task ~ n_lights^0.6, the growth of node visits per eye):
    // every queue starts with its heaviest eyes and ends with light ones, so
    // the launch's tail is made of short tasks.  One item keeps equal slices.
    std::vector<uint32_t> torder(n);
    for (size_t k = 0; k < n; ++k) torder[k] = (uint32_t)k;
    std::stable_sort(torder.begin(), torder.end(), [&](uint32_t x, uint32_t y) {
        return items[x].h->n_lights > items[y].h->n_lights;
    });
    std::vector<double> task_cost(n);
    double total_cost = 0.0;
    for (size_t k = 0; k < n; ++k) {
        task_cost[k] = pow((double)std::max<uint32_t>(items[k].h->n_lights, 1u), 0.6);
        total_cost += task_cost[k] * (double)tasks_of[k];
    }
    std::vector<uint32_t> begin_of(n);
    uint32_t qbegin[kQueues + 1];
    {
        uint64_t tb = 0;
        double cum = 0.0;
        uint32_t g = 1;
        qbegin[0] = 0;
        for (size_t pos = 0; pos < n; ++pos) {
            const uint32_t k = torder[pos];
            begin_of[k] = (uint32_t)tb;
            const double c = task_cost[k], item_cost = c * (double)tasks_of[k];
            while (g < kQueues && cum + item_cost >= total_cost * g / kQueues) {
                const double need = total_cost * g / kQueues - cum;
                const uint64_t at = tb + std::min<uint64_t>(tasks_of[k], (uint64_t)ceil(need / c));
                qbegin[g] = (uint32_t)std::max<uint64_t>(at, qbegin[g - 1]);
                ++g;
            }
            tb += tasks_of[k];
            cum += item_cost;
        }
        for (; g <= kQueues; ++g) qbegin[g] = (uint32_t)tasks;
        qbegin[kQueues] = (uint32_t)tasks;
    }

    S.h_items.assign(n, ItemDesc{});
    S.h_task_begin.assign(n + 1, 0);
    for (size_t pos = 0; pos < n; ++pos) {
        const size_t k = torder[pos];
        const HostItem& it = items[k];
        const hrr_hierarchy* h = it.h;
        const ItemMeta& m = M[k];
        ItemDesc& D = S.h_items[pos];
        D.nodes = h->d_nodes;
        D.frontier = h->d_frontier;
        D.n_frontier = h->n_frontier;
        D.lights = h->d_lights;
        D.eyes = it.eyes.xyz;
        D.pairs = pairs ? pairs + 2 * it.out_offset : nullptr;
        D.weights = weights ? weights + it.out_offset : nullptr;
        D.slack_pairs = static_cast<uint32_t*>(S.slack_pairs.p) + 2 * m.slack_off;
        D.slack_weights = with_w ? static_cast<float*>(S.slack_weights.p) + m.slack_off : nullptr;
        D.order = ordered ? static_cast<const uint32_t*>(S.order_idx.p) + vbegin[k] : nullptr;
        D.counters = d_counters + k * CNT_STRIDE;
        D.partials = d_partials + 2 * m.partial_off;
        D.plan = static_cast<unsigned long long*>(S.plan.p) + m.plan_off;
        D.capacity = it.out_capacity;
        D.slack = m.slack;
        D.partial_cap = m.partial_cap;
        D.chunk_shift = m.chunk_shift;
        D.n_lights = h->n_lights;
        D.n_nodes = h->n_nodes;
        D.leaf_size = h->leaf_size;
        D.n_virtual = h->n_lights ? (uint32_t)((uint64_t)it.eyes.n * n_samples) : 0u;
        D.width = it.eyes.width;
        D.shift_offset = it.eyes.shift_offset;
        D.pixel_base = it.eyes.pixel_base;
        D.n_samples = n_samples;
        D.psi_s0 = psi_s0;
        D.s = it.s;
        product_test_bounds(it.s, &D.t_cull, &D.t_keep, &D.d2_fast);
        for (int q = 0; q < 3; ++q) {
            D.root_lo[q] = h->box[q];
            D.root_hi[q] = h->box[3 + q];
        }
        D.task_begin = begin_of[k];
        S.h_task_begin[pos] = begin_of[k];
    }
    S.h_task_begin[n] = (uint32_t)tasks;

    // pinned staging: readback words first, then the upload of the tables
    const size_t items_bytes = n * sizeof(ItemDesc);
    const size_t tb_bytes = (n + 1) * sizeof(uint32_t);
    const size_t oi_bytes = ordered ? n * sizeof(OrderItem) : 0;
    const size_t vb_bytes = ordered ? (n + 1) * sizeof(uint32_t) : 0;
    const size_t read_words = n * CNT_STRIDE + 1 + ST_N;
    const size_t pin_words = read_words + (items_bytes + tb_bytes + oi_bytes + vb_bytes + 7) / 8 + 8;
    if (S.h_pinned_n < pin_words) {
        if (S.h_pinned) (void)hipHostFree(S.h_pinned);
        S.h_pinned = nullptr;
        S.h_pinned_n = 0;
        if ((e = hipHostMalloc((void**)&S.h_pinned, pin_words * 8, hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "pinned staging");
        S.h_pinned_n = pin_words;
    }
    unsigned char* up = reinterpret_cast<unsigned char*>(S.h_pinned + read_words);
    memcpy(up, S.h_items.data(), items_bytes);
    memcpy(up + items_bytes, S.h_task_begin.data(), tb_bytes);
    // OrderItem holds a pointer: keep it 8-byte aligned
    const size_t oi_at = (items_bytes + tb_bytes + 7) / 8 * 8;
    const size_t vb_at = oi_at + oi_bytes;
    if (ordered) {
        memcpy(up + oi_at, oitems.data(), oi_bytes);
        memcpy(up + vb_at, vbegin.data(), vb_bytes);
    }

    if ((e = S.items.ensure(items_bytes)) != hipSuccess) return hip_fail(e, "item table");
    if ((e = S.task_begin.ensure(tb_bytes)) != hipSuccess) return hip_fail(e, "task table");
    if ((e = hipMemcpyAsync(S.items.p, up, items_bytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
        return hip_fail(e, "upload items");
    if ((e = hipMemcpyAsync(S.task_begin.p, up + items_bytes, tb_bytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
        return hip_fail(e, "upload tasks");
    if ((e = hipMemsetAsync(d_counters, 0, n * CNT_STRIDE * sizeof(unsigned long long), stream)) != hipSuccess)
        return hip_fail(e, "clear counters");
    if ((e = hipMemsetAsync(d_misc, 0, 16 * sizeof(unsigned long long), stream)) != hipSuccess)
        return hip_fail(e, "clear misc");
    if ((e = hipMemsetAsync(S.queues.p, 0, kQueues * kQueueStride * sizeof(uint32_t), stream)) != hipSuccess)
        return hip_fail(e, "clear queues");
    if (ordered) {
        if ((e = hipMemcpyAsync(S.order_items.p, up + oi_at, oi_bytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return hip_fail(e, "upload order items");
        if ((e = hipMemcpyAsync(S.order_vbegin.p, up + vb_at, vb_bytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return hip_fail(e, "upload order offsets");
        if ((e = hrr_launch_order(static_cast<const OrderItem*>(S.order_items.p),
                                  static_cast<const uint32_t*>(S.order_vbegin.p), (uint32_t)n, (uint32_t)vtotal, bits,
                                  rbits, ctx->d_tile, ctx->tile_tz, static_cast<uint32_t*>(S.order_keys.p),
                                  static_cast<uint32_t*>(S.order_hist.p), static_cast<uint32_t*>(S.order_idx.p),
                                  ctx->n_cu, stream)) != hipSuccess)
            return hip_fail(e, "eye ordering");
    }

    if (tasks > 0) {
        // 128 entries per tree level (see the kernel's stack), whole 64-entry units, one spare
        const uint64_t bound = 128ull * (dmax + 2);
        const uint32_t spill_cap = (uint32_t)(((bound + 63) / 64) * 64 + 64);
        const size_t spill_bytes = (size_t)waves * spill_cap * sizeof(unsigned long long);
        if ((e = S.spill.ensure(spill_bytes)) != hipSuccess) return hip_fail(e, "spill stacks");

        TravArgs A;
        memset(&A, 0, sizeof A);
        A.items = static_cast<const ItemDesc*>(S.items.p);
        A.task_begin = static_cast<const uint32_t*>(S.task_begin.p);
        A.n_items = (uint32_t)n;
        A.n_tasks = (uint32_t)tasks;
        for (uint32_t q = 0; q <= kQueues; ++q) A.queue_begin[q] = qbegin[q];
        A.interleave_shift = il_shift;
        A.queues = static_cast<uint32_t*>(S.queues.p);
        A.tile = ctx->d_tile;
        A.spill = static_cast<unsigned long long*>(S.spill.p);
        A.spill_cap = spill_cap;
        A.stack_cap = cap;
        A.lds_per_wave = (uint32_t)lds_wave;
        A.stats = stats ? d_misc + 2 : nullptr;
        A.error = reinterpret_cast<uint32_t*>(d_misc + 1);
        if (timing) {
            if (!S.ev_begin && (e = hipEventCreate(&S.ev_begin)) != hipSuccess) return hip_fail(e, "timing event");
            if (!S.ev_end && (e = hipEventCreate(&S.ev_end)) != hipSuccess) return hip_fail(e, "timing event");
            if ((e = hipEventRecord(S.ev_begin, stream)) != hipSuccess) return hip_fail(e, "timing event");
        }
        if ((e = hrr_launch_traverse(&A, epw, method, stats, with_w, blocks, stream)) != hipSuccess)
            return hip_fail(e, "traverse launch");
        if (timing) {
            if ((e = hipEventRecord(S.ev_end, stream)) != hipSuccess) return hip_fail(e, "timing event");
            S.timed = true;
        }
        // make every item's stored pairs dense (on the device, before the readback)
        bool any_capacity = false;
        for (size_t k = 0; k < n; ++k) any_capacity = any_capacity || items[k].out_capacity > 0;
        if (any_capacity &&
            (e = hrr_launch_compact(static_cast<const ItemDesc*>(S.items.p), (uint32_t)n, A.error, stream)) !=
                hipSuccess)
            return hip_fail(e, "output compaction");
    }
    if ((e = hipMemcpyAsync(S.h_pinned, d_counters, n * CNT_STRIDE * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            stream)) != hipSuccess)
        return hip_fail(e, "read counters");
    if ((e = hipMemcpyAsync(S.h_pinned + n * CNT_STRIDE, d_misc + 1, (1 + ST_N) * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, stream)) != hipSuccess)
        return hip_fail(e, "read status");
    return HRR_OK;
}

// The allocation-free traversal.  Same kernels as launch_items for one item,
// with every buffer the launch needs carved out of the device's fixed scratch
// (kNoAllocScratchBytes): the header, then per wave a stack spill region
// sized for the hierarchy's depth (the walk's bound, 128 entries per level),
// then the partial-chunk list and compaction plan (one entry per wave: a
// one-item launch leaves its item once per wave), then the output slack (two
// chunks per wave).  The grid is the resident one, cut to as many whole
// blocks as the scratch holds; output chunks have at most 2^10 pairs.  Eyes
// run in index order (the result does not depend on the order).
hrr_status launch_noalloc(hrr_ctx* ctx, const hrr_hierarchy* h, const hrr_eyes& eyes, float s,
                          const hrr_traverse_opts* opts, uint32_t* pairs, float* weights, uint64_t capacity,
                          unsigned long long* result_dev, hipStream_t stream) {
    if (h->owner != ctx) return fail(HRR_E_INVALID, "hrr_traverse_noalloc: hierarchy belongs to another context");
    if (!ctx->noalloc_scratch) return fail(HRR_E_DEVICE, "hrr_traverse_noalloc: no scratch on this device");
    if (!(s > 0.0f) || !isfinite(s)) return fail(HRR_E_INVALID, "hrr_traverse_noalloc: s must be finite and > 0");
    if (eyes.n > 0 && !eyes.xyz) return fail(HRR_E_INVALID, "hrr_traverse_noalloc: null eye positions");
    if (eyes.width == 0) return fail(HRR_E_INVALID, "hrr_traverse_noalloc: width must be >= 1");
    if (capacity > 0 && !pairs) return fail(HRR_E_INVALID, "hrr_traverse_noalloc: null pairs buffer");
    const uint32_t flags = opts ? opts->flags : 0u;
    if (flags & (HRR_F_STATS | HRR_F_TIMING))
        return fail(HRR_E_INVALID, "hrr_traverse_noalloc: statistics and timing need a readback; not supported");
    const uint32_t method = opts ? opts->rmq_method : HRR_RMQ_PAPER;
    if (method > 5) return fail(HRR_E_INVALID, "unknown rmq method %u", method);
    const uint32_t n_samples = opts && opts->n_samples > 1 ? opts->n_samples : 1u;
    const uint64_t nv = (uint64_t)eyes.n * n_samples;
    if (nv > 0xFFFFFFFFull) return fail(HRR_E_INVALID, "hrr_traverse_noalloc: eyes x samples exceeds 2^32 - 1");
    uint32_t epw = 1, cap = 192;
    resolve_shape(ctx, opts, h->n_lights, eyes.n, &epw, &cap);
    if (!(epw == 1 || epw == 2 || epw == 4 || epw == 8))
        return fail(HRR_E_INVALID, "eyes_per_wave must be 1, 2, 4 or 8");
    if (cap % 64 != 0 || cap < 192 || cap > 4096)
        return fail(HRR_E_INVALID, "stack_entries must be a multiple of 64 in [192, 4096]");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const int with_w = weights != nullptr;
    const size_t lds_wave = hrr_trav_lds_per_wave(cap, epw);
    const size_t lds_block = hrr_trav_lds_per_block(1, lds_wave);
    int bpc = 0;
    if ((e = hrr_traverse_occupancy(epw, method, 0, with_w, lds_block, &bpc)) != hipSuccess)
        return hip_fail(e, "occupancy");
    if (bpc <= 0) return fail(HRR_E_INVALID, "stack of %u entries does not fit in LDS", cap);
    const uint64_t tasks = h->n_lights ? (nv + epw - 1) / epw : 0;

    // ---- scratch layout: as many whole blocks as the scratch holds ----
    const uint64_t spill_cap = (128ull * (h->depth + 2) + 63) / 64 * 64 + 64;    // entries per wave
    const uint64_t pair_bytes = 8ull + (with_w ? 4ull : 0ull);
    const uint64_t resident = std::max<uint64_t>(1, (uint64_t)ctx->n_cu * bpc) * kWavesPerBlock;
    const uint64_t needed = std::max<uint64_t>(kWavesPerBlock, (tasks + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock);
    uint64_t waves = std::min(resident, needed);
    uint32_t shift = std::min<uint32_t>(chunk_shift_for(capacity, std::min<uint64_t>(waves, std::max<uint64_t>(tasks, 1))),
                                        kNoAllocMaxChunkShift);
    auto bytes_for = [&](uint64_t w, uint32_t sh) {
        return kNoAllocHeaderBytes + w * spill_cap * 8ull + w * 2ull * 8ull + (3ull * w + 4ull) * 8ull +
               (capacity ? 2ull * w * (1ull << sh) * pair_bytes : 0ull) + 1024ull;
    };
    while (waves > kWavesPerBlock && bytes_for(waves, shift) > kNoAllocScratchBytes)
        waves -= kWavesPerBlock;
    if (bytes_for(waves, shift) > kNoAllocScratchBytes)
        return fail(HRR_E_INVALID, "hrr_traverse_noalloc: a hierarchy of depth %u needs more than the "
                    "%llu-byte scratch for one block", h->depth, (unsigned long long)kNoAllocScratchBytes);
    const uint32_t blocks = (uint32_t)(waves / kWavesPerBlock);
    unsigned char* base = static_cast<unsigned char*>(ctx->noalloc_scratch);
    uint64_t at = kNoAllocHeaderBytes;
    auto carve = [&](uint64_t bytes) {
        unsigned char* p = base + at;
        at += (bytes + 255) / 256 * 256;
        return p;
    };
    const uint64_t pk = std::max<uint64_t>(1, std::min<uint64_t>(waves, tasks));
    uint2* spill = reinterpret_cast<uint2*>(carve(waves * spill_cap * 8ull));
    unsigned long long* partials = reinterpret_cast<unsigned long long*>(carve(pk * 2ull * 8ull));
    unsigned long long* plan = reinterpret_cast<unsigned long long*>(carve((3ull * pk + 4ull) * 8ull));
    const unsigned long long slack = capacity ? 2ull * pk << shift : 0ull;
    uint32_t* slack_pairs = reinterpret_cast<uint32_t*>(carve(std::max<unsigned long long>(slack, 1) * 8ull));
    float* slack_weights = with_w ? reinterpret_cast<float*>(carve(std::max<unsigned long long>(slack, 1) * 4ull)) : nullptr;
    if (at > kNoAllocScratchBytes) return fail(HRR_E_DEVICE, "hrr_traverse_noalloc: scratch layout exceeds its size");

    ItemDesc D;
    memset(&D, 0, sizeof D);
    D.nodes = h->d_nodes;
    D.frontier = h->d_frontier;
    D.n_frontier = h->n_frontier;
    D.lights = h->d_lights;
    D.eyes = eyes.xyz;
    D.pairs = pairs;
    D.weights = weights;
    D.slack_pairs = slack_pairs;
    D.slack_weights = slack_weights;
    D.order = nullptr;
    D.counters = reinterpret_cast<unsigned long long*>(base + kNoAllocCounters);
    D.partials = partials;
    D.plan = plan;
    D.capacity = capacity;
    D.slack = slack;
    D.partial_cap = (uint32_t)pk;
    D.chunk_shift = shift;
    D.n_lights = h->n_lights;
    D.n_nodes = h->n_nodes;
    D.leaf_size = h->leaf_size;
    D.n_virtual = h->n_lights ? (uint32_t)nv : 0u;
    D.width = eyes.width;
    D.shift_offset = eyes.shift_offset;
    D.pixel_base = eyes.pixel_base;
    D.n_samples = n_samples;
    D.psi_s0 = opts ? opts->psi_s0 : 0u;
    D.s = s;
    product_test_bounds(s, &D.t_cull, &D.t_keep, &D.d2_fast);
    for (int q = 0; q < 3; ++q) {
        D.root_lo[q] = h->box[q];
        D.root_hi[q] = h->box[3 + q];
    }
    D.task_begin = 0;

    if ((e = hrr_launch_noalloc_setup(&D, (uint32_t)tasks, base, stream)) != hipSuccess)
        return hip_fail(e, "allocation-free set-up");
    const ItemDesc* d_item = reinterpret_cast<const ItemDesc*>(base + kNoAllocItem);
    uint32_t* error = reinterpret_cast<uint32_t*>(base + kNoAllocMisc + 8);
    if (tasks > 0) {
        TravArgs A;
        memset(&A, 0, sizeof A);
        A.items = d_item;
        A.task_begin = reinterpret_cast<const uint32_t*>(base + kNoAllocTasks);
        A.n_items = 1;
        A.n_tasks = (uint32_t)tasks;
        for (uint32_t q = 0; q <= kQueues; ++q) A.queue_begin[q] = (uint32_t)(tasks * q / kQueues);
        A.interleave_shift = 0;
        A.queues = reinterpret_cast<uint32_t*>(base + kNoAllocQueues);
        A.tile = ctx->d_tile;
        A.spill = reinterpret_cast<unsigned long long*>(spill);
        A.spill_cap = (uint32_t)spill_cap;
        A.stack_cap = cap;
        A.lds_per_wave = (uint32_t)lds_wave;
        A.stats = nullptr;
        A.error = error;
        if ((e = hrr_launch_traverse(&A, epw, method, 0, with_w, blocks, stream)) != hipSuccess)
            return hip_fail(e, "allocation-free traverse launch");
        if (capacity > 0 && (e = hrr_launch_compact(d_item, 1, error, stream)) != hipSuccess)
            return hip_fail(e, "allocation-free output compaction");
    }
    if ((e = hrr_launch_noalloc_finish(base, result_dev, stream)) != hipSuccess)
        return hip_fail(e, "allocation-free result");
    return HRR_OK;
}

double timed_kernel_ms(LaunchScratch& S) {
    if (!S.timed) return 0.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, S.ev_begin, S.ev_end) != hipSuccess) return 0.0;
    return (double)ms;
}

hrr_status finish_items(hrr_ctx*, LaunchScratch& S) {
    const size_t n = S.n_items;
    S.counts.assign(n, 0);
    S.stored.assign(n, 0);
    const unsigned long long* rd = S.h_pinned;
    S.error = (uint32_t)rd[n * CNT_STRIDE];
    for (int q = 0; q < ST_N; ++q) S.stat[q] = rd[n * CNT_STRIDE + 1 + q];
    for (size_t k = 0; k < n; ++k) {
        S.counts[k] = rd[k * CNT_STRIDE + CNT_PAIRS];
        S.stored[k] = rd[k * CNT_STRIDE + CNT_STORED];
    }
    return HRR_OK;
}

}  // namespace hrr
