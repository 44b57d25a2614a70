// hrr_compact.hpp -- host planning of the output compaction that follows a
// traversal launch (no device calls; unit-tested on the CPU).
//
// The kernel hands out output chunks of C = 2^shift pairs, one atomic per
// chunk; a wave that leaves an item publishes its last, partly filled chunk
// as (chunk, fill).  Positions below the caller's capacity are in the
// caller's slice, positions in [capacity, capacity + slack) in a library
// slack area, later ones are dropped (the count stays exact).  To make the
// first target = min(count, capacity) positions dense, the pairs stored at
// or past `target` are moved into the holes below it (the unfilled tails of
// partly filled chunks).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <thread>
#include <utility>
#include <vector>

namespace hrr {

// Source offsets with this bit set are slack-area offsets.
constexpr unsigned long long kSlackFlag = 1ull << 63;

// Reusable scratch of plan_compaction (keeps its capacity between calls).
struct CompactScratch {
    std::vector<unsigned long long> fill;
    std::vector<std::pair<unsigned long long, unsigned long long>> holes, data;
};

// Appends (source, destination, length) triples to `segments` (sources are
// out_offset + position, or kSlackFlag | (slack_off + position - capacity);
// destinations out_offset + position) and returns the number of positions
// below `target` left unfilled (0 whenever the slack holds twice the chunks
// of all partial chunks).  partials: n_partials (chunk, fill) pairs in any
// order; chunks: the number of chunks handed out.
inline unsigned long long plan_compaction(unsigned long long target, unsigned long long chunks, uint32_t shift,
                                          unsigned long long capacity, unsigned long long slack,
                                          const unsigned long long* partials, unsigned long long n_partials,
                                          unsigned long long out_offset, unsigned long long slack_off,
                                          CompactScratch& scratch, std::vector<unsigned long long>& segments) {
    if (target == 0) return 0;
    const unsigned long long C = 1ull << shift;
    const unsigned long long limit = capacity + slack;   // stored positions are below this
    // Holes: tails of partly filled chunks below the target.  Data: chunks
    // c0 = target / C .. up to the limit (at most n_partials + 1 of them when
    // the count fits), full except the partly filled ones.  Holes and data
    // pair up in any order, so nothing is sorted.
    std::vector<unsigned long long>& fill = scratch.fill;
    std::vector<std::pair<unsigned long long, unsigned long long>>& holes = scratch.holes;
    std::vector<std::pair<unsigned long long, unsigned long long>>& data = scratch.data;
    holes.clear();
    data.clear();
    const unsigned long long c0 = target / C;
    const unsigned long long c_end = std::min<unsigned long long>(chunks, (limit + C - 1) / C);
    fill.assign(c_end > c0 ? (size_t)(c_end - c0) : 0u, C);
    for (unsigned long long q = 0; q < n_partials; ++q) {
        const unsigned long long c = partials[2 * q], f = partials[2 * q + 1];
        const unsigned long long lo = c * C + f;
        const unsigned long long hi = std::min((c + 1) * C, target);
        if (lo < hi) holes.push_back({lo, hi});
        if (c >= c0 && c < c_end) fill[c - c0] = f;
    }
    for (unsigned long long c = c0; c < c_end; ++c) {
        const unsigned long long lo = std::max(c * C, target);
        const unsigned long long hi = std::min(c * C + fill[c - c0], limit);
        // a chunk that straddles the capacity gives two segments
        if (lo < std::min(hi, capacity)) data.push_back({lo, std::min(hi, capacity)});
        if (std::max(lo, capacity) < hi) data.push_back({std::max(lo, capacity), hi});
    }
    unsigned long long unfilled = 0;
    size_t hi_ = 0, di = 0;
    unsigned long long hpos = holes.empty() ? 0 : holes[0].first;
    unsigned long long dpos = data.empty() ? 0 : data[0].first;
    while (hi_ < holes.size()) {
        if (di >= data.size()) {
            unfilled += holes[hi_].second - hpos;
            if (++hi_ < holes.size()) hpos = holes[hi_].first;
            continue;
        }
        const unsigned long long len = std::min(holes[hi_].second - hpos, data[di].second - dpos);
        segments.push_back(dpos < capacity ? out_offset + dpos : (kSlackFlag | (slack_off + dpos - capacity)));
        segments.push_back(out_offset + hpos);
        segments.push_back(len);
        hpos += len;
        dpos += len;
        if (hpos == holes[hi_].second && ++hi_ < holes.size()) hpos = holes[hi_].first;
        if (dpos == data[di].second && ++di < data.size()) dpos = data[di].first;
    }
    return unfilled;
}

// One item of a launch, as the host reads it back: its true pair count, the
// chunks handed out, its partial-chunk list (n_partials entries from
// partial_at in the packed list; only items that stored pairs have one) and
// its output layout.
struct ItemPlan {
    unsigned long long count, chunks, n_partials, partial_at;
    unsigned long long capacity, slack, out_offset, slack_off;
    uint32_t shift;
};

// Plans the moves of every item of a launch: appends their segments to
// `segments` in item order and sets stored[k] = min(count, capacity) minus the
// positions left unfilled.  With eight or more items and 8192 or more partial
// entries the items are cut into up to max_threads contiguous ranges of about
// equal partial counts, planned on host threads with scratch of their own and
// joined in item order, so the result equals the one-thread plan.  Returns
// true when some item left positions unfilled.
inline bool plan_items(const ItemPlan* items, size_t n, const unsigned long long* partials, unsigned max_threads,
                       CompactScratch& scratch, std::vector<unsigned long long>& segments,
                       unsigned long long* stored) {
    auto plan_range = [&](size_t k0, size_t k1, CompactScratch& sc, std::vector<unsigned long long>& seg) {
        bool lost = false;
        for (size_t k = k0; k < k1; ++k) {
            const ItemPlan& it = items[k];
            const unsigned long long target = std::min(it.count, it.capacity);
            stored[k] = 0;
            if (target == 0) continue;
            const unsigned long long unfilled =
                plan_compaction(target, it.chunks, it.shift, it.capacity, it.slack, partials + 2 * it.partial_at,
                                it.n_partials, it.out_offset, it.slack_off, sc, seg);
            stored[k] = target - unfilled;
            if (unfilled) lost = true;
        }
        return lost;
    };
    unsigned long long total = 0;
    for (size_t k = 0; k < n; ++k)
        if (std::min(items[k].count, items[k].capacity)) total += items[k].n_partials;
    const size_t n_threads =
        (n >= 8 && total >= 8192) ? std::min<size_t>(std::max(1u, max_threads), std::min<size_t>(8, n)) : 1;
    if (n_threads <= 1) return plan_range(0, n, scratch, segments);
    std::vector<size_t> cut(n_threads + 1, n);
    cut[0] = 0;
    size_t t = 1;
    unsigned long long acc = 0;
    for (size_t k = 0; k < n && t < n_threads; ++k) {
        if (std::min(items[k].count, items[k].capacity)) acc += items[k].n_partials;
        if (acc * n_threads >= total * t) cut[t++] = k + 1;
    }
    std::vector<CompactScratch> sc(n_threads - 1);
    std::vector<std::vector<unsigned long long>> seg(n_threads - 1);
    std::vector<char> lost(n_threads, 0);
    std::vector<std::thread> pool;
    for (size_t q = 1; q < n_threads; ++q)
        pool.emplace_back([&, q] { lost[q] = plan_range(cut[q], cut[q + 1], sc[q - 1], seg[q - 1]); });
    lost[0] = plan_range(cut[0], cut[1], scratch, segments);
    for (auto& th : pool) th.join();
    bool any = lost[0] != 0;
    for (size_t q = 1; q < n_threads; ++q) {
        any = any || lost[q];
        segments.insert(segments.end(), seg[q - 1].begin(), seg[q - 1].end());
    }
    return any;
}

}  // namespace hrr
