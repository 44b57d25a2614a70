// hrr_compact.hpp -- per-item arithmetic of the output compaction that follows
// a traversal launch; used by the device kernels (compact_plan_kernel,
// compact_move_kernel) and by the CPU tests, which emulate those kernels with
// these same functions.
//
// The traversal hands out output chunks of C = 2^shift pairs, one atomic per
// chunk; a wave that leaves an item publishes its last, partly filled chunk
// as (chunk, fill).  Positions below the caller's capacity are in the
// caller's slice, positions in [capacity, capacity + slack) in a library
// slack area, later ones are dropped (the count stays exact).  To make the
// first target = min(count, capacity) positions dense, the pairs stored at or
// past `target` are moved into the holes below it:
//   holes -- the unfilled tails [c C + f, min((c + 1) C, target)) of the
//            partly filled chunks, in the order of the item's partial list;
//   data  -- the stored positions [max(c C, target), min(c C + fill_c, limit))
//            of the chunks c = c0, c0 + 1, ... (c0 = target / C) up to the
//            last chunk handed out below limit = capacity + slack, where
//            fill_c = C except for partly filled chunks.
// Moved element e (0 <= e < min(total hole length, total data length)) goes
// from the e-th data position to the e-th hole position.  Sources lie at or
// past target and destinations below it, so moves never overlap.
//
// Bounds.  Every chunk handed out is full or on the partial list (a wave
// holds a chunk only while its fill is positive and publishes it when it
// leaves), so with count <= capacity the chunks past c0 number at most
// n_partials + 1; with count > capacity they end at limit, at most
// slack / C + 2.  The launch sizes slack = 2 * partial_cap * C, so an item
// never has more than 2 * partial_cap + 2 data chunks.
#pragma once

#include <stdint.h>

#ifndef HRR_HD   // host and device inline functions (also defined by hrr_rmq.hpp)
#if defined(__HIPCC__)
#define HRR_HD __host__ __device__ __forceinline__
#else
#define HRR_HD inline
#endif
#endif

namespace hrr {

// Per-item quantities of the compaction.
struct CompactGeom {
    unsigned long long target;   // min(count, capacity): positions that must end up dense
    unsigned long long C;        // pairs per chunk
    unsigned long long limit;    // capacity + slack: stored positions are below this
    unsigned long long c0;       // first data chunk
    unsigned long long nd;       // number of data chunks
    unsigned long long P;        // entries of the partial list that count
};

HRR_HD unsigned long long umin64(unsigned long long a, unsigned long long b) { return a < b ? a : b; }
HRR_HD unsigned long long umax64(unsigned long long a, unsigned long long b) { return a > b ? a : b; }

HRR_HD CompactGeom compact_geom(unsigned long long count, unsigned long long chunks, unsigned long long listed,
                                unsigned long long partial_cap, unsigned long long capacity,
                                unsigned long long slack, uint32_t shift) {
    CompactGeom g;
    g.target = umin64(count, capacity);
    g.C = 1ull << shift;
    g.limit = capacity + slack;
    g.c0 = g.target >> shift;
    const unsigned long long c_end = umin64(chunks, (g.limit + g.C - 1) >> shift);
    g.nd = (g.target && c_end > g.c0) ? c_end - g.c0 : 0ull;
    g.P = g.target ? umin64(listed, partial_cap) : 0ull;
    return g;
}

// first position and length of the hole of partial entry (chunk c, fill f)
HRR_HD unsigned long long hole_lo(const CompactGeom& g, unsigned long long c, unsigned long long f) {
    return c * g.C + f;
}
HRR_HD unsigned long long hole_len(const CompactGeom& g, unsigned long long c, unsigned long long f) {
    const unsigned long long lo = c * g.C + f, hi = umin64((c + 1) * g.C, g.target);
    return hi > lo ? hi - lo : 0ull;
}

// first position and length of the stored pairs of data chunk c0 + i with fill `fill`
HRR_HD unsigned long long data_lo(const CompactGeom& g, unsigned long long i) {
    return umax64((g.c0 + i) * g.C, g.target);
}
HRR_HD unsigned long long data_len(const CompactGeom& g, unsigned long long i, unsigned long long fill) {
    const unsigned long long lo = data_lo(g, i), hi = umin64((g.c0 + i) * g.C + fill, g.limit);
    return hi > lo ? hi - lo : 0ull;
}

// Largest q in [0, n) with prefix[q] <= e, for a nondecreasing prefix with
// prefix[0] = 0 <= e.
HRR_HD unsigned long long prefix_rank(const unsigned long long* prefix, unsigned long long n, unsigned long long e) {
    unsigned long long lo = 0, hi = n;
    while (hi - lo > 1) {
        const unsigned long long mid = lo + (hi - lo) / 2;
        if (prefix[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// Which moved elements a thread of compact_move_kernel handles.  Two
// mappings over `threads` threads (a multiple of the 64-lane wave):
//   run mode  (lanes = false): thread t takes the runs [t R, t R + R),
//             [t R + T R, ...), ... of R = run consecutive elements, T the
//             thread count;
//   lane mode (lanes = true): wave w = t / 64 takes blocks of 64 R
//             consecutive elements, [w 64 R, (w + 1) 64 R), then the block
//             T R further on, and so on, and its lane l = t % 64 takes the
//             elements l, l + 64, l + 128, ... of each block, so that the 64
//             lanes of one access touch 64 consecutive elements.
// Either way every element of [0, moved) belongs to exactly one thread.  A
// thread walks its elements as: for (e0 = first; e0 < moved; e0 += step)
// for (e = e0; e < run_end(e0); e += stride).
struct MoveMap {
    unsigned long long first;    // first element of the thread
    unsigned long long stride;   // between the thread's elements inside one run or block
    unsigned long long span;     // elements of one run (run mode) or block (lane mode)
    unsigned long long step;     // from one run or block of the thread to its next
    unsigned long long lane;     // offset of the thread inside its block (0 in run mode)
};

HRR_HD MoveMap move_map(bool lanes, unsigned long long tid, unsigned long long threads, unsigned long long run) {
    MoveMap m;
    m.lane = lanes ? tid % 64ull : 0ull;
    m.stride = lanes ? 64ull : 1ull;
    m.span = lanes ? 64ull * run : run;
    m.first = lanes ? (tid / 64ull) * m.span + m.lane : tid * run;
    m.step = threads * run;
    return m;
}

// End (exclusive) of the run or block that starts the thread's walk at e0.
HRR_HD unsigned long long move_run_end(const MoveMap& m, unsigned long long e0, unsigned long long moved) {
    return umin64(e0 - m.lane + m.span, moved);
}

}  // namespace hrr
