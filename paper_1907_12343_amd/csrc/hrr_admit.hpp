// hrr_admit.hpp -- admission policy of the serving loop: which queued
// requests join the next batch (host only; no device calls, CPU-tested).
//
// The queue is scanned in arrival order.  A request joins the batch when the
// batch still has room for it (max_items requests, max_eyes eyes; the first
// request of a batch is always within the eye limit) and the arena can hold
// its eye copy and its output reservation.  A request that does not fit is
// skipped, so a large request at the head does not hold up smaller ones
// behind it -- unless it has already waited longer than max_skip_s: then the
// scan stops at it, nothing behind it is admitted, and the arena drains until
// it fits (it is then the oldest request, so it is first in line).  That age
// bound is what keeps large requests from starving; max_skip_s = 0 gives a
// strict FIFO (the scan stops at the first request that does not fit).
#pragma once

#include <stdint.h>

#include <vector>

#include "hrr_arena.hpp"

namespace hrr {

struct AdmitLimits {
    uint32_t max_items;   // requests per batch (>= 1)
    uint64_t max_eyes;    // eyes per batch
    double max_skip_s;    // a request waiting longer than this is never overtaken
    uint32_t max_scan;    // queue entries looked at per batch (bounds the work under the lock)
};

// What the policy needs to know about one queued request.
struct AdmitView {
    uint64_t n_eyes;
    uint64_t eye_bytes;   // device bytes of its eye copy (0: none)
    uint64_t out_bytes;   // device bytes of its output reservation (0: none)
    double submit_s;      // arrival time, same clock as `now`
};

struct Admitted {
    size_t pos;           // position in the queue
    uint64_t eye_off, out_off;
};

// Choose the next batch from a queue of qlen requests; view(i) describes the
// i-th.  The chosen requests' arena blocks are allocated here (their offsets
// are returned); out lists them in queue order.
template <class ViewFn>
void admit_batch(Arena& arena, const AdmitLimits& L, double now, size_t qlen, ViewFn view,
                 std::vector<Admitted>& out) {
    out.clear();
    uint64_t eyes = 0;
    const size_t scan = qlen < (size_t)L.max_scan ? qlen : (size_t)L.max_scan;
    for (size_t i = 0; i < scan && out.size() < L.max_items; ++i) {
        const AdmitView v = view(i);
        const bool overdue = now - v.submit_s >= L.max_skip_s;
        bool fits = out.empty() || eyes + v.n_eyes <= L.max_eyes;
        uint64_t eoff = 0, ooff = 0;
        if (fits && v.eye_bytes && !arena.alloc(v.eye_bytes, &eoff)) fits = false;
        if (fits && v.out_bytes && !arena.alloc(v.out_bytes, &ooff)) {
            if (v.eye_bytes) arena.release(eoff, v.eye_bytes);
            fits = false;
        }
        if (!fits) {
            if (overdue) break;   // nothing may overtake an overdue request
            continue;
        }
        out.push_back(Admitted{i, eoff, ooff});
        eyes += v.n_eyes;
    }
}

}  // namespace hrr
