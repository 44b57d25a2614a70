// hrr_layout.hpp -- host-side choices of a traversal launch's layout (eye
// order key, work-queue layout, output chunk size, partial-chunk bound).
// Plain functions of the launch's sizes, unit-tested on the CPU.
#pragma once

#include <stdint.h>

#include "hrr_types.hpp"

namespace hrr {

// Eye-order key widths for n items holding `virtual_eyes` virtual eyes in all:
// Morton cells of about 2^11 or more virtual eyes each (at least two bits per
// axis where the bucket budget allows), then up to 9 bits of the shift class
// (no more than the tile values' significant bits), within kOrderMaxBuckets
// buckets.  bits = 0: no reordering.  On the 1920x1080 frame over 2^20 lights
// (3 bits per axis, 9 class bits) this runs 4-5 % faster than finer cells
// alone; a launch of 256 small items is insensitive to the split as long as
// cells have two or more bits per axis.
inline void order_key_bits(uint64_t n, uint64_t virtual_eyes, uint32_t tile_bits, uint32_t* bits_out,
                           uint32_t* rbits_out) {
    uint32_t bits = 0, rbits = 0;
    if (n > 0 && virtual_eyes > 0 && virtual_eyes < 0xFFFFFFFFull) {
        const uint64_t per_item = virtual_eyes / n > 0 ? virtual_eyes / n : 1;
        while (bits < 2 && (n << (3 * (bits + 1))) <= kOrderMaxBuckets) ++bits;
        while (bits && bits < 10 && (per_item >> (3 * (bits + 1))) >= (1u << 11) &&
               (n << (3 * (bits + 1))) <= kOrderMaxBuckets)
            ++bits;
        if (bits && tile_bits) {
            rbits = tile_bits < 9u ? tile_bits : 9u;
            while (rbits && (n << (3 * bits + rbits)) > kOrderMaxBuckets) --rbits;
        }
    }
    *bits_out = bits;
    *rbits_out = rbits;
}

// Whether a launch orders its eyes at all: the ordering pass (five small
// kernels and their set-up) costs about 35 us per call, which only pays when
// the launch has enough work for cache locality to matter.  `cost` is the
// launch's estimated work, the sum over items of virtual eyes x
// n_lights^0.6 (the cost model of the work queues).  4096 eyes x 1024 lights
// (cost 2.6e5): 0.134 ms per call unordered against 0.170 ordered; 4096 of the
// frame's eyes x 2^20 lights (cost 1.7e7): 1.37 unordered against 1.34
// ordered, and ordering halves the time from 2^15 such eyes on.
constexpr double kOrderMinCost = 2097152.0;   // 2^21
inline bool order_pays(double cost) { return cost >= kOrderMinCost; }

// Work-queue layout: launches of several items with 2^19 or more tasks use
// interleaved chunks of 2^13 tasks (queue q owns chunks q, q + 8, ...), so all
// XCDs work on the same heavy items at a time and the Infinity Cache holds
// fewer hierarchies at once (256 caches: kernel 70.3 -> 66.5 ms); others use
// eight contiguous slices of equal cost.  Returns the chunk shift, 0 for
// slices.
inline uint32_t queue_interleave_shift(uint64_t n, uint64_t tasks) {
    return (n > 1 && tasks >= (1ull << 19)) ? 13u : 0u;
}

// How often one wave can leave one item (publishing a partly filled chunk).
// A wave visits each queue once (cyclic order from its own) and takes a
// queue's tasks in increasing order, so within one queue visit the items it
// meets are nondecreasing and it leaves an item at most once.  Contiguous
// slices are in task order too: at most twice per item (the one wrap), once
// in a one-item launch; interleaved chunks: at most once per queue visit.
inline uint64_t departures_per_wave(uint64_t n, uint32_t interleave_shift) {
    return interleave_shift ? kQueues : (n > 1 ? 2 : 1);
}

// Eyes per wavefront for a hierarchy of n_lights lights when neither the
// caller nor the tuner fixes it.  Small hierarchies give an eye only tens to
// hundreds of node visits, too few to keep 64 lanes busy (one eye per wave:
// 13 % of the lanes active at 2^10..2^12 lights, 37 % at 2^14..2^16, 89 % at
// 2^18..2^20), so several eyes share a wave.  Thresholds measured on batched
// launches of mixture caches at s = 1e-4 (kernel ms at 1 / 4 / 8 eyes per wave:
// 2^10..2^12 lights 3.82 / 1.40 / 0.76, 2^14..2^16 6.34 / 3.37 / 3.11,
// 2^16..2^17 3.36 / 3.04 / 3.08, 2^17..2^18 8.90 / 8.94 / 9.08, 2^18..2^20
// 40.4 / 45.2 / 51.3).
inline uint32_t default_eyes_per_wave(uint32_t n_lights) {
    return n_lights >= (1u << 17) ? 1u : n_lights >= (1u << 16) ? 4u : 8u;
}

// LDS stack entries per wave when neither the caller nor the tuner fixes
// them.  One eye per wave also keeps a 4160-byte record area in LDS; 192
// entries (1.5 KB) leave room for 7 waves per SIMD in 160 KB, 256 entries
// for 6 (frame, power-of-two splits: 123.7 ms at 192 entries against 127.9 ms
// at 256 and 154.3 ms at 512).  Several eyes per wave run at 96 registers (5
// waves per SIMD) with their eyes in LDS, where 512 entries cost nothing.
inline uint32_t default_stack_entries(uint32_t eyes_per_wave) {
    return eyes_per_wave == 1 ? 192u : 512u;
}

// Stack sizes the autotuner tries for a shape, in order of preference.
inline void tune_stack_candidates(uint32_t eyes_per_wave, uint32_t out[3]) {
    if (eyes_per_wave == 1) {
        out[0] = 192; out[1] = 256; out[2] = 512;
    } else {
        out[0] = 512; out[1] = 256; out[2] = 1024;
    }
}

// Output chunk size of an item: about sixteen chunks per wave that touches
// the item, 2^kMinChunkShift .. 2^kMaxChunkShift pairs.
inline uint32_t chunk_shift_for(uint64_t capacity, uint64_t touching_waves) {
    uint32_t shift = kMinChunkShift;
    while (shift < kMaxChunkShift && (capacity >> (shift + 1)) >= 16 * touching_waves) ++shift;
    return shift;
}

}  // namespace hrr
