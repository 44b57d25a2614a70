// hrr_types.hpp -- data layouts shared by the library's host code and its
// gfx950 kernels (not by the oracle).
#pragma once

#include <stdint.h>

namespace hrr {

// One internal node of the light hierarchy, 64 bytes (half a 128-byte cache
// line).  The node covers sequence indices [a, b) (Section 1: a node is a
// contiguous sub-range of the sorted lights) and is split at c into
// [a, c) and [c, b).  It stores the fp32 bounding boxes of BOTH children, so
// one 64-byte fetch lets a lane bound and cull two subtrees.  A child whose
// range has at most leaf_size lights is a leaf and has no record.
//
// Records sit in sibling pairs: the root is record 0 (record 1 is unused),
// and a node with at least one internal child owns the pair of records
// `first` (its left child, when internal) and `first` + 1 (its right child,
// when internal), 128-byte aligned, so both children's records share one
// cache line: when a walk descends into both children, as it does for about
// two of every five records it reads, one line serves both.  Pairs are
// numbered in depth-first preorder of their owners (subtrees stay contiguous
// in memory).  A record slot whose child is a leaf is all zero, as is record
// 1; `first` is 0xFFFFFFFF when both children are leaves.
struct alignas(64) Node {
    float lo_l[3];
    uint32_t a;
    float hi_l[3];
    uint32_t c;
    float lo_r[3];
    uint32_t b;
    float hi_r[3];
    uint32_t first;
};
static_assert(sizeof(Node) == 64, "node record must be 64 bytes");

// Device-side description of one traversal work item (one hierarchy, one
// eye set, one output slice).  Eyes are "virtual": with N samples per pair,
// virtual eye u is eye u / N, sample u % N.
struct ItemDesc {
    const Node* nodes;
    const float* frontier;        // the hierarchy's top (kFrontierFloats per entry), n_frontier entries
    const float* lights;          // 4 floats per light (x, y, z, 0), sequence order
    const float* eyes;            // 3 floats per eye
    uint32_t* pairs;              // item's output slice, 2 u32 per pair
    float* weights;               // item's weight slice or null
    uint32_t* slack_pairs;        // positions >= capacity land here (library memory)
    float* slack_weights;
    const uint32_t* order;        // processing order of the virtual eyes, or null (index order)
    unsigned long long* counters; // CNT_* (device)
    unsigned long long* partials; // (chunk, fill) of partly filled chunks
    unsigned long long* plan;     // compaction prefixes: partial_cap + 1 hole, 2 partial_cap + 3 data entries
    unsigned long long capacity;  // pairs the slice can hold
    unsigned long long slack;     // pairs the slack area can hold
    uint32_t partial_cap, chunk_shift;
    uint32_t n_lights, n_nodes, leaf_size, n_virtual;
    uint32_t width, shift_offset, pixel_base, n_samples;
    uint32_t psi_s0, task_begin;
    uint32_t n_frontier, pad_frontier;
    float s;
    // product-form keep test (set by the host): v is culled when
    // float(v) * d2 > t_cull, kept (one light) when < t_keep, for d2 <= d2_fast
    float t_cull, t_keep, d2_fast;
    float root_lo[3], root_hi[3];
};

// The top of a hierarchy, where a one-eye-per-wave walk starts: the nodes of
// depth kFrontierDepth and the leaves above that depth, in index order, at
// most 2^kFrontierDepth = 64 entries (one per lane).  Every root-to-leaf path
// crosses exactly one entry, so testing the entries in place of the nodes
// above them culls no more (each test is conservative on its own) and skips
// the walk's first, nearly empty steps.  Entry layout, three float4:
// (lo.x, lo.y, lo.z, a), (hi.x, hi.y, hi.z, b), (record, 0, 0, 0), with a, b
// (the range [a, b)) and the node's record (0xFFFFFFFF for a leaf) as bits.
constexpr uint32_t kFrontierDepth = 6;
constexpr uint32_t kFrontierMax = 1u << kFrontierDepth;
constexpr uint32_t kFrontierFloats = 12;

// Eye-ordering description of one item: eyes are bucketed by the Morton
// cell of their position inside the item's light box (cell = (x - lo) * scale,
// clamped), then by the low significant bits of their tile value (bit
// reversed), so that consecutive tasks walk nearby parts of the hierarchy and
// eyes whose shifts agree modulo a power of two (which therefore see the same
// minima on all but the smallest index blocks) run together.
struct OrderItem {
    const float* eyes;
    float lo[3], scale[3];
    uint32_t n_samples, width, pixel_base, pad;
};

// Per-item device counters, one 128-byte line per item.
// CNT_STORED / CNT_MOVED / CNT_ND are written by the compaction after the
// traversal: pairs dense at the front of the slice, pairs moved, data chunks.
enum CounterIdx {
    CNT_PAIRS = 0, CNT_CHUNKS = 1, CNT_PARTIALS = 2, CNT_STORED = 3, CNT_MOVED = 4, CNT_ND = 5, CNT_STRIDE = 16
};

// Kernel arguments of the persistent traversal launch.
struct TravArgs {
    const ItemDesc* items;
    const uint32_t* task_begin;   // n_items + 1 prefix of tasks per item
    uint32_t n_items, n_tasks;
    uint32_t* queues;             // kQueues work-queue heads, kQueueStride words apart
    uint32_t queue_begin[9];      // queue q owns tasks [queue_begin[q], queue_begin[q + 1]) ...
    const uint32_t* tile;         // 64 x 64 shifts
    unsigned long long* spill;    // per-wave spill stacks (uint2 entries)
    uint32_t spill_cap;           // entries per wave
    uint32_t stack_cap;           // LDS stack entries per wave (a multiple of 64, >= 192)
    uint32_t lds_per_wave;        // bytes
    uint32_t interleave_shift;    // ... or, if > 0, chunks q, q + 8, q + 16, ... of 2^shift tasks
    unsigned long long* stats;    // 8 counters or null
    uint32_t* error;              // set non-zero on an internal failure
};

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr uint32_t kMaxItemsPerLaunch = 1024;
// One work queue per XCD: queue q owns a contiguous slice of the task list
// (TravArgs::queue_begin), or every eighth chunk of 2^interleave_shift tasks;
// blocks are dispatched to the 8 XCDs round-robin, so block b starts on queue
// b % 8.  Slices give each L2 a contiguous (spatially ordered) part of the
// eyes; interleaved chunks keep all XCDs on the same items at a time.
constexpr uint32_t kQueues = 8;
constexpr uint32_t kQueueStride = 32;   // 128 bytes between queue heads
static_assert(sizeof(TravArgs::queue_begin) == (kQueues + 1) * sizeof(uint32_t), "one slice per queue");
// Eye ordering: counting sort over (item, Morton cell) buckets.
constexpr uint32_t kOrderMaxBuckets = 1u << 20;
constexpr uint32_t kMinChunkShift = 7;  // a chunk holds >= 128 pairs (one emission step)
constexpr uint32_t kMaxChunkShift = 13;
constexpr uint32_t kSlotShift = 28;     // stack entry: node | slot << 28
constexpr uint32_t kMaxNodes = 1u << kSlotShift;
// Lights per hierarchy: at most 2^25 - 1, so that the node records (64 bytes
// each, at most 2 n_lights of them with the unused pair slots) span less than
// 4 GiB and the walk addresses them with 32-bit offsets.
constexpr uint32_t kMaxLights = 1u << 25;

// Scratch of the allocation-free traversal (hrr_traverse_noalloc): one
// device array per GPU, 128 MiB, laid out as a header (queue heads, counters,
// status words, the item and task tables), then per-wave stack spill regions,
// the partial-chunk list, the compaction plan and the output slack.
constexpr unsigned long long kNoAllocScratchBytes = 128ull << 20;
constexpr unsigned long long kNoAllocHeaderBytes = 4096;
constexpr unsigned long long kNoAllocQueues = 0;        // kQueues * kQueueStride u32
constexpr unsigned long long kNoAllocCounters = 1024;   // CNT_STRIDE u64
constexpr unsigned long long kNoAllocMisc = 1152;       // 16 u64: [1] = error word
constexpr unsigned long long kNoAllocItem = 1280;       // one ItemDesc
constexpr unsigned long long kNoAllocTasks = 1792;      // task table {0, n_tasks}
constexpr uint32_t kNoAllocMaxChunkShift = 10;          // output chunks of at most 1024 pairs

enum StatIdx { ST_EYES = 0, ST_PAIRS, ST_VISITS, ST_RMQ, ST_LEAF, ST_SPILLS, ST_MAXSTACK, ST_N };

// Kernel-reported (1, 2) and host-detected (4) internal failures.
enum ErrCode { ERR_NONE = 0, ERR_SPILL_OVERFLOW = 1, ERR_PARTIALS_OVERFLOW = 2, ERR_UNFILLED = 4 };

static_assert(sizeof(ItemDesc) <= kNoAllocTasks - kNoAllocItem, "item table slot");
static_assert(kQueues * kQueueStride * sizeof(uint32_t) <= kNoAllocCounters, "queue heads slot");

}  // namespace hrr
