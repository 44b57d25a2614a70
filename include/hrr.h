/*
 * hrr.h -- C ABI of the MI355X (gfx950) hierarchical Russian-roulette library.
 *
 * The library culls the product set of eye vertices {e_j} x light vertices
 * {l_i} by hierarchical Russian roulette with a deterministic, per-eye rotated
 * base-2 radical inverse, following J. Pantaleoni, "Blue-Noise Dithered QMC
 * Hierarchical Russian Roulette":
 *
 *   - lights are sorted by a spatial hierarchy and the sort position is the
 *     sequence index i; every hierarchy node covers a contiguous index range
 *     [a_n, b_n) (Section 1);
 *   - eye j draws xi_ij = (Phi_2(i) + r_j) mod 1, Phi_2 the base-2 radical
 *     inverse and r_j a Cranley-Patterson rotation from a 64x64 dither tile
 *     (Section 1, equation for phi_j, and the teaser figure);
 *   - the traversal computes, at every node, v(a_n, b_n) = min over the range
 *     of xi (Section 1, equation for v(a,b); Section 2 and Algorithms 2-3 give
 *     the range-minimum method) and culls the subtree when that minimum
 *     cannot pass the node's acceptance bound;
 *   - an extra rotation psi(n) can be folded into the shift to draw several
 *     samples per pair (Section 3).
 *
 * Fixed point.  All values in [0,1) are 32-bit fixed point: x is stored as
 * floor(x * 2^32).  Phi_2(i) is bit_reverse32(i); the rotated value is
 * xi_ij = (bit_reverse32(i) + r_j) mod 2^32, exact.
 *
 * Acceptance.  For pair (j, i) the probability is p = min(1, s / d^2),
 * d^2 = (dx*dx + dy*dy) + dz*dz with d = l_i - e_j, all in IEEE binary32 with
 * each operation rounded (no fused multiply-add) and a correctly rounded
 * division.  The pair is kept when xi_ij / 2^32 < p, i.e. when
 * xi_ij < ceil(p * 2^32).  Culling never changes this set: a node is dropped
 * only when its range minimum already fails a bound that is at least the
 * probability of every light inside the node's box.
 *
 * Memory.  Pointers documented as "device" must point to device memory of the
 * context's GPU (for example torch tensors' data_ptr()); "host" pointers are
 * ordinary process memory.  The caller owns every buffer it passes in;
 * hierarchies and server results are owned by the context until freed or
 * released.  Streams are hipStream_t passed as void* (NULL = default stream).
 *
 * Errors.  Every call returns an hrr_status; nothing throws across the ABI.
 * hrr_last_error() returns a message for the last failing call on that
 * context (thread-local to the calling thread).
 *
 * Threads.  hrr_submit / hrr_poll / hrr_wait / hrr_result_copy / hrr_cancel /
 * hrr_release and the server statistics call are thread-safe (also against
 * the server's own workers).  All other calls on one context
 * must not run concurrently.
 */
#ifndef HRR_H
#define HRR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hrr_status {
    HRR_OK = 0,
    HRR_E_INVALID = 1,   /* bad argument: null pointer, size, empty range, non-finite input */
    HRR_E_NOMEM = 2,     /* device memory or the server budget cannot hold the request */
    HRR_E_OVERFLOW = 3,  /* output capacity too small; the true count is still reported */
    HRR_E_DEVICE = 4,    /* a HIP runtime call failed, or a kernel reported an internal error */
    HRR_E_NOTREADY = 5,  /* served request not finished yet */
    HRR_E_CANCELLED = 6, /* served request was cancelled */
    HRR_E_BUSY = 7       /* server not running, or queue full */
} hrr_status;

typedef struct hrr_ctx hrr_ctx;
typedef struct hrr_hierarchy hrr_hierarchy;

/* ------------------------------------------------------------------------- */
/* Context                                                                    */
/* ------------------------------------------------------------------------- */

/* Create a context on HIP device `device` with the 64x64 dither tile `tile`
 * (host, 4096 u32, row-major: entry (x mod 64) * 64 + (y mod 64) is the shift
 * of pixel (x, y)).  The tile is copied to the device.  Section 1 of the
 * paper: shifts come from a tile laid over the image plane. */
hrr_status hrr_create(int device, const uint32_t* tile, hrr_ctx** out);
void hrr_destroy(hrr_ctx* ctx);
const char* hrr_last_error(const hrr_ctx* ctx);
const char* hrr_status_string(hrr_status s);
/* Library version as 10000 * major + 100 * minor + patch. */
int hrr_version(void);

/* ------------------------------------------------------------------------- */
/* Range minimum of the rotated radical inverse                               */
/* ------------------------------------------------------------------------- */

/* All methods return the same (argmin, min).  Methods 0-3 differ in how the
 * paper's steps are scheduled on the VALU; method 4 is a different closed form
 * kept for comparison.
 *
 * Method 0 follows the paper's case analysis (Section 2: k_r in the range,
 * an index above the threshold, or none) and its two sweeps, but evaluates
 * the sweeps' candidate positions with O(1) bit tests instead of visiting
 * them one by one: both sweeps end at the highest zero bit of k_r whose
 * prefix class (k_r's bits below it, a 1 at it) meets [a,b) -- positions at
 * or above k_p, the left-to-right sweep's, outrank the right-to-left sweep's
 * below it -- and "meets [a,b)" is a closed-form membership test of a residue
 * class.  What remains a loop is Algorithm 3's walk, which refines the
 * winning class to its reflected-smallest member (and, with no class,
 * walks from a to the index with the most trailing zeros, Algorithm 1's
 * answer).  HRR_RMQ_PAPER_FULL runs the sweeps as printed, one candidate at
 * a time; all methods return the same result on every query. */
#define HRR_RMQ_PAPER 0u      /* default: the paper's case analysis and sweeps (Section 2, Algorithms 2
                                 and 3) with all candidate flip positions tested at once in bit
                                 arithmetic, then Algorithm 3's refinement of the winning prefix */
#define HRR_RMQ_DIRECT 1u     /* ablation: every step in O(1) bit arithmetic, no refinement walk */
#define HRR_RMQ_PAPER_FULL 2u /* ablation: the sweeps as loops, refining every candidate in turn */
#define HRR_RMQ_PAPER_LOOP 3u /* ablation: the sweeps as loops, refining only the candidate whose
                                 prefix class meets the range */
#define HRR_RMQ_DYADIC 4u     /* ablation, not the paper's method: the range split into maximal
                                 aligned blocks, each block's minimum in closed form */
#define HRR_RMQ_PAPER_NO_REUSE 5u /* traversal only: HRR_RMQ_PAPER, and the child that holds the
                                     parent's argmin gets its own query instead of inheriting it
                                     (ablation of that reuse); hrr_range_min rejects it */

/* For q < n: k = argmin over i in [a[q], b[q]) of (bit_reverse32(i) + r[q])
 * mod 2^32 and v = that minimum (Section 1, v(a,b); Section 2, the argmin
 * form k).  The argmin is unique (the map is a bijection).
 * a, b, r: device u32[n]; argmin_out, min_out: device u32[n].
 * A query with a[q] >= b[q] is empty: it yields argmin = b[q] and
 * min = 0xFFFFFFFF (the paper marks an invalid k with b), and is counted in
 * *n_invalid_dev (device u64, optional, added to atomically).
 * Asynchronous on `stream`; returns HRR_E_INVALID for null pointers or an
 * unknown method, HRR_E_DEVICE if the launch fails. */
hrr_status hrr_range_min(hrr_ctx* ctx, const uint32_t* a, const uint32_t* b,
                         const uint32_t* r, uint64_t n, uint32_t method,
                         uint32_t* argmin_out, uint32_t* min_out,
                         unsigned long long* n_invalid_dev, void* stream);

/* ------------------------------------------------------------------------- */
/* Light hierarchy                                                            */
/* ------------------------------------------------------------------------- */

typedef struct hrr_hierarchy_info {
    uint32_t n_lights;
    uint32_t leaf_size;
    uint32_t n_nodes;       /* node records (sibling pairs, see hrr_hierarchy_records) */
    uint32_t depth;         /* deepest internal node (root = 0) */
    uint64_t device_bytes;  /* nodes + sorted lights + permutation */
    float box[6];           /* root bounding box lo xyz, hi xyz */
    uint32_t split;         /* HRR_SPLIT_RADIX or HRR_SPLIT_POW2 */
} hrr_hierarchy_info;

/* Split rules of a hierarchy build, OR-ed into its leaf_size argument. */
#define HRR_SPLIT_RADIX 0x000u /* default: at the first index whose Morton code has the highest
                                  bit in which code[a] and code[b-1] differ (midpoint if equal) */
#define HRR_SPLIT_POW2 0x100u  /* after the largest power of two below the node's length b - a:
                                  every left child is an aligned block of 2^k indices, and for a
                                  power-of-two light count every node is one */

/* Build a binary light hierarchy (Section 1: lights sorted by a hierarchy,
 * each node a contiguous range of sequence indices).  lights_xyz: host,
 * 3*n_lights fp32.  Lights are ordered by ascending (Morton code, original
 * index); the Morton code interleaves 21-bit cell indices of x, y, z
 * (x highest) against `box` (host, 6 floats lo xyz hi xyz; NULL = unit cube;
 * coordinates outside are clamped for ordering only).  A node [a,b) with
 * b - a > leaf is split by the rule in leaf_size's flag bits (HRR_SPLIT_*).
 * leaf_size: the leaf size in [1, 8], optionally OR HRR_SPLIT_POW2; other
 * bits return HRR_E_INVALID.  Non-finite coordinates return HRR_E_INVALID.
 * The accepted pairs of a traversal do not depend on the split rule.
 * The hierarchy lives on the context's device until hrr_free_hierarchy. */
hrr_status hrr_build_hierarchy(hrr_ctx* ctx, const float* lights_xyz,
                               uint32_t n_lights, uint32_t leaf_size,
                               const float* box, hrr_hierarchy** out);
/* The same hierarchy built on the GPU (the step before the path, for light
 * caches that already live in device memory): lights_xyz_dev is device
 * memory, 3*n_lights fp32; box and leaf_size (with its split flag) as above.  The result is the
 * one hrr_build_hierarchy returns for the same lights, record for record
 * (same order, splits, exact boxes and record numbering): Morton codes,
 * a stable radix sort, one launch per tree level for the splits, then a
 * bottom-up refit.  Work is ordered on `stream`; the call returns when the
 * hierarchy is complete.  Non-finite coordinates return HRR_E_INVALID. */
hrr_status hrr_build_hierarchy_device(hrr_ctx* ctx, const float* lights_xyz_dev,
                                      uint32_t n_lights, uint32_t leaf_size,
                                      const float* box, void* stream, hrr_hierarchy** out);
hrr_status hrr_hierarchy_get_info(const hrr_hierarchy* h, hrr_hierarchy_info* out);
/* nodes_out (host, 64 bytes per record, n_nodes records).  A record is one
 * internal node [a, b) split at c: lo xyz of the left child's box, a; hi xyz
 * of the left box, c; lo xyz of the right child's box, b; hi xyz of the right
 * box, first.  Records sit in 128-byte sibling pairs: the root is record 0
 * (record 1 is unused), and a node with an internal child owns records first
 * (its left child, when internal) and first + 1 (its right child, when
 * internal); pairs follow the depth-first preorder of their owners.  first is
 * 0xFFFFFFFF when both children are leaves (at most leaf_size lights); an
 * unused record is all zero. */
hrr_status hrr_hierarchy_records(const hrr_hierarchy* h, void* nodes_out);
/* perm_out (host u32[n_lights]): perm_out[i] = original index of the light
 * with sequence index i. */
hrr_status hrr_hierarchy_permutation(const hrr_hierarchy* h, uint32_t* perm_out);
/* sorted_xyz_out (host fp32[3*n_lights]): light positions in sequence order. */
hrr_status hrr_hierarchy_sorted_lights(const hrr_hierarchy* h, float* sorted_xyz_out);
void hrr_free_hierarchy(hrr_ctx* ctx, hrr_hierarchy* h);

/* ------------------------------------------------------------------------- */
/* Traversal                                                                  */
/* ------------------------------------------------------------------------- */

/* An eye set (device memory).  Eye j (0 <= j < n) has position
 * xyz[3j..3j+2] and pixel p = pixel_base + j at (p mod width, p div width);
 * its shift is r_j = tile[(x mod 64) * 64 + (y mod 64)] + shift_offset
 * (mod 2^32).  shift_offset is an extra rotation absorbed into the shift
 * (Section 3). */
typedef struct hrr_eyes {
    const float* xyz;
    uint32_t n;
    uint32_t width;
    uint32_t shift_offset;
    uint32_t pixel_base;
} hrr_eyes;

#define HRR_F_STATS 1u      /* count node visits, range minima, leaf tests (slower) */
#define HRR_F_NO_REORDER 2u /* process eyes in index order instead of grouping them by space
                               (ablation; the result is the same either way) */
#define HRR_F_TIMING 4u     /* time the traversal kernel alone with HIP events on the
                               call's stream (hrr_stats.kernel_ms) */

typedef struct hrr_traverse_opts {
    uint32_t eyes_per_wave; /* 0 = tuned or by hierarchy size; else 1, 2, 4 or 8 eyes share one wavefront */
    uint32_t stack_entries; /* 0 = autotuned; else LDS stack entries per wave, multiple of 64 in [192, 4096] */
    uint32_t rmq_method;    /* HRR_RMQ_PAPER (default) or one of the HRR_RMQ_* ablations */
    uint32_t n_samples;     /* 0 or 1 = one sample per pair; > 1: Section 3 multi-sample */
    uint32_t psi_s0;        /* start of the golden-ratio lattice psi(n) = s0 + n * alpha mod 1 */
    uint32_t flags;         /* HRR_F_* */
} hrr_traverse_opts;

typedef struct hrr_stats {
    uint64_t eyes;          /* (virtual) eyes traversed */
    uint64_t pairs;         /* accepted pairs (true count, also past capacity) */
    uint64_t node_visits;   /* internal nodes popped (each tests both children); a
                               one-eye-per-wave walk, which starts by testing the
                               hierarchy's top (the nodes of depth 6 and the leaves
                               above), adds half a visit per tested entry */
    uint64_t rmq_calls;     /* range minima computed with the paper's method */
    uint64_t leaf_tests;    /* exact tests of lights inside leaves of several lights (or of a
                               hierarchy that is a single leaf); a one-light child is decided by
                               its bound at the parent and is not counted here */
    uint64_t spills;        /* stack chunks moved between LDS and device memory */
    uint64_t max_stack;     /* deepest stack seen by any wave */
    double kernel_ms;       /* traversal kernel duration with HRR_F_TIMING, else 0 */
} hrr_stats;

/* Hierarchical Russian roulette of every eye of `eyes` against `h`
 * (Section 1: each eye vertex draws one rotated radical-inverse number per
 * light, a pair survives with probability p, and the light hierarchy is
 * walked top-down, a node being culled when the minimum of the eye's numbers
 * over the node's index range already fails the node's acceptance bound).
 *
 * Output: the accepted pairs as u32 (j, i) in pairs_out (device,
 * 2*capacity u32), i the sequence index (see hrr_hierarchy_permutation), in
 * unspecified order.  With n_samples = N > 1 the first component is
 * j * N + n for sample n, and sample n uses r_j + psi(n).
 * weights_out (device fp32[capacity], optional): 1/p for each emitted pair,
 * the Russian-roulette weight (IEEE binary32 reciprocal of p).
 * *n_pairs (host) receives the true number of accepted pairs; if it exceeds
 * `capacity` only the first `capacity` are stored and HRR_E_OVERFLOW is
 * returned (resize and call again).  stats (host, optional) is filled when
 * opts->flags has HRR_F_STATS.  s must be finite and > 0.
 * Synchronous: returns after the kernel has finished on `stream`. */
hrr_status hrr_traverse(hrr_ctx* ctx, const hrr_hierarchy* h, const hrr_eyes* eyes,
                        float s, const hrr_traverse_opts* opts, uint32_t* pairs_out,
                        float* weights_out, uint64_t capacity, uint64_t* n_pairs,
                        hrr_stats* stats, void* stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): hrr_traverse of one
 * eye set with nothing allocated and nothing read back.  Every buffer the
 * launch needs beyond the caller's inputs and outputs comes from one fixed
 * 128 MiB scratch array per GPU, which the library holds for the life of the
 * process; the call only enqueues kernels on `stream` (no memset, no copy, no
 * host synchronization) and returns.
 *   result_dev (device, 2 u64): after the stream reaches the end of the call,
 *     result_dev[0] = the true number of accepted pairs and result_dev[1] = 0,
 *     or a non-zero internal error code (the scratch is sized so that it
 *     should never be).
 *   pairs_out / weights_out / capacity: as hrr_traverse (the first
 *     min(count, capacity) positions hold distinct accepted pairs, all of
 *     them when count <= capacity; the overflow is visible as
 *     result_dev[0] > capacity).
 *   opts: as hrr_traverse; HRR_F_STATS and HRR_F_TIMING are rejected
 *     (HRR_E_INVALID), and eyes are processed in index order.
 * The grid is cut to as many whole blocks as the scratch holds: with the
 * stack spill area sized for the hierarchy's depth, about 23 KB per wave at
 * depth 20; a hierarchy too deep for one block returns HRR_E_INVALID.
 * Output chunks hold at most 1024 pairs.  All calls on one GPU share its
 * scratch: calls that overlap in time on one GPU (several streams, several
 * threads) race and must be serialised by the caller. */
hrr_status hrr_traverse_noalloc(hrr_ctx* ctx, const hrr_hierarchy* h, const hrr_eyes* eyes, float s,
                                const hrr_traverse_opts* opts, uint32_t* pairs_out, float* weights_out,
                                uint64_t capacity, unsigned long long* result_dev, void* stream);

/* One unit of a batched launch: an eye set against one hierarchy, with its
 * own slice [out_offset, out_offset + out_capacity) of the output buffers. */
typedef struct hrr_work_item {
    const hrr_hierarchy* h;
    hrr_eyes eyes;
    float s;
    uint32_t reserved;
    uint64_t out_offset;
    uint64_t out_capacity;
} hrr_work_item;

/* Many independent (hierarchy, eye set) items in one persistent launch fed by
 * a device work queue; every item is the culling of hrr_traverse (Section 1,
 * as above) for its own eyes and hierarchy.  With opts->eyes_per_wave = 0 each item's shape is
 * resolved on its own (tuned entry of its light class or a neighbouring one,
 * else 8 eyes per wave below 2^16 lights, 4 below 2^17, then 1) and the call
 * enqueues one such launch per group of equal shape on `stream`, largest
 * hierarchies first.  items: host array of at most 1024 items (HRR_E_INVALID
 * beyond).  counts_out (host u64[n_items])
 * receives each item's true pair count; items whose count exceeds their
 * capacity store only the first out_capacity pairs and make the call return
 * HRR_E_OVERFLOW.  stats (optional) sums the work of all launches (max_stack:
 * the largest) and kernel_ms their traversal kernels.  Other arguments as
 * hrr_traverse.  Synchronous. */
hrr_status hrr_traverse_batched(hrr_ctx* ctx, const hrr_work_item* items,
                                uint32_t n_items, const hrr_traverse_opts* opts,
                                uint32_t* pairs_out, float* weights_out,
                                uint64_t* counts_out, hrr_stats* stats, void* stream);

/* ------------------------------------------------------------------------- */
/* Autotuner                                                                  */
/* ------------------------------------------------------------------------- */

typedef struct hrr_tune_result {
    uint32_t eyes_per_wave;
    uint32_t stack_entries;
    uint32_t leaf_size;
    float ms;               /* best measured time of the probe launch */
} hrr_tune_result;

/* Time candidate launch shapes (eyes per wave x stack entries) for eyes of
 * `eyes` against each hierarchy in hs[0..n_h) -- normally the same lights
 * built with different leaf sizes -- and remember the fastest for hierarchies
 * of this size class (log2 of the light count) and this eye count class.
 * Later launches with eyes_per_wave = 0 or stack_entries = 0 on hierarchies
 * of the same or a neighbouring size class use the remembered choice (the
 * nearest entry); other sizes use the built-in rule.  Candidates are tried
 * in order of preference (fewer eyes per wave first; for one eye per wave 192
 * stack entries, then 256, then 512, otherwise 512, then 256, then 1024) and a
 * later one replaces the best only when it is more than 2 % faster.  The
 * probe uses at most max_probe_eyes eyes and a scratch output the library
 * allocates.  best (host, optional) receives the winner. */
hrr_status hrr_autotune(hrr_ctx* ctx, const hrr_hierarchy* const* hs, uint32_t n_h,
                        const hrr_eyes* eyes, float s, uint32_t max_probe_eyes,
                        hrr_tune_result* best, void* stream);
/* Batched autotuner.  sets holds n_sets x n_items work items (host array,
 * set-major): the same eye sets against the same lights in every set, set q
 * built with its own leaf size (normally 1, 2, 4, 8).  For every set the
 * call times ONE launch of all its items (their own eyes, a scratch output
 * the library allocates; out_offset and out_capacity are ignored) for every
 * eyes per wave and stack candidate, in the order and with the 2 % rule of
 * hrr_autotune, and remembers the fastest (leaf size, eyes per wave, stack)
 * for the light class and eye class of every item.  Meant for the items of
 * one light class of a batch: a launch of all of them fills the GPU as the
 * batched call will, which a probe launch of a single small cache does not.
 * Later calls with eyes_per_wave = 0 or stack_entries = 0 use the remembered
 * shape as above.  best (host, optional) receives the winner.  Synchronous;
 * HRR_E_INVALID when a set's items differ from set 0 in lights or eyes, or
 * when n_items exceeds the 1024 items of one launch. */
hrr_status hrr_autotune_batched(hrr_ctx* ctx, const hrr_work_item* sets, uint32_t n_sets,
                                uint32_t n_items, hrr_tune_result* best, void* stream);
/* The leaf size the tuner prefers for hierarchies of n_lights lights (0 if none tuned). */
uint32_t hrr_tuned_leaf_size(const hrr_ctx* ctx, uint32_t n_lights);

/* ------------------------------------------------------------------------- */
/* Serving: resident hierarchies, continuous batching of eye tiles            */
/* ------------------------------------------------------------------------- */
/*
 * A request is one eye tile (a few hundred to a few hundred thousand eyes)
 * against one hierarchy already resident on the GPU, with its own additive
 * shift offset folded into every r_j (Section 3: an extra rotation is
 * absorbed into the shift) and its own s.  Its result is exactly what
 * hrr_traverse would return for the same eyes, hierarchy, width, offset and
 * s (same set of pairs; order unspecified).
 *
 * The server owns one device arena of hbm_budget_bytes, allocated at start,
 * that holds the eyes of running requests and the pairs of finished ones
 * until they are released.  max_inflight worker threads (one HIP stream
 * each) repeatedly take as many queued requests as fit (in arrival order; up
 * to max_batch_items requests and max_batch_eyes eyes, and as much arena as
 * is free; a request that does not fit is passed over by later ones that do
 * until it has waited overtake_ms) and run them as the items of one
 * persistent traversal launch per eyes-per-wave group (Section 1: every
 * request is the culling of its eye set against one hierarchy); while one
 * launch runs, newly arrived requests are batched into the next.  Each
 * request reserves output space from a running estimate of pairs per eye for
 * its hierarchy; a request whose count exceeds its reservation is re-run once
 * with the exact count reserved (hrr_ticket_info.launches > 1).
 *
 * Lifetime: a hierarchy must stay alive while requests on it are queued or
 * running.  Results hold arena space until hrr_release; a client that never
 * releases eventually blocks admission of further requests.  hrr_server_stop
 * (and hrr_destroy) invalidate every ticket and every result address.
 */

typedef struct hrr_server_config {
    uint64_t hbm_budget_bytes;   /* device arena for request eyes + results (>= 1 MiB) */
    uint32_t max_inflight;       /* launches in flight at once (one worker + stream each), 1..8 */
    uint32_t max_batch_eyes;     /* eyes per launch before a batch is closed (>= 1); every
                                    request of a launch completes with its slowest item, and
                                    the first request of a batch is always admitted, so a
                                    limit near the typical request keeps large requests
                                    alone (2^16 for requests of 2^8..2^18 eyes) */
    uint32_t max_batch_items;    /* requests per launch, 1..1024 */
    uint32_t eyes_per_wave;      /* 0 = tuned / default by hierarchy size; else 1, 2, 4 or 8 */
    float pairs_per_eye_guess;   /* output reservation per eye before any request on a
                                    hierarchy has finished (> 0; adapted online) */
    float overtake_ms;           /* a queued request that does not fit is skipped by later
                                    requests that do, until it has waited this long; from then
                                    on nothing behind it is admitted until it runs (>= 0,
                                    finite; 0 = strict FIFO admission) */
} hrr_server_config;

typedef struct hrr_server_stats {
    uint64_t submitted, completed, cancelled, rejected, launches, retries;
    uint64_t pairs;                 /* pairs of completed requests */
    double p50_ms, p99_ms, mean_ms; /* submit -> complete latency of completed requests */
    double busy_s;                  /* wall time with at least one launch in flight */
    uint64_t peak_bytes;            /* high-water mark of the arena in use */
} hrr_server_stats;

typedef struct hrr_ticket_info {
    double submit_s, start_s, done_s;  /* host monotonic clock (seconds): submit, first
                                          launch enqueued, result complete */
    uint64_t n_pairs;
    uint32_t launches;                 /* > 1 if the request was re-run after an output overflow */
} hrr_ticket_info;

/* Start the serving workers and allocate the arena.  HRR_E_BUSY if a server
 * already runs on ctx, HRR_E_INVALID for a bad config, HRR_E_NOMEM if the
 * arena cannot be allocated. */
hrr_status hrr_server_start(hrr_ctx* ctx, const hrr_server_config* cfg);
/* Stop: queued requests are cancelled, running launches finish, then the
 * workers exit and the arena is freed.  HRR_OK also if no server runs. */
hrr_status hrr_server_stop(hrr_ctx* ctx);
/* Queue a request.  eyes_xyz: host, 3*n_eyes fp32, copied before the call
 * returns (finite values only).  width: pixels per row of the tile, as in
 * hrr_eyes.  shift_offset: added to every r_j mod 2^32.  s: finite, > 0.
 * *ticket (host) receives an id unique within this server.  HRR_E_NOMEM (and
 * the request counted as rejected) if the tile could never fit the arena,
 * HRR_E_BUSY if no server runs, HRR_E_INVALID for bad arguments. */
hrr_status hrr_submit(hrr_ctx* ctx, const hrr_hierarchy* h, const float* eyes_xyz,
                      uint32_t n_eyes, uint32_t width, uint32_t shift_offset,
                      float s, uint64_t* ticket);
/* HRR_E_NOTREADY while queued or running.  When complete: HRR_OK, *pairs_dev
 * (host variable) = device address of the request's n_pairs (j, i) u32 pairs
 * inside the arena (NULL if none; valid until hrr_release), *n_pairs = their
 * count.  HRR_E_CANCELLED for a cancelled request; the failing status (with
 * hrr_last_error set) for one that failed; HRR_E_INVALID for an unknown ticket.
 * pairs_dev, n_pairs and info may each be NULL. */
hrr_status hrr_poll(hrr_ctx* ctx, uint64_t ticket, const uint32_t** pairs_dev,
                    uint64_t* n_pairs, hrr_ticket_info* info);
/* Block until the request is no longer queued or running, or timeout_ms
 * elapses (then HRR_E_NOTREADY).  Returns what hrr_poll would. */
hrr_status hrr_wait(hrr_ctx* ctx, uint64_t ticket, uint32_t timeout_ms);
/* Copy a complete request's pairs to dst (device, 2*capacity u32) on
 * `stream` and wait for the copy.  HRR_E_OVERFLOW (first capacity pairs
 * copied) if capacity is smaller than the count; other statuses as hrr_poll. */
hrr_status hrr_result_copy(hrr_ctx* ctx, uint64_t ticket, uint32_t* dst, uint64_t capacity,
                           void* stream);
/* Cancel a queued request (HRR_OK).  HRR_E_BUSY if it is already running or
 * complete, HRR_E_INVALID for an unknown ticket. */
hrr_status hrr_cancel(hrr_ctx* ctx, uint64_t ticket);
/* Forget a complete, failed or cancelled request and free its result
 * memory.  HRR_E_BUSY while it is queued or running. */
hrr_status hrr_release(hrr_ctx* ctx, uint64_t ticket);
/* Counters since hrr_server_start.  HRR_E_BUSY if no server runs. */
hrr_status hrr_server_get_stats(hrr_ctx* ctx, hrr_server_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* HRR_H */
