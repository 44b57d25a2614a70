// hrr_kernels.hip -- gfx950 kernels for hierarchical Russian roulette with a
// rotated base-2 radical inverse (Pantaleoni, "Blue-Noise Dithered QMC
// Hierarchical Russian Roulette").
//
//   rmq_kernel       range-minimum queries (Section 1, v(a,b); Section 2,
//                    Algorithms 2-3), eight per thread, streaming u32 arrays.
//   traverse_kernel  persistent wavefronts that pull (item, eye group) tasks
//                    from eight per-XCD work queues and cull every eye's pairs
//                    by a top-down walk of its item's light hierarchy
//                    (Section 1).
//   around it        the eye order (bucket keys, a multi-block scan, scatter)
//                    and the compaction that makes every item's output dense
//                    after a traversal (compact_plan_kernel,
//                    compact_move_kernel).
//
// Wavefront design.  One wave owns a group of 1..8 eyes.  Its stack of
// pending hierarchy nodes lives in LDS and is shared by the 64 lanes: each
// iteration pops up to 64 nodes (one per lane), each lane obtains its node's
// 64-byte record (both children's boxes; neighbouring lanes fetch their two
// records as shared 32-byte halves), derives the children's range minima
// -- the child that contains the parent's argmin inherits it, the other needs
// one range-minimum query -- bounds both children, and the survivors are
// pushed back with ballot/mbcnt compaction.  Leaves with one light are tested
// exactly at the parent; accepted pairs go straight from the lanes into an
// output chunk the wave owns (one atomic per chunk of thousands of pairs, see
// emit2).  The stack spills in halves to a per-wave region
// of device memory when it would overflow LDS; its size is bounded by
// 128 entries per tree level (see stack_spill).
//
// Floating point: every acceptance probability is computed in binary32 with
// separately rounded operations (no contraction) and an IEEE division, so that
// a one-light leaf's test is bit-identical to the all-pairs definition.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hrr_compact.hpp"
#include "hrr_rmq.hpp"
#include "hrr_scan.hpp"
#include "hrr_types.hpp"

#pragma clang fp contract(off)

namespace hrr {

// ---------------------------------------------------------------------------
// wavefront helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// lanes (of the active ones) whose p holds; the builtin takes the condition as
// a lane mask directly (the int-valued __ballot materialises it in a register
// and compares it again)
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// number of set bits of m in lanes below this one
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ float unif(float x) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(x)));
}

// Order LDS traffic of one wave across lanes: the wave executes in lock step
// and LDS serves one wave's requests in order, so only compiler reordering
// has to be prevented.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// acceptance bound
// ---------------------------------------------------------------------------

// squared distance from the eye to the box [lo, hi] (0 inside), summed
// (x + y) + z; for a one-point box this is the pair's own d^2 bit for bit.
// Hierarchy records and lights always live in device global memory; loading
// them through an address-space-1 pointer makes the compiler emit global
// loads instead of generic (flat) ones, which would also tie up the LDS
// counter that the stack operations wait on.
typedef float f32x4 __attribute__((ext_vector_type(4)));
// DPP control: quad_perm(1, 0, 3, 2) -- every lane reads its pair partner.
constexpr int kDppSwapPairs = 0xB1;

__device__ __forceinline__ float swap_pairs(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), kDppSwapPairs, 0xF, 0xF, false));
}
__device__ __forceinline__ float4 swap_pairs(float4 v) {
    return make_float4(swap_pairs(v.x), swap_pairs(v.y), swap_pairs(v.z), swap_pairs(v.w));
}

__device__ __forceinline__ float4 load_global4(const float4* p, uint32_t i) {
    const f32x4 v = ((const __attribute__((address_space(1))) f32x4*)(p))[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float box_d2(float ex, float ey, float ez, float lx, float ly, float lz,
                                        float hx, float hy, float hz) {
    const float dx = fmaxf(fmaxf(lx - ex, ex - hx), 0.0f);
    const float dy = fmaxf(fmaxf(ly - ey, ey - hy), 0.0f);
    const float dz = fmaxf(fmaxf(lz - ez, ez - hz), 0.0f);
    const float x2 = dx * dx;
    const float y2 = dy * dy;
    const float z2 = dz * dz;
    return (x2 + y2) + z2;
}

// p = min(1, (s / d2) * mult).  mult = 1 for an exact one-light test; for a
// multi-light box mult = 1 + 2^-20, a safety factor on the bound (every step
// above is monotone, so the box bound is already >= each light's p).
__device__ __forceinline__ float accept_p(float s, float d2, float mult) {
    float q = s / d2;
    q = q * mult;
    return fminf(q, 1.0f);
}

// Russian roulette with a 32-bit fixed-point random number: keep iff
// v / 2^32 < p, i.e. v < ceil(p * 2^32) (exact: the scaling is a power of 2).
__device__ __forceinline__ bool keeps(uint32_t v, float p) {
    if (p >= 1.0f) return true;
    return v < (uint32_t)ceilf(p * 4294967296.0f);
}

constexpr float kBoxMargin = 1.0f + 0x1p-20f;

// ---- product-form keep test ------------------------------------------------
//
// With x = fl(s / d2) 2^32 the pair is kept iff v < x (v is an integer, so
// v < ceil(x) is the same as v < x).  Instead of the IEEE quotient (about ten
// VALU instructions) the kernel compares the product P = fl(fl(v) d2) with
// two per-item constants, t_cull >= S (1 + 2^-18) and t_keep <= S (1 - 2^-18),
// S = s 2^32.  Each of fl(v), the product and fl(s / d2) has a relative error
// of at most 2^-24, so
//   P > t_cull  implies  v > (s / d2) 2^32 (1 + 2^-24) >= x   (culled), and
//   P < t_keep  implies  v < (s / d2) 2^32 (1 - 2^-24) <= x   (kept).
// For d2 <= s (p = 1) the first never holds, since fl(v) d2 <= 2^32 s.
// A box at squared distance d2 bounds every light inside it (each light's
// squared distance, computed with the same monotone binary32 steps, is at
// least d2), so "P > t_cull" culls a whole subtree safely; anything else
// keeps the box.  A one-light test whose product falls between the two
// constants (a relative band of about 2^-17 around the threshold) decides
// with the IEEE quotient.  The product form is used only for
// d2 <= d2_fast = s 2^60 (s / d2 stays a normal number, P cannot overflow);
// beyond it, and for s outside [2^-60, 2^60], the IEEE path decides.

// Product-form part of the keep test, with selects only: sets `keep` and
// returns false when decided, returns true when the IEEE path must decide.
__device__ __forceinline__ bool rr_fast(uint32_t v, const ItemDesc& D, float d2, bool exact, bool& keep) {
    const float P = (float)v * d2;
    const bool fast = d2 <= D.d2_fast;
    const bool cull = fast && P > D.t_cull;
    const bool sure = fast && (!exact || P < D.t_keep);
    keep = !cull;
    return !cull && !sure;
}

// Keep test of value v at squared distance d2.
//   exact = true : one light; the result equals keeps(v, min(1, s / d2)).
//   exact = false: a box; false only if no light in the box can keep v.
__device__ __forceinline__ bool rr_test(uint32_t v, const ItemDesc& D, float d2, bool exact) {
    if (d2 <= D.d2_fast) {
        const float P = (float)v * d2;
        if (P > D.t_cull) return false;
        if (!exact || P < D.t_keep) return true;
    }
    return keeps(v, accept_p(D.s, d2, exact ? 1.0f : kBoxMargin));
}

// Fixed-point golden-ratio lattice alpha = round(2^32 (sqrt(5) - 1) / 2).
constexpr uint32_t kGoldenAlpha = 2654435769u;

// ---------------------------------------------------------------------------
// range-minimum kernel
// ---------------------------------------------------------------------------

template <int METHOD>
__device__ __forceinline__ void rmq_one(uint32_t a, uint32_t b, uint32_t R, uint32_t& k, uint32_t& v,
                                        uint32_t& bad) {
    if (a < b) {
        k = rmq<METHOD>(a, b, threshold_index(R));
        v = rotated(k, R);
    } else {
        k = b;
        v = 0xFFFFFFFFu;
        ++bad;
    }
}

// Four queries per lane per step through 16-byte loads when every array is
// 16-byte aligned (vec != 0); the scalar tail and unaligned arrays go one
// query at a time.  Every array is touched once, so loads and stores are
// non-temporal (2^28 queries: 0.895 ms against 0.970 ms with ordinary ones;
// non-temporal stores alone 0.96 ms, loads alone 0.98 ms).
constexpr uint32_t kRmqGroups = 1;   // 4-query groups per thread (2^28 queries: 1: 0.925 ms, 2: 0.941, 4: 0.955)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 load_stream4(const uint4* p, uint64_t i) {
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p) + i);
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void store_stream4(uint4* p, uint64_t i, uint4 x) {
    const u32x4 v = {x.x, x.y, x.z, x.w};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(p) + i);
}

template <int METHOD>
__global__ __launch_bounds__(256) void rmq_kernel(const uint32_t* __restrict__ A, const uint32_t* __restrict__ B,
                                                  const uint32_t* __restrict__ R, uint64_t n,
                                                  uint32_t* __restrict__ K, uint32_t* __restrict__ V,
                                                  unsigned long long* __restrict__ n_bad, int vec) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    uint64_t done = 0;
    if (vec) {
        const uint64_t n4 = n >> 2;
        const uint4* A4 = reinterpret_cast<const uint4*>(A);
        const uint4* B4 = reinterpret_cast<const uint4*>(B);
        const uint4* R4 = reinterpret_cast<const uint4*>(R);
        uint4* K4 = reinterpret_cast<uint4*>(K);
        uint4* V4 = reinterpret_cast<uint4*>(V);
        // kRmqGroups 4-query groups per thread, all loads first; block b
        // covers groups [b, b + 1) x blockDim x kRmqGroups, so every load and
        // store instruction of a block is contiguous
        for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x * kRmqGroups; base < n4;
             base += stride * kRmqGroups) {
            uint4 a[kRmqGroups], b[kRmqGroups], r[kRmqGroups];
#pragma unroll
            for (uint32_t g = 0; g < kRmqGroups; ++g) {
                const uint64_t q = base + g * blockDim.x + threadIdx.x;
                if (q < n4) {
                    a[g] = load_stream4(A4, q);
                    b[g] = load_stream4(B4, q);
                    r[g] = load_stream4(R4, q);
                }
            }
#pragma unroll
            for (uint32_t g = 0; g < kRmqGroups; ++g) {
                const uint64_t q = base + g * blockDim.x + threadIdx.x;
                if (q < n4) {
                    uint4 k, v;
                    rmq_one<METHOD>(a[g].x, b[g].x, r[g].x, k.x, v.x, bad);
                    rmq_one<METHOD>(a[g].y, b[g].y, r[g].y, k.y, v.y, bad);
                    rmq_one<METHOD>(a[g].z, b[g].z, r[g].z, k.z, v.z, bad);
                    rmq_one<METHOD>(a[g].w, b[g].w, r[g].w, k.w, v.w, bad);
                    store_stream4(K4, q, k);
                    store_stream4(V4, q, v);
                }
            }
        }
        done = n4 << 2;
    }
    for (uint64_t q = done + tid; q < n; q += stride) {
        uint32_t k, v;
        rmq_one<METHOD>(__builtin_nontemporal_load(A + q), __builtin_nontemporal_load(B + q),
                        __builtin_nontemporal_load(R + q), k, v, bad);
        __builtin_nontemporal_store(k, K + q);
        __builtin_nontemporal_store(v, V + q);
    }
    if (n_bad) {
        const uint64_t m = ballot(bad != 0);
        if (m) {
            // wave-reduce the few non-zero counts
            uint32_t tot = bad;
            for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
            if (lane_id() == 0) atomicAdd(n_bad, (unsigned long long)tot);
        }
    }
}


// ---------------------------------------------------------------------------
// traversal kernel
// ---------------------------------------------------------------------------

struct EyeState {
    float ex, ey, ez;
    uint32_t R;     // rotation r_j (+ extras), fixed point
    uint32_t kr;    // threshold index Phi_2^{-1}(1 - r_j)
    uint32_t u;     // virtual eye index emitted as the pair's first component
};

// Record fetch of the walk.  One eye per wave: the four lanes of a quad
// fetch their four 64-byte records as 16-byte quarters, so every load of a
// quad touches a single record, and the quarters go straight from memory into
// LDS (global_load_lds_dwordx4 writes lane L's 16 bytes at the instruction's
// LDS base + 16 L), where each lane reads its own record back.  The area holds
// one 1040-byte slab per record slot t of a quad: 1024 bytes for the 64 lanes
// and 16 bytes that stagger the slabs over the LDS banks.  Several eyes per
// wave (which keep their eyes in LDS and run at lower occupancy): lanes 2i,
// 2i + 1 fetch both of their records as 32-byte halves and swap halves with a
// DPP lane exchange.
constexpr uint32_t kSlab = 1040;
constexpr uint32_t kXposeBytes = 4 * kSlab;
template <int EPW>
struct FetchOf {
    static constexpr bool quad_lds = EPW == 1;
};

constexpr uint32_t kEyeTableBytes = 8 * 8 * sizeof(uint32_t);   // 8 words per eye slot

// LDS of one wave: the stack ring, then the eye table (several eyes per wave)
// or the record area (one eye per wave).
struct WaveLds {
    uint2* stack;
    uint32_t* eyes;   // 8 words per slot
    unsigned char* xpose;
};

// ---- per-wave stack in LDS with spill to device memory ----
//
// Logical positions [0, g) live in the wave's spill region, [g, g + n) in an
// LDS ring of cap entries (cap a multiple of 64, at least 192); the entry at
// logical position g sits in ring slot `base`, the next ones follow it round
// the ring.  Stack memory moves in units of 64 entries, one per lane, so a
// lane always re-reads exactly what it wrote.  One unit is always enough:
// after a pop the ring holds at most cap - 64 entries (or none), a step pushes
// at most 128, so an overflowing push needs at most 64 more slots, and it
// only overflows when the ring holds more than cap - 128 >= 64 entries.
//
// Size bound.  Pops take the top <= 64 entries (lanes in stack order) and
// each pushes its surviving children next to each other, so depths never
// decrease from bottom to top.  A pop that reaches an entry of depth d - 1
// also removes every entry of depth >= d above it; hence all entries of depth
// d come from one pop and number at most 128, and the stack never holds more
// than 128 * (max depth + 1) entries.
constexpr uint32_t kStackUnit = 64;

struct StackState {
    uint32_t g;      // entries in device memory
    uint32_t n;      // entries in LDS
    uint32_t base;   // ring slot of logical position g
    uint32_t max_total;
    uint32_t spills;
};

// ring slot of x in [0, 2 cap): x or x - cap
__device__ __forceinline__ uint32_t ring(uint32_t x, uint32_t cap) { return min(x, x - cap); }

__device__ __forceinline__ bool stack_spill(StackState& st, const WaveLds& L, uint2* spill, uint32_t cap,
                                            uint32_t spill_cap, uint32_t* err) {
    if (st.g + kStackUnit > spill_cap) {
        if (lane_id() == 0) atomicOr(err, (uint32_t)ERR_SPILL_OVERFLOW);
        return false;
    }
    wave_sync();
    spill[st.g + lane_id()] = L.stack[ring(st.base + lane_id(), cap)];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    st.g += kStackUnit;
    st.n -= kStackUnit;
    st.base = ring(st.base + kStackUnit, cap);
    ++st.spills;
    return true;
}

__device__ __forceinline__ void stack_refill(StackState& st, const WaveLds& L, const uint2* spill, uint32_t cap) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    st.g -= kStackUnit;
    st.base = ring(st.base + cap - kStackUnit, cap);
    L.stack[ring(st.base + lane_id(), cap)] = spill[st.g + lane_id()];
    wave_sync();
    st.n += kStackUnit;
    ++st.spills;
}

// ---- pair output in per-wave chunks ----
//
// An item's output positions are cut into chunks of 2^chunk_shift pairs.  A
// wave takes a whole chunk from the item's chunk counter (one device-scope
// atomic per chunk instead of one per flush: a single address serialises
// those atomics) and writes its accepted pairs into it directly from the
// lanes, compacted with ballot/mbcnt.  A wave leaving an item publishes its
// partly filled chunk as (chunk, fill) (the launch bounds how often a wave can
// leave an item), so that the compaction kernels can move the pairs found
// past the final count into those holes.  Positions at or
// past the caller's capacity go to a library slack area, positions past that
// are dropped (the count stays exact).
constexpr unsigned long long kNoChunk = ~0ull;

struct OutState {
    unsigned long long chunk;   // current chunk, or kNoChunk
    unsigned long long count;   // pairs emitted for the current item
    uint2* wp;                  // first pair slot of the chunk when it lies wholly in one buffer
    float* ww;                  // same for the weights
    uint32_t fill;
};

__device__ __forceinline__ unsigned long long uni64(unsigned long long x) {
    return ((unsigned long long)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

__device__ __forceinline__ unsigned long long alloc_chunk(const ItemDesc& D) {
    unsigned long long c = 0;
    if (lane_id() == 0) c = atomicAdd(D.counters + CNT_CHUNKS, 1ull);
    return uni64(c);
}

// Pairs and weights are written once and not read again by the launch:
// non-temporal stores keep them from displacing node records in the caches
// (frame 144.5 -> 141.9 ms, 256-cache batch 57.2 -> 55.8 ms).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Stores go through global (address-space 1) pointers: a generic pointer
// makes them flat stores, which also count against the LDS counter that every
// stack access of the walk waits on.
typedef __attribute__((address_space(1))) u32x2 g_u32x2;
typedef __attribute__((address_space(1))) float g_f32;

__device__ __forceinline__ void put_pair(uint2* p, unsigned long long i, uint2 x) {
    const u32x2 v = {x.x, x.y};
    __builtin_nontemporal_store(v, (g_u32x2*)(p) + i);
}

__device__ __forceinline__ void put_weight(float* p, unsigned long long i, float w) {
    __builtin_nontemporal_store(w, (g_f32*)(p) + i);
}

// Make `c` the current chunk; direct pointers when the whole chunk lies below
// the capacity or inside the slack area (a chunk that straddles the capacity
// or the end of the slack takes the per-pair path).
template <bool W>
__device__ __forceinline__ void set_chunk(OutState& O, const ItemDesc& D, unsigned long long c) {
    O.chunk = c;
    O.wp = nullptr;
    O.ww = nullptr;
    if (c == kNoChunk) return;
    const unsigned long long p0 = c << D.chunk_shift;
    const unsigned long long C = 1ull << D.chunk_shift;
    if (p0 + C <= D.capacity) {
        O.wp = reinterpret_cast<uint2*>(D.pairs) + p0;
        if (W) O.ww = D.weights + p0;
    } else if (p0 >= D.capacity && p0 - D.capacity + C <= D.slack) {
        O.wp = reinterpret_cast<uint2*>(D.slack_pairs) + (p0 - D.capacity);
        if (W) O.ww = D.slack_weights + (p0 - D.capacity);
    }
}

template <bool W>
__device__ __forceinline__ void store_pair(const ItemDesc& D, unsigned long long p, uint2 pr, float w) {
    if (p < D.capacity) {
        put_pair(reinterpret_cast<uint2*>(D.pairs), p, pr);
        if (W) put_weight(D.weights, p, w);
    } else if (p - D.capacity < D.slack) {
        const unsigned long long q = p - D.capacity;
        put_pair(reinterpret_cast<uint2*>(D.slack_pairs), q, pr);
        if (W) put_weight(D.slack_weights, q, w);
    }
}

// Emit up to two pairs per lane, compacted over the wave (uniform control
// flow): every lane's first pair, then every lane's second, so that each of the
// two store instructions writes one contiguous run.  (With a lane's two pairs
// side by side, both instructions wrote every cache line in part: 1.52 bytes
// reached memory per byte of pairs.)  A step holds at most 128 pairs and a
// chunk at least 128, so a step crosses at most one chunk boundary.
template <bool W>
__device__ __forceinline__ void emit2(OutState& O, const ItemDesc& D, bool e0, uint2 p0, float w0, bool e1, uint2 p1,
                                      float w1) {
    const uint64_t m0 = ballot(e0), m1 = ballot(e1);
    const uint32_t cnt = (uint32_t)(__popcll(m0) + __popcll(m1));
    if (cnt == 0) return;
    if (D.capacity == 0) {   // counting launch: nothing is stored
        O.count += cnt;
        return;
    }
    if (O.chunk == kNoChunk) {
        set_chunk<W>(O, D, alloc_chunk(D));
        O.fill = 0;
    }
    const uint32_t shift = D.chunk_shift;
    const uint32_t C = 1u << shift;
    const uint32_t pos0 = O.fill + count_below(m0);
    const uint32_t pos1 = O.fill + (uint32_t)__popcll(m0) + count_below(m1);
    if (O.wp && uni(O.fill) + cnt <= C) {
        if (e0) {
            put_pair(O.wp, pos0, p0);
            if (W) put_weight(O.ww, pos0, w0);
        }
        if (e1) {
            put_pair(O.wp, pos1, p1);
            if (W) put_weight(O.ww, pos1, w1);
        }
        O.fill += cnt;
        O.count += cnt;
        if (O.fill == C) set_chunk<W>(O, D, kNoChunk);
        return;
    }
    unsigned long long next = kNoChunk;
    if (O.fill + cnt > C) next = alloc_chunk(D);
    const unsigned long long base = O.chunk << shift;
    const unsigned long long nbase = next << shift;
    if (e0) store_pair<W>(D, pos0 < C ? base + pos0 : nbase + (pos0 - C), p0, w0);
    if (e1) store_pair<W>(D, pos1 < C ? base + pos1 : nbase + (pos1 - C), p1, w1);
    O.count += cnt;
    O.fill += cnt;
    if (O.fill >= C) {
        O.fill -= C;
        set_chunk<W>(O, D, next);
    }
}

// A wave leaves an item: publish its count and its partly filled chunk.
__device__ __forceinline__ void close_item(OutState& O, const ItemDesc& D, uint32_t* err) {
    if (lane_id() == 0) {
        if (O.chunk != kNoChunk && O.fill > 0) {
            const unsigned long long at = atomicAdd(D.counters + CNT_PARTIALS, 1ull);
            if (at < D.partial_cap) {
                D.partials[2 * at] = O.chunk;
                D.partials[2 * at + 1] = O.fill;
            } else {
                atomicOr(err, (uint32_t)ERR_PARTIALS_OVERFLOW);
            }
        }
        if (O.count) atomicAdd(D.counters + CNT_PAIRS, O.count);
    }
    O.chunk = kNoChunk;
    O.wp = nullptr;
    O.ww = nullptr;
    O.fill = 0;
    O.count = 0;
}

__device__ __forceinline__ EyeState load_eye(const ItemDesc& D, const uint32_t* tile, uint32_t u) {
    EyeState E;
    const uint32_t ns = D.n_samples;
    const uint32_t j = ns > 1 ? u / ns : u;
    const uint32_t n = ns > 1 ? u - j * ns : 0u;
    E.ex = D.eyes[3u * j + 0];
    E.ey = D.eyes[3u * j + 1];
    E.ez = D.eyes[3u * j + 2];
    const uint32_t pix = D.pixel_base + j;
    const uint32_t x = pix % D.width;
    const uint32_t y = pix / D.width;
    uint32_t R = tile[(x & 63u) * 64u + (y & 63u)] + D.shift_offset;
    if (ns > 1) R += D.psi_s0 + n * kGoldenAlpha;
    E.R = R;
    E.kr = threshold_index(R);
    E.u = u;
    return E;
}

// Exact per-light tests of the leaf children that survived their box bound
// and hold more than one light.  Lane-local loops; emissions are compacted
// every step.
template <bool W>
__device__ __forceinline__ void leaf_lights(OutState& O, const ItemDesc& D, const EyeState& E, uint32_t la,
                                            uint32_t ln, uint32_t ra, uint32_t rn, uint64_t& tests) {
    const uint32_t total = ln + rn;
    for (uint32_t q = 0; ballot(q < total); ++q) {
        const bool act = q < total;
        bool emit = false;
        uint32_t i = 0;
        float w = 0.0f;
        if (act) {
            i = q < ln ? la + q : ra + (q - ln);
            const float4 P = load_global4(reinterpret_cast<const float4*>(D.lights), i);
            const float d2 = box_d2(E.ex, E.ey, E.ez, P.x, P.y, P.z, P.x, P.y, P.z);
            emit = rr_test(rotated(i, E.R), D, d2, true);
            if (W) w = 1.0f / accept_p(D.s, d2, 1.0f);
            ++tests;
        }
        emit2<W>(O, D, emit, make_uint2(E.u, i), w, false, make_uint2(0u, 0u), 0.0f);
    }
}

// Occupancy.  With one eye per wave the LDS holds 7 waves per SIMD (a wave
// takes its stack ring and the 4160-byte record area, 5696 bytes at the
// default 192 entries; 28 waves fill 160 KB), so the register budget is the
// one of 7 waves (72 VGPRs): asking for 8 only forced spills (frame
// 108.6 -> 108.3 ms with 7).  Several eyes per wave use little LDS and run
// at whatever occupancy their registers allow.
template <int EPW, int METHOD, bool STATS, bool W>
__global__ __launch_bounds__(kWave * kWavesPerBlock)
__attribute__((amdgpu_waves_per_eu(EPW == 1 ? 7 : 1, 8)))
void traverse_kernel(TravArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    // dynamic LDS: task table (n_items + 1 entries, padded to 16 bytes), then one area per wave
    uint32_t* task_begin_lds = reinterpret_cast<uint32_t*>(smem);
    for (uint32_t t = threadIdx.x; t <= A.n_items; t += blockDim.x) task_begin_lds[t] = A.task_begin[t];
    __syncthreads();
    unsigned char* wave_area = smem + (((size_t)A.n_items + 1u) * sizeof(uint32_t) + 15u) / 16u * 16u;

    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t wave_gid = blockIdx.x * kWavesPerBlock + wv;
    const uint32_t cap = A.stack_cap;

    unsigned char* base = wave_area + (size_t)wv * A.lds_per_wave;
    WaveLds L;
    L.stack = reinterpret_cast<uint2*>(base);
    L.eyes = reinterpret_cast<uint32_t*>(base + (size_t)cap * sizeof(uint2));
    L.xpose = base + (size_t)cap * sizeof(uint2);   // one eye per wave: no eye table
    // the record area's LDS address, wave-uniform (the destination of the
    // record fetch must be a scalar)
    const uint32_t xlds = uni((uint32_t)(size_t)(__attribute__((address_space(3))) unsigned char*)L.xpose);
    uint2* spill = reinterpret_cast<uint2*>(A.spill) + (size_t)wave_gid * A.spill_cap;

    uint64_t st_eyes = 0, st_visits = 0, st_rmq = 0, st_leaf = 0, st_spills = 0;
    uint32_t st_maxstack = 0;

    uint32_t cur = 0xFFFFFFFFu;
    ItemDesc D;
    OutState O;
    O.chunk = kNoChunk;
    O.wp = nullptr;
    O.ww = nullptr;
    O.fill = 0;
    O.count = 0;

    // work queues: start on this block's XCD queue, move on when it is empty
    uint32_t q = blockIdx.x % kQueues;
    uint32_t queues_left = kQueues;
    for (;;) {
        uint32_t i = 0;
        if (lane == 0) i = atomicAdd(A.queues + q * kQueueStride, 1u);
        i = uni(i);
        // the i-th task of queue q; increasing in i, so the first one past the
        // end means the queue is exhausted
        const uint32_t sh = A.interleave_shift;
        const uint64_t t64 = sh ? (((((uint64_t)(i >> sh)) * kQueues + q) << sh) | (i & ((1u << sh) - 1u)))
                                : (uint64_t)A.queue_begin[q] + i;
        const uint64_t end = sh ? (uint64_t)A.n_tasks : (uint64_t)A.queue_begin[q + 1];
        if (t64 >= end) {
            if (--queues_left == 0) break;
            q = (q + 1) % kQueues;
            continue;
        }
        const uint32_t t = (uint32_t)t64;

        // item of task t: largest k with task_begin[k] <= t
        uint32_t lo = 0, hi = A.n_items;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (task_begin_lds[mid] <= t) lo = mid; else hi = mid;
        }
        const uint32_t it = uni(lo);
        if (it != cur) {
            if (cur != 0xFFFFFFFFu) close_item(O, D, A.error);
            cur = it;
            D = A.items[it];
        }
        const uint32_t u0 = (t - D.task_begin) * EPW;
        const uint32_t cnt = min((uint32_t)EPW, D.n_virtual - u0);
        const uint32_t N = D.n_lights;
        const uint32_t leaf = D.leaf_size;
        const float s = D.s;

        // -------- eyes of this task --------
        EyeState E0;   // EPW == 1: wave-uniform eye
        if (EPW == 1) {
            const uint32_t u = D.order ? uni(D.order[u0]) : u0;
            E0 = load_eye(D, A.tile, u);
            E0.ex = unif(E0.ex); E0.ey = unif(E0.ey); E0.ez = unif(E0.ez);
            E0.R = uni(E0.R); E0.kr = uni(E0.kr);
        } else {
            if (lane < cnt) {
                const uint32_t u = D.order ? D.order[u0 + lane] : u0 + lane;
                const EyeState e = load_eye(D, A.tile, u);
                uint32_t* w = L.eyes + lane * 8u;
                w[0] = __float_as_uint(e.ex); w[1] = __float_as_uint(e.ey); w[2] = __float_as_uint(e.ez);
                w[3] = e.R; w[4] = e.kr; w[5] = e.u;
            }
            wave_sync();
        }
        if (STATS) st_eyes += cnt;

        StackState S;
        S.g = 0; S.n = 0; S.base = 0; S.max_total = 0; S.spills = 0;

        // -------- roots --------
        {
            const bool act = lane < cnt;
            EyeState E = E0;
            if (EPW > 1 && act) {
                const uint32_t* w = L.eyes + lane * 8u;
                E.ex = __uint_as_float(w[0]); E.ey = __uint_as_float(w[1]); E.ez = __uint_as_float(w[2]);
                E.R = w[3]; E.kr = w[4]; E.u = w[5];
            }
            if (D.n_nodes == 0) {
                // the whole light set is one leaf: exact tests of its <= 8 lights
                uint64_t tests = 0;
                if (EPW == 1) {
                    // spread the lights of the single eye over the lanes
                    const bool a1 = lane < N;
                    bool emit = false;
                    float w = 0.0f;
                    if (a1) {
                        const float4 P = load_global4(reinterpret_cast<const float4*>(D.lights), lane);
                        const float d2 = box_d2(E.ex, E.ey, E.ez, P.x, P.y, P.z, P.x, P.y, P.z);
                        emit = rr_test(rotated(lane, E.R), D, d2, true);
                        if (W) w = 1.0f / accept_p(s, d2, 1.0f);
                        ++tests;
                    }
                    emit2<W>(O, D, emit, make_uint2(E.u, lane), w, false, make_uint2(0u, 0u), 0.0f);
                } else {
                    leaf_lights<W>(O, D, E, 0u, act ? N : 0u, 0u, 0u, tests);
                }
                if (STATS) st_leaf += tests;
                continue;
            }
            if (EPW == 1 && D.n_frontier > 0) {
                // one eye per wave: lane t tests entry t of the hierarchy's top
                // (its range minimum, its box; a leaf entry is tested as a leaf
                // child is), surviving nodes are pushed in index order
                const bool fa = lane < D.n_frontier;
                uint32_t a = 0, b = 1, rec = 0xFFFFFFFFu;
                float4 f0 = make_float4(0.f, 0.f, 0.f, 0.f), f1 = f0;
                if (fa) {
                    const float4* f = reinterpret_cast<const float4*>(D.frontier) + 3u * lane;
                    f0 = f[0];
                    f1 = f[1];
                    a = __float_as_uint(f0.w);
                    b = __float_as_uint(f1.w);
                    rec = __float_as_uint(f[2].x);
                }
                const uint32_t n = b - a;
                uint32_t k = a;
                if (METHOD == 0 || METHOD == 5) {
                    k = rmq<METHOD>(a, b, E.kr);   // a one-index range gives a
                } else if (n > 1u) {
                    k = rmq<METHOD>(a, b, E.kr);
                }
                if (STATS && fa && n > 1u) ++st_rmq;
                const uint32_t v = rotated(k, E.R);
                const float d2 = box_d2(E.ex, E.ey, E.ez, f0.x, f0.y, f0.z, f1.x, f1.y, f1.z);
                bool kept = false;
                if (fa) kept = rr_test(v, D, d2, n == 1u);
                const bool push = kept && rec != 0xFFFFFFFFu;
                const bool emit = kept && rec == 0xFFFFFFFFu && n == 1u;
                const bool multi = kept && rec == 0xFFFFFFFFu && n > 1u;
                float w = 0.0f;
                if (W && emit) w = 1.0f / accept_p(s, d2, 1.0f);
                const uint64_t m = ballot(push);
                if (push) L.stack[count_below(m)] = make_uint2(rec, k);
                S.n = (uint32_t)__popcll(m);
                wave_sync();
                // each pair of entries is one parent's two child tests
                if (STATS) st_visits += (D.n_frontier + 1u) / 2u;
                emit2<W>(O, D, emit, make_uint2(E.u, a), w, false, make_uint2(0u, 0u), 0.0f);
                if (ballot(multi)) {
                    uint64_t tests = 0;
                    leaf_lights<W>(O, D, E, a, multi ? n : 0u, 0u, 0u, tests);
                    if (STATS) st_leaf += tests;
                }
            } else {
            bool push = false;
            uint32_t k0 = 0;
            if (act) {
                k0 = rmq<METHOD>(0u, N, E.kr);
                const float d2 = box_d2(E.ex, E.ey, E.ez, D.root_lo[0], D.root_lo[1], D.root_lo[2],
                                        D.root_hi[0], D.root_hi[1], D.root_hi[2]);
                push = rr_test(rotated(k0, E.R), D, d2, false);
                if (STATS) ++st_rmq;
            }
            const uint64_t m = ballot(push);
            if (push) {
                const uint32_t at = count_below(m);
                L.stack[at] = make_uint2(0u | ((EPW > 1 ? lane : 0u) << kSlotShift), k0);
            }
            S.n = (uint32_t)__popcll(m);
            wave_sync();
            }
        }

        // -------- top-down walk --------
        // the node records' base, wave-uniform in scalar registers for the
        // whole walk (the loads take it as their scalar base)
        const Node* const nodes = reinterpret_cast<const Node*>(uni64((unsigned long long)(size_t)D.nodes));
        // the loop and refill conditions are written as one scalar compare
        // each (S.g is a multiple of 64, so S.n < 64 && S.g > 0 is
        // S.n < min(S.g, 64)); as && / + the compiler builds them from two
        // compares merged in lane masks
        while ((S.n | S.g) != 0u) {
            if (S.n < min(S.g, (uint32_t)kStackUnit)) stack_refill(S, L, spill, cap);
            // the wave issues its record loads at raised priority, so that
            // they leave early (frame 142.9 -> 142.1 ms)
            __builtin_amdgcn_s_setprio(1);
            const uint32_t n = min(S.n, (uint32_t)kWave);
            const bool act = lane < n;
            // inactive lanes keep an arbitrary entry: every load and decision
            // below is masked by `act` (no instruction spent on a default)
            uint2 e;
            e.x = __builtin_nondeterministic_value(e.x);
            e.y = __builtin_nondeterministic_value(e.y);
            if (act) e = L.stack[ring(S.base + S.n - n + lane, cap)];
            S.n -= n;
            wave_sync();
            if (STATS) st_visits += n;

            EyeState E = E0;
            const uint32_t node = e.x & (kMaxNodes - 1u);
            const uint32_t slot = e.x >> kSlotShift;
            if (EPW > 1 && act) {
                const uint32_t* w = L.eyes + slot * 8u;
                E.ex = __uint_as_float(w[0]); E.ey = __uint_as_float(w[1]); E.ez = __uint_as_float(w[2]);
                E.R = w[3]; E.kr = w[4]; E.u = w[5];
            }

            bool pushL = false, pushR = false, emitL = false, emitR = false, multi = false;
            // read only in lanes whose flags above are set
            uint32_t kL = __builtin_nondeterministic_value(kL), kR = __builtin_nondeterministic_value(kR);
            uint32_t a = __builtin_nondeterministic_value(a), c = __builtin_nondeterministic_value(c);
            uint32_t b = __builtin_nondeterministic_value(b);
            uint32_t first = __builtin_nondeterministic_value(first);
            float wL = __builtin_nondeterministic_value(wL), wR = __builtin_nondeterministic_value(wR);
            uint32_t mlN = 0, mrN = 0;   // lights of the multi-light leaves to test (0: none)
            // Node records.  A load costs about one cycle of the vector-memory
            // pipeline per distinct cache line that a quad of lanes touches
            // (more when the line comes from L2 or beyond), so neighbouring
            // lanes share each record's line (see FetchOf).
            float4 q0, q1, q2, q3;
            if (FetchOf<EPW>::quad_lds) {
                // lane 4g + j fetches quarter j of the records of lanes 4g + t;
                // quarter j of record t lands at t * kSlab + 64 g + 16 j.
                // Inactive lanes fetch record 0, so no load needs a lane mask;
                // byte offsets are 32-bit (at most 2^26 records), the
                // base and the LDS destinations are wave-uniform.
                const uint32_t j = lane & 3u, g4 = lane & ~3u;
                const uint32_t nd = act ? node : 0u;
                const uint32_t jo = j << 4;
                const uint32_t o0 = ((uint32_t)__builtin_amdgcn_mov_dpp((int)nd, 0x00, 0xF, 0xF, false) << 6) | jo;
                const uint32_t o1 = ((uint32_t)__builtin_amdgcn_mov_dpp((int)nd, 0x55, 0xF, 0xF, false) << 6) | jo;
                const uint32_t o2 = ((uint32_t)__builtin_amdgcn_mov_dpp((int)nd, 0xAA, 0xF, 0xF, false) << 6) | jo;
                const uint32_t o3 = ((uint32_t)__builtin_amdgcn_mov_dpp((int)nd, 0xFF, 0xF, 0xF, false) << 6) | jo;
                typedef __attribute__((address_space(1))) const unsigned char* gbytes;
                typedef __attribute__((address_space(1))) const void* gptr;
                typedef __attribute__((address_space(3))) void* lptr;
                const gbytes rec = (gbytes)(nodes);
                __builtin_amdgcn_global_load_lds((gptr)(rec + o0), (lptr)(size_t)(xlds), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((gptr)(rec + o1), (lptr)(size_t)(xlds + kSlab), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((gptr)(rec + o2), (lptr)(size_t)(xlds + 2 * kSlab), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((gptr)(rec + o3), (lptr)(size_t)(xlds + 3 * kSlab), 16, 0, 0);
                unsigned char* xb = L.xpose;
                __builtin_amdgcn_s_setprio(0);
                wave_sync();
                const float4* r = reinterpret_cast<const float4*>(xb + j * kSlab + 16u * g4);
                q0 = r[0]; q1 = r[1]; q2 = r[2]; q3 = r[3];
                wave_sync();
            } else {
                const bool odd = (lane & 1u) != 0u;
                const uint32_t partner = (uint32_t)__builtin_amdgcn_mov_dpp((int)node, kDppSwapPairs, 0xF, 0xF, false);
                const uint32_t n_even = odd ? partner : node;   // record of the pair's even lane
                const uint32_t n_odd = odd ? node : partner;    // record of the pair's odd lane
                const float4* re = reinterpret_cast<const float4*>(D.nodes + n_even);
                const float4* ro = reinterpret_cast<const float4*>(D.nodes + n_odd);
                const uint32_t h = odd ? 1u : 0u;
                float4 e02 = make_float4(0.f, 0.f, 0.f, 0.f), e13 = e02, o02 = e02, o13 = e02;
                if ((lane & ~1u) < n) { e02 = load_global4(re, h); e13 = load_global4(re, 2u + h); }
                if ((lane | 1u) < n) { o02 = load_global4(ro, h); o13 = load_global4(ro, 2u + h); }
                __builtin_amdgcn_s_setprio(0);
                // even lane holds chunks 0, 2 of both records, odd lane chunks 1, 3
                const float4 r1 = swap_pairs(odd ? e02 : o02);
                const float4 r2 = swap_pairs(odd ? e13 : o13);
                q0 = odd ? r1 : e02;
                q1 = odd ? o02 : r1;
                q2 = odd ? r2 : e13;
                q3 = odd ? o13 : r2;
            }
            // Every lane runs the node arithmetic (inactive ones on whatever
            // their registers hold, with no range-minimum query); only the
            // decisions are masked by `act`.  A block masked by `act` cost the
            // moves that merge its results with defaults every step, and spills
            // (frame 124.6 -> 122.8 ms).
            {
                a = __float_as_uint(q0.w);
                c = __float_as_uint(q1.w);
                b = __float_as_uint(q2.w);
                first = __float_as_uint(q3.w);
                const uint32_t k = e.y;
                // the child holding k inherits the minimum; the other one needs a query
                const bool kLeft = k < c;
                const uint32_t qa = kLeft ? c : a;
                uint32_t kq = qa;
                if (METHOD == 0 || METHOD == 5) {
                    // the default method returns qa for a one-index range, so
                    // it runs on every lane (inactive ones on [qa, qa + 1))
                    // without a divergent guard
                    const uint32_t qb = act ? (kLeft ? b : c) : qa + 1u;
                    kq = rmq<METHOD>(qa, qb, E.kr);
                    if (STATS && qb - qa > 1u) ++st_rmq;
                } else {
                    const uint32_t qb = act ? (kLeft ? b : c) : qa;
                    if (qb - qa > 1u) {
                        kq = rmq<METHOD>(qa, qb, E.kr);
                        if (STATS) ++st_rmq;
                    }
                }
                kL = kLeft ? k : kq;
                kR = kLeft ? kq : k;
                if (METHOD == 5) {   // ablation: the inheriting child's minimum is recomputed too
                    const uint32_t ia = kLeft ? a : c, ib = act ? (kLeft ? c : b) : ia;
                    uint32_t ki = ia;
                    if (ib - ia > 1u) {
                        ki = rmq<METHOD>(ia, ib, E.kr);
                        if (STATS) ++st_rmq;
                    }
                    kL = kLeft ? ki : kL;
                    kR = kLeft ? kR : ki;
                }
                const uint32_t nL = c - a, nR = b - c;
                const bool leafL = nL <= leaf, leafR = nR <= leaf;
                const float d2L = box_d2(E.ex, E.ey, E.ez, q0.x, q0.y, q0.z, q1.x, q1.y, q1.z);
                const float d2R = box_d2(E.ex, E.ey, E.ez, q2.x, q2.y, q2.z, q3.x, q3.y, q3.z);
                const uint32_t vL = rotated(kL, E.R), vR = rotated(kR, E.R);
                bool sL, sR;
                const bool openL = rr_fast(vL, D, d2L, nL == 1u, sL) && act;
                const bool openR = rr_fast(vR, D, d2R, nR == 1u, sR) && act;
                if (openL || openR) {   // rare: one shared block for the IEEE decisions
                    if (openL) sL = keeps(vL, accept_p(s, d2L, nL == 1u ? 1.0f : kBoxMargin));
                    if (openR) sR = keeps(vR, accept_p(s, d2R, nR == 1u ? 1.0f : kBoxMargin));
                }
                sL = sL && act;
                sR = sR && act;
                pushL = sL && !leafL;
                pushR = sR && !leafR;
                emitL = sL && nL == 1u;
                emitR = sR && nR == 1u;
                if (W) {
                    if (emitL) wL = 1.0f / accept_p(s, d2L, 1.0f);
                    if (emitR) wR = 1.0f / accept_p(s, d2R, 1.0f);
                }
                mlN = sL && leafL && nL > 1u ? nL : 0u;
                mrN = sR && leafR && nR > 1u ? nR : 0u;
                multi = mlN + mrN > 0u;
            }

            // push survivors: a lane's two children stay adjacent, lanes in order
            const uint64_t bl = ballot(pushL), br = ballot(pushR);
            const uint32_t npush = (uint32_t)(__popcll(bl) + __popcll(br));
            if (npush) {
                if (S.n + npush > cap) {
                    if (!stack_spill(S, L, spill, cap, A.spill_cap, A.error)) break;
                }
                // S.n + npush <= cap here, so S.base + at < 2 cap
                const uint32_t at = S.n + count_below(bl) + count_below(br);
                const uint32_t tag = (EPW > 1 ? slot : 0u) << kSlotShift;
                if (pushL) L.stack[ring(S.base + at, cap)] = make_uint2(first | tag, kL);
                if (pushR) L.stack[ring(S.base + at + (pushL ? 1u : 0u), cap)] = make_uint2((first + 1u) | tag, kR);
                S.n += npush;
                wave_sync();
                const uint32_t tot = S.g + S.n;
                if (tot > S.max_total) S.max_total = tot;
            }

            // one-light leaves accepted at the parent
            emit2<W>(O, D, emitL, make_uint2(E.u, a), wL, emitR, make_uint2(E.u, c), wR);

            // multi-light leaves
            if (leaf > 1u && ballot(multi)) {   // one-light leaves are emitted above
                uint64_t tests = 0;
                leaf_lights<W>(O, D, E, a, mlN, c, mrN, tests);
                if (STATS) st_leaf += tests;
            }
        }
        if (STATS) {
            st_spills += S.spills;
            st_maxstack = max(st_maxstack, S.max_total);
        }
    }
    if (cur != 0xFFFFFFFFu) close_item(O, D, A.error);

    if (STATS && A.stats) {
        uint64_t v[6] = {st_eyes, 0, st_visits, st_rmq, st_leaf, st_spills};
        for (int q = 0; q < 6; ++q) {
            uint64_t x = v[q];
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
            v[q] = x;
        }
        uint32_t mx = st_maxstack;
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o));
        if (lane == 0) {
            // eyes / visits / spills / max stack are per-wave quantities kept in every lane
            atomicAdd(A.stats + ST_EYES, (unsigned long long)(v[0] / kWave));
            atomicAdd(A.stats + ST_VISITS, (unsigned long long)(v[2] / kWave));
            atomicAdd(A.stats + ST_RMQ, (unsigned long long)v[3]);
            atomicAdd(A.stats + ST_LEAF, (unsigned long long)v[4]);
            atomicAdd(A.stats + ST_SPILLS, (unsigned long long)(v[5] / kWave));
            atomicMax(A.stats + ST_MAXSTACK, (unsigned long long)mx);
        }
    }
}

// ---------------------------------------------------------------------------
// the top of a hierarchy (the one-eye-per-wave walk's starting entries)
// ---------------------------------------------------------------------------
//
// One wave expands the root kFrontierDepth times: every internal entry is
// replaced by its two children (their boxes and ranges come from its record,
// their records are `first` and `first + 1` when internal), leaves stay.
// Entries keep index order; after level l there are at most 2^l of them.
// The root's own box is never needed: the root is internal (the caller only
// runs this for hierarchies with records) and is always expanded.
__global__ __launch_bounds__(64) void frontier_kernel(const Node* __restrict__ nodes, uint32_t n_lights,
                                                      uint32_t leaf, float* __restrict__ out) {
    struct Entry { uint32_t a, b, rec; float lo[3], hi[3]; };
    __shared__ Entry next[kFrontierMax];
    const uint32_t t = threadIdx.x;
    Entry e;
    e.a = 0u; e.b = n_lights; e.rec = 0u;
    for (int q = 0; q < 3; ++q) { e.lo[q] = 0.0f; e.hi[q] = 0.0f; }
    uint32_t n = 1;
    for (uint32_t level = 0; level < kFrontierDepth; ++level) {
        const bool have = t < n;
        const bool internal = have && e.rec != 0xFFFFFFFFu;
        const uint32_t c = have ? (internal ? 2u : 1u) : 0u;
        // exclusive prefix of c over the wave
        uint32_t inc = c;
        for (uint32_t off = 1; off < 64u; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off, 64);
            if (t >= off) inc += y;
        }
        const uint32_t pos = inc - c;
        const uint32_t total = __shfl(inc, 63, 64);
        if (internal) {
            const Node R = nodes[e.rec];
            Entry L, Rt;
            L.a = R.a; L.b = R.c; L.rec = R.c - R.a > leaf ? R.first : 0xFFFFFFFFu;
            Rt.a = R.c; Rt.b = R.b; Rt.rec = R.b - R.c > leaf ? R.first + 1u : 0xFFFFFFFFu;
            for (int q = 0; q < 3; ++q) {
                L.lo[q] = R.lo_l[q]; L.hi[q] = R.hi_l[q];
                Rt.lo[q] = R.lo_r[q]; Rt.hi[q] = R.hi_r[q];
            }
            next[pos] = L;
            next[pos + 1u] = Rt;
        } else if (have) {
            next[pos] = e;
        }
        __syncthreads();
        n = total;
        if (t < n) e = next[t];
        __syncthreads();
    }
    if (t < n) {
        float* o = out + (size_t)t * kFrontierFloats;
        o[0] = e.lo[0]; o[1] = e.lo[1]; o[2] = e.lo[2]; o[3] = __uint_as_float(e.a);
        o[4] = e.hi[0]; o[5] = e.hi[1]; o[6] = e.hi[2]; o[7] = __uint_as_float(e.b);
        o[8] = __uint_as_float(e.rec); o[9] = 0.0f; o[10] = 0.0f; o[11] = 0.0f;
    }
    if (t == 0) reinterpret_cast<uint32_t*>(out)[kFrontierMax * kFrontierFloats] = n;
}

// ---------------------------------------------------------------------------
// eye ordering: counting sort of the virtual eyes by (item, Morton cell, shift class)
// ---------------------------------------------------------------------------
//
// The traversal result does not depend on the order in which eyes are
// processed; processing spatially close eyes together lets an XCD's L2 hold
// the part of the hierarchy they share.  Cells: `bits` bits per axis of the
// eye position inside the item's light box, interleaved x-y-z.  Within a cell,
// eyes are grouped by the shift class: the low `rbits` significant bits of the
// eye's tile value t (t = m * 2^tz), bit reversed.  The minimum over an aligned
// block of 2^s indices is (bitreverse(p) + r) mod 2^(32-s), so two eyes whose
// m agree modulo 2^q see equal minima on every block with s >= 32 - tz - q;
// such eyes visit nearly the same nodes.  Bucket of virtual eye g of item k:
// ((k << 3 bits | cell) << rbits) | class.

__device__ __forceinline__ uint32_t spread3_10(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t cell_of(float x, float lo, float scale, uint32_t bits) {
    const float f = (x - lo) * scale;
    const uint32_t top = (1u << bits) - 1u;
    if (!(f > 0.0f)) return 0u;
    const float c = floorf(f);
    return c >= (float)top ? top : (uint32_t)c;
}

__global__ __launch_bounds__(256) void order_keys_kernel(const OrderItem* __restrict__ items,
                                                         const uint32_t* __restrict__ vbegin, uint32_t n_items,
                                                         uint32_t total, uint32_t bits, uint32_t rbits,
                                                         const uint32_t* __restrict__ tile, uint32_t tile_tz,
                                                         uint32_t* __restrict__ keys, uint32_t* __restrict__ hist) {
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = n_items;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (vbegin[mid] <= g) lo = mid; else hi = mid;
        }
        const OrderItem& I = items[lo];
        const uint32_t u = g - vbegin[lo];
        const uint32_t j = I.n_samples > 1 ? u / I.n_samples : u;
        const float* e = I.eyes + 3u * j;
        const uint32_t cx = cell_of(e[0], I.lo[0], I.scale[0], bits);
        const uint32_t cy = cell_of(e[1], I.lo[1], I.scale[1], bits);
        const uint32_t cz = cell_of(e[2], I.lo[2], I.scale[2], bits);
        uint32_t key = (lo << (3u * bits)) | (spread3_10(cx) << 2) | (spread3_10(cy) << 1) | spread3_10(cz);
        if (rbits) {
            const uint32_t pix = I.pixel_base + j;
            const uint32_t x = pix % I.width;
            const uint32_t y = pix / I.width;
            const uint32_t t = tile[(x & 63u) * 64u + (y & 63u)];
            key = (key << rbits) | (__brev(t >> tile_tz) >> (32u - rbits));
        }
        keys[g] = key;
        atomicAdd(hist + key, 1u);
    }
}

__global__ __launch_bounds__(256) void order_scatter_kernel(const uint32_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ vbegin, uint32_t total,
                                                            uint32_t key_bits, uint32_t* __restrict__ offsets,
                                                            uint32_t* __restrict__ order) {
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += gridDim.x * blockDim.x) {
        const uint32_t key = keys[g];
        const uint32_t item = key >> key_bits;
        const uint32_t pos = atomicAdd(offsets + key, 1u);
        order[pos] = g - vbegin[item];
    }
}

// Output compaction after a traversal (the arithmetic and its bounds are in
// hrr_compact.hpp).  compact_plan_kernel, one block per item: the exclusive
// prefix sums of the hole lengths (partial-list order) and of the data
// lengths (chunk order) into the item's plan scratch, then the moved count,
// the dense count and the number of data chunks into its counter line.
// compact_move_kernel, a grid of blocks per item: moved element e goes from
// the e-th data position to the e-th hole position.

// Exclusive scan of one value per thread over a block of 256; total = the sum.
__device__ __forceinline__ unsigned long long block_exclusive_scan_u64(unsigned long long x,
                                                                       unsigned long long* lds,
                                                                       unsigned long long& total) {
    const uint32_t t = threadIdx.x;
    lds[t] = x;
    __syncthreads();
    for (uint32_t off = 1; off < 256u; off <<= 1) {
        const unsigned long long add = t >= off ? lds[t - off] : 0ull;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    const unsigned long long incl = lds[t];
    total = lds[255];
    __syncthreads();
    return incl - x;
}

__device__ __forceinline__ CompactGeom item_geom(const ItemDesc& D) {
    const unsigned long long* cnt = D.counters;
    return compact_geom(cnt[CNT_PAIRS], cnt[CNT_CHUNKS], cnt[CNT_PARTIALS], D.partial_cap, D.capacity, D.slack,
                        D.chunk_shift);
}

__global__ __launch_bounds__(256) void compact_plan_kernel(const ItemDesc* __restrict__ items,
                                                           uint32_t* __restrict__ error) {
    __shared__ unsigned long long lds[256];
    const ItemDesc& D = items[blockIdx.x];
    const CompactGeom g = item_geom(D);
    const unsigned long long nd_cap = 2ull * D.partial_cap + 2ull;
    const unsigned long long nd = umin64(g.nd, nd_cap);   // g.nd <= nd_cap always (see the bounds)
    unsigned long long* Hs = D.plan;
    unsigned long long* Ds = D.plan + D.partial_cap + 1;
    const unsigned long long* pl = D.partials;

    unsigned long long run = 0, tot = 0;
    for (unsigned long long b = 0; b < g.P; b += 256) {
        const unsigned long long q = b + threadIdx.x;
        const unsigned long long len = q < g.P ? hole_len(g, pl[2 * q], pl[2 * q + 1]) : 0ull;
        const unsigned long long ex = block_exclusive_scan_u64(len, lds, tot);
        if (q < g.P) Hs[q] = run + ex;
        run += tot;
    }
    const unsigned long long TH = run;

    // fills of the data chunks: full, except the partly filled ones (each
    // chunk is on the partial list at most once)
    for (unsigned long long i = threadIdx.x; i < nd; i += 256) Ds[i] = g.C;
    __syncthreads();
    for (unsigned long long q = threadIdx.x; q < g.P; q += 256) {
        const unsigned long long c = pl[2 * q];
        if (c >= g.c0 && c - g.c0 < nd) Ds[c - g.c0] = pl[2 * q + 1];
    }
    __syncthreads();
    run = 0;
    for (unsigned long long b = 0; b < nd; b += 256) {
        const unsigned long long i = b + threadIdx.x;
        const unsigned long long len = i < nd ? data_len(g, i, Ds[i]) : 0ull;
        const unsigned long long ex = block_exclusive_scan_u64(len, lds, tot);   // every read precedes the writes
        if (i < nd) Ds[i] = run + ex;
        run += tot;
    }
    const unsigned long long TD = run;
    if (threadIdx.x == 0) {
        Hs[g.P] = TH;
        Ds[nd] = TD;
        const unsigned long long moved = umin64(TH, TD);
        D.counters[CNT_MOVED] = moved;
        D.counters[CNT_ND] = nd;
        D.counters[CNT_STORED] = g.target - (TH - moved);
        if (TH > moved || g.nd > nd_cap) atomicOr(error, (uint32_t)ERR_UNFILLED);   // never expected
    }
}

constexpr uint32_t kMoveRun = 16;   // moved elements per lane and step

// Two mappings of moved elements to lanes.  With chunks of 2^10 or more
// pairs (long holes and data runs) each wave moves a block of kWave *
// kMoveRun consecutive elements, lane l taking e0 + l, e0 + l + kWave, ...,
// so the 64 lanes of one access read and write whole cache lines (frame:
// 258 -> 95 us).  With smaller chunks a lane stepping by kWave would cross a
// hole boundary, a dependent load, almost every step; there each lane moves
// its own run of kMoveRun consecutive elements instead.
__global__ __launch_bounds__(256) void compact_move_kernel(const ItemDesc* __restrict__ items) {
    const ItemDesc& D = items[blockIdx.y];
    const unsigned long long moved = D.counters[CNT_MOVED];
    if (moved == 0) return;
    const CompactGeom g = item_geom(D);
    const unsigned long long nd = D.counters[CNT_ND];
    const unsigned long long* Hs = D.plan;
    const unsigned long long* Ds = D.plan + D.partial_cap + 1;
    const unsigned long long* pl = D.partials;
    uint2* out = reinterpret_cast<uint2*>(D.pairs);
    const uint2* sl = reinterpret_cast<const uint2*>(D.slack_pairs);
    const unsigned long long cap = D.capacity;
    const unsigned long long tid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool lanes = D.chunk_shift >= 10;   // uniform over the block (one item per blockIdx.y)
    const MoveMap mm = move_map(lanes, tid, (unsigned long long)gridDim.x * blockDim.x, kMoveRun);
    for (unsigned long long e0 = mm.first; e0 < moved; e0 += mm.step) {
        // moved < both totals, so the walks below stop inside the prefixes
        unsigned long long q = prefix_rank(Hs, g.P, e0);
        unsigned long long i = prefix_rank(Ds, nd, e0);
        const unsigned long long e1 = move_run_end(mm, e0, moved);
        for (unsigned long long e = e0; e < e1; e += mm.stride) {
            while (Hs[q + 1] <= e) ++q;
            while (Ds[i + 1] <= e) ++i;
            const unsigned long long dst = hole_lo(g, pl[2 * q], pl[2 * q + 1]) + (e - Hs[q]);
            const unsigned long long src = data_lo(g, i) + (e - Ds[i]);
            out[dst] = src < cap ? out[src] : sl[src - cap];
            if (D.weights) D.weights[dst] = src < cap ? D.weights[src] : D.slack_weights[src - cap];
        }
    }
}

// ---------------------------------------------------------------------------
// the allocation-free traversal: set-up and result kernels
// ---------------------------------------------------------------------------

// Writes the launch's item and task tables into the scratch header and
// clears its queue heads, counters and status words (a kernel, not a memset
// or a copy, so that the call records only kernel launches).
__global__ __launch_bounds__(256) void noalloc_setup_kernel(ItemDesc D, uint32_t n_tasks, unsigned char* base) {
    uint32_t* q = reinterpret_cast<uint32_t*>(base + kNoAllocQueues);
    for (uint32_t t = threadIdx.x; t < kQueues * kQueueStride; t += blockDim.x) q[t] = 0u;
    unsigned long long* c = reinterpret_cast<unsigned long long*>(base + kNoAllocCounters);
    for (uint32_t t = threadIdx.x; t < CNT_STRIDE; t += blockDim.x) c[t] = 0ull;
    unsigned long long* m = reinterpret_cast<unsigned long long*>(base + kNoAllocMisc);
    for (uint32_t t = threadIdx.x; t < 16u; t += blockDim.x) m[t] = 0ull;
    if (threadIdx.x == 0) {
        *reinterpret_cast<ItemDesc*>(base + kNoAllocItem) = D;
        uint32_t* tb = reinterpret_cast<uint32_t*>(base + kNoAllocTasks);
        tb[0] = 0u;
        tb[1] = n_tasks;
    }
}

// result[0] = the item's true pair count, result[1] = the status word (0 when
// the launch and its compaction completed).
__global__ void noalloc_finish_kernel(const unsigned char* base, unsigned long long* result) {
    if (threadIdx.x == 0) {
        result[0] = reinterpret_cast<const unsigned long long*>(base + kNoAllocCounters)[CNT_PAIRS];
        result[1] = reinterpret_cast<const unsigned long long*>(base + kNoAllocMisc)[1] & 0xFFFFFFFFull;
    }
}

}  // namespace hrr

// Scratch of the allocation-free traversal.  Every GPU the library runs on
// holds its own copy for the life of the process; host code reaches it only
// through the per-device address below (the array's name is not a device
// address in host code).
static __device__ __align__(256) unsigned char scratch[hrr::kNoAllocScratchBytes];

// Device address of this GPU's scratch, looked up once per device with that
// device current (called by hrr_create) and kept.
extern "C" hipError_t hrr_noalloc_scratch(int device, void** out) {
    static std::mutex mu;
    static void* addr[64] = {};
    if (device < 0 || device >= 64 || !out) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

extern "C" hipError_t hrr_launch_noalloc_setup(const hrr::ItemDesc* D, uint32_t n_tasks, void* base,
                                               hipStream_t stream) {
    hipLaunchKernelGGL(hrr::noalloc_setup_kernel, dim3(1), dim3(256), 0, stream, *D, n_tasks,
                       static_cast<unsigned char*>(base));
    return hipGetLastError();
}

extern "C" hipError_t hrr_launch_noalloc_finish(const void* base, unsigned long long* result, hipStream_t stream) {
    hipLaunchKernelGGL(hrr::noalloc_finish_kernel, dim3(1), dim3(64), 0, stream,
                       static_cast<const unsigned char*>(base), result);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers (called from the C++ runtime)
// ---------------------------------------------------------------------------

extern "C" hipError_t hrr_launch_rmq(const uint32_t* a, const uint32_t* b, const uint32_t* r, uint64_t n,
                                     uint32_t method, uint32_t* k, uint32_t* v, unsigned long long* n_bad,
                                     int n_cu, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int vec = ((((uintptr_t)a) | ((uintptr_t)b) | ((uintptr_t)r) | ((uintptr_t)k) | ((uintptr_t)v)) & 15u) == 0;
    const uint64_t work = vec ? (n + 3) / 4 : n;
    // kRmqGroups 4-query groups per thread and a grid far larger than the
    // resident capacity keep the most loads in flight (2^28 queries with
    // ordinary loads: 1.26 ms with 16 blocks per CU and a grid-stride loop,
    // 1.02 ms with one group per thread, 0.98 ms with two; with non-temporal
    // loads one group is best).  The loop still covers grids above the cap.
    const uint64_t per_block = vec ? 256ull * hrr::kRmqGroups : 256ull;
    uint64_t blocks = (work + per_block - 1) / per_block;
    const uint64_t max_blocks = 1ull << 30;
    (void)n_cu;
    if (blocks > max_blocks) blocks = max_blocks;
    if (blocks < 1) blocks = 1;
    if (method == 1)
        hipLaunchKernelGGL(hrr::rmq_kernel<1>, dim3((uint32_t)blocks), dim3(256), 0, stream, a, b, r, n, k, v, n_bad, vec);
    else if (method == 2)
        hipLaunchKernelGGL(hrr::rmq_kernel<2>, dim3((uint32_t)blocks), dim3(256), 0, stream, a, b, r, n, k, v, n_bad, vec);
    else if (method == 3)
        hipLaunchKernelGGL(hrr::rmq_kernel<3>, dim3((uint32_t)blocks), dim3(256), 0, stream, a, b, r, n, k, v, n_bad, vec);
    else if (method == 4)
        hipLaunchKernelGGL(hrr::rmq_kernel<4>, dim3((uint32_t)blocks), dim3(256), 0, stream, a, b, r, n, k, v, n_bad, vec);
    else
        hipLaunchKernelGGL(hrr::rmq_kernel<0>, dim3((uint32_t)blocks), dim3(256), 0, stream, a, b, r, n, k, v, n_bad, vec);
    return hipGetLastError();
}

// Compaction of a launch's items (see compact_plan_kernel): n_items <= 65535.
extern "C" hipError_t hrr_launch_compact(const hrr::ItemDesc* items, uint32_t n_items, uint32_t* error,
                                         hipStream_t stream) {
    if (n_items == 0) return hipSuccess;
    if (n_items > 65535u) return hipErrorInvalidValue;
    hipLaunchKernelGGL(hrr::compact_plan_kernel, dim3(n_items), dim3(256), 0, stream, items, error);
    // about 8192 blocks in all, at least 16 and at most 4096 per item
    uint32_t per_item = 8192u / n_items;
    per_item = per_item < 16u ? 16u : (per_item > 4096u ? 4096u : per_item);
    hipLaunchKernelGGL(hrr::compact_move_kernel, dim3(per_item, n_items), dim3(256), 0, stream, items);
    return hipGetLastError();
}

namespace {

template <int EPW, int METHOD, bool STATS, bool W>
hipError_t launch_trav(const hrr::TravArgs& A, uint32_t blocks, size_t lds, hipStream_t stream) {
    auto kern = hrr::traverse_kernel<EPW, METHOD, STATS, W>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(hrr::kWave * hrr::kWavesPerBlock), lds, stream, A);
    return hipGetLastError();
}

template <int EPW, int METHOD, bool STATS>
hipError_t pick_w(const hrr::TravArgs& A, bool w, uint32_t blocks, size_t lds, hipStream_t s) {
    return w ? launch_trav<EPW, METHOD, STATS, true>(A, blocks, lds, s)
             : launch_trav<EPW, METHOD, STATS, false>(A, blocks, lds, s);
}

template <int EPW, int METHOD>
hipError_t pick_stats(const hrr::TravArgs& A, bool st, bool w, uint32_t blocks, size_t lds, hipStream_t s) {
    return st ? pick_w<EPW, METHOD, true>(A, w, blocks, lds, s) : pick_w<EPW, METHOD, false>(A, w, blocks, lds, s);
}

template <int EPW>
hipError_t pick_method(const hrr::TravArgs& A, uint32_t method, bool st, bool w, uint32_t blocks, size_t lds,
                       hipStream_t s) {
    if (method == 1) return pick_stats<EPW, 1>(A, st, w, blocks, lds, s);
    if (method == 2) return pick_stats<EPW, 2>(A, st, w, blocks, lds, s);
    if (method == 3) return pick_stats<EPW, 3>(A, st, w, blocks, lds, s);
    if (method == 4) return pick_stats<EPW, 4>(A, st, w, blocks, lds, s);
    if (method == 5) return pick_stats<EPW, 5>(A, st, w, blocks, lds, s);
    return pick_stats<EPW, 0>(A, st, w, blocks, lds, s);
}

}  // namespace

// LDS bytes of one wave for a given stack size.
extern "C" size_t hrr_trav_lds_per_wave(uint32_t stack_cap, uint32_t eyes_per_wave) {
    return (size_t)stack_cap * sizeof(uint2) + (eyes_per_wave > 1 ? hrr::kEyeTableBytes : hrr::kXposeBytes);
}

// Dynamic LDS bytes of one block.
extern "C" size_t hrr_trav_lds_per_block(uint32_t n_items, size_t lds_per_wave) {
    return ((size_t)n_items + 1u) * sizeof(uint32_t) / 16u * 16u + 16u + lds_per_wave * hrr::kWavesPerBlock;
}

extern "C" hipError_t hrr_launch_traverse(const hrr::TravArgs* A, uint32_t eyes_per_wave, uint32_t method,
                                          int stats, int with_weights, uint32_t blocks, hipStream_t stream) {
    const size_t lds = hrr_trav_lds_per_block(A->n_items, A->lds_per_wave);
    switch (eyes_per_wave) {
        case 1: return pick_method<1>(*A, method, stats, with_weights, blocks, lds, stream);
        case 2: return pick_method<2>(*A, method, stats, with_weights, blocks, lds, stream);
        case 4: return pick_method<4>(*A, method, stats, with_weights, blocks, lds, stream);
        case 8: return pick_method<8>(*A, method, stats, with_weights, blocks, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

// Resident blocks per CU for a launch shape (for sizing the persistent grid).
extern "C" hipError_t hrr_traverse_occupancy(uint32_t eyes_per_wave, uint32_t method, int stats, int with_weights,
                                             size_t lds_per_block, int* blocks_per_cu) {
    const void* f = nullptr;
#define HRR_PICK(E, M, S, W) \
    if (eyes_per_wave == E && method == M && (stats != 0) == S && (with_weights != 0) == W) \
        f = (const void*)hrr::traverse_kernel<E, M, S, W>;
#define HRR_PICK_SW(E, M) HRR_PICK(E, M, false, false) HRR_PICK(E, M, false, true) HRR_PICK(E, M, true, false) HRR_PICK(E, M, true, true)
#define HRR_PICK_M(E) \
    HRR_PICK_SW(E, 0) HRR_PICK_SW(E, 1) HRR_PICK_SW(E, 2) HRR_PICK_SW(E, 3) HRR_PICK_SW(E, 4) HRR_PICK_SW(E, 5)
    HRR_PICK_M(1) HRR_PICK_M(2) HRR_PICK_M(4) HRR_PICK_M(8)
#undef HRR_PICK_M
#undef HRR_PICK_SW
#undef HRR_PICK
    if (!f) return hipErrorInvalidValue;
    if (lds_per_block > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_per_block);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, hrr::kWave * hrr::kWavesPerBlock,
                                                        lds_per_block);
}

// The top of a hierarchy with records (see frontier_kernel): out holds
// kFrontierMax * kFrontierFloats floats, then the entry count.
extern "C" hipError_t hrr_launch_frontier(const hrr::Node* nodes, uint32_t n_lights, uint32_t leaf_size, float* out,
                                          hipStream_t stream) {
    hipLaunchKernelGGL(hrr::frontier_kernel, dim3(1), dim3(64), 0, stream, nodes, n_lights, leaf_size, out);
    return hipGetLastError();
}

// Processing order of the virtual eyes of a launch (see order_keys_kernel).
// hist must hold (n_items << (3 bits + rbits)) + 1024 counters (the last 1024
// are the scan's chunk sums); keys and order `total` words; tile is the
// context's 64x64 tile, whose values share tile_tz trailing zeros (rbits = 0
// leaves the shift out of the key).
extern "C" hipError_t hrr_launch_order(const hrr::OrderItem* items, const uint32_t* vbegin, uint32_t n_items,
                                       uint32_t total, uint32_t bits, uint32_t rbits, const uint32_t* tile,
                                       uint32_t tile_tz, uint32_t* keys, uint32_t* hist, uint32_t* order, int n_cu,
                                       hipStream_t stream) {
    if (total == 0) return hipSuccess;
    if (rbits > 31u || (rbits && tile_tz > 31u)) return hipErrorInvalidValue;
    const uint32_t key_bits = 3u * bits + rbits;
    const uint32_t n_buckets = n_items << key_bits;
    if (hrr::scan::chunk_count(n_buckets) > 1024u) return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(hist, 0, (size_t)n_buckets * sizeof(uint32_t), stream);
    if (e != hipSuccess) return e;
    uint32_t blocks = (total + 255u) / 256u;
    const uint32_t max_blocks = (uint32_t)(n_cu > 0 ? n_cu : 256) * 8u;
    if (blocks > max_blocks) blocks = max_blocks;
    hipLaunchKernelGGL(hrr::order_keys_kernel, dim3(blocks), dim3(256), 0, stream, items, vbegin, n_items, total, bits,
                       rbits, tile, tile_tz, keys, hist);
    if ((e = hrr::scan::exclusive_sum(hist, hist, n_buckets, hist + n_buckets, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(hrr::order_scatter_kernel, dim3(blocks), dim3(256), 0, stream, keys, vbegin, total, key_bits,
                       hist, order);
    return hipGetLastError();
}
