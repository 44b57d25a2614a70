// hrr_build_device.hip -- the light hierarchy built on the GPU, record for
// record identical to the host builder (hrr_build.cpp): same Morton codes,
// same (code, original index) order, same split rule (radix split with the
// midpoint for equal codes, or the power-of-two split), same exact fp32 boxes
// and the same record numbering (sibling pairs in preorder of their owners).
//
// Section 1 of the paper only needs the lights sorted by a spatial hierarchy
// with every node a contiguous index range; building it on the device lets a
// renderer rebuild per-frame light caches without a host round trip.
//
// Steps (all stream-ordered; the host reads back one count per level):
//   1. codes   : 63-bit Morton code per light (21-bit cells, x highest)
//   2. sort    : stable LSD radix sort of (code, index) pairs, 8-bit digits
//   3. gather  : lights in sequence order as float4, codes in sequence order
//   4. levels  : breadth-first, one launch per level: split every internal
//                node of the level, append its internal children to the next
//                level (exclusive scan of the child counts)
//   5. refit   : deepest level first, each node's children boxes (a leaf
//                child from its <= leaf_size lights, an internal child as
//                the union of its own children) and the number of pair
//                owners (nodes with an internal child) in its subtree
//   6. records : root level first, record numbers (a node's children take
//                the sibling pair 2 (1 + owners before it in preorder) and
//                the next record) and the 64-byte records at those numbers
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "hrr_devbuild.hpp"
#include "hrr_scan.hpp"
#include "hrr_types.hpp"

namespace hrr {
namespace devbuild {

// ---- Morton code, written out as in the host builder --------------------

__device__ __forceinline__ uint64_t spread_bits3(uint32_t v) {
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t cell21(float x, float lo, float hi) {
    float u = (x - lo) / (hi - lo);
    if (!(u > 0.0f)) u = 0.0f;
    if (u > 1.0f) u = 1.0f;
    const uint32_t q = (uint32_t)(u * 2097152.0f);
    return q < 2097151u ? q : 2097151u;
}

__global__ void codes_kernel(const float* __restrict__ xyz, uint32_t n, QBox qb, uint64_t* __restrict__ code,
                             uint32_t* __restrict__ idx, uint32_t* __restrict__ bad) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = xyz[3 * (size_t)i], y = xyz[3 * (size_t)i + 1], z = xyz[3 * (size_t)i + 2];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) atomicOr(bad, 1u);
    code[i] = (spread_bits3(cell21(x, qb.lo[0], qb.hi[0])) << 2) | (spread_bits3(cell21(y, qb.lo[1], qb.hi[1])) << 1) |
              spread_bits3(cell21(z, qb.lo[2], qb.hi[2]));
    idx[i] = i;
}

__global__ void gather_kernel(const float* __restrict__ xyz, const uint32_t* __restrict__ perm, uint32_t n,
                              float4* __restrict__ lights) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = perm[i];
    lights[i] = make_float4(xyz[3 * (size_t)j], xyz[3 * (size_t)j + 1], xyz[3 * (size_t)j + 2], 0.0f);
}

// ---- breadth-first split ----------------------------------------------
//
// Internal nodes are numbered breadth-first (t); level l holds
// [off[l], off[l+1]).  Bfs (hrr_devbuild.hpp) holds, per node, the range a,
// split c, end b, children t (or -1 for a leaf child), subtree counts of
// pair owners, record numbers, owners before the node in preorder and the
// node's own box.

__device__ __forceinline__ uint32_t split_of(const uint64_t* __restrict__ code, uint32_t a, uint32_t b,
                                             uint32_t pow2) {
    if (pow2) return a + (1u << (31 - __clz((int)(b - a - 1u))));   // largest 2^k < b - a (b - a >= 2)
    const uint64_t ca = code[a], cb = code[b - 1];
    if (ca == cb) return a + (b - a) / 2;
    const int h = 63 - __clzll((long long)(ca ^ cb));
    // first index in (a, b) whose code has bit h set (the codes agree above h)
    uint32_t lo = a, hi = b - 1;
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if ((code[mid] >> h) & 1u) hi = mid; else lo = mid;
    }
    return hi;
}

// Pass 1 of a level: split, count internal children.
__global__ void split_kernel(Bfs T, const uint64_t* __restrict__ code, uint32_t t0, uint32_t t1, uint32_t leaf,
                             uint32_t pow2, uint32_t* __restrict__ kids) {
    const uint32_t t = t0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t1) return;
    const uint32_t a = T.a[t], b = T.b[t];
    const uint32_t c = split_of(code, a, b, pow2);
    T.c[t] = c;
    kids[t - t0] = (c - a > leaf ? 1u : 0u) + (b - c > leaf ? 1u : 0u);
}

// Pass 2 of a level: place the internal children at t1 + exclusive prefix.
// Every split leaves both sides non-empty, so a build has at most n - 1
// internal nodes; `cap` (that bound) only guards the tables.
__global__ void place_kernel(Bfs T, uint32_t t0, uint32_t t1, uint32_t leaf, const uint32_t* __restrict__ prefix,
                             uint32_t cap) {
    const uint32_t t = t0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t1) return;
    const uint32_t a = T.a[t], c = T.c[t], b = T.b[t];
    uint32_t at = t1 + prefix[t - t0];
    int32_t l = -1, r = -1;
    if (c - a > leaf && at < cap) {
        l = (int32_t)at;
        T.a[at] = a;
        T.b[at] = c;
        ++at;
    }
    if (b - c > leaf && at < cap) {
        r = (int32_t)at;
        T.a[at] = c;
        T.b[at] = b;
    }
    T.l[t] = l;
    T.r[t] = r;
}

// min / max with the host builder's tie rule (std::min / std::max keep the
// first operand unless the second is strictly smaller / larger), so that
// signed zeros come out the same.
__device__ __forceinline__ float min_first(float x, float y) { return y < x ? y : x; }
__device__ __forceinline__ float max_first(float x, float y) { return x < y ? y : x; }

__device__ __forceinline__ void leaf_box(const float4* __restrict__ lights, uint32_t a, uint32_t b, float* lo,
                                         float* hi) {
    const float4 p = lights[a];
    lo[0] = hi[0] = p.x;
    lo[1] = hi[1] = p.y;
    lo[2] = hi[2] = p.z;
    for (uint32_t i = a + 1; i < b; ++i) {
        const float4 q = lights[i];
        lo[0] = min_first(lo[0], q.x); hi[0] = max_first(hi[0], q.x);
        lo[1] = min_first(lo[1], q.y); hi[1] = max_first(hi[1], q.y);
        lo[2] = min_first(lo[2], q.z); hi[2] = max_first(hi[2], q.z);
    }
}

// Children boxes of a node: a leaf child from its lights, an internal child
// from its own box (computed one level deeper, earlier).
__device__ __forceinline__ void child_box(const Bfs& T, const float4* __restrict__ lights, int32_t child, uint32_t a,
                                          uint32_t b, float* lo, float* hi) {
    if (child < 0) {
        leaf_box(lights, a, b, lo, hi);
    } else {
        const float* bx = T.box + 6 * (size_t)child;
        for (int k = 0; k < 3; ++k) {
            lo[k] = bx[k];
            hi[k] = bx[3 + k];
        }
    }
}

// Refit one level (deepest first): own box and the pair owners in the subtree.
__global__ void refit_kernel(Bfs T, const float4* __restrict__ lights, uint32_t t0, uint32_t t1) {
    const uint32_t t = t0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t1) return;
    const uint32_t a = T.a[t], c = T.c[t], b = T.b[t];
    const int32_t l = T.l[t], r = T.r[t];
    float llo[3], lhi[3], rlo[3], rhi[3];
    child_box(T, lights, l, a, c, llo, lhi);
    child_box(T, lights, r, c, b, rlo, rhi);
    float* bx = T.box + 6 * (size_t)t;
    for (int k = 0; k < 3; ++k) {
        bx[k] = min_first(llo[k], rlo[k]);
        bx[3 + k] = max_first(lhi[k], rhi[k]);
    }
    T.cnt[t] = (l >= 0 || r >= 0 ? 1u : 0u) + (l >= 0 ? T.cnt[l] : 0u) + (r >= 0 ? T.cnt[r] : 0u);
}

// Records of one level (root level first): the children's record numbers
// and owner ranks, and the 64-byte record at this node's number.
__global__ void record_kernel(Bfs T, const float4* __restrict__ lights, uint32_t t0, uint32_t t1,
                              Node* __restrict__ nodes) {
    const uint32_t t = t0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t1) return;
    const uint32_t me = T.pre[t];
    const uint32_t a = T.a[t], c = T.c[t], b = T.b[t];
    const int32_t l = T.l[t], r = T.r[t];
    uint32_t first = 0xFFFFFFFFu;
    if (l >= 0 || r >= 0) {
        const uint32_t rank = T.own[t];   // owners before this node in preorder
        first = 2u * (1u + rank);
        if (l >= 0) {
            T.pre[l] = first;
            T.own[l] = rank + 1u;
        }
        if (r >= 0) {
            T.pre[r] = first + 1u;
            T.own[r] = rank + 1u + (l >= 0 ? T.cnt[l] : 0u);
        }
    }
    float llo[3], lhi[3], rlo[3], rhi[3];
    child_box(T, lights, l, a, c, llo, lhi);
    child_box(T, lights, r, c, b, rlo, rhi);
    Node nd;
    for (int k = 0; k < 3; ++k) {
        nd.lo_l[k] = llo[k];
        nd.hi_l[k] = lhi[k];
        nd.lo_r[k] = rlo[k];
        nd.hi_r[k] = rhi[k];
    }
    nd.a = a;
    nd.c = c;
    nd.b = b;
    nd.first = first;
    nodes[me] = nd;
}

__global__ void root_leaf_box_kernel(const float4* __restrict__ lights, uint32_t n, float* __restrict__ box) {
    if (blockIdx.x == 0 && threadIdx.x == 0) leaf_box(lights, 0, n, box, box + 3);
}

__global__ void init_root_kernel(Bfs T, uint32_t n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        T.a[0] = 0u;
        T.b[0] = n;
        T.pre[0] = 0u;
        T.own[0] = 0u;
    }
}


// ---- stable LSD radix sort of (code, index) pairs ----------------------
//
// Eight passes of 8-bit digits cover the 63 code bits, least significant
// digit first.  One pass is three steps: the digit counts of every tile of
// kSortTile keys, an exclusive scan of those counts laid out digit-major
// (digit d of tile b at d * n_tiles + b, so the scan hands every (digit,
// tile) pair the first output position of its keys), and a scatter that
// ranks each tile's keys stably.  A tile is read in kSortRounds rounds of
// 256 consecutive keys; a key's rank is its digit's next free position in the
// tile, plus the keys of its round with the same digit in earlier waves, plus
// those in earlier lanes of its own wave (found with eight ballots, one per
// digit bit).  Keys of one digit therefore leave in index order, which makes
// every pass stable and the result ordered by (code, original index).

constexpr uint32_t kSortThreads = 256;
constexpr uint32_t kSortRounds = 16;
constexpr uint32_t kSortTile = kSortThreads * kSortRounds;
constexpr uint32_t kSortDigits = 256;
constexpr uint32_t kSortPasses = 8;

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes of the wave (among `valid`) whose digit equals this lane's.
__device__ __forceinline__ uint64_t same_digit_lanes(uint32_t d, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (uint32_t bit = 0; bit < 8u; ++bit) {
        const bool set = (d >> bit) & 1u;
        const uint64_t m = __builtin_amdgcn_ballot_w64(set);
        peers &= set ? m : ~m;
    }
    return peers;
}

__global__ __launch_bounds__(kSortThreads) void sort_count_kernel(const uint64_t* __restrict__ key, uint32_t n,
                                                                  uint32_t shift, uint32_t n_tiles,
                                                                  uint32_t* __restrict__ counts) {
    __shared__ uint32_t hist[kSortDigits];
    const uint32_t t = threadIdx.x;
    hist[t] = 0u;
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortTile;
    for (uint32_t r = 0; r < kSortRounds; ++r) {
        const uint32_t i = base + r * kSortThreads + t;
        const bool ok = i < n;
        const uint32_t d = ok ? (uint32_t)(key[i] >> shift) & (kSortDigits - 1u) : 0u;
        const uint64_t peers = same_digit_lanes(d, __builtin_amdgcn_ballot_w64(ok));
        if (ok && lanes_below(peers) == 0u) atomicAdd(&hist[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    counts[(size_t)t * n_tiles + blockIdx.x] = hist[t];
}

__global__ __launch_bounds__(kSortThreads) void sort_scatter_kernel(const uint64_t* __restrict__ kin,
                                                                    const uint32_t* __restrict__ vin, uint32_t n,
                                                                    uint32_t shift, uint32_t n_tiles,
                                                                    const uint32_t* __restrict__ first,
                                                                    uint64_t* __restrict__ kout,
                                                                    uint32_t* __restrict__ vout) {
    // next[d]: the tile's next output position for digit d (thread d owns it).
    // pos[r & 1][w][d]: keys of digit d in wave w of round r, then the first
    // position of those keys; the other parity is cleared for the next round.
    __shared__ uint32_t next[kSortDigits];
    __shared__ uint32_t pos[2][kSortThreads / 64][kSortDigits];
    const uint32_t t = threadIdx.x, w = t >> 6;
    next[t] = first[(size_t)t * n_tiles + blockIdx.x];
    for (uint32_t q = 0; q < kSortThreads / 64; ++q) {
        pos[0][q][t] = 0u;
        pos[1][q][t] = 0u;
    }
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortTile;
    for (uint32_t r = 0; r < kSortRounds; ++r) {
        const uint32_t p = r & 1u;
        const uint32_t i = base + r * kSortThreads + t;
        const bool ok = i < n;
        const uint64_t k = ok ? kin[i] : 0ull;
        const uint32_t v = ok ? vin[i] : 0u;
        const uint32_t d = (uint32_t)(k >> shift) & (kSortDigits - 1u);
        const uint64_t peers = same_digit_lanes(d, __builtin_amdgcn_ballot_w64(ok));
        const uint32_t below = lanes_below(peers);
        if (ok && below == 0u) pos[p][w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        uint32_t run = next[t];
        for (uint32_t q = 0; q < kSortThreads / 64; ++q) {
            const uint32_t c = pos[p][q][t];
            pos[p][q][t] = run;
            run += c;
            pos[p ^ 1u][q][t] = 0u;
        }
        next[t] = run;
        __syncthreads();
        if (ok) {
            const uint32_t at = pos[p][w][d] + below;
            kout[at] = k;
            vout[at] = v;
        }
    }
}

}  // namespace devbuild
}  // namespace hrr

using namespace hrr;
using namespace hrr::devbuild;

namespace {

constexpr uint32_t kThreads = 256;

uint32_t blocks_for(uint32_t n) { return (n + kThreads - 1) / kThreads; }

}  // namespace

// Scratch sizes and steps are driven from the host file (hrr_api.cpp) through
// these entry points; every one is asynchronous on `stream`.
extern "C" hipError_t hrr_dev_codes(const float* xyz, uint32_t n, const float* qbox, uint64_t* code, uint32_t* idx,
                                    uint32_t* bad, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    QBox qb;
    for (int k = 0; k < 3; ++k) {
        qb.lo[k] = qbox[k];
        qb.hi[k] = qbox[3 + k];
    }
    codes_kernel<<<blocks_for(n), kThreads, 0, stream>>>(xyz, n, qb, code, idx, bad);
    return hipGetLastError();
}

size_t align256(size_t b) { return (b + 255u) & ~(size_t)255u; }

// Stable radix sort of (code, index) by code (63 low bits); temp == nullptr
// queries temp_bytes.  Scratch: a second key and index buffer (the passes
// alternate between it and the outputs, the last pass landing in the
// outputs), the per-tile digit counts and the scan's chunk sums.
extern "C" hipError_t hrr_dev_sort(void* temp, size_t* temp_bytes, const uint64_t* code_in, uint64_t* code_out,
                                   const uint32_t* idx_in, uint32_t* idx_out, uint32_t n, hipStream_t stream) {
    static_assert(kSortPasses % 2 == 0, "the last pass must write the outputs");
    if (!temp_bytes) return hipErrorInvalidValue;
    const uint32_t n_tiles = (n + kSortTile - 1u) / kSortTile;
    const uint32_t n_counts = n_tiles * kSortDigits;
    const size_t b_keys = align256((size_t)n * 8u), b_idx = align256((size_t)n * 4u);
    const size_t b_counts = align256((size_t)n_counts * 4u), b_sums = align256((size_t)scan::chunk_count(n_counts) * 4u);
    const size_t need = std::max<size_t>(b_keys + b_idx + b_counts + b_sums, 256u);
    if (!temp) {
        *temp_bytes = need;
        return hipSuccess;
    }
    if (*temp_bytes < need) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    unsigned char* tp = static_cast<unsigned char*>(temp);
    uint64_t* k_tmp = reinterpret_cast<uint64_t*>(tp);
    uint32_t* v_tmp = reinterpret_cast<uint32_t*>(tp + b_keys);
    uint32_t* counts = reinterpret_cast<uint32_t*>(tp + b_keys + b_idx);
    uint32_t* sums = reinterpret_cast<uint32_t*>(tp + b_keys + b_idx + b_counts);
    const uint64_t* ks = code_in;
    const uint32_t* vs = idx_in;
    for (uint32_t pass = 0; pass < kSortPasses; ++pass) {
        uint64_t* kd = (pass & 1u) ? code_out : k_tmp;
        uint32_t* vd = (pass & 1u) ? idx_out : v_tmp;
        const uint32_t shift = 8u * pass;
        sort_count_kernel<<<n_tiles, kSortThreads, 0, stream>>>(ks, n, shift, n_tiles, counts);
        hipError_t e = scan::exclusive_sum(counts, counts, n_counts, sums, stream);
        if (e != hipSuccess) return e;
        sort_scatter_kernel<<<n_tiles, kSortThreads, 0, stream>>>(ks, vs, n, shift, n_tiles, counts, kd, vd);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        ks = kd;
        vs = vd;
    }
    return hipSuccess;
}

// out[i] = in[0] + ... + in[i - 1]; temp == nullptr queries temp_bytes.
extern "C" hipError_t hrr_dev_exclusive_sum(void* temp, size_t* temp_bytes, const uint32_t* in, uint32_t* out,
                                            uint32_t n, hipStream_t stream) {
    if (!temp_bytes) return hipErrorInvalidValue;
    const size_t need = std::max<size_t>(align256((size_t)scan::chunk_count(n) * 4u), 256u);
    if (!temp) {
        *temp_bytes = need;
        return hipSuccess;
    }
    if (*temp_bytes < need) return hipErrorInvalidValue;
    return scan::exclusive_sum(in, out, n, static_cast<uint32_t*>(temp), stream);
}

extern "C" hipError_t hrr_dev_gather(const float* xyz, const uint32_t* perm, uint32_t n, float4* lights,
                                     hipStream_t stream) {
    if (n == 0) return hipSuccess;
    gather_kernel<<<blocks_for(n), kThreads, 0, stream>>>(xyz, perm, n, lights);
    return hipGetLastError();
}

extern "C" hipError_t hrr_dev_init_root(Bfs T, uint32_t n, hipStream_t stream) {
    init_root_kernel<<<1, 64, 0, stream>>>(T, n);
    return hipGetLastError();
}

extern "C" hipError_t hrr_dev_split(Bfs T, const uint64_t* code, uint32_t t0, uint32_t t1, uint32_t leaf,
                                    uint32_t pow2, uint32_t* kids, hipStream_t stream) {
    split_kernel<<<blocks_for(t1 - t0), kThreads, 0, stream>>>(T, code, t0, t1, leaf, pow2, kids);
    return hipGetLastError();
}

extern "C" hipError_t hrr_dev_place(Bfs T, uint32_t t0, uint32_t t1, uint32_t leaf, const uint32_t* prefix,
                                    uint32_t cap, hipStream_t stream) {
    place_kernel<<<blocks_for(t1 - t0), kThreads, 0, stream>>>(T, t0, t1, leaf, prefix, cap);
    return hipGetLastError();
}

extern "C" hipError_t hrr_dev_refit(Bfs T, const float4* lights, uint32_t t0, uint32_t t1, hipStream_t stream) {
    refit_kernel<<<blocks_for(t1 - t0), kThreads, 0, stream>>>(T, lights, t0, t1);
    return hipGetLastError();
}

extern "C" hipError_t hrr_dev_records(Bfs T, const float4* lights, uint32_t t0, uint32_t t1, Node* nodes,
                                      hipStream_t stream) {
    record_kernel<<<blocks_for(t1 - t0), kThreads, 0, stream>>>(T, lights, t0, t1, nodes);
    return hipGetLastError();
}

extern "C" hipError_t hrr_dev_root_leaf_box(const float4* lights, uint32_t n, float* box, hipStream_t stream) {
    root_leaf_box_kernel<<<1, 64, 0, stream>>>(lights, n, box);
    return hipGetLastError();
}
