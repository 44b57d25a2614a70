// hrr_build.cpp -- host construction of the light hierarchy.
//
// Section 1 of the paper assumes the light vertices are sorted by a spatial
// hierarchy so that every leaf has a sequence index i in [0, N_l) and every
// internal node is a contiguous index range [a_n, b_n); spatial sorting is
// what lets the low-discrepancy sequence's stratification carry over to the
// lights.  Here the order is a Morton (Z-order) sort and the hierarchy is the
// binary radix split of that order:
//   code   : 21-bit cell indices of x, y, z against a box, interleaved with x
//            in the highest bit of each triple (63-bit code);
//   order  : ascending (code, original index);
//   split  : a node [a,b) with more than leaf_size lights is cut at the first
//            index whose code has the highest bit where code[a] and
//            code[b-1] differ; equal codes are cut at the midpoint.  The
//            power-of-two rule cuts after a + 2^k, 2^k the largest power of
//            two below b - a (every left child an aligned index block);
//   boxes  : exact fp32 min/max of the lights below each child.
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "hrr_build.hpp"

#pragma clang fp contract(off)

namespace hrr {

namespace {

// Spread the low 21 bits of v so that bit k lands on bit 3k.
uint64_t spread_bits3(uint32_t v) {
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

uint32_t cell21(float x, float lo, float hi) {
    float u = (x - lo) / (hi - lo);
    if (!(u > 0.0f)) u = 0.0f;
    if (u > 1.0f) u = 1.0f;
    const uint32_t q = (uint32_t)(u * 2097152.0f);
    return q < 2097151u ? q : 2097151u;
}

struct Box {
    float lo[3], hi[3];
};

Box box_of(const std::vector<float>& xyz, uint32_t a, uint32_t b) {
    Box bx;
    for (int k = 0; k < 3; ++k) {
        bx.lo[k] = xyz[3 * (size_t)a + k];
        bx.hi[k] = bx.lo[k];
    }
    for (uint32_t i = a + 1; i < b; ++i)
        for (int k = 0; k < 3; ++k) {
            const float v = xyz[3 * (size_t)i + k];
            bx.lo[k] = std::min(bx.lo[k], v);
            bx.hi[k] = std::max(bx.hi[k], v);
        }
    return bx;
}

Box merge(const Box& p, const Box& q) {
    Box r;
    for (int k = 0; k < 3; ++k) {
        r.lo[k] = std::min(p.lo[k], q.lo[k]);
        r.hi[k] = std::max(p.hi[k], q.hi[k]);
    }
    return r;
}

struct Builder {
    const std::vector<uint64_t>& code;
    const std::vector<float>& xyz;   // sorted
    uint32_t leaf;
    bool pow2;
    std::vector<Node>& nodes;
    uint32_t depth_max = 0;

    uint32_t split(uint32_t a, uint32_t b) const {
        if (pow2) {
            const uint32_t len = b - a;
            const uint32_t k = 1u << (31 - __builtin_clz(len - 1u));   // largest 2^k < len (len >= 2)
            return a + k;
        }
        const uint64_t ca = code[a], cb = code[b - 1];
        if (ca == cb) return a + (b - a) / 2;
        const int h = 63 - __builtin_clzll(ca ^ cb);
        // first index in (a, b) whose code has bit h set (codes share the bits above h)
        uint32_t lo = a, hi = b - 1;   // code[lo] has bit h clear, code[hi] set
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if ((code[mid] >> h) & 1u) hi = mid; else lo = mid;
        }
        return hi;
    }

    // Builds the internal node [a,b) into record `me`; returns its box.  A
    // node with an internal child takes the next sibling pair of records
    // when it is built (pairs in preorder of their owners).
    Box build(uint32_t a, uint32_t b, uint32_t depth, uint32_t me) {
        depth_max = std::max(depth_max, depth);
        const uint32_t c = split(a, b);
        const bool in_l = c - a > leaf, in_r = b - c > leaf;
        uint32_t first = 0xFFFFFFFFu;
        if (in_l || in_r) {
            first = (uint32_t)nodes.size();
            nodes.resize(first + 2);
        }
        const Box bl = in_l ? build(a, c, depth + 1, first) : box_of(xyz, a, c);
        const Box br = in_r ? build(c, b, depth + 1, first + 1) : box_of(xyz, c, b);
        Node& n = nodes[me];
        for (int k = 0; k < 3; ++k) {
            n.lo_l[k] = bl.lo[k];
            n.hi_l[k] = bl.hi[k];
            n.lo_r[k] = br.lo[k];
            n.hi_r[k] = br.hi[k];
        }
        n.a = a;
        n.c = c;
        n.b = b;
        n.first = first;
        return merge(bl, br);
    }
};

}  // namespace

uint64_t morton_code(float x, float y, float z, const float* box) {
    static const float unit[6] = {0.f, 0.f, 0.f, 1.f, 1.f, 1.f};
    const float* bx = box ? box : unit;
    return (spread_bits3(cell21(x, bx[0], bx[3])) << 2) | (spread_bits3(cell21(y, bx[1], bx[4])) << 1) |
           spread_bits3(cell21(z, bx[2], bx[5]));
}

bool build_hierarchy(const float* xyz, uint32_t n, uint32_t leaf, bool pow2, const float* box, HostHierarchy& out) {
    for (size_t q = 0; q < 3 * (size_t)n; ++q)
        if (!std::isfinite(xyz[q])) return false;
    struct Key {
        uint64_t code;
        uint32_t id;
    };
    std::vector<Key> keys(n);
    for (uint32_t i = 0; i < n; ++i)
        keys[i] = {morton_code(xyz[3 * (size_t)i], xyz[3 * (size_t)i + 1], xyz[3 * (size_t)i + 2], box), i};
    std::sort(keys.begin(), keys.end(), [](const Key& p, const Key& q) {
        return p.code != q.code ? p.code < q.code : p.id < q.id;
    });
    out.n_lights = n;
    out.leaf_size = leaf;
    out.pow2 = pow2;
    out.perm.resize(n);
    out.sorted_xyz.resize(3 * (size_t)n);
    std::vector<uint64_t> code(n);
    for (uint32_t i = 0; i < n; ++i) {
        out.perm[i] = keys[i].id;
        code[i] = keys[i].code;
        for (int k = 0; k < 3; ++k) out.sorted_xyz[3 * (size_t)i + k] = xyz[3 * (size_t)keys[i].id + k];
    }
    out.nodes.clear();
    out.depth = 0;
    if (n == 0) {
        for (int k = 0; k < 6; ++k) out.box[k] = 0.0f;
        return true;
    }
    Builder B{code, out.sorted_xyz, leaf, pow2, out.nodes};
    Box root;
    if (n <= leaf) {
        root = box_of(out.sorted_xyz, 0, n);
    } else {
        out.nodes.reserve(2 * (size_t)(n / leaf) + 2);
        out.nodes.resize(2);   // the root, and the unused record 1
        root = B.build(0, n, 0, 0);
    }
    out.depth = B.depth_max;
    for (int k = 0; k < 3; ++k) {
        out.box[k] = root.lo[k];
        out.box[3 + k] = root.hi[k];
    }
    return true;
}

}  // namespace hrr
