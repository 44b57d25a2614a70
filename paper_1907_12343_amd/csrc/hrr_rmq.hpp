// hrr_rmq.hpp -- range minimum of the Cranley-Patterson rotated base-2
// radical inverse over an index interval, for gfx950 device code.
//
// Problem (Pantaleoni, "Blue-Noise Dithered QMC Hierarchical Russian
// Roulette", Section 1 and Section 2): for an eye with rotation r, find
//     k = argmin_{i in [a,b)} phi(i),   phi(i) = (Phi_2(i) + r) mod 1,
// and v = phi(k).  Everything is 32-bit fixed point: Phi_2(i) is
// bit_reverse32(i) and phi(i) = bit_reverse32(i) + R (mod 2^32), R = r 2^32.
//
// Orders used below.  Comparing Phi_2 values compares indices from their
// lowest bit upward ("reflected" order): the index whose lowest differing bit
// is 0 has the smaller radical inverse.  The threshold index
// k_r = Phi_2^{-1}(1 - r) = bit_reverse32(-R) splits the range into indices
// whose radical inverse is at least 1 - r (their phi wraps below r, Section
// 2's second case) and the rest (phi >= r, third case).  The minimum is:
//   (1) k_r itself when it lies in [a,b) (phi = 0, first case);
//   (2) otherwise the reflected-smallest index above k_r, if any index in
//       [a,b) is above it: it agrees with k_r on its low bits and has a 1 at
//       the highest possible bit where k_r has a 0 (the "left-to-right"
//       search of Section 2, highest bit first, then the refinement of
//       Algorithm 3 inside the set of indices sharing that prefix);
//   (3) otherwise the reflected-smallest index of the whole range, i.e. the
//       one with the most trailing zeros (the problem of Algorithm 1), which
//       Section 2's "right-to-left" sweep reaches by trying exactly i
//       trailing zeros for i = 0, 1, ...
//
// Four implementations compute the same k:
//   rmq_paper  -- the paper's method: case test, left-to-right sweep with
//                 refinement, right-to-left sweep.  Written from the paper's
//                 description with gfx950-friendly changes that keep the
//                 result: the sweep visits only the zero bits of k_r (the
//                 paper's steps at set bits only merge a's bits, which the
//                 candidate construction does directly), the refinement
//                 stops at the first candidate at or past b, the right-to-left
//                 sweep stops once no index in [a,b) has i trailing zeros, and
//                 every shift by 32 is guarded (VALU shifts wrap at 32).  The
//                 case a == 0 with no index above the threshold returns 0, the
//                 reflected-smallest index overall (the printed sweep stops at
//                 i = B - 1 and would miss it).
//   rmq_paper_pruned -- the same sweeps as loops, refining only the one
//                 candidate whose prefix class meets [a,b).
//   rmq_paper_select -- the same sweeps with every candidate position tested
//                 at once by bit arithmetic, then Algorithm 3's refinement of
//                 the winning prefix class (the default: no divergent scan
//                 loops on the VALU, only the short refinement walk).
//   rmq_direct -- the same three cases, each resolved in O(1) bit
//                 arithmetic, refinement included (an ablation, no loops).
//
// All functions are __host__ __device__ so that host-side unit harnesses can
// exercise exactly the code the kernels run.
#pragma once

#include <stdint.h>

#ifndef HRR_HD
#if defined(__HIPCC__)
#define HRR_HD __host__ __device__ __forceinline__
#else
#define HRR_HD inline
#endif
#endif

namespace hrr {

HRR_HD uint32_t bit_reverse(uint32_t x) { return __builtin_bitreverse32(x); }

// 2^n - 1 for n in [0, 32]  (a plain 1u << 32 is 1 on the VALU).
HRR_HD uint32_t low_mask(int n) { return n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u); }

// index of the highest / lowest set bit; x must be non-zero
HRR_HD int top_bit(uint32_t x) { return 31 - __builtin_clz(x); }
HRR_HD int bottom_bit(uint32_t x) { return __builtin_ctz(x); }

HRR_HD bool in_range(uint32_t x, uint32_t a, uint32_t b) { return x - a < b - a; }

// k_r: the index whose radical inverse equals 1 - r (mod 1).
HRR_HD uint32_t threshold_index(uint32_t R) { return bit_reverse(0u - R); }

HRR_HD uint32_t rotated(uint32_t i, uint32_t R) { return bit_reverse(i) + R; }

// Refinement (Algorithm 3's role).  x carries a fixed low prefix (bits below
// `keep`).  Among the indices of [a,b) that share that prefix, the reflected
// order prefers a 0 at the lowest free bit, then at the next one, and so on.
// Adding 2^j at a set bit j turns the run of ones starting at j into zeros and
// sets the next zero bit: the smallest index above x with a 0 at bit j.  The
// walk takes each such step that lands in [a,b), lowest bit first.  Steps only
// grow x, so once x + 2^j reaches b every later step does too.
HRR_HD uint32_t refine(uint32_t x, int keep, uint32_t a, uint32_t b) {
    uint32_t todo = keep >= 32 ? 0u : (x & ~low_mask(keep));
    while (todo) {
        const int j = bottom_bit(todo);
        const uint32_t step = 1u << j;
        if (x >= b || step >= b - x) break;
        const uint32_t y = x + step;
        if (y >= a) x = y;
        todo = j >= 31 ? 0u : (x & ~low_mask(j + 1));
    }
    return x;
}

// The same walk for a class that meets [a,b), started from seed_candidate:
// the seed is either the smallest member at or above a (then below b), or
// one class step below it with bit `keep` set, so the first step lands on
// that member.  Every step therefore ends at or above a, and only the bound
// b is tested; the bits above j are 0u - (2u << j) (none for j = 31).  The
// first step that would reach b ends the walk by emptying `todo`, so the
// loop has a single exit (on the GPU: one lane mask to maintain per trip).
HRR_HD uint32_t refine_inside(uint32_t x, int keep, uint32_t b) {
    uint32_t todo = x & ~low_mask(keep);   // keep = 32: nothing to walk
    while (todo) {
        const int j = bottom_bit(todo);
        const uint32_t step = 1u << j;
        const bool inside = step < b - x;
        x = inside ? x + step : x;
        todo = inside ? x & (0u - (2u << j)) : 0u;
    }
    return x;
}

// Candidate with a given low prefix: a's bits above bit `i`, a 1 at bit i,
// and `low` (bits below i).  When that falls below a, one more bit above i is
// set to lift it into the range before refining.  Section 2: keep a's set
// bits met during the sweep; set an extra 1 at i + 1 when the prefix of k_r is
// smaller than a's.
HRR_HD uint32_t seed_candidate(uint32_t a, int i, uint32_t low) {
    const uint32_t x = (a & ~low_mask(i + 1)) | (1u << i) | low;
    return x < a && i < 31 ? x | (2u << i) : x;
}

// The paper's range-minimum method (Section 2, Algorithms 2 and 3).
HRR_HD uint32_t rmq_paper(uint32_t a, uint32_t b, uint32_t kr) {
    // first case: phi vanishes inside the range
    if (in_range(kr, a, b)) return kr;
    const int kp = kr ? bottom_bit(kr) : 32;
    const int bh = top_bit(b);
    // Left-to-right sweep: flip the highest possible zero bit of k_r, from
    // bit b_h down to k_p, keeping k_r's bits below it; the first candidate
    // that refines into [a,b) is the answer.
    if (kp <= bh) {
        uint32_t zeros = ~kr & low_mask(bh + 1) & ~low_mask(kp);
        while (zeros) {
            const int i = top_bit(zeros);
            zeros ^= 1u << i;
            const uint32_t x = refine(seed_candidate(a, i, kr & low_mask(i)), i + 1, a, b);
            if (in_range(x, a, b)) return x;
        }
    }
    // Right-to-left sweep: candidates with exactly i trailing zeros.  Below
    // k_p they are above the threshold and the last one found wins at i ==
    // k_p; past k_p (no index above the threshold) the one with the most
    // trailing zeros is the minimum.
    uint32_t k = b;   // b marks "nothing found"
    for (int i = 0; i < 32; ++i) {
        if (i == kp && k != b) return k;
        if (a != 0 && ((a - 1u) | low_mask(i)) >= b - 1u) break;
        const uint32_t x = refine(seed_candidate(a, i, 0u), i + 1, a, b);
        if (in_range(x, a, b)) k = x;
    }
    return a == 0 ? 0u : k;
}

// Does [a,b) hold an index whose bits below i+1 equal `prefix`
// (prefix < 2^(i+1))?  The first index at or above a with that residue is
// a + ((prefix - a) mod 2^(i+1)).
HRR_HD bool prefix_in_range(uint32_t prefix, int i, uint32_t a, uint32_t b) {
    return ((prefix - a) & low_mask(i + 1)) < b - a;
}

// The paper's method with its sweeps pruned by that O(1) membership test:
// the left-to-right sweep still visits the zero bits of k_r from b_h down to
// k_p, the right-to-left sweep still tries "exactly i trailing zeros" for
// i = 0, 1, ..., but only the position whose prefix class meets [a,b) is
// refined (Algorithm 3 finds its reflected-smallest member), through a single
// refinement call.  A prefix class that misses the range cannot refine into
// it, so skipping it never changes the answer; the right-to-left sweep
// remembers the last position that meets the range and refines it once.
HRR_HD uint32_t rmq_paper_pruned(uint32_t a, uint32_t b, uint32_t kr) {
    if (in_range(kr, a, b)) return kr;
    const int kp = kr ? bottom_bit(kr) : 32;
    const int bh = top_bit(b);
    int pos = -1;
    uint32_t low = 0u;
    if (kp <= bh) {
        uint32_t zeros = ~kr & low_mask(bh + 1) & ~low_mask(kp);
        while (zeros) {
            const int i = top_bit(zeros);
            zeros ^= 1u << i;
            const uint32_t prefix = (kr & low_mask(i)) | (1u << i);
            if (prefix_in_range(prefix, i, a, b)) {
                pos = i;
                low = kr & low_mask(i);
                break;
            }
        }
    }
    if (pos < 0) {
        for (int i = 0; i < 32; ++i) {
            if (i == kp) {
                if (pos >= 0) break;     // an index above the threshold exists
                if (a == 0) return 0u;   // none: 0 is the reflected-smallest index
            }
            if (a != 0 && ((a - 1u) | low_mask(i)) >= b - 1u) break;
            if (prefix_in_range(1u << i, i, a, b)) pos = i;
        }
        low = 0u;
    }
    return refine(seed_candidate(a, pos, low), pos + 1, a, b);
}

// Index with the most trailing zeros in [lo, hi] (lo <= hi): below the highest
// bit where lo and hi differ, hi with that bit kept and the rest cleared --
// unless lo itself is already zero from that bit down.  Written with selects
// only (no divergent branches on the GPU).
HRR_HD uint32_t most_trailing_zeros(uint32_t lo, uint32_t hi) {
    const uint32_t x = lo ^ hi;
    const int h = x ? top_bit(x) : 0;
    const uint32_t r = hi & ~low_mask(h);
    return (x == 0u || (lo & low_mask(h + 1)) == 0u) ? lo : r;
}

// Same result in O(1): the candidate set for "first difference at bit i" is
// an arithmetic progression of step 2^(i+1).  When that step exceeds the range
// length it holds at most one index, a + ((k_r - a + 2^i) mod 2^(i+1)), and
// above the length's top bit g only the lowest set bit of (k_r - a) above g
// can produce one; below g every zero bit of k_r produces a non-empty set, and
// the refinement is the most-trailing-zeros index of the progression's
// quotient range.
HRR_HD uint32_t rmq_direct(uint32_t a, uint32_t b, uint32_t kr) {
    if (in_range(kr, a, b)) return kr;
    const uint32_t len = b - a;
    const int g = top_bit(len);
    const uint32_t d = kr - a;
    const uint32_t dlow = d & low_mask(g + 1);
    if (g < 31) {
        const uint32_t dhi = d >> (g + 1);
        if (dhi) {
            const int i = bottom_bit(dhi) + g + 1;
            if (!((kr >> i) & 1u) && dlow < len) return a + ((d & low_mask(i + 1)) ^ (1u << i));
        }
    }
    if (!((kr >> g) & 1u)) {
        const uint32_t t = dlow ^ (1u << g);
        if (t < len) return a + t;
    }
    const uint32_t z = ~kr & low_mask(g);
    if (z) {
        const int i = top_bit(z);
        const uint32_t P = (kr & low_mask(i)) | (1u << i);
        const uint32_t t = (d & low_mask(i + 1)) ^ (1u << i);
        const uint32_t qlo = (a + t) >> (i + 1);
        const uint32_t qhi = (b - 1u - P) >> (i + 1);
        return P + (most_trailing_zeros(qlo, qhi) << (i + 1));
    }
    return most_trailing_zeros(a, b - 1u);
}

// The paper's method with both sweeps evaluated for all bit positions at
// once.  The sweeps look for the highest zero bit i of k_r whose prefix class
// (k_r's bits below i, a 1 at i) meets [a,b); left-to-right positions
// (>= k_p) outrank right-to-left ones (< k_p) and higher outranks lower, so
// the winner is simply the highest such bit.  With g the top bit of b - a:
// above g a class meets the range only at the lowest set bit of k_r - a above
// g (one member, a + ((k_r - a + 2^i) mod 2^(i+1))); at g the same single-
// member test applies; below g every class meets the range, so the highest
// zero bit of k_r below g wins and Algorithm 3's refinement walks it to its
// reflected-smallest member.  No class: the range's reflected-smallest index,
// the one with the most trailing zeros (Algorithm 1's answer) -- which is the
// same walk started from a with no bit held fixed: each step clears the lowest
// set bit while the result stays below b.
HRR_HD uint32_t rmq_paper_select(uint32_t a, uint32_t b, uint32_t kr) {
    // Every case is evaluated with selects; only the refinement walk, needed
    // when no single-member class wins, is a (short) loop.
    const uint32_t len = b - a;
    const uint32_t d = kr - a;
    const bool first = d < len;                  // k_r itself is in the range
    const int g = top_bit(len);
    const uint32_t mg = low_mask(g + 1);
    const uint32_t dlow = d & mg;
    const uint32_t dhi = d & ~mg;
    // above g: the lowest set bit i of (k_r - a) above g; its class holds the
    // single index a + ((d & low_mask(i + 1)) ^ 2^i) = a + dlow (the bits of d
    // between g and i are zero and bit i is set)
    const int i_hi = dhi ? bottom_bit(dhi) : 0;
    const bool above = dhi != 0u && !((kr >> i_hi) & 1u) && dlow < len;
    // at g: the single candidate a + (dlow ^ 2^g)
    const uint32_t t_g = dlow ^ (1u << g);
    const bool at_g = !((kr >> g) & 1u) && t_g < len;
    // below g: every zero bit of k_r has a non-empty class; the highest wins
    const uint32_t z = ~kr & low_mask(g);
    const bool single = first || above || at_g;
    // the walk: from the class seed (below g the class step 2^(i+1) is at most
    // the range length, so its smallest member at or above a lies inside
    // [a,b)), or from a with nothing held fixed (no class); not at all when a
    // single candidate wins
    const int i = top_bit(z | 1u);
    const bool cls = !single && z != 0u;
    const uint32_t seed = seed_candidate(a, i, kr & low_mask(i));   // evaluated on every lane (no branch)
    const uint32_t x0 = cls ? seed : a;
    const int keep = single ? 32 : (cls ? i + 1 : 0);
    uint32_t k = refine_inside(x0, keep, b);
    k = at_g ? a + t_g : k;
    k = above ? a + dlow : k;
    return first ? kr : k;
}

// Not the paper's method (an ablation): the range split into maximal aligned
// blocks [p, p + 2^s).  Inside one block bitreverse(p + q) = bitreverse(p) +
// bitreverse_s(q) 2^(32-s), so with u = bitreverse(p) + R the block's values
// are u + x 2^(32-s) (mod 2^32) over all x < 2^s: the minimum is u mod
// 2^(32-s), at x = -(u div 2^(32-s)) mod 2^s, i.e. at index p +
// bitreverse_s(x).  The range minimum is the smallest block minimum (the
// values are distinct).  R comes back from k_r = bitreverse(-R).
HRR_HD uint32_t rmq_dyadic(uint32_t a, uint32_t b, uint32_t kr) {
    const uint32_t R = 0u - bit_reverse(kr);
    uint32_t best_v = 0, best_k = a;
    bool found = false;
    uint32_t p = a;
    while (p < b) {
        const int room = top_bit(b - p);                  // largest s with 2^s <= b - p
        const int s = p ? (bottom_bit(p) < room ? bottom_bit(p) : room) : room;
        const uint32_t u = bit_reverse(p) + R;
        uint32_t v = u, k = p;
        if (s > 0) {
            const int sh = 32 - s;                        // s <= 31: b < 2^32
            v = u & low_mask(sh);
            const uint32_t x = (0u - (u >> sh)) & low_mask(s);
            k = p + (bit_reverse(x) >> sh);
        }
        if (!found || v < best_v) {
            best_v = v;
            best_k = k;
            found = true;
        }
        if (b - p <= (1u << s)) break;                    // the last block (no wrap past 2^32 - 1)
        p += 1u << s;
    }
    return best_k;
}

// METHOD 0: the paper's sweeps, candidate positions selected bit-parallel,
//           Algorithm 3 refinement (default);
//        1: closed form of every step (ablation, no refinement walk);
//        2: the paper's sweeps refining every candidate in turn (ablation);
//        3: the paper's sweeps as loops, refining only the candidate that
//           meets the range (ablation);
//        4: the dyadic block decomposition (ablation, not the paper's method);
//        5: the default method; the traversal then also recomputes the minimum
//           of the child that holds the parent's argmin (ablation of the reuse).
template <int METHOD>
HRR_HD uint32_t rmq(uint32_t a, uint32_t b, uint32_t kr) {
    if (METHOD == 1) return rmq_direct(a, b, kr);
    if (METHOD == 2) return rmq_paper(a, b, kr);
    if (METHOD == 3) return rmq_paper_pruned(a, b, kr);
    if (METHOD == 4) return rmq_dyadic(a, b, kr);
    return rmq_paper_select(a, b, kr);
}

}  // namespace hrr
