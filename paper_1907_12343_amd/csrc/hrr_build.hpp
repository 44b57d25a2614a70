// hrr_build.hpp -- host-side light hierarchy (see hrr_build.cpp).
#pragma once

#include <stdint.h>

#include <vector>

#include "hrr_types.hpp"

namespace hrr {

struct HostHierarchy {
    uint32_t n_lights = 0, leaf_size = 1, depth = 0;
    bool pow2 = false;                // split rule: largest power of two below the length
    std::vector<Node> nodes;          // node records in sibling pairs (hrr_types.hpp)
    std::vector<float> sorted_xyz;    // 3 per light, sequence order
    std::vector<uint32_t> perm;       // perm[i] = original index of sequence index i
    float box[6] = {0, 0, 0, 0, 0, 0};
};

uint64_t morton_code(float x, float y, float z, const float* box);

// false if a coordinate is not finite; pow2 selects the power-of-two split
bool build_hierarchy(const float* xyz, uint32_t n, uint32_t leaf, bool pow2, const float* box, HostHierarchy& out);

}  // namespace hrr
