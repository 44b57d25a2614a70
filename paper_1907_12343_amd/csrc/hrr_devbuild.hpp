// hrr_devbuild.hpp -- tables of the device hierarchy build, shared by its
// kernels (hrr_build_device.hip) and its host driver (hrr_api.cpp).
#pragma once

#include <stdint.h>

namespace hrr {
namespace devbuild {

// Internal nodes in breadth-first order (device arrays).
struct Bfs {
    uint32_t* a;     // range [a, b) split at c
    uint32_t* c;
    uint32_t* b;
    int32_t* l;      // breadth-first number of the internal left child, or -1
    int32_t* r;      // same for the right child
    uint32_t* cnt;   // pair owners (nodes with an internal child) in the subtree
    uint32_t* pre;   // record number
    uint32_t* own;   // pair owners before the node in depth-first preorder
    float* box;      // 6 floats per node: lo xyz, hi xyz of its own box
};

// Morton quantisation box, lo xyz and hi xyz.
struct QBox {
    float lo[3], hi[3];
};

}  // namespace devbuild
}  // namespace hrr
