// hrr_build_device_host.cpp -- host driver of the device hierarchy build
// (kernels in hrr_build_device.hip).  The result is the same hierarchy, record
// for record, as hrr_build_hierarchy builds on the host.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "hrr_ctx.hpp"
#include "hrr_devbuild.hpp"

#define HRR_EXPORT extern "C" __attribute__((visibility("default")))

using hrr::Node;
using hrr::devbuild::Bfs;

extern "C" hipError_t hrr_dev_codes(const float* xyz, uint32_t n, const float* qbox, uint64_t* code, uint32_t* idx,
                                    uint32_t* bad, hipStream_t stream);
extern "C" hipError_t hrr_dev_sort(void* temp, size_t* temp_bytes, const uint64_t* code_in, uint64_t* code_out,
                                   const uint32_t* idx_in, uint32_t* idx_out, uint32_t n, hipStream_t stream);
extern "C" hipError_t hrr_dev_exclusive_sum(void* temp, size_t* temp_bytes, const uint32_t* in, uint32_t* out,
                                            uint32_t n, hipStream_t stream);
extern "C" hipError_t hrr_dev_gather(const float* xyz, const uint32_t* perm, uint32_t n, float4* lights,
                                     hipStream_t stream);
extern "C" hipError_t hrr_dev_init_root(Bfs T, uint32_t n, hipStream_t stream);
extern "C" hipError_t hrr_dev_split(Bfs T, const uint64_t* code, uint32_t t0, uint32_t t1, uint32_t leaf,
                                    uint32_t pow2, uint32_t* kids, hipStream_t stream);
extern "C" hipError_t hrr_dev_place(Bfs T, uint32_t t0, uint32_t t1, uint32_t leaf, const uint32_t* prefix,
                                    uint32_t cap, hipStream_t stream);
extern "C" hipError_t hrr_dev_refit(Bfs T, const float4* lights, uint32_t t0, uint32_t t1, hipStream_t stream);
extern "C" hipError_t hrr_dev_records(Bfs T, const float4* lights, uint32_t t0, uint32_t t1, Node* nodes,
                                      hipStream_t stream);
extern "C" hipError_t hrr_dev_root_leaf_box(const float4* lights, uint32_t n, float* box, hipStream_t stream);

namespace {

// Device allocations of one build, released on every exit path.
struct Temps {
    std::vector<void*> ptrs;
    ~Temps() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    hipError_t get(T** p, size_t count) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e != hipSuccess) return e;
        ptrs.push_back(q);
        *p = static_cast<T*>(q);
        return hipSuccess;
    }
};

}  // namespace

HRR_EXPORT hrr_status hrr_build_hierarchy_device(hrr_ctx* ctx, const float* lights_xyz_dev, uint32_t n_lights,
                                                 uint32_t leaf_arg, const float* box, void* stream_v,
                                                 hrr_hierarchy** out) {
    using namespace hrr;
    if (!ctx || !out) return fail(HRR_E_INVALID, "hrr_build_hierarchy_device: null argument");
    *out = nullptr;
    if (n_lights > 0 && !lights_xyz_dev) return fail(HRR_E_INVALID, "hrr_build_hierarchy_device: null lights");
    uint32_t leaf_size, split;
    if (!parse_leaf_arg(leaf_arg, &leaf_size, &split))
        return fail(HRR_E_INVALID, "leaf_size must be in [1, 8], optionally with HRR_SPLIT_POW2");
    if (n_lights >= kMaxLights) return fail(HRR_E_INVALID, "at most %u lights", kMaxLights - 1);
    float qbox[6] = {0.f, 0.f, 0.f, 1.f, 1.f, 1.f};
    if (box) {
        for (int k = 0; k < 3; ++k)
            if (!isfinite(box[k]) || !isfinite(box[3 + k]) || !(box[3 + k] > box[k]))
                return fail(HRR_E_INVALID, "box must be finite with hi > lo");
        memcpy(qbox, box, sizeof qbox);
    }
    hipStream_t stream = (hipStream_t)stream_v;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const uint32_t n = n_lights;
    const uint32_t max_internal = n > leaf_size ? n - 1 : 0;

    hrr_hierarchy* h = new hrr_hierarchy();
    h->owner = ctx;
    h->n_lights = n;
    h->leaf_size = leaf_size;
    h->split = split;
    h->host_copies = false;
    auto fail_free = [&](hrr_status st) {
        hrr_free_hierarchy(ctx, h);
        return st;
    };
    // node records: allocated once their number is known (after the refit)
    if ((max_internal == 0 && (e = hipMalloc((void**)&h->d_nodes, sizeof(Node))) != hipSuccess) ||
        (e = hipMalloc((void**)&h->d_lights, std::max<size_t>(n, 1) * 4 * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void**)&h->d_perm, std::max<size_t>(n, 1) * sizeof(uint32_t))) != hipSuccess)
        return fail_free(hip_fail(e, "hierarchy allocation"));
    h->device_bytes = (max_internal == 0 ? sizeof(Node) : 0) + std::max<size_t>(n, 1) * 20;

    Temps tmp;
    uint64_t *code_in = nullptr, *code = nullptr;
    uint32_t *idx_in = nullptr, *bad = nullptr, *kids = nullptr, *prefix = nullptr, *pin = nullptr;
    float* d_box = nullptr;
    Bfs T{};
    if ((e = tmp.get(&code_in, n)) != hipSuccess || (e = tmp.get(&code, n)) != hipSuccess ||
        (e = tmp.get(&idx_in, n)) != hipSuccess || (e = tmp.get(&bad, 1)) != hipSuccess ||
        (e = tmp.get(&d_box, 6)) != hipSuccess)
        return fail_free(hip_fail(e, "build scratch"));
    if (max_internal &&
        ((e = tmp.get(&T.a, max_internal)) != hipSuccess || (e = tmp.get(&T.c, max_internal)) != hipSuccess ||
         (e = tmp.get(&T.b, max_internal)) != hipSuccess || (e = tmp.get(&T.l, max_internal)) != hipSuccess ||
         (e = tmp.get(&T.r, max_internal)) != hipSuccess || (e = tmp.get(&T.cnt, max_internal)) != hipSuccess ||
         (e = tmp.get(&T.pre, max_internal)) != hipSuccess || (e = tmp.get(&T.own, max_internal)) != hipSuccess || (e = tmp.get(&T.box, 6 * (size_t)max_internal)) != hipSuccess ||
         (e = tmp.get(&kids, max_internal)) != hipSuccess || (e = tmp.get(&prefix, max_internal)) != hipSuccess))
        return fail_free(hip_fail(e, "build scratch"));
    if ((e = hipHostMalloc((void**)&pin, 16 * sizeof(uint32_t), hipHostMallocDefault)) != hipSuccess)
        return fail_free(hip_fail(e, "build staging"));
    struct PinFree {
        uint32_t* p;
        ~PinFree() { (void)hipHostFree(p); }
    } pin_free{pin};

    // 1-3: codes, sort, gather
    if ((e = hipMemsetAsync(bad, 0, sizeof(uint32_t), stream)) != hipSuccess) return fail_free(hip_fail(e, "build"));
    if (n) {
        if ((e = hrr_dev_codes(lights_xyz_dev, n, qbox, code_in, idx_in, bad, stream)) != hipSuccess)
            return fail_free(hip_fail(e, "Morton codes"));
        size_t sort_bytes = 0;
        if ((e = hrr_dev_sort(nullptr, &sort_bytes, code_in, code, idx_in, h->d_perm, n, stream)) != hipSuccess)
            return fail_free(hip_fail(e, "sort size"));
        void* sort_tmp = nullptr;
        if ((e = tmp.get((unsigned char**)&sort_tmp, sort_bytes)) != hipSuccess) return fail_free(hip_fail(e, "sort scratch"));
        if ((e = hrr_dev_sort(sort_tmp, &sort_bytes, code_in, code, idx_in, h->d_perm, n, stream)) != hipSuccess)
            return fail_free(hip_fail(e, "sort"));
        if ((e = hrr_dev_gather(lights_xyz_dev, h->d_perm, n, reinterpret_cast<float4*>(h->d_lights), stream)) !=
            hipSuccess)
            return fail_free(hip_fail(e, "gather"));
    }

    // 4: breadth-first levels
    std::vector<uint32_t> off{0};
    if (max_internal) {
        size_t scan_bytes = 0;
        if ((e = hrr_dev_exclusive_sum(nullptr, &scan_bytes, kids, prefix, max_internal, stream)) != hipSuccess)
            return fail_free(hip_fail(e, "scan size"));
        void* scan_tmp = nullptr;
        if ((e = tmp.get((unsigned char**)&scan_tmp, scan_bytes)) != hipSuccess) return fail_free(hip_fail(e, "scan scratch"));
        if ((e = hrr_dev_init_root(T, n, stream)) != hipSuccess) return fail_free(hip_fail(e, "root"));
        uint32_t t0 = 0, t1 = 1;
        off.push_back(1);
        while (t1 > t0) {
            const uint32_t m = t1 - t0;
            if ((e = hrr_dev_split(T, code, t0, t1, leaf_size, split == HRR_SPLIT_POW2 ? 1u : 0u, kids, stream)) != hipSuccess ||
                (e = hrr_dev_exclusive_sum(scan_tmp, &scan_bytes, kids, prefix, m, stream)) != hipSuccess ||
                (e = hipMemcpyAsync(pin, prefix + (m - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, stream)) !=
                    hipSuccess ||
                (e = hipMemcpyAsync(pin + 1, kids + (m - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, stream)) !=
                    hipSuccess ||
                (e = hrr_dev_place(T, t0, t1, leaf_size, prefix, max_internal, stream)) != hipSuccess ||
                (e = hipStreamSynchronize(stream)) != hipSuccess)
                return fail_free(hip_fail(e, "level split"));
            const uint64_t next = (uint64_t)pin[0] + pin[1];
            if ((uint64_t)t1 + next > max_internal) return fail_free(fail(HRR_E_DEVICE, "device build: node count overflow"));
            t0 = t1;
            t1 += (uint32_t)next;
            if (t1 > t0) off.push_back(t1);
        }
        const size_t levels = off.size() - 1;
        // 5: refit, deepest level first; 6: records, root level first
        for (size_t L = levels; L-- > 0;)
            if ((e = hrr_dev_refit(T, reinterpret_cast<const float4*>(h->d_lights), off[L], off[L + 1], stream)) !=
                hipSuccess)
                return fail_free(hip_fail(e, "refit"));
        // records: the root, the unused record 1, then one sibling pair per
        // node with an internal child (the root's subtree count)
        if ((e = hipMemcpyAsync(pin + 3, T.cnt, sizeof(uint32_t), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
            (e = hipStreamSynchronize(stream)) != hipSuccess)
            return fail_free(hip_fail(e, "record count"));
        if (pin[3] > max_internal) return fail_free(fail(HRR_E_DEVICE, "device build: record count overflow"));
        const uint32_t n_records = 2u * (1u + pin[3]);
        if ((e = hipMalloc((void**)&h->d_nodes, (size_t)n_records * sizeof(Node))) != hipSuccess ||
            (e = hipMemsetAsync(h->d_nodes, 0, (size_t)n_records * sizeof(Node), stream)) != hipSuccess)
            return fail_free(hip_fail(e, "node records"));
        h->device_bytes += (size_t)n_records * sizeof(Node);
        for (size_t L = 0; L < levels; ++L)
            if ((e = hrr_dev_records(T, reinterpret_cast<const float4*>(h->d_lights), off[L], off[L + 1], h->d_nodes,
                                     stream)) != hipSuccess)
                return fail_free(hip_fail(e, "records"));
        if ((e = hipMemcpyAsync(d_box, T.box, 6 * sizeof(float), hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return fail_free(hip_fail(e, "root box"));
        h->n_nodes = n_records;
        h->depth = (uint32_t)(levels - 1);
        const hrr_status st = attach_frontier(h, stream);
        if (st != HRR_OK) return fail_free(st);
        if ((e = hipMemcpyAsync(pin + 4, h->d_frontier + (size_t)kFrontierMax * kFrontierFloats, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, stream)) != hipSuccess)
            return fail_free(hip_fail(e, "hierarchy top"));
    } else if (n) {
        if ((e = hrr_dev_root_leaf_box(reinterpret_cast<const float4*>(h->d_lights), n, d_box, stream)) != hipSuccess)
            return fail_free(hip_fail(e, "root box"));
    }
    float root_box[6] = {0, 0, 0, 0, 0, 0};
    if (n && (e = hipMemcpyAsync(root_box, d_box, sizeof root_box, hipMemcpyDeviceToHost, stream)) != hipSuccess)
        return fail_free(hip_fail(e, "root box"));
    if ((e = hipMemcpyAsync(pin + 2, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return fail_free(hip_fail(e, "device build"));
    if (pin[2]) return fail_free(fail(HRR_E_INVALID, "non-finite light coordinate"));
    if (h->d_frontier) h->n_frontier = pin[4];
    memcpy(h->box, root_box, sizeof root_box);
    *out = h;
    return HRR_OK;
}
