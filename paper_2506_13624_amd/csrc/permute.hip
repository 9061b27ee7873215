// Per-node data between a caller's node order and the library's
// stage-major breadth-first order (the node sets of Sec. II-B do not fix an
// order; the library's kernels need the stage-major one).  One pass over
// the array: a gather into the library's order, or a scatter back.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "bmpc_internal.hpp"

namespace {

constexpr int kThreads = 256;

// element e of library node k sits at lib_index, the same element of the
// caller's node order[k] at caller_index; the thread index runs fastest
// over whichever of the two is contiguous in the layout, so one side of
// every copy is coalesced and the other reads or writes whole node rows
// (node-major) or gathers within one entry's array (entry-major)
__global__ void __launch_bounds__(kThreads)
k_permute_nodes(const int32_t* __restrict__ order, long N, long W, int elem_major, int to_caller,
                const double* __restrict__ src, double* __restrict__ dst)
{
    const long total = N * W;
    const long stride = (long)gridDim.x * kThreads;
    for (long t = (long)blockIdx.x * kThreads + threadIdx.x; t < total; t += stride) {
        long k, e;
        if (elem_major) {
            e = t / N;
            k = t - e * N;
        } else {
            k = t / W;
            e = t - k * W;
        }
        const long o = order[k];
        const long lib_index = elem_major ? e * N + k : k * W + e;
        const long caller_index = elem_major ? e * N + o : o * W + e;
        if (to_caller)
            dst[caller_index] = src[lib_index];
        else
            dst[lib_index] = src[caller_index];
    }
}

}  // namespace

using namespace bmpc;

extern "C" {

BMPC_API bmpc_status bmpc_tree_permute(bmpc_tree* tree, int32_t direction, int32_t layout,
                                       int32_t width, const double* src, double* dst, void* stream)
{
    if (!tree || !src || !dst) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    if (direction != BMPC_TO_LIBRARY_ORDER && direction != BMPC_TO_CALLER_ORDER)
        return fail(BMPC_ERR_INVALID_ARG, "direction must be BMPC_TO_LIBRARY_ORDER or BMPC_TO_CALLER_ORDER");
    if (layout != BMPC_LAYOUT_NODE_MAJOR && layout != BMPC_LAYOUT_ELEM_MAJOR)
        return fail(BMPC_ERR_INVALID_ARG, "layout must be BMPC_LAYOUT_NODE_MAJOR or BMPC_LAYOUT_ELEM_MAJOR");
    if (width <= 0) return fail(BMPC_ERR_INVALID_ARG, "width must be positive (got %d)", width);
    if ((const void*)src == (const void*)dst)
        return fail(BMPC_ERR_INVALID_ARG, "src and dst must be different arrays");
    const long N = tree->h.N;
    const long total = N * (long)width;
    hipStream_t s = (hipStream_t)stream;
    if (tree->order.empty()) {
        // the caller's order is the library's: a plain copy
        BMPC_HIP_TRY(hipMemcpyAsync(dst, src, sizeof(double) * total, hipMemcpyDeviceToDevice, s));
        return BMPC_OK;
    }
    if (!tree->d_order) {
        void* p = nullptr;
        if (hipMalloc(&p, sizeof(int32_t) * N) != hipSuccess)
            return fail(BMPC_ERR_OOM, "hipMalloc of %ld bytes failed", (long)(sizeof(int32_t) * N));
        tree->allocations.push_back(p);
        BMPC_HIP_TRY(hipMemcpy(p, tree->order.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice));
        tree->d_order = (const int32_t*)p;
    }
    const long blocks = std::min<long>((total + kThreads - 1) / kThreads, 8192);
    hipLaunchKernelGGL(k_permute_nodes, dim3((unsigned)blocks), dim3(kThreads), 0, s, tree->d_order, N,
                       (long)width, layout == BMPC_LAYOUT_ELEM_MAJOR, direction == BMPC_TO_CALLER_ORDER,
                       src, dst);
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

}  // extern "C"
