// Internal declarations of libbmpc (host and device).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bmpc.h"

namespace bmpc {

// ---------------------------------------------------------------- errors
bmpc_status fail(bmpc_status st, const char* fmt, ...);
void clear_error();

#define BMPC_HIP_TRY(expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::bmpc::fail(BMPC_ERR_HIP, "%s failed: %s (%s:%d)", #expr,          \
                                hipGetErrorString(e_), __FILE__, __LINE__);             \
    } while (0)

// ---------------------------------------------------------------- layout
// Index of element e (0 <= e < esize) of node i among N nodes.
template <int LAYOUT>
__host__ __device__ __forceinline__ long lidx(int i, int e, int esize, int N)
{
    if constexpr (LAYOUT == BMPC_LAYOUT_NODE_MAJOR)
        return (long)i * esize + e;
    else
        return (long)e * N + i;
}

// ---------------------------------------------------------------- tree
// Device view of a tree in stage-major breadth-first order.
struct TreeDev {
    int N;
    int num_leaves;
    int depth;            // largest stage
    const int* parent;    // N
    const int* child_off; // N+1: children of n are child_off[n] .. child_off[n+1]-1
    const int4* info;     // N: {first child, end of children, parent, number of children of the parent}
    const int* stage;     // N
    const int* level_off; // depth+2: nodes of stage t are level_off[t] .. level_off[t+1]-1
    const int* leaves;    // num_leaves, increasing node ids
    const int* leaf_stage;// num_leaves
    const int* path;      // (depth+1) x num_leaves: node at stage t on the path of leaf l
    const int* first_leaf;// N: smallest leaf index below n (the node's designated writer)
    const int* write_from;// num_leaves: path l writes the nodes of stages >= write_from[l]
    // segment scan structure
    int num_segments;
    const int* seg_start; // S: first (top) node of segment s
    const int* seg_end;   // S: last (bottom) node of segment s
    const int* seg_len;   // S
    const int* seg_of;    // N
    const int* seg_pos;   // N: position of the node inside its segment (0 = top)
    const int* seg_nodes; // N: nodes of all segments, segment by segment, top to bottom
    const int* seg_off;   // S+1: offsets into seg_nodes
    const int* seg_depth; // S: number of branching ancestors of the segment
    int max_seg_len;
    int max_seg_depth;
};

struct HostTree {
    std::vector<int> parent, child_off, stage, leaves, leaf_stage, path, first_leaf, write_from;
    std::vector<int4> info;
    std::vector<int> level_off;
    std::vector<int> seg_start, seg_end, seg_len, seg_of, seg_pos, seg_nodes, seg_off, seg_depth;
    int N = 0, depth = 0, max_seg_len = 0, max_seg_depth = 0;
};

}  // namespace bmpc

struct bmpc_tree {
    bmpc::HostTree h;
    bmpc::TreeDev d{};
    std::vector<void*> allocations;
    int device = 0;
    bool on_device = false;
    // trees made from a caller's own node order: order[k] = the caller's
    // index of library node k (empty = the caller's order is the library's);
    // d_order is its device copy, uploaded by the first permute call
    std::vector<int32_t> order;
    const int32_t* d_order = nullptr;
};

namespace bmpc {
// Upload the tree's index arrays to the current device (once).
bmpc_status tree_on_device(bmpc_tree* t);
}
