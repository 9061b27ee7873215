// Tree topology: validation, index sets (Sec. II-B: parent, children,
// stage sets, leaves), root-to-leaf paths and maximal unbranched segments,
// uploaded once to the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "bmpc_internal.hpp"

namespace bmpc {

static thread_local std::string g_err;

bmpc_status fail(bmpc_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err.clear(); }

static bmpc_status analyse(const int32_t* parent, int32_t N, HostTree& h)
{
    if (N <= 0) return fail(BMPC_ERR_INVALID_ARG, "num_nodes must be positive (got %d)", N);
    if (!parent) return fail(BMPC_ERR_INVALID_ARG, "parent is NULL");
    if (parent[0] != -1) return fail(BMPC_ERR_TOPOLOGY, "parent[0] must be -1");
    for (int i = 1; i < N; ++i) {
        if (parent[i] < 0 || parent[i] >= i)
            return fail(BMPC_ERR_TOPOLOGY, "node %d: parent %d must satisfy 0 <= parent < %d", i,
                        parent[i], i);
        if (i > 1 && parent[i] < parent[i - 1])
            return fail(BMPC_ERR_TOPOLOGY,
                        "node %d: parent[] must be non-decreasing (stage-major breadth-first order)",
                        i);
    }
    h.N = N;
    h.parent.assign(parent, parent + N);
    h.child_off.assign(N + 1, 0);
    for (int i = 1; i < N; ++i) h.child_off[parent[i] + 1]++;
    for (int i = 0; i < N; ++i) h.child_off[i + 1] += h.child_off[i];
    // with non-decreasing parents the children of n are a contiguous range
    // starting right after the nodes of earlier parents: child_off[n] + 1
    // is the first child id
    for (int i = 0; i < N; ++i) h.child_off[i] += 1;
    h.child_off[N] += 1;
    h.stage.assign(N, 0);
    for (int i = 1; i < N; ++i) h.stage[i] = h.stage[parent[i]] + 1;
    h.info.resize(N);
    for (int i = 0; i < N; ++i) {
        const int p = parent[i];
        h.info[i] = make_int4(h.child_off[i], h.child_off[i + 1], p,
                              p < 0 ? 0 : h.child_off[p + 1] - h.child_off[p]);
    }
    h.depth = *std::max_element(h.stage.begin(), h.stage.end());
    h.level_off.assign(h.depth + 2, 0);
    for (int i = 0; i < N; ++i) h.level_off[h.stage[i] + 1]++;
    for (int s = 0; s <= h.depth; ++s) h.level_off[s + 1] += h.level_off[s];
    h.leaves.clear();
    for (int i = 0; i < N; ++i)
        if (h.child_off[i] == h.child_off[i + 1]) h.leaves.push_back(i);
    const int Z = (int)h.leaves.size();
    h.leaf_stage.resize(Z);
    h.first_leaf.assign(N, INT_MAX);
    for (int l = 0; l < Z; ++l) {
        h.leaf_stage[l] = h.stage[h.leaves[l]];
        h.first_leaf[h.leaves[l]] = l;
    }
    for (int i = N - 1; i >= 1; --i)
        h.first_leaf[parent[i]] = std::min(h.first_leaf[parent[i]], h.first_leaf[i]);
    h.path.assign((size_t)(h.depth + 1) * Z, -1);
    for (int l = 0; l < Z; ++l)
        for (int n = h.leaves[l]; n >= 0; n = parent[n]) h.path[(size_t)h.stage[n] * Z + l] = n;
    // a path is the designated writer of a node exactly when it is the
    // smallest leaf below it; going up from the leaf, that holds for an
    // unbroken run of ancestors, so one stage per path describes it
    h.write_from.resize(Z);
    for (int l = 0; l < Z; ++l) {
        int n = h.leaves[l];
        while (parent[n] >= 0 && h.first_leaf[parent[n]] == l) n = parent[n];
        h.write_from[l] = h.stage[n];
    }

    // maximal unbranched segments: start at the root or at a child of a node
    // with >= 2 children; continue through single-child nodes
    h.seg_of.assign(N, -1);
    h.seg_pos.assign(N, 0);
    h.seg_start.clear();
    for (int i = 0; i < N; ++i) {
        const int p = parent[i];
        const int np = p < 0 ? 0 : h.child_off[p + 1] - h.child_off[p];
        if (p < 0 || np != 1) {
            h.seg_of[i] = (int)h.seg_start.size();
            h.seg_pos[i] = 0;
            h.seg_start.push_back(i);
        } else {
            h.seg_of[i] = h.seg_of[p];
            h.seg_pos[i] = h.seg_pos[p] + 1;
        }
    }
    const int S = (int)h.seg_start.size();
    h.seg_len.assign(S, 0);
    h.seg_end.assign(S, -1);
    for (int i = 0; i < N; ++i) {
        h.seg_len[h.seg_of[i]]++;
        h.seg_end[h.seg_of[i]] = i;  // deepest node seen last in BFS order
    }
    h.seg_off.assign(S + 1, 0);
    for (int s = 0; s < S; ++s) h.seg_off[s + 1] = h.seg_off[s] + h.seg_len[s];
    h.seg_nodes.assign(N, -1);
    for (int i = 0; i < N; ++i) h.seg_nodes[h.seg_off[h.seg_of[i]] + h.seg_pos[i]] = i;
    h.max_seg_len = *std::max_element(h.seg_len.begin(), h.seg_len.end());
    h.seg_depth.assign(S, 0);
    for (int s = 0; s < S; ++s) {
        const int p = parent[h.seg_start[s]];
        h.seg_depth[s] = p < 0 ? 0 : h.seg_depth[h.seg_of[p]] + 1;  // parent segments come first
    }
    h.max_seg_depth = *std::max_element(h.seg_depth.begin(), h.seg_depth.end());
    return BMPC_OK;
}

template <class T>
static bmpc_status upload(bmpc_tree* t, const std::vector<T>& v, const T** out)
{
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
    if (hipMalloc(&p, bytes) != hipSuccess)
        return fail(BMPC_ERR_OOM, "hipMalloc of %zu bytes failed", bytes);
    t->allocations.push_back(p);
    if (!v.empty()) BMPC_HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = (const T*)p;
    return BMPC_OK;
}

bmpc_status tree_on_device(bmpc_tree* t)
{
    if (t->on_device) return BMPC_OK;
    HostTree& h = t->h;
    TreeDev& d = t->d;
    BMPC_HIP_TRY(hipGetDevice(&t->device));
    d.N = h.N;
    d.num_leaves = (int)h.leaves.size();
    d.depth = h.depth;
    d.num_segments = (int)h.seg_start.size();
    d.max_seg_len = h.max_seg_len;
    d.max_seg_depth = h.max_seg_depth;
    bmpc_status st;
#define UP(field) \
    if ((st = upload(t, h.field, &d.field)) != BMPC_OK) return st;
    UP(parent) UP(child_off) UP(info) UP(stage) UP(level_off) UP(leaves) UP(leaf_stage) UP(path) UP(first_leaf) UP(write_from)
    UP(seg_start) UP(seg_end) UP(seg_len) UP(seg_of) UP(seg_pos) UP(seg_nodes) UP(seg_off) UP(seg_depth)
#undef UP
    t->on_device = true;
    return BMPC_OK;
}

// Breadth-first relabelling of a tree given in any node order: one root
// (parent -1), every other node with one parent in [0, N).  Children keep
// the order of their caller indices, so the result is the library's
// stage-major order with contiguous children.  Every node is some node's
// child exactly once, so a node that the walk from the root does not reach
// lies on a parent cycle.
static bmpc_status breadth_first_order(const int32_t* parent, int N, std::vector<int32_t>& order,
                                       std::vector<int32_t>& lib_parent)
{
    if (N <= 0) return fail(BMPC_ERR_INVALID_ARG, "num_nodes must be positive (got %d)", N);
    if (!parent) return fail(BMPC_ERR_INVALID_ARG, "parent is NULL");
    int root = -1;
    std::vector<int32_t> off(N + 1, 0);
    for (int i = 0; i < N; ++i) {
        const int p = parent[i];
        if (p == -1) {
            if (root >= 0)
                return fail(BMPC_ERR_TOPOLOGY, "nodes %d and %d both have parent -1", root, i);
            root = i;
        } else if (p < 0 || p >= N || p == i) {
            return fail(BMPC_ERR_TOPOLOGY, "node %d: parent %d is not a node index other than %d",
                        i, p, i);
        } else {
            off[p + 1]++;
        }
    }
    if (root < 0) return fail(BMPC_ERR_TOPOLOGY, "no node has parent -1");
    for (int i = 0; i < N; ++i) off[i + 1] += off[i];
    std::vector<int32_t> kids(N > 1 ? N - 1 : 1), fill(off.begin(), off.end() - 1);
    for (int i = 0; i < N; ++i)
        if (parent[i] >= 0) kids[fill[parent[i]]++] = i;
    order.assign(N, -1);
    std::vector<int32_t> lib_id(N, -1);
    order[0] = root;
    lib_id[root] = 0;
    int tail = 1;
    for (int head = 0; head < tail; ++head) {
        const int n = order[head];
        for (int c = off[n]; c < off[n + 1]; ++c) {
            lib_id[kids[c]] = tail;
            order[tail++] = kids[c];
        }
    }
    if (tail != N)
        return fail(BMPC_ERR_TOPOLOGY,
                    "only %d of %d nodes descend from the root: the parents form a cycle", tail, N);
    lib_parent.assign(N, -1);
    for (int k = 1; k < N; ++k) lib_parent[k] = lib_id[parent[order[k]]];
    return BMPC_OK;
}

}  // namespace bmpc

using namespace bmpc;

extern "C" {

BMPC_API const char* bmpc_last_error(void) { return g_err.c_str(); }

BMPC_API int32_t bmpc_version(void) { return 100; }

BMPC_API int32_t bmpc_device_count(void)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

BMPC_API bmpc_status bmpc_tree_create(const int32_t* parent, int32_t num_nodes, bmpc_tree** out)
{
    if (!out) return fail(BMPC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    auto* t = new bmpc_tree();
    bmpc_status st = analyse(parent, num_nodes, t->h);
    if (st != BMPC_OK) {
        delete t;
        return st;
    }
    *out = t;
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_tree_order(const int32_t* parent, int32_t num_nodes, int32_t* order,
                                     int32_t* lib_parent)
{
    if (!order) return fail(BMPC_ERR_INVALID_ARG, "order is NULL");
    std::vector<int32_t> ord, lp;
    bmpc_status st = breadth_first_order(parent, num_nodes, ord, lp);
    if (st != BMPC_OK) return st;
    std::memcpy(order, ord.data(), sizeof(int32_t) * num_nodes);
    if (lib_parent) std::memcpy(lib_parent, lp.data(), sizeof(int32_t) * num_nodes);
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_tree_create_any(const int32_t* parent, int32_t num_nodes, int32_t* order,
                                          bmpc_tree** out)
{
    if (!out) return fail(BMPC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::vector<int32_t> ord, lp;
    bmpc_status st = breadth_first_order(parent, num_nodes, ord, lp);
    if (st != BMPC_OK) return st;
    auto* t = new bmpc_tree();
    st = analyse(lp.data(), num_nodes, t->h);
    if (st != BMPC_OK) {
        delete t;
        return st;
    }
    bool identity = true;
    for (int k = 0; k < num_nodes; ++k) identity = identity && ord[k] == k;
    if (!identity) t->order = ord;
    if (order) std::memcpy(order, ord.data(), sizeof(int32_t) * num_nodes);
    *out = t;
    return BMPC_OK;
}

BMPC_API void bmpc_tree_destroy(bmpc_tree* t)
{
    if (!t) return;
    for (void* p : t->allocations) (void)hipFree(p);
    delete t;
}

BMPC_API bmpc_status bmpc_tree_info(const bmpc_tree* t, int32_t* num_nodes, int32_t* num_leaves,
                                    int32_t* depth, int32_t* num_segments)
{
    if (!t) return fail(BMPC_ERR_INVALID_ARG, "tree is NULL");
    if (num_nodes) *num_nodes = t->h.N;
    if (num_leaves) *num_leaves = (int32_t)t->h.leaves.size();
    if (depth) *depth = t->h.depth;
    if (num_segments) *num_segments = (int32_t)t->h.seg_start.size();
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_tree_segments(const bmpc_tree* t, int32_t* seg_of_node)
{
    if (!t || !seg_of_node) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    std::memcpy(seg_of_node, t->h.seg_of.data(), sizeof(int32_t) * t->h.N);
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_weights_from_probs(const bmpc_tree* t, const double* leaf_prob,
                                             double* node_weight)
{
    if (!t || !leaf_prob || !node_weight) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    const HostTree& h = t->h;
    for (int i = 0; i < h.N; ++i) node_weight[i] = 0.0;
    for (size_t l = 0; l < h.leaves.size(); ++l) {
        if (!(leaf_prob[l] >= 0.0))
            return fail(BMPC_ERR_INVALID_ARG, "leaf_prob[%zu] must be a non-negative number", l);
        node_weight[h.leaves[l]] = leaf_prob[l];
    }
    // children have larger ids than their parent: one reverse sweep sums subtrees
    for (int i = h.N - 1; i >= 1; --i) node_weight[h.parent[i]] += node_weight[i];
    return BMPC_OK;
}

}  // extern "C"
