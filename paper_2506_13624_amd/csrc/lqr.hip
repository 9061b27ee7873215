// Tree LQR on the GPU: backward tree Riccati, forward rollout, costates.
//
// Backward (Sec. III-A, eq. tree_Riccati with the gains of eq.
// tree_feedback_laws).  For node n with children j:
//   H = R_n + sum_j B_j^T P_j B_j,  G = M_n + sum_j B_j^T P_j A_j,
//   g = r_n + sum_j B_j^T (p_j + P_j c_j)
//   K_n = -H^-1 G,  k_n = -H^-1 g
//   P_n = sym(Q_n + sum_j A_j^T P_j A_j + G^T K_n),  p_n = q_n + sum_j A_j^T (p_j + P_j c_j) + G^T k_n
// Leaves: P = Q, p = q.
//
// Level-parallel schedule without grid barriers: every leaf segment is
// walked upwards by one worker (a lane for small nx, a wavefront with LDS
// staging for larger nx); all nodes of one depth are processed at the same
// time.  When a worker reaches a branching node it counts itself in with an
// atomic; the last child to arrive merges all children (always in child
// order, so results are bitwise reproducible) and carries on upwards, the
// others stop.  Inside a segment the next node's inputs are loaded while the
// current node is computed.
//
// Forward (Sec. III-B, last paragraph; eq. forward_comb_rule): a group of G
// lanes per root-to-leaf path (lane g owns row g) applies u = K x + k and
// x_j = A_j x + B_j u + c_j down the path, with the inputs of the next D
// steps in flight.  Every node is written by exactly one path (the first
// leaf below it).  The costates lam = P x + p are then computed for all
// nodes in parallel.
#include <hip/hip_runtime.h>

#include <cstring>

#include <algorithm>
#include <climits>
#include <initializer_list>
#include <type_traits>
#include <utility>

#include "bmpc_internal.hpp"
#include "cvf_device.hpp"
#include "lqr_device.hpp"
#include "profile.hpp"

namespace bmpc {

// ------------------------------------------------------------------------
// Hand-over of a finished child's value function to the worker that merges
// it at a branching node (possibly on another XCD).  The child's (P, p) are
// written and read with device-scope relaxed atomics, which go to the
// device-coherent level and bypass the per-XCD L2, and the writer waits for
// its own stores to complete before it counts itself in.  This avoids a
// device-scope release fence per worker, which would write back the whole
// L2 of the XCD.
// ------------------------------------------------------------------------
__device__ __forceinline__ void st_shared_dev(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_shared_dev(const double* p)
{
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_shared_dev(float* p, float v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_shared_dev(const float* p)
{
    return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// all earlier memory operations of this lane have completed
__device__ __forceinline__ void wait_own_stores()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <int NX, int LAY, class T>
__device__ __forceinline__ void store_value_dev(const LqrArgsT<T>& a, int N, int n, const T (&P)[NX][NX],
                                                const T (&p)[NX])
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j) st_shared_dev(&a.P[lidx<LAY>(n, i * NX + j, NX * NX, N)], P[i][j]);
        st_shared_dev(&a.p[lidx<LAY>(n, i, NX, N)], p[i]);
    }
}

template <int NX, int LAY, class T>
__device__ __forceinline__ void load_value_dev(const LqrArgsT<T>& a, int N, int j, T (&P)[NX][NX],
                                               T (&p)[NX])
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int k = 0; k < NX; ++k) P[i][k] = ld_shared_dev(&a.P[lidx<LAY>(j, i * NX + k, NX * NX, N)]);
        p[i] = ld_shared_dev(&a.p[lidx<LAY>(j, i, NX, N)]);
    }
}

// ------------------------------------------------------------------------
// lane-per-segment backward
// ------------------------------------------------------------------------
template <int NX, int NU, int LAY, class T = double>
__global__ void __launch_bounds__(64) k_bwd_lane(TreeDev t, LqrArgsT<T> a, int* arrive)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= t.num_leaves) return;
    const int N = t.N;
    int n = t.leaves[l];
    int4 inf = t.info[n];
    int from = -1;
    bool pref = false;  // stage/edge hold the inputs of n (single child == from)
    T P[NX][NX], p[NX];
    StageRegs<NX, NU, T> stage;
    EdgeRegs<NX, NU, T> edge;
    for (;;) {
        const int c0 = inf.x, c1 = inf.y, par = inf.z, nsib = inf.w;
        // the next node's topology record, in flight while this node is computed
        const int4 inf_next = par >= 0 ? t.info[par] : make_int4(0, 0, -1, 0);
        if (c0 == c1) {
            load_value<NX, LAY>(a.Q, a.q, N, n, P, p);
#pragma unroll
            for (int e = 0; e < NU * NX; ++e) a.K[lidx<LAY>(n, e, NU * NX, N)] = T(0);
#pragma unroll
            for (int e = 0; e < NU; ++e) a.k[lidx<LAY>(n, e, NU, N)] = T(0);
            if (nsib == 1) {
                load_stage<NX, NU, LAY>(a, N, par, stage);
                load_edge<NX, NU, LAY, false>(a, N, par, n, edge);
            }
        } else {
            RicAcc<NX, NU, T> acc;
            if (pref) {
                acc.init(stage);
                const EdgeRegs<NX, NU, T> e0 = edge;
                // inputs of the parent are independent of this step: start them now
                if (nsib == 1) {
                    load_stage<NX, NU, LAY>(a, N, par, stage);
                    load_edge<NX, NU, LAY, false>(a, N, par, n, edge);
                }
                acc.add_child(e0, P, p);
            } else {
                load_stage<NX, NU, LAY>(a, N, n, stage);
                acc.init(stage);
                for (int j = c0; j < c1; ++j) {
                    load_edge<NX, NU, LAY, false>(a, N, n, j, edge);
                    if (!(c1 - c0 == 1 && from == j)) load_value_dev<NX, LAY>(a, N, j, P, p);
                    acc.add_child(edge, P, p);
                }
                if (nsib == 1) {
                    load_stage<NX, NU, LAY>(a, N, par, stage);
                    load_edge<NX, NU, LAY, false>(a, N, par, n, edge);
                }
            }
            T Kn[NU][NX], kn[NU];
            if (!acc.finish(Kn, kn, P, p)) atomicMin(a.bad, n);
#pragma unroll
            for (int i = 0; i < NU; ++i) {
#pragma unroll
                for (int b = 0; b < NX; ++b) a.K[lidx<LAY>(n, i * NX + b, NU * NX, N)] = Kn[i][b];
                a.k[lidx<LAY>(n, i, NU, N)] = kn[i];
            }
        }
        if (nsib > 1)
            store_value_dev<NX, LAY>(a, N, n, P, p);
        else
            store_value<NX, LAY>(a, N, n, P, p);
        if (par < 0) break;
        pref = nsib == 1;
        if (nsib > 1) {
            wait_own_stores();
            const int old = atomicAdd(&arrive[par], 1);
            if (old != nsib - 1) break;
        }
        from = n;
        n = par;
        inf = inf_next;
    }
}

// ------------------------------------------------------------------------
// nx = 4, nu = 2: a group of 16 lanes per leaf chain
// ------------------------------------------------------------------------
// Same walk and merges as k_bwd_lane, but the work of a step is spread over
// the 16 lanes of a DPP row: lane q = 4 i + j holds entry (i, j) of P and
// of the step's 4 x 4 products, entry (a, j) of G for both rows a, and
// entry (a, j % 2) of H.  Row i of P comes from the lane's quad (quad_perm
// broadcasts); the column of S = P [A B] and the vector s = P c + p that
// the second products need come from the lanes at distance 4, 8 and 12 in
// the row (row rotations), so every lane reads only the entries of A, B it
// multiplies.  H, g and the gains are small and formed by every lane.

// lane K of this lane's quad
template <int K, class T>
__device__ __forceinline__ T quad_bcast(T v)
{
    return __builtin_amdgcn_update_dpp(T(0), v, K | (K << 2) | (K << 4) | (K << 6), 0xf, 0xf, false);
}
// the other lane of this lane's pair in the quad (lane ^ 1)
template <class T>
__device__ __forceinline__ T quad_swap1(T v)
{
    return __builtin_amdgcn_update_dpp(T(0), v, 0xB1, 0xf, 0xf, false);
}
// lane J of this lane's row of 16
template <int J, class T>
__device__ __forceinline__ T row_lane(T v)
{
    return __builtin_amdgcn_update_dpp(T(0), v, 0x150 + J, 0xf, 0xf, false);
}
// rotation by R lanes within the row of 16
template <int R, class T>
__device__ __forceinline__ T row_rot(T v)
{
    return __builtin_amdgcn_update_dpp(T(0), v, 0x120 + R, 0xf, 0xf, false);
}
template <int R>
__device__ __forceinline__ int row_rot_int(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x120 + R, 0xf, 0xf, false);
}

template <class T>
struct QuadEdge {
    T Acol[4], Bcol[4], c[4];  // A[k][j], B[k][j % 2], c[k]
    T Arot[4], Brot[2][4];     // A[r_d][i], B[r_d][a]: r_d the row held by the lane rotated in by 4 d
};
template <class T>
struct QuadStage {
    T Q, M[2], R[2], r[2], q;  // Q[i][j], M[a][j], R[a][j % 2], r[a], q[i]
};
template <class T>
struct QuadAcc {
    T W, w, G[2], H[2], g[2];  // W[i][j], w[i], G[a][j], H[a][j % 2], g[a]
};

template <int LAY, class T = double>
__global__ void __launch_bounds__(64) k_bwd_quad(TreeDev t, LqrArgsT<T> a, int* arrive)
{
    constexpr int NX = 4, NU = 2;
    const int tid = blockIdx.x * 64 + threadIdx.x;
    const int chain = tid >> 4;
    if (chain >= t.num_leaves) return;  // the whole group leaves together
    const int q = tid & 15, i = q >> 2, j = q & 3, jb = j & 1;
    const int N = t.N;
    // row of the matrices held by the lane that a rotation by 4 d brings in
    // (d = 0: this lane), found with the same rotation that moves the values
    int rrow[4];
    rrow[0] = i;
    rrow[1] = row_rot_int<12>(i);
    rrow[2] = row_rot_int<8>(i);
    rrow[3] = row_rot_int<4>(i);

    auto load_edge_q = [&](int ch, QuadEdge<T>& e) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            e.Acol[k] = a.A[lidx<LAY>(ch, k * NX + j, NX * NX, N)];
            e.Bcol[k] = a.B[lidx<LAY>(ch, k * NU + jb, NX * NU, N)];
            e.c[k] = a.c[lidx<LAY>(ch, k, NX, N)];
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            e.Arot[d] = a.A[lidx<LAY>(ch, rrow[d] * NX + i, NX * NX, N)];
#pragma unroll
            for (int b = 0; b < NU; ++b) e.Brot[b][d] = a.B[lidx<LAY>(ch, rrow[d] * NU + b, NX * NU, N)];
        }
    };
    auto load_stage_q = [&](int m, QuadStage<T>& st) {
        st.Q = a.Q[lidx<LAY>(m, i * NX + j, NX * NX, N)];
        st.q = a.q[lidx<LAY>(m, i, NX, N)];
#pragma unroll
        for (int b = 0; b < NU; ++b) {
            st.M[b] = a.M[lidx<LAY>(m, b * NX + j, NU * NX, N)];
            st.R[b] = a.R[lidx<LAY>(m, b * NU + jb, NU * NU, N)];
            st.r[b] = a.r[lidx<LAY>(m, b, NU, N)];
        }
    };
    auto acc_init = [&](const QuadStage<T>& st, QuadAcc<T>& z) {
        z.W = st.Q;
        z.w = st.q;
#pragma unroll
        for (int b = 0; b < NU; ++b) {
            z.G[b] = st.M[b];
            z.H[b] = st.R[b];
            z.g[b] = st.r[b];
        }
    };
    // the child's value function (entry Pv of P, entry pv of p) through edge e
    auto acc_add = [&](const QuadEdge<T>& e, T Pv, T pv, QuadAcc<T>& z) {
        T prow[4];
        prow[0] = quad_bcast<0>(Pv);
        prow[1] = quad_bcast<1>(Pv);
        prow[2] = quad_bcast<2>(Pv);
        prow[3] = quad_bcast<3>(Pv);
        T SA = T(0), SB = T(0), sv = pv;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            SA = fma(prow[k], e.Acol[k], SA);
            SB = fma(prow[k], e.Bcol[k], SB);
            sv = fma(prow[k], e.c[k], sv);
        }
        T rSA[4], rSB[4], rs[4];
        rSA[0] = SA;
        rSB[0] = SB;
        rs[0] = sv;
        rSA[1] = row_rot<12>(SA);
        rSB[1] = row_rot<12>(SB);
        rs[1] = row_rot<12>(sv);
        rSA[2] = row_rot<8>(SA);
        rSB[2] = row_rot<8>(SB);
        rs[2] = row_rot<8>(sv);
        rSA[3] = row_rot<4>(SA);
        rSB[3] = row_rot<4>(SB);
        rs[3] = row_rot<4>(sv);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            z.W = fma(e.Arot[d], rSA[d], z.W);
            z.w = fma(e.Arot[d], rs[d], z.w);
#pragma unroll
            for (int b = 0; b < NU; ++b) {
                z.G[b] = fma(e.Brot[b][d], rSA[d], z.G[b]);
                z.H[b] = fma(e.Brot[b][d], rSB[d], z.H[b]);
                z.g[b] = fma(e.Brot[b][d], rs[d], z.g[b]);
            }
        }
    };
    T Pv, pv;  // this lane's entries of the current value function
    // gains and value function of node m from the accumulated z
    auto finish = [&](const QuadAcc<T>& z, int m) {
        const T ho0 = quad_swap1(z.H[0]), ho1 = quad_swap1(z.H[1]);
        T L[2][2], inv[2];
        L[0][0] = jb == 0 ? z.H[0] : ho0;
        L[0][1] = jb == 1 ? z.H[0] : ho0;
        L[1][0] = jb == 0 ? z.H[1] : ho1;
        L[1][1] = jb == 1 ? z.H[1] : ho1;
        bool ok;
        if constexpr (std::is_same<T, double>::value)
            ok = chol_inplace_rsq<2>(L, inv);
        else
            ok = chol_inplace<2, T>(L, inv);
        if (!ok && q == 0) atomicMin(a.bad, m);
        T Kj[2] = {z.G[0], z.G[1]}, kv[2] = {z.g[0], z.g[1]};
        chol_solve<2>(L, inv, Kj);
        chol_solve<2>(L, inv, kv);
#pragma unroll
        for (int b = 0; b < NU; ++b) {
            Kj[b] = -Kj[b];
            kv[b] = -kv[b];
        }
        // G[a][i]: entry i of row a, held by lane i of the row
        T Gi[2];
#pragma unroll
        for (int b = 0; b < NU; ++b) {
            const T g0 = row_lane<0>(z.G[b]), g1 = row_lane<1>(z.G[b]);
            const T g2 = row_lane<2>(z.G[b]), g3 = row_lane<3>(z.G[b]);
            Gi[b] = i == 0 ? g0 : (i == 1 ? g1 : (i == 2 ? g2 : g3));
        }
        T X = z.W, pn = z.w;
#pragma unroll
        for (int b = 0; b < NU; ++b) {
            X = fma(Gi[b], Kj[b], X);
            pn = fma(Gi[b], kv[b], pn);
        }
        // (X is symmetric up to rounding; it is kept as it is rather than
        // averaged with the transposed lane's entry, an LDS permute on the
        // walk's path)
        Pv = X;
        pv = pn;
        if (i < NU) a.K[lidx<LAY>(m, i * NX + j, NU * NX, N)] = i == 0 ? Kj[0] : Kj[1];
        if (q < NU) a.k[lidx<LAY>(m, q, NU, N)] = q == 0 ? kv[0] : kv[1];
    };
    auto store_value_q = [&](int m, bool shared) {
        T* pP = &a.P[lidx<LAY>(m, i * NX + j, NX * NX, N)];
        T* pp = &a.p[lidx<LAY>(m, i, NX, N)];
        if (shared) {
            st_shared_dev(pP, Pv);
            if (j == 0) st_shared_dev(pp, pv);
        } else {
            *pP = Pv;
            if (j == 0) *pp = pv;
        }
    };

    int n = t.leaves[chain];
    int4 inf = t.info[n];
    int from = -1;
    bool pref = false;  // stage / edge hold the inputs of n (its single child is from)
    bool pre2 = false;  // mst / me0 / me1 hold the inputs of n (two children, one is from)
    QuadStage<T> stage, mst;
    QuadEdge<T> edge, me0, me1;
    for (;;) {
        const int c0 = inf.x, c1 = inf.y, par = inf.z, nsib = inf.w;
        // the next node's topology record, in flight while this node is computed
        const int4 inf_next = par >= 0 ? t.info[par] : make_int4(0, 0, -1, 0);
        if (c0 == c1) {
            Pv = a.Q[lidx<LAY>(n, i * NX + j, NX * NX, N)];
            pv = a.q[lidx<LAY>(n, i, NX, N)];
            if (i < NU) a.K[lidx<LAY>(n, i * NX + j, NU * NX, N)] = T(0);
            if (q < NU) a.k[lidx<LAY>(n, q, NU, N)] = T(0);
            if (nsib == 1) {
                load_stage_q(par, stage);
                load_edge_q(n, edge);
            }
        } else {
            QuadAcc<T> z;
            if (pref) {
                acc_init(stage, z);
                const QuadEdge<T> e0 = edge;
                // inputs of the parent are independent of this step: start them now
                if (nsib == 1) {
                    load_stage_q(par, stage);
                    load_edge_q(n, edge);
                }
                acc_add(e0, Pv, pv, z);
            } else if (pre2) {
                // two children: the stage and both edges were requested with
                // the count; the sibling's value function is read now, this
                // group's own is in registers; sums in child order
                acc_init(mst, z);
                const bool own0 = from == c0;
                T P0 = Pv, p0 = pv, P1 = Pv, p1 = pv;
                if (own0) {
                    P1 = ld_shared_dev(&a.P[lidx<LAY>(c0 + 1, i * NX + j, NX * NX, N)]);
                    p1 = ld_shared_dev(&a.p[lidx<LAY>(c0 + 1, i, NX, N)]);
                } else {
                    P0 = ld_shared_dev(&a.P[lidx<LAY>(c0, i * NX + j, NX * NX, N)]);
                    p0 = ld_shared_dev(&a.p[lidx<LAY>(c0, i, NX, N)]);
                }
                if (nsib == 1) {
                    load_stage_q(par, stage);
                    load_edge_q(n, edge);
                }
                acc_add(me0, P0, p0, z);
                acc_add(me1, P1, p1, z);
            } else {
                QuadStage<T> st;
                load_stage_q(n, st);
                acc_init(st, z);
                for (int ch = c0; ch < c1; ++ch) {
                    QuadEdge<T> e;
                    load_edge_q(ch, e);
                    T Pc = Pv, pc = pv;
                    if (!(c1 - c0 == 1 && from == ch)) {
                        Pc = ld_shared_dev(&a.P[lidx<LAY>(ch, i * NX + j, NX * NX, N)]);
                        pc = ld_shared_dev(&a.p[lidx<LAY>(ch, i, NX, N)]);
                    }
                    acc_add(e, Pc, pc, z);
                }
                if (nsib == 1) {
                    load_stage_q(par, stage);
                    load_edge_q(n, edge);
                }
            }
            finish(z, n);
        }
        store_value_q(n, nsib > 1);
        if (par < 0) break;
        pref = nsib == 1;
        pre2 = nsib == 2;
        if (nsib > 1) {
            // hand the value function over: all of the group's stores
            // complete before its one count
            wait_own_stores();
            // with one sibling, the parent's stage and both edges are
            // requested with the count, for the case that this group
            // arrives last
            if (pre2) {
                load_stage_q(par, mst);
                load_edge_q(inf_next.x, me0);
                load_edge_q(inf_next.x + 1, me1);
            }
            int old = 0;
            if (q == 0) old = atomicAdd(&arrive[par], 1);
            old = __shfl(old, (int)(threadIdx.x & 48), 64);
            if (old != nsib - 1) break;
        }
        from = n;
        n = par;
        inf = inf_next;
    }
}

// ------------------------------------------------------------------------
// log-depth backward: segment scan of conditional value functions
// ------------------------------------------------------------------------
// One wavefront per maximal unbranched segment, with the same dataflow over
// segments as the level-parallel kernels (the last child segment to reach a
// branching node merges its children and carries on with the segment that
// ends there).  Inside a segment the single-child nodes become conditional
// value functions (Sec. II-A, eqs. sol_min and comb_rule with the corrected
// signs), one per lane; a Hillis-Steele suffix scan composes every node's
// element with all elements below it in log2(length) rounds, and applying
// the value function of the segment's end node then gives every node's
// (P, p) at once (eq. V_ki_min).  Gains K, k follow from one Riccati step
// on the child's value (eq. tree_feedback_laws).  The single-child nodes
// of a segment are done in chunks of ch <= 64 from the bottom; ch is the
// tree's longest such run (at most 64), and the LDS of a workgroup is two
// scan buffers of ch elements (the chunk's value functions go to the one not
// holding the scan's result), so short segments leave room for more
// segments per compute unit.
template <int NX>
struct ValueLds {
    double P[NX][NX], p[NX];
};

// Two wavefronts per SIMD (the compiler keeps a lane within 256 registers,
// spilling a few hundred bytes): with the LDS sized to the chunk, a compute
// unit then holds up to eight segments.
template <int NX, int NU, int LAY>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_bwd_seg(TreeDev t, LqrArgs a, int* arrive, int ch)
{
    static_assert(sizeof(ValueLds<NX>) <= sizeof(Cvf<NX>), "a chunk's values fit in a scan buffer");
    extern __shared__ __align__(16) unsigned char seg_lds[];
    // element i of scan buffer b (indexed off the LDS symbol itself, so that
    // every access stays an LDS access)
    auto sbuf = [&](int b, int i) -> Cvf<NX>& { return reinterpret_cast<Cvf<NX>*>(seg_lds)[b * ch + i]; };
    __shared__ ValueLds<NX> send;
    __shared__ int sgo;
    const int lane = threadIdx.x;
    const int N = t.N;
    int s = t.seg_of[t.leaves[blockIdx.x]];
    for (;;) {
        const int off = t.seg_off[s], len = t.seg_len[s];
        const int e = t.seg_nodes[off + len - 1];
        // value function of the segment's bottom node: terminal cost at a
        // leaf, the exact merge of all children at a branching node
        if (lane == 0) {
            const int4 inf = t.info[e];
            double P[NX][NX], p[NX];
            if (inf.x == inf.y) {
                load_value<NX, LAY>(a.Q, a.q, N, e, P, p);
#pragma unroll
                for (int i = 0; i < NU * NX; ++i) a.K[lidx<LAY>(e, i, NU * NX, N)] = 0.0;
#pragma unroll
                for (int i = 0; i < NU; ++i) a.k[lidx<LAY>(e, i, NU, N)] = 0.0;
            } else {
                StageRegs<NX, NU> st;
                load_stage<NX, NU, LAY>(a, N, e, st);
                RicAcc<NX, NU> acc;
                acc.init(st);
                for (int j = inf.x; j < inf.y; ++j) {
                    EdgeRegs<NX, NU> ed;
                    load_edge<NX, NU, LAY, false>(a, N, e, j, ed);
                    double Pj[NX][NX], pj[NX];
                    load_value_dev<NX, LAY>(a, N, j, Pj, pj);
                    acc.add_child(ed, Pj, pj);
                }
                double Kn[NU][NX], kn[NU];
                if (!acc.finish(Kn, kn, P, p)) atomicMin(a.bad, e);
#pragma unroll
                for (int i = 0; i < NU; ++i) {
#pragma unroll
                    for (int b = 0; b < NX; ++b) a.K[lidx<LAY>(e, i * NX + b, NU * NX, N)] = Kn[i][b];
                    a.k[lidx<LAY>(e, i, NU, N)] = kn[i];
                }
            }
            if (len == 1 && inf.z >= 0)
                store_value_dev<NX, LAY>(a, N, e, P, p);
            else
                store_value<NX, LAY>(a, N, e, P, p);
#pragma unroll
            for (int i = 0; i < NX; ++i) {
#pragma unroll
                for (int j = 0; j < NX; ++j) send.P[i][j] = P[i][j];
                send.p[i] = p[i];
            }
        }
        __syncthreads();
        // single-child nodes at positions [0, len-1), bottom chunk first
        for (int hi = len - 1; hi > 0;) {
            const int lo = hi > ch ? hi - ch : 0;
            const int cnt = hi - lo;
            const int pos = lo + lane;
            const bool act = lane < cnt;
            const int n = act ? t.seg_nodes[off + pos] : 0;
            const int j = act ? t.seg_nodes[off + pos + 1] : 0;
            StageRegs<NX, NU> st;
            EdgeRegs<NX, NU> ed;
            if (act) {
                load_stage<NX, NU, LAY>(a, N, n, st);
                load_edge<NX, NU, LAY, false>(a, N, n, j, ed);
                if (!cvf_element<NX, NU>(st.Q, st.R, st.M, st.q, st.r, ed.A, ed.B, ed.c, sbuf(0, lane)))
                    atomicMin(a.bad, n);
            }
            __syncthreads();
            int cur = 0;
            for (int span = 1; span < cnt; span <<= 1) {
                if (act) {
                    if (lane + span < cnt)
                        cvf_combine<NX>(sbuf(cur, lane), sbuf(cur, lane + span), sbuf(cur ^ 1, lane));
                    else
                        sbuf(cur ^ 1, lane) = sbuf(cur, lane);
                }
                __syncthreads();
                cur ^= 1;
            }
            ValueLds<NX>* const sval = reinterpret_cast<ValueLds<NX>*>(&sbuf(cur ^ 1, 0));
            double P[NX][NX], p[NX];
            if (act) {
                cvf_apply_value<NX>(sbuf(cur, lane), send.P, send.p, P, p);
#pragma unroll
                for (int i = 0; i < NX; ++i) {
#pragma unroll
                    for (int k = 0; k < NX; ++k) sval[lane].P[i][k] = P[i][k];
                    sval[lane].p[i] = p[i];
                }
            }
            __syncthreads();
            if (act) {
                const ValueLds<NX>& cv = lane + 1 < cnt ? sval[lane + 1] : send;
                double Pc[NX][NX], pc[NX];
#pragma unroll
                for (int i = 0; i < NX; ++i) {
#pragma unroll
                    for (int k = 0; k < NX; ++k) Pc[i][k] = cv.P[i][k];
                    pc[i] = cv.p[i];
                }
                RicAcc<NX, NU> acc;
                acc.init(st);
                acc.add_child(ed, Pc, pc);
                double Kn[NU][NX], kn[NU], P1[NX][NX], p1[NX];
                if (!acc.finish(Kn, kn, P1, p1)) atomicMin(a.bad, n);
#pragma unroll
                for (int i = 0; i < NU; ++i) {
#pragma unroll
                    for (int b = 0; b < NX; ++b) a.K[lidx<LAY>(n, i * NX + b, NU * NX, N)] = Kn[i][b];
                    a.k[lidx<LAY>(n, i, NU, N)] = kn[i];
                }
                if (pos == 0 && t.info[n].z >= 0)
                    store_value_dev<NX, LAY>(a, N, n, P, p);
                else
                    store_value<NX, LAY>(a, N, n, P, p);
            }
            __syncthreads();
            if (lane == 0) send = sval[0];
            __syncthreads();
            hi = lo;
        }
        // count in at the branching node above the segment
        const int top = t.seg_nodes[off];
        const int4 tinf = t.info[top];
        const int par = tinf.z;
        if (par < 0) break;
        if (lane == 0) {
            wait_own_stores();
            const int old = atomicAdd(&arrive[par], 1);
            sgo = old == tinf.w - 1;
        }
        __syncthreads();
        if (!sgo) break;
        s = t.seg_of[par];
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// wavefront-per-segment backward (LDS staging; used for larger nx)
// ------------------------------------------------------------------------

// f(e) for the CNT elements of a node over the 64 lanes, without branches:
// lanes past the end repeat the last element (f must write the same value
// for the same element).
template <int CNT, class F>
__device__ __forceinline__ void each_elem(int lane, F f)
{
#pragma unroll
    for (int s = 0; s < (CNT + 63) / 64; ++s) {
        const int e = lane + 64 * s;
        f(e < CNT ? e : CNT - 1);
    }
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Single-wavefront workgroups: LDS accesses of one wavefront complete in
// issue order, so ordering them only needs a compiler-level fence.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------------
// Register-resident matrix-core backward pass (nx = 12, nu = 4): one
// wavefront per leaf chain, the value function P kept in the accumulator
// registers of v_mfma_f64_16x16x4 from one step to the next.
//
// Lane l (li = l % 16, lk = l / 16) holds element v of a 16 x 16 matrix
// tile as entry (lk + 4 v, li).  For a symmetric P that is also entry
// (li, lk + 4 v), which is exactly the A operand of k-block v of the product
// P [A B c]: so P needs no trip through LDS between steps.  The edge data
// [A B c] are read from memory straight into the operand layout (entry
// (4 m + lk, li) for k-block m), the stage data straight into the
// accumulator layout of Z = [[Q M^T q],[M R r]], two steps ahead along the
// leaf's root path.  Per child:
//   S = P [A B] (+ P c + p in column 0 of a second accumulator)
//   Z += [A B]^T S
// Only rows NX.. of Z ([G H g]) go through LDS, for the gains.
// ------------------------------------------------------------------------
struct WregIn {
    double d[3];   // [A B] of the edge, entry (4 m + lk, li), m < 3
    double cb[3];  // c of the edge, entry 4 m + lk (used in lanes li == 0)
    double z[4];   // stage data [[Q M^T],[M R]], entry (lk + 4 v, li)
    double zc[4];  // [q; r], entry lk + 4 v (used in lanes li == 0)
};

template <int NX, int NU, int LAY>
__global__ void __launch_bounds__(64) k_bwd_wreg(TreeDev t, LqrArgs a, int* arrive)
{
    static_assert(NX == 12 && NU == 4, "three k-blocks of P and one 16 x 16 tile of [A B]");
    constexpr int NZ = NX + NU;
    __shared__ double sH[NU][NZ + 1];   // rows NX.. of Z: [G H g]
    __shared__ int sgo;
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int l = blockIdx.x, NL = t.num_leaves, N = t.N;
    int s = t.leaf_stage[l];
    int n = t.leaves[l];
    // The walk's topology, 64 stages at a time, one stage per lane: lane i
    // holds the node at stage base - i of this leaf's root path, its first
    // child and its number of children.  A step reads them with readlane
    // (no memory latency on the path of the walk).
    int base = s, pathv = -1, c0v = 0, cntv = 0;
    auto reload = [&](int st) {
        base = st;
        const int sl = st - lane;
        pathv = sl >= 0 ? t.path[(long)sl * NL + l] : -1;
        c0v = pathv >= 0 ? t.child_off[pathv] : 0;
        cntv = pathv >= 0 ? t.child_off[pathv + 1] - c0v : 0;
        // used here, so that the loads are waited for inside this (rare)
        // branch: a load that might still be in flight where a step reads
        // the values would make the compiler wait for every load in flight
        // there, the prefetched inputs included
        asm volatile("" : "+v"(pathv), "+v"(c0v), "+v"(cntv));
    };
    reload(s);
    // stages base .. base - 63 are held; a step reads stages s .. s - 3
    auto lane_of = [&](int st) -> int { return base - st; };
    auto node_at = [&](int st) -> int { return st >= 0 ? __builtin_amdgcn_readlane(pathv, lane_of(st)) : -1; };

    // Per-lane addresses of node 0's entries and the distance from one node
    // to the next, computed once: the edge into child j, operand layout (an
    // entry of A or of B, picked per lane), and the stage data of a node,
    // accumulator layout (rows lk + 4 v < NX for v < 3).  A load is then one
    // multiply-add of the node id.
    constexpr bool NM = LAY == BMPC_LAYOUT_NODE_MAJOR;
    auto at = [&](const double* arr, int e) -> const double* { return NM ? arr + e : arr + (long)e * N; };
    auto stride = [](int esize) -> int { return NM ? esize : 1; };
    const double* pd0[3];
    const double* pc0[3];
    const double* pz0[4];
    const double* pq0[4];
    const int sd = li < NX ? stride(NX * NX) : stride(NX * NU);
    const int sz0 = li < NX ? stride(NX * NX) : stride(NU * NX);
    const int sz3 = li < NX ? stride(NU * NX) : stride(NU * NU);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int k = 4 * m + lk;
        pd0[m] = li < NX ? at(a.A, k * NX + li) : at(a.B, k * NU + (li - NX));
        pc0[m] = at(a.c, k);
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const int r = lk + 4 * v;
        pz0[v] = li < NX ? at(a.Q, r * NX + li) : at(a.M, (li - NX) * NX + r);
        pq0[v] = at(a.q, r);
    }
    pz0[3] = li < NX ? at(a.M, lk * NX + li) : at(a.R, lk * NU + (li - NX));
    pq0[3] = at(a.r, lk);
    // and of the outputs: this lane's entries of P and p (accumulator
    // layout) and its column of K (or k)
    auto atw = [&](double* arr, int e) -> double* { return NM ? arr + e : arr + (long)e * N; };
    double* pP0[3];
    double* pp0[3];
    double* pK0[NU];
    const int sK = li < NX ? stride(NU * NX) : stride(NU);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        pP0[v] = atw(a.P, (lk + 4 * v) * NX + (li < NX ? li : 0));
        pp0[v] = atw(a.p, lk + 4 * v);
    }
#pragma unroll
    for (int i = 0; i < NU; ++i) pK0[i] = li < NX ? atw(a.K, i * NX + li) : atw(a.k, i);
    auto load_edge = [&](int j, WregIn& in) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            in.d[m] = pd0[m][(long)j * sd];
            in.cb[m] = pc0[m][(long)j * stride(NX)];
        }
    };
    auto load_stage = [&](int m, WregIn& in) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            in.z[v] = pz0[v][(long)m * (v < 3 ? sz0 : sz3)];
            in.zc[v] = pq0[v][(long)m * (v < 3 ? stride(NX) : stride(NU))];
        }
    };
    // the child's contribution D^T (P D + [0 0 p]) added to (zm, zc)
    auto add_child = [&](const f64x4& Pr, const double (&pv)[4], const WregIn& e, f64x4& zm, f64x4& zc) {
        f64x4 sm = {0.0, 0.0, 0.0, 0.0}, sc;
#pragma unroll
        for (int v = 0; v < 4; ++v) sc[v] = (li == 0 && v < 3) ? pv[v] : 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const double cbm = li == 0 ? e.cb[m] : 0.0;
            sm = __builtin_amdgcn_mfma_f64_16x16x4f64(Pr[m], e.d[m], sm, 0, 0, 0);
            sc = __builtin_amdgcn_mfma_f64_16x16x4f64(Pr[m], cbm, sc, 0, 0, 0);
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            zm = __builtin_amdgcn_mfma_f64_16x16x4f64(e.d[m], sm[m], zm, 0, 0, 0);
            zc = __builtin_amdgcn_mfma_f64_16x16x4f64(e.d[m], sc[m], zc, 0, 0, 0);
        }
    };
    // value function of child j (another walker's), accumulator layout
    auto load_value_dev = [&](int j, f64x4& Pr, double (&pv)[4]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = lk + 4 * v;
            Pr[v] = (v < 3 && li < NX) ? ld_shared_dev(&a.P[lidx<LAY>(j, r * NX + li, NX * NX, N)]) : 0.0;
            pv[v] = v < 3 ? ld_shared_dev(&a.p[lidx<LAY>(j, r, NX, N)]) : 0.0;
        }
    };
    auto store_value = [&](int m, const f64x4& Pr, const double (&pv)[4], bool shared) {
        const long oP = (long)m * stride(NX * NX), op = (long)m * stride(NX);
        if (shared) {
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                if (li < NX) st_shared_dev(pP0[v] + oP, Pr[v]);
                if (li == 0) st_shared_dev(pp0[v] + op, pv[v]);
            }
        } else {
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                if (li < NX) pP0[v][oP] = Pr[v];
                if (li == 0) pp0[v][op] = pv[v];
            }
        }
    };

    // the leaf: P = Q_f, p = q_f, no gains
    f64x4 Preg;
    double pvec[4];
    // number of children of the parent (1 for the root, which has none)
    auto nsib_of = [&](int st) -> int { return st > 0 ? __builtin_amdgcn_readlane(cntv, lane_of(st - 1)) : 1; };
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = lk + 4 * v;
        Preg[v] = (v < 3 && li < NX) ? a.Q[lidx<LAY>(n, r * NX + li, NX * NX, N)] : 0.0;
        pvec[v] = v < 3 ? a.q[lidx<LAY>(n, r, NX, N)] : 0.0;
    }
    each_elem<NU * NX>(lane, [&](int e) { a.K[lidx<LAY>(n, e, NU * NX, N)] = 0.0; });
    each_elem<NU>(lane, [&](int e) { a.k[lidx<LAY>(n, e, NU, N)] = 0.0; });
    store_value(n, Preg, pvec, nsib_of(s) > 1);
    // inputs of the next two steps along the root path: step to stage s - 1
    // reads buffer A, to stage s - 2 buffer B, then they alternate
    // (Near the root the root's own data are loaded instead, unused: every
    // path then issues the same loads, and the compiler's count of loads
    // still in flight -- its waits -- need not assume that a buffer's loads
    // were the last ones issued.)
    WregIn bufA, bufB;
    load_stage(node_at(max(s - 1, 0)), bufA);
    load_edge(n, bufA);
    load_stage(node_at(max(s - 2, 0)), bufB);
    load_edge(node_at(max(s - 1, 0)), bufB);

    // One step up from n (stage s) to its parent; false when the walk ends.
    auto up = [&](WregIn& in) -> bool {
        if (s == 0) return false;
        if (base - (s - 3) >= 64) reload(s);
        const int nsib = nsib_of(s);
        const int par = node_at(s - 1);
        // with one sibling, its edge is requested with the count (after
        // the wait for this walker's stores, which would wait for it too),
        // for the case that this walker arrives last
        WregIn sib;
        int sib_j = -1;
        if (nsib > 1) {
            // hand the value function over: the stores complete before the count
            wait_own_stores();
            if (nsib == 2) {
                const int pf = __builtin_amdgcn_readlane(c0v, lane_of(s - 1));
                sib_j = pf == n ? pf + 1 : pf;
                load_edge(sib_j, sib);
            }
            __syncthreads();
            if (lane == 0) sgo = (atomicAdd(&arrive[par], 1) == nsib - 1);
            __syncthreads();
            if (!sgo) return false;
        }
        const int child = n;
        n = par;
        --s;
        const int k = lane_of(s);
        const int cfirst = __builtin_amdgcn_readlane(c0v, k), ccount = __builtin_amdgcn_readlane(cntv, k);
        f64x4 zm, zc;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            zm[v] = in.z[v];
            zc[v] = li == 0 ? in.zc[v] : 0.0;
        }
        if (ccount == 1) {
            add_child(Preg, pvec, in, zm, zc);
        } else {
            // every child in child order (deterministic sums): this walker's
            // own child from registers, the others from memory
            for (int j = cfirst; j < cfirst + ccount; ++j) {
                f64x4 Pj;
                double pj[4];
                WregIn ej;
                if (j == child) {
                    Pj = Preg;
#pragma unroll
                    for (int v = 0; v < 4; ++v) pj[v] = pvec[v];
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        ej.d[m] = in.d[m];
                        ej.cb[m] = in.cb[m];
                    }
                } else if (j == sib_j) {
                    load_value_dev(j, Pj, pj);
                    ej = sib;
                } else {
                    load_value_dev(j, Pj, pj);
                    load_edge(j, ej);
                }
                add_child(Pj, pj, ej, zm, zc);
            }
        }
        // the step after next: its inputs into the buffer just consumed
        load_stage(node_at(max(s - 2, 0)), in);
        load_edge(node_at(max(s - 1, 0)), in);
        // gains from rows NX.. of Z (element 3 of every lane): every lane
        // factors H = L L^T and forms the columns of Gh = L^-1 [G g] it
        // needs itself -- its own column li (for the gains and P), the
        // columns lk + 4 v (v < 3, rows of P) and gh -- so that no column
        // goes back through LDS
        sH[lk][li] = zm[3];
        if (li == 0) sH[lk][NZ] = zc[3];
        wave_sync();
        double L[NU][NU], inv[NU];
#pragma unroll
        for (int i = 0; i < NU; ++i)
#pragma unroll
            for (int j = 0; j < NU; ++j) L[i][j] = sH[i][NX + j];
        const bool ok = chol_inplace_rsq<NU>(L, inv);
        if (!ok && lane == 0) atomicMin(a.bad, n);
        auto column = [&](int c, double (&v)[NU]) {
#pragma unroll
            for (int i = 0; i < NU; ++i) v[i] = sH[i][c];
            chol_fwd<NU>(L, inv, v);
        };
        double gl[NU], gg[NU], gi[3][NU];
        column(li < NX ? li : NZ, gl);
        column(NZ, gg);
#pragma unroll
        for (int v = 0; v < 3; ++v) column(lk + 4 * v, gi[v]);
        wave_sync();  // sH is rewritten by the next step
        {
            // [K k] = -L^-T Gh: lanes li < NX take column li of K, the
            // others k (the same values)
            double x[NU];
#pragma unroll
            for (int i = 0; i < NU; ++i) x[i] = gl[i];
            chol_bwd<NU>(L, inv, x);
#pragma unroll
            for (int i = 0; i < NU; ++i) pK0[i][(long)n * sK] = -x[i];
        }
        // P = W - Gh^T Gh and p = w - Gh^T gh, in the accumulator layout
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            double tP = 0.0, tp = 0.0;
#pragma unroll
            for (int r = 0; r < NU; ++r) {
                tP = fma(gi[v][r], gl[r], tP);
                tp = fma(gi[v][r], gg[r], tp);
            }
            Preg[v] = li < NX ? zm[v] - tP : 0.0;
            pvec[v] = zc[v] - tp;
        }
        Preg[3] = 0.0;
        pvec[3] = 0.0;
        store_value(n, Preg, pvec, nsib_of(s) > 1);
        return true;
    };
    for (;;) {
        if (!up(bufA)) break;
        if (!up(bufB)) break;
    }
}

// ------------------------------------------------------------------------
// Backward pass for larger state dimensions (the mass-spring chain,
// nx = 30, nu = 14): one workgroup of four wavefronts walks a leaf
// segment upwards, with the same last-arriver merges as k_bwd_wreg.  Per
// child, the two dense products run on the FP64 matrix cores
// (v_mfma_f64_16x16x4, 16 x 16 output tiles spread over the wavefronts):
//   S = P [A B c] + [0 0 p]         (NX x NC, NC = NX + NU + 1)
//   Z += [A B]^T S                  (Z = [[W G^T w],[G H g]], NZ x NC)
// then one wavefront factors H = L L^T, lanes take the columns of
// L^-1 [G g] and of the gains, and all threads form
//   P = (W + W^T)/2 - Gh^T Gh,  p = w - Gh^T gh  (Gh = L^-1 G, gh = L^-1 g).
// Operand layout of v_mfma_f64_16x16x4 (lane l, li = l % 16, lk = l / 16):
// A entry (li, lk), B entry (lk, li), result entries (lk + 4 v, li), v < 4.
// ------------------------------------------------------------------------
__host__ __device__ constexpr int pad16(int v) { return (v + 15) / 16 * 16; }

// Value of v in lane src of the wavefront (scalar reads of both halves;
// they read the register whether or not lane src is active)
__device__ __forceinline__ double lane_value(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Workgroup barrier that waits for this wavefront's LDS operations only, so
// that global loads in flight (the next node's inputs) stay in flight
// across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int NX, int NU, int LAY>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_bwd_mfma(TreeDev t, LqrArgs a, int* arrive)
{
    constexpr int NZ = NX + NU, NC = NZ + 1;
    constexpr int NXP = pad16(NX), NCP = pad16(NC), NZP = pad16(NZ);
    constexpr int KS = NXP / 4;                   // k steps of both products
    constexpr int NG = NX + 1;                    // columns of [G g]
    constexpr int NT = NU + NG;                   // columns of [H G g]
    constexpr int CW = NC + 1;                    // row pitch of D and Z
    static_assert(NXP == 32 && NCP / 16 <= 4, "two row tiles of S per column block, one wavefront per block");
    __shared__ __align__(16) double sD[NX][CW];   // [A B c] of the child edge
    __shared__ __align__(16) double sP[NX][NX + 1];  // the child's P (odd pitch: its columns are read across lanes)
    __shared__ __align__(16) double sp[NXP];
    __shared__ __align__(16) double sZ[NZ][CW];
    __shared__ __align__(16) double sG[NU][NG];   // L^-1 [G g]
    __shared__ int sgo;

    // thread indices are re-derived through an opaque copy at every step of
    // the walk, so that the compiler recomputes the many per-lane LDS
    // addresses where they are used instead of keeping them all live
    // across the walk (they would not fit in the registers)
    int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int li = lane & 15, lk = lane >> 4;
    auto refresh_ids = [&]() {
        int v = threadIdx.x;
        asm volatile("" : "+v"(v));
        tid = v;
        lane = v & 63;
        wave = v >> 6;
        li = lane & 15;
        lk = lane >> 4;
    };
    const int N = t.N;
    int n = t.leaves[blockIdx.x];


    // Every thread's share of a block of elements is requested at once and
    // stored to LDS afterwards, so that a thread has all its loads in flight
    // together instead of one after the other.
    // stage data of node m into Z: [[Q M^T q],[M R r]], element e of the
    // node's Q (NX x NX), M (NU x NX), q, R (NU x NU), r in that order, so
    // that the lanes of a wavefront read consecutive entries of one array
    constexpr int SE = NX * NX + NU * NX + NX + NU * NU + NU;
    auto stage_get = [&](int m, int e) -> double {
        if (e < NX * NX) return a.Q[lidx<LAY>(m, e, NX * NX, N)];
        e -= NX * NX;
        if (e < NU * NX) return a.M[lidx<LAY>(m, e, NU * NX, N)];
        e -= NU * NX;
        if (e < NX) return a.q[lidx<LAY>(m, e, NX, N)];
        e -= NX;
        if (e < NU * NU) return a.R[lidx<LAY>(m, e, NU * NU, N)];
        return a.r[lidx<LAY>(m, e - NU * NU, NU, N)];
    };
    auto stage_put = [&](int e, double v) {
        if (e < NX * NX) {
            sZ[e / NX][e % NX] = v;
            return;
        }
        e -= NX * NX;
        if (e < NU * NX) {
            const int i = e / NX, j = e % NX;
            sZ[NX + i][j] = v;
            sZ[j][NX + i] = v;
            return;
        }
        e -= NU * NX;
        if (e < NX) {
            sZ[e][NZ] = v;
            return;
        }
        e -= NX;
        if (e < NU * NU) {
            sZ[NX + e / NU][NX + e % NU] = v;
            return;
        }
        sZ[NX + e - NU * NU][NZ] = v;
    };
    // edge into node j: A (NX x NX), B (NX x NU), c into D = [A B c]
    constexpr int EE = NX * NX + NX * NU + NX;
    auto edge_get = [&](int j, int e) -> double {
        if (e < NX * NX) return a.A[lidx<LAY>(j, e, NX * NX, N)];
        e -= NX * NX;
        if (e < NX * NU) return a.B[lidx<LAY>(j, e, NX * NU, N)];
        return a.c[lidx<LAY>(j, e - NX * NU, NX, N)];
    };
    auto edge_put = [&](int e, double v) {
        if (e < NX * NX) {
            sD[e / NX][e % NX] = v;
            return;
        }
        e -= NX * NX;
        if (e < NX * NU) {
            sD[e / NU][NX + e % NU] = v;
            return;
        }
        sD[e - NX * NU][NZ] = v;
    };
    // Loaders of the elements [e0, e1) of the stage or edge data by NT_
    // threads (rank t): every thread's share is requested at once, then
    // stored.  Stage elements: Q [0, QE), M [QE, ME), q [ME, RE0), R and r
    // [RE0, SE); the "upper" part (Q, q) is what the value function's
    // formation still reads from Z.
    constexpr int QE = NX * NX, ME = QE + NU * NX, RE0 = ME + NX;
    auto load_part = [&](auto get, auto put, int node, int e0, int e1, auto ntc, int t) {
        constexpr int NT_ = decltype(ntc)::value;
        constexpr int CNT = (SE + NT_ - 1) / NT_;
        double v[CNT];
#pragma unroll
        for (int it = 0; it < CNT; ++it) {
            const int e = e0 + t + NT_ * it;
            v[it] = e < e1 ? get(node, e) : 0.0;
        }
#pragma unroll
        for (int it = 0; it < CNT; ++it) {
            const int e = e0 + t + NT_ * it;
            if (e < e1) put(e, v[it]);
        }
    };
    // every thread's share is requested at once, then stored
    constexpr int CNT_S = (SE + 255) / 256, CNT_E = (EE + 255) / 256;
    auto load_stage = [&](int m) {
        double v[CNT_S];
#pragma unroll
        for (int it = 0; it < CNT_S; ++it) {
            const int e = tid + 256 * it;
            v[it] = e < SE ? stage_get(m, e) : 0.0;
        }
#pragma unroll
        for (int it = 0; it < CNT_S; ++it) {
            const int e = tid + 256 * it;
            if (e < SE) stage_put(e, v[it]);
        }
    };
    auto load_edge = [&](int j) {
        double v[CNT_E];
#pragma unroll
        for (int it = 0; it < CNT_E; ++it) {
            const int e = tid + 256 * it;
            v[it] = e < EE ? edge_get(j, e) : 0.0;
        }
#pragma unroll
        for (int it = 0; it < CNT_E; ++it) {
            const int e = tid + 256 * it;
            if (e < EE) edge_put(e, v[it]);
        }
    };
    // value function of child j, written by another workgroup
    auto load_value = [&](int j) {
        constexpr int CNT = (NX * NX + NX + 255) / 256;
        double v[CNT];
#pragma unroll
        for (int it = 0; it < CNT; ++it) {
            const int e = tid + 256 * it;
            v[it] = e < NX * NX ? ld_shared_dev(&a.P[lidx<LAY>(j, e, NX * NX, N)])
                  : (e < NX * NX + NX ? ld_shared_dev(&a.p[lidx<LAY>(j, e - NX * NX, NX, N)]) : 0.0);
        }
#pragma unroll
        for (int it = 0; it < CNT; ++it) {
            const int e = tid + 256 * it;
            if (e < NX * NX) sP[e / NX][e % NX] = v[it];
            else if (e < NX * NX + NX) sp[e - NX * NX] = v[it];
        }
    };
    // Per child: wavefront w < NCP / 16 takes column block w (16 columns) of
    // S and of Z.  It computes both row tiles of S = P [A B c] + [0 0 p] for
    // its block and keeps them in the accumulator registers, whose layout
    // (lane l, element v: row l / 16 + 4 v) is the B-operand layout of the
    // k-blocks of Z += [A B]^T S, so S never goes through LDS.
    auto add_child = [&]() {
        lds_barrier();
        if (wave < NCP / 16) {
            const int col = 16 * wave + li;
            const bool cin = col < NC;
            f64x4 s0 = {0.0, 0.0, 0.0, 0.0}, s1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k = 4 * ks + lk;
                const double bv = (k < NX && cin) ? sD[k][col] : 0.0;
                const double a0 = (li < NX && k < NX) ? sP[li][k] : 0.0;
                const double a1 = (16 + li < NX && k < NX) ? sP[16 + li][k] : 0.0;
                s0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv, s0, 0, 0, 0);
                s1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv, s1, 0, 0, 0);
            }
            if (col == NZ) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    s0[v] += sp[lk + 4 * v];
                    if (16 + lk + 4 * v < NX) s1[v] += sp[16 + lk + 4 * v];
                }
            }
#pragma unroll
            for (int ti = 0; ti < NZP / 16; ++ti) {
                const int rowa = 16 * ti + li;
                f64x4 acc;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * ti + lk + 4 * v;
                    acc[v] = (r < NZ && cin) ? sZ[r][col] : 0.0;
                }
#pragma unroll
                for (int kb = 0; kb < KS; ++kb) {
                    const int k = 4 * kb + lk;
                    const double av = (k < NX && rowa < NC) ? sD[k][rowa] : 0.0;
                    const double bv = kb < 4 ? s0[kb & 3] : s1[kb & 3];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * ti + lk + 4 * v;
                    if (r < NZ && cin) sZ[r][col] = acc[v];
                }
            }
        }
        lds_barrier();
    };
    // Gains and value function of node m from the accumulated Z, by one
    // wavefront without barriers: lane c holds column c of T = [H G g]
    // (NU x NT) in registers and the lanes run the right-looking Cholesky
    // factorisation of H with the columns of [G g] carried along; the pivot
    // and the column of step j come from lane j by scalar reads.  Afterwards
    // lane j < NU holds column j of L and lane NU + c column c of
    // Gh = L^-1 [G g], both unscaled; the latter solve L^T X = Gh for their
    // column (X = -[K k]) with the entries of L read from the lanes that
    // hold them.
    // Then all threads form P = (W + W^T)/2 - Gh^T Gh and p = w - Gh^T gh.
    // next_stage >= 0: the next step is a chain step (node next_stage, edge
    // into m); while wavefront 0 computes the gains, the other three load
    // its edge into D and the parts of its stage data that the formation
    // of P no longer reads (M, R, r) into Z.
    auto finish = [&](int m, bool shared_out, int next_stage) {
        double col[NU];
        if (wave == 0) {
            const int c = lane;
#pragma unroll
            for (int r = 0; r < NU; ++r)
                col[r] = c < NU ? sZ[NX + r][NX + c]
                       : (c < NT ? sZ[NX + r][c - NU < NX ? c - NU : NZ] : 0.0);
        }
        // rows NX.. of Z and all of D are free from here on
        lds_barrier();
        if (wave == 0) {
            const int c = lane;
            double inv[NU];
            bool ok = true;
#pragma unroll
            for (int j = 0; j < NU; ++j) {
                const double d = lane_value(col[j], j);
                ok = ok && d > 0.0;
                const double dd = d > 0.0 ? d : 1.0;
                const double y = rsqrt_refined(dd);
                inv[j] = y;
                const double tjc = col[j] * y;  // L[c][j] in lane c > j
#pragma unroll
                for (int r = j + 1; r < NU; ++r) {
                    const double lrj = lane_value(col[r], j) * y;  // L[r][j], from lane j
                    if (c > j) col[r] -= lrj * tjc;
                }
            }
            if (lane == 0 && !ok) atomicMin(a.bad, m);
            // No column is scaled in place: lane j keeps column j of the
            // Schur complement of step j unscaled (L[r][j] = col[r] inv[j]
            // for r > j) and lane NU + c its column of [G g] after step j
            // (Gh[j][c] = col[j] inv[j]).  The solve reads the former across
            // lanes, in a branch that lane j does not take; inside the branch
            // the compiler may take a lane-dependent select for the side
            // that the branch's own lanes see (and it does), so an opaque
            // copy pins every lane's columns before the branch.
#pragma unroll
            for (int j = 0; j < NU; ++j) asm volatile("" : "+v"(col[j]));
            if (c >= NU && c < NT) {
                const int g = c - NU;  // column of [G g]
                double gh[NU];
#pragma unroll
                for (int r = 0; r < NU; ++r) {
                    gh[r] = col[r] * inv[r];
                    sG[r][g] = gh[r];
                }
                // L^T x = gh
                double x[NU];
#pragma unroll
                for (int j = NU - 1; j >= 0; --j) {
                    double t = 0.0;
#pragma unroll
                    for (int k = j + 1; k < NU; ++k) t = fma(lane_value(col[k], j), x[k], t);
                    x[j] = (gh[j] - t * inv[j]) * inv[j];
                }
#pragma unroll
                for (int r = 0; r < NU; ++r) {
                    if (g < NX) a.K[lidx<LAY>(m, r * NX + g, NU * NX, N)] = -x[r];
                    else a.k[lidx<LAY>(m, r, NU, N)] = -x[r];
                }
            }
        } else if (next_stage >= 0) {
            const int t3 = tid - 64;
            load_part(edge_get, edge_put, m, 0, EE, std::integral_constant<int, 192>{}, t3);
            load_part(stage_get, stage_put, next_stage, QE, ME, std::integral_constant<int, 192>{}, t3);
            load_part(stage_get, stage_put, next_stage, RE0, SE, std::integral_constant<int, 192>{}, t3);
        }
        lds_barrier();
        // P and p from Gh (the child's P in sP was last read by the products)
#pragma unroll 1
        for (int e = tid; e < NX * NX; e += 256) {
            const int i = e / NX, j = e % NX;
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < NU; ++r) s = fma(sG[r][i], sG[r][j], s);
            const double pv = 0.5 * (sZ[i][j] + sZ[j][i]) - s;
            sP[i][j] = pv;
            if (shared_out) st_shared_dev(&a.P[lidx<LAY>(m, e, NX * NX, N)], pv);
            else a.P[lidx<LAY>(m, e, NX * NX, N)] = pv;
        }
        if (tid < NX) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < NU; ++r) s = fma(sG[r][tid], sG[r][NX], s);
            const double pv = sZ[tid][NZ] - s;
            sp[tid] = pv;
            if (shared_out) st_shared_dev(&a.p[lidx<LAY>(m, tid, NX, N)], pv);
            else a.p[lidx<LAY>(m, tid, NX, N)] = pv;
        }
        lds_barrier();
    };

    // the leaf: P = Q_f, p = q_f, no gains
    {
        const int4 inf = t.info[n];
        const bool shared_out = inf.w > 1;
        #pragma unroll 1
        for (int e = tid; e < NX * NX; e += 256) {
            const double v = a.Q[lidx<LAY>(n, e, NX * NX, N)];
            sP[e / NX][e % NX] = v;
            if (shared_out) st_shared_dev(&a.P[lidx<LAY>(n, e, NX * NX, N)], v);
            else a.P[lidx<LAY>(n, e, NX * NX, N)] = v;
        }
        #pragma unroll 1
        for (int e = tid; e < NX; e += 256) {
            const double v = a.q[lidx<LAY>(n, e, NX, N)];
            sp[e] = v;
            if (shared_out) st_shared_dev(&a.p[lidx<LAY>(n, e, NX, N)], v);
            else a.p[lidx<LAY>(n, e, NX, N)] = v;
        }
        #pragma unroll 1
        for (int e = tid; e < NU * NX; e += 256) a.K[lidx<LAY>(n, e, NU * NX, N)] = 0.0;
        #pragma unroll 1
        for (int e = tid; e < NU; e += 256) a.k[lidx<LAY>(n, e, NU, N)] = 0.0;
    }
    bool have_next = false;
    for (;;) {
        refresh_ids();
        const int4 inf = t.info[n];
        const int par = inf.z, nsib = inf.w;
        if (par < 0) break;
        if (nsib > 1) {
            // hand the value function over: every thread's stores complete
            // before the count
            wait_own_stores();
            __syncthreads();
            if (tid == 0) sgo = (atomicAdd(&arrive[par], 1) == nsib - 1);
            __syncthreads();
            if (!sgo) break;
        }
        const int child = n;
        n = par;
        const int4 pinf = t.info[n];
        const bool shared_out = pinf.w > 1;
        lds_barrier();
        if (nsib == 1) {
            // the only child's value function is still in sP, sp
            if (have_next) {
                // edge and lower stage data were loaded during the last step
                load_part(stage_get, stage_put, n, 0, QE, std::integral_constant<int, 256>{}, tid);
                load_part(stage_get, stage_put, n, ME, RE0, std::integral_constant<int, 256>{}, tid);
            } else {
                load_stage(n);
                load_edge(child);
            }
            add_child();
        } else {
            load_stage(n);
            for (int j = pinf.x; j < pinf.y; ++j) {
                lds_barrier();
                load_edge(j);
                load_value(j);
                add_child();
            }
        }
        // the next step is a chain step: n is its parent's only child
        have_next = pinf.z >= 0 && pinf.w == 1;
        finish(n, shared_out, have_next ? pinf.z : -1);
    }
}

// ------------------------------------------------------------------------
// forward rollout: G lanes per root-to-leaf path, inputs D steps ahead
// ------------------------------------------------------------------------
// Value of lane j of each row of 16 lanes, for every lane of the row
// (one DPP move, row_newbcast, instead of a trip through the LDS crossbar).
template <int J>
__device__ __forceinline__ double row_bcast(double v)
{
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + J, 0xf, 0xf, false);
}
template <int J>
__device__ __forceinline__ float row_bcast(float v)
{
    return __builtin_amdgcn_update_dpp(0.0f, v, 0x150 + J, 0xf, 0xf, false);
}
template <int J>
__device__ __forceinline__ int row_bcast_int(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x150 + J, 0xf, 0xf, false);
}
// lane J of the group of G lanes that starts at lane base
// lane J of the wavefront (a group of 64 lanes): one scalar read per dword
template <int J>
__device__ __forceinline__ float wave_lane(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), J));
}
template <int J>
__device__ __forceinline__ double wave_lane(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), J);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), J);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int G, int J, class T>
__device__ __forceinline__ T group_value(T v, int base)
{
    if constexpr (G == 16)
        return row_bcast<J>(v);
    else if constexpr (G == 64)
        return wave_lane<J>(v);
    else
        return __shfl(v, base + J, 64);
}
template <int G, int J>
__device__ __forceinline__ int group_value_int(int v, int base)
{
    if constexpr (G == 16)
        return row_bcast_int<J>(v);
    else if constexpr (G == 64)
        return __builtin_amdgcn_readlane(v, J);
    else
        return __shfl(v, base + J, 64);
}
template <int G, class T, int... J>
__device__ __forceinline__ void group_gather(T v, int base, T* out, std::integer_sequence<int, J...>)
{
    ((out[J] = group_value<G, J>(v, base)), ...);
}
template <class F, int... K>
__device__ __forceinline__ void unroll_impl(F&& f, std::integer_sequence<int, K...>)
{
    (f(std::integral_constant<int, K>{}), ...);
}
template <int CNT, class F>
__device__ __forceinline__ void unroll(F&& f)
{
    unroll_impl(f, std::make_integer_sequence<int, CNT>{});
}

// One step of a path: lane g < NX holds row g of [A B c] of the edge into
// the next node; lane NX + i holds row i of [K k] of the node (lanes past
// NX + NU repeat the last row).  Both roles evaluate r = w . x + c0, which is
// A x + c on the first lanes and u = K x + k on the others.
template <int NX, int NU, class T = double>
struct FwdRow {
    T w[NX], b[NU], c0;
};

template <int NX, int NU, int LAY, class T>
__device__ __forceinline__ void fwd_row_fill(const LqrArgsT<T>& a, int N, int n, int m, int g, FwdRow<NX, NU, T>& f)
{
    // the last step of a path needs no inputs, and stages past its end
    // none at all: those read the entries of node n, or of the root, which
    // are in bounds, so that the loads need no branch
    const int nn = n >= 0 ? n : 0;
    const int me = m >= 0 ? m : nn;
    const bool krow = g >= NX;
    const int i = krow ? (g - NX < NU ? g - NX : NU - 1) : g;
    const T* wp = krow ? a.K : a.A;
    const int wn = krow ? nn : me, wsz = krow ? NU * NX : NX * NX;
#pragma unroll
    for (int j = 0; j < NX; ++j) f.w[j] = wp[lidx<LAY>(wn, i * NX + j, wsz, N)];
    const int ib = krow ? 0 : i;
#pragma unroll
    for (int j = 0; j < NU; ++j) f.b[j] = a.B[lidx<LAY>(me, ib * NU + j, NX * NU, N)];
    f.c0 = krow ? a.k[lidx<LAY>(nn, i, NU, N)] : a.c[lidx<LAY>(me, i, NX, N)];
}

template <int NX, int NU, int LAY, int G, int D, class T = double>
__global__ void __launch_bounds__(64) k_fwd_rows(TreeDev t, LqrArgsT<T> a)
{
    static_assert(NX + NU <= G && 64 % G == 0 && G % D == 0, "group must hold the rows of [A B c] and [K k]");
    const int tid = blockIdx.x * 64 + threadIdx.x;
    const int path = tid / G;
    const int g = tid % G;
    const int base = (int)threadIdx.x - g;
    const int N = t.N, Z = t.num_leaves;
    if (path >= Z) return;  // whole group leaves together
    const int last = t.leaf_stage[path];
    const int wfrom = t.write_from[path];
    // node ids, one block of G stages per register: lane g of the group
    // holds the node at stage s0 + g; two blocks are held and the next one
    // is requested a block ahead
    auto ids = [&](int s0) -> int {
        const int s = s0 + g;
        return s <= last ? t.path[(long)s * Z + path] : -1;
    };
    int blk0 = ids(0), blk1 = ids(G);
    FwdRow<NX, NU, T> ring[D];
    // node at stage s0 + K (K a constant, K < 2G) of the blocks held
    auto node_at = [&](auto kc) -> int {
        constexpr int K = decltype(kc)::value;
        if constexpr (K < G)
            return group_value_int<G, K>(blk0, base);
        else
            return group_value_int<G, K - G>(blk1, base);
    };
    unroll<D>([&](auto dc) {
        constexpr int d = decltype(dc)::value;
        fwd_row_fill<NX, NU, LAY>(a, N, node_at(std::integral_constant<int, d>{}),
                                  node_at(std::integral_constant<int, d + 1>{}), g, ring[d]);
    });
    T xg = g < NX ? a.x0[g] : T(0);
    for (int s0 = 0; s0 <= last; s0 += G) {
        const int blk2 = ids(s0 + 2 * G);
        unroll<G>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int s = s0 + k;
            // no branch in a step except around the stores: a value that is
            // kept on one side of a branch and loaded on the other would be
            // merged by a copy, and the copy waits for every load in flight
            const bool live = s <= last, fin = s == last;
            FwdRow<NX, NU, T>& f = ring[k % D];
            const int n = node_at(std::integral_constant<int, k>{});
            const bool writer = live && s >= wfrom;
            T xs[NX];
            group_gather<G>(xg, base, xs, std::make_integer_sequence<int, NX>{});
            if (writer && g < NX) a.x[lidx<LAY>(n, g, NX, N)] = xg;
            T r = f.c0;
#pragma unroll
            for (int j = 0; j < NX; ++j) r += f.w[j] * xs[j];
            if (writer && g >= NX && g < NX + NU) a.u[lidx<LAY>(n, g - NX, NU, N)] = fin ? T(0) : r;
            T us[NU];
            unroll<NU>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                us[i] = group_value<G, NX + i>(r, base);
            });
#pragma unroll
            for (int j = 0; j < NU; ++j) r += f.b[j] * us[j];
            xg = (live && !fin) ? r : xg;
            // refill with the inputs of stage s + D
            if constexpr (k + D + 1 < 2 * G) {
                fwd_row_fill<NX, NU, LAY>(a, N, node_at(std::integral_constant<int, k + D>{}),
                                          node_at(std::integral_constant<int, k + D + 1>{}), g, f);
            } else {
                // stage s + D + 1 lies in the block after next
                const int n1 = node_at(std::integral_constant<int, k + D>{});
                const int n2 = group_value_int<G, k + D + 1 - 2 * G>(blk2, base);
                fwd_row_fill<NX, NU, LAY>(a, N, n1, n2, g, f);
            }
        });
        blk0 = blk1;
        blk1 = blk2;
    }
}

// Costates lam_n = P_n x_n + p_n for every node; also re-arms the branch
// counters and the positive-definiteness flag for the next solve.
template <int NX, int LAY, class T = double>
__global__ void __launch_bounds__(256) k_costate(TreeDev t, LqrArgsT<T> a, int* arrive)
{
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = t.N;
    if (tid == 0) {
        *a.bad_out = *a.bad;
        *a.bad = INT_MAX;
    }
    if (tid >= (long)N * NX) return;
    int n, i;
    if constexpr (LAY == BMPC_LAYOUT_NODE_MAJOR) {
        n = (int)(tid / NX);
        i = (int)(tid % NX);
    } else {
        i = (int)(tid / N);
        n = (int)(tid % N);
    }
    if (i == 0) arrive[n] = 0;
    T acc = a.p[lidx<LAY>(n, i, NX, N)];
#pragma unroll
    for (int j = 0; j < NX; ++j)
        acc += a.P[lidx<LAY>(n, i * NX + j, NX * NX, N)] * a.x[lidx<LAY>(n, j, NX, N)];
    a.lam[lidx<LAY>(n, i, NX, N)] = acc;
}

// ------------------------------------------------------------------------
// mixed precision: FP32 Riccati solves, FP64 residuals, iterative refinement
// ------------------------------------------------------------------------

// Elementwise FP64 -> FP32 copy of one matrix array.
__global__ void __launch_bounds__(256) k_to_f32(const double* __restrict__ src, float* __restrict__ dst, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

// Largest |value| over the workgroup (256 threads), merged into *slot by
// one atomic: IEEE order of non-negative doubles is the order of their bit
// patterns, and a NaN's pattern lies above that of every finite value and
// infinity, so it survives the maximum.
__device__ __forceinline__ void block_abs_max_into(double v, unsigned long long* slot)
{
    __shared__ unsigned long long wmax[4];
    unsigned long long b = (unsigned long long)__double_as_longlong(fabs(v));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(b, off, 64);
        b = o > b ? o : b;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long m01 = wmax[0] > wmax[1] ? wmax[0] : wmax[1];
        const unsigned long long m23 = wmax[2] > wmax[3] ? wmax[2] : wmax[3];
        atomicMax(slot, m01 > m23 ? m01 : m23);
    }
}

// KKT residual of the tree LQR at the FP64 iterate (x, u, lam), one thread
// per (node n, state row i).  With z = 0 (FIRST) the residual is the data
// itself.  Rows, for the Lagrangian cost + sum_j lam_j^T (A_j x_p + B_j u_p
// + c_j - x_j) + lam_0^T (x0 - x_0):
//   g_u[n] = R u + M x + r + sum_{j child} B_j^T lam_j         (control nodes)
//   g_x[n] = Q x + M^T u + q + sum_{j child} A_j^T lam_j - lam_n
//   d[n]   = A_n x_p + B_n u_p + c_n - x_n   (root: x0 - x_0)
// They are the linear terms of the correction problem, written in FP32 as
// its (r, q, c, x0); the largest |row| is merged into *norm if it is set.
template <int NX, int NU, int LAY, bool FIRST>
__global__ void __launch_bounds__(256) k_lqr_residual(TreeDev t, LqrArgs a, float* __restrict__ q32,
                                                      float* __restrict__ r32, float* __restrict__ c32,
                                                      float* __restrict__ x032, unsigned long long* norm)
{
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = t.N;
    double worst = 0.0;
    if (tid < (long)N * NX) {
        int n, i;
        if constexpr (LAY == BMPC_LAYOUT_NODE_MAJOR) {
            n = (int)(tid / NX);
            i = (int)(tid % NX);
        } else {
            i = (int)(tid / N);
            n = (int)(tid % N);
        }
        const int4 inf = t.info[n];
        const bool leaf = inf.x == inf.y;
        auto X = [&](int m, int k) { return FIRST ? 0.0 : a.x[lidx<LAY>(m, k, NX, N)]; };
        auto U = [&](int m, int k) { return FIRST ? 0.0 : a.u[lidx<LAY>(m, k, NU, N)]; };
        auto Lm = [&](int m, int k) { return FIRST ? 0.0 : a.lam[lidx<LAY>(m, k, NX, N)]; };
        // stationarity in x
        double gx = a.q[lidx<LAY>(n, i, NX, N)];
        if constexpr (!FIRST) {
#pragma unroll
            for (int k = 0; k < NX; ++k) gx += a.Q[lidx<LAY>(n, i * NX + k, NX * NX, N)] * X(n, k);
            if (!leaf) {
#pragma unroll
                for (int k = 0; k < NU; ++k) gx += a.M[lidx<LAY>(n, k * NX + i, NU * NX, N)] * U(n, k);
            }
            for (int j = inf.x; j < inf.y; ++j) {
#pragma unroll
                for (int k = 0; k < NX; ++k) gx += a.A[lidx<LAY>(j, k * NX + i, NX * NX, N)] * Lm(j, k);
            }
            gx -= Lm(n, i);
        }
        q32[lidx<LAY>(n, i, NX, N)] = (float)gx;
        // dynamics defect of the edge into n
        double d;
        if (inf.z < 0) {
            d = a.x0[i] - X(n, i);
            x032[i] = (float)d;
        } else {
            const int pn = inf.z;
            d = a.c[lidx<LAY>(n, i, NX, N)];
            if constexpr (!FIRST) {
#pragma unroll
                for (int k = 0; k < NX; ++k) d += a.A[lidx<LAY>(n, i * NX + k, NX * NX, N)] * X(pn, k);
#pragma unroll
                for (int k = 0; k < NU; ++k) d += a.B[lidx<LAY>(n, i * NU + k, NX * NU, N)] * U(pn, k);
                d -= X(n, i);
            }
        }
        c32[lidx<LAY>(n, i, NX, N)] = (float)d;
        worst = fmax(fabs(gx), fabs(d));
        if (gx != gx || d != d) worst = gx + d;
        // stationarity in u
        if (i < NU) {
            double gu = 0.0;
            if (!leaf) {
                gu = a.r[lidx<LAY>(n, i, NU, N)];
                if constexpr (!FIRST) {
#pragma unroll
                    for (int k = 0; k < NU; ++k) gu += a.R[lidx<LAY>(n, i * NU + k, NU * NU, N)] * U(n, k);
#pragma unroll
                    for (int k = 0; k < NX; ++k) gu += a.M[lidx<LAY>(n, i * NX + k, NU * NX, N)] * X(n, k);
                    for (int j = inf.x; j < inf.y; ++j) {
#pragma unroll
                        for (int k = 0; k < NX; ++k) gu += a.B[lidx<LAY>(j, k * NU + i, NX * NU, N)] * Lm(j, k);
                    }
                }
            }
            r32[lidx<LAY>(n, i, NU, N)] = (float)gu;
            if (fabs(gu) > worst || gu != gu) worst = gu != gu ? gu : fabs(gu);
        }
    }
    if (norm) block_abs_max_into(worst, norm);
}

// z <- z + dz (or z <- dz on the first solve), elementwise over the
// flat arrays: x and lam have N*NX entries, u N*NU, in the same layout as
// their FP32 corrections.
template <bool FIRST>
__global__ void __launch_bounds__(256) k_lqr_update(long nxe, long nue, double* __restrict__ x,
                                                    double* __restrict__ u, double* __restrict__ lam,
                                                    const float* __restrict__ dx, const float* __restrict__ du,
                                                    const float* __restrict__ dl)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nxe) {
        x[i] = FIRST ? (double)dx[i] : x[i] + (double)dx[i];
        lam[i] = FIRST ? (double)dl[i] : lam[i] + (double)dl[i];
    }
    if (i < nue) u[i] = FIRST ? (double)du[i] : u[i] + (double)du[i];
}

__global__ void k_zero_norms(unsigned long long* norm, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) norm[i] = 0ull;
}

// ------------------------------------------------------------------------
// dispatch
// ------------------------------------------------------------------------
struct LqrKernels {
    int nx, nu, layout, group;
    void (*bwd_lane)(TreeDev, LqrArgs, int*);
    void (*bwd_mfma)(TreeDev, LqrArgs, int*);
    void (*bwd_seg)(TreeDev, LqrArgs, int*, int);
    void (*fwd)(TreeDev, LqrArgs);
    void (*costate)(TreeDev, LqrArgs, int*);
    // FP32 solve and the FP64 residual of the mixed-precision refinement
    void (*bwd_lane32)(TreeDev, LqrArgsT<float>, int*);
    void (*fwd32)(TreeDev, LqrArgsT<float>);
    void (*costate32)(TreeDev, LqrArgsT<float>, int*);
    void (*residual_first)(TreeDev, LqrArgs, float*, float*, float*, float*, unsigned long long*);
    void (*residual)(TreeDev, LqrArgs, float*, float*, float*, float*, unsigned long long*);
    // nx = 12, nu = 4: register-resident matrix-core backward pass
    void (*bwd_wreg)(TreeDev, LqrArgs, int*);
    // nx = 4, nu = 2: 16 lanes per leaf chain
    void (*bwd_quad)(TreeDev, LqrArgs, int*);
    void (*bwd_quad32)(TreeDev, LqrArgsT<float>, int*);
    // bytes of one segment-scan element (the kernel's LDS per chunk node)
    size_t seg_cvf_bytes;
};

template <int NX, int NU, int LAY, bool LANE>
static LqrKernels make_k()
{
    // rows of 16 lanes: the broadcasts inside a group are DPP row moves
    constexpr int G = 16;
    LqrKernels k{NX, NU, LAY, G, nullptr, nullptr, nullptr, k_fwd_rows<NX, NU, LAY, G, 4>,
                 k_costate<NX, LAY>};
    if constexpr (NX == 12 && NU == 4) k.bwd_wreg = k_bwd_wreg<NX, NU, LAY>;
    if constexpr (NX == 4 && NU == 2) {
        k.bwd_quad = k_bwd_quad<LAY>;
        k.bwd_quad32 = k_bwd_quad<LAY, float>;
    }
    if constexpr (LANE) {
        k.bwd_lane = k_bwd_lane<NX, NU, LAY>;
        k.bwd_lane32 = k_bwd_lane<NX, NU, LAY, float>;
        k.fwd32 = k_fwd_rows<NX, NU, LAY, G, 4, float>;
        k.costate32 = k_costate<NX, LAY, float>;
        k.residual_first = k_lqr_residual<NX, NU, LAY, true>;
        k.residual = k_lqr_residual<NX, NU, LAY, false>;
    }
    if constexpr (NX <= 4) {
        k.bwd_seg = k_bwd_seg<NX, NU, LAY>;
        k.seg_cvf_bytes = sizeof(Cvf<NX>);
    }
    return k;
}

// larger state dimensions: the matrix-core backward pass (four wavefronts
// per leaf segment) and a whole wavefront per path in the forward pass
template <int NX, int NU, int LAY>
static LqrKernels make_k_mfma()
{
    constexpr int G = 64;
    return LqrKernels{NX, NU, LAY, G, nullptr, k_bwd_mfma<NX, NU, LAY>, nullptr,
                      k_fwd_rows<NX, NU, LAY, G, 2>, k_costate<NX, LAY>, nullptr, nullptr, nullptr, nullptr, nullptr,
                      nullptr};
}

static const LqrKernels* find_kernels(int nx, int nu, int layout)
{
    static const LqrKernels table[] = {
        make_k<3, 1, 0, true>(),   make_k<3, 1, 1, true>(),
        make_k<4, 2, 0, true>(),   make_k<4, 2, 1, true>(),
        make_k<6, 3, 0, true>(),   make_k<6, 3, 1, true>(),
        make_k<12, 4, 0, false>(), make_k<12, 4, 1, false>(),
        make_k_mfma<30, 14, 0>(),  make_k_mfma<30, 14, 1>(),
    };
    for (const auto& k : table)
        if (k.nx == nx && k.nu == nu && k.layout == layout) return &k;
    return nullptr;
}

}  // namespace bmpc

using namespace bmpc;

struct bmpc_lqr_plan {
    const bmpc_tree* tree = nullptr;
    int nx = 0, nu = 0, layout = 0;
    const LqrKernels* kern = nullptr;
    double *K = nullptr, *k = nullptr, *P = nullptr, *p = nullptr;
    int* arrive = nullptr;
    int* bad = nullptr;  // [0] live flag, [1] copy taken after the last backward pass
    // FP32 workspace, allocated by the first FP32 or mixed-precision solve:
    // gains and value functions, then (mixed only) the FP32 copies of the
    // matrices, the correction problem's linear terms and its solution
    float *K32 = nullptr, *k32 = nullptr, *P32 = nullptr, *p32 = nullptr;
    float *A32 = nullptr, *B32 = nullptr, *Q32 = nullptr, *R32 = nullptr, *M32 = nullptr;
    float *q32 = nullptr, *r32 = nullptr, *c32 = nullptr, *x032 = nullptr;
    float *x32 = nullptr, *u32 = nullptr, *l32 = nullptr;
    // host-pointer solves: one pinned staging block and one device block of
    // the same size (inputs, then x0, then outputs), allocated by the first
    double* stage_host = nullptr;
    double* stage_dev = nullptr;
};

namespace {

bool alloc_f32(float** p, size_t n) { return *p || hipMalloc(p, sizeof(float) * (n ? n : 1)) == hipSuccess; }

bmpc_status ensure_f32(bmpc_lqr_plan* pl, bool mixed)
{
    const size_t N = pl->tree->h.N, n = pl->nx, m = pl->nu;
    bool ok = alloc_f32(&pl->K32, N * m * n) && alloc_f32(&pl->k32, N * m) && alloc_f32(&pl->P32, N * n * n) &&
              alloc_f32(&pl->p32, N * n);
    if (ok && mixed)
        ok = alloc_f32(&pl->A32, N * n * n) && alloc_f32(&pl->B32, N * n * m) && alloc_f32(&pl->Q32, N * n * n) &&
             alloc_f32(&pl->R32, N * m * m) && alloc_f32(&pl->M32, N * m * n) && alloc_f32(&pl->q32, N * n) &&
             alloc_f32(&pl->r32, N * m) && alloc_f32(&pl->c32, N * n) && alloc_f32(&pl->x032, n) &&
             alloc_f32(&pl->x32, N * n) && alloc_f32(&pl->u32, N * m) && alloc_f32(&pl->l32, N * n);
    return ok ? BMPC_OK : fail(BMPC_ERR_OOM, "device allocation of the FP32 LQR workspace failed");
}

void launch_f32(bmpc_lqr_plan* pl, const LqrArgsT<float>& a, hipStream_t s)
{
    const TreeDev& t = pl->tree->d;
    const int Z = t.num_leaves;
    if (pl->kern->bwd_quad32) {
        ProfScope ps("lqr_backward_level_quad_f32", s);
        const long threads = (long)Z * 16;
        hipLaunchKernelGGL(pl->kern->bwd_quad32, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, s, t, a,
                           pl->arrive);
    } else {
        ProfScope ps("lqr_backward_level_lane_f32", s);
        hipLaunchKernelGGL(pl->kern->bwd_lane32, dim3((Z + 63) / 64), dim3(64), 0, s, t, a, pl->arrive);
    }
    {
        ProfScope ps("lqr_forward_paths_f32", s);
        const long threads = (long)Z * pl->kern->group;
        hipLaunchKernelGGL(pl->kern->fwd32, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, s, t, a);
    }
    {
        ProfScope ps("lqr_costate_f32", s);
        const long threads = (long)t.N * pl->nx;
        hipLaunchKernelGGL(pl->kern->costate32, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, t, a,
                           pl->arrive);
    }
}

unsigned grid_for(long n, int block) { return (unsigned)std::max(1L, std::min((n + block - 1) / block, 65536L)); }

}  // namespace

extern "C" {

BMPC_API int32_t bmpc_lqr_supported(int32_t nx, int32_t nu, int32_t variant)
{
    const LqrKernels* k = find_kernels(nx, nu, 0);
    if (!k) return 0;
    if (variant == BMPC_RICCATI_AUTO || variant == BMPC_RICCATI_LEVEL) return 1;
    if (variant == BMPC_RICCATI_SEGSCAN) return k->bwd_seg ? 1 : 0;
    return 0;
}

BMPC_API bmpc_status bmpc_lqr_plan_create(const bmpc_tree* tree, int32_t nx, int32_t nu,
                                          int32_t layout, bmpc_lqr_plan** out)
{
    if (!tree || !out) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (layout != BMPC_LAYOUT_NODE_MAJOR && layout != BMPC_LAYOUT_ELEM_MAJOR)
        return fail(BMPC_ERR_INVALID_ARG, "unknown layout %d", layout);
    const LqrKernels* kern = find_kernels(nx, nu, layout);
    if (!kern) return fail(BMPC_ERR_UNSUPPORTED, "no tree-LQR kernel compiled for nx=%d nu=%d", nx, nu);
    bmpc_status st = tree_on_device(const_cast<bmpc_tree*>(tree));
    if (st != BMPC_OK) return st;
    auto* pl = new bmpc_lqr_plan();
    pl->tree = tree;
    pl->nx = nx;
    pl->nu = nu;
    pl->layout = layout;
    pl->kern = kern;
    const size_t N = tree->h.N;
    bool ok = hipMalloc(&pl->K, sizeof(double) * N * nx * nu) == hipSuccess &&
              hipMalloc(&pl->k, sizeof(double) * N * nu) == hipSuccess &&
              hipMalloc(&pl->P, sizeof(double) * N * nx * nx) == hipSuccess &&
              hipMalloc(&pl->p, sizeof(double) * N * nx) == hipSuccess &&
              hipMalloc(&pl->arrive, sizeof(int) * N) == hipSuccess &&
              hipMalloc(&pl->bad, 2 * sizeof(int)) == hipSuccess;
    if (!ok) {
        bmpc_lqr_plan_destroy(pl);
        return fail(BMPC_ERR_OOM, "device allocation for the LQR plan failed");
    }
    const int init_bad[2] = {INT_MAX, INT_MAX};
    if (hipMemset(pl->arrive, 0, sizeof(int) * N) != hipSuccess ||
        hipMemcpy(pl->bad, init_bad, sizeof init_bad, hipMemcpyHostToDevice) != hipSuccess) {
        bmpc_lqr_plan_destroy(pl);
        return fail(BMPC_ERR_HIP, "initialising the LQR plan failed");
    }
    *out = pl;
    return BMPC_OK;
}

BMPC_API void bmpc_lqr_plan_destroy(bmpc_lqr_plan* pl)
{
    if (!pl) return;
    (void)hipFree(pl->K);
    (void)hipFree(pl->k);
    (void)hipFree(pl->P);
    (void)hipFree(pl->p);
    (void)hipFree(pl->arrive);
    (void)hipFree(pl->bad);
    for (float* f : {pl->K32, pl->k32, pl->P32, pl->p32, pl->A32, pl->B32, pl->Q32, pl->R32, pl->M32, pl->q32,
                     pl->r32, pl->c32, pl->x032, pl->x32, pl->u32, pl->l32})
        (void)hipFree(f);
    (void)hipHostFree(pl->stage_host);
    (void)hipFree(pl->stage_dev);
    delete pl;
}

BMPC_API bmpc_status bmpc_lqr_solve(bmpc_lqr_plan* pl, const double* A, const double* B,
                                    const double* c, const double* Q, const double* R,
                                    const double* M, const double* q, const double* r,
                                    const double* x0, double* x, double* u, double* lam,
                                    double* K, double* k, double* P, double* p, int32_t variant,
                                    void* stream)
{
    if (!pl) return fail(BMPC_ERR_INVALID_ARG, "plan is NULL");
    if (!A || !B || !c || !Q || !R || !M || !q || !r || !x0 || !x || !u || !lam)
        return fail(BMPC_ERR_INVALID_ARG, "NULL input or output array");
    if (variant != BMPC_RICCATI_AUTO && variant != BMPC_RICCATI_LEVEL && variant != BMPC_RICCATI_SEGSCAN)
        return fail(BMPC_ERR_INVALID_ARG, "unknown Riccati variant %d", variant);
    if (variant == BMPC_RICCATI_SEGSCAN && !pl->kern->bwd_seg)
        return fail(BMPC_ERR_UNSUPPORTED, "the segment-scan backward pass is compiled for nx <= 4 only");
    hipStream_t s = (hipStream_t)stream;
    LqrArgs a{A, B, c, Q, R, M, q, r, x0, x, u, lam, K ? K : pl->K, k ? k : pl->k,
              P ? P : pl->P, p ? p : pl->p, pl->bad, pl->bad + 1};
    const TreeDev& t = pl->tree->d;
    const int Z = t.num_leaves;
    if (variant == BMPC_RICCATI_SEGSCAN) {
        ProfScope ps("lqr_backward_segscan", s);
        // single-child nodes of the longest segment (all but its bottom node)
        const int ch = std::min(64, std::max(1, t.max_seg_len - 1));
        hipLaunchKernelGGL(pl->kern->bwd_seg, dim3(Z), dim3(64), 2 * ch * pl->kern->seg_cvf_bytes, s, t, a,
                           pl->arrive, ch);
    } else if (pl->kern->bwd_mfma) {
        ProfScope ps("lqr_backward_level_mfma", s);
        hipLaunchKernelGGL(pl->kern->bwd_mfma, dim3(Z), dim3(256), 0, s, t, a, pl->arrive);
    } else if (pl->kern->bwd_wreg) {
        ProfScope ps("lqr_backward_level_wreg", s);
        hipLaunchKernelGGL(pl->kern->bwd_wreg, dim3(Z), dim3(64), 0, s, t, a, pl->arrive);
    } else if (pl->kern->bwd_quad) {
        ProfScope ps("lqr_backward_level_quad", s);
        const long threads = (long)Z * 16;
        hipLaunchKernelGGL(pl->kern->bwd_quad, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, s, t, a,
                           pl->arrive);
    } else {
        // every table entry without one of the three above has the lane kernel
        ProfScope ps("lqr_backward_level_lane", s);
        hipLaunchKernelGGL(pl->kern->bwd_lane, dim3((Z + 63) / 64), dim3(64), 0, s, t, a, pl->arrive);
    }
    {
        ProfScope ps("lqr_forward_paths", s);
        const long threads = (long)Z * pl->kern->group;
        hipLaunchKernelGGL(pl->kern->fwd, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, s, t, a);
    }
    {
        ProfScope ps("lqr_costate", s);
        const long threads = (long)t.N * pl->nx;
        hipLaunchKernelGGL(pl->kern->costate, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                           t, a, pl->arrive);
    }
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_lqr_solve_host(bmpc_lqr_plan* pl, const double* A, const double* B,
                                         const double* c, const double* Q, const double* R,
                                         const double* M, const double* q, const double* r,
                                         const double* x0, double* x, double* u, double* lam,
                                         int32_t variant, void* stream)
{
    if (!pl) return fail(BMPC_ERR_INVALID_ARG, "plan is NULL");
    if (!A || !B || !c || !Q || !R || !M || !q || !r || !x0 || !x || !u || !lam)
        return fail(BMPC_ERR_INVALID_ARG, "NULL input or output array");
    const size_t N = pl->tree->h.N, n = pl->nx, m = pl->nu;
    // input arrays and their sizes in doubles, in staging order
    const double* in[8] = {A, B, c, Q, R, M, q, r};
    const size_t in_len[8] = {N * n * n, N * n * m, N * n, N * n * n, N * m * m, N * m * n, N * n, N * m};
    size_t in_total = 0;
    for (size_t len : in_len) in_total += len;
    const size_t out_len[3] = {N * n, N * m, N * n};
    const size_t total = in_total + n + out_len[0] + out_len[1] + out_len[2];
    if (!pl->stage_host) {
        if (hipHostMalloc((void**)&pl->stage_host, sizeof(double) * total, hipHostMallocDefault) != hipSuccess) {
            pl->stage_host = nullptr;
            return fail(BMPC_ERR_OOM, "pinned staging block of %zu bytes failed", sizeof(double) * total);
        }
        if (hipMalloc((void**)&pl->stage_dev, sizeof(double) * total) != hipSuccess) {
            (void)hipHostFree(pl->stage_host);
            pl->stage_host = nullptr;
            pl->stage_dev = nullptr;
            return fail(BMPC_ERR_OOM, "device staging block of %zu bytes failed", sizeof(double) * total);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    // the previous call on this plan has finished with the pinned block:
    // every call ends with a stream synchronisation
    double* h = pl->stage_host;
    const double* d_in[8];
    size_t off = 0;
    for (int i = 0; i < 8; ++i) {
        std::memcpy(h + off, in[i], sizeof(double) * in_len[i]);
        d_in[i] = pl->stage_dev + off;
        off += in_len[i];
    }
    std::memcpy(h + off, x0, sizeof(double) * n);
    const double* d_x0 = pl->stage_dev + off;
    off += n;
    const size_t out_off = off;
    double* d_out[3];
    for (int i = 0; i < 3; ++i) {
        d_out[i] = pl->stage_dev + off;
        off += out_len[i];
    }
    BMPC_HIP_TRY(hipMemcpyAsync(pl->stage_dev, h, sizeof(double) * out_off, hipMemcpyHostToDevice, s));
    bmpc_status st = bmpc_lqr_solve(pl, d_in[0], d_in[1], d_in[2], d_in[3], d_in[4], d_in[5], d_in[6], d_in[7], d_x0,
                                    d_out[0], d_out[1], d_out[2], nullptr, nullptr, nullptr, nullptr, variant, s);
    if (st != BMPC_OK) {
        (void)hipStreamSynchronize(s);
        return st;
    }
    BMPC_HIP_TRY(hipMemcpyAsync(h + out_off, pl->stage_dev + out_off, sizeof(double) * (total - out_off),
                                hipMemcpyDeviceToHost, s));
    BMPC_HIP_TRY(hipStreamSynchronize(s));
    double* out[3] = {x, u, lam};
    off = out_off;
    for (int i = 0; i < 3; ++i) {
        std::memcpy(out[i], h + off, sizeof(double) * out_len[i]);
        off += out_len[i];
    }
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_lqr_solve_f32(bmpc_lqr_plan* pl, const float* A, const float* B, const float* c,
                                        const float* Q, const float* R, const float* M, const float* q,
                                        const float* r, const float* x0, float* x, float* u, float* lam, float* K,
                                        float* k, float* P, float* p, void* stream)
{
    if (!pl) return fail(BMPC_ERR_INVALID_ARG, "plan is NULL");
    if (!A || !B || !c || !Q || !R || !M || !q || !r || !x0 || !x || !u || !lam)
        return fail(BMPC_ERR_INVALID_ARG, "NULL input or output array");
    if (!pl->kern->bwd_lane32)
        return fail(BMPC_ERR_UNSUPPORTED, "no FP32 tree-LQR kernel compiled for nx=%d nu=%d", pl->nx, pl->nu);
    bmpc_status st = ensure_f32(pl, false);
    if (st != BMPC_OK) return st;
    LqrArgsT<float> a{A, B, c, Q, R, M, q, r, x0, x, u, lam, K ? K : pl->K32, k ? k : pl->k32,
                      P ? P : pl->P32, p ? p : pl->p32, pl->bad, pl->bad + 1};
    launch_f32(pl, a, (hipStream_t)stream);
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_lqr_solve_mixed(bmpc_lqr_plan* pl, const double* A, const double* B, const double* c,
                                          const double* Q, const double* R, const double* M, const double* q,
                                          const double* r, const double* x0, double* x, double* u, double* lam,
                                          int32_t refine_steps, double* res_norms, void* stream)
{
    if (!pl) return fail(BMPC_ERR_INVALID_ARG, "plan is NULL");
    if (!A || !B || !c || !Q || !R || !M || !q || !r || !x0 || !x || !u || !lam)
        return fail(BMPC_ERR_INVALID_ARG, "NULL input or output array");
    if (refine_steps < 0 || refine_steps > BMPC_LQR_REFINE_MAX)
        return fail(BMPC_ERR_INVALID_ARG, "refine_steps %d outside [0, %d]", refine_steps, BMPC_LQR_REFINE_MAX);
    if (!pl->kern->bwd_lane32)
        return fail(BMPC_ERR_UNSUPPORTED, "no FP32 tree-LQR kernel compiled for nx=%d nu=%d", pl->nx, pl->nu);
    bmpc_status st = ensure_f32(pl, true);
    if (st != BMPC_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const TreeDev& t = pl->tree->d;
    const long N = t.N, n = pl->nx, m = pl->nu;
    {
        ProfScope ps("lqr_matrices_to_f32", s);
        const std::pair<const double*, float*> mats[] = {
            {A, pl->A32}, {B, pl->B32}, {Q, pl->Q32}, {R, pl->R32}, {M, pl->M32}};
        const long sizes[] = {N * n * n, N * n * m, N * n * n, N * m * m, N * m * n};
        for (int i = 0; i < 5; ++i)
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(sizes[i], 256)), dim3(256), 0, s, mats[i].first,
                               mats[i].second, sizes[i]);
    }
    auto* norms = reinterpret_cast<unsigned long long*>(res_norms);
    if (norms) hipLaunchKernelGGL(k_zero_norms, dim3(1), dim3(128), 0, s, norms, refine_steps + 2);
    const LqrArgs a64{A, B, c, Q, R, M, q, r, x0, x, u, lam, nullptr, nullptr, nullptr, nullptr, pl->bad, pl->bad + 1};
    const LqrArgsT<float> a32{pl->A32, pl->B32, pl->c32, pl->Q32, pl->R32, pl->M32, pl->q32, pl->r32,
                              pl->x032, pl->x32, pl->u32, pl->l32, pl->K32, pl->k32, pl->P32, pl->p32,
                              pl->bad, pl->bad + 1};
    const unsigned rgrid = (unsigned)((N * n + 255) / 256), ugrid = (unsigned)((std::max(n, m) * N + 255) / 256);
    for (int it = 0; it <= refine_steps + 1; ++it) {
        unsigned long long* slot = norms ? norms + it : nullptr;
        if (it == refine_steps + 1 && !slot) break;
        {
            ProfScope ps("lqr_residual_f64", s);
            hipLaunchKernelGGL(it == 0 ? pl->kern->residual_first : pl->kern->residual, dim3(rgrid), dim3(256), 0,
                               s, t, a64, pl->q32, pl->r32, pl->c32, pl->x032, slot);
        }
        if (it == refine_steps + 1) break;
        launch_f32(pl, a32, s);
        {
            ProfScope ps("lqr_refine_update", s);
            if (it == 0)
                hipLaunchKernelGGL(k_lqr_update<true>, dim3(ugrid), dim3(256), 0, s, N * n, N * m, x, u, lam,
                                   pl->x32, pl->u32, pl->l32);
            else
                hipLaunchKernelGGL(k_lqr_update<false>, dim3(ugrid), dim3(256), 0, s, N * n, N * m, x, u, lam,
                                   pl->x32, pl->u32, pl->l32);
        }
    }
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_lqr_check(bmpc_lqr_plan* pl, int32_t* bad_node, void* stream)
{
    if (!pl) return fail(BMPC_ERR_INVALID_ARG, "plan is NULL");
    BMPC_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int bad = 0;
    BMPC_HIP_TRY(hipMemcpy(&bad, pl->bad + 1, sizeof(int), hipMemcpyDeviceToHost));
    if (bad_node) *bad_node = bad == INT_MAX ? -1 : bad;
    if (bad != INT_MAX)
        return fail(BMPC_ERR_NOT_PD, "Riccati Hessian not positive definite at node %d", bad);
    return BMPC_OK;
}

}  // extern "C"
