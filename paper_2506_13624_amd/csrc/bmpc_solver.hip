// Branch-MPC solver: augmented-Lagrangian multiple-shooting iLQR (Sec. IV,
// Alg. 1) on a trajectory tree, one workgroup per problem instance.
//
// The whole iteration runs on the device.  Inner loop (Sec. IV-A): linearise
// the dynamics and quadratise the augmented objective (eq. AL, Gauss-Newton
// Hessian) around the current tree, solve the tree LQR (eq. tree_Riccati /
// tree_feedback_laws, level by level with an exact merge at branching
// nodes), roll the deviations out linearly, choose the merit penalty mu so
// that the merit slope is sufficiently negative, evaluate the merit (eq.
// merit) for every step size of the set in parallel and take the largest
// one with sufficient decrease (eq. sufficient_decrease).  The loop stops
// when the KKT residual is below omega.  Outer loop (Sec. IV-B): constraint
// violation, then either the multiplier update or a larger penalty, and the
// tolerance schedule.
//
// Node-parallel passes give one node per thread (strided); level passes
// walk the stages with a workgroup barrier per stage.  Sums are reduced
// with a fixed butterfly per wavefront and a fixed-order sum over
// wavefronts, so results are bitwise reproducible.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <map>
#include <mutex>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "bmpc_device.hpp"
#include "bmpc_hess_device.hpp"
#include "bmpc_internal.hpp"
#include "lqr_device.hpp"
#include "cvf_device.hpp"
#include "profile.hpp"

namespace bmpc {

constexpr int NALPHA_MAX = 12;
constexpr int LS_ROUNDS_MAX = 8;

// Workspace arrays per instance (node-major, doubles per node)
enum WsOff : int {
    W_FX = 0,          // 4: f(x_n, u_n)
    W_A = 4,           // 16: dF/dx at (x_n, u_n), shared by all out-edges of n
    W_B = 20,          // 8: dF/du
    W_C = 28,          // 4: defect of the edge into n: f(x_p, u_p) - x_n
    W_Q = 32,          // 16
    W_R = 48,          // 4
    W_QV = 52,         // 4: q
    W_RV = 56,         // 2: r
    W_K = 58,          // 8
    W_KV = 66,         // 2: k
    W_P = 68,          // 16
    W_PV = 84,         // 4: p
    W_DX = 88,         // 4
    W_DU = 92,         // 2
    W_LH = 94,         // 4: LQR costates
    W_S0 = 98,         // 56: conditional value function (A, c, C, P, p), scan buffer 0
    W_S1 = 154,        // 56: scan buffer 1
    W_M = 210,         // 8: cross block d2/du dx of the model (zero for Gauss-Newton)
    W_NODE = 218
};

struct InstDesc {
    int N, T;
    const int* parent;
    const int* child_off;
    const int* level_off;
    const double* weight;  // N
    const double* ref;     // N x 4
    const double* obs;     // N x 2
    const int* has_obs;    // N
    const double* x0;      // 4
    BikeParams prm;
    double* x;    // N x 4
    double* u;    // N x 2
    double* lam;  // N x 4
    double* ye;   // N x 5
    double* ws;   // N x W_NODE
    // maximal unbranched segments (segment-scan variant)
    const int* seg_of;
    const int* seg_pos;
    const int* seg_len;
    const int* seg_nodes;
    const int* seg_off;
    const int* seg_end;
    const int* seg_depth;
    int max_seg_len, max_seg_depth;
};

struct SolverCfg {
    double eps_tol, tau, omega0, eta0, a_omega, b_omega, a_eta, b_eta, rho0, mu0, beta;
    int n_alpha, max_outer, max_inner, max_ls_fail, max_total, ls_rounds;
    int warm;  // bits: 1 x,u given, 2 lam given, 4 ye given, 8 u given (x rolled out), 16 guarded
    int hess;  // 0 Gauss-Newton, 1 exact Hessian with eigenvalue modification
    double eig_floor;
};

// Phases of an inner iteration whose time the solver accumulates
enum Phase : int { PH_LINEARISE = 0, PH_BACKWARD, PH_FORWARD, PH_LINESEARCH, PH_UPDATE, PH_COUNT };

struct SolveOut {
    int status, outer_it, inner_it, ls_failures, bad_node, start;
    double r_kkt, viol, rho, mu, merit;
    unsigned long long ticks[PH_COUNT];  // constant-rate clock ticks per phase, summed over the solve
};

// Phase clock: the constant-rate device counter, read by the team's first
// thread only (the others get 0, so their sums are unused and cheap).
struct PhaseClock {
    unsigned long long t = 0, acc[PH_COUNT] = {};
    __device__ void start(bool on) { if (on) t = wall_clock64(); }
    __device__ void lap(bool on, int ph)
    {
        if (on) {
            const unsigned long long now = wall_clock64();
            acc[ph] += now - t;
            t = now;
        }
    }
};

__device__ __forceinline__ void load4(const double* p, double (&v)[4])
{
    v[0] = p[0]; v[1] = p[1]; v[2] = p[2]; v[3] = p[3];
}
__device__ __forceinline__ void store4(double* p, const double (&v)[4])
{
    p[0] = v[0]; p[1] = v[1]; p[2] = v[2]; p[3] = v[3];
}

__device__ __forceinline__ NodeData node_data(const InstDesc& I, int n)
{
    NodeData d;
    d.w = I.weight[n];
#pragma unroll
    for (int i = 0; i < BX; ++i) d.ref[i] = I.ref[n * 4 + i];
    d.ox = I.obs[n * 2];
    d.oy = I.obs[n * 2 + 1];
    d.has_obs = I.has_obs[n] != 0;
    d.leaf = I.child_off[n] == I.child_off[n + 1];
    return d;
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = (v != v || o != o) ? NAN : fmax(v, o);
    }
    return v;
}

// Sum (or max) K values over the workgroup; every thread gets the totals.
template <int BS, int K, bool MAX>
__device__ __forceinline__ void block_reduce(double (&v)[K], double* sred)
{
    constexpr int NW = BS / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = MAX ? wave_max(v[k]) : wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sred[k * NW + w] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double t = sred[k * NW];
        for (int i = 1; i < NW; ++i) {
            const double o = sred[k * NW + i];
            t = MAX ? ((t != t || o != o) ? NAN : fmax(t, o)) : t + o;
        }
        v[k] = t;
    }
    __syncthreads();
}

// Teams of threads that run the solver passes: one workgroup (one problem
// per workgroup, the batched solver) or the whole grid (one large problem;
// cooperative launch, so every workgroup is resident and grid-wide
// synchronisation is safe).  Reductions are deterministic in both: the grid
// team combines the per-workgroup results in workgroup order.
template <int BS_>
struct TeamWG {
    static constexpr int BS = BS_;
    static constexpr bool kGrid = false;
    __device__ static int rank() { return threadIdx.x; }
    __device__ static int size() { return BS_; }
    __device__ static void sync() { __syncthreads(); }
    template <int K, bool MAX>
    __device__ static void reduce(double (&v)[K], double* sred, double*)
    {
        block_reduce<BS_, K, MAX>(v, sred);
    }
};

template <int BS_>
struct TeamGrid {
    static constexpr int BS = BS_;
    static constexpr bool kGrid = true;
    __device__ static int rank() { return blockIdx.x * BS_ + threadIdx.x; }
    // a rank whose neighbours are in different workgroups: work that falls
    // on a contiguous range of node ids (one stage of the tree) is spread
    // over all CUs instead of a few
    __device__ static int rank_spread() { return threadIdx.x * gridDim.x + blockIdx.x; }
    __device__ static int size() { return gridDim.x * BS_; }
    __device__ static void sync() { cooperative_groups::this_grid().sync(); }
    // gpart: gridDim.x x K doubles of device memory
    template <int K, bool MAX>
    __device__ static void reduce(double (&v)[K], double* sred, double* gpart)
    {
        block_reduce<BS_, K, MAX>(v, sred);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < K; ++k) gpart[(long)blockIdx.x * K + k] = v[k];
        sync();
        // every workgroup combines the per-workgroup results the same way:
        // thread t takes workgroups t, t + BS, ... in order, then the
        // workgroup's fixed reduction tree; so all of them hold the same
        // value, and no thread walks all workgroups alone
        double w[K];
#pragma unroll
        for (int k = 0; k < K; ++k) w[k] = MAX ? -INFINITY : 0.0;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += BS_) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double o = gpart[(long)b * K + k];
                w[k] = MAX ? ((w[k] != w[k] || o != o) ? NAN : fmax(w[k], o)) : w[k] + o;
            }
        }
        block_reduce<BS_, K, MAX>(w, sred);
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = w[k];
        sync();  // partials may be overwritten by the next reduction
    }
};

// ---------------------------------------------------------------- passes
// Linearise dynamics, quadratise L_a; returns this thread's partial L_a and
// constraint violation.  hess = 1 replaces the Gauss-Newton Hessian blocks by
// the exact ones with eigenvalue modification (floor eig_floor), which
// take the children's multipliers.
template <class T>
__device__ void pass_linearise(const InstDesc& I, double rho, double& La, double& viol, int hess = 0,
                               double eig_floor = 0.0)
{
    La = 0.0;
    viol = 0.0;
    for (int n = T::rank(); n < I.N; n += T::size()) {
        const NodeData nd = node_data(I, n);
        double x[BX], u[BU], ye[BG];
        load4(I.x + n * 4, x);
        u[0] = I.u[n * 2];
        u[1] = I.u[n * 2 + 1];
#pragma unroll
        for (int s = 0; s < BG; ++s) ye[s] = I.ye[n * BG + s];
        double q[BX], r[BU], Qh[BX][BX], Rh[BU][BU], Mh[BU][BX] = {};
        La += node_quad(I.prm, nd, x, u, ye, rho, q, r, Qh, Rh);
        if (!nd.leaf && !steer_in_domain(u)) La = INFINITY;
        if (hess) {
            double mu[BX] = {0.0, 0.0, 0.0, 0.0};
            for (int j = I.child_off[n]; j < I.child_off[n + 1]; ++j)
#pragma unroll
                for (int i = 0; i < BX; ++i) mu[i] += I.lam[j * 4 + i];
            exact_node_model(I.prm, nd, x, u, ye, rho, mu, eig_floor, Qh, Rh, Mh);
        }
        double* w = I.ws + (long)n * W_NODE;
#pragma unroll
        for (int i = 0; i < BU; ++i)
#pragma unroll
            for (int j = 0; j < BX; ++j) w[W_M + i * 4 + j] = Mh[i][j];
#pragma unroll
        for (int i = 0; i < BX; ++i) {
            w[W_QV + i] = q[i];
#pragma unroll
            for (int j = 0; j < BX; ++j) w[W_Q + i * 4 + j] = Qh[i][j];
        }
#pragma unroll
        for (int i = 0; i < BU; ++i) {
            w[W_RV + i] = r[i];
#pragma unroll
            for (int j = 0; j < BU; ++j) w[W_R + i * 2 + j] = Rh[i][j];
        }
        double g[BG], dist, ex, ey;
        bool on[BG];
        node_constraints(I.prm, nd, x, u, g, on, dist, ex, ey);
#pragma unroll
        for (int s = 0; s < BG; ++s)
            if (on[s]) {
                const double c = fabs(fmax(g[s], -ye[s] / rho));
                viol = (viol != viol || c != c) ? NAN : fmax(viol, c);
            }
        double xn[BX] = {0.0, 0.0, 0.0, 0.0}, A[BX][BX] = {}, B[BX][BU] = {};
        if (!nd.leaf) bike_step_jac(I.prm, x, u, xn, A, B);
#pragma unroll
        for (int i = 0; i < BX; ++i) {
            w[W_FX + i] = xn[i];
#pragma unroll
            for (int j = 0; j < BX; ++j) w[W_A + i * 4 + j] = A[i][j];
#pragma unroll
            for (int j = 0; j < BU; ++j) w[W_B + i * 2 + j] = B[i][j];
        }
    }
}

// Defects and KKT residual (needs the linearisation of the parents):
// returns partial max residual and partial sums lam.d, |d|^2.
template <class T>
__device__ void pass_defects_kkt(const InstDesc& I, double& rk, double& ld, double& dd)
{
    rk = 0.0;
    ld = 0.0;
    dd = 0.0;
    for (int n = T::rank(); n < I.N; n += T::size()) {
        double* w = I.ws + (long)n * W_NODE;
        double lam[BX];
        load4(I.lam + n * 4, lam);
        if (n > 0) {
            const double* wp = I.ws + (long)I.parent[n] * W_NODE;
#pragma unroll
            for (int i = 0; i < BX; ++i) {
                const double d = wp[W_FX + i] - I.x[n * 4 + i];
                w[W_C + i] = d;
                ld += lam[i] * d;
                dd += d * d;
                rk = (rk != rk || d != d) ? NAN : fmax(rk, fabs(d));
            }
        } else {
#pragma unroll
            for (int i = 0; i < BX; ++i) w[W_C + i] = 0.0;
        }
        const int c0 = I.child_off[n], c1 = I.child_off[n + 1];
        double s[BX] = {0.0, 0.0, 0.0, 0.0};
        for (int j = c0; j < c1; ++j)
#pragma unroll
            for (int i = 0; i < BX; ++i) s[i] += I.lam[j * 4 + i];
        if (n > 0) {
#pragma unroll
            for (int i = 0; i < BX; ++i) {
                double gx = w[W_QV + i] - lam[i];
                if (c1 > c0)
#pragma unroll
                    for (int k = 0; k < BX; ++k) gx += w[W_A + k * 4 + i] * s[k];
                rk = (rk != rk || gx != gx) ? NAN : fmax(rk, fabs(gx));
            }
        }
        if (c1 > c0) {
#pragma unroll
            for (int i = 0; i < BU; ++i) {
                double gu = w[W_RV + i];
#pragma unroll
                for (int k = 0; k < BX; ++k) gu += w[W_B + k * 2 + i] * s[k];
                rk = (rk != rk || gu != gu) ? NAN : fmax(rk, fabs(gu));
            }
        }
    }
}

// Backward tree Riccati, one stage per barrier.  Returns false (and sets
// *bad) if some H_n is not positive definite.
// One node of the backward pass: gains and value function from its stage
// data and its children's value functions (workspace rows).
__device__ __forceinline__ void ric_node_ws(const InstDesc& I, int n, int* bad)
{
    double* w = I.ws + (long)n * W_NODE;
    const int c0 = I.child_off[n], c1 = I.child_off[n + 1];
    if (c0 == c1) {
#pragma unroll
        for (int e = 0; e < 16; ++e) w[W_P + e] = w[W_Q + e];
#pragma unroll
        for (int e = 0; e < 4; ++e) w[W_PV + e] = w[W_QV + e];
        return;
    }
    StageRegs<BX, BU> st;
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) st.Q[i][j] = w[W_Q + i * 4 + j];
        st.q[i] = w[W_QV + i];
    }
#pragma unroll
    for (int i = 0; i < BU; ++i) {
#pragma unroll
        for (int j = 0; j < BU; ++j) st.R[i][j] = w[W_R + i * 2 + j];
#pragma unroll
        for (int j = 0; j < BX; ++j) st.M[i][j] = w[W_M + i * 4 + j];
        st.r[i] = w[W_RV + i];
    }
    RicAcc<BX, BU> acc;
    acc.init(st);
    EdgeRegs<BX, BU> ed;
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) ed.A[i][j] = w[W_A + i * 4 + j];
#pragma unroll
        for (int j = 0; j < BU; ++j) ed.B[i][j] = w[W_B + i * 2 + j];
    }
    for (int j = c0; j < c1; ++j) {
        const double* wj = I.ws + (long)j * W_NODE;
        double P[BX][BX], p[BX];
#pragma unroll
        for (int i = 0; i < BX; ++i) {
#pragma unroll
            for (int k = 0; k < BX; ++k) P[i][k] = wj[W_P + i * 4 + k];
            p[i] = wj[W_PV + i];
            ed.c[i] = wj[W_C + i];
        }
        acc.add_child(ed, P, p);
    }
    double K[BU][BX], k[BU], P[BX][BX], p[BX];
    if (!acc.finish(K, k, P, p)) atomicMin(bad, n);
#pragma unroll
    for (int i = 0; i < BU; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) w[W_K + i * 4 + j] = K[i][j];
        w[W_KV + i] = k[i];
    }
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) w[W_P + i * 4 + j] = P[i][j];
        w[W_PV + i] = p[i];
    }
}

template <class T>
__device__ void pass_riccati(const InstDesc& I, int* bad)
{
    for (int t = I.T; t >= 0; --t) {
        const int n0 = I.level_off[t], n1 = I.level_off[t + 1];
        for (int n = n0 + T::rank(); n < n1; n += T::size()) ric_node_ws(I, n, bad);
        T::sync();
    }
}

// The same backward pass by segment depth: one thread walks a maximal
// unbranched segment from its bottom node (a leaf, or a branching node
// whose children start deeper segments, done in an earlier round) up to
// its top, so a round of the whole team covers a segment depth instead
// of a stage: on a tree that branches every few stages far fewer team
// barriers, and the same operations per node, so the same results.
template <class T>
__device__ void pass_riccati_seg(const InstDesc& I, int* bad)
{
    for (int d = I.max_seg_depth; d >= 0; --d) {
        for (int n = T::rank_spread(); n < I.N; n += T::size()) {
            const int s = I.seg_of[n];
            if (I.seg_end[s] != n || I.seg_depth[s] != d) continue;
            const int top = I.seg_nodes[I.seg_off[s]];
            for (int m = n;; m = I.parent[m]) {
                ric_node_ws(I, m, bad);
                if (m == top) break;
            }
        }
        T::sync();
    }
}

// ---------------------------------------------------------------- segment scan
__device__ __forceinline__ void cvf_load(const double* w, Cvf<BX>& e)
{
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) {
            e.A[i][j] = w[i * 4 + j];
            e.C[i][j] = w[20 + i * 4 + j];
            e.P[i][j] = w[36 + i * 4 + j];
        }
        e.c[i] = w[16 + i];
        e.p[i] = w[52 + i];
    }
}
__device__ __forceinline__ void cvf_store(double* w, const Cvf<BX>& e)
{
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) {
            w[i * 4 + j] = e.A[i][j];
            w[20 + i * 4 + j] = e.C[i][j];
            w[36 + i * 4 + j] = e.P[i][j];
        }
        w[16 + i] = e.c[i];
        w[52 + i] = e.p[i];
    }
}

__device__ __forceinline__ void stage_from_ws(const double* w, StageRegs<BX, BU>& st)
{
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) st.Q[i][j] = w[W_Q + i * 4 + j];
        st.q[i] = w[W_QV + i];
    }
#pragma unroll
    for (int i = 0; i < BU; ++i) {
#pragma unroll
        for (int j = 0; j < BU; ++j) st.R[i][j] = w[W_R + i * 2 + j];
#pragma unroll
        for (int j = 0; j < BX; ++j) st.M[i][j] = w[W_M + i * 4 + j];
        st.r[i] = w[W_RV + i];
    }
}

__device__ __forceinline__ void edge_from_ws(const double* w, const double* wj, EdgeRegs<BX, BU>& ed)
{
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) ed.A[i][j] = w[W_A + i * 4 + j];
#pragma unroll
        for (int j = 0; j < BU; ++j) ed.B[i][j] = w[W_B + i * 2 + j];
        ed.c[i] = wj[W_C + i];
    }
}

// Riccati merge at node n over all its children (children's P, p ready);
// stores K, k, P, p of n.  Leaves: P = Q, p = q.
__device__ __forceinline__ void riccati_merge_ws(const InstDesc& I, int n, int* bad)
{
    double* w = I.ws + (long)n * W_NODE;
    const int c0 = I.child_off[n], c1 = I.child_off[n + 1];
    if (c0 == c1) {
#pragma unroll
        for (int e = 0; e < 16; ++e) w[W_P + e] = w[W_Q + e];
#pragma unroll
        for (int e = 0; e < 4; ++e) w[W_PV + e] = w[W_QV + e];
        return;
    }
    StageRegs<BX, BU> st;
    stage_from_ws(w, st);
    RicAcc<BX, BU> acc;
    acc.init(st);
    for (int j = c0; j < c1; ++j) {
        const double* wj = I.ws + (long)j * W_NODE;
        EdgeRegs<BX, BU> ed;
        edge_from_ws(w, wj, ed);
        double P[BX][BX], p[BX];
#pragma unroll
        for (int i = 0; i < BX; ++i) {
#pragma unroll
            for (int k = 0; k < BX; ++k) P[i][k] = wj[W_P + i * 4 + k];
            p[i] = wj[W_PV + i];
        }
        acc.add_child(ed, P, p);
    }
    double K[BU][BX], k[BU], P[BX][BX], p[BX];
    if (!acc.finish(K, k, P, p)) atomicMin(bad, n);
#pragma unroll
    for (int i = 0; i < BU; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) w[W_K + i * 4 + j] = K[i][j];
        w[W_KV + i] = k[i];
    }
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) w[W_P + i * 4 + j] = P[i][j];
        w[W_PV + i] = p[i];
    }
}

// Log-depth backward pass: conditional value functions are composed along
// every maximal unbranched segment by a Hillis-Steele suffix scan; branching
// nodes are merged exactly (deepest segments first); then every segment
// node gets its value function by composing its suffix with the value
// function of the segment's end, and its gains from its child's value
// function (eq. feedback_laws).
template <int BS>
__device__ void pass_riccati_segscan(const InstDesc& I, int* bad)
{
    const int N = I.N;
    for (int n = threadIdx.x; n < N; n += BS) {
        if (I.child_off[n + 1] - I.child_off[n] != 1) continue;
        const double* w = I.ws + (long)n * W_NODE;
        const double* wj = I.ws + (long)I.child_off[n] * W_NODE;
        StageRegs<BX, BU> st;
        stage_from_ws(w, st);
        EdgeRegs<BX, BU> ed;
        edge_from_ws(w, wj, ed);
        Cvf<BX> e;
        if (!cvf_element<BX, BU>(st.Q, st.R, st.M, st.q, st.r, ed.A, ed.B, ed.c, e)) atomicMin(bad, n);
        cvf_store(I.ws + (long)n * W_NODE + W_S0, e);
    }
    __syncthreads();
    int src = W_S0, dst = W_S1;
    for (int span = 1; span < I.max_seg_len - 1; span <<= 1) {
        for (int n = threadIdx.x; n < N; n += BS) {
            if (I.child_off[n + 1] - I.child_off[n] != 1) continue;
            const int s = I.seg_of[n], pos = I.seg_pos[n], len = I.seg_len[s];
            Cvf<BX> a;
            cvf_load(I.ws + (long)n * W_NODE + src, a);
            if (pos + span < len - 1) {
                const int partner = I.seg_nodes[I.seg_off[s] + pos + span];
                Cvf<BX> b, o;
                cvf_load(I.ws + (long)partner * W_NODE + src, b);
                cvf_combine<BX>(a, b, o);
                cvf_store(I.ws + (long)n * W_NODE + dst, o);
            } else {
                cvf_store(I.ws + (long)n * W_NODE + dst, a);
            }
        }
        __syncthreads();
        const int t = src;
        src = dst;
        dst = t;
    }
    for (int d = I.max_seg_depth; d >= 0; --d) {
        for (int n = threadIdx.x; n < N; n += BS) {
            const int s = I.seg_of[n];
            if (I.seg_depth[s] == d && I.seg_end[s] == n) riccati_merge_ws(I, n, bad);
        }
        __syncthreads();
        for (int n = threadIdx.x; n < N; n += BS) {
            const int s = I.seg_of[n];
            if (I.seg_depth[s] != d || I.child_off[n + 1] - I.child_off[n] != 1) continue;
            const double* we = I.ws + (long)I.seg_end[s] * W_NODE;
            double Pv[BX][BX], pv[BX], P[BX][BX], p[BX];
#pragma unroll
            for (int i = 0; i < BX; ++i) {
#pragma unroll
                for (int k = 0; k < BX; ++k) Pv[i][k] = we[W_P + i * 4 + k];
                pv[i] = we[W_PV + i];
            }
            Cvf<BX> a;
            cvf_load(I.ws + (long)n * W_NODE + src, a);
            cvf_apply_value<BX>(a, Pv, pv, P, p);
            double* w = I.ws + (long)n * W_NODE;
#pragma unroll
            for (int i = 0; i < BX; ++i) {
#pragma unroll
                for (int k = 0; k < BX; ++k) w[W_P + i * 4 + k] = P[i][k];
                w[W_PV + i] = p[i];
            }
        }
        __syncthreads();
    }
    // gains of the segment nodes from their only child's value function
    for (int n = threadIdx.x; n < N; n += BS) {
        if (I.child_off[n + 1] - I.child_off[n] != 1) continue;
        double* w = I.ws + (long)n * W_NODE;
        const double* wj = I.ws + (long)I.child_off[n] * W_NODE;
        StageRegs<BX, BU> st;
        stage_from_ws(w, st);
        EdgeRegs<BX, BU> ed;
        edge_from_ws(w, wj, ed);
        double Pc[BX][BX], pc[BX];
#pragma unroll
        for (int i = 0; i < BX; ++i) {
#pragma unroll
            for (int k = 0; k < BX; ++k) Pc[i][k] = wj[W_P + i * 4 + k];
            pc[i] = wj[W_PV + i];
        }
        RicAcc<BX, BU> acc;
        acc.init(st);
        acc.add_child(ed, Pc, pc);
        double K[BU][BX], k[BU], P[BX][BX], p[BX];
        if (!acc.finish(K, k, P, p)) atomicMin(bad, n);
#pragma unroll
        for (int i = 0; i < BU; ++i) {
#pragma unroll
            for (int j = 0; j < BX; ++j) w[W_K + i * 4 + j] = K[i][j];
            w[W_KV + i] = k[i];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- LDS passes
// For problems whose per-node chain values fit in LDS, the stage-by-stage
// backward and forward passes keep the values that flow from one stage to
// the next there (P, p and defect c per node for the backward pass; dx for
// the forward pass) and fetch each thread's inputs for the next stage from
// HBM while the current stage is computed.  Same arithmetic as the passes
// above, so the same results bit for bit.  Each row also holds the node's
// child range, written once per problem, so that a stage reads no topology
// from global memory, and the forward pass's control step, so that a stage
// writes no global memory either (the results of either pass go to the
// workspace in one sweep over all nodes after it).  The backward pass keeps
// the gains K (8) and k (2) in four slots of their own plus the dx and du
// slots, which the forward pass fills only after that sweep.
constexpr int LN = 35;  // doubles per node: P 16, p 4, c 4, dx 4, child range, du 2, gains 4
constexpr int LN_P = 0, LN_PV = 16, LN_C = 20, LN_DX = 24, LN_CH = 28, LN_DU = 29, LN_G = 31;
// LDS slot of gain entry e (K row-major, then k)
__device__ __forceinline__ constexpr int lds_gain_slot(int e)
{
    return e < 4 ? LN_G + e : (e < 8 ? LN_DX + e - 4 : LN_DU + e - 8);
}

// child range [first, end) of node n, as kept in its LDS row
__device__ __forceinline__ int2 lds_children(const double* sn, int n)
{
    return *reinterpret_cast<const int2*>(sn + (long)n * LN + LN_CH);
}

template <class T>
__device__ void lds_topology(const InstDesc& I, double* sn)
{
    for (int n = T::rank(); n < I.N; n += T::size())
        *reinterpret_cast<int2*>(sn + (long)n * LN + LN_CH) = make_int2(I.child_off[n], I.child_off[n + 1]);
    T::sync();
}

// After a backward pass that left the value functions in the workspace (the
// segment scan): copy P, p and the defect c of every node into its LDS row,
// all nodes at once, for the LDS forward pass.
template <int BS>
__device__ void lds_from_ws(const InstDesc& I, double* sn)
{
    for (int n = threadIdx.x; n < I.N; n += BS) {
        const double* w = I.ws + (long)n * W_NODE;
        double* me = sn + (long)n * LN;
#pragma unroll
        for (int e = 0; e < BX * BX; ++e) me[LN_P + e] = w[W_P + e];
#pragma unroll
        for (int i = 0; i < BX; ++i) {
            me[LN_PV + i] = w[W_PV + i];
            me[LN_C + i] = w[W_C + i];
        }
    }
    __syncthreads();
}

struct RicPre {
    StageRegs<BX, BU> st;
    double A[BX][BX], B[BX][BU];
};

__device__ __forceinline__ void ric_fetch(const InstDesc& I, int n, RicPre& r)
{
    const double* w = I.ws + (long)n * W_NODE;
    stage_from_ws(w, r.st);
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) r.A[i][j] = w[W_A + i * 4 + j];
#pragma unroll
        for (int j = 0; j < BU; ++j) r.B[i][j] = w[W_B + i * 2 + j];
    }
}

__device__ __forceinline__ void ric_node_lds(const InstDesc& I, int n, const RicPre& r, double* sn, int* bad)
{
    double* me = sn + (long)n * LN;
    const int2 ch = lds_children(sn, n);
    const int c0 = ch.x, c1 = ch.y;
    if (c0 == c1) {
#pragma unroll
        for (int i = 0; i < BX; ++i) {
#pragma unroll
            for (int j = 0; j < BX; ++j) me[LN_P + i * 4 + j] = r.st.Q[i][j];
            me[LN_PV + i] = r.st.q[i];
        }
        return;
    }
    RicAcc<BX, BU> acc;
    acc.init(r.st);
    EdgeRegs<BX, BU> ed;
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) ed.A[i][j] = r.A[i][j];
#pragma unroll
        for (int j = 0; j < BU; ++j) ed.B[i][j] = r.B[i][j];
    }
    for (int j = c0; j < c1; ++j) {
        const double* cj = sn + (long)j * LN;
        double P[BX][BX], p[BX];
#pragma unroll
        for (int i = 0; i < BX; ++i) {
#pragma unroll
            for (int k = 0; k < BX; ++k) P[i][k] = cj[LN_P + i * 4 + k];
            p[i] = cj[LN_PV + i];
            ed.c[i] = cj[LN_C + i];
        }
        acc.add_child(ed, P, p);
    }
    double K[BU][BX], k[BU], P[BX][BX], p[BX];
    if (!acc.finish(K, k, P, p)) atomicMin(bad, n);
#pragma unroll
    for (int i = 0; i < BU; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) me[lds_gain_slot(i * 4 + j)] = K[i][j];
        me[lds_gain_slot(8 + i)] = k[i];
    }
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) me[LN_P + i * 4 + j] = P[i][j];
        me[LN_PV + i] = p[i];
    }
}

// Workgroup barrier that orders LDS only: it waits for this wave's LDS
// operations but not for its outstanding global loads, so the next stage's
// inputs stay in flight across it.  (A full __syncthreads() would drain
// them.)  Used only where threads exchange data through LDS.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int BS>
__device__ void pass_riccati_lds(const InstDesc& I, int* bad, double* sn)
{
    for (int n = threadIdx.x; n < I.N; n += BS) {
        const double* w = I.ws + (long)n * W_NODE;
#pragma unroll
        for (int i = 0; i < BX; ++i) sn[(long)n * LN + LN_C + i] = w[W_C + i];
    }
    __syncthreads();
    for (int t = I.T; t >= 0; --t) {
        const int n0 = I.level_off[t], n1 = I.level_off[t + 1];
        for (int n = n0 + (int)threadIdx.x; n < n1; n += BS) {
            RicPre r;
            ric_fetch(I, n, r);
            ric_node_lds(I, n, r, sn, bad);
        }
        lds_barrier();
    }
    __syncthreads();
    // gains to the workspace, where the forward pass fetches them
    for (int n = threadIdx.x; n < I.N; n += BS) {
        const int2 ch = lds_children(sn, n);
        if (ch.x == ch.y) continue;
        const double* me = sn + (long)n * LN;
        double* w = I.ws + (long)n * W_NODE;
#pragma unroll
        for (int e = 0; e < 8; ++e) w[W_K + e] = me[lds_gain_slot(e)];
        w[W_KV] = me[lds_gain_slot(8)];
        w[W_KV + 1] = me[lds_gain_slot(9)];
    }
    __syncthreads();
}

struct FwdPre {
    double K[BU][BX], k[BU], A[BX][BX], B[BX][BU];
};

__device__ __forceinline__ void fwd_fetch(const InstDesc& I, int n, FwdPre& r)
{
    const double* w = I.ws + (long)n * W_NODE;
#pragma unroll
    for (int i = 0; i < BU; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) r.K[i][j] = w[W_K + i * 4 + j];
        r.k[i] = w[W_KV + i];
    }
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) r.A[i][j] = w[W_A + i * 4 + j];
#pragma unroll
        for (int j = 0; j < BU; ++j) r.B[i][j] = w[W_B + i * 2 + j];
    }
}

__device__ __forceinline__ void fwd_node_lds(int n, const FwdPre& r, double* sn)
{
    double* me = sn + (long)n * LN;
    double dx[BX];
#pragma unroll
    for (int i = 0; i < BX; ++i) dx[i] = me[LN_DX + i];
    const int2 ch = lds_children(sn, n);
    const int c0 = ch.x, c1 = ch.y;
    double du[BU] = {0.0, 0.0};
    if (c1 > c0) {
#pragma unroll
        for (int i = 0; i < BU; ++i) {
            double acc = r.k[i];
#pragma unroll
            for (int j = 0; j < BX; ++j) acc += r.K[i][j] * dx[j];
            du[i] = acc;
        }
        for (int j = c0; j < c1; ++j) {
            double* cj = sn + (long)j * LN;
#pragma unroll
            for (int i = 0; i < BX; ++i) {
                double acc = cj[LN_C + i];
#pragma unroll
                for (int k = 0; k < BX; ++k) acc += r.A[i][k] * dx[k];
#pragma unroll
                for (int k = 0; k < BU; ++k) acc += r.B[i][k] * du[k];
                cj[LN_DX + i] = acc;
            }
        }
    }
    me[LN_DU] = du[0];
    me[LN_DU + 1] = du[1];
}

// Forward results of one node from its LDS row to the workspace: the LQR
// costate estimate P dx + p, dx and du.
__device__ __forceinline__ void fwd_store_lds(const InstDesc& I, int n, const double* sn)
{
    double* w = I.ws + (long)n * W_NODE;
    const double* me = sn + (long)n * LN;
    double dx[BX];
#pragma unroll
    for (int i = 0; i < BX; ++i) dx[i] = me[LN_DX + i];
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        double acc = me[LN_PV + i];
#pragma unroll
        for (int j = 0; j < BX; ++j) acc += me[LN_P + i * 4 + j] * dx[j];
        w[W_LH + i] = acc;
        w[W_DX + i] = dx[i];
    }
    w[W_DU] = me[LN_DU];
    w[W_DU + 1] = me[LN_DU + 1];
}

template <int BS>
__device__ void pass_forward_lds(const InstDesc& I, double* sn)
{
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < BX; ++i) sn[LN_DX + i] = 0.0;
    FwdPre buf[2];
    if (threadIdx.x == 0) fwd_fetch(I, 0, buf[0]);
    __syncthreads();
    auto stage = [&](int t, FwdPre& cur, FwdPre& nxt) {
        const int n0 = I.level_off[t], n1 = I.level_off[t + 1];
        const int n = n0 + (int)threadIdx.x;
        if (t < I.T) {
            const int m = n1 + (int)threadIdx.x;
            if (m < I.level_off[t + 2]) fwd_fetch(I, m, nxt);
        }
        if (n < n1) fwd_node_lds(n, cur, sn);
        for (int e = n + BS; e < n1; e += BS) {
            FwdPre r;
            fwd_fetch(I, e, r);
            fwd_node_lds(e, r, sn);
        }
        lds_barrier();
    };
    for (int t = 0; t <= I.T; t += 2) {
        stage(t, buf[0], buf[1]);
        if (t + 1 <= I.T) stage(t + 1, buf[1], buf[0]);
    }
    __syncthreads();
    for (int n = threadIdx.x; n < I.N; n += BS) fwd_store_lds(I, n, sn);
    __syncthreads();
}

// Forward linear rollout of the deviations (delta x_0 = 0) and the LQR
// costates lam_hat = P dx + p.
// One node of the forward pass: costate estimate, control step and the
// state steps of its children.
__device__ __forceinline__ void fwd_node_ws(const InstDesc& I, int n)
{
    double* w = I.ws + (long)n * W_NODE;
    double dx[BX];
    load4(w + W_DX, dx);
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        double acc = w[W_PV + i];
#pragma unroll
        for (int j = 0; j < BX; ++j) acc += w[W_P + i * 4 + j] * dx[j];
        w[W_LH + i] = acc;
    }
    const int c0 = I.child_off[n], c1 = I.child_off[n + 1];
    double du[BU] = {0.0, 0.0};
    if (c1 > c0) {
#pragma unroll
        for (int i = 0; i < BU; ++i) {
            double acc = w[W_KV + i];
#pragma unroll
            for (int j = 0; j < BX; ++j) acc += w[W_K + i * 4 + j] * dx[j];
            du[i] = acc;
        }
        for (int j = c0; j < c1; ++j) {
            double* wj = I.ws + (long)j * W_NODE;
#pragma unroll
            for (int i = 0; i < BX; ++i) {
                double acc = wj[W_C + i];
#pragma unroll
                for (int k = 0; k < BX; ++k) acc += w[W_A + i * 4 + k] * dx[k];
#pragma unroll
                for (int k = 0; k < BU; ++k) acc += w[W_B + i * 2 + k] * du[k];
                wj[W_DX + i] = acc;
            }
        }
    }
    w[W_DU] = du[0];
    w[W_DU + 1] = du[1];
}

template <class T>
__device__ void pass_forward(const InstDesc& I)
{
    if (T::rank() == 0)
#pragma unroll
        for (int i = 0; i < BX; ++i) I.ws[W_DX + i] = 0.0;
    T::sync();
    for (int t = 0; t <= I.T; ++t) {
        const int n0 = I.level_off[t], n1 = I.level_off[t + 1];
        for (int n = n0 + T::rank(); n < n1; n += T::size()) fwd_node_ws(I, n);
        T::sync();
    }
}

// The forward pass by segment depth: one thread walks a segment from its
// top down.  The walk keeps the state step in registers and has the next
// node's K, k, A, B and defect c in flight while a node is computed.  The
// costate estimates lam_hat = P dx + p, which nothing in the walk needs, are
// left to the caller's next node-parallel sweep (lam_hat_ws).  The same
// operations per node as fwd_node_ws, so the same results.
__device__ __forceinline__ void lam_hat_ws(const InstDesc& I, int n)
{
    double* w = I.ws + (long)n * W_NODE;
    double dx[BX];
    load4(w + W_DX, dx);
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        double acc = w[W_PV + i];
#pragma unroll
        for (int j = 0; j < BX; ++j) acc += w[W_P + i * 4 + j] * dx[j];
        w[W_LH + i] = acc;
    }
}

struct FwdWalkIn {
    double K[BU][BX], k[BU], A[BX][BX], B[BX][BU], c[BX];
    int c0, c1;
};
__device__ __forceinline__ void fwd_walk_load(const InstDesc& I, int n, FwdWalkIn& r)
{
    const double* w = I.ws + (long)n * W_NODE;
    r.c0 = I.child_off[n];
    r.c1 = I.child_off[n + 1];
#pragma unroll
    for (int i = 0; i < BU; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) r.K[i][j] = w[W_K + i * 4 + j];
        r.k[i] = w[W_KV + i];
    }
#pragma unroll
    for (int i = 0; i < BX; ++i) {
#pragma unroll
        for (int j = 0; j < BX; ++j) r.A[i][j] = w[W_A + i * 4 + j];
#pragma unroll
        for (int j = 0; j < BU; ++j) r.B[i][j] = w[W_B + i * 2 + j];
        r.c[i] = w[W_C + i];
    }
}

template <class T>
__device__ void pass_forward_seg(const InstDesc& I)
{
    if (T::rank() == 0)
#pragma unroll
        for (int i = 0; i < BX; ++i) I.ws[W_DX + i] = 0.0;
    T::sync();
    for (int d = 0; d <= I.max_seg_depth; ++d) {
        for (int n = T::rank_spread(); n < I.N; n += T::size()) {
            const int s = I.seg_of[n];
            if (I.seg_pos[n] != 0 || I.seg_depth[s] != d) continue;
            const int off = I.seg_off[s], len = I.seg_len[s];
            FwdWalkIn cur, nxt;
            fwd_walk_load(I, n, cur);
            double dx[BX];
            load4(I.ws + (long)n * W_NODE + W_DX, dx);
            // node ids of the walk: this step's, the next one's (its inputs
            // are requested now) and the one after (requested a step ahead)
            int m = n, m1 = len > 1 ? I.seg_nodes[off + 1] : -1;
            for (int q = 0; q < len; ++q) {
                const bool more = q + 1 < len;
                const int m2 = q + 2 < len ? I.seg_nodes[off + q + 2] : -1;
                if (more) fwd_walk_load(I, m1, nxt);
                double* w = I.ws + (long)m * W_NODE;
#pragma unroll
                for (int i = 0; i < BX; ++i) w[W_DX + i] = dx[i];
                const int c0 = cur.c0, c1 = cur.c1;
                double du[BU] = {0.0, 0.0};
                double dxn[BX] = {0.0, 0.0, 0.0, 0.0};
                if (c1 > c0) {
#pragma unroll
                    for (int i = 0; i < BU; ++i) {
                        double acc = cur.k[i];
#pragma unroll
                        for (int j = 0; j < BX; ++j) acc += cur.K[i][j] * dx[j];
                        du[i] = acc;
                    }
                    for (int j = c0; j < c1; ++j) {
                        double* wj = I.ws + (long)j * W_NODE;
                        // the only child is the next node of the walk: its
                        // defect is in flight with its other inputs
                        double cj[BX];
                        if (more) {
#pragma unroll
                            for (int i = 0; i < BX; ++i) cj[i] = nxt.c[i];
                        } else {
                            load4(wj + W_C, cj);
                        }
#pragma unroll
                        for (int i = 0; i < BX; ++i) {
                            double acc = cj[i];
#pragma unroll
                            for (int k = 0; k < BX; ++k) acc += cur.A[i][k] * dx[k];
#pragma unroll
                            for (int k = 0; k < BU; ++k) acc += cur.B[i][k] * du[k];
                            dxn[i] = acc;
                            if (!more) wj[W_DX + i] = acc;
                        }
                    }
                }
                w[W_DU] = du[0];
                w[W_DU + 1] = du[1];
#pragma unroll
                for (int i = 0; i < BX; ++i) dx[i] = dxn[i];
                cur = nxt;
                m = m1;
                m1 = m2;
            }
        }
        T::sync();
    }
}

// Adjoint sweep lam_leaf = q, lam_n = q_n + A_n^T sum_children lam (makes the
// state gradient of the Lagrangian vanish at the current point).
__device__ __forceinline__ void adjoint_node(const InstDesc& I, int n)
{
    const double* w = I.ws + (long)n * W_NODE;
    const int c0 = I.child_off[n], c1 = I.child_off[n + 1];
    double s[BX] = {0.0, 0.0, 0.0, 0.0};
    for (int j = c0; j < c1; ++j)
#pragma unroll
        for (int i = 0; i < BX; ++i) s[i] += I.lam[j * 4 + i];
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        double acc = w[W_QV + i];
        if (c1 > c0)
#pragma unroll
            for (int k = 0; k < BX; ++k) acc += w[W_A + k * 4 + i] * s[k];
        I.lam[n * 4 + i] = acc;
    }
}

template <class T>
__device__ void pass_adjoint(const InstDesc& I)
{
    if constexpr (T::kGrid) {
        // by segment depth, each segment walked bottom-up by one thread
        for (int d = I.max_seg_depth; d >= 0; --d) {
            for (int n = T::rank_spread(); n < I.N; n += T::size()) {
                const int s = I.seg_of[n];
                if (I.seg_end[s] != n || I.seg_depth[s] != d) continue;
                const int top = I.seg_nodes[I.seg_off[s]];
                for (int m = n;; m = I.parent[m]) {
                    adjoint_node(I, m);
                    if (m == top) break;
                }
            }
            T::sync();
        }
        return;
    }
    for (int t = I.T; t >= 0; --t) {
        const int n0 = I.level_off[t], n1 = I.level_off[t + 1];
        for (int n = n0 + T::rank(); n < n1; n += T::size()) adjoint_node(I, n);
        T::sync();
    }
}

// Start point.  warm bits: 1 = x, u given; 8 = u given, x by rollout from
// x0; 4 = ye given (clamped at zero); 2 = lam given, otherwise lam from the
// adjoint sweep at the start.  No bit: cold start u = 0 and exact rollout.
template <class T>
__device__ void build_start(const InstDesc& I, int warm, double rho)
{
    const int tid = T::rank(), N = I.N;
    for (int n = tid; n < N; n += T::size()) {
        if (!(warm & (1 | 8)) || I.child_off[n] == I.child_off[n + 1]) {
            I.u[n * 2] = 0.0;
            I.u[n * 2 + 1] = 0.0;
        }
        if (n == 0)
#pragma unroll
            for (int i = 0; i < BX; ++i) I.x[i] = I.x0[i];
#pragma unroll
        for (int s = 0; s < BG; ++s) I.ye[n * BG + s] = (warm & 4) ? fmax(I.ye[n * BG + s], 0.0) : 0.0;
    }
    T::sync();
    if ((warm & 8) || !(warm & 1)) {
        auto roll = [&](int n) {
            const int p = I.parent[n];
            double xp[BX], up[BU] = {I.u[p * 2], I.u[p * 2 + 1]}, xn[BX];
            load4(I.x + p * 4, xp);
            bike_step(I.prm, xp, up, xn);
            store4(I.x + n * 4, xn);
        };
        if constexpr (T::kGrid) {
            // by segment depth, each segment walked top-down by one thread
            for (int d = 0; d <= I.max_seg_depth; ++d) {
                for (int n = T::rank_spread(); n < N; n += T::size()) {
                    const int s = I.seg_of[n];
                    if (I.seg_pos[n] != 0 || I.seg_depth[s] != d) continue;
                    const int off = I.seg_off[s], len = I.seg_len[s];
                    for (int q = 0; q < len; ++q) {
                        const int m = I.seg_nodes[off + q];
                        if (m != 0) roll(m);
                    }
                }
                T::sync();
            }
        } else {
            for (int t = 1; t <= I.T; ++t) {
                const int n0 = I.level_off[t], n1 = I.level_off[t + 1];
                for (int n = n0 + tid; n < n1; n += T::size()) roll(n);
                T::sync();
            }
        }
    }
    if (!(warm & 2)) {
        double La, vi;
        pass_linearise<T>(I, rho, La, vi);
        T::sync();
        pass_adjoint<T>(I);
    }
}

// Quality of a start point: max(KKT residual, constraint violation), with
// NaN mapped to +inf.
template <class T>
__device__ double start_measure(const InstDesc& I, double rho, double* sred, double* gpart)
{
    double La, vi, rk, ld, dd;
    pass_linearise<T>(I, rho, La, vi);
    T::sync();
    pass_defects_kkt<T>(I, rk, ld, dd);
    double mx[2] = {rk, vi};
    T::template reduce<2, true>(mx, sred, gpart);
    if (!(mx[0] == mx[0]) || !(mx[1] == mx[1])) return INFINITY;
    return fmax(mx[0], mx[1]);
}

// Save (save = true) the caller's x, u, lam, ye into the node workspace
// slots of the step (dx, du, costate step, scan scratch), or restore them.
template <class T>
__device__ void stash_state(const InstDesc& I, bool save)
{
    for (int n = T::rank(); n < I.N; n += T::size()) {
        double* w = I.ws + (long)n * W_NODE;
#pragma unroll
        for (int i = 0; i < BX; ++i) {
            if (save) {
                w[W_DX + i] = I.x[n * 4 + i];
                w[W_LH + i] = I.lam[n * 4 + i];
            } else {
                I.x[n * 4 + i] = w[W_DX + i];
                I.lam[n * 4 + i] = w[W_LH + i];
            }
        }
#pragma unroll
        for (int i = 0; i < BU; ++i) {
            if (save)
                w[W_DU + i] = I.u[n * 2 + i];
            else
                I.u[n * 2 + i] = w[W_DU + i];
        }
#pragma unroll
        for (int k = 0; k < BG; ++k) {
            if (save)
                w[W_S0 + k] = I.ye[n * BG + k];
            else
                I.ye[n * BG + k] = w[W_S0 + k];
        }
    }
    T::sync();
}

// ---------------------------------------------------------------- solver kernel
// The whole of Alg. 1 for problem idx, run by team T (one workgroup or the grid).
// The descriptor's pointers all address global memory, but the compiler
// cannot tell that from a pointer loaded from memory and reaches them with
// flat instructions, which count against the LDS counter as well (so every
// wait for an LDS operation also waits for them).  Each pointer is passed
// through an empty asm statement as a global-address-space pointer and
// converted back, so that the compiler knows where it points and uses
// global loads and stores.
template <class P>
__device__ __forceinline__ P* as_global(P* p)
{
    __attribute__((address_space(1))) P* g = (__attribute__((address_space(1))) P*)p;
    asm volatile("" : "+s"(g));
    return (P*)g;
}

__device__ __forceinline__ InstDesc global_view(InstDesc d)
{
    d.parent = as_global(d.parent);
    d.child_off = as_global(d.child_off);
    d.level_off = as_global(d.level_off);
    d.weight = as_global(d.weight);
    d.ref = as_global(d.ref);
    d.obs = as_global(d.obs);
    d.has_obs = as_global(d.has_obs);
    d.x0 = as_global(d.x0);
    d.x = as_global(d.x);
    d.u = as_global(d.u);
    d.lam = as_global(d.lam);
    d.ye = as_global(d.ye);
    d.ws = as_global(d.ws);
    d.seg_of = as_global(d.seg_of);
    d.seg_pos = as_global(d.seg_pos);
    d.seg_len = as_global(d.seg_len);
    d.seg_nodes = as_global(d.seg_nodes);
    d.seg_off = as_global(d.seg_off);
    d.seg_end = as_global(d.seg_end);
    d.seg_depth = as_global(d.seg_depth);
    return d;
}

template <class T, bool SEGSCAN>
__device__ __forceinline__ void solve_one(const InstDesc* __restrict__ insts, int idx, const SolverCfg& cfg,
                                          SolveOut* __restrict__ outs, int* __restrict__ bad_flags,
                                          double* __restrict__ hist, int hist_cap, double* sred, double* sn,
                                          int lds_nodes, double* gpart)
{
    const InstDesc I = global_view(insts[idx]);
    // the per-node chain values fit in LDS: the stage-by-stage passes run
    // there (both with the level backward, the forward one after the
    // segment scan)
    const bool fits = !T::kGrid && I.N <= lds_nodes;
    const bool in_lds = fits && !SEGSCAN;
    int* bad = bad_flags + idx;
    const int tid = T::rank();
    const int N = I.N;
    if (tid == 0) *bad = INT_MAX;
    if (fits) lds_topology<T>(I, sn);

    double rho = cfg.rho0, mu = cfg.mu0, omega = cfg.omega0, eta = cfg.eta0;
    double r_kkt = INFINITY, viol = INFINITY, merit = 0.0;
    int status = BMPC_ERR_MAXITER, inner_total = 0, outer = 0, ls_fail = 0, ls_run = 0, nhist = 0;
    int start_used = (cfg.warm & (1 | 4 | 8)) ? 1 : 0;

    if (cfg.warm & 16) {
        // guarded start: keep the given start only if it is at least as
        // good as the cold one by max(KKT residual, violation) at rho0
        stash_state<T>(I, true);
        build_start<T>(I, 0, rho);
        const double m_cold = start_measure<T>(I, rho, sred, gpart);
        stash_state<T>(I, false);
        build_start<T>(I, cfg.warm & 15, rho);
        const double m_given = start_measure<T>(I, rho, sred, gpart);
        if (m_cold < m_given) {
            build_start<T>(I, 0, rho);
            start_used = 0;
        }
    } else {
        build_start<T>(I, cfg.warm, rho);
    }

    PhaseClock clk;
    const bool timer = tid == 0;
    for (outer = 0; outer < cfg.max_outer; ++outer) {
        for (int inner = 0;; ++inner) {
            double La_p, vi_p, rk_p, ld_p, dd_p;
            clk.start(timer);
            pass_linearise<T>(I, rho, La_p, vi_p, cfg.hess, cfg.eig_floor);
            T::sync();
            pass_defects_kkt<T>(I, rk_p, ld_p, dd_p);
            double mx[2] = {rk_p, vi_p};
            T::template reduce<2, true>(mx, sred, gpart);
            r_kkt = mx[0];
            viol = mx[1];
            clk.lap(timer, PH_LINEARISE);
            if (!(r_kkt == r_kkt)) {
                status = BMPC_ERR_NONFINITE;
                goto done;
            }
            if (r_kkt <= omega || inner >= cfg.max_inner) break;
            // total iteration cap (0 = none): stop before a further step
            if (cfg.max_total > 0 && inner_total >= cfg.max_total) {
                status = BMPC_ERR_MAXITER;
                goto done;
            }

            if constexpr (SEGSCAN)
                pass_riccati_segscan<T::BS>(I, bad);
            else if constexpr (!T::kGrid) {
                if (in_lds)
                    pass_riccati_lds<T::BS>(I, bad, sn);
                else
                    pass_riccati<T>(I, bad);
            } else {
                pass_riccati_seg<T>(I, bad);
            }
            if (__hip_atomic_load(bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != INT_MAX) {
                status = BMPC_ERR_NOT_PD;
                goto done;
            }
            clk.lap(timer, PH_BACKWARD);
            if constexpr (!T::kGrid) {
                if (fits) {
                    if (SEGSCAN) lds_from_ws<T::BS>(I, sn);
                    pass_forward_lds<T::BS>(I, sn);
                } else {
                    pass_forward<T>(I);
                }
            } else {
                pass_forward_seg<T>(I);
            }
            clk.lap(timer, PH_FORWARD);

            // merit slope pieces and the current merit
            double sm[6] = {0.0, 0.0, 0.0, La_p, ld_p, dd_p};
            for (int n = tid; n < N; n += T::size()) {
                if constexpr (T::kGrid) lam_hat_ws(I, n);  // left by the segment walk
                const double* w = I.ws + (long)n * W_NODE;
                double dx[BX];
                load4(w + W_DX, dx);
#pragma unroll
                for (int i = 0; i < BX; ++i) {
                    sm[0] += w[W_QV + i] * dx[i];
#pragma unroll
                    for (int j = 0; j < BX; ++j) sm[1] += dx[i] * w[W_Q + i * 4 + j] * dx[j];
                }
                if (I.child_off[n] < I.child_off[n + 1]) {
#pragma unroll
                    for (int i = 0; i < BU; ++i) {
                        sm[0] += w[W_RV + i] * w[W_DU + i];
#pragma unroll
                        for (int j = 0; j < BU; ++j) sm[1] += w[W_DU + i] * w[W_R + i * 2 + j] * w[W_DU + j];
#pragma unroll
                        for (int j = 0; j < BX; ++j) sm[1] += 2.0 * w[W_DU + i] * w[W_M + i * 4 + j] * dx[j];
                    }
                }
                if (n > 0)
#pragma unroll
                    for (int i = 0; i < BX; ++i) sm[2] += (w[W_LH + i] - 2.0 * I.lam[n * 4 + i]) * w[W_C + i];
            }
            T::template reduce<6, false>(sm, sred, gpart);
            const double gtd = sm[0], dhd = sm[1], lhd = sm[2], La0 = sm[3], ld0 = sm[4], dd0 = sm[5];
            if (dd0 > 0.0) {
                const double mu_hat = (gtd + lhd + 0.5 * dhd) / dd0;
                if (mu < mu_hat) mu = fmax(mu_hat, 2.0 * mu);
            }
            const double phi0 = La0 + ld0 + 0.5 * mu * dd0;
            const double dphi0 = gtd + lhd - mu * dd0;

            // backtracking (Sec. IV-A): a round evaluates the merit at na
            // step sizes 2^-k0 ... 2^-(k0+na-1) and keeps the largest accepted
            // one; a further round of smaller steps runs only when a round
            // accepts none
            const int na = cfg.n_alpha;
            double a_star = -1.0, phi_star = NAN;
            for (int rd = 0; rd < cfg.ls_rounds && a_star < 0.0; ++rd) {
            const int k0 = rd * na;
            double tr[3 * NALPHA_MAX];
#pragma unroll
            for (int e = 0; e < 3 * NALPHA_MAX; ++e) tr[e] = 0.0;
            // one (node, step size) pair per thread: ten short rollouts in
            // parallel instead of ten in a row
            // (node, step size) pairs while the tree is small against the
            // workgroup, whole nodes (all step sizes in one thread) otherwise
            const int per = (N * na <= 16 * T::size()) ? 1 : na;
            for (int it = tid; it < N * na / per; it += T::size())
            for (int sub = 0; sub < per; ++sub) {
                const int n = per == 1 ? it / na : it, ka = per == 1 ? it - n * na : sub;
                const double alpha = ldexp(1.0, -(k0 + ka));
                const double* w = I.ws + (long)n * W_NODE;
                const NodeData nd = node_data(I, n);
                double x[BX], u[BU], ye[BG], dx[BX];
                load4(I.x + n * 4, x);
                load4(w + W_DX, dx);
                u[0] = I.u[n * 2];
                u[1] = I.u[n * 2 + 1];
#pragma unroll
                for (int s = 0; s < BG; ++s) ye[s] = I.ye[n * BG + s];
                const int c0 = I.child_off[n], c1 = I.child_off[n + 1];
                double xt[BX], ut[BU];
#pragma unroll
                for (int i = 0; i < BX; ++i) xt[i] = x[i] + alpha * dx[i];
#pragma unroll
                for (int i = 0; i < BU; ++i) ut[i] = u[i] + alpha * w[W_DU + i];
                // outside the model's domain the trial point has merit +inf
                const double v = (c1 > c0 && !steer_in_domain(ut)) ? INFINITY
                                                                   : node_value(I.prm, nd, xt, ut, ye, rho);
                double ld = 0.0, dd = 0.0;
                if (c1 > c0) {
                    double ft[BX];
                    bike_step(I.prm, xt, ut, ft);
                    for (int j = c0; j < c1; ++j) {
                        const double* wj = I.ws + (long)j * W_NODE;
#pragma unroll
                        for (int i = 0; i < BX; ++i) {
                            const double xj = I.x[j * 4 + i] + alpha * wj[W_DX + i];
                            const double lj = I.lam[j * 4 + i] + alpha * (wj[W_LH + i] - I.lam[j * 4 + i]);
                            const double d = ft[i] - xj;
                            ld += lj * d;
                            dd += d * d;
                        }
                    }
                }
                // accumulate into slot ka without dynamic indexing (keeps tr in registers)
#pragma unroll
                for (int q = 0; q < NALPHA_MAX; ++q)
                    if (q == ka) {
                        tr[q] += v;
                        tr[NALPHA_MAX + q] += ld;
                        tr[2 * NALPHA_MAX + q] += dd;
                    }
            }
            T::template reduce<3 * NALPHA_MAX, false>(tr, sred, gpart);
            double alpha = ldexp(1.0, -k0);
            // constant indices only, so that tr stays in registers (a loop
            // bounded by na would index it at run time and move it to
            // scratch memory, for the accumulation above as well)
#pragma unroll
            for (int ka = 0; ka < NALPHA_MAX; ++ka) {
                if (ka < na) {
                    const double phi = tr[ka] + tr[NALPHA_MAX + ka] + 0.5 * mu * tr[2 * NALPHA_MAX + ka];
                    if (a_star < 0.0 && phi <= phi0 + cfg.beta * alpha * dphi0) {
                        a_star = alpha;
                        phi_star = phi;
                    }
                }
                alpha *= 0.5;
            }
            }
            if (a_star < 0.0) {
                ++ls_fail;
                if (++ls_run >= cfg.max_ls_fail) {
                    status = BMPC_ERR_LINESEARCH;
                    goto done;
                }
                a_star = ldexp(1.0, -(cfg.ls_rounds * na - 1));
                phi_star = NAN;
            } else {
                ls_run = 0;
            }
            clk.lap(timer, PH_LINESEARCH);
            for (int n = tid; n < N; n += T::size()) {
                const double* w = I.ws + (long)n * W_NODE;
#pragma unroll
                for (int i = 0; i < BX; ++i) {
                    I.x[n * 4 + i] += a_star * w[W_DX + i];
                    I.lam[n * 4 + i] += a_star * (w[W_LH + i] - I.lam[n * 4 + i]);
                }
#pragma unroll
                for (int i = 0; i < BU; ++i) I.u[n * 2 + i] += a_star * w[W_DU + i];
            }
            merit = phi_star;
            ++inner_total;
            if (hist && tid == 0 && nhist < hist_cap) {
                double* h = hist + ((long)idx * hist_cap + nhist) * 6;
                h[0] = outer;
                h[1] = r_kkt;
                h[2] = a_star;
                h[3] = mu;
                h[4] = rho;
                h[5] = phi_star;
                ++nhist;
            }
            T::sync();
            clk.lap(timer, PH_UPDATE);
        }
        clk.start(timer);

        // outer update (BCL)
        if (viol <= eta) {
            for (int n = tid; n < N; n += T::size()) {
                const NodeData nd = node_data(I, n);
                double x[BX], u[BU], g[BG], dist, ex, ey;
                bool on[BG];
                load4(I.x + n * 4, x);
                u[0] = I.u[n * 2];
                u[1] = I.u[n * 2 + 1];
                node_constraints(I.prm, nd, x, u, g, on, dist, ex, ey);
#pragma unroll
                for (int s = 0; s < BG; ++s) {
                    const double y = I.ye[n * BG + s];
                    I.ye[n * BG + s] = on[s] ? fmax(0.0, y + rho * g[s]) : 0.0;
                }
            }
            T::sync();
            if (fmax(r_kkt, viol) < cfg.eps_tol) {
                status = BMPC_OK;
                ++outer;
                goto done;
            }
            omega = omega / pow(rho, cfg.b_omega);
            eta = eta / pow(rho, cfg.b_eta);
        } else {
            rho = cfg.tau * rho;
            omega = cfg.omega0 / pow(rho, cfg.a_omega);
            eta = cfg.eta0 / pow(rho, cfg.a_eta);
        }
        clk.lap(timer, PH_UPDATE);
        // Alg. 1 floors omega at eps_tol; eta gets the same floor, since the
        // stopping test asks only viol < eps_tol
        omega = fmax(omega, cfg.eps_tol);
        eta = fmax(eta, cfg.eps_tol);
    }

done:
    T::sync();
    if (tid == 0) {
        SolveOut o;
        o.status = status;
        o.outer_it = outer;
        o.inner_it = inner_total;
        o.ls_failures = ls_fail;
        const int bn = __hip_atomic_load(bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        o.bad_node = bn == INT_MAX ? -1 : bn;
        o.start = start_used;
        o.r_kkt = r_kkt;
        o.viol = viol;
        o.rho = rho;
        o.mu = mu;
        o.merit = merit;
#pragma unroll
        for (int k = 0; k < PH_COUNT; ++k) o.ticks[k] = clk.acc[k];
        outs[idx] = o;
    }
    T::sync();
}

// Persistent batched solver: every workgroup takes the next problem from a
// queue (problems in decreasing size order) until the queue is empty, so a
// workgroup that finishes early starts another problem instead of idling
// while the slowest ones iterate.  Each problem is solved start to end by
// one workgroup, so results do not depend on the schedule.
template <int BS, bool SEGSCAN>
__global__ void __launch_bounds__(BS) k_bmpc_wg(const InstDesc* __restrict__ insts, SolverCfg cfg,
                                                SolveOut* __restrict__ outs, int* __restrict__ bad_flags,
                                                double* __restrict__ hist, int hist_cap,
                                                const int* __restrict__ order, int count, int* queue, int lds_nodes)
{
    __shared__ double sred[3 * NALPHA_MAX * (BS / 64)];
    __shared__ int s_next;
    extern __shared__ double s_nodes[];  // lds_nodes x LN
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(queue, 1);
        __syncthreads();
        const int q = s_next;
        __syncthreads();
        if (q >= count) break;
        solve_one<TeamWG<BS>, SEGSCAN>(insts, order[q], cfg, outs, bad_flags, hist, hist_cap, sred, s_nodes,
                                       lds_nodes, nullptr);
    }
}

__global__ void k_reset_queue(int* queue) { *queue = 0; }

// One large problem solved by the whole grid (cooperative launch).
__global__ void __launch_bounds__(256) k_bmpc_grid(const InstDesc* __restrict__ insts, SolverCfg cfg,
                                                   SolveOut* __restrict__ outs, int* __restrict__ bad_flags,
                                                   double* __restrict__ hist, int hist_cap, double* gpart)
{
    __shared__ double sred[3 * NALPHA_MAX * 4];
    solve_one<TeamGrid<256>, false>(insts, 0, cfg, outs, bad_flags, hist, hist_cap, sred, nullptr, 0, gpart);
}

// Linearisation and quadratisation only (row a2), for testing and for
// callers that bring their own LQR solver.
template <int BS>
__global__ void __launch_bounds__(BS) k_bmpc_linearise(InstDesc I, double rho, double* kkt_out, int hess,
                                                       double eig_floor)
{
    __shared__ double sred[2 * (BS / 64)];
    double La, vi, rk, ld, dd;
    pass_linearise<TeamWG<BS>>(I, rho, La, vi, hess, eig_floor);
    __syncthreads();
    pass_defects_kkt<TeamWG<BS>>(I, rk, ld, dd);
    double mx[2] = {rk, vi};
    block_reduce<BS, 2, true>(mx, sred);
    if (threadIdx.x == 0 && kkt_out) {
        kkt_out[0] = mx[0];
        kkt_out[1] = mx[1];
    }
}

// A measured initial state passed by value (use = 0: none).
struct MeasuredX0 {
    double v[4];
    int use;
};

// Shifted warm start after one simulated step: x0' = F(x0, u_0) (or the
// measured state when one is given); every
// non-leaf node takes the weight-averaged values of its children (the old
// nodes one stage later on the same scenarios), a node whose children are
// leaves repeats its own input, leaves keep costates and multipliers,
// extrapolate their reference and are rolled out from the new parent.
// The workspace rows serve as scratch for the new values.
template <int BS>
__global__ void __launch_bounds__(BS) k_bmpc_shift(const InstDesc* __restrict__ insts, MeasuredX0 meas)
{
    const InstDesc I = insts[blockIdx.x];
    const int N = I.N, tid = threadIdx.x;
    double* ref = const_cast<double*>(I.ref);
    double* x0 = const_cast<double*>(I.x0);
    // scratch columns inside each workspace row
    constexpr int T_X = W_Q, T_U = W_Q + 4, T_L = W_Q + 6, T_Y = W_Q + 10, T_R = W_K;
    for (int n = tid; n < N; n += BS) {
        double* w = I.ws + (long)n * W_NODE;
        const int c0 = I.child_off[n], c1 = I.child_off[n + 1];
        if (c0 == c1) {
            const int p = I.parent[n];
            for (int a = 0; a < 4; ++a) {
                w[T_L + a] = I.lam[n * 4 + a];
                w[T_R + a] = p >= 0 ? 2.0 * ref[n * 4 + a] - ref[p * 4 + a] : ref[n * 4 + a];
            }
            for (int a = 0; a < BG; ++a) w[T_Y + a] = I.ye[n * BG + a];
            w[T_U] = 0.0;
            w[T_U + 1] = 0.0;
            continue;
        }
        double wsum = 0.0, wu = 0.0;
        int nctrl = 0;
        for (int j = c0; j < c1; ++j) {
            wsum += I.weight[j];
            if (I.child_off[j] < I.child_off[j + 1]) {
                wu += I.weight[j];
                ++nctrl;
            }
        }
        double sx[4] = {}, sl[4] = {}, sr[4] = {}, sy[BG] = {}, su[2] = {};
        for (int j = c0; j < c1; ++j) {
            const double f = wsum > 0.0 ? I.weight[j] / wsum : 1.0 / (c1 - c0);
            for (int a = 0; a < 4; ++a) {
                sx[a] += f * I.x[j * 4 + a];
                sl[a] += f * I.lam[j * 4 + a];
                sr[a] += f * ref[j * 4 + a];
            }
            for (int a = 0; a < BG; ++a) sy[a] += f * I.ye[j * BG + a];
            if (I.child_off[j] < I.child_off[j + 1]) {
                const double fu = wu > 0.0 ? I.weight[j] / wu : 1.0 / nctrl;
                su[0] += fu * I.u[j * 2];
                su[1] += fu * I.u[j * 2 + 1];
            }
        }
        for (int a = 0; a < 4; ++a) {
            w[T_X + a] = sx[a];
            w[T_L + a] = sl[a];
            w[T_R + a] = sr[a];
        }
        for (int a = 0; a < BG; ++a) w[T_Y + a] = sy[a];
        w[T_U] = nctrl > 0 ? su[0] : I.u[n * 2];
        w[T_U + 1] = nctrl > 0 ? su[1] : I.u[n * 2 + 1];
    }
    __syncthreads();
    if (tid == 0) {
        double xr[BX], ur[BU] = {I.u[0], I.u[1]}, xn[BX];
        load4(I.x0, xr);
        bike_step(I.prm, xr, ur, xn);
        for (int a = 0; a < 4; ++a) I.ws[T_X + a] = meas.use ? meas.v[a] : xn[a];
    }
    __syncthreads();
    // leaves are rolled out from their (already shifted) parents
    for (int n = tid; n < N; n += BS) {
        if (I.child_off[n] != I.child_off[n + 1] || n == 0) continue;
        const double* wp = I.ws + (long)I.parent[n] * W_NODE;
        double xp[BX], up[BU] = {wp[T_U], wp[T_U + 1]}, xn[BX];
        load4(wp + T_X, xp);
        bike_step(I.prm, xp, up, xn);
        for (int a = 0; a < 4; ++a) I.ws[(long)n * W_NODE + T_X + a] = xn[a];
    }
    __syncthreads();
    for (int n = tid; n < N; n += BS) {
        const double* w = I.ws + (long)n * W_NODE;
        for (int a = 0; a < 4; ++a) {
            I.x[n * 4 + a] = w[T_X + a];
            I.lam[n * 4 + a] = w[T_L + a];
            ref[n * 4 + a] = w[T_R + a];
        }
        for (int a = 0; a < BG; ++a) I.ye[n * BG + a] = w[T_Y + a];
        I.u[n * 2] = w[T_U];
        I.u[n * 2 + 1] = w[T_U + 1];
        if (n == 0)
            for (int a = 0; a < 4; ++a) x0[a] = w[T_X + a];
    }
}

}  // namespace bmpc

using namespace bmpc;

// ------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------
struct bmpc_problem {
    bmpc_tree* tree = nullptr;
    bmpc_bicycle_params prm{};
    int N = 0;
    double* d_weight = nullptr;
    double* d_ref = nullptr;
    double* d_obs = nullptr;
    int* d_has = nullptr;
    double* d_x0 = nullptr;
    int n_control = 0;  // nodes with children
    int n_obs = 0;      // nodes carrying the obstacle constraint
    bmpc_batch* self = nullptr;  // one-instance batch used by bmpc_solve
    double* d_kkt = nullptr;     // KKT residual and violation of bmpc_linearize (2 doubles)
};

struct bmpc_batch {
    int count = 0;
    std::vector<bmpc_problem*> problems;
    std::vector<int> offset;  // node offset of each instance in the state arrays
    long total_nodes = 0;
    InstDesc* d_desc = nullptr;
    SolveOut* d_out = nullptr;
    int* d_bad = nullptr;
    double* d_state = nullptr;  // x | u | lam | ye for all instances
    double* d_ws = nullptr;
    double* d_hist = nullptr;
    int hist_cap = 0;
    std::vector<InstDesc> h_desc;
    int tuned_variant = 0;  // set by bmpc_batch_tune (0 = not tuned)
    int tuned_block = 0;
    int* d_order = nullptr;  // problems by decreasing node count (work queue order)
    double* d_gpart = nullptr;  // per-workgroup partial sums of the grid solver
    int* d_queue = nullptr;  // next queue position, reset before every solve
};

// Scatter one row of network outputs per problem into its start point:
// u of every control node (node order), then the PHR multiplier estimates of
// every active constraint slot in (node, slot) order (slots 0-3 of control
// nodes, slot 4 of nodes with an obstacle).  Inactive slots and leaf inputs
// become zero; x and lam are left to the solver's rollout and adjoint sweep.
template <int BS>
__global__ void __launch_bounds__(BS) k_start_from_outputs(const InstDesc* __restrict__ insts,
                                                           const float* __restrict__ Y, int width)
{
    __shared__ int s_c[BS], s_a[BS];
    __shared__ int s_nctl;
    const InstDesc I = insts[blockIdx.x];
    const float* y = Y + (long)blockIdx.x * width;
    const int tid = threadIdx.x, N = I.N;
    if (tid == 0) s_nctl = 0;
    __syncthreads();
    int mine = 0;
    for (int n = tid; n < N; n += BS) mine += I.child_off[n + 1] > I.child_off[n] ? 1 : 0;
    atomicAdd(&s_nctl, mine);
    __syncthreads();
    const int ye_base = 2 * s_nctl;
    int carry_c = 0, carry_a = 0;
    for (int base = 0; base < N; base += BS) {
        const int n = base + tid;
        const bool in = n < N;
        const bool ctl = in && I.child_off[n + 1] > I.child_off[n];
        const bool obs = in && I.has_obs[n] != 0;
        const int c = ctl ? 1 : 0, a = (ctl ? 4 : 0) + (obs ? 1 : 0);
        s_c[tid] = c;
        s_a[tid] = a;
        __syncthreads();
        for (int off = 1; off < BS; off <<= 1) {  // inclusive Hillis-Steele scan
            const int vc = tid >= off ? s_c[tid - off] : 0;
            const int va = tid >= off ? s_a[tid - off] : 0;
            __syncthreads();
            s_c[tid] += vc;
            s_a[tid] += va;
            __syncthreads();
        }
        if (in) {
            const int ic = carry_c + s_c[tid] - c;  // exclusive prefixes
            int ia = ye_base + carry_a + s_a[tid] - a;
            I.u[n * 2] = ctl ? (double)y[2 * ic] : 0.0;
            I.u[n * 2 + 1] = ctl ? (double)y[2 * ic + 1] : 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) I.ye[n * BG + k] = ctl ? (double)y[ia + k] : 0.0;
            if (ctl) ia += 4;
            I.ye[n * BG + 4] = obs ? (double)y[ia] : 0.0;
        }
        carry_c += s_c[BS - 1];
        carry_a += s_a[BS - 1];
        __syncthreads();
    }
}

// Batched solver instantiations: threads per problem x backward variant.
struct WgKernel {
    int block;
    bool segscan;
    void (*fn)(const InstDesc*, SolverCfg, SolveOut*, int*, double*, int, const int*, int, int*, int);
    const char* name;
};
static const WgKernel kWgKernels[] = {
    {64, false, k_bmpc_wg<64, false>, "bmpc_solve_wg64_level"},
    {128, false, k_bmpc_wg<128, false>, "bmpc_solve_wg128_level"},
    {256, false, k_bmpc_wg<256, false>, "bmpc_solve_wg256_level"},
    {64, true, k_bmpc_wg<64, true>, "bmpc_solve_wg64_segscan"},
    {128, true, k_bmpc_wg<128, true>, "bmpc_solve_wg128_segscan"},
    {256, true, k_bmpc_wg<256, true>, "bmpc_solve_wg256_segscan"},
};

static const WgKernel* find_wg(int block, bool segscan)
{
    for (const auto& k : kWgKernels)
        if (k.block == block && k.segscan == segscan) return &k;
    return &kWgKernels[2];
}

// Dynamic LDS of a solver launch: the per-node chain values of problems up
// to this size.  A workgroup of 256 threads has a CU to itself (register
// use), so it takes most of the 160 KB; narrower ones leave room for the
// other workgroups of the CU.  Requests above the default limit are enabled
// once per kernel; if that fails the launch stays within 64 KB.
static size_t solver_lds_bytes(const WgKernel& k)
{
    static std::mutex mu;
    static std::map<const void*, size_t> ok;
    std::lock_guard<std::mutex> lk(mu);
    auto it = ok.find((const void*)k.fn);
    if (it != ok.end()) return it->second;
    size_t want = k.block == 256 ? 144 * 1024 : (k.block == 128 ? 72 * 1024 : 36 * 1024);
    if (want > 64 * 1024 &&
        hipFuncSetAttribute((const void*)k.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)want) != hipSuccess) {
        (void)hipGetLastError();
        want = 60 * 1024;
    }
    ok[(const void*)k.fn] = want;
    return want;
}

// Workgroups that fit on the device at once for this kernel (the persistent
// grid); never more than the number of problems.
static int resident_groups(const WgKernel& k, int count)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, long> cache;  // (device, kernel) -> groups
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return count;
    long cap = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find({dev, (const void*)k.fn});
        if (it != cache.end()) {
            cap = it->second;
        } else {
            int per_cu = 0, cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k.fn, k.block, solver_lds_bytes(k)) !=
                    hipSuccess ||
                per_cu < 1 || cus < 1)
                return count;
            cap = (long)per_cu * cus;
            cache[{dev, (const void*)k.fn}] = cap;
        }
    }
    return (int)(cap < count ? cap : count);
}

static BikeParams to_dev(const bmpc_bicycle_params& p)
{
    BikeParams b;
    b.L = p.wheelbase;
    b.dt = p.dt;
    for (int i = 0; i < 4; ++i) b.Qd[i] = p.Qd[i];
    for (int i = 0; i < 2; ++i) b.Rd[i] = p.Rd[i];
    b.a_max = p.a_max;
    b.steer_max = p.steer_max;
    b.obs_r = p.obs_radius;
    return b;
}

static SolverCfg to_cfg(const bmpc_settings& s, int warm)
{
    SolverCfg c;
    c.eps_tol = s.eps_tol;
    c.tau = s.tau;
    c.omega0 = s.omega0;
    c.eta0 = s.eta0;
    c.a_omega = s.a_omega;
    c.b_omega = s.b_omega;
    c.a_eta = s.a_eta;
    c.b_eta = s.b_eta;
    c.rho0 = s.rho0;
    c.mu0 = s.mu0;
    c.beta = s.armijo_beta;
    c.n_alpha = s.n_alpha;
    c.max_outer = s.max_outer;
    c.max_inner = s.max_inner;
    c.max_total = s.max_iter_total;
    c.max_ls_fail = s.max_ls_fail;
    c.ls_rounds = s.ls_rounds;
    c.warm = warm;
    c.hess = s.hessian;
    c.eig_floor = s.eig_floor;
    return c;
}

template <class T>
static bool dalloc(T** p, size_t n)
{
    return hipMalloc((void**)p, std::max<size_t>(1, n) * sizeof(T)) == hipSuccess;
}

// Reset the work queue and start the persistent solver kernel (both are
// plain kernel launches, so the pair can be captured into a graph).
static bmpc_status launch_solver(bmpc_batch* b, const WgKernel& k, const SolverCfg& cfg, hipStream_t st)
{
    const size_t lds = solver_lds_bytes(k);
    const int grid = resident_groups(k, b->count);
    const int lds_nodes = (int)(lds / (LN * sizeof(double)));
    ProfScope ps(k.name, st);
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, st, b->d_queue);
    hipLaunchKernelGGL(k.fn, dim3(grid), dim3(k.block), lds, st, b->d_desc, cfg, b->d_out, b->d_bad, b->d_hist,
                       b->hist_cap, b->d_order, b->count, b->d_queue, lds_nodes);
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

// Problems at least this large, alone in a batch, are solved by the whole
// grid (cooperative launch) instead of one workgroup.
constexpr long GRID_MIN_NODES = 16384;

static bmpc_status launch_grid_solver(bmpc_batch* b, const SolverCfg& cfg, hipStream_t st)
{
    int dev = 0, cus = 0, per_cu = 0;
    BMPC_HIP_TRY(hipGetDevice(&dev));
    BMPC_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    BMPC_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_bmpc_grid, 256, 0));
    if (per_cu < 1 || cus < 1) return fail(BMPC_ERR_HIP, "the grid solver does not fit on the device");
    const int grid = per_cu * cus;
    if (!b->d_gpart && !dalloc(&b->d_gpart, (size_t)grid * 3 * NALPHA_MAX))
        return fail(BMPC_ERR_OOM, "device allocation for the grid reductions failed");
    const InstDesc* desc = b->d_desc;
    SolverCfg c = cfg;
    SolveOut* outs = b->d_out;
    int* bad = b->d_bad;
    double* hist = b->d_hist;
    int hist_cap = b->hist_cap;
    double* gpart = b->d_gpart;
    void* args[] = {&desc, &c, &outs, &bad, &hist, &hist_cap, &gpart};
    ProfScope ps("bmpc_solve_grid", st);
    BMPC_HIP_TRY(hipLaunchCooperativeKernel((const void*)k_bmpc_grid, dim3(grid), dim3(256), args, 0, st));
    return BMPC_OK;
}

extern "C" {

BMPC_API void bmpc_settings_default(bmpc_settings* s)
{
    if (!s) return;
    s->eps_tol = 1e-6;
    s->tau = 100.0;
    s->omega0 = 1.0;
    s->eta0 = 0.1;
    s->a_omega = 1.0;
    s->b_omega = 1.0;
    s->a_eta = 0.1;
    s->b_eta = 0.9;
    s->rho0 = 100.0;
    s->mu0 = 100.0;
    s->armijo_beta = 1e-4;
    s->n_alpha = 10;
    s->max_outer = 50;
    s->max_inner = 100;
    s->max_ls_fail = 3;
    s->riccati_variant = BMPC_RICCATI_AUTO;
    s->block_size = 0;
    s->max_iter_total = 0;
    s->ls_rounds = 3;
    s->hessian = BMPC_HESSIAN_GAUSS_NEWTON;
    s->eig_floor = 1e-9;
}

BMPC_API void bmpc_bicycle_default(bmpc_bicycle_params* p)
{
    if (!p) return;
    p->wheelbase = 2.7;
    p->dt = 0.1;
    const double Q[4] = {1.0, 1.0, 0.1, 0.1}, R[2] = {0.1, 1.0};
    for (int i = 0; i < 4; ++i) p->Qd[i] = Q[i];
    for (int i = 0; i < 2; ++i) p->Rd[i] = R[i];
    p->a_max = 3.0;
    p->steer_max = 0.5;
    p->obs_radius = 1.5;
}

BMPC_API bmpc_status bmpc_node_refs(const bmpc_tree* t, const double* leaf_prob, const double* leaf_offset,
                                    double dt, double speed, double* node_ref)
{
    if (!t || !leaf_prob || !leaf_offset || !node_ref) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    const HostTree& h = t->h;
    std::vector<double> w(h.N, 0.0), wy(h.N, 0.0);
    for (size_t l = 0; l < h.leaves.size(); ++l) {
        w[h.leaves[l]] = leaf_prob[l];
        wy[h.leaves[l]] = leaf_prob[l] * leaf_offset[l];
    }
    for (int i = h.N - 1; i >= 1; --i) {
        w[h.parent[i]] += w[i];
        wy[h.parent[i]] += wy[i];
    }
    for (int i = 0; i < h.N; ++i) {
        node_ref[4 * i + 0] = speed * dt * h.stage[i];
        node_ref[4 * i + 1] = w[i] > 0.0 ? wy[i] / w[i] : 0.0;
        node_ref[4 * i + 2] = 0.0;
        node_ref[4 * i + 3] = speed;
    }
    return BMPC_OK;
}

static bmpc_status check_problem_data(int N, const double* node_weight, const double* node_ref,
                                      const int32_t* has_obs, const double* x0)
{
    for (int i = 0; i < N; ++i)
        if (!std::isfinite(node_weight[i]) || node_weight[i] < 0.0)
            return fail(BMPC_ERR_NONFINITE, "node_weight[%d] must be a finite non-negative number", i);
    for (int i = 0; i < 4 * N; ++i)
        if (!std::isfinite(node_ref[i])) return fail(BMPC_ERR_NONFINITE, "node_ref has a non-finite entry");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(x0[i])) return fail(BMPC_ERR_NONFINITE, "x0 has a non-finite entry");
    for (int i = 0; i < N; ++i)
        if (has_obs[i] != 0 && has_obs[i] != 1) return fail(BMPC_ERR_INVALID_ARG, "has_obs[%d] must be 0 or 1", i);
    return BMPC_OK;
}

static bmpc_status upload_problem_data(bmpc_problem* p, const double* node_weight, const double* node_ref,
                                       const double* node_obs, const int32_t* has_obs, const double* x0)
{
    const int N = p->N;
    BMPC_HIP_TRY(hipMemcpy(p->d_weight, node_weight, sizeof(double) * N, hipMemcpyHostToDevice));
    BMPC_HIP_TRY(hipMemcpy(p->d_ref, node_ref, sizeof(double) * 4 * N, hipMemcpyHostToDevice));
    BMPC_HIP_TRY(hipMemcpy(p->d_obs, node_obs, sizeof(double) * 2 * N, hipMemcpyHostToDevice));
    BMPC_HIP_TRY(hipMemcpy(p->d_has, has_obs, sizeof(int) * N, hipMemcpyHostToDevice));
    BMPC_HIP_TRY(hipMemcpy(p->d_x0, x0, sizeof(double) * 4, hipMemcpyHostToDevice));
    p->n_obs = 0;
    for (int i = 0; i < N; ++i) p->n_obs += has_obs[i];
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_problem_create(bmpc_tree* tree, const bmpc_bicycle_params* prm,
                                         const double* node_weight, const double* node_ref,
                                         const double* node_obs, const int32_t* has_obs, const double* x0,
                                         bmpc_problem** out)
{
    if (!tree || !prm || !node_weight || !node_ref || !node_obs || !has_obs || !x0 || !out)
        return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (!(prm->dt > 0.0) || !(prm->wheelbase > 0.0) || !(prm->obs_radius >= 0.0))
        return fail(BMPC_ERR_INVALID_ARG, "bicycle parameters must be positive");
    const int N = tree->h.N;
    bmpc_status st = check_problem_data(N, node_weight, node_ref, has_obs, x0);
    if (st != BMPC_OK) return st;
    st = tree_on_device(tree);
    if (st != BMPC_OK) return st;
    auto* p = new bmpc_problem();
    p->tree = tree;
    p->prm = *prm;
    p->N = N;
    for (int i = 0; i < N; ++i) p->n_control += tree->h.child_off[i + 1] > tree->h.child_off[i] ? 1 : 0;
    bool ok = dalloc(&p->d_weight, N) && dalloc(&p->d_ref, 4 * (size_t)N) && dalloc(&p->d_obs, 2 * (size_t)N) &&
              dalloc(&p->d_has, N) && dalloc(&p->d_x0, 4);
    if (!ok) {
        bmpc_problem_destroy(p);
        return fail(BMPC_ERR_OOM, "device allocation for the problem failed");
    }
    if ((st = upload_problem_data(p, node_weight, node_ref, node_obs, has_obs, x0)) != BMPC_OK) {
        bmpc_problem_destroy(p);
        return st;
    }
    *out = p;
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_problem_update(bmpc_problem* p, const double* node_weight, const double* node_ref,
                                         const double* node_obs, const int32_t* has_obs, const double* x0)
{
    if (!p || !node_weight || !node_ref || !node_obs || !has_obs || !x0)
        return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    bmpc_status st = check_problem_data(p->N, node_weight, node_ref, has_obs, x0);
    if (st != BMPC_OK) return st;
    return upload_problem_data(p, node_weight, node_ref, node_obs, has_obs, x0);
}

BMPC_API bmpc_status bmpc_problem_get_x0(const bmpc_problem* p, double* x0)
{
    if (!p || !x0) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    BMPC_HIP_TRY(hipMemcpy(x0, p->d_x0, sizeof(double) * 4, hipMemcpyDeviceToHost));
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_problem_output_width(const bmpc_problem* p, int32_t* width)
{
    if (!p || !width) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    *width = 6 * p->n_control + p->n_obs;
    return BMPC_OK;
}

BMPC_API void bmpc_batch_destroy(bmpc_batch* b);

BMPC_API void bmpc_problem_destroy(bmpc_problem* p)
{
    if (!p) return;
    if (p->self) bmpc_batch_destroy(p->self);
    (void)hipFree(p->d_weight);
    (void)hipFree(p->d_ref);
    (void)hipFree(p->d_obs);
    (void)hipFree(p->d_has);
    (void)hipFree(p->d_x0);
    (void)hipFree(p->d_kkt);
    delete p;
}

BMPC_API bmpc_status bmpc_problem_set_x0(bmpc_problem* p, const double* x0)
{
    if (!p || !x0) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(x0[i])) return fail(BMPC_ERR_NONFINITE, "x0 has a non-finite entry");
    BMPC_HIP_TRY(hipMemcpy(p->d_x0, x0, sizeof(double) * 4, hipMemcpyHostToDevice));
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_batch_create(bmpc_problem* const* problems, int32_t count, int32_t hist_cap,
                                       bmpc_batch** out)
{
    if (!problems || count <= 0 || !out || hist_cap < 0) return fail(BMPC_ERR_INVALID_ARG, "bad argument");
    *out = nullptr;
    auto* b = new bmpc_batch();
    b->count = count;
    b->hist_cap = hist_cap;
    b->problems.assign(problems, problems + count);
    b->offset.resize(count);
    long tot = 0;
    for (int i = 0; i < count; ++i) {
        if (!problems[i]) {
            delete b;
            return fail(BMPC_ERR_INVALID_ARG, "problem %d is NULL", i);
        }
        b->offset[i] = (int)tot;
        tot += problems[i]->N;
    }
    b->total_nodes = tot;
    bool ok = dalloc(&b->d_desc, count) && dalloc(&b->d_out, count) && dalloc(&b->d_bad, count) &&
              dalloc(&b->d_order, count) && dalloc(&b->d_queue, 1) &&
              dalloc(&b->d_state, (size_t)tot * 15) && dalloc(&b->d_ws, (size_t)tot * W_NODE) &&
              (hist_cap == 0 || dalloc(&b->d_hist, (size_t)count * hist_cap * 6));
    if (!ok) {
        bmpc_batch_destroy(b);
        return fail(BMPC_ERR_OOM, "device allocation for the batch failed");
    }
    if (hipMemset(b->d_state, 0, sizeof(double) * tot * 15) != hipSuccess) {
        bmpc_batch_destroy(b);
        return fail(BMPC_ERR_HIP, "hipMemset failed");
    }
    b->h_desc.resize(count);
    for (int i = 0; i < count; ++i) {
        const bmpc_problem* p = problems[i];
        InstDesc& d = b->h_desc[i];
        d.N = p->N;
        d.T = p->tree->h.depth;
        d.parent = p->tree->d.parent;
        d.child_off = p->tree->d.child_off;
        d.level_off = p->tree->d.level_off;
        d.weight = p->d_weight;
        d.ref = p->d_ref;
        d.obs = p->d_obs;
        d.has_obs = p->d_has;
        d.x0 = p->d_x0;
        d.prm = to_dev(p->prm);
        const long o = b->offset[i];
        d.x = b->d_state + o * 4;
        d.u = b->d_state + tot * 4 + o * 2;
        d.lam = b->d_state + tot * 6 + o * 4;
        d.ye = b->d_state + tot * 10 + o * 5;
        d.ws = b->d_ws + o * W_NODE;
        const TreeDev& td = p->tree->d;
        d.seg_of = td.seg_of;
        d.seg_pos = td.seg_pos;
        d.seg_len = td.seg_len;
        d.seg_nodes = td.seg_nodes;
        d.seg_off = td.seg_off;
        d.seg_end = td.seg_end;
        d.seg_depth = td.seg_depth;
        d.max_seg_len = td.max_seg_len;
        d.max_seg_depth = td.max_seg_depth;
    }
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return problems[a]->N > problems[c]->N; });
    if (hipMemcpy(b->d_desc, b->h_desc.data(), sizeof(InstDesc) * count, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_order, order.data(), sizeof(int) * count, hipMemcpyHostToDevice) != hipSuccess) {
        bmpc_batch_destroy(b);
        return fail(BMPC_ERR_HIP, "uploading the batch descriptors failed");
    }
    *out = b;
    return BMPC_OK;
}

BMPC_API void bmpc_batch_destroy(bmpc_batch* b)
{
    if (!b) return;
    (void)hipFree(b->d_order);
    (void)hipFree(b->d_gpart);
    (void)hipFree(b->d_queue);
    (void)hipFree(b->d_desc);
    (void)hipFree(b->d_out);
    (void)hipFree(b->d_bad);
    (void)hipFree(b->d_state);
    (void)hipFree(b->d_ws);
    (void)hipFree(b->d_hist);
    delete b;
}

BMPC_API bmpc_status bmpc_batch_launch(bmpc_batch* b, const bmpc_settings* s, int32_t warm, void* stream)
{
    if (!b || !s) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    if (s->n_alpha < 1 || s->n_alpha > NALPHA_MAX)
        return fail(BMPC_ERR_INVALID_ARG, "n_alpha must be in [1, %d]", NALPHA_MAX);
    if (s->ls_rounds < 1 || s->ls_rounds > LS_ROUNDS_MAX)
        return fail(BMPC_ERR_INVALID_ARG, "ls_rounds must be in [1, %d]", LS_ROUNDS_MAX);
    if (s->hessian != BMPC_HESSIAN_GAUSS_NEWTON && s->hessian != BMPC_HESSIAN_EXACT)
        return fail(BMPC_ERR_INVALID_ARG, "unknown Hessian choice %d", s->hessian);
    if (s->hessian == BMPC_HESSIAN_EXACT && !(s->eig_floor > 0.0 && s->eig_floor < INFINITY))
        return fail(BMPC_ERR_INVALID_ARG, "eig_floor must be positive and finite");
    if (s->riccati_variant != BMPC_RICCATI_AUTO && s->riccati_variant != BMPC_RICCATI_LEVEL &&
        s->riccati_variant != BMPC_RICCATI_SEGSCAN)
        return fail(BMPC_ERR_INVALID_ARG, "unknown Riccati variant %d", s->riccati_variant);
    if (warm < 0 || warm > 31) return fail(BMPC_ERR_INVALID_ARG, "warm bits %d outside [0, 31]", warm);
    if (s->block_size != 0 && s->block_size != 64 && s->block_size != 128 && s->block_size != 256 &&
        s->block_size != BMPC_BLOCK_GRID)
        return fail(BMPC_ERR_INVALID_ARG, "block_size must be 0, 64, 128, 256 or BMPC_BLOCK_GRID");
    int variant = s->riccati_variant, block = s->block_size;
    hipStream_t st = (hipStream_t)stream;
    const SolverCfg cfg = to_cfg(*s, warm);
    if (block == BMPC_BLOCK_GRID) {
        if (b->count != 1) return fail(BMPC_ERR_INVALID_ARG, "the whole-grid solver takes a batch of one problem");
        if (variant == BMPC_RICCATI_SEGSCAN)
            return fail(BMPC_ERR_UNSUPPORTED, "the whole-grid solver uses the level-parallel backward pass");
        return launch_grid_solver(b, cfg, st);
    }
    // a single large problem: the whole grid works on it
    if (b->count == 1 && b->total_nodes >= GRID_MIN_NODES && variant != BMPC_RICCATI_SEGSCAN && block == 0)
        return launch_grid_solver(b, cfg, st);
    if (variant == BMPC_RICCATI_AUTO) variant = b->tuned_variant ? b->tuned_variant : BMPC_RICCATI_LEVEL;
    if (block == 0) block = b->tuned_block ? b->tuned_block : 256;
    const WgKernel* k = find_wg(block, variant == BMPC_RICCATI_SEGSCAN);
    return launch_solver(b, *k, cfg, st);
}

}  // extern "C"

// The tuning criterion: launch time divided by the inner iterations summed
// over the batch.  Candidates sum reductions in different orders, so their
// iterates can part by rounding and take different iteration counts (a
// problem that does not converge can run far longer on one candidate than on
// another); the time per iteration compares the kernels' speed, not those
// paths.
struct TuneRig {
    bmpc_batch* b;
    SolverCfg cfg;
    hipStream_t st;
    double* saved = nullptr;
    size_t bytes = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<SolveOut> outs;

    bmpc_status open()
    {
        bytes = sizeof(double) * (size_t)b->total_nodes * 15;
        if (hipMalloc(&saved, bytes) != hipSuccess) return fail(BMPC_ERR_OOM, "no memory to save the batch state");
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
            hipMemcpyAsync(saved, b->d_state, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return fail(BMPC_ERR_HIP, "setting up the tuning runs failed");
        outs.resize(b->count);
        return BMPC_OK;
    }
    // one solve of the batch with kernel k from the saved state
    bmpc_status run(const WgKernel& k, double* ms, double* iters)
    {
        float t = 0.f;
        if (hipMemcpyAsync(b->d_state, saved, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipEventRecord(e0, st) != hipSuccess)
            return fail(BMPC_ERR_HIP, "tuning run failed");
        if (launch_solver(b, k, cfg, st) != BMPC_OK || hipEventRecord(e1, st) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess ||
            hipMemcpy(outs.data(), b->d_out, sizeof(SolveOut) * b->count, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(BMPC_ERR_HIP, "tuning run of %s failed", k.name);
        double it = 0.0;
        for (const auto& o : outs) it += o.inner_it;
        *ms = t;
        *iters = std::max(it, 1.0);
        return BMPC_OK;
    }
    bmpc_status close(bmpc_status rc)
    {
        if (saved && (hipMemcpyAsync(b->d_state, saved, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                      hipStreamSynchronize(st) != hipSuccess) && rc == BMPC_OK)
            rc = fail(BMPC_ERR_HIP, "restoring the batch state failed");
        (void)hipFree(saved);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return rc;
    }
};

constexpr int NUM_WG_KERNELS = sizeof(kWgKernels) / sizeof(kWgKernels[0]);

static void keep_choice(bmpc_batch* b, const WgKernel& k)
{
    b->tuned_variant = k.segscan ? BMPC_RICCATI_SEGSCAN : BMPC_RICCATI_LEVEL;
    b->tuned_block = k.block;
}

static bmpc_status check_tune_args(const bmpc_batch* b, const bmpc_settings* s, int32_t warm)
{
    if (!b || !s) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    if (warm < 0 || warm > 31) return fail(BMPC_ERR_INVALID_ARG, "warm bits %d outside [0, 31]", warm);
    if (s->n_alpha < 1 || s->n_alpha > NALPHA_MAX)
        return fail(BMPC_ERR_INVALID_ARG, "n_alpha must be in [1, %d]", NALPHA_MAX);
    if (s->ls_rounds < 1 || s->ls_rounds > LS_ROUNDS_MAX)
        return fail(BMPC_ERR_INVALID_ARG, "ls_rounds must be in [1, %d]", LS_ROUNDS_MAX);
    if (s->hessian != BMPC_HESSIAN_GAUSS_NEWTON && s->hessian != BMPC_HESSIAN_EXACT)
        return fail(BMPC_ERR_INVALID_ARG, "unknown Hessian choice %d", s->hessian);
    if (s->hessian == BMPC_HESSIAN_EXACT && !(s->eig_floor > 0.0 && s->eig_floor < INFINITY))
        return fail(BMPC_ERR_INVALID_ARG, "eig_floor must be positive and finite");
    return BMPC_OK;
}

// Key of a batch's shape for the tuning cache: FNV-1a over the problem
// count, the warm bits and each problem's node count, depth, leaf count and
// segment count, in batch order.
static unsigned long long shape_key(const bmpc_batch* b, int warm)
{
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&](long long v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (unsigned long long)((v >> (8 * i)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix(b->count);
    mix(warm);
    for (const bmpc_problem* p : b->problems) {
        mix(p->N);
        mix(p->tree->h.depth);
        mix((long long)p->tree->h.leaves.size());
        mix((long long)p->tree->h.seg_start.size());
    }
    return h;
}

extern "C" {

BMPC_API bmpc_status bmpc_batch_tune(bmpc_batch* b, const bmpc_settings* s, int32_t warm, int32_t reps,
                                     int32_t* variant_out, int32_t* block_out, double* ms_out, void* stream)
{
    bmpc_status rc = check_tune_args(b, s, warm);
    if (rc != BMPC_OK) return rc;
    if (reps < 1 || reps > 100) return fail(BMPC_ERR_INVALID_ARG, "reps must be in [1, 100]");
    TuneRig rig{b, to_cfg(*s, warm), (hipStream_t)stream};
    const WgKernel* best = nullptr;
    double best_t = INFINITY;
    if ((rc = rig.open()) == BMPC_OK) {
        for (int idx = 0; idx < NUM_WG_KERNELS && rc == BMPC_OK; ++idx) {
            double ms_sum = 0.0, it_sum = 0.0;
            for (int r = 0; r < reps && rc == BMPC_OK; ++r) {
                double ms = 0.0, it = 0.0;
                rc = rig.run(kWgKernels[idx], &ms, &it);
                ms_sum += ms;
                it_sum += it;
            }
            const double per_it = ms_sum / it_sum;
            if (ms_out) ms_out[idx] = per_it;
            if (per_it < best_t) {
                best_t = per_it;
                best = &kWgKernels[idx];
            }
        }
    }
    if (rc == BMPC_OK && best) {
        keep_choice(b, *best);
        if (variant_out) *variant_out = b->tuned_variant;
        if (block_out) *block_out = b->tuned_block;
    }
    return rig.close(rc);
}

BMPC_API bmpc_status bmpc_batch_autotune(bmpc_batch* b, const bmpc_settings* s, int32_t warm, int32_t budget_ms,
                                         const char* cache_path, int32_t* variant_out, int32_t* block_out,
                                         double* ms_per_iter_out, int32_t* from_cache, void* stream)
{
    bmpc_status rc = check_tune_args(b, s, warm);
    if (rc != BMPC_OK) return rc;
    if (budget_ms < 0) return fail(BMPC_ERR_INVALID_ARG, "budget_ms must be >= 0");
    const unsigned long long key = shape_key(b, warm);
    char keytxt[32];
    snprintf(keytxt, sizeof keytxt, "%016llx", key);
    if (from_cache) *from_cache = 0;
    // a cached choice for this shape: the last matching line wins
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "r")) {
            char line[256], k[64];
            int v = 0, blk = 0, found = 0;
            double t = 0.0, best_t = 0.0;
            while (fgets(line, sizeof line, f)) {
                int vv = 0, bb = 0;
                if (sscanf(line, "bmpc-autotune %63s %d %d %lf", k, &vv, &bb, &t) == 4 && strcmp(k, keytxt) == 0 &&
                    find_wg(bb, vv == BMPC_RICCATI_SEGSCAN) &&
                    (vv == BMPC_RICCATI_LEVEL || vv == BMPC_RICCATI_SEGSCAN)) {
                    v = vv;
                    blk = bb;
                    best_t = t;
                    found = 1;
                }
            }
            fclose(f);
            if (found) {
                keep_choice(b, *find_wg(blk, v == BMPC_RICCATI_SEGSCAN));
                if (variant_out) *variant_out = b->tuned_variant;
                if (block_out) *block_out = b->tuned_block;
                if (ms_per_iter_out) *ms_per_iter_out = best_t;
                if (from_cache) *from_cache = 1;
                return BMPC_OK;
            }
        }
    }
    // every candidate once, then further rounds over all of them while the
    // budget lasts (at most 100 runs each)
    TuneRig rig{b, to_cfg(*s, warm), (hipStream_t)stream};
    double ms_sum[NUM_WG_KERNELS] = {}, it_sum[NUM_WG_KERNELS] = {};
    if ((rc = rig.open()) == BMPC_OK) {
        const auto t0 = std::chrono::steady_clock::now();
        for (int round = 0; round < 100 && rc == BMPC_OK; ++round) {
            if (round > 0 && std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                                     .count() >= budget_ms)
                break;
            for (int idx = 0; idx < NUM_WG_KERNELS && rc == BMPC_OK; ++idx) {
                double ms = 0.0, it = 0.0;
                rc = rig.run(kWgKernels[idx], &ms, &it);
                ms_sum[idx] += ms;
                it_sum[idx] += it;
            }
        }
    }
    rc = rig.close(rc);
    if (rc != BMPC_OK) return rc;
    int best = 0;
    for (int idx = 1; idx < NUM_WG_KERNELS; ++idx)
        if (ms_sum[idx] / it_sum[idx] < ms_sum[best] / it_sum[best]) best = idx;
    keep_choice(b, kWgKernels[best]);
    const double per_it = ms_sum[best] / it_sum[best];
    if (variant_out) *variant_out = b->tuned_variant;
    if (block_out) *block_out = b->tuned_block;
    if (ms_per_iter_out) *ms_per_iter_out = per_it;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (!f) return fail(BMPC_ERR_INVALID_ARG, "cannot append to the tuning cache %s", cache_path);
        fprintf(f, "bmpc-autotune %s %d %d %.9g\n", keytxt, b->tuned_variant, b->tuned_block, per_it);
        fclose(f);
    }
    return BMPC_OK;
}

BMPC_API int32_t bmpc_batch_tune_candidates(int32_t* variants, int32_t* blocks, int32_t cap)
{
    int n = 0;
    for (const auto& k : kWgKernels) {
        if (n < cap) {
            if (variants) variants[n] = k.segscan ? BMPC_RICCATI_SEGSCAN : BMPC_RICCATI_LEVEL;
            if (blocks) blocks[n] = k.block;
        }
        ++n;
    }
    return n;
}

BMPC_API bmpc_status bmpc_batch_stats(bmpc_batch* b, bmpc_stats* stats, void* stream)
{
    if (!b || !stats) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    BMPC_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    std::vector<SolveOut> o(b->count);
    BMPC_HIP_TRY(hipMemcpy(o.data(), b->d_out, sizeof(SolveOut) * b->count, hipMemcpyDeviceToHost));
    int dev = 0, khz = 0;
    BMPC_HIP_TRY(hipGetDevice(&dev));
    BMPC_HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    int worst = BMPC_OK;
    for (int i = 0; i < b->count; ++i) {
        for (int k = 0; k < PH_COUNT; ++k) stats[i].time_ms[k] = khz > 0 ? (double)o[i].ticks[k] / khz : 0.0;
        stats[i].status = o[i].status;
        stats[i].outer_it = o[i].outer_it;
        stats[i].inner_it = o[i].inner_it;
        stats[i].ls_failures = o[i].ls_failures;
        stats[i].bad_node = o[i].bad_node;
        stats[i].start = o[i].start;
        stats[i].r_kkt = o[i].r_kkt;
        stats[i].viol = o[i].viol;
        stats[i].rho = o[i].rho;
        stats[i].mu = o[i].mu;
        stats[i].merit = o[i].merit;
        if (o[i].status != BMPC_OK && worst == BMPC_OK) worst = o[i].status;
    }
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_batch_state(bmpc_batch* b, int32_t i, double* x, double* u, double* lam, double* ye,
                                      int32_t into_batch, void* stream)
{
    if (!b || i < 0 || i >= b->count) return fail(BMPC_ERR_INVALID_ARG, "bad instance index");
    hipStream_t st = (hipStream_t)stream;
    const InstDesc& d = b->h_desc[i];
    const size_t N = d.N;
    struct {
        double* ext;
        double* in;
        size_t n;
    } parts[4] = {{x, d.x, 4 * N}, {u, d.u, 2 * N}, {lam, d.lam, 4 * N}, {ye, d.ye, 5 * N}};
    for (auto& pt : parts) {
        if (!pt.ext) continue;
        if (into_batch)
            BMPC_HIP_TRY(hipMemcpyAsync(pt.in, pt.ext, sizeof(double) * pt.n, hipMemcpyDeviceToDevice, st));
        else
            BMPC_HIP_TRY(hipMemcpyAsync(pt.ext, pt.in, sizeof(double) * pt.n, hipMemcpyDeviceToDevice, st));
    }
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_batch_state_all(bmpc_batch* b, double* x, double* u, double* lam, double* ye,
                                          int32_t into_batch, void* stream)
{
    if (!b) return fail(BMPC_ERR_INVALID_ARG, "batch is NULL");
    hipStream_t st = (hipStream_t)stream;
    const size_t T = (size_t)b->total_nodes;
    struct {
        double* ext;
        double* in;
        size_t n;
    } parts[4] = {{x, b->d_state, 4 * T}, {u, b->d_state + 4 * T, 2 * T}, {lam, b->d_state + 6 * T, 4 * T},
                  {ye, b->d_state + 10 * T, 5 * T}};
    for (auto& pt : parts) {
        if (!pt.ext) continue;
        if (into_batch)
            BMPC_HIP_TRY(hipMemcpyAsync(pt.in, pt.ext, sizeof(double) * pt.n, hipMemcpyDeviceToDevice, st));
        else
            BMPC_HIP_TRY(hipMemcpyAsync(pt.ext, pt.in, sizeof(double) * pt.n, hipMemcpyDeviceToDevice, st));
    }
    return BMPC_OK;
}

BMPC_API int64_t bmpc_batch_total_nodes(const bmpc_batch* b) { return b ? b->total_nodes : 0; }

BMPC_API bmpc_status bmpc_batch_start_from_network(bmpc_batch* b, const float* Y, int32_t rows, int32_t width,
                                                   void* stream)
{
    if (!b || !Y) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    if (rows < 1 || rows > b->count) return fail(BMPC_ERR_INVALID_ARG, "rows %d outside [1, %d]", rows, b->count);
    for (int i = 0; i < rows; ++i) {
        const int w = 6 * b->problems[i]->n_control + b->problems[i]->n_obs;
        if (w != width)
            return fail(BMPC_ERR_INVALID_ARG, "problem %d needs %d network outputs, got %d", i, w, width);
    }
    hipStream_t st = (hipStream_t)stream;
    {
        ProfScope ps("bmpc_start_from_network", st);
        hipLaunchKernelGGL(k_start_from_outputs<256>, dim3(rows), dim3(256), 0, st, b->d_desc, Y, width);
    }
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_batch_shift(bmpc_batch* b, void* stream)
{
    if (!b) return fail(BMPC_ERR_INVALID_ARG, "batch is NULL");
    hipStream_t st = (hipStream_t)stream;
    {
        ProfScope ps("bmpc_shift", st);
        hipLaunchKernelGGL(k_bmpc_shift<256>, dim3(b->count), dim3(256), 0, st, b->d_desc, MeasuredX0{{0, 0, 0, 0}, 0});
    }
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_warm_shift(bmpc_problem* p, double* x, double* u, double* lam, double* ye,
                                     const double* x0_new, void* stream)
{
    if (!p || !x || !u || !lam || !ye) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    MeasuredX0 m{{0, 0, 0, 0}, 0};
    if (x0_new) {
        for (int a = 0; a < 4; ++a) {
            if (!std::isfinite(x0_new[a])) return fail(BMPC_ERR_NONFINITE, "x0_new has a non-finite entry");
            m.v[a] = x0_new[a];
        }
        m.use = 1;
    }
    bmpc_status st;
    if (!p->self) {
        bmpc_problem* one[1] = {p};
        if ((st = bmpc_batch_create(one, 1, 0, &p->self)) != BMPC_OK) return st;
    }
    if ((st = bmpc_batch_state(p->self, 0, x, u, lam, ye, 1, stream)) != BMPC_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    {
        ProfScope ps("bmpc_shift", sm);
        hipLaunchKernelGGL(k_bmpc_shift<256>, dim3(1), dim3(256), 0, sm, p->self->d_desc, m);
    }
    BMPC_HIP_TRY(hipGetLastError());
    return bmpc_batch_state(p->self, 0, x, u, lam, ye, 0, stream);
}

BMPC_API bmpc_status bmpc_batch_history(bmpc_batch* b, int32_t i, double* hist, void* stream)
{
    if (!b || i < 0 || i >= b->count || !hist) return fail(BMPC_ERR_INVALID_ARG, "bad argument");
    if (!b->d_hist) return fail(BMPC_ERR_INVALID_ARG, "batch was created without history");
    BMPC_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    BMPC_HIP_TRY(hipMemcpy(hist, b->d_hist + (size_t)i * b->hist_cap * 6, sizeof(double) * b->hist_cap * 6,
                           hipMemcpyDeviceToHost));
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_solve(bmpc_problem* p, const bmpc_settings* s, int32_t warm, double* x, double* u,
                                double* lam, double* ye, bmpc_stats* stats, void* stream)
{
    if (!p || !s || !x || !u || !lam || !ye || !stats) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    bmpc_status st;
    if (!p->self) {
        bmpc_problem* one[1] = {p};
        if ((st = bmpc_batch_create(one, 1, 0, &p->self)) != BMPC_OK) return st;
    }
    if (warm && (st = bmpc_batch_state(p->self, 0, (warm & 1) ? x : nullptr, (warm & (1 | 8)) ? u : nullptr,
                                       (warm & 2) ? lam : nullptr, (warm & 4) ? ye : nullptr, 1, stream)) != BMPC_OK)
        return st;
    if ((st = bmpc_batch_launch(p->self, s, warm, stream)) != BMPC_OK) return st;
    if ((st = bmpc_batch_state(p->self, 0, x, u, lam, ye, 0, stream)) != BMPC_OK) return st;
    if ((st = bmpc_batch_stats(p->self, stats, stream)) != BMPC_OK) return st;
    if (stats->status != BMPC_OK) {
        if (stats->status == BMPC_ERR_NOT_PD)
            return fail(BMPC_ERR_NOT_PD, "Riccati Hessian not positive definite at node %d", stats->bad_node);
        return fail(stats->status, "solver stopped with status %d after %d inner iterations", stats->status,
                    stats->inner_it);
    }
    return BMPC_OK;
}

}  // extern "C"

// Workspace rows of bmpc_linearize_noalloc: one file-scope device array per
// GPU, NOALLOC_MAX_NODES rows of W_NODE doubles (3.4 MB), held until the
// process ends.  Host code never uses the array's name as an address: the
// device address of each GPU's copy is looked up once with that device
// current and kept per device.
constexpr int NOALLOC_MAX_NODES = BMPC_NOALLOC_MAX_NODES;
static __device__ __align__(256) double scratch[(size_t)NOALLOC_MAX_NODES * W_NODE];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of this GPU's scratch array (looked up on the first call
// on the device, with it current).
static bmpc_status scratch_for_current_device(double** out)
{
    int dev = 0;
    BMPC_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(BMPC_ERR_UNSUPPORTED, "device %d beyond the %d devices with a scratch array", dev,
                    NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(BMPC_ERR_HIP, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return BMPC_OK;
}

extern "C" {

static bmpc_status linearize_impl(bmpc_problem* p, int hess, double eig_floor, const double* x, const double* u,
                                  const double* lam, const double* ye, double rho, double* A, double* B, double* c,
                                  double* Q, double* R, double* M, double* q, double* r, double* kkt_viol,
                                  void* stream)
{
    if (!p || !x || !u || !lam || !ye || !A || !B || !c || !Q || !R || !q || !r || (hess && !M))
        return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    if (!(rho > 0.0)) return fail(BMPC_ERR_INVALID_ARG, "rho must be positive");
    if (hess && !(eig_floor > 0.0 && eig_floor < INFINITY))
        return fail(BMPC_ERR_INVALID_ARG, "eig_floor must be positive and finite");
    bmpc_status st;
    if (!p->self) {
        bmpc_problem* one[1] = {p};
        if ((st = bmpc_batch_create(one, 1, 0, &p->self)) != BMPC_OK) return st;
    }
    hipStream_t sm = (hipStream_t)stream;
    if ((st = bmpc_batch_state(p->self, 0, const_cast<double*>(x), const_cast<double*>(u),
                               const_cast<double*>(lam), const_cast<double*>(ye), 1, stream)) != BMPC_OK)
        return st;
    const InstDesc& d = p->self->h_desc[0];
    if (kkt_viol && !p->d_kkt && !dalloc(&p->d_kkt, 2))
        return fail(BMPC_ERR_OOM, "device allocation for the KKT residual failed");
    double* kk = kkt_viol ? p->d_kkt : nullptr;
    {
        ProfScope ps("bmpc_linearise", sm);
        hipLaunchKernelGGL(k_bmpc_linearise<256>, dim3(1), dim3(256), 0, sm, d, rho, kk, hess, eig_floor);
    }
    BMPC_HIP_TRY(hipGetLastError());
    // unpack the workspace rows into the caller's node-major arrays
    const size_t N = d.N;
    const size_t pitch = sizeof(double) * W_NODE;
    struct {
        double* dst;
        int off, w;
    } parts[8] = {{A, W_A, 16}, {B, W_B, 8}, {c, W_C, 4}, {Q, W_Q, 16}, {R, W_R, 4}, {q, W_QV, 4}, {r, W_RV, 2},
                  {M, W_M, 8}};
    for (auto& pt : parts)
        if (pt.dst)
            BMPC_HIP_TRY(hipMemcpy2DAsync(pt.dst, sizeof(double) * pt.w, d.ws + pt.off, pitch,
                                          sizeof(double) * pt.w, N, hipMemcpyDeviceToDevice, sm));
    if (kkt_viol) {
        BMPC_HIP_TRY(hipMemcpyAsync(kkt_viol, kk, 2 * sizeof(double), hipMemcpyDeviceToHost, sm));
        BMPC_HIP_TRY(hipStreamSynchronize(sm));
    }
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_linearize(bmpc_problem* p, const double* x, const double* u, const double* lam,
                                    const double* ye, double rho, double* A, double* B, double* c, double* Q,
                                    double* R, double* q, double* r, double* kkt_viol, void* stream)
{
    return linearize_impl(p, 0, 0.0, x, u, lam, ye, rho, A, B, c, Q, R, nullptr, q, r, kkt_viol, stream);
}

BMPC_API bmpc_status bmpc_linearize_exact(bmpc_problem* p, double eig_floor, const double* x, const double* u,
                                          const double* lam, const double* ye, double rho, double* A, double* B,
                                          double* c, double* Q, double* R, double* M, double* q, double* r,
                                          double* kkt_viol, void* stream)
{
    return linearize_impl(p, 1, eig_floor, x, u, lam, ye, rho, A, B, c, Q, R, M, q, r, kkt_viol, stream);
}

BMPC_API bmpc_status bmpc_linearize_noalloc(const bmpc_problem* p, const double* x, const double* u,
                                            const double* lam, const double* ye, double rho, double* A, double* B,
                                            double* c, double* Q, double* R, double* q, double* r,
                                            double* kkt_viol, void* stream)
{
    if (!p || !x || !u || !lam || !ye || !A || !B || !c || !Q || !R || !q || !r)
        return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    if (!(rho > 0.0)) return fail(BMPC_ERR_INVALID_ARG, "rho must be positive");
    if (p->N > NOALLOC_MAX_NODES)
        return fail(BMPC_ERR_INVALID_ARG, "problem of %d nodes exceeds the %d nodes of the fixed workspace", p->N,
                    NOALLOC_MAX_NODES);
    double* ws = nullptr;
    bmpc_status st = scratch_for_current_device(&ws);
    if (st != BMPC_OK) return st;
    // the problem's own device data; the point and the workspace rows are
    // the caller's arrays and the scratch array (the kernel only reads x, u,
    // lam, ye)
    InstDesc d{};
    d.N = p->N;
    d.T = p->tree->h.depth;
    d.parent = p->tree->d.parent;
    d.child_off = p->tree->d.child_off;
    d.level_off = p->tree->d.level_off;
    d.weight = p->d_weight;
    d.ref = p->d_ref;
    d.obs = p->d_obs;
    d.has_obs = p->d_has;
    d.x0 = p->d_x0;
    d.prm = to_dev(p->prm);
    d.x = const_cast<double*>(x);
    d.u = const_cast<double*>(u);
    d.lam = const_cast<double*>(lam);
    d.ye = const_cast<double*>(ye);
    d.ws = ws;
    hipStream_t sm = (hipStream_t)stream;
    {
        ProfScope ps("bmpc_linearise", sm);
        hipLaunchKernelGGL(k_bmpc_linearise<256>, dim3(1), dim3(256), 0, sm, d, rho, kkt_viol, 0, 0.0);
    }
    BMPC_HIP_TRY(hipGetLastError());
    const size_t N = d.N;
    const size_t pitch = sizeof(double) * W_NODE;
    struct {
        double* dst;
        int off, w;
    } parts[7] = {{A, W_A, 16}, {B, W_B, 8}, {c, W_C, 4}, {Q, W_Q, 16}, {R, W_R, 4}, {q, W_QV, 4}, {r, W_RV, 2}};
    for (auto& pt : parts)
        BMPC_HIP_TRY(hipMemcpy2DAsync(pt.dst, sizeof(double) * pt.w, ws + pt.off, pitch, sizeof(double) * pt.w, N,
                                      hipMemcpyDeviceToDevice, sm));
    return BMPC_OK;
}

}  // extern "C"
