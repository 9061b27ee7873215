// Tree LQR on the GPU: backward tree Riccati and forward rollout.
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
// walked upwards by one worker (a lane, or a wavefront for larger nx); all
// nodes of one depth are therefore processed at the same time.  When a
// worker reaches a branching node it counts itself in with an atomic; the
// last child to arrive merges all children (always in child order, so the
// result is bitwise reproducible) and carries on upwards, the others stop.
//
// Forward (Sec. III-B, last paragraph; eq. forward_comb_rule): one lane per
// root-to-leaf path applies u = K x + k and x_j = A_j x + B_j u + c_j down its
// path; each node is written by exactly one lane (the path of the first leaf
// below it), which also writes the costate lam = P x + p.
#include <hip/hip_runtime.h>

#include <climits>

#include "bmpc_internal.hpp"
#include "lqr_device.hpp"
#include "profile.hpp"

namespace bmpc {

// ------------------------------------------------------------------------
// lane-per-segment backward
// ------------------------------------------------------------------------
template <int NX, int NU, int LAY>
__global__ void __launch_bounds__(64) k_bwd_lane(TreeDev t, LqrArgs a, int* arrive)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= t.num_leaves) return;
    const int N = t.N;
    int n = t.leaves[l];
    int from = -1;
    double P[NX][NX], p[NX];
    for (;;) {
        const int c0 = t.child_off[n], c1 = t.child_off[n + 1];
        if (c0 == c1) {
            leaf_value<NX, NU, LAY>(a, N, n, P, p);
        } else {
            const bool use_regs = (c1 - c0 == 1) && from == c0;
            riccati_node<NX, NU, LAY, false>(a, N, n, c0, c1, use_regs, P, p);
        }
        store_value<NX, LAY>(a, N, n, P, p);
        const int par = t.parent[n];
        if (par < 0) break;
        const int nsib = t.child_off[par + 1] - t.child_off[par];
        if (nsib > 1) {
            __threadfence();
            const int old = atomicAdd(&arrive[par], 1);
            if (old != nsib - 1) break;
            __threadfence();
        }
        from = n;
        n = par;
    }
}

// ------------------------------------------------------------------------
// wavefront-per-segment backward (LDS staging; used for larger nx)
// ------------------------------------------------------------------------
template <int NX, int NU, int LAY>
__global__ void __launch_bounds__(64) k_bwd_wave(TreeDev t, LqrArgs a, int* arrive)
{
    constexpr int NZ = NX + NU;       // rows of [A B]^T
    constexpr int ND = NX + NU + 1;   // columns of [A B c]
    __shared__ double sD[NX][ND];
    __shared__ double sP[NX][NX];
    __shared__ double sp[NX];
    __shared__ double sS[NX][ND];
    __shared__ double sZ[NZ][ND];
    __shared__ double sK[NU][NX + 1];
    __shared__ int sgo;

    const int l = blockIdx.x;
    const int lane = threadIdx.x;
    const int N = t.N;
    int n = t.leaves[l];
    int from = -1;
    for (;;) {
        const int c0 = t.child_off[n], c1 = t.child_off[n + 1];
        if (c0 == c1) {
            for (int e = lane; e < NX * NX; e += 64)
                sP[e / NX][e % NX] = a.Q[lidx<LAY>(n, e, NX * NX, N)];
            for (int e = lane; e < NX; e += 64) sp[e] = a.q[lidx<LAY>(n, e, NX, N)];
            for (int e = lane; e < NU * NX; e += 64) a.K[lidx<LAY>(n, e, NU * NX, N)] = 0.0;
            for (int e = lane; e < NU; e += 64) a.k[lidx<LAY>(n, e, NU, N)] = 0.0;
            __syncthreads();
        } else {
            // Z <- stage cost: rows 0..NX-1 hold [W . w], rows NX.. hold [G H g]
            for (int e = lane; e < NZ * ND; e += 64) {
                const int r = e / ND, col = e % ND;
                double v = 0.0;
                if (r < NX) {
                    if (col < NX) v = a.Q[lidx<LAY>(n, r * NX + col, NX * NX, N)];
                    else if (col == NZ) v = a.q[lidx<LAY>(n, r, NX, N)];
                } else {
                    const int ru = r - NX;
                    if (col < NX) v = a.M[lidx<LAY>(n, ru * NX + col, NU * NX, N)];
                    else if (col < NZ) v = a.R[lidx<LAY>(n, ru * NU + (col - NX), NU * NU, N)];
                    else v = a.r[lidx<LAY>(n, ru, NU, N)];
                }
                sZ[r][col] = v;
            }
            const bool use_lds = (c1 - c0 == 1) && from == c0;
            for (int j = c0; j < c1; ++j) {
                for (int e = lane; e < NX * ND; e += 64) {
                    const int r = e / ND, col = e % ND;
                    double v;
                    if (col < NX) v = a.A[lidx<LAY>(j, r * NX + col, NX * NX, N)];
                    else if (col < NZ) v = a.B[lidx<LAY>(j, r * NU + (col - NX), NX * NU, N)];
                    else v = a.c[lidx<LAY>(j, r, NX, N)];
                    sD[r][col] = v;
                }
                if (!use_lds) {
                    for (int e = lane; e < NX * NX; e += 64)
                        sP[e / NX][e % NX] = a.P[lidx<LAY>(j, e, NX * NX, N)];
                    for (int e = lane; e < NX; e += 64) sp[e] = a.p[lidx<LAY>(j, e, NX, N)];
                }
                __syncthreads();
                // S = P [A B c];  last column + p  ->  p + P c
                for (int e = lane; e < NX * ND; e += 64) {
                    const int r = e / ND, col = e % ND;
                    double acc = 0.0;
#pragma unroll
                    for (int k = 0; k < NX; ++k) acc += sP[r][k] * sD[k][col];
                    if (col == NZ) acc += sp[r];
                    sS[r][col] = acc;
                }
                __syncthreads();
                // Z += [A B]^T S on the blocks that are used
                for (int e = lane; e < NZ * ND; e += 64) {
                    const int r = e / ND, col = e % ND;
                    if (r < NX && col >= NX && col < NZ) continue;
                    double acc = 0.0;
#pragma unroll
                    for (int k = 0; k < NX; ++k) acc += sD[k][r] * sS[k][col];
                    sZ[r][col] += acc;
                }
                __syncthreads();
            }
            // gains: lane i < NX solves column i of K, lane NX solves k
            if (lane <= NX) {
                double L[NU][NU];
#pragma unroll
                for (int i = 0; i < NU; ++i)
#pragma unroll
                    for (int j = 0; j < NU; ++j) L[i][j] = sZ[NX + i][NX + j];
                const bool ok = chol_inplace<NU>(L);
                if (!ok) atomicMin(a.bad, n);
                double v[NU];
                const int col = lane < NX ? lane : NZ;
#pragma unroll
                for (int i = 0; i < NU; ++i) v[i] = sZ[NX + i][col];
                chol_solve<NU>(L, v);
#pragma unroll
                for (int i = 0; i < NU; ++i) sK[i][lane] = -v[i];
            }
            __syncthreads();
            for (int e = lane; e < NU * NX; e += 64)
                a.K[lidx<LAY>(n, e, NU * NX, N)] = sK[e / NX][e % NX];
            for (int e = lane; e < NU; e += 64) a.k[lidx<LAY>(n, e, NU, N)] = sK[e][NX];
            // P = sym(W + G^T K), p = w + G^T k   (child P in sP no longer needed)
            double pv[(NX * NX + 63) / 64];
            double qv[(NX + 63) / 64];
#pragma unroll
            for (int s = 0; s < (NX * NX + 63) / 64; ++s) {
                const int e = lane + 64 * s;
                if (e < NX * NX) {
                    const int i = e / NX, j = e % NX;
                    double xij = sZ[i][j], xji = sZ[j][i];
                    double tij = 0.0, tji = 0.0;
#pragma unroll
                    for (int r = 0; r < NU; ++r) {
                        tij += sZ[NX + r][i] * sK[r][j];
                        tji += sZ[NX + r][j] * sK[r][i];
                    }
                    pv[s] = 0.5 * ((xij + tij) + (xji + tji));
                }
            }
#pragma unroll
            for (int s = 0; s < (NX + 63) / 64; ++s) {
                const int i = lane + 64 * s;
                if (i < NX) {
                    double tt = 0.0;
#pragma unroll
                    for (int r = 0; r < NU; ++r) tt += sZ[NX + r][i] * sK[r][NX];
                    qv[s] = sZ[i][NZ] + tt;
                }
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < (NX * NX + 63) / 64; ++s) {
                const int e = lane + 64 * s;
                if (e < NX * NX) sP[e / NX][e % NX] = pv[s];
            }
#pragma unroll
            for (int s = 0; s < (NX + 63) / 64; ++s) {
                const int i = lane + 64 * s;
                if (i < NX) sp[i] = qv[s];
            }
            __syncthreads();
        }
        for (int e = lane; e < NX * NX; e += 64) a.P[lidx<LAY>(n, e, NX * NX, N)] = sP[e / NX][e % NX];
        for (int e = lane; e < NX; e += 64) a.p[lidx<LAY>(n, e, NX, N)] = sp[e];
        const int par = t.parent[n];
        if (par < 0) break;
        const int nsib = t.child_off[par + 1] - t.child_off[par];
        if (nsib > 1) {
            __threadfence();
            __syncthreads();
            if (lane == 0) sgo = (atomicAdd(&arrive[par], 1) == nsib - 1);
            __syncthreads();
            if (!sgo) break;
            __threadfence();
        }
        from = n;
        n = par;
    }
}

// ------------------------------------------------------------------------
// lane-per-path forward
// ------------------------------------------------------------------------
template <int NX, int NU, int LAY>
__global__ void __launch_bounds__(64) k_fwd_lane(TreeDev t, LqrArgs a, int* arrive)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= t.num_leaves) return;
    const int N = t.N, Z = t.num_leaves;
    const int last = t.leaf_stage[l];
    double x[NX], u[NU];
#pragma unroll
    for (int i = 0; i < NX; ++i) x[i] = a.x0[i];
    for (int s = 0; s <= last; ++s) {
        const int n = t.path[(long)s * Z + l];
        const bool writer = t.first_leaf[n] == l;
        if (writer) {
            arrive[n] = 0;
#pragma unroll
            for (int i = 0; i < NX; ++i) a.x[lidx<LAY>(n, i, NX, N)] = x[i];
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                double acc = a.p[lidx<LAY>(n, i, NX, N)];
#pragma unroll
                for (int j = 0; j < NX; ++j) acc += a.P[lidx<LAY>(n, i * NX + j, NX * NX, N)] * x[j];
                a.lam[lidx<LAY>(n, i, NX, N)] = acc;
            }
        }
        if (s == last) {
            if (writer)
#pragma unroll
                for (int i = 0; i < NU; ++i) a.u[lidx<LAY>(n, i, NU, N)] = 0.0;
            break;
        }
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            double acc = a.k[lidx<LAY>(n, i, NU, N)];
#pragma unroll
            for (int j = 0; j < NX; ++j) acc += a.K[lidx<LAY>(n, i * NX + j, NU * NX, N)] * x[j];
            u[i] = acc;
        }
        if (writer)
#pragma unroll
            for (int i = 0; i < NU; ++i) a.u[lidx<LAY>(n, i, NU, N)] = u[i];
        const int m = t.path[(long)(s + 1) * Z + l];
        double xn[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            double acc = a.c[lidx<LAY>(m, i, NX, N)];
#pragma unroll
            for (int j = 0; j < NX; ++j) acc += a.A[lidx<LAY>(m, i * NX + j, NX * NX, N)] * x[j];
#pragma unroll
            for (int j = 0; j < NU; ++j) acc += a.B[lidx<LAY>(m, i * NU + j, NX * NU, N)] * u[j];
            xn[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) x[i] = xn[i];
    }
}

__global__ void k_init_flag(int* bad) { *bad = INT_MAX; }

// ------------------------------------------------------------------------
// dispatch
// ------------------------------------------------------------------------
struct LqrKernels {
    int nx, nu, layout;
    void (*bwd_lane)(TreeDev, LqrArgs, int*);
    void (*bwd_wave)(TreeDev, LqrArgs, int*);
    void (*fwd)(TreeDev, LqrArgs, int*);
};

template <int NX, int NU, int LAY, bool LANE>
static LqrKernels make_k()
{
    LqrKernels k{NX, NU, LAY, nullptr, k_bwd_wave<NX, NU, LAY>, k_fwd_lane<NX, NU, LAY>};
    if constexpr (LANE) k.bwd_lane = k_bwd_lane<NX, NU, LAY>;
    return k;
}

static const LqrKernels* find_kernels(int nx, int nu, int layout)
{
    static const LqrKernels table[] = {
        make_k<3, 1, 0, true>(),   make_k<3, 1, 1, true>(),
        make_k<4, 2, 0, true>(),   make_k<4, 2, 1, true>(),
        make_k<6, 3, 0, true>(),   make_k<6, 3, 1, true>(),
        make_k<12, 4, 0, false>(), make_k<12, 4, 1, false>(),
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
    int* bad = nullptr;
};

extern "C" {

BMPC_API int32_t bmpc_lqr_supported(int32_t nx, int32_t nu, int32_t variant)
{
    const LqrKernels* k = find_kernels(nx, nu, 0);
    if (!k) return 0;
    if (variant == BMPC_RICCATI_AUTO || variant == BMPC_RICCATI_LEVEL) return 1;
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
              hipMalloc(&pl->bad, sizeof(int)) == hipSuccess;
    if (!ok) {
        bmpc_lqr_plan_destroy(pl);
        return fail(BMPC_ERR_OOM, "device allocation for the LQR plan failed");
    }
    if (hipMemset(pl->arrive, 0, sizeof(int) * N) != hipSuccess ||
        hipMemset(pl->bad, 0x7f, sizeof(int)) != hipSuccess) {
        bmpc_lqr_plan_destroy(pl);
        return fail(BMPC_ERR_HIP, "hipMemset failed");
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
    if (variant != BMPC_RICCATI_AUTO && variant != BMPC_RICCATI_LEVEL)
        return fail(BMPC_ERR_UNSUPPORTED, "Riccati variant %d is not available for the tree LQR",
                    variant);
    hipStream_t s = (hipStream_t)stream;
    LqrArgs a{A, B, c, Q, R, M, q, r, x0, x, u, lam, K ? K : pl->K, k ? k : pl->k,
              P ? P : pl->P, p ? p : pl->p, pl->bad};
    const TreeDev& t = pl->tree->d;
    const int Z = t.num_leaves;
    hipLaunchKernelGGL(k_init_flag, dim3(1), dim3(1), 0, s, pl->bad);
    const bool lane = pl->kern->bwd_lane != nullptr && pl->nx <= 6;
    if (lane) {
        ProfScope ps("lqr_backward_level_lane", s);
        hipLaunchKernelGGL(pl->kern->bwd_lane, dim3((Z + 63) / 64), dim3(64), 0, s, t, a, pl->arrive);
    } else {
        ProfScope ps("lqr_backward_level_wave", s);
        hipLaunchKernelGGL(pl->kern->bwd_wave, dim3(Z), dim3(64), 0, s, t, a, pl->arrive);
    }
    {
        ProfScope ps("lqr_forward_paths", s);
        hipLaunchKernelGGL(pl->kern->fwd, dim3((Z + 63) / 64), dim3(64), 0, s, t, a, pl->arrive);
    }
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_lqr_check(bmpc_lqr_plan* pl, int32_t* bad_node, void* stream)
{
    if (!pl) return fail(BMPC_ERR_INVALID_ARG, "plan is NULL");
    BMPC_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int bad = 0;
    BMPC_HIP_TRY(hipMemcpy(&bad, pl->bad, sizeof(int), hipMemcpyDeviceToHost));
    if (bad_node) *bad_node = bad == INT_MAX ? -1 : bad;
    if (bad != INT_MAX)
        return fail(BMPC_ERR_NOT_PD, "Riccati Hessian not positive definite at node %d", bad);
    return BMPC_OK;
}

}  // extern "C"
