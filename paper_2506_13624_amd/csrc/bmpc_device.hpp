// Device math of the branch-MPC problem: kinematic-bicycle RK4 step with
// its Jacobians, node terms of the augmented Lagrangian and their
// Gauss-Newton quadratisation.
#pragma once

#include <hip/hip_runtime.h>

namespace bmpc {

struct BikeParams {
    double L, dt;
    double Qd[4], Rd[2];
    double a_max, steer_max, obs_r;
};

constexpr int BX = 4;  // state [px, py, psi, v]
constexpr int BU = 2;  // input [a, delta]
constexpr int BG = 5;  // constraint slots: u0 <= a_max, -u0 <= a_max, u1 <= s_max, -u1 <= s_max, obstacle

// Continuous-time bicycle  d/dt [px,py,psi,v] = [v cos psi, v sin psi, v tan(delta)/L, a].
__device__ __forceinline__ void bike_rhs(double L, const double (&x)[BX], const double (&u)[BU],
                                         double (&f)[BX])
{
    double s, c;
    sincos(x[2], &s, &c);
    f[0] = x[3] * c;
    f[1] = x[3] * s;
    f[2] = x[3] * tan(u[1]) / L;
    f[3] = u[0];
}

// Same, with the directional derivative along (dx, du).
__device__ __forceinline__ void bike_rhs_tangent(double L, const double (&x)[BX], const double (&u)[BU],
                                                 double tan_delta, double sec2, const double (&dx)[BX],
                                                 const double (&du)[BU], double (&df)[BX])
{
    double s, c;
    sincos(x[2], &s, &c);
    df[0] = dx[3] * c - x[3] * s * dx[2];
    df[1] = dx[3] * s + x[3] * c * dx[2];
    df[2] = (dx[3] * tan_delta + x[3] * sec2 * du[1]) / L;
    df[3] = du[0];
}

// One RK4 step x+ = F(x, u) (input held over the step).
__device__ __forceinline__ void bike_step(const BikeParams& P, const double (&x)[BX], const double (&u)[BU],
                                          double (&xn)[BX])
{
    const double h = P.dt;
    double k1[BX], k2[BX], k3[BX], k4[BX], y[BX];
    bike_rhs(P.L, x, u, k1);
#pragma unroll
    for (int i = 0; i < BX; ++i) y[i] = x[i] + 0.5 * h * k1[i];
    bike_rhs(P.L, y, u, k2);
#pragma unroll
    for (int i = 0; i < BX; ++i) y[i] = x[i] + 0.5 * h * k2[i];
    bike_rhs(P.L, y, u, k3);
#pragma unroll
    for (int i = 0; i < BX; ++i) y[i] = x[i] + h * k3[i];
    bike_rhs(P.L, y, u, k4);
#pragma unroll
    for (int i = 0; i < BX; ++i) xn[i] = x[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

// RK4 step and its Jacobians A = dF/dx (4x4), B = dF/du (4x2), by forward
// propagation of the six unit tangent directions through the four stages.
__device__ __forceinline__ void bike_step_jac(const BikeParams& P, const double (&x)[BX], const double (&u)[BU],
                                              double (&xn)[BX], double (&A)[BX][BX], double (&B)[BX][BU])
{
    const double h = P.dt;
    const double tan_delta = tan(u[1]);
    const double cd = cos(u[1]);
    const double sec2 = 1.0 / (cd * cd);
    // stage points
    double y1[BX], y2[BX], y3[BX], y4[BX], k1[BX], k2[BX], k3[BX], k4[BX];
#pragma unroll
    for (int i = 0; i < BX; ++i) y1[i] = x[i];
    bike_rhs(P.L, y1, u, k1);
#pragma unroll
    for (int i = 0; i < BX; ++i) y2[i] = x[i] + 0.5 * h * k1[i];
    bike_rhs(P.L, y2, u, k2);
#pragma unroll
    for (int i = 0; i < BX; ++i) y3[i] = x[i] + 0.5 * h * k2[i];
    bike_rhs(P.L, y3, u, k3);
#pragma unroll
    for (int i = 0; i < BX; ++i) y4[i] = x[i] + h * k3[i];
    bike_rhs(P.L, y4, u, k4);
#pragma unroll
    for (int i = 0; i < BX; ++i) xn[i] = x[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    // tangents
#pragma unroll
    for (int d = 0; d < BX + BU; ++d) {
        double dx[BX] = {0.0, 0.0, 0.0, 0.0}, du[BU] = {0.0, 0.0};
        if (d < BX) dx[d] = 1.0;
        else du[d - BX] = 1.0;
        double t1[BX], t2[BX], t3[BX], t4[BX], dy[BX];
        bike_rhs_tangent(P.L, y1, u, tan_delta, sec2, dx, du, t1);
#pragma unroll
        for (int i = 0; i < BX; ++i) dy[i] = dx[i] + 0.5 * h * t1[i];
        bike_rhs_tangent(P.L, y2, u, tan_delta, sec2, dy, du, t2);
#pragma unroll
        for (int i = 0; i < BX; ++i) dy[i] = dx[i] + 0.5 * h * t2[i];
        bike_rhs_tangent(P.L, y3, u, tan_delta, sec2, dy, du, t3);
#pragma unroll
        for (int i = 0; i < BX; ++i) dy[i] = dx[i] + h * t3[i];
        bike_rhs_tangent(P.L, y4, u, tan_delta, sec2, dy, du, t4);
#pragma unroll
        for (int i = 0; i < BX; ++i) {
            const double v = dx[i] + (h / 6.0) * (t1[i] + 2.0 * t2[i] + 2.0 * t3[i] + t4[i]);
            if (d < BX) A[i][d] = v;
            else B[i][d - BX] = v;
        }
    }
}

// Node data of the augmented Lagrangian (PHR penalty on every active slot).
struct NodeData {
    double w;        // probability weight of the node
    double ref[BX];  // tracking reference
    double ox, oy;   // obstacle centre
    bool has_obs, leaf;
};

// Constraint values; inactive slots get -inf-like sentinel flags.
__device__ __forceinline__ void node_constraints(const BikeParams& P, const NodeData& nd, const double (&x)[BX],
                                                 const double (&u)[BU], double (&g)[BG], bool (&on)[BG],
                                                 double& dist, double& ex, double& ey)
{
#pragma unroll
    for (int s = 0; s < 4; ++s) on[s] = !nd.leaf;
    g[0] = u[0] - P.a_max;
    g[1] = -u[0] - P.a_max;
    g[2] = u[1] - P.steer_max;
    g[3] = -u[1] - P.steer_max;
    on[4] = nd.has_obs;
    ex = x[0] - nd.ox;
    ey = x[1] - nd.oy;
    dist = sqrt(ex * ex + ey * ey);
    g[4] = P.obs_r - dist;
}

// The kinematic bicycle is defined for steering angles inside (-pi/2, pi/2):
// tan(delta) has its pole at pi/2 and past it the yaw rate changes sign.  A
// point with a control outside is not a point of the problem (merit +inf).
__device__ __forceinline__ bool steer_in_domain(const double (&u)[BU])
{
    return fabs(u[1]) < 1.5707963267948966;
}

// Value of the node's augmented objective
//   w * (1/2 |x - ref|_Q^2 + 1/2 |u|_R^2) + rho/2 sum_active max(0, g + y/rho)^2.
__device__ __forceinline__ double node_value(const BikeParams& P, const NodeData& nd, const double (&x)[BX],
                                             const double (&u)[BU], const double (&ye)[BG], double rho)
{
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        const double e = x[i] - nd.ref[i];
        v += 0.5 * nd.w * P.Qd[i] * e * e;
    }
    if (!nd.leaf) {
#pragma unroll
        for (int i = 0; i < BU; ++i) v += 0.5 * nd.w * P.Rd[i] * u[i] * u[i];
    }
    double g[BG], dist, ex, ey;
    bool on[BG];
    node_constraints(P, nd, x, u, g, on, dist, ex, ey);
    double pen = 0.0;
#pragma unroll
    for (int s = 0; s < BG; ++s) {
        const double t = g[s] + ye[s] / rho;
        if (on[s] && t > 0.0) pen += t * t;
    }
    return v + 0.5 * rho * pen;
}

// Gradient and Gauss-Newton Hessian of the node's augmented objective:
//   q = w Q (x - ref) + rho * sum_active t grad_x g,  r = w R u + rho * sum_active t grad_u g,
//   Qh = w Q + rho * sum_active grad_x g grad_x g^T,  Rh = w R + rho * sum_active grad_u g grad_u g^T
// with t = g + y/rho and "active" meaning t > 0.  Returns the value.
__device__ __forceinline__ double node_quad(const BikeParams& P, const NodeData& nd, const double (&x)[BX],
                                            const double (&u)[BU], const double (&ye)[BG], double rho,
                                            double (&q)[BX], double (&r)[BU], double (&Qh)[BX][BX],
                                            double (&Rh)[BU][BU])
{
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        const double e = x[i] - nd.ref[i];
        v += 0.5 * nd.w * P.Qd[i] * e * e;
        q[i] = nd.w * P.Qd[i] * e;
#pragma unroll
        for (int j = 0; j < BX; ++j) Qh[i][j] = (i == j) ? nd.w * P.Qd[i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < BU; ++i) {
        r[i] = 0.0;
#pragma unroll
        for (int j = 0; j < BU; ++j) Rh[i][j] = 0.0;
    }
    if (!nd.leaf) {
#pragma unroll
        for (int i = 0; i < BU; ++i) {
            v += 0.5 * nd.w * P.Rd[i] * u[i] * u[i];
            r[i] = nd.w * P.Rd[i] * u[i];
            Rh[i][i] = nd.w * P.Rd[i];
        }
    }
    double g[BG], dist, ex, ey;
    bool on[BG];
    node_constraints(P, nd, x, u, g, on, dist, ex, ey);
    double pen = 0.0;
    // input bounds: slot 2k+s constrains u_k with sign +1 (s = 0) or -1 (s = 1)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double t = g[s] + ye[s] / rho;
        if (on[s] && t > 0.0) {
            const int k = s >> 1;
            const double sg = (s & 1) ? -1.0 : 1.0;
            pen += t * t;
            r[k] += rho * t * sg;
            Rh[k][k] += rho;
        }
    }
    {
        const double t = g[4] + ye[4] / rho;
        if (on[4] && t > 0.0) {
            // grad_p (r - |p - o|) = -(p - o)/|p - o|; at the centre use -e_x
            const double jx = dist > 0.0 ? -ex / dist : -1.0;
            const double jy = dist > 0.0 ? -ey / dist : 0.0;
            pen += t * t;
            q[0] += rho * t * jx;
            q[1] += rho * t * jy;
            Qh[0][0] += rho * jx * jx;
            Qh[0][1] += rho * jx * jy;
            Qh[1][0] += rho * jy * jx;
            Qh[1][1] += rho * jy * jy;
        }
    }
    return v + 0.5 * rho * pen;
}

}  // namespace bmpc
