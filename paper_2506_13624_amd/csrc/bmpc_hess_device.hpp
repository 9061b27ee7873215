// Exact node Hessian of the Lagrangian with eigenvalue modification
// (Sec. IV-A, search direction): the alternative to the Gauss-Newton model
// of bmpc_device.hpp.
//
// For node n the quadratic model's Hessian is that of
//   L_a,n(x_n, u_n) + sum_{j child of n} lam_j^T F(x_n, u_n),
// i.e. the Gauss-Newton blocks plus
//   - the curvature of the active obstacle penalty, rho t grad^2 g, where
//     g = r - |p - o|, t = g + y/rho and grad^2 g = -(I - e e^T) / |p - o|;
//   - the dynamics curvature mu^T grad^2 F with mu = sum of the children's
//     multipliers.
// Its eigenvalues are then raised to at least delta * max(1, largest
// |eigenvalue|): a floor relative to the block's scale keeps the modified
// block numerically positive definite whatever the penalty's size.
//
// Structure used here: the position (px, py) enters neither the bicycle's
// right-hand side nor the input bounds, and the state weight is diagonal,
// so the 6x6 Hessian over (px, py, psi, v, a, delta) is block diagonal,
// 2x2 (position: weights and obstacle) plus 4x4 (psi, v, a, delta:
// weights, input bounds and dynamics curvature).  The eigenvalue
// modification acts on each block by itself.
#pragma once

#include <hip/hip_runtime.h>

#include "bmpc_device.hpp"

namespace bmpc {

// Second-order jet over the four variables (psi, v, a, delta): value,
// gradient and the packed upper triangle of the Hessian.
struct Jet2 {
    double v, g[4], h[10];
};

__device__ __forceinline__ constexpr int jidx(int i, int j)
{
    return i <= j ? i * 4 - i * (i - 1) / 2 + (j - i) : j * 4 - j * (j - 1) / 2 + (i - j);
}

__device__ __forceinline__ Jet2 jet_var(int k, double v)
{
    Jet2 r{};
    r.v = v;
    r.g[k] = 1.0;
    return r;
}

// a + s b
__device__ __forceinline__ Jet2 jet_axpy(const Jet2& a, double s, const Jet2& b)
{
    Jet2 r;
    r.v = a.v + s * b.v;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.g[i] = a.g[i] + s * b.g[i];
#pragma unroll
    for (int i = 0; i < 10; ++i) r.h[i] = a.h[i] + s * b.h[i];
    return r;
}

__device__ __forceinline__ Jet2 jet_mul(const Jet2& a, const Jet2& b)
{
    Jet2 r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.g[i] = a.v * b.g[i] + b.v * a.g[i];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i; j < 4; ++j)
            r.h[jidx(i, j)] = a.v * b.h[jidx(i, j)] + b.v * a.h[jidx(i, j)] + a.g[i] * b.g[j] + a.g[j] * b.g[i];
    return r;
}

// phi(a) for a scalar function with phi(a.v) = f0, phi' = f1, phi'' = f2
__device__ __forceinline__ Jet2 jet_fn(const Jet2& a, double f0, double f1, double f2)
{
    Jet2 r;
    r.v = f0;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.g[i] = f1 * a.g[i];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i; j < 4; ++j) r.h[jidx(i, j)] = f1 * a.h[jidx(i, j)] + f2 * a.g[i] * a.g[j];
    return r;
}

// Packed Hessian over (psi, v, a, delta) of mu^T F(x, u), F the RK4 step.
// F = x + h/6 (k1 + 2 k2 + 2 k3 + k4) with k = [V cos Psi, V sin Psi,
// V tan(delta) / L, a] at the stage points; only Psi and V of a stage point
// enter k, and V = v + c h a is affine.
__device__ __forceinline__ void bike_step_hessian(const BikeParams& P, const double (&x)[BX], const double (&u)[BU],
                                                  const double (&mu)[BX], double (&H)[10])
{
    const double h = P.dt, iL = 1.0 / P.L;
    const Jet2 psi = jet_var(0, x[2]), v = jet_var(1, x[3]), a = jet_var(2, u[0]), dl = jet_var(3, u[1]);
    const double td = tan(dl.v), s2 = 1.0 + td * td;
    const Jet2 T = jet_fn(dl, td, s2, 2.0 * td * s2);
#pragma unroll
    for (int i = 0; i < 10; ++i) H[i] = 0.0;
    Jet2 Psi = psi;
    const double cst[4] = {0.0, 0.5, 0.5, 1.0}, wst[4] = {1.0, 2.0, 2.0, 1.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const Jet2 V = jet_axpy(v, cst[s] * h, a);
        double sp, cp;
        sincos(Psi.v, &sp, &cp);
        const Jet2 c = jet_fn(Psi, cp, -sp, -cp), sn = jet_fn(Psi, sp, cp, -sp);
        const Jet2 k0 = jet_mul(V, c), k1 = jet_mul(V, sn), k2 = jet_mul(V, T);
        const double f = wst[s] * h / 6.0;
#pragma unroll
        for (int i = 0; i < 10; ++i) H[i] += f * (mu[0] * k0.h[i] + mu[1] * k1.h[i] + mu[2] * iL * k2.h[i]);
        if (s < 3) Psi = jet_axpy(psi, cst[s + 1] * h * iL, k2);
    }
}

// Symmetric A = V diag(w) V^T by cyclic Jacobi rotations (each zeroes one
// off-diagonal pair) until the off-diagonal part is negligible: on return
// the diagonal of A holds w (the rest is rounding) and V the eigenvectors.
template <int n>
__device__ __forceinline__ void jacobi_eig(double (&A)[n][n], double (&V)[n][n])
{
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) V[i][j] = i == j ? 1.0 : 0.0;
#pragma unroll 1
    for (int sweep = 0; sweep < 16; ++sweep) {
        double off = 0.0, dia = 0.0;
#pragma unroll
        for (int i = 0; i < n; ++i) {
            dia += A[i][i] * A[i][i];
#pragma unroll
            for (int j = i + 1; j < n; ++j) off += A[i][j] * A[i][j];
        }
        if (!(off > 1e-32 * (dia + off))) break;
#pragma unroll
        for (int p = 0; p < n - 1; ++p)
#pragma unroll
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p][q];
                if (apq == 0.0) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
                const double t = copysign(1.0, th) / (fabs(th) + sqrt(1.0 + th * th));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                // A <- J^T A J, V <- V J with J the rotation in the (p, q) plane
#pragma unroll
                for (int k = 0; k < n; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
#pragma unroll
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
#pragma unroll
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
}

// A <- V diag(max(w, delta)) V^T from the output of jacobi_eig.
template <int n>
__device__ __forceinline__ void eig_rebuild(double (&A)[n][n], const double (&V)[n][n], double delta)
{
    double w[n];
#pragma unroll
    for (int i = 0; i < n; ++i) w[i] = fmax(A[i][i], delta);
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < n; ++k) acc += V[i][k] * w[k] * V[j][k];
            A[i][j] = acc;
        }
}

// Turn the Gauss-Newton blocks (Qh, Rh of node_quad) into the exact model
// with eigenvalue modification; M receives the cross block d2/du dx.
// mu: sum of the children's multipliers (unused at a leaf).
__device__ __forceinline__ void exact_node_model(const BikeParams& P, const NodeData& nd, const double (&x)[BX],
                                                 const double (&u)[BU], const double (&ye)[BG], double rho,
                                                 const double (&mu)[BX], double delta, double (&Qh)[BX][BX],
                                                 double (&Rh)[BU][BU], double (&Mh)[BU][BX])
{
    // position block: weights, obstacle Gauss-Newton term and its curvature
    double Pp[2][2] = {{Qh[0][0], Qh[0][1]}, {Qh[1][0], Qh[1][1]}};
    if (nd.has_obs) {
        const double ex = x[0] - nd.ox, ey = x[1] - nd.oy;
        const double dist = sqrt(ex * ex + ey * ey);
        const double t = (P.obs_r - dist) + ye[4] / rho;
        if (t > 0.0 && dist > 0.0) {
            const double e0 = ex / dist, e1 = ey / dist, f = -rho * t / dist;
            Pp[0][0] += f * (1.0 - e0 * e0);
            Pp[0][1] += f * (-e0 * e1);
            Pp[1][0] += f * (-e1 * e0);
            Pp[1][1] += f * (1.0 - e1 * e1);
        }
    }
    double Vp[2][2];
    jacobi_eig<2>(Pp, Vp);
#pragma unroll
    for (int i = 0; i < BU; ++i)
#pragma unroll
        for (int j = 0; j < BX; ++j) Mh[i][j] = 0.0;
    double big = fmax(1.0, fmax(fabs(Pp[0][0]), fabs(Pp[1][1])));
    if (nd.leaf) {
        // (psi, v) block: the diagonal weights
        big = fmax(big, fmax(fabs(Qh[2][2]), fabs(Qh[3][3])));
        const double fl = delta * big;
        eig_rebuild<2>(Pp, Vp, fl);
        Qh[0][0] = Pp[0][0];
        Qh[0][1] = Pp[0][1];
        Qh[1][0] = Pp[1][0];
        Qh[1][1] = Pp[1][1];
        Qh[2][2] = fmax(Qh[2][2], fl);
        Qh[3][3] = fmax(Qh[3][3], fl);
        return;
    }
    // (psi, v, a, delta) block
    double Hd[10];
    bike_step_hessian(P, x, u, mu, Hd);
    double B4[4][4], V4[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) B4[i][j] = Hd[jidx(i, j)];
    B4[0][0] += Qh[2][2];
    B4[1][1] += Qh[3][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) B4[2 + i][2 + j] += Rh[i][j];
    jacobi_eig<4>(B4, V4);
#pragma unroll
    for (int i = 0; i < 4; ++i) big = fmax(big, fabs(B4[i][i]));
    const double fl = delta * big;
    eig_rebuild<2>(Pp, Vp, fl);
    Qh[0][0] = Pp[0][0];
    Qh[0][1] = Pp[0][1];
    Qh[1][0] = Pp[1][0];
    Qh[1][1] = Pp[1][1];
    eig_rebuild<4>(B4, V4, fl);
    Qh[2][2] = B4[0][0];
    Qh[2][3] = B4[0][1];
    Qh[3][2] = B4[1][0];
    Qh[3][3] = B4[1][1];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) Rh[i][j] = B4[2 + i][2 + j];
        Mh[i][2] = B4[2 + i][0];
        Mh[i][3] = B4[2 + i][1];
    }
}

}  // namespace bmpc
