/*
 * CPU FP64 oracle for the warm-start network (multilayer perceptron, GELU
 * hidden layers, linear output, mean-squared-error loss, Adam).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark, never by the library.
 *
 * Definitions written out plainly (no blocking, no fusion):
 *   layer l (0 <= l < L):  Z_{l+1} = A_l W_l + 1 b_l^T,
 *                          A_{l+1} = gelu(Z_{l+1}) for l < L-1, Y = Z_L,
 *   gelu(z)  = z Phi(z) = z/2 (1 + erf(z / sqrt 2)),
 *   gelu'(z) = Phi(z) + z phi(z),  phi(z) = exp(-z^2/2) / sqrt(2 pi),
 *   loss     = (1/n) sum (Y - T)^2 over all n = B * w_L outputs,
 *   backward by the chain rule:
 *     dY = 2 (Y - T) / n,  dW_l = A_l^T dZ_{l+1},  db_l = column sums of
 *     dZ_{l+1},  dZ_l = (dZ_{l+1} W_l^T) * gelu'(Z_l).
 *   Adam (Kingma and Ba, Algorithm 1): m <- b1 m + (1-b1) g,
 *     v <- b2 v + (1-b2) g^2, p <- p - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 *
 * quant = 1 rounds to the nearest BF16 value (ties to even) at the points
 * where a low-precision network stores BF16: the input X, the weights W,
 * every hidden activation A_l, the output gradient dY and every hidden
 * gradient dZ_l.  Everything else (biases, Z, sums) stays FP64.  quant = 0
 * is the exact FP64 network.
 *
 * Parameter vector: W_0 .. W_{L-1} (w_l x w_{l+1}, row-major), b_0 .. b_{L-1}.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* nearest BF16 value (8 significant bits, exponent range of binary32), ties
   to even through nearbyint in the default rounding mode */
double orc_bf16(double x)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e = ilogb(x);
    if (e < -126) e = -126; /* subnormal range: fixed quantum 2^-133 */
    const double quantum = ldexp(1.0, e - 7);
    double r = nearbyint(x / quantum) * quantum;
    const double max_bf16 = ldexp(255.0, 120); /* (2 - 2^-7) 2^127 */
    if (fabs(r) > max_bf16) r = copysign(INFINITY, x);
    return r;
}

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }

static double gelu_prime(double z)
{
    const double Phi = 0.5 * (1.0 + erf(z / sqrt(2.0)));
    const double phi = exp(-0.5 * z * z) / sqrt(2.0 * 3.14159265358979323846);
    return Phi + z * phi;
}

double orc_gelu(double z) { return gelu(z); }
double orc_gelu_prime(double z) { return gelu_prime(z); }

static double q(double x, int quant) { return quant ? orc_bf16(x) : x; }

/* offsets of W_l and b_l in the parameter vector */
static void offsets(int L, const int* w, long* woff, long* boff)
{
    long off = 0;
    for (int l = 0; l < L; ++l) {
        woff[l] = off;
        off += (long)w[l] * w[l + 1];
    }
    for (int l = 0; l < L; ++l) {
        boff[l] = off;
        off += w[l + 1];
    }
}

/* Forward pass keeping A_l (acts[l], B x w_l, l = 0..L-1) and Z_l
   (zs[l], B x w_l, l = 1..L).  Returns 0 or ORC_ERR_INVALID_ARG. */
static int forward(int L, const int* w, const double* params, int B, const double* X, int quant,
                   double** acts, double** zs)
{
    long woff[16], boff[16];
    if (L < 1 || L > 16 || B < 1) return ORC_ERR_INVALID_ARG;
    offsets(L, w, woff, boff);
    for (long i = 0; i < (long)B * w[0]; ++i) acts[0][i] = q(X[i], quant);
    for (int l = 0; l < L; ++l) {
        const int K = w[l], N = w[l + 1];
        const double* W = params + woff[l];
        const double* b = params + boff[l];
        double* Z = zs[l + 1];
        for (int m = 0; m < B; ++m)
            for (int n = 0; n < N; ++n) {
                double s = b[n];
                for (int k = 0; k < K; ++k) s += acts[l][(long)m * K + k] * q(W[(long)k * N + n], quant);
                Z[(long)m * N + n] = s;
            }
        if (l < L - 1)
            for (long i = 0; i < (long)B * N; ++i) acts[l + 1][i] = q(gelu(Z[i]), quant);
    }
    return ORC_OK;
}

static int alloc_buffers(int L, const int* w, int B, double** acts, double** zs)
{
    for (int l = 0; l <= L; ++l) {
        acts[l] = (double*)calloc((size_t)B * w[l], sizeof(double));
        zs[l] = (double*)calloc((size_t)B * w[l], sizeof(double));
        if (!acts[l] || !zs[l]) return 0;
    }
    return 1;
}

static void free_buffers(int L, double** acts, double** zs)
{
    for (int l = 0; l <= L; ++l) {
        free(acts[l]);
        free(zs[l]);
    }
}

int orc_mlp_forward(int L, const int* w, int B, const double* params, const double* X, int quant, double* Y)
{
    double *acts[17] = {0}, *zs[17] = {0};
    if (L < 1 || L > 16) return ORC_ERR_INVALID_ARG;
    int st = ORC_ERR_INVALID_ARG;
    if (alloc_buffers(L, w, B, acts, zs)) {
        st = forward(L, w, params, B, X, quant, acts, zs);
        if (st == ORC_OK) memcpy(Y, zs[L], sizeof(double) * (size_t)B * w[L]);
    }
    free_buffers(L, acts, zs);
    return st;
}

/* loss (returned through *loss) and its gradient with respect to every
   parameter (grad, length of the parameter vector) */
int orc_mlp_backward(int L, const int* w, int B, const double* params, const double* X, const double* T,
                     int quant, double* grad, double* loss)
{
    double *acts[17] = {0}, *zs[17] = {0};
    long woff[16], boff[16];
    if (L < 1 || L > 16) return ORC_ERR_INVALID_ARG;
    int st = ORC_ERR_INVALID_ARG;
    double* dZ = NULL;
    double* dZprev = NULL;
    int wmax = 0;
    for (int l = 0; l <= L; ++l) wmax = w[l] > wmax ? w[l] : wmax;
    if (!alloc_buffers(L, w, B, acts, zs)) goto done;
    dZ = (double*)calloc((size_t)B * wmax, sizeof(double));
    dZprev = (double*)calloc((size_t)B * wmax, sizeof(double));
    if (!dZ || !dZprev) goto done;
    st = forward(L, w, params, B, X, quant, acts, zs);
    if (st != ORC_OK) goto done;
    offsets(L, w, woff, boff);
    {
        const long n = (long)B * w[L];
        double s = 0.0;
        for (long i = 0; i < n; ++i) {
            const double d = zs[L][i] - T[i];
            s += d * d;
            dZ[i] = q(2.0 * d / (double)n, quant);
        }
        *loss = s / (double)n;
    }
    for (int l = L - 1; l >= 0; --l) {
        const int K = w[l], N = w[l + 1];
        const double* W = params + woff[l];
        double* gW = grad + woff[l];
        double* gb = grad + boff[l];
        /* dW_l = A_l^T dZ_{l+1} */
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < N; ++j) {
                double s = 0.0;
                for (int m = 0; m < B; ++m) s += acts[l][(long)m * K + k] * dZ[(long)m * N + j];
                gW[(long)k * N + j] = s;
            }
        /* db_l = column sums of dZ_{l+1} */
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
            for (int m = 0; m < B; ++m) s += dZ[(long)m * N + j];
            gb[j] = s;
        }
        if (l == 0) break;
        /* dZ_l = (dZ_{l+1} W_l^T) * gelu'(Z_l) */
        for (int m = 0; m < B; ++m)
            for (int k = 0; k < K; ++k) {
                double s = 0.0;
                for (int j = 0; j < N; ++j) s += dZ[(long)m * N + j] * q(W[(long)k * N + j], quant);
                dZprev[(long)m * K + k] = q(s * gelu_prime(zs[l][(long)m * K + k]), quant);
            }
        double* t = dZ;
        dZ = dZprev;
        dZprev = t;
    }
    st = ORC_OK;
done:
    free(dZ);
    free(dZprev);
    free_buffers(L, acts, zs);
    return st;
}

void orc_adam(long n, double* p, const double* g, double* m, double* v, int t, double lr, double b1, double b2,
              double eps)
{
    for (long i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        const double mhat = m[i] / (1.0 - pow(b1, t));
        const double vhat = v[i] / (1.0 - pow(b2, t));
        p[i] -= lr * mhat / (sqrt(vhat) + eps);
    }
}
