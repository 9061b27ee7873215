// Warm-start network: a multilayer perceptron with GELU hidden activations
// and a linear output, trained with Adam on the mean squared error.
// Weights and activations are BF16, products accumulate in FP32 on the
// matrix cores (MFMA 16x16x16 BF16), master weights and optimiser state are
// FP32.
//
// Layer l:  Z_{l+1} = A_l W_l + b_l,  A_{l+1} = gelu(Z_{l+1}) (hidden) or
// Y = Z_L (output), with gelu(z) = z/2 (1 + erf(z/sqrt 2)).
// Backward: dW_l = A_l^T dZ_{l+1}, db_l = column sums of dZ_{l+1},
// dZ_l = (dZ_{l+1} W_l^T) * gelu'(Z_l).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "bmpc_internal.hpp"
#include "profile.hpp"

namespace bmpc {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest, ties to even (NaN stays NaN)
__host__ __device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf2f(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum Epi { EPI_GELU = 0, EPI_LINEAR = 1, EPI_GELU_BACK = 2, EPI_STORE = 3 };

// C = op(A) op(B) for bf16 inputs with fp32 accumulation.
//   op(A)[m][k] = TA ? A[k*lda + m] : A[m*lda + k]
//   op(B)[k][n] = TB ? B[n*ldb + k] : B[k*ldb + n]
// One wavefront per 32 x 32 tile of C (2 x 2 MFMA 16x16x16 tiles), so that
// batch-sized GEMMs still spread over every CU.  K advances 32 at a time
// through LDS; operands are fetched from global memory as 8-element (16-byte)
// runs along their contiguous dimension and the next K stage is fetched into
// registers while the current one is multiplied.  LDS holds A as [m][k] and
// B as [n][k], so each lane reads its four consecutive k of an MFMA operand
// with one 8-byte load.  Out-of-range elements are zero.
// Split K: blockIdx.z takes K range [z*kchunk, (z+1)*kchunk); with more
// than one split the raw products go to Zout + z*M*ldc (summed later in a
// fixed order) and the epilogue must be EPI_STORE.
// Epilogues:
//   EPI_GELU:      Z = acc + bias (fp32 out), O = bf16(gelu(Z))
//   EPI_LINEAR:    Z = acc + bias (fp32 out)
//   EPI_GELU_BACK: O = bf16(acc * gelu'(Zin))
//   EPI_STORE:     Z = acc (fp32 out)
constexpr int MLP_MAX_SPLITS = 8;  // split-K factor limit of the weight gradient
constexpr int GT = 32;       // tile edge
constexpr int GK = 32;       // K per stage
constexpr int GLD = GK + 8;  // LDS row stride in elements (80 bytes: 16-byte aligned rows)

struct Run8 {
    uint4 v;  // 8 bf16
};

// 8 consecutive elements p[0..7] (valid ones: first `valid`), as one 16-byte
// load when all are valid and the address is 16-byte aligned
__device__ __forceinline__ uint4 load_run8(const uint16_t* __restrict__ p, int valid)
{
    if (valid >= 8 && ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)) return *reinterpret_cast<const uint4*>(p);
    uint16_t t[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = e < valid ? p[e] : (uint16_t)0;
    uint4 r;
    memcpy(&r, t, 16);
    return r;
}

template <bool TRANS>
struct TileLoad {
    // operand X with logical rows r (m for A, n for B) and reduction index k:
    //   TRANS == false: X[r*ld + k] (k contiguous),  TRANS == true: X[k*ld + r]
    // Each lane fetches two runs of 8 per stage.
    uint4 run[2];
    __device__ __forceinline__ void fetch(const uint16_t* __restrict__ X, int ld, int rows, int K, int r0, int k0,
                                          int kend, int lane)
    {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = lane + 64 * e;  // 128 runs of 8 per 32 x 32 tile
            if (!TRANS) {
                const int r = r0 + (c >> 2), k = k0 + (c & 3) * 8;
                const int valid = (r < rows) ? (kend - k) : 0;
                run[e] = valid > 0 ? load_run8(X + (long)r * ld + k, valid) : make_uint4(0, 0, 0, 0);
            } else {
                const int k = k0 + (c >> 2), r = r0 + (c & 3) * 8;
                const int valid = (k < kend) ? (rows - r) : 0;
                run[e] = valid > 0 ? load_run8(X + (long)k * ld + r, valid) : make_uint4(0, 0, 0, 0);
            }
        }
        (void)K;
    }
    __device__ __forceinline__ void store(uint16_t (*S)[GLD], int lane) const
    {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = lane + 64 * e;
            if (!TRANS) {
                *reinterpret_cast<uint4*>(&S[c >> 2][(c & 3) * 8]) = run[e];
            } else {
                uint16_t t[8];
                memcpy(t, &run[e], 16);
                const int k = c >> 2, r = (c & 3) * 8;
#pragma unroll
                for (int q = 0; q < 8; ++q) S[r + q][k] = t[q];
            }
        }
    }
};

// ordering of one wavefront's own LDS accesses (its LDS operations complete
// in issue order; only the compiler must not move them)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int GW = 4;  // wavefronts per workgroup, each on every GW-th K stage

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(64 * GW) k_gemm_bf16(int M, int N, int K, const uint16_t* __restrict__ A, int lda,
                                                       const uint16_t* __restrict__ B, int ldb,
                                                       const float* __restrict__ bias, const float* __restrict__ Zin,
                                                       float* __restrict__ Zout, uint16_t* __restrict__ O, int ldc,
                                                       int kchunk)
{
    __shared__ __align__(16) uint16_t sA[GW][GT][GLD];  // per wave: [m][k]
    __shared__ __align__(16) uint16_t sB[GW][GT][GLD];  // per wave: [n][k]
    __shared__ float red[GW][GT][GT + 1];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    f32x4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    // op(B)[k][n]: with TB the storage is B[n][k] (k contiguous), otherwise B[k][n]
    TileLoad<TA> la;
    TileLoad<!TB> lb;
    int k0 = kbeg + w * GK;
    if (k0 < kend) {
        la.fetch(A, lda, M, K, m0, k0, kend, lane);
        lb.fetch(B, ldb, N, K, n0, k0, kend, lane);
    }
    const int r = lane & 15, kq = (lane >> 4) * 4;
    for (; k0 < kend; k0 += GW * GK) {
        la.store(sA[w], lane);
        lb.store(sB[w], lane);
        wave_lds_sync();
        if (k0 + GW * GK < kend) {  // this wave's next stage in flight during the products
            la.fetch(A, lda, M, K, m0, k0 + GW * GK, kend, lane);
            lb.fetch(B, ldb, N, K, n0, k0 + GW * GK, kend, lane);
        }
#pragma unroll
        for (int kk = 0; kk < GK; kk += 16) {
            bf16x4_t a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x4_t*>(&sA[w][16 * i + r][kk + kq]);
                b[i] = *reinterpret_cast<const bf16x4_t*>(&sB[w][16 * i + r][kk + kq]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        wave_lds_sync();
    }
    // lane holds C[row = 4*(lane/16) + q][col = lane%16] of each 16x16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[w][16 * i + 4 * (lane >> 4) + q][16 * j + (lane & 15)] = acc[i][j][q];
    __syncthreads();
    // the waves' partial tiles summed in wave order; one element per thread
    // and pass, consecutive threads on consecutive columns
    float* Zdst = Zout ? Zout + (long)blockIdx.z * M * ldc : nullptr;
    for (int e = threadIdx.x; e < GT * GT; e += 64 * GW) {
        const int rr = e / GT, cc = e % GT;
        const int gm = m0 + rr, gn = n0 + cc;
        if (gm >= M || gn >= N) continue;
        float v = red[0][rr][cc];
#pragma unroll
        for (int q = 1; q < GW; ++q) v += red[q][rr][cc];
        const long o = (long)gm * ldc + gn;
        if constexpr (EPI == EPI_GELU) {
            v += bias[gn];
            Zdst[o] = v;
            O[o] = f2bf(gelu(v));
        } else if constexpr (EPI == EPI_LINEAR) {
            Zdst[o] = v + bias[gn];
        } else if constexpr (EPI == EPI_GELU_BACK) {
            O[o] = f2bf(v * gelu_grad(Zin[o]));
        } else {
            Zdst[o] = v;
        }
    }
}

// out[i] = sum over s of part[s*n + i], in split order
__global__ void k_sum_splits(const float* __restrict__ part, int splits, long n, float* __restrict__ out)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float t = part[i];
    for (int s = 1; s < splits; ++s) t += part[(long)s * n + i];
    out[i] = t;
}

// Network input: bf16((x - shift_c) * scale_c) for column c (FP32 affine
// map first, so standardisation happens before the rounding).
__global__ void k_input_bf16(const float* __restrict__ x, const float* __restrict__ shift,
                             const float* __restrict__ scale, uint16_t* __restrict__ y, long n, int cols)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = (int)(i % cols);
    y[i] = f2bf((x[i] - shift[c]) * scale[c]);
}

// dY = 2 (Y - T) / (B * N) in bf16; per-block partial sums of (Y - T)^2
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             uint16_t* __restrict__ dY, float* __restrict__ partial, long n,
                                             float scale)
{
    __shared__ float s[256];
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float e2 = 0.f;
    if (i < n) {
        const float d = Y[i] - T[i];
        e2 = d * d;
        dY[i] = f2bf(2.0f * d * scale);
    }
    s[threadIdx.x] = e2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ void k_sum_partials(const float* __restrict__ partial, int n, float scale, float* __restrict__ out)
{
    __shared__ float s[256];
    float t = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) t += partial[i];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0] * scale;
}

// db[n] = sum_m dZ[m][n].  A block covers 32 columns with 8 row groups;
// thread (c, g) sums rows g, g + 8, ... of column c (reads of 32 consecutive
// columns are coalesced), then the 8 partial sums are added in group order,
// so the result does not depend on timing.
__global__ void __launch_bounds__(256) k_colsum_bf16(const uint16_t* __restrict__ dZ, int M, int N,
                                                     float* __restrict__ db)
{
    __shared__ float part[8][33];
    const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int n = blockIdx.x * 32 + c;
    float acc = 0.f;
    if (n < N)
        for (int m = g; m < M; m += 8) acc += bf2f(dZ[(long)m * N + n]);
    part[g][c] = acc;
    __syncthreads();
    if (g == 0 && n < N) {
        float t = part[0][c];
#pragma unroll
        for (int q = 1; q < 8; ++q) t += part[q][c];
        db[n] = t;
    }
}

// Adam on fp32 master parameters; refreshes the bf16 copy of weights.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ pbf, long n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    if (pbf) pbf[i] = f2bf(pi);
}

}  // namespace bmpc

using namespace bmpc;

struct bmpc_mlp {
    int L = 0, max_batch = 0;
    std::vector<int> w;          // widths, L+1
    std::vector<long> woff, boff;  // offsets of W_l, b_l in the flat parameter vector
    long nparam = 0;
    float* p = nullptr;          // fp32 master parameters (all W then b, layer by layer)
    float* g = nullptr;          // gradients
    float* m = nullptr;          // Adam moments
    float* v = nullptr;
    uint16_t* pbf = nullptr;     // bf16 copy of the parameters
    std::vector<uint16_t*> act;  // A_l bf16, B x w_l (act[0] = input)
    std::vector<float*> z;       // Z_l fp32, B x w_l (l >= 1)
    std::vector<uint16_t*> dz;   // dZ_l bf16, B x w_l (l >= 1)
    float* partial = nullptr;
    float* loss = nullptr;
    float* gpart = nullptr;     // split-K partial weight gradients
    float* in_shift = nullptr;  // w_0: input affine map (x - shift) * scale
    float* in_scale = nullptr;
    long step = 0;
};

static bmpc_status mlp_forward_impl(bmpc_mlp* net, const float* X, int B, hipStream_t s)
{
    const int L = net->L;
    const long nin = (long)B * net->w[0];
    hipLaunchKernelGGL(k_input_bf16, dim3((unsigned)((nin + 255) / 256)), dim3(256), 0, s, X, net->in_shift,
                       net->in_scale, net->act[0], nin, net->w[0]);
    for (int l = 0; l < L; ++l) {
        const int K = net->w[l], N = net->w[l + 1];
        dim3 grid((N + GT - 1) / GT, (B + GT - 1) / GT, 1);
        const uint16_t* W = net->pbf + net->woff[l];
        const float* b = net->p + net->boff[l];
        if (l < L - 1) {
            ProfScope ps("mlp_gemm_forward", s);
            hipLaunchKernelGGL((k_gemm_bf16<false, false, EPI_GELU>), grid, dim3(64 * GW), 0, s, B, N, K, net->act[l], K, W,
                               N, b, nullptr, net->z[l + 1], net->act[l + 1], N, K);
        } else {
            ProfScope ps("mlp_gemm_forward", s);
            hipLaunchKernelGGL((k_gemm_bf16<false, false, EPI_LINEAR>), grid, dim3(64 * GW), 0, s, B, N, K, net->act[l],
                               K, W, N, b, nullptr, net->z[l + 1], nullptr, N, K);
        }
    }
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

// loss and gradients into net->g (no update)
static bmpc_status mlp_backward_impl(bmpc_mlp* net, const float* T, int B, hipStream_t s)
{
    const int L = net->L;
    const int NO = net->w[L];
    const long n = (long)B * NO;
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, net->z[L], T, net->dz[L], net->partial, n, 1.0f / (float)n);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, net->partial, nb, 1.0f / (float)n, net->loss);
    for (int l = L - 1; l >= 0; --l) {
        const int K = net->w[l], N = net->w[l + 1];
        // dW_l = A_l^T dZ_{l+1}: (K x B) (B x N)
        {
            // split the batch (the reduction) so that small weight matrices
            // still occupy the whole chip; partial products are summed in a
            // fixed order, so the gradient does not depend on the schedule
            const int tiles = ((N + GT - 1) / GT) * ((K + GT - 1) / GT);
            int splits = (512 + tiles - 1) / tiles;
            splits = std::min(splits, std::max(1, B / 128));
            splits = std::max(1, std::min(splits, MLP_MAX_SPLITS));
            const int kchunk = ((B + splits - 1) / splits + GK - 1) / GK * GK;
            splits = (B + kchunk - 1) / kchunk;
            dim3 grid((N + GT - 1) / GT, (K + GT - 1) / GT, splits);
            float* dst = splits > 1 ? net->gpart : net->g + net->woff[l];
            ProfScope ps("mlp_gemm_weight_grad", s);
            hipLaunchKernelGGL((k_gemm_bf16<true, false, EPI_STORE>), grid, dim3(64 * GW), 0, s, K, N, B, net->act[l], K,
                               net->dz[l + 1], N, nullptr, nullptr, dst, nullptr, N, kchunk);
            if (splits > 1) {
                const long nel = (long)K * N;
                hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, s, net->gpart,
                                   splits, nel, net->g + net->woff[l]);
            }
        }
        hipLaunchKernelGGL(k_colsum_bf16, dim3((N + 31) / 32), dim3(256), 0, s, net->dz[l + 1], B, N,
                           net->g + net->boff[l]);
        if (l > 0) {
            // dZ_l = (dZ_{l+1} W_l^T) * gelu'(Z_l): (B x N) (N x K)
            ProfScope ps("mlp_gemm_input_grad", s);
            dim3 grid((K + GT - 1) / GT, (B + GT - 1) / GT, 1);
            hipLaunchKernelGGL((k_gemm_bf16<false, true, EPI_GELU_BACK>), grid, dim3(64 * GW), 0, s, B, K, N,
                               net->dz[l + 1], N, net->pbf + net->woff[l], N, nullptr, net->z[l], nullptr,
                               net->dz[l], K, N);
        }
    }
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

extern "C" {

BMPC_API bmpc_status bmpc_mlp_create(const int32_t* widths, int32_t n_layers, int32_t max_batch, bmpc_mlp** out)
{
    if (!widths || n_layers < 1 || n_layers > 16 || max_batch < 1 || !out)
        return fail(BMPC_ERR_INVALID_ARG, "bad network shape");
    *out = nullptr;
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1 || widths[l] > 65536) return fail(BMPC_ERR_INVALID_ARG, "layer width %d out of range", l);
    auto* net = new bmpc_mlp();
    net->L = n_layers;
    net->max_batch = max_batch;
    net->w.assign(widths, widths + n_layers + 1);
    long off = 0;
    for (int l = 0; l < n_layers; ++l) {
        net->woff.push_back(off);
        off += (long)widths[l] * widths[l + 1];
    }
    for (int l = 0; l < n_layers; ++l) {
        net->boff.push_back(off);
        off += widths[l + 1];
    }
    net->nparam = off;
    long max_wprod = 1;
    for (int l = 0; l < n_layers; ++l) max_wprod = std::max(max_wprod, (long)widths[l] * widths[l + 1]);
    bool ok = hipMalloc(&net->p, sizeof(float) * off) == hipSuccess &&
              hipMalloc(&net->g, sizeof(float) * off) == hipSuccess &&
              hipMalloc(&net->m, sizeof(float) * off) == hipSuccess &&
              hipMalloc(&net->v, sizeof(float) * off) == hipSuccess &&
              hipMalloc(&net->pbf, sizeof(uint16_t) * off) == hipSuccess &&
              hipMalloc(&net->loss, sizeof(float)) == hipSuccess &&
              hipMalloc(&net->gpart, sizeof(float) * MLP_MAX_SPLITS * max_wprod) == hipSuccess &&
              hipMalloc(&net->in_shift, sizeof(float) * widths[0]) == hipSuccess &&
              hipMalloc(&net->in_scale, sizeof(float) * widths[0]) == hipSuccess &&
              hipMalloc(&net->partial, sizeof(float) * (((long)max_batch * widths[n_layers] + 255) / 256 + 1)) ==
                  hipSuccess;
    net->act.assign(n_layers + 1, nullptr);
    net->z.assign(n_layers + 1, nullptr);
    net->dz.assign(n_layers + 1, nullptr);
    for (int l = 0; l <= n_layers && ok; ++l) {
        const size_t e = (size_t)max_batch * widths[l];
        ok = hipMalloc(&net->act[l], sizeof(uint16_t) * e) == hipSuccess;
        if (ok && l > 0)
            ok = hipMalloc(&net->z[l], sizeof(float) * e) == hipSuccess &&
                 hipMalloc(&net->dz[l], sizeof(uint16_t) * e) == hipSuccess;
    }
    if (!ok) {
        bmpc_mlp_destroy(net);
        return fail(BMPC_ERR_OOM, "device allocation for the network failed");
    }
    std::vector<float> ones(widths[0], 1.0f);
    if (hipMemset(net->in_shift, 0, sizeof(float) * widths[0]) != hipSuccess ||
        hipMemcpy(net->in_scale, ones.data(), sizeof(float) * widths[0], hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(net->p, 0, sizeof(float) * off) != hipSuccess ||
        hipMemset(net->m, 0, sizeof(float) * off) != hipSuccess ||
        hipMemset(net->v, 0, sizeof(float) * off) != hipSuccess ||
        hipMemset(net->pbf, 0, sizeof(uint16_t) * off) != hipSuccess) {
        bmpc_mlp_destroy(net);
        return fail(BMPC_ERR_HIP, "initialising the network failed");
    }
    *out = net;
    return BMPC_OK;
}

BMPC_API void bmpc_mlp_destroy(bmpc_mlp* net)
{
    if (!net) return;
    (void)hipFree(net->p);
    (void)hipFree(net->g);
    (void)hipFree(net->m);
    (void)hipFree(net->v);
    (void)hipFree(net->pbf);
    (void)hipFree(net->loss);
    (void)hipFree(net->partial);
    (void)hipFree(net->gpart);
    (void)hipFree(net->in_shift);
    (void)hipFree(net->in_scale);
    for (auto* a : net->act) (void)hipFree(a);
    for (auto* a : net->z) (void)hipFree(a);
    for (auto* a : net->dz) (void)hipFree(a);
    delete net;
}

BMPC_API int64_t bmpc_mlp_num_params(const bmpc_mlp* net) { return net ? net->nparam : 0; }

BMPC_API bmpc_status bmpc_mlp_set_params(bmpc_mlp* net, const float* params)
{
    if (!net || !params) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    for (long i = 0; i < net->nparam; ++i)
        if (!std::isfinite(params[i])) return fail(BMPC_ERR_NONFINITE, "parameter %ld is not finite", i);
    BMPC_HIP_TRY(hipMemcpy(net->p, params, sizeof(float) * net->nparam, hipMemcpyHostToDevice));
    std::vector<uint16_t> h(net->nparam);
    for (long i = 0; i < net->nparam; ++i) h[i] = f2bf(params[i]);
    BMPC_HIP_TRY(hipMemcpy(net->pbf, h.data(), sizeof(uint16_t) * net->nparam, hipMemcpyHostToDevice));
    BMPC_HIP_TRY(hipMemset(net->m, 0, sizeof(float) * net->nparam));
    BMPC_HIP_TRY(hipMemset(net->v, 0, sizeof(float) * net->nparam));
    net->step = 0;
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_mlp_set_input_map(bmpc_mlp* net, const float* shift, const float* scale)
{
    if (!net || !shift || !scale) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    for (int c = 0; c < net->w[0]; ++c)
        if (!std::isfinite(shift[c]) || !std::isfinite(scale[c]))
            return fail(BMPC_ERR_NONFINITE, "input map entry %d is not finite", c);
    BMPC_HIP_TRY(hipMemcpy(net->in_shift, shift, sizeof(float) * net->w[0], hipMemcpyHostToDevice));
    BMPC_HIP_TRY(hipMemcpy(net->in_scale, scale, sizeof(float) * net->w[0], hipMemcpyHostToDevice));
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_mlp_get_params(bmpc_mlp* net, float* params)
{
    if (!net || !params) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    BMPC_HIP_TRY(hipMemcpy(params, net->p, sizeof(float) * net->nparam, hipMemcpyDeviceToHost));
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_mlp_forward(bmpc_mlp* net, const float* X, int32_t B, float* Y, void* stream)
{
    if (!net || !X || !Y) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    if (B < 1 || B > net->max_batch) return fail(BMPC_ERR_INVALID_ARG, "batch %d outside [1, %d]", B, net->max_batch);
    hipStream_t s = (hipStream_t)stream;
    bmpc_status st = mlp_forward_impl(net, X, B, s);
    if (st != BMPC_OK) return st;
    BMPC_HIP_TRY(hipMemcpyAsync(Y, net->z[net->L], sizeof(float) * (size_t)B * net->w[net->L],
                                hipMemcpyDeviceToDevice, s));
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_mlp_gradients(bmpc_mlp* net, const float* X, const float* T, int32_t B, float* grad,
                                        float* loss, void* stream)
{
    if (!net || !X || !T) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    if (B < 1 || B > net->max_batch) return fail(BMPC_ERR_INVALID_ARG, "batch %d outside [1, %d]", B, net->max_batch);
    hipStream_t s = (hipStream_t)stream;
    bmpc_status st;
    if ((st = mlp_forward_impl(net, X, B, s)) != BMPC_OK) return st;
    if ((st = mlp_backward_impl(net, T, B, s)) != BMPC_OK) return st;
    if (grad)
        BMPC_HIP_TRY(hipMemcpyAsync(grad, net->g, sizeof(float) * net->nparam, hipMemcpyDeviceToHost, s));
    if (loss) BMPC_HIP_TRY(hipMemcpyAsync(loss, net->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    BMPC_HIP_TRY(hipStreamSynchronize(s));
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_mlp_train_step(bmpc_mlp* net, const float* X, const float* T, int32_t B, float lr,
                                         float* loss, void* stream)
{
    if (!net || !X || !T) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    if (B < 1 || B > net->max_batch) return fail(BMPC_ERR_INVALID_ARG, "batch %d outside [1, %d]", B, net->max_batch);
    if (!(lr > 0.0f)) return fail(BMPC_ERR_INVALID_ARG, "learning rate must be positive");
    hipStream_t s = (hipStream_t)stream;
    bmpc_status st;
    if ((st = mlp_forward_impl(net, X, B, s)) != BMPC_OK) return st;
    if ((st = mlp_backward_impl(net, T, B, s)) != BMPC_OK) return st;
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f / (1.0f - powf(b1, (float)net->step));
    const float c2 = 1.0f / (1.0f - powf(b2, (float)net->step));
    {
        ProfScope ps("mlp_adam", s);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((net->nparam + 255) / 256)), dim3(256), 0, s, net->p, net->g,
                           net->m, net->v, net->pbf, net->nparam, lr, b1, b2, eps, c1, c2);
    }
    BMPC_HIP_TRY(hipGetLastError());
    if (loss) {
        BMPC_HIP_TRY(hipMemcpyAsync(loss, net->loss, sizeof(float), hipMemcpyDeviceToHost, s));
        BMPC_HIP_TRY(hipStreamSynchronize(s));
    }
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t trans_a,
                                    const uint16_t* B, int32_t trans_b, float* C, void* stream)
{
    if (!A || !B || !C || M < 1 || N < 1 || K < 1) return fail(BMPC_ERR_INVALID_ARG, "bad GEMM arguments");
    hipStream_t s = (hipStream_t)stream;
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, 1);
    const int lda = trans_a ? M : K, ldb = trans_b ? K : N;
    if (!trans_a && !trans_b)
        hipLaunchKernelGGL((k_gemm_bf16<false, false, EPI_STORE>), grid, dim3(64 * GW), 0, s, M, N, K, A, lda, B, ldb,
                           nullptr, nullptr, C, nullptr, N, K);
    else if (trans_a && !trans_b)
        hipLaunchKernelGGL((k_gemm_bf16<true, false, EPI_STORE>), grid, dim3(64 * GW), 0, s, M, N, K, A, lda, B, ldb,
                           nullptr, nullptr, C, nullptr, N, K);
    else if (!trans_a && trans_b)
        hipLaunchKernelGGL((k_gemm_bf16<false, true, EPI_STORE>), grid, dim3(64 * GW), 0, s, M, N, K, A, lda, B, ldb,
                           nullptr, nullptr, C, nullptr, N, K);
    else
        return fail(BMPC_ERR_UNSUPPORTED, "both operands transposed is not supported");
    BMPC_HIP_TRY(hipGetLastError());
    return BMPC_OK;
}

}  // extern "C"
