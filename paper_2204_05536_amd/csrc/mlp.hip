// Learned per-leaf preconditioner: a shared 3-layer MLP applied leaf by
// leaf, used as a right preconditioner inside flexible GMRES.
//
// Input of leaf X (64 slots, slot i = the i-th point of X in tree order,
// empty slots zero): [(x_i - c_x) / h (64), (y_i - c_y) / h (64),
// r_i / |r_X| (64)], with c the box centre and h its half side.
// Network: 192 -> 256 (ReLU) -> 256 (ReLU) -> 64, in residual form around
// a fitted scale s: z_i = s |r_X| (r_i / |r_X| + out_i), so the map is
// positively homogeneous in r and the untrained network (last layer zero)
// is the preconditioner s I.  Training targets come from the method
// itself: for random r, z = K(X, X)^{-1} r(X) leaf by leaf (the method's
// leaf-block solves; default) or z = A^{-1} r by FP64 GMRES; s is the
// least-squares scalar with z ~ s r, and every leaf contributes the pair
// (r_X, z_X / (s |r_X|) - r_X / |r_X|).  Leaf targets are a deterministic
// function of the leaf's geometry and residual; global targets add the
// coupling beyond the leaf, which the leaf's input cannot see.
#include "h2d_impl.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace h2d {

constexpr int kIn = 192, kH = 256, kOut = 64;
constexpr int kInPatch = 5 * kIn;   // the leaf and its 4 edge sharers, 64 slots x 3 features each

// Packed parameter layout of a network with `in` inputs:
// W1 (256 x in), b1, W2 (256 x 256), b2, W3 (64 x 256), b3.
struct Dims {
    int in;
    int64_t w1, b1, w2, b2, w3, b3, params;
};
constexpr Dims make_dims(int in)
{
    return Dims{in,
                0,
                (int64_t)kH * in,
                (int64_t)kH * in + kH,
                (int64_t)kH * in + kH + (int64_t)kH * kH,
                (int64_t)kH * in + 2 * kH + (int64_t)kH * kH,
                (int64_t)kH * in + 2 * kH + (int64_t)kH * kH + (int64_t)kOut * kH,
                (int64_t)kH * in + 2 * kH + (int64_t)kH * kH + (int64_t)kOut * kH + kOut};
}
constexpr Dims kLeafDims = make_dims(kIn), kPatchDims = make_dims(kInPatch);
static_assert(kLeafDims.params == H2D_MLP_PARAMS, "parameter count");
static_assert(kPatchDims.params == H2D_MLP_PARAMS_PATCH, "parameter count (patch input)");

// ---------------------------------------------------------------------
// FP32 GEMM: C (M x N, row-major, ldc) = alpha op(A) op(B) + beta C, with
// op(A) M x K and op(B) K x N.  A row-major (lda) or, transA, its
// transpose; same for B.  64 x 64 tiles, 256 threads, 4 x 4 outputs each,
// K in steps of 16 through LDS.  Fixed summation order.
// ---------------------------------------------------------------------
// With gridDim.z > 1 the inner dimension is cut into slices of kslice
// (slice z covers rows [z kslice, (z + 1) kslice) of op(A)'s columns and
// op(B)'s rows) and slice z writes its own C at C + z cstride: the partial
// products of a split-K product, all in one launch.
__global__ void __launch_bounds__(256)
k_gemm(int M, int N, int K, const float* __restrict__ A, int lda, int transA, const float* __restrict__ B, int ldb,
       int transB, float* __restrict__ C, int ldc, float alpha, float beta, int kslice, int64_t cstride)
{
    __shared__ float As[16][64 + 1];
    __shared__ float Bs[16][64 + 1];
    if (gridDim.z > 1) {
        const int k0 = blockIdx.z * kslice;
        K = max(0, min(K, k0 + kslice) - k0);
        A += transA ? (int64_t)k0 * lda : k0;
        B += transB ? k0 : (int64_t)k0 * ldb;
        C += blockIdx.z * cstride;
    }
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e / 64, mm = e % 64;
            const int gm = m0 + mm, gk = k0 + kk;
            float a = 0.f;
            if (gm < M && gk < K) a = transA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
            As[kk][mm] = a;
            const int gn = n0 + mm;
            float b = 0.f;
            if (gn < N && gk < K) b = transB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
            Bs[kk][mm] = b;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gm = m0 + ty * 4 + i, gn = n0 + tx * 4 + j;
            if (gm < M && gn < N) {
                float* c = C + (int64_t)gm * ldc + gn;
                *c = alpha * acc[i][j] + (beta == 0.f ? 0.f : beta * *c);
            }
        }
}

static void gemm(int M, int N, int K, const float* A, int lda, bool tA, const float* B, int ldb, bool tB, float* C,
                 int ldc, float alpha, float beta, hipStream_t s)
{
    dim3 g((N + 63) / 64, (M + 63) / 64);
    k_gemm<<<g, 256, 0, s>>>(M, N, K, A, lda, tA ? 1 : 0, B, ldb, tB ? 1 : 0, C, ldc, alpha, beta, K, 0);
    HIPCK(hipGetLastError());
}

// C (M x N, ldc = N) = sum over the S slices of partial products, slice q
// covering K rows [q K / S, (q + 1) K / S) of op(A) and op(B); partials
// summed in slice order (fixed).  For the weight gradients, where the
// inner dimension is the batch and M x N is only a few 64 x 64 tiles.
__global__ void k_sum_slices(int64_t mn, int S, const float* __restrict__ P, float* __restrict__ C)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn; e += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        for (int q = 0; q < S; ++q) v += P[(int64_t)q * mn + e];
        C[e] = v;
    }
}

static void gemm_tn_split(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, float* work,
                          int S, hipStream_t s)
{
    // op(A) = A^T (A stored K x M), op(B) = B (K x N); slice z of K in
    // grid plane z
    const int kq = (K + S - 1) / S;
    dim3 g((N + 63) / 64, (M + 63) / 64, S);
    k_gemm<<<g, 256, 0, s>>>(M, N, K, A, lda, 1, B, ldb, 0, work, N, 1.f, 0.f, kq, (int64_t)M * N);
    const int64_t mn = (int64_t)M * N;
    k_sum_slices<<<(int)std::min<int64_t>(1024, (mn + 255) / 256), 256, 0, s>>>(mn, S, work, C);
    HIPCK(hipGetLastError());
}

// Z (M x N) += bias (per column), then optional ReLU.
__global__ void k_bias_act(int64_t M, int N, const float* __restrict__ bias, float* __restrict__ Z, int relu)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M * N; e += (int64_t)gridDim.x * blockDim.x) {
        float v = Z[e] + bias[e % N];
        Z[e] = relu ? fmaxf(v, 0.f) : v;
    }
}

// G (M x N) *= [H > 0]  (ReLU derivative, H = the layer's output)
__global__ void k_relu_back(int64_t M, int N, const float* __restrict__ Hh, float* __restrict__ G)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M * N; e += (int64_t)gridDim.x * blockDim.x)
        if (!(Hh[e] > 0.f)) G[e] = 0.f;
}

// db (N) = column sums of G (M x N) in two fixed-order stages: block
// (c, q) sums rows q, q + Q, ... of columns 64 c .. 64 c + 63 (4 row
// groups per block, combined in LDS), then one pass adds the Q partials.
constexpr int kColQ = 64;
__global__ void __launch_bounds__(256)
k_colsum_part(int64_t M, int N, const float* __restrict__ G, float* __restrict__ part)
{
    __shared__ float red[4][64];
    const int c = threadIdx.x % 64, g = threadIdx.x / 64;
    const int j = blockIdx.x * 64 + c, q = blockIdx.y;
    float v = 0.f;
    if (j < N)
        for (int64_t i = q + (int64_t)kColQ * g; i < M; i += 4 * kColQ) v += G[i * N + j];
    red[g][c] = v;
    __syncthreads();
    if (g == 0 && j < N) part[(int64_t)q * N + j] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

__global__ void k_colsum_final(int N, const float* __restrict__ part, float* __restrict__ db)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float v = 0.f;
    for (int q = 0; q < kColQ; ++q) v += part[(int64_t)q * N + j];
    db[j] = v;
}

// count[0] = sum of the n values (one workgroup, fixed order), at least 1:
// the mask's valid slots, from the per-row counts of a batch.
__global__ void __launch_bounds__(256) k_masksum(int64_t n, const float* __restrict__ Mk, float* __restrict__ count)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t e = threadIdx.x; e < n; e += 256) s += Mk[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) count[0] = fmaxf(red[0], 1.f);
}

// dO = mask (O - T) / count; partial loss sums per block (fixed order).
// The count is read from device memory (count_d) when given, else taken
// from inv_count.
__global__ void k_mse(int64_t n, const float* __restrict__ O, const float* __restrict__ T, const float* __restrict__ Mk,
                      float inv_count, const float* __restrict__ count_d, float* __restrict__ dO,
                      float* __restrict__ part)
{
    __shared__ float red[256];
    if (count_d) inv_count = 1.f / count_d[0];
    float s = 0.f;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float d = (O[e] - T[e]) * Mk[e];
        dO[e] = d * inv_count;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float c1, float c2, float eps)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float a = b1 * m1[e] + (1.f - b1) * gg, v = b2 * m2[e] + (1.f - b2) * gg * gg;
        m1[e] = a;
        m2[e] = v;
        w[e] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
    }
}

// ---------------------------------------------------------------------
// Forward and backward on a batch (X: B x 192, targets T and mask Mk:
// B x 64).  Workspace: H1, H2 (B x 256), O (B x 64), G1, G2, GO.
// ---------------------------------------------------------------------
constexpr int kSplitMax = 16;   // K slices of the weight-gradient products
struct MlpWork {
    int64_t cap = 0;
    DBuf<float> h1, h2, o, g1, g2, go, part, split, colp, count;
    void ensure(int64_t B)
    {
        if (B <= cap) return;
        h1.alloc(B * kH); h2.alloc(B * kH); o.alloc(B * kOut);
        g1.alloc(B * kH); g2.alloc(B * kH); go.alloc(B * kOut);
        part.alloc(1024);
        split.alloc((size_t)kSplitMax * kH * kInPatch);
        colp.alloc((size_t)kColQ * kH);
        count.alloc(1);
        cap = B;
    }
};

static void colsum(int64_t M, int N, const float* G, float* db, MlpWork& w, hipStream_t s)
{
    k_colsum_part<<<dim3((N + 63) / 64, kColQ), 256, 0, s>>>(M, N, G, w.colp.p);
    k_colsum_final<<<(N + 255) / 256, 256, 0, s>>>(N, w.colp.p, db);
}

// K slices for a weight-gradient product with inner dimension B
static int splits_for(int64_t B) { return (int)std::max<int64_t>(1, std::min<int64_t>(kSplitMax, B / 256)); }

static int grid_for(int64_t n) { return (int)std::min<int64_t>(4096, (n + 255) / 256); }

static void forward(const Dims& d, const float* W, const float* X, int64_t B, MlpWork& w, hipStream_t s)
{
    gemm((int)B, kH, d.in, X, d.in, false, W + d.w1, d.in, true, w.h1.p, kH, 1.f, 0.f, s);
    k_bias_act<<<grid_for(B * kH), 256, 0, s>>>(B, kH, W + d.b1, w.h1.p, 1);
    gemm((int)B, kH, kH, w.h1.p, kH, false, W + d.w2, kH, true, w.h2.p, kH, 1.f, 0.f, s);
    k_bias_act<<<grid_for(B * kH), 256, 0, s>>>(B, kH, W + d.b2, w.h2.p, 1);
    gemm((int)B, kOut, kH, w.h2.p, kH, false, W + d.w3, kH, true, w.o.p, kOut, 1.f, 0.f, s);
    k_bias_act<<<grid_for(B * kOut), 256, 0, s>>>(B, kOut, W + d.b3, w.o.p, 0);
    HIPCK(hipGetLastError());
}

// loss = sum mask (O - T)^2 / (2 count); grad in the packed layout.  The
// loss is read back (synchronising) only when want_loss.
// count > 0: the mask sum given by the caller; count <= 0: summed on the
// device from Mk (no host round trip).
static float loss_grad(const Dims& d, const float* W, const float* X, const float* T, const float* Mk, int64_t B,
                       float count, float* grad, MlpWork& w, hipStream_t s, bool want_loss = true,
                       const float* rowcnt = nullptr)
{
    w.ensure(B);
    forward(d, W, X, B, w, s);
    const int nb = std::min<int64_t>(1024, (B * kOut + 255) / 256);
    if (count <= 0.f) {
        if (rowcnt) k_masksum<<<1, 256, 0, s>>>(B, rowcnt, w.count.p);
        else k_masksum<<<1, 256, 0, s>>>(B * kOut, Mk, w.count.p);
        k_mse<<<nb, 256, 0, s>>>(B * kOut, w.o.p, T, Mk, 1.f, w.count.p, w.go.p, w.part.p);
    } else {
        k_mse<<<nb, 256, 0, s>>>(B * kOut, w.o.p, T, Mk, 1.f / count, nullptr, w.go.p, w.part.p);
    }
    const int S = splits_for(B);
    // layer 3
    gemm_tn_split(kOut, kH, (int)B, w.go.p, kOut, w.h2.p, kH, grad + d.w3, w.split.p, S, s);
    colsum(B, kOut, w.go.p, grad + d.b3, w, s);
    gemm((int)B, kH, kOut, w.go.p, kOut, false, W + d.w3, kH, false, w.g2.p, kH, 1.f, 0.f, s);
    k_relu_back<<<grid_for(B * kH), 256, 0, s>>>(B, kH, w.h2.p, w.g2.p);
    // layer 2
    gemm_tn_split(kH, kH, (int)B, w.g2.p, kH, w.h1.p, kH, grad + d.w2, w.split.p, S, s);
    colsum(B, kH, w.g2.p, grad + d.b2, w, s);
    gemm((int)B, kH, kH, w.g2.p, kH, false, W + d.w2, kH, false, w.g1.p, kH, 1.f, 0.f, s);
    k_relu_back<<<grid_for(B * kH), 256, 0, s>>>(B, kH, w.h1.p, w.g1.p);
    // layer 1
    gemm_tn_split(kH, d.in, (int)B, w.g1.p, kH, X, d.in, grad + d.w1, w.split.p, S, s);
    colsum(B, kH, w.g1.p, grad + d.b1, w, s);
    HIPCK(hipGetLastError());
    if (want_loss && count <= 0.f) {
        HIPCK(hipMemcpyAsync(&count, w.count.p, sizeof(float), hipMemcpyDeviceToHost, s));
    }
    if (!want_loss) return 0.f;
    std::vector<float> part(nb);
    HIPCK(hipMemcpyAsync(part.data(), w.part.p, sizeof(float) * nb, hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    double l = 0;
    for (float v : part) l += v;
    return (float)(l / (2.0 * count));
}

// ---------------------------------------------------------------------
// BF16 inference on the matrix cores: C (M x N) = act(X W^T + b) with
// v_mfma_f32_16x16x16bf16_1k (FP32 accumulation).  X: M x K row-major,
// FP32 (the leaf features, rounded to BF16 on load) or BF16 (hidden
// activations); W: N x K row-major BF16; b FP32.  Lane layout (checked on
// the device with small integer matrices): A lane l holds
// A[l % 16][4 (l / 16) + e], B lane l holds B[4 (l / 16) + e][l % 16], and
// result register v of lane l is D[4 (l / 16) + v][l % 16].  One wave
// computes 16 rows x N; K is a multiple of 16.
// ---------------------------------------------------------------------
typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf_bits(float x)
{
    return __builtin_bit_cast(short, __float2bfloat16(x));
}
__device__ __forceinline__ void store_out(float* p, float v) { *p = v; }
__device__ __forceinline__ void store_out(__hip_bfloat16* p, float v) { *p = __float2bfloat16(v); }

template <typename TX, int N, bool kRelu, typename TO>
__global__ void __launch_bounds__(256)
k_dense_bf16(int64_t M, int K, const TX* __restrict__ X, const __hip_bfloat16* __restrict__ W,
             const float* __restrict__ bias, TO* __restrict__ C)
{
    constexpr int NT = N / 16;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (m0 >= M) return;
    const int li = lane % 16, lk = lane / 16;
    const int64_t row = min(m0 + li, M - 1);   // rows past M re-read row M - 1; never stored
    f4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        const int kk = k0 + 4 * lk;
        bf4 a;
        if constexpr (sizeof(TX) == 4) {
            const float4 v = *reinterpret_cast<const float4*>(X + row * K + kk);
            a = bf4{bf_bits(v.x), bf_bits(v.y), bf_bits(v.z), bf_bits(v.w)};
        } else {
            a = *reinterpret_cast<const bf4*>(X + row * K + kk);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const bf4 b = *reinterpret_cast<const bf4*>(W + (int64_t)(16 * t + li) * K + kk);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t m = m0 + 4 * lk + v;
            const int n = 16 * t + li;
            if (m < M) {
                float y = acc[t][v] + bias[n];
                if (kRelu) y = fmaxf(y, 0.f);
                store_out(C + m * N + n, y);
            }
        }
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ src, __hip_bfloat16* __restrict__ dst)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = __float2bfloat16(src[e]);
}

// ---------------------------------------------------------------------
// Leaf features and corrections
// ---------------------------------------------------------------------
__device__ __forceinline__ uint32_t compact_bits(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0F0F0F0Fu;
    v = (v | (v >> 4)) & 0x00FF00FFu;
    v = (v | (v >> 8)) & 0x0000FFFFu;
    return v;
}

// One wave per leaf: features (nleaf x 192) and |r_X|.  Optionally also
// the normalised target t_i = z_i / |r_X| and the slot mask.
__global__ void __launch_bounds__(256)
k_features(int32_t nleaf, const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
           const uint32_t* __restrict__ key, int kappa, double R, const double* __restrict__ xyt,
           const int32_t* __restrict__ perm, const double* __restrict__ r, const double* __restrict__ zt, double zscale,
           float* __restrict__ F, float* __restrict__ rn, float* __restrict__ T, float* __restrict__ Mk)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t X = blockIdx.x * 4 + wave;
    if (X >= nleaf) return;
    const int32_t m = count[X], r0 = begin[X];
    const bool on = lane < m;
    const double ri = on ? r[perm[r0 + lane]] : 0.0;
    double ss = ri * ri;
    for (int d = 32; d > 0; d >>= 1) ss += __shfl_xor(ss, d, kWave);
    const double nrm = sqrt(ss), inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    const uint32_t k = key[X];
    const double h = R / (double)(1u << kappa);
    const double cx = -R + (2.0 * compact_bits(k) + 1.0) * h, cy = -R + (2.0 * compact_bits(k >> 1) + 1.0) * h;
    float* f = F + (int64_t)X * kIn;
    f[lane] = on ? (float)((xyt[2 * (r0 + lane)] - cx) / h) : 0.f;
    f[64 + lane] = on ? (float)((xyt[2 * (r0 + lane) + 1] - cy) / h) : 0.f;
    f[128 + lane] = on ? (float)(ri * inv) : 0.f;
    if (lane == 0) rn[X] = (float)nrm;
    if (T) {
        T[(int64_t)X * kOut + lane] = on ? (float)((zt[perm[r0 + lane]] * zscale - ri) * inv) : 0.f;
        Mk[(int64_t)X * kOut + lane] = (on && nrm > 0.0) ? 1.f : 0.f;
    }
}

// z(X) = s (r(X) + |r_X| O(X)) in caller order.
__global__ void k_correction(int32_t nleaf, const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
                             const int32_t* __restrict__ perm, const float* __restrict__ O, const float* __restrict__ rn,
                             double s, const double* __restrict__ r, double* __restrict__ z)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t X = blockIdx.x * 4 + wave;
    if (X >= nleaf) return;
    if (lane < count[X]) {
        const int32_t p = perm[begin[X] + lane];
        z[p] = s * (r[p] + (double)O[(int64_t)X * kOut + lane] * (double)rn[X]);
    }
}

// Patch input (one wave per leaf X): 5 groups of 64 slots -- X, then its
// edge-sharing leaves to the left, right, below and above (a missing one
// leaves its group zero) -- each group (x offset / h, y offset / h,
// r_i / |r_P|) with offsets from the centre of X, h its half side, and
// |r_P| the residual norm over the whole patch.  Optionally the target
// t_i = zd_i zscale / |r_P| on X's slots and their mask.
__global__ void __launch_bounds__(256)
k_patch_features(int32_t nleaf, const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
                 const uint32_t* __restrict__ key, const int32_t* __restrict__ near_ptr,
                 const int32_t* __restrict__ near_src, int kappa, double R, const double* __restrict__ xyt,
                 const int32_t* __restrict__ perm, const double* __restrict__ r, const double* __restrict__ zd,
                 double zscale, float* __restrict__ F, float* __restrict__ rn, float* __restrict__ T,
                 float* __restrict__ Mk)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t X = blockIdx.x * 4 + wave;
    if (X >= nleaf) return;
    const uint32_t kx = key[X];
    const int32_t ix = (int32_t)compact_bits(kx), iy = (int32_t)compact_bits(kx >> 1);
    const double h = R / (double)(1u << kappa);
    const double cx = -R + (2.0 * ix + 1.0) * h, cy = -R + (2.0 * iy + 1.0) * h;
    // group of each near block: 0 self, 1 left, 2 right, 3 below, 4 above
    int32_t box[5] = {-1, -1, -1, -1, -1};
    for (int32_t q = near_ptr[X]; q < near_ptr[X + 1]; ++q) {
        const int32_t Y = near_src[q];
        const uint32_t ky = key[Y];
        const int32_t dx = (int32_t)compact_bits(ky) - ix, dy = (int32_t)compact_bits(ky >> 1) - iy;
        const int gidx = Y == X ? 0 : dx < 0 ? 1 : dx > 0 ? 2 : dy < 0 ? 3 : 4;
        box[gidx] = Y;
    }
    double ss = 0.0;
    double rv[5];
    for (int gi = 0; gi < 5; ++gi) {
        rv[gi] = 0.0;
        if (box[gi] >= 0 && lane < count[box[gi]]) rv[gi] = r[perm[begin[box[gi]] + lane]];
        ss += rv[gi] * rv[gi];
    }
    for (int d = 32; d > 0; d >>= 1) ss += __shfl_xor(ss, d, kWave);
    const double nrm = sqrt(ss), inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    float* f = F + (int64_t)X * kInPatch;
    for (int gi = 0; gi < 5; ++gi) {
        const bool on = box[gi] >= 0 && lane < count[box[gi]];
        const int32_t t = on ? begin[box[gi]] + lane : 0;
        f[gi * kIn + lane] = on ? (float)((xyt[2 * t] - cx) / h) : 0.f;
        f[gi * kIn + 64 + lane] = on ? (float)((xyt[2 * t + 1] - cy) / h) : 0.f;
        f[gi * kIn + 128 + lane] = on ? (float)(rv[gi] * inv) : 0.f;
    }
    if (lane == 0) rn[X] = (float)nrm;
    if (T) {
        const bool on = lane < count[X];
        T[(int64_t)X * kOut + lane] = on ? (float)(zd[perm[begin[X] + lane]] * zscale * inv) : 0.f;
        Mk[(int64_t)X * kOut + lane] = (on && nrm > 0.0) ? 1.f : 0.f;
    }
}

// z(X) += s |r_P| O(X) in caller order (z holds the block-Jacobi step).
__global__ void k_patch_correction(int32_t nleaf, const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
                                   const int32_t* __restrict__ perm, const float* __restrict__ O,
                                   const float* __restrict__ rn, double s, double* __restrict__ z)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t X = blockIdx.x * 4 + wave;
    if (X >= nleaf) return;
    if (lane < count[X]) z[perm[begin[X] + lane]] += s * (double)O[(int64_t)X * kOut + lane] * (double)rn[X];
}

// out = a - b
__global__ void k_diff(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = a[e] - b[e];
}

// Counter-based uniform numbers in [-1, 1): splitmix64 of (seed, index).
__device__ __forceinline__ double uniform_pm1(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_random(int64_t n, uint64_t seed, double* __restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = uniform_pm1(seed, (uint64_t)e);
}

// Batch of step `it`: sample index of row b = splitmix64 of (seed, it B + b)
// modulo nsamp, then rows of F (192), T and Mk (64) gathered (no host
// round trip per step).
__global__ void k_sample_batch(int32_t B, int in, int64_t nsamp, uint64_t seed, int64_t it, const float* __restrict__ F,
                               const float* __restrict__ T, const float* __restrict__ Mk, float* __restrict__ Fb,
                               float* __restrict__ Tb, float* __restrict__ Mb, float* __restrict__ rowcnt)
{
    const int32_t b = blockIdx.x;
    if (b >= B) return;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * ((uint64_t)it * (uint64_t)B + (uint64_t)b + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int64_t sidx = (int64_t)(z % (uint64_t)nsamp);
    for (int e = threadIdx.x; e < in; e += blockDim.x) Fb[(int64_t)b * in + e] = F[sidx * in + e];
    float c = 0.f;
    for (int e = threadIdx.x; e < kOut; e += blockDim.x) {
        Tb[(int64_t)b * kOut + e] = T[sidx * kOut + e];
        const float mv = Mk[sidx * kOut + e];
        Mb[(int64_t)b * kOut + e] = mv;
        c += mv;
    }
    // the block is one wave (64 threads): its valid-slot count
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, kWave);
    if (threadIdx.x == 0) rowcnt[b] = c;
}


struct MlpState {
    Dims d = kLeafDims;   // parameter layout of the current network
    int input = H2D_MLP_INPUT_LEAF;
    double scale = 1.0;   // s: z ~ s r over the training solves
    DBuf<float> w, m1, m2, grad;
    MlpWork work;
    DBuf<float> feat, rn, out;               // inference: features, |r_X|, network output (FP32)
    DBuf<__hip_bfloat16> w16, h1b, h2b;      // inference: BF16 weights (W1, W2, W3) and hidden activations
    int64_t feat_cap = 0;
    bool w16_ok = false;                     // w16 holds the current FP32 weights rounded to BF16
    bool ready = false;
    DBuf<int32_t> nsrc;                      // device copy of the near-list sources (patch input)
};

// BF16 forward of nleaf leaves into S.out (FP32 nleaf x 64).
static void forward_bf16(MlpState& S, int64_t nleaf, hipStream_t s)
{
    const Dims& d = S.d;
    const int64_t n1 = (int64_t)kH * d.in, n2 = (int64_t)kH * kH, n3 = (int64_t)kOut * kH;
    if (!S.w16_ok) {
        S.w16.alloc(n1 + n2 + n3);
        k_to_bf16<<<256, 256, 0, s>>>(n1, S.w.p + d.w1, S.w16.p);
        k_to_bf16<<<256, 256, 0, s>>>(n2, S.w.p + d.w2, S.w16.p + n1);
        k_to_bf16<<<64, 256, 0, s>>>(n3, S.w.p + d.w3, S.w16.p + n1 + n2);
        S.w16_ok = true;
    }
    const unsigned g = (unsigned)((nleaf + 63) / 64);
    k_dense_bf16<float, kH, true, __hip_bfloat16><<<g, 256, 0, s>>>(nleaf, d.in, S.feat.p, S.w16.p, S.w.p + d.b1,
                                                                     S.h1b.p);
    k_dense_bf16<__hip_bfloat16, kH, true, __hip_bfloat16><<<g, 256, 0, s>>>(nleaf, kH, S.h1b.p, S.w16.p + n1,
                                                                              S.w.p + d.b2, S.h2b.p);
    k_dense_bf16<__hip_bfloat16, kOut, false, float><<<g, 256, 0, s>>>(nleaf, kH, S.h2b.p, S.w16.p + n1 + n2,
                                                                        S.w.p + d.b3, S.out.p);
    HIPCK(hipGetLastError());
}

// The network has 64 point slots per leaf: leaves above 64 points are
// refused, as block-Jacobi refuses them.
static void check_leaf_slots(const Handle& H)
{
    const Level& LL = H.lev[H.kappa];
    for (int64_t x = 0; x < LL.nbox; ++x)
        if (LL.h_count[x] > kOut)
            fail(H2D_EUNSUPPORTED, "the MLP preconditioner needs leaves of at most 64 points (a leaf holds " +
                                       std::to_string(LL.h_count[x]) + ")");
}

MlpState& mlp_state(Handle& H)
{
    if (!H.mlp) H.mlp = std::make_shared<MlpState>();
    return *H.mlp;
}

void mlp_apply(Handle& H, const double* r, double* z, hipStream_t s)
{
    MlpState& S = mlp_state(H);
    if (!S.ready) fail(H2D_EINVAL, "the MLP preconditioner was not trained (h2d_mlp_train) or loaded");
    check_leaf_slots(H);
    const Level& LL = H.lev[H.kappa];
    const int32_t nleaf = (int32_t)LL.nbox;
    if (S.feat_cap < nleaf || (int64_t)S.feat.n < (int64_t)nleaf * S.d.in) {
        S.feat.alloc((size_t)nleaf * S.d.in);
        S.rn.alloc(nleaf);
        S.out.alloc((size_t)nleaf * kOut);
        S.h1b.alloc((size_t)nleaf * kH);
        S.h2b.alloc((size_t)nleaf * kH);
        S.feat_cap = nleaf;
    }
    if (S.input == H2D_MLP_INPUT_PATCH) {
        // block-Jacobi step, then the learned correction from the patch
        if (!H.bj_ready) fail(H2D_EINVAL, "the patch-input MLP needs block-Jacobi (h2d_bj_setup)");
        precond_apply(H, H2D_PC_BLOCK_JACOBI, r, z, s);
        k_patch_features<<<(nleaf + 3) / 4, 256, 0, s>>>(nleaf, LL.begin.p, LL.count.p, LL.key.p, H.near_ptr.p,
                                                         S.nsrc.p, H.kappa, H.R, H.xyt.p, H.perm.p, r, nullptr, 0.0,
                                                         S.feat.p, S.rn.p, nullptr, nullptr);
        forward_bf16(S, nleaf, s);
        k_patch_correction<<<(nleaf + 3) / 4, 256, 0, s>>>(nleaf, LL.begin.p, LL.count.p, H.perm.p, S.out.p, S.rn.p,
                                                           S.scale, z);
        HIPCK(hipGetLastError());
        return;
    }
    k_features<<<(nleaf + 3) / 4, 256, 0, s>>>(nleaf, LL.begin.p, LL.count.p, LL.key.p, H.kappa, H.R, H.xyt.p,
                                               H.perm.p, r, nullptr, 0.0, S.feat.p, S.rn.p, nullptr, nullptr);
    forward_bf16(S, nleaf, s);
    k_correction<<<(nleaf + 3) / 4, 256, 0, s>>>(nleaf, LL.begin.p, LL.count.p, H.perm.p, S.out.p, S.rn.p, S.scale,
                                                 r, z);
    HIPCK(hipGetLastError());
}

// ---------------------------------------------------------------------
// Patch targets: for leaf X with near list {X} u E_X (the self block and
// the edge-sharing leaves, the blocks the method stores dense), the patch
// P = X followed by the points of E_X, the patch system K(P, P) z_P = r_P
// solved exactly, and z_X kept (a restricted additive Schwarz step).  One
// workgroup per leaf: the augmented matrix [K(P, P) | r_P of every
// right-hand side] is built column-major in the workgroup's slice of a
// global work array, reduced by Gaussian elimination with partial
// pivoting, and back-substituted.
// ---------------------------------------------------------------------
constexpr int kPatchMax = 5 * 64;   // self + 4 edge sharers, 64 points each

__global__ void __launch_bounds__(256)
k_patch_solve(int32_t x0, int32_t nx, const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
              const int32_t* __restrict__ near_ptr, const int32_t* __restrict__ near_src, KernelParams kp,
              const double* __restrict__ xyt, const int32_t* __restrict__ perm, int64_t n, int ns,
              const double* __restrict__ R, double* __restrict__ Z, double* __restrict__ work, int64_t slot_elems,
              int lds, int* __restrict__ singular)
{
    extern __shared__ double lds_aug[];
    __shared__ int32_t pts[kPatchMax];
    __shared__ int32_t pv;
    __shared__ int32_t npts;
    const int32_t X = x0 + blockIdx.x;
    if (blockIdx.x >= nx) return;
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    if (t == 0) {
        int32_t c = 0;
        for (int32_t i = 0; i < count[X]; ++i) pts[c++] = begin[X] + i;
        for (int32_t q = near_ptr[X]; q < near_ptr[X + 1]; ++q) {
            const int32_t y = near_src[q];
            if (y == X) continue;
            for (int32_t i = 0; i < count[y]; ++i) pts[c++] = begin[y] + i;
        }
        npts = c;
    }
    __syncthreads();
    const int m = npts, mx = count[X], nc = m + ns;
    // m x (m + ns), column-major, ld = m: in LDS when the launch gave room
    // for the largest patch of the chunk, else in the workgroup's slice of
    // the global work array
    double* A = lds ? lds_aug : work + (int64_t)blockIdx.x * slot_elems;
    for (int64_t e = t; e < (int64_t)m * nc; e += blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        const int32_t pi = pts[i];
        double v;
        if (j < m) {
            const int32_t pj = pts[j];
            v = kernel_entry(kp, xyt[2 * pi], xyt[2 * pi + 1], xyt[2 * pj], xyt[2 * pj + 1], pi == pj);
        } else {
            v = R[(int64_t)(j - m) * n + perm[pi]];
        }
        A[(int64_t)j * m + i] = v;
    }
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        if (wave == 0) {
            double best = -1.0;
            int bi = -1;
            for (int i = k + lane; i < m; i += kWave) {
                const double v = fabs(A[(int64_t)k * m + i]);
                if (v > best) { best = v; bi = i; }
            }
            for (int d = 32; d > 0; d >>= 1) {
                const double ov = __shfl_xor(best, d, kWave);
                const int oi = __shfl_xor(bi, d, kWave);
                if (ov > best || (ov == best && oi >= 0 && (bi < 0 || oi < bi))) { best = ov; bi = oi; }
            }
            if (lane == 0) {
                pv = bi;
                if (!(best > 0.0)) atomicOr(singular, 1);
            }
        }
        __syncthreads();
        const int p = pv;
        if (p != k && p >= 0)
            for (int j = k + t; j < nc; j += blockDim.x) {
                const double a = A[(int64_t)j * m + k];
                A[(int64_t)j * m + k] = A[(int64_t)j * m + p];
                A[(int64_t)j * m + p] = a;
            }
        __syncthreads();
        const double d = A[(int64_t)k * m + k];
        if (d != 0.0)
            for (int i = k + 1 + t; i < m; i += blockDim.x) A[(int64_t)k * m + i] /= d;
        __syncthreads();
        const int rem = m - k - 1, cols = nc - k - 1;
        for (int64_t e = t; e < (int64_t)rem * cols; e += blockDim.x) {
            const int i = k + 1 + (int)(e % rem), j = k + 1 + (int)(e / rem);
            A[(int64_t)j * m + i] -= A[(int64_t)k * m + i] * A[(int64_t)j * m + k];
        }
        __syncthreads();
    }
    // back substitution, one thread per right-hand side; only the first mx
    // unknowns (the leaf's own points) are kept
    for (int q = t; q < ns; q += blockDim.x) {
        double* b = A + (int64_t)(m + q) * m;
        for (int k = m - 1; k >= 0; --k) {
            double v = b[k];
            for (int j = k + 1; j < m; ++j) v -= A[(int64_t)j * m + k] * b[j];
            const double d = A[(int64_t)k * m + k];
            b[k] = d != 0.0 ? v / d : 0.0;
        }
        for (int i = 0; i < mx; ++i) Z[(int64_t)q * n + perm[pts[i]]] = b[i];
    }
}

// Patch targets z_q (n each, caller order) for the ns right-hand sides r_q.
static void patch_targets(Handle& H, const double* R, double* Z, int ns, hipStream_t s)
{
    const Level& LL = H.lev[H.kappa];
    const int32_t nleaf = (int32_t)LL.nbox;
    int32_t pmax = 0;
    for (int32_t x = 0; x < nleaf; ++x) {
        int32_t c = 0;
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) c += LL.h_count[H.h_near_src[q]];
        pmax = std::max(pmax, c);
    }
    if (pmax > kPatchMax) fail(H2D_EUNSUPPORTED, "a near-field patch exceeds 320 points");
    DBuf<int32_t> nsrc;
    nsrc.alloc(std::max<size_t>(H.h_near_src.size(), 1));
    HIPCK(hipMemcpyAsync(nsrc.p, H.h_near_src.data(), sizeof(int32_t) * H.h_near_src.size(), hipMemcpyHostToDevice,
                         s));
    const int64_t slot = (int64_t)pmax * (pmax + ns);
    // the augmented matrix in LDS when it fits (the common case), else in
    // global memory, a chunk of leaves at a time
    int dev = 0, lds_max = 0;
    HIPCK(hipGetDevice(&dev));
    HIPCK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int64_t static_lds = (int64_t)sizeof(int32_t) * (kPatchMax + 2) + 64;
    const int64_t need = slot * (int64_t)sizeof(double);
    bool lds = need + static_lds <= lds_max;
    if (lds && need > 48 * 1024)
        lds = hipFuncSetAttribute(reinterpret_cast<const void*>(k_patch_solve),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) == hipSuccess;
    (void)hipGetLastError();
    const int32_t chunk =
        lds ? nleaf : (int32_t)std::max<int64_t>(1, std::min<int64_t>(nleaf, (int64_t)(512ll << 20) / 8 / slot));
    DBuf<double> work;
    if (!lds) work.alloc((size_t)chunk * slot);
    DBuf<int> sing;
    sing.alloc(1);
    HIPCK(hipMemsetAsync(sing.p, 0, sizeof(int), s));
    for (int32_t x0 = 0; x0 < nleaf; x0 += chunk) {
        const int32_t nx = std::min(chunk, nleaf - x0);
        k_patch_solve<<<nx, 256, lds ? (size_t)need : 0, s>>>(x0, nx, LL.begin.p, LL.count.p, H.near_ptr.p, nsrc.p,
                                                              H.kern, H.xyt.p, H.perm.p, H.n, ns, R, Z, work.p, slot,
                                                              lds ? 1 : 0, sing.p);
        HIPCK(hipGetLastError());
    }
    int hs = 0;
    HIPCK(hipMemcpyAsync(&hs, sing.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    if (hs) fail(H2D_EINVAL, "a near-field patch system is singular");
}

// Xavier-uniform initial weights from the counter-based generator.
__global__ void k_init_w(float* __restrict__ w, uint64_t seed, Dims d)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < d.params; e += (int64_t)gridDim.x * blockDim.x) {
        float lim = 0.f;
        if (e < d.b1) lim = sqrtf(6.f / (d.in + kH));
        else if (e >= d.w2 && e < d.b2) lim = sqrtf(6.f / (kH + kH));
        // the last layer starts at zero: the untrained preconditioner is s I
        w[e] = lim * (float)uniform_pm1(seed, (uint64_t)e);
    }
}

static void ensure_weights(MlpState& S, hipStream_t s)
{
    if (S.w.p && (int64_t)S.w.n == S.d.params) return;
    S.w.alloc(S.d.params);
    S.m1.alloc(S.d.params);
    S.m2.alloc(S.d.params);
    S.grad.alloc(S.d.params);
    HIPCK(hipMemsetAsync(S.m1.p, 0, sizeof(float) * S.d.params, s));
    HIPCK(hipMemsetAsync(S.m2.p, 0, sizeof(float) * S.d.params, s));
    S.ready = false;
}

void mlp_train(Handle& H, const h2d_mlp_train_opts& o, h2d_mlp_train_info* info, hipStream_t s)
{
    check_leaf_slots(H);
    MlpState& S = mlp_state(H);
    const bool patch_in = o.input == H2D_MLP_INPUT_PATCH;
    const Dims d = patch_in ? kPatchDims : kLeafDims;
    if (S.d.in != d.in) S.ready = false;   // another network: start from fresh weights
    S.d = d;
    S.input = patch_in ? H2D_MLP_INPUT_PATCH : H2D_MLP_INPUT_LEAF;
    const Level& LL = H.lev[H.kappa];
    const int32_t nleaf = (int32_t)LL.nbox;
    const int64_t n = H.n;
    const int ns = o.n_solves;
    auto t0 = std::chrono::steady_clock::now();
    // training pairs from the method's own FP64 solves
    const int64_t nsamp = (int64_t)ns * nleaf;
    DBuf<float> F, T, Mk, rn;
    F.alloc((size_t)nsamp * d.in);
    T.alloc((size_t)nsamp * kOut);
    Mk.alloc((size_t)nsamp * kOut);
    rn.alloc(nsamp);
    h2d_solve_opts so{};
    so.mode = H2D_SOLVE_PLAIN;
    so.restart = 50;
    so.max_iter = 500;
    so.precond = H2D_PC_NONE;
    int solves_ok = 0;
    if ((o.target == H2D_MLP_TARGET_LEAF || patch_in) && !H.bj_ready) bj_setup(H, s);
    DBuf<double> R, Z, W, Zb;
    R.alloc((size_t)n * ns);
    Z.alloc((size_t)n * ns);
    W.alloc((size_t)n);
    if (patch_in) Zb.alloc((size_t)n * ns);
    double zr = 0.0, rr = 0.0;
    std::vector<double> hw(n);
    for (int q = 0; q < ns; ++q) {
        double* rq = R.p + (int64_t)q * n;
        double* zq = Z.p + (int64_t)q * n;
        k_random<<<grid_for(n), 256, 0, s>>>(n, o.seed + 7919ull * (uint64_t)q, rq);
        // Residuals met inside a Krylov solve are not white noise: sample q
        // is A^p r for p = q mod 4 (random r, rescaled to unit RMS after each
        // product), so the pairs cover the smoother vectors as well.
        for (int p = 0; p < q % 4; ++p) {
            launch_matvec(H, rq, W.p, 1, n, H2D_P_FP64, s);
            HIPCK(hipMemcpyAsync(hw.data(), W.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
            HIPCK(hipStreamSynchronize(s));
            double nn = 0.0;
            for (int64_t i = 0; i < n; ++i) nn += hw[i] * hw[i];
            const double f = nn > 0.0 ? std::sqrt((double)n / nn) : 1.0;
            for (int64_t i = 0; i < n; ++i) hw[i] *= f;
            HIPCK(hipMemcpyAsync(rq, hw.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
        }
        if (patch_in) precond_apply(H, H2D_PC_BLOCK_JACOBI, rq, Zb.p + (int64_t)q * n, s);
        if (o.target == H2D_MLP_TARGET_GLOBAL) {
            h2d_solve_info si{};
            h2d_status st = solve(H, rq, zq, o.solve_tol, so, &si, s);
            if (st == H2D_OK) ++solves_ok;
        } else if (o.target == H2D_MLP_TARGET_LEAF) {
            precond_apply(H, H2D_PC_BLOCK_JACOBI, rq, zq, s);
            ++solves_ok;
        } else {
            ++solves_ok;   // patch targets: every right-hand side at once below
        }
    }
    if (o.target == H2D_MLP_TARGET_PATCH) patch_targets(H, R.p, Z.p, ns, s);
    // s: the least-squares scalar z ~ s r of the targets (leaf input) or of
    // the block-Jacobi steps the patch-input correction is added to
    {
        const DBuf<double>& Zs = patch_in ? Zb : Z;
        std::vector<double> hr(n), hz(n);
        for (int q = 0; q < ns; ++q) {
            HIPCK(hipMemcpyAsync(hr.data(), R.p + (int64_t)q * n, sizeof(double) * n, hipMemcpyDeviceToHost, s));
            HIPCK(hipMemcpyAsync(hz.data(), Zs.p + (int64_t)q * n, sizeof(double) * n, hipMemcpyDeviceToHost, s));
            HIPCK(hipStreamSynchronize(s));
            for (int64_t i = 0; i < n; ++i) { zr += hz[i] * hr[i]; rr += hr[i] * hr[i]; }
        }
    }
    S.scale = rr > 0.0 ? zr / rr : 1.0;
    if (!(S.scale != 0.0) || !std::isfinite(S.scale)) S.scale = 1.0;
    if (patch_in) {
        // target: what the target solve adds to the block-Jacobi step
        k_diff<<<grid_for(n * ns), 256, 0, s>>>(n * ns, Z.p, Zb.p, Z.p);
        S.nsrc.alloc(std::max<size_t>(H.h_near_src.size(), 1));
        HIPCK(hipMemcpyAsync(S.nsrc.p, H.h_near_src.data(), sizeof(int32_t) * H.h_near_src.size(),
                             hipMemcpyHostToDevice, s));
    }
    for (int q = 0; q < ns; ++q) {
        if (patch_in)
            k_patch_features<<<(nleaf + 3) / 4, 256, 0, s>>>(
                nleaf, LL.begin.p, LL.count.p, LL.key.p, H.near_ptr.p, S.nsrc.p, H.kappa, H.R, H.xyt.p, H.perm.p,
                R.p + (int64_t)q * n, Z.p + (int64_t)q * n, 1.0 / S.scale, F.p + (int64_t)q * nleaf * d.in,
                rn.p + (int64_t)q * nleaf, T.p + (int64_t)q * nleaf * kOut, Mk.p + (int64_t)q * nleaf * kOut);
        else
            k_features<<<(nleaf + 3) / 4, 256, 0, s>>>(nleaf, LL.begin.p, LL.count.p, LL.key.p, H.kappa, H.R, H.xyt.p,
                                                       H.perm.p, R.p + (int64_t)q * n, Z.p + (int64_t)q * n,
                                                       1.0 / S.scale, F.p + (int64_t)q * nleaf * d.in,
                                                       rn.p + (int64_t)q * nleaf, T.p + (int64_t)q * nleaf * kOut,
                                                       Mk.p + (int64_t)q * nleaf * kOut);
        HIPCK(hipGetLastError());
    }
    HIPCK(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    // training
    ensure_weights(S, s);
    if (!S.ready) {
        k_init_w<<<256, 256, 0, s>>>(S.w.p, o.seed ^ 0xA5A5A5A5ull, d);
        HIPCK(hipMemsetAsync(S.m1.p, 0, sizeof(float) * d.params, s));
        HIPCK(hipMemsetAsync(S.m2.p, 0, sizeof(float) * d.params, s));
    }
    const int B = std::max(1, std::min<int>(o.batch, (int)nsamp));
    DBuf<float> Fb, Tb, Mb, rc;
    Fb.alloc((size_t)B * d.in);
    Tb.alloc((size_t)B * kOut);
    Mb.alloc((size_t)B * kOut);
    rc.alloc(B);
    float first = 0.f, last = 0.f;
    const float b1 = 0.9f, b2 = 0.999f;
    const uint64_t bseed = o.seed * 6364136223846793005ull + 1442695040888963407ull;
    for (int it = 0; it < o.steps; ++it) {
        // batch drawn and gathered on the device; the mask sum (valid slots)
        // is taken there too, so a step has no host round trip
        k_sample_batch<<<B, 64, 0, s>>>(B, d.in, nsamp, bseed, it, F.p, T.p, Mk.p, Fb.p, Tb.p, Mb.p, rc.p);
        const bool report = it == 0 || it + 1 == o.steps;
        const float L = loss_grad(d, S.w.p, Fb.p, Tb.p, Mb.p, B, 0.f, S.grad.p, S.work, s, report, rc.p);
        if (it == 0) first = L;
        if (report) last = L;
        const float c1 = 1.f - std::pow(b1, (float)(it + 1)), c2 = 1.f - std::pow(b2, (float)(it + 1));
        k_adam<<<grid_for(d.params), 256, 0, s>>>(d.params, S.w.p, S.grad.p, S.m1.p, S.m2.p, o.lr, b1, b2, c1, c2,
                                                  1e-8f);
        HIPCK(hipGetLastError());
    }
    HIPCK(hipStreamSynchronize(s));
    S.ready = true;
    S.w16_ok = false;
    auto t2 = std::chrono::steady_clock::now();
    if (info) {
        info->seconds_data = std::chrono::duration<double>(t1 - t0).count();
        info->seconds_train = std::chrono::duration<double>(t2 - t1).count();
        info->loss_first = first;
        info->loss_last = last;
        info->n_samples = (int32_t)nsamp;
        info->solves_converged = solves_ok;
        info->scale = S.scale;
    }
}

void mlp_weights(Handle& H, float* out, const float* in, double* scale, hipStream_t s)
{
    MlpState& S = mlp_state(H);
    if (in && scale) S.scale = *scale;
    if (out && scale) *scale = S.scale;
    if (in) {
        // weights set from the host are always a leaf-input network
        S.d = kLeafDims;
        S.input = H2D_MLP_INPUT_LEAF;
        ensure_weights(S, s);
        HIPCK(hipMemcpyAsync(S.w.p, in, sizeof(float) * S.d.params, hipMemcpyHostToDevice, s));
        HIPCK(hipMemsetAsync(S.m1.p, 0, sizeof(float) * S.d.params, s));
        HIPCK(hipMemsetAsync(S.m2.p, 0, sizeof(float) * S.d.params, s));
        S.ready = true;
        S.w16_ok = false;
    }
    if (out) {
        if (!S.w.p) fail(H2D_EINVAL, "no MLP weights");
        HIPCK(hipMemcpyAsync(out, S.w.p, sizeof(float) * S.d.params, hipMemcpyDeviceToHost, s));
    }
    HIPCK(hipStreamSynchronize(s));
}

float mlp_loss_grad(const float* W, const float* X, const float* T, const float* Mk, int32_t B, float* grad,
                    hipStream_t s)
{
    MlpWork w;
    std::vector<float> hm((size_t)B * kOut);
    HIPCK(hipMemcpyAsync(hm.data(), Mk, sizeof(float) * hm.size(), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    double cnt = 0;
    for (float v : hm) cnt += v;
    return loss_grad(kLeafDims, W, X, T, Mk, B, (float)std::max(1.0, cnt), grad, w, s);
}

}  // namespace h2d
