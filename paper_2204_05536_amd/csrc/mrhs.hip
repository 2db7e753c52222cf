// Multi-RHS form of Algorithm 2 on the matrix cores: Y = A_hat X for
// blocks of 16 right-hand sides.  With 16 columns the products become real
// contractions, T_b = V_b^T X(Y_b) (k x 16) and Y(X) += U_b T_b, computed
// with v_mfma_f64_16x16x4f64 on the FP64 pools and, on the FP16 / BF16
// pools, with v_mfma_f32_16x16x4f32: each stored value is widened to FP32
// as it is loaded, right-hand sides, T and the sums stay FP32, and the
// products accumulate in FP32 (the accuracy of the single-RHS half path).
// Schedule, storage and the tree are those of the single-RHS path
// (matvec.hip); only the inner products differ.  The half pools keep their
// per-block scales: phase B multiplies each 4-column group of U or D by its
// block's scale (the phase-B table entries carry it), and the self-block
// diagonal held apart in FP32 is added when the result is scattered back.
//
// MFMA operand layout (16 x 16 output, K = 4 per instruction), lane l:
//   A (16 x 4):  A[l % 16][l / 16]
//   B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): register v holds D[4 v + l / 16][l % 16] for the FP64
//                instruction, D[4 (l / 16) + v][l % 16] for the FP32 one
//                (checked on the device)
// Right-hand sides are kept point-major inside the kernels (16 consecutive
// values per point), so a B fragment is 64 consecutive doubles.
#include "h2d_impl.h"

#include <algorithm>
#include <type_traits>

namespace h2d {

constexpr int kR = 16;
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;

// Storage type T -> arithmetic type A, accumulator tile V4, the matrix
// instruction, and loads of one stored value (through a buffer resource at
// a byte offset, or through a pointer) widened to A.
template <typename T> struct MrT;
template <> struct MrT<double> {
    using A = double;
    using V4 = d4;
    static __device__ __forceinline__ V4 mma(A a, A b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ A load(rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    }
    static __device__ __forceinline__ A get(const double* p) { return *p; }
    // output row of accumulator register v in lane group lk = lane / 16
    static __device__ __forceinline__ int row(int v, int lk) { return 4 * v + lk; }
};
template <> struct MrT<__half> {
    using A = float;
    using V4 = f4;
    static __device__ __forceinline__ V4 mma(A a, A b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ A load(rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0));
    }
    static __device__ __forceinline__ A get(const __half* p) { return __half2float(*p); }
    static __device__ __forceinline__ int row(int v, int lk) { return 4 * lk + v; }
};
template <> struct MrT<__hip_bfloat16> {
    using A = float;
    using V4 = f4;
    static __device__ __forceinline__ V4 mma(A a, A b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ A load(rsrc_t r, uint32_t voff, uint32_t soff)
    {
        const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
        return __builtin_bit_cast(float, h << 16);
    }
    static __device__ __forceinline__ A get(const __hip_bfloat16* p) { return __bfloat162float(*p); }
    static __device__ __forceinline__ int row(int v, int lk) { return 4 * lk + v; }
};
// Work-vector values (x, T) through a buffer resource.
template <typename A> __device__ __forceinline__ A vload(rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ double vload<double>(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ float vload<float>(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

__device__ __forceinline__ int32_t uni_i(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni_l(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A device address from an instance table as a global-memory pointer.
template <typename T> __device__ __forceinline__ T* gp(uint64_t a)
{
    return (T*)(__attribute__((address_space(1))) T*)a;
}

// Work item i of a table-driven kernel: (instance, item); without a list,
// instance 0 and item i.
__device__ __forceinline__ int2 work_at(const int2* __restrict__ work, int32_t i)
{
    const int2 w = work ? work[i] : make_int2(0, i);
    // wave-uniform: the instance's fields then load through the scalar cache
    return make_int2(__builtin_amdgcn_readfirstlane(w.x), __builtin_amdgcn_readfirstlane(w.y));
}

// xs[iperm[c] * 16 + r] = x[(r0 + r) * ld + c] for r < nr, 0 beyond.  One
// workgroup per 64 caller-order points of an instance: the right-hand-side
// rows are read coalesced, transposed through LDS, and each point's 16
// values are written as one segment at its tree position.
template <typename A>
__global__ void __launch_bounds__(256)
k_gather_mr(const MRInst* __restrict__ insts, const int2* __restrict__ work, int32_t nwork, MRIo io0,
            const MRIo* __restrict__ iot, int32_t r0, int32_t nr)
{
    __shared__ double tile[kR][kWave + 1];
    if ((int32_t)blockIdx.x >= nwork) return;
    const int2 wk = work_at(work, blockIdx.x);
    const MRInst& I = insts[wk.x];
    const MRIo io = iot ? iot[wk.x] : io0;
    const int32_t n = I.n, c0 = wk.y * kWave;
    const double* x = gp<const double>(io.x) + (int64_t)r0 * io.ld;
    A* xs = gp<A>(I.xs);
    const int32_t* iperm = gp<const int32_t>(I.iperm);
    for (int e = threadIdx.x; e < kR * kWave; e += blockDim.x) {
        const int r = e / kWave, c = e % kWave;
        tile[r][c] = (r < nr && c0 + c < n) ? x[(int64_t)r * io.ld + c0 + c] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kR * kWave; e += blockDim.x) {
        const int c = e / kR, r = e % kR;
        if (c0 + c < n) xs[(int64_t)iperm[c0 + c] * kR + r] = (A)tile[r][c];
    }
}

// y[(r0 + r) * ld + c] = (yleaf + yanc)[iperm[c] * 16 + r] for r < nr: the
// inverse of the gather, from the tree-ordered point-major leaf and
// ancestor sums back to caller order (half pools: plus the FP32 self
// diagonal times x).
template <typename A>
__global__ void __launch_bounds__(256)
k_scatter_mr(const MRInst* __restrict__ insts, const int2* __restrict__ work, int32_t nwork, MRIo io0,
             const MRIo* __restrict__ iot, int32_t r0, int32_t nr)
{
    __shared__ double tile[kR][kWave + 1];
    if ((int32_t)blockIdx.x >= nwork) return;
    const int2 wk = work_at(work, blockIdx.x);
    const MRInst& I = insts[wk.x];
    const MRIo io = iot ? iot[wk.x] : io0;
    const int32_t n = I.n, c0 = wk.y * kWave;
    const A* yt = gp<const A>(I.yl);
    const A* ya = I.has_b1 ? gp<const A>(I.yp) : nullptr;
    const float* diag = I.diag ? gp<const float>(I.diag) : nullptr;
    const A* xs = gp<const A>(I.xs);
    const int32_t* iperm = gp<const int32_t>(I.iperm);
    for (int e = threadIdx.x; e < kR * kWave; e += blockDim.x) {
        const int c = e / kR, r = e % kR;
        if (c0 + c < n) {
            const int32_t i = iperm[c0 + c];
            const int64_t g = (int64_t)i * kR + r;
            A v = ya ? yt[g] + ya[g] : yt[g];
            if (diag) v += (A)diag[i] * xs[g];
            tile[r][c] = (double)v;
        }
    }
    __syncthreads();
    double* y = gp<double>(io.y) + (int64_t)r0 * io.ld;
    for (int e = threadIdx.x; e < kR * kWave; e += blockDim.x) {
        const int r = e / kWave, c = e % kWave;
        if (r < nr && c0 + c < n) y[(int64_t)r * io.ld + c0 + c] = tile[r][c];
    }
}

__global__ void k_iperm(const int32_t* __restrict__ perm, int32_t n, int32_t* __restrict__ iperm)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) iperm[perm[i]] = i;
}

// Every load below is unconditional: addresses are clamped into the
// operand (rows past the end re-read the last row, and their results are
// never stored; K indices past the end re-read the last column with the
// other operand zeroed), so the compiler can issue a whole group of loads
// before the matrix instructions that consume them.  Loads go through
// buffer resources: a wave-uniform base and extent in scalar registers,
// a scalar offset per K-step and a 32-bit per-lane offset that stays fixed
// over the loop, so a group of 4 K-steps needs no per-lane address math.
// An offset at or past the extent reads 0 (never the case by construction).
template <typename T>
__device__ __forceinline__ rsrc_t rsrc(const T* base, int64_t elems)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, (int)(elems * (int64_t)sizeof(T)),
                                             0x00020000);
}

// T rows q0 + 16 t (t < NT) += V(0..rows-1, q)^T X(0..rows-1, :) for one
// block: V row-major with k columns and row stride ldv at Vb, X point-major
// in LDS at xl, zero-padded to a multiple of 16 rows.
template <typename T, int NT>
__device__ __forceinline__ void srcA_tiles(typename MrT<T>::V4 (&acc)[4], const T* __restrict__ Vb, int32_t k,
                                           int32_t ldv, int32_t q0, const typename MrT<T>::A* xl, int32_t rows,
                                           int lane)
{
    using A = typename MrT<T>::A;
    constexpr uint32_t es = sizeof(T);
    const int li = lane % 16, lk = lane / 16;
    uint32_t ao[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) ao[t] = (uint32_t)(lk * ldv + min(q0 + 16 * t + li, k - 1)) * es;
    const uint32_t sa = (uint32_t)ldv * 4u * es;   // 4 rows of V, in bytes
    int32_t j = 0;
    // software-pipelined: the loads of the next 16 rows are issued before
    // the matrix instructions of the current 16
    auto load = [&](int32_t jj, A (&a)[4][NT], A (&b)[4]) {
        const rsrc_t rv = rsrc(Vb + (int64_t)jj * ldv, 16 * (int64_t)ldv);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            b[u] = xl[(jj + 4 * u + lk) * kR + li];
#pragma unroll
            for (int t = 0; t < NT; ++t) a[u][t] = MrT<T>::load(rv, ao[t], u * sa);
        }
    };
    auto compute = [&](const A (&a)[4][NT], const A (&b)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = MrT<T>::mma(a[u][t], b[u], acc[t]);
    };
    if (j + 16 <= rows) {
        A a0[4][NT], b0[4], a1[4][NT], b1[4];
        load(j, a0, b0);
        for (; j + 32 <= rows; j += 32) {
            load(j + 16, a1, b1);
            compute(a0, b0);
            if (j + 48 <= rows) load(j + 32, a0, b0);
            compute(a1, b1);
        }
        if (j + 16 <= rows) {   // one loaded group left in a0
            compute(a0, b0);
            j += 16;
        }
    }
    if (j < rows) {   // last group: rows past the end re-read row rows - 1, their X rows are zero
        A a[4][NT], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t jl = min(j + 4 * u + lk, rows - 1);
            b[u] = xl[(j + 4 * u + lk) * kR + li];
#pragma unroll
            for (int t = 0; t < NT; ++t) a[u][t] = MrT<T>::get(Vb + jl * ldv + min(q0 + 16 * t + li, k - 1));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = MrT<T>::mma(a[u][t], b[u], acc[t]);
    }
}

// The 4 half values of one aligned 8-byte group, widened to FP32.
template <typename T>
__device__ __forceinline__ f4 quad_f32(uint64_t w)
{
    const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
    if constexpr (std::is_same<T, __half>::value)
        return f4{__half2float(__ushort_as_half((unsigned short)(lo & 0xffffu))),
                  __half2float(__ushort_as_half((unsigned short)(lo >> 16))),
                  __half2float(__ushort_as_half((unsigned short)(hi & 0xffffu))),
                  __half2float(__ushort_as_half((unsigned short)(hi >> 16)))};
    else
        return f4{__uint_as_float(lo << 16), __uint_as_float(lo & 0xffff0000u), __uint_as_float(hi << 16),
                  __uint_as_float(hi & 0xffff0000u)};
}

// acc[t] (columns q0 + 16 t .. + 15 of T_b, t < NT) += V_b(rows, q)^T X(rows)
// on the half V pools, where 4 rows of one column are one aligned 8-byte
// group: V_b(j, q) at Vb[(j / 4) rg + 4 q + j mod 4].  A step takes 16
// rows: lane group lk loads the row group j / 4 + lk of its column, and
// instruction u takes row j + 4 lk + u of it as its k index lk; two steps
// are loaded before their instructions.  Row groups past the item re-read
// its last one (their X rows in LDS are zero); columns past k re-read
// column k - 1 (dropped on output).
template <typename T, int NT>
__device__ __forceinline__ void srcA_tiles_q(f4 (&acc)[4], const T* __restrict__ Vb, int32_t k, int64_t rg,
                                             int32_t q0, const float* xl, int32_t rows, int lane)
{
    const int li = lane % 16, lk = lane / 16;
    const int32_t nq = (rows + 3) >> 2;
    int64_t co[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) co[t] = 4 * (int64_t)min(q0 + 16 * t + li, k - 1);
    for (int32_t j = 0; j < rows; j += 32) {
        uint64_t w[2][NT];
        float b[2][4];
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const int32_t jq = min(((j + 16 * st) >> 2) + lk, nq - 1);
#pragma unroll
            for (int t = 0; t < NT; ++t)
                w[st][t] = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(Vb + jq * rg + co[t]));
#pragma unroll
            for (int u = 0; u < 4; ++u) b[st][u] = xl[(j + 16 * st + 4 * lk + u) * kR + li];
        }
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            f4 a[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) a[t] = quad_f32<T>(w[st][t]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][u], b[st][u], acc[t], 0, 0, 0);
        }
    }
}

// Phase A on the half pools: one workgroup per item of the source-grouped
// schedule (at most kPhaseARows rows of a source box, all its low-rank
// blocks side by side: w columns).  The item's X rows are staged in LDS
// once; the 4 waves take 64-column groups of the wide row in turn, T (w x
// 16) = V(rows, :)^T X(rows, :) on the matrix cores with no per-block
// padding of the columns, and each column of T goes to its block's t
// entry through the source box's column map, or to the item's partial row.
template <typename T>
__global__ void __launch_bounds__(256)
k_phaseA_mr_wide(int64_t nitems, const AWDesc* __restrict__ items, const int32_t* __restrict__ map,
                 const T* __restrict__ V, const float* __restrict__ xs, float* __restrict__ tp,
                 float* __restrict__ pp)
{
    __shared__ float xl[kPhaseARows * kR];
    const int64_t it = blockIdx.x;
    if (it >= nitems) return;
    const AWDesc D = items[it];
    const int64_t voff = uni_l(D.voff);
    const int32_t rows = uni_i(D.rows), w = uni_i(D.w), x0 = uni_i(D.x0), mo = uni_i(D.map), part = uni_i(D.part);
    const int32_t rpad = (rows + 31) & ~31;
    const float* src = xs + (int64_t)x0 * kR;
    for (int32_t e = threadIdx.x; e < rpad * kR; e += blockDim.x) xl[e] = e < rows * kR ? src[e] : 0.f;
    __syncthreads();
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int li = lane % 16, lk = lane / 16;
    const T* Vb = V + voff;
    const int64_t rg = 4 * (int64_t)uni_i(D.ws);
    for (int32_t c0 = 64 * wave; c0 < w; c0 += 4 * 64) {
        f4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
        const int32_t nt = min(4, (w - c0 + 15) / 16);
        if (nt == 4) srcA_tiles_q<T, 4>(acc, Vb, w, rg, c0, xl, rows, lane);
        else if (nt == 3) srcA_tiles_q<T, 3>(acc, Vb, w, rg, c0, xl, rows, lane);
        else if (nt == 2) srcA_tiles_q<T, 2>(acc, Vb, w, rg, c0, xl, rows, lane);
        else srcA_tiles_q<T, 1>(acc, Vb, w, rg, c0, xl, rows, lane);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t c = c0 + 16 * t + MrT<T>::row(v, lk);
                if (t < nt && c < w) {
                    float* dst = part >= 0 ? pp + (int64_t)(part + c) * kR : tp + (int64_t)map[mo + c] * kR;
                    dst[li] = acc[t][v];
                }
            }
    }
}

// T of the columns of source boxes whose phase-A rows were split (half
// pools): the sum of the partial rows, per column and right-hand side.  One
// workgroup per chunk (b, e0) of the list: it owns values e0 .. e0 + 63 of
// box b's w x 16 result (one coalesced row of a part per wave load), its
// four waves take every fourth part, and the four wave sums are added in a
// fixed order.
__global__ void __launch_bounds__(256)
k_reduce_mr_wide(int64_t nc, const int2* __restrict__ chunks, const AWRed* __restrict__ R,
                 const int32_t* __restrict__ map, const float* __restrict__ pp, float* __restrict__ tp)
{
    __shared__ float part[4][kWave];
    if ((int64_t)blockIdx.x >= nc) return;
    const int2 C = chunks[blockIdx.x];
    const AWRed D = R[__builtin_amdgcn_readfirstlane(C.x)];
    const int32_t E = D.w * kR;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t e = __builtin_amdgcn_readfirstlane(C.y) + lane;
    const int64_t stride = (int64_t)D.w * kR;
    const float* base = pp + (int64_t)D.pbeg * kR + min(e, E - 1);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int32_t p = wave;
    for (; p + 12 < D.nparts; p += 16) {
        s0 += base[(int64_t)p * stride];
        s1 += base[(int64_t)(p + 4) * stride];
        s2 += base[(int64_t)(p + 8) * stride];
        s3 += base[(int64_t)(p + 12) * stride];
    }
    for (; p < D.nparts; p += 4) s0 += base[(int64_t)p * stride];
    part[wave][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (wave == 0 && e < E)
        tp[(int64_t)map[D.map + e / kR] * kR + e % kR] =
            (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// Phase A grouped by source box: one workgroup per item stages the item's
// rows of X in LDS once; its four waves take the blocks sharing that source
// in turn, T (k x 16, row-major) = V(rows, :)^T X(rows, :), up to 4 M tiles
// of 16 columns q per pass (on the half pools the block's U scale is
// applied in phase B, with the U values).
// Dynamic LDS: 16 values per row, rows rounded up to 16 (FP64) or 32
// (half pools).
template <typename T>
__device__ __forceinline__ void
phaseA_item(const MRItem& it, const MRBlk* __restrict__ blks, const T* __restrict__ V,
            const typename MrT<T>::A* __restrict__ xs, typename MrT<T>::A* __restrict__ tpool,
            typename MrT<T>::A* __restrict__ ppool, typename MrT<T>::A* xl, const float* __restrict__ scale)
{
    using A = typename MrT<T>::A;
    using V4 = typename MrT<T>::V4;
    const int32_t rows = it.j1 - it.j0, rpad = (rows + 15) & ~15;
    const A* src = xs + (int64_t)(it.col0 + it.j0) * kR;
    for (int e = threadIdx.x; e < rpad * kR; e += blockDim.x) xl[e] = e < rows * kR ? src[e] : (A)0;
    __syncthreads();
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int li = lane % 16, lk = lane / 16;
    for (int32_t b = it.b0 + wave; b < it.b1; b += 4) {
        const MRBlk B = blks[b];
        const int64_t voff = uni_l(B.voff);
        const int32_t k = uni_i(B.k), out = uni_i(B.out);
        A* Tt = out >= 0 ? tpool + (int64_t)out * kR : ppool + ((int64_t)(-out - 1) + (int64_t)it.p * k) * kR;
        for (int32_t q0 = 0; q0 < k; q0 += 64) {
            V4 acc[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = V4{0, 0, 0, 0};
            const int32_t nt = min(4, (k - q0 + 15) / 16);
            const T* Vb = V + voff + (int64_t)it.j0 * k;   // row-major, k values per row
            if (nt == 4) srcA_tiles<T, 4>(acc, Vb, k, k, q0, xl, rows, lane);
            else if (nt == 3) srcA_tiles<T, 3>(acc, Vb, k, k, q0, xl, rows, lane);
            else if (nt == 2) srcA_tiles<T, 2>(acc, Vb, k, k, q0, xl, rows, lane);
            else srcA_tiles<T, 1>(acc, Vb, k, k, q0, xl, rows, lane);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int32_t q = q0 + 16 * t + MrT<T>::row(v, lk);
                    if (t < nt && q < k) Tt[(int64_t)q * kR + li] = acc[t][v];
                }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_phaseA_mr(const MRInst* __restrict__ insts, const int2* __restrict__ work, int32_t nwork)
{
    using A = typename MrT<T>::A;
    extern __shared__ double xl_raw[];
    if ((int32_t)blockIdx.x >= nwork) return;
    const int2 wk = work_at(work, blockIdx.x);
    const MRInst& I = insts[wk.x];
    phaseA_item<T>(gp<const MRItem>(I.items)[wk.y], gp<const MRBlk>(I.blks), gp<const T>(I.V), gp<const A>(I.xs),
                   gp<A>(I.tp), gp<A>(I.pp), (A*)xl_raw, I.scale ? gp<const float>(I.scale) : nullptr);
}

// t = sum of the partial products of one split block.  One workgroup per
// chunk (b, e0) of the instance's list: it owns elements e0 .. e0 + 63 of
// block b's k x 16 result, its four waves take every fourth part, and the
// four wave sums are added in a fixed order.
template <typename A>
__global__ void __launch_bounds__(256)
k_reduce_mr(const MRInst* __restrict__ insts, const int2* __restrict__ work, int32_t nwork)
{
    __shared__ A part[4][kWave];
    if ((int32_t)blockIdx.x >= nwork) return;
    const int2 wk = work_at(work, blockIdx.x);
    const MRInst& I = insts[wk.x];
    const A* __restrict__ ppool = gp<const A>(I.pp);
    A* __restrict__ tpool = gp<A>(I.tp);
    const int2 C = gp<const int2>(I.rchunks)[wk.y];
    const RDesc D = gp<const RDesc>(I.ritems)[__builtin_amdgcn_readfirstlane(C.x)];
    const int32_t E = D.k * kR;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t e = __builtin_amdgcn_readfirstlane(C.y) + lane;
    const int64_t stride = (int64_t)D.k * kR;
    const A* base = ppool + (int64_t)D.pbeg * kR + min(e, E - 1);
    A sv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int32_t p = wave;
    for (; p + 28 < D.nparts; p += 32) {
#pragma unroll
        for (int u = 0; u < 8; ++u) sv[u] += base[(int64_t)(p + 4 * u) * stride];
    }
    for (; p < D.nparts; p += 4) sv[0] += base[(int64_t)p * stride];
    part[wave][lane] = ((sv[0] + sv[1]) + (sv[2] + sv[3])) + ((sv[4] + sv[5]) + (sv[6] + sv[7]));
    __syncthreads();
    if (wave == 0 && e < E)
        tpool[(int64_t)D.tout * kR + e] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// acc[t] (rows 16 t .. 16 t + 15 of a tile, t < NT) += A (rows x K) B (K x 16)
// where A(i, c) = Ab[c * lda + i] (stored values) and B(c, r) = bs Bb[c * ldb + r]
// (work values, times the dense block's scale bs on the half pools).
template <typename T, int NT>
__device__ __forceinline__ void mm_tiles(typename MrT<T>::V4 (&acc)[4], const T* __restrict__ Ab, int64_t lda,
                                         int32_t rows, const typename MrT<T>::A* __restrict__ Bb, int64_t ldb, int32_t K,
                                         typename MrT<T>::A bs, int lane)
{
    using A = typename MrT<T>::A;
    constexpr uint32_t ea = sizeof(T), eb = sizeof(A);
    const int li = lane % 16, lk = lane / 16;
    uint32_t ao[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) ao[t] = (uint32_t)(lk * lda + min(16 * t + li, rows - 1)) * ea;
    const uint32_t bo = (uint32_t)(lk * ldb + li) * eb;
    const uint32_t sa = (uint32_t)lda * 4u * ea, sb = (uint32_t)ldb * 4u * eb;   // 4 columns, in bytes
    int32_t c = 0;
    for (; c + 16 <= K; c += 16) {
        const rsrc_t ra = rsrc(Ab + (int64_t)c * lda, 15 * lda + rows);
        const rsrc_t rb = rsrc(Bb + (int64_t)c * ldb, 15 * ldb + kR);
        A a[4][NT], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            b[u] = vload<A>(rb, bo, u * sb) * bs;
#pragma unroll
            for (int t = 0; t < NT; ++t) a[u][t] = MrT<T>::load(ra, ao[t], u * sa);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = MrT<T>::mma(a[u][t], b[u], acc[t]);
    }
    for (; c < K; c += 4) {   // tail: columns past K re-read column K - 1 with B zeroed
        const int32_t cc = c + lk;
        const int64_t cl = min(cc, K - 1);
        A b = Bb[cl * ldb + li] * bs;
        b = cc < K ? b : (A)0;
        A a[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) a[t] = MrT<T>::get(Ab + cl * lda + min(16 * t + li, rows - 1));
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = MrT<T>::mma(a[t], b, acc[t]);
    }
}

template <typename T>
__device__ __forceinline__ void mm_tile(typename MrT<T>::V4 (&acc)[4], const T* __restrict__ Ab, int64_t lda,
                                        int32_t rows, const typename MrT<T>::A* __restrict__ Bb, int64_t ldb, int32_t K,
                                        typename MrT<T>::A bs, int lane)
{
    if (rows > 48) mm_tiles<T, 4>(acc, Ab, lda, rows, Bb, ldb, K, bs, lane);
    else if (rows > 32) mm_tiles<T, 3>(acc, Ab, lda, rows, Bb, ldb, K, bs, lane);
    else if (rows > 16) mm_tiles<T, 2>(acc, Ab, lda, rows, Bb, ldb, K, bs, lane);
    else mm_tiles<T, 1>(acc, Ab, lda, rows, Bb, ldb, K, bs, lane);
}

// acc[t] (rows 16 t .. 16 t + 15 of a slice, t < NT) += the products of
// the slice's rows of the 4-column groups of table entries j0 .. j1 - 1 (a
// phase-B table of the half pools) with their multiplier rows, times the
// entries' scales.  A step takes 4 entries: lane group lk loads its row's
// 4 values of entry jb + lk, and instruction u = 0..3 takes column u of
// that group as its k index lk; two steps are loaded before either is
// used, and the next two steps' entries are fetched meanwhile.  Entries past j1 re-read the last one with their multiplier values
// zeroed, as are columns past an entry's nv; rows past the slice re-read
// its last row.
template <typename T, int NT>
__device__ __forceinline__ void mm_qt_tiles(f4 (&acc)[4], const QEnt* __restrict__ qt, int32_t j0, int32_t j1,
                                            int32_t rc, int32_t rows, const T* __restrict__ Up,
                                            const T* __restrict__ Dp, const float* __restrict__ tp,
                                            const float* __restrict__ xs, int lane)
{
    constexpr int US = 2;
    const int li = lane % 16, lk = lane / 16;
    int64_t ro[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) ro[t] = (int64_t)(rc + min(16 * t + li, rows - 1)) * 4;
    if (j0 >= j1) return;
    QEnt e[US];
#pragma unroll
    for (int st = 0; st < US; ++st) e[st] = qt[min(j0 + 4 * st + lk, j1 - 1)];
    for (int32_t jb = j0; jb < j1; jb += 4 * US) {
        uint64_t w[US][NT];
        float b[US][4];
#pragma unroll
        for (int st = 0; st < US; ++st) {
            const int32_t j = jb + 4 * st + lk;
            const T* qa = (e[st].src >= 0 ? Up : Dp) + ((int64_t)e[st].q << 2);
#pragma unroll
            for (int t = 0; t < NT; ++t) w[st][t] = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(qa + ro[t]));
            const float* tb = e[st].src >= 0 ? tp + (int64_t)e[st].src * kR : xs + (int64_t)(~e[st].src) * kR;
            const int32_t nv = j < j1 ? e[st].nv : 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) b[st][u] = u < nv ? tb[u * kR + li] * e[st].sc : 0.f;
        }
        // the next entries are loaded while this step's values are in flight
#pragma unroll
        for (int st = 0; st < US; ++st) e[st] = qt[min(jb + 4 * (US + st) + lk, j1 - 1)];
#pragma unroll
        for (int st = 0; st < US; ++st) {
            f4 a[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) a[t] = quad_f32<T>(w[st][t]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][u], b[st][u], acc[t], 0, 0, 0);
        }
    }
}

template <typename T>
__device__ __forceinline__ void mm_qt(f4 (&acc)[4], const QEnt* __restrict__ qt, int32_t j0, int32_t j1, int32_t rc,
                                      int32_t rows, const T* __restrict__ Up, const T* __restrict__ Dp,
                                      const float* __restrict__ tp, const float* __restrict__ xs, int lane)
{
    if (rows > 48) mm_qt_tiles<T, 4>(acc, qt, j0, j1, rc, rows, Up, Dp, tp, xs, lane);
    else if (rows > 32) mm_qt_tiles<T, 3>(acc, qt, j0, j1, rc, rows, Up, Dp, tp, xs, lane);
    else if (rows > 16) mm_qt_tiles<T, 2>(acc, qt, j0, j1, rc, rows, Up, Dp, tp, xs, lane);
    else mm_qt_tiles<T, 1>(acc, qt, j0, j1, rc, rows, Up, Dp, tp, xs, lane);
}

// Scale of a dense block of the half pools (index into the scale table).
template <typename T>
__device__ __forceinline__ typename MrT<T>::A dense_scale(const float* __restrict__ scale, int64_t i)
{
    if constexpr (sizeof(T) == 8) return 1.0;
    else return scale[i];
}

// Phase B1 (ancestor levels): one wave per 64-row chunk of a box at level
// kappa - 1; U tiles as in the single-RHS path.  ypart is row-major n x 16.
template <typename T>
__device__ __forceinline__ void
b1_mr(int32_t it, int lane, const int2* __restrict__ items, int tl, const int32_t* const* __restrict__ Lbegin,
      const int32_t* const* __restrict__ Lcount, const int32_t* const* __restrict__ Lparent,
      const int32_t* const* __restrict__ Lil, const BDesc* __restrict__ bil, const T* __restrict__ Up,
      const T* __restrict__ Dp, const typename MrT<T>::A* __restrict__ tpool,
      const typename MrT<T>::A* __restrict__ xs, typename MrT<T>::A* __restrict__ ypart,
      const float* __restrict__ scale)
{
    using A = typename MrT<T>::A;
    using V4 = typename MrT<T>::V4;
    const int2 w = items[it];
    const int32_t P = uni_i(w.x), rc = uni_i(w.y);
    const int32_t p0 = uni_i(gp<const int32_t>((uint64_t)Lbegin[tl])[P]), cnt = uni_i(gp<const int32_t>((uint64_t)Lcount[tl])[P]);
    const int32_t rows = min(kWave, cnt - rc);
    V4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = V4{0, 0, 0, 0};
    int32_t a_box = P;
    for (int l = tl; l >= 1; --l) {
        const int32_t ab = uni_i(gp<const int32_t>((uint64_t)Lbegin[l])[a_box]), ld_m = uni_i(gp<const int32_t>((uint64_t)Lcount[l])[a_box]);
        const int32_t q0 = uni_i(gp<const int32_t>((uint64_t)Lil[l])[a_box]), q1 = uni_i(gp<const int32_t>((uint64_t)Lil[l])[a_box + 1]);
        for (int32_t q = q0; q < q1; ++q) {
            const BDesc d = bil[q];
            const int64_t off = uni_l(d.off);
            const int32_t cols = uni_i(d.cols), tsrc = uni_i(d.tsrc);
            if (cols > 0)
                mm_tile<T>(acc, Up + off + (int64_t)cols * (p0 - ab) + rc, cnt, rows, tpool + (int64_t)tsrc * kR, kR,
                           cols, (A)1, lane);
            else if (cols < 0)
                mm_tile<T>(acc, Dp + off + (p0 - ab) + rc, ld_m, rows, xs + (int64_t)tsrc * kR, kR, -cols,
                           dense_scale<T>(scale, q), lane);
        }
        a_box = uni_i(gp<const int32_t>((uint64_t)Lparent[l])[a_box]);
    }
    const int li = lane % 16, lk = lane / 16;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int32_t i = 16 * t + MrT<T>::row(v, lk);
            if (i < rows) ypart[(int64_t)(p0 + rc + i) * kR + li] = acc[t][v];
        }
}

// Phase B2 (leaf level): one wave per leaf box; near blocks and the leaf's
// own interaction-list blocks, into yt (tree order, point-major).
template <typename T>
__device__ __forceinline__ void
b2_mr(int32_t X, int lane, const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
      const int32_t* __restrict__ il_ptr, const int32_t* __restrict__ near_ptr, const BDesc* __restrict__ bnear,
      const BDesc* __restrict__ bil, const T* __restrict__ Up, const T* __restrict__ Dp,
      const typename MrT<T>::A* __restrict__ tpool, const typename MrT<T>::A* __restrict__ xs,
      typename MrT<T>::A* __restrict__ yt, const float* __restrict__ scale, int32_t n_il)
{
    using A = typename MrT<T>::A;
    using V4 = typename MrT<T>::V4;
    const int32_t r0 = uni_i(begin[X]), cnt = uni_i(count[X]);
    const int32_t n0 = uni_i(near_ptr[X]), n1 = uni_i(near_ptr[X + 1]);
    const int32_t q0 = uni_i(il_ptr[X]), q1 = uni_i(il_ptr[X + 1]);
    const int li = lane % 16, lk = lane / 16;
    for (int32_t rc = 0; rc < cnt; rc += kWave) {
        const int32_t rows = min(kWave, cnt - rc);
        V4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = V4{0, 0, 0, 0};
        for (int32_t q = n0; q < n1; ++q) {
            const BDesc d = bnear[q];
            mm_tile<T>(acc, Dp + uni_l(d.off) + rc, cnt, rows, xs + (int64_t)uni_i(d.tsrc) * kR, kR, -uni_i(d.cols),
                       dense_scale<T>(scale, (int64_t)n_il + q), lane);
        }
        for (int32_t q = q0; q < q1; ++q) {
            const BDesc d = bil[q];
            const int64_t off = uni_l(d.off);
            const int32_t cols = uni_i(d.cols), tsrc = uni_i(d.tsrc);
            if (cols > 0)
                mm_tile<T>(acc, Up + off + rc, cnt, rows, tpool + (int64_t)tsrc * kR, kR, cols, (A)1, lane);
            else if (cols < 0)
                mm_tile<T>(acc, Dp + off + rc, cnt, rows, xs + (int64_t)tsrc * kR, kR, -cols, dense_scale<T>(scale, q),
                           lane);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t i = 16 * t + MrT<T>::row(v, lk);
                if (i < rows) yt[(int64_t)(r0 + rc + i) * kR + li] = acc[t][v];
            }
    }
}

// Phase B on the half pools: rows rc .. rc + rows - 1 of a box whose first
// row is r0 (one level above the leaves: its table-1 entries; a leaf: its
// table-2 entries j0 .. j1 - 1), into out (tree order, point-major).
template <typename T>
__device__ __forceinline__ void mr_half_slice(int lane, int32_t r0, int32_t rc, int32_t rows,
                                              const QEnt* __restrict__ qt, int32_t j0, int32_t j1,
                                              const T* __restrict__ Up, const T* __restrict__ Dp,
                                              const float* __restrict__ tp, const float* __restrict__ xs,
                                              float* __restrict__ out)
{
    f4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    mm_qt<T>(acc, qt, j0, j1, rc, rows, Up, Dp, tp, xs, lane);
    const int li = lane % 16, lk = lane / 16;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int32_t i = 16 * t + MrT<T>::row(v, lk);
            if (i < rows) out[(int64_t)(r0 + rc + i) * kR + li] = acc[t][v];
        }
}

// Workgroups w0 .. w0 + n - 1 -> tiles 0 .. n - 1, each XCD (workgroup ids
// are dealt round-robin over the 8 XCDs) walking one contiguous range.
__device__ __forceinline__ int32_t xcd_sub_mr(int32_t w, int32_t w0, int32_t n)
{
    const int32_t x = w % 8;
    int32_t start = 0;
    for (int xx = 0; xx < x; ++xx) {
        const int32_t f = ((xx - w0) % 8 + 8) % 8;
        start += f < n ? (n - f + 7) / 8 : 0;
    }
    const int32_t f = ((x - w0) % 8 + 8) % 8;
    return start + (w - w0 - f) / 8;
}

// Phase B in one launch: the first nb1 workgroups do 64-row chunks of the
// level-(kappa-1) boxes (ancestor levels, into ypart), the rest do leaf
// boxes (into yleaf); the halves are independent and summed by the scatter.
template <typename T>
__global__ void __launch_bounds__(256)
k_phaseB_mr(const MRInst* __restrict__ insts, int32_t nb1, const int2* __restrict__ work1, int32_t n1,
            const int2* __restrict__ work2, int32_t n2)
{
    using A = typename MrT<T>::A;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t w = blockIdx.x;
    if (w < nb1) {
        const int32_t it = xcd_sub_mr(w, 0, nb1) * 4 + wave;
        if (it >= n1) return;
        const int2 wk = work_at(work1, it);
        const MRInst& I = insts[wk.x];
        const int32_t* const* L = gp<const int32_t* const>(I.lvl);
        if constexpr (sizeof(T) == 2) {
            const int2 wi = gp<const int2>(I.b1items)[wk.y];
            const int32_t P = uni_i(wi.x), rc = uni_i(wi.y), tl = I.kappa - 1;
            const int32_t p0 = uni_i(gp<const int32_t>((uint64_t)L[tl])[P]);
            const int32_t cnt = uni_i(gp<const int32_t>((uint64_t)L[(kMaxLevel + 1) + tl])[P]);
            const int32_t* qp = gp<const int32_t>(I.qp1);
            mr_half_slice<T>(lane, p0, rc, min(kWave, cnt - rc), gp<const QEnt>(I.qt1), uni_i(qp[P]), uni_i(qp[P + 1]),
                             gp<const T>(I.U), gp<const T>(I.D), gp<const A>(I.tp), gp<const A>(I.xs), gp<A>(I.yp));
            return;
        }
        b1_mr<T>(wk.y, lane, gp<const int2>(I.b1items), I.kappa - 1, L, L + (kMaxLevel + 1), L + 2 * (kMaxLevel + 1),
                 L + 3 * (kMaxLevel + 1), gp<const BDesc>(I.bil), gp<const T>(I.U), gp<const T>(I.D),
                 gp<const A>(I.tp), gp<const A>(I.xs), gp<A>(I.yp), I.scale ? gp<const float>(I.scale) : nullptr);
    } else {
        const int32_t it = xcd_sub_mr(w, nb1, (int32_t)gridDim.x - nb1) * 4 + wave;
        if (it >= n2) return;
        const int2 wk = work_at(work2, it);
        const MRInst& I = insts[wk.x];
        const int32_t* const* L = gp<const int32_t* const>(I.lvl);
        const int kp = I.kappa;
        if constexpr (sizeof(T) == 2) {
            const int32_t X = wk.y;
            const int32_t r0 = uni_i(gp<const int32_t>((uint64_t)L[kp])[X]);
            const int32_t cnt = uni_i(gp<const int32_t>((uint64_t)L[(kMaxLevel + 1) + kp])[X]);
            const int32_t* qp = gp<const int32_t>(I.qp2);
            const int32_t j0 = uni_i(qp[X]), j1 = uni_i(qp[X + 1]);
            for (int32_t rc = 0; rc < cnt; rc += kWave)
                mr_half_slice<T>(lane, r0, rc, min(kWave, cnt - rc), gp<const QEnt>(I.qt2), j0, j1, gp<const T>(I.U),
                                 gp<const T>(I.D), gp<const A>(I.tp), gp<const A>(I.xs), gp<A>(I.yl));
            return;
        }
        b2_mr<T>(wk.y, lane, gp<const int32_t>((uint64_t)L[kp]), gp<const int32_t>((uint64_t)L[(kMaxLevel + 1) + kp]),
                 gp<const int32_t>((uint64_t)L[3 * (kMaxLevel + 1) + kp]), gp<const int32_t>(I.near_ptr),
                 gp<const BDesc>(I.bnear), gp<const BDesc>(I.bil), gp<const T>(I.U), gp<const T>(I.D),
                 gp<const A>(I.tp), gp<const A>(I.xs), gp<A>(I.yl), I.scale ? gp<const float>(I.scale) : nullptr,
                 I.n_il);
    }
}

// Source-grouped phase-A schedule for the multi-RHS product: low-rank
// blocks sorted by (level, source box), each source cut into chunks of
// mr_rows rows; blocks whose source spans several chunks get a partial sum
// per chunk and a reduction.  Items are ordered largest work first.
static void build_mr_schedule(Handle& H, hipStream_t s)
{
    const int32_t R = std::max(16, std::min<int32_t>(H.mr_rows, kMrRowsMax)) & ~15;
    std::vector<int64_t> idx;
    for (int64_t b = 0; b < H.n_il; ++b)
        if (H.h_il_kind[b] != kDense && H.h_il_k[b] > 0) idx.push_back(b);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        return H.h_il_level[a] != H.h_il_level[b] ? H.h_il_level[a] < H.h_il_level[b] : H.h_il_src[a] < H.h_il_src[b];
    });
    std::vector<MRBlk> blks;
    std::vector<MRItem> items;
    std::vector<int64_t> work;
    std::vector<RDesc> red;
    int64_t poff = 0;
    for (size_t g0 = 0; g0 < idx.size();) {
        size_t g1 = g0;
        const int32_t lv = H.h_il_level[idx[g0]], src = H.h_il_src[idx[g0]];
        while (g1 < idx.size() && H.h_il_level[idx[g1]] == lv && H.h_il_src[idx[g1]] == src) ++g1;
        const Level& L = H.lev[lv];
        const int32_t n = L.h_count[src], c0 = L.h_begin[src];
        const int32_t parts = (n + R - 1) / R;
        const int32_t b0 = (int32_t)blks.size();
        int64_t ksum = 0;
        for (size_t g = g0; g < g1; ++g) {
            const int64_t b = idx[g];
            const int32_t k = H.h_il_k[b];
            ksum += k;
            if (parts == 1) {
                blks.push_back(MRBlk{H.h_il_voff[b], k, H.h_il_toff[b], (int32_t)b, 0});
            } else {
                blks.push_back(MRBlk{H.h_il_voff[b], k, (int32_t)(-poff - 1), (int32_t)b, 0});
                red.push_back(RDesc{H.h_il_toff[b], k, (int32_t)poff, parts});
                poff += (int64_t)parts * k;
            }
        }
        const int32_t b1 = (int32_t)blks.size();
        for (int32_t p = 0; p < parts; ++p) {
            const int32_t j0 = p * R, j1 = std::min(n, j0 + R);
            items.push_back(MRItem{c0, j0, j1, b0, b1, p});
            work.push_back((int64_t)(j1 - j0) * ksum);
        }
        g0 = g1;
    }
    if (poff > INT32_MAX) fail(H2D_EUNSUPPORTED, "multi-RHS partial pool too large");
    std::vector<int64_t> ord(items.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int64_t)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return work[a] > work[b]; });
    std::vector<MRItem> sorted(items.size());
    H.h_mr_work.resize(items.size());
    for (size_t i = 0; i < ord.size(); ++i) {
        sorted[i] = items[ord[i]];
        H.h_mr_work[i] = work[ord[i]];
    }
    H.mr_items.alloc(std::max<size_t>(sorted.size(), 1));
    H.mr_blks.alloc(std::max<size_t>(blks.size(), 1));
    H.mr_ritems.alloc(std::max<size_t>(red.size(), 1));
    if (!sorted.empty())
        HIPCK(hipMemcpyAsync(H.mr_items.p, sorted.data(), sizeof(MRItem) * sorted.size(), hipMemcpyHostToDevice, s));
    if (!blks.empty())
        HIPCK(hipMemcpyAsync(H.mr_blks.p, blks.data(), sizeof(MRBlk) * blks.size(), hipMemcpyHostToDevice, s));
    if (!red.empty())
        HIPCK(hipMemcpyAsync(H.mr_ritems.p, red.data(), sizeof(RDesc) * red.size(), hipMemcpyHostToDevice, s));
    H.n_mr_items = (int64_t)sorted.size();
    H.n_mr_ritems = (int64_t)red.size();
    // the reductions in chunks of 64 of their k x 16 values (no workgroup
    // launched empty): the first chunk of every reduction, then the second, ...
    std::vector<int2> chunks;
    int32_t nch = 0;
    for (const RDesc& r : red) nch = std::max(nch, (r.k * kR + kWave - 1) / kWave);
    for (int32_t c = 0; c < nch; ++c)
        for (size_t r = 0; r < red.size(); ++r)
            if (c * kWave < red[r].k * kR) chunks.push_back(make_int2((int32_t)r, c * kWave));
    if (chunks.size() > (size_t)INT32_MAX) fail(H2D_EUNSUPPORTED, "multi-RHS reduction list above 2^31 chunks");
    H.mr_rchunks.alloc(std::max<size_t>(chunks.size(), 1));
    if (!chunks.empty())
        HIPCK(hipMemcpyAsync(H.mr_rchunks.p, chunks.data(), sizeof(int2) * chunks.size(), hipMemcpyHostToDevice, s));
    H.n_mr_rchunks = (int64_t)chunks.size();
    H.mr_p_elems = poff;
    HIPCK(hipStreamSynchronize(s));
}

static uint64_t addr(const void* p) { return (uint64_t)(uintptr_t)p; }

MRInst mr_inst_of(const Handle& H)
{
    MRInst I{};
    I.U = addr(H.U64.p); I.V = addr(H.V64.p); I.D = addr(H.D64.p);
    I.xs = addr(H.xs_mr.p); I.tp = addr(H.tp_mr.p); I.pp = addr(H.pp_mr.p);
    I.yp = addr(H.yp_mr.p); I.yl = addr(H.yl_mr.p);
    I.items = addr(H.mr_items.p); I.blks = addr(H.mr_blks.p); I.ritems = addr(H.mr_ritems.p);
    I.rchunks = addr(H.mr_rchunks.p);
    I.b1items = addr(H.b1items.p); I.bil = addr(H.bil.p); I.bnear = addr(H.bnear.p);
    I.near_ptr = addr(H.near_ptr.p); I.iperm = addr(H.iperm.p); I.lvl = addr(H.lvl_ptrs.p);
    I.scale = 0; I.diag = 0;
    I.n = (int32_t)H.n; I.kappa = H.kappa; I.has_b1 = H.n_b1 ? 1 : 0; I.n_il = (int32_t)H.n_il;
    return I;
}

void ensure_mr(Handle& H, hipStream_t s)
{
    const int32_t n = (int32_t)H.n;
    // per-group operand extents (16 columns of a box) must stay below 4 GiB
    if (H.n > (1 << 24)) fail(H2D_EUNSUPPORTED, "multi-RHS products support at most 2^24 points");
    if (H.mr_cap != 0) return;
    build_mr_schedule(H, s);
    H.xs_mr.alloc((size_t)n * kR);
    H.tp_mr.alloc(std::max<int64_t>(H.t_elems, 1) * kR);
    H.pp_mr.alloc(std::max<int64_t>(H.mr_p_elems, 1) * kR);
    H.yp_mr.alloc((size_t)n * kR);
    H.yl_mr.alloc((size_t)n * kR);
    H.iperm.alloc(std::max(n, 1));
    k_iperm<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(H.perm.p, n, H.iperm.p);
    HIPCK(hipGetLastError());
    std::vector<const int32_t*> ptrs(4 * (kMaxLevel + 1), nullptr);
    for (int l = 0; l <= H.kappa; ++l) {
        ptrs[l] = H.lev[l].begin.p;
        ptrs[kMaxLevel + 1 + l] = H.lev[l].count.p;
        ptrs[2 * (kMaxLevel + 1) + l] = H.lev[l].parent.p;
        ptrs[3 * (kMaxLevel + 1) + l] = H.lev[l].il_ptr.p;
    }
    H.lvl_ptrs.alloc(ptrs.size());
    HIPCK(hipMemcpyAsync(H.lvl_ptrs.p, ptrs.data(), sizeof(void*) * ptrs.size(), hipMemcpyHostToDevice, s));
    const MRInst I = mr_inst_of(H);
    H.mr_inst.alloc(1);
    HIPCK(hipMemcpyAsync(H.mr_inst.p, &I, sizeof(MRInst), hipMemcpyHostToDevice, s));
    HIPCK(hipStreamSynchronize(s));
    H.mr_cap = kR;
    H.mr16_cap = 0;   // the half-pool entries follow the schedule
}

// The half-pool entries (FP16, then BF16) of the multi-RHS product: the
// FP64 schedule with the padded half V offsets, FP32 work vectors.
static void ensure_mr16(Handle& H, hipStream_t s)
{
    ensure_mr(H, s);
    if (H.mr16_cap) return;
    const int32_t n = (int32_t)H.n;
    H.xs_mr32.alloc((size_t)n * kR);
    H.tp_mr32.alloc(std::max<int64_t>(H.t_elems, 1) * kR);
    H.pp_mr32.alloc(std::max<int64_t>(H.p16_elems, 1) * kR);
    H.yp_mr32.alloc((size_t)n * kR);
    H.yl_mr32.alloc((size_t)n * kR);
    MRInst I[2];
    for (int h = 0; h < 2; ++h) {
        I[h] = mr_inst_of(H);
        I[h].U = addr(h ? (const void*)H.Ub16.p : (const void*)H.U16.p);
        I[h].V = addr(h ? (const void*)H.Vb16.p : (const void*)H.V16.p);
        I[h].D = addr(h ? (const void*)H.Db16.p : (const void*)H.D16.p);
        I[h].xs = addr(H.xs_mr32.p); I[h].tp = addr(H.tp_mr32.p); I[h].pp = addr(H.pp_mr32.p);
        I[h].yp = addr(H.yp_mr32.p); I[h].yl = addr(H.yl_mr32.p);
        I[h].qp1 = addr(H.qp1.p); I[h].qt1 = addr(H.qt1.p);
        I[h].qp2 = addr(H.qp2.p); I[h].qt2 = addr(H.qt2.p);
        I[h].scale = addr(H.scale16.p);
        I[h].diag = addr(H.diag32.p);
    }
    H.mr_inst16.alloc(2);
    HIPCK(hipMemcpyAsync(H.mr_inst16.p, I, sizeof(I), hipMemcpyHostToDevice, s));
    HIPCK(hipStreamSynchronize(s));
    H.mr16_cap = 1;
}

static int32_t mr_rows_of(const Handle& H) { return std::max(16, std::min<int32_t>(H.mr_rows, kMrRowsMax)) & ~15; }

template <typename T>
static void run_mr(Handle& H, const MRInst* I, const double* x, double* y, int nrhs, int64_t ld, hipStream_t s)
{
    using A = typename MrT<T>::A;
    const int32_t n = (int32_t)H.n;
    const int32_t nleaf = (int32_t)H.lev[H.kappa].nbox;
    const int32_t R = mr_rows_of(H);
    const int32_t pblocks = (n + kWave - 1) / kWave;
    const MRIo io{addr(x), addr(y), ld};
    for (int r0 = 0; r0 < nrhs; r0 += kR) {
        const int32_t nr = std::min(kR, nrhs - r0);
        k_gather_mr<A><<<(unsigned)pblocks, 256, 0, s>>>(I, nullptr, pblocks, io, nullptr, r0, nr);
        if constexpr (sizeof(T) == 2) {
            // the half V pools: the source-grouped items of the single-RHS form
            const T* V = (const T*)(std::is_same<T, __half>::value ? (const void*)H.V16.p : (const void*)H.Vb16.p);
            if (H.n_aw_items)
                k_phaseA_mr_wide<T><<<(unsigned)H.n_aw_items, 256, 0, s>>>(H.n_aw_items, H.aw_items.p, H.aw_map.p, V,
                                                                            H.xs_mr32.p, H.tp_mr32.p, H.pp_mr32.p);
            if (H.n_aw_red)
                k_reduce_mr_wide<<<(unsigned)H.n_aw_rchunks, 256, 0, s>>>(H.n_aw_rchunks, H.aw_rchunks.p, H.aw_red.p,
                                                                          H.aw_map.p, H.pp_mr32.p,
                                                                      H.tp_mr32.p);
        } else {
            if (H.n_mr_items)
                k_phaseA_mr<T><<<(unsigned)H.n_mr_items, 256, (size_t)R * kR * sizeof(A), s>>>(I, nullptr,
                                                                                             (int32_t)H.n_mr_items);
            if (H.n_mr_rchunks)
                k_reduce_mr<A><<<(unsigned)H.n_mr_rchunks, 256, 0, s>>>(I, nullptr, (int32_t)H.n_mr_rchunks);
        }
        const int32_t nb1 = (int32_t)((H.n_b1 + 3) / 4), nb2 = (nleaf + 3) / 4;
        k_phaseB_mr<T><<<(unsigned)(nb1 + nb2), 256, 0, s>>>(I, nb1, nullptr, (int32_t)H.n_b1, nullptr, nleaf);
        k_scatter_mr<A><<<(unsigned)pblocks, 256, 0, s>>>(I, nullptr, pblocks, io, nullptr, r0, nr);
        HIPCK(hipGetLastError());
    }
}

void launch_matvec_mr(Handle& H, const double* x, double* y, int nrhs, int64_t ld, int prec, hipStream_t s)
{
    if (prec == H2D_P_FP64) {
        ensure_mr(H, s);
        run_mr<double>(H, H.mr_inst.p, x, y, nrhs, ld, s);
    } else {
        ensure_mr16(H, s);
        if (prec == H2D_P_FP16) run_mr<__half>(H, H.mr_inst16.p, x, y, nrhs, ld, s);
        else run_mr<__hip_bfloat16>(H, H.mr_inst16.p + 1, x, y, nrhs, ld, s);
    }
}

template <typename T>
static void upload(DBuf<T>& d, const std::vector<T>& h, hipStream_t s)
{
    d.alloc(std::max<size_t>(h.size(), 1));
    if (!h.empty()) HIPCK(hipMemcpyAsync(d.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s));
}

void mr_plan(MRBatchPlan& P, Handle* const* hs, const MRIo* io, int count, hipStream_t s)
{
    constexpr int kXcd = 8;
    std::vector<MRInst> insts(count);
    std::vector<MRIo> ios(io, io + count);
    std::vector<int2> wg, wr;
    std::vector<std::pair<int64_t, int2>> wa;
    std::vector<int32_t> rows(count);
    for (int i = 0; i < count; ++i) {
        Handle& H = *hs[i];
        ensure_mr(H, s);
        insts[i] = mr_inst_of(H);
        rows[i] = mr_rows_of(H);
        const int32_t n = (int32_t)H.n;
        for (int32_t b = 0; b < (n + kWave - 1) / kWave; ++b) wg.push_back(make_int2(i, b));
        for (int32_t a = 0; a < (int32_t)H.n_mr_items; ++a) wa.push_back({H.h_mr_work[a], make_int2(i, a)});
        for (int32_t r = 0; r < (int32_t)H.n_mr_rchunks; ++r) wr.push_back(make_int2(i, r));
    }
    // phase B: the XCD-aware mapping gives each XCD one eighth of the list;
    // deal every instance's items over the eighths (contiguous inside each)
    // so that each XCD gets a share of every instance
    auto dealt = [&](auto count_of) {
        std::vector<int2> w;
        for (int x = 0; x < kXcd; ++x)
            for (int i = 0; i < count; ++i) {
                const int32_t m = count_of(*hs[i]);
                for (int32_t q = (int32_t)((int64_t)m * x / kXcd); q < (int32_t)((int64_t)m * (x + 1) / kXcd); ++q)
                    w.push_back(make_int2(i, q));
            }
        return w;
    };
    const std::vector<int2> wb1 = dealt([](const Handle& H) { return (int32_t)H.n_b1; });
    const std::vector<int2> wb2 = dealt([](const Handle& H) { return (int32_t)H.lev[H.kappa].nbox; });
    // phase A: one launch per source-chunk size (its LDS need), items of all
    // instances largest work first inside each (a static LPT schedule)
    std::stable_sort(wa.begin(), wa.end(), [&](const auto& a, const auto& b) {
        const int32_t ra = rows[a.second.x], rb = rows[b.second.x];
        return ra != rb ? ra > rb : a.first > b.first;
    });
    std::vector<int2> wav(wa.size());
    P.a_rows.clear(); P.a_beg.clear(); P.a_cnt.clear();
    for (size_t q = 0; q < wa.size(); ++q) {
        wav[q] = wa[q].second;
        const int32_t r = rows[wa[q].second.x];
        if (P.a_rows.empty() || P.a_rows.back() != r) {
            P.a_rows.push_back(r);
            P.a_beg.push_back((int32_t)q);
            P.a_cnt.push_back(0);
        }
        ++P.a_cnt.back();
    }
    upload(P.insts, insts, s);
    upload(P.io, ios, s);
    upload(P.wg, wg, s);
    upload(P.wa, wav, s);
    upload(P.wr, wr, s);
    upload(P.wb1, wb1, s);
    upload(P.wb2, wb2, s);
    P.ng = (int32_t)wg.size(); P.nr = (int32_t)wr.size();
    P.nb1 = (int32_t)wb1.size(); P.nb2 = (int32_t)wb2.size();
    HIPCK(hipStreamSynchronize(s));
}

void mr_plan_launch(const MRBatchPlan& P, int32_t r0, int32_t nr, hipStream_t s)
{
    const MRIo none{0, 0, 0};
    k_gather_mr<double><<<(unsigned)P.ng, 256, 0, s>>>(P.insts.p, P.wg.p, P.ng, none, P.io.p, r0, nr);
    for (size_t g = 0; g < P.a_rows.size(); ++g)
        k_phaseA_mr<double><<<(unsigned)P.a_cnt[g], 256, (size_t)P.a_rows[g] * kR * sizeof(double), s>>>(
            P.insts.p, P.wa.p + P.a_beg[g], P.a_cnt[g]);
    if (P.nr) k_reduce_mr<double><<<(unsigned)P.nr, 256, 0, s>>>(P.insts.p, P.wr.p, P.nr);
    const int32_t g1 = (P.nb1 + 3) / 4, g2 = (P.nb2 + 3) / 4;
    k_phaseB_mr<double><<<(unsigned)(g1 + g2), 256, 0, s>>>(P.insts.p, g1, P.wb1.p, P.nb1, P.wb2.p, P.nb2);
    k_scatter_mr<double><<<(unsigned)P.ng, 256, 0, s>>>(P.insts.p, P.wg.p, P.ng, none, P.io.p, r0, nr);
    HIPCK(hipGetLastError());
}

}  // namespace h2d
