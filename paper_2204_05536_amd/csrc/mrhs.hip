// Multi-RHS form of Algorithm 2 on FP64 matrix cores: Y = A_hat X for
// blocks of 16 right-hand sides.  With 16 columns the products become real
// contractions, T_b = V_b^T X(Y_b) (k x 16) and Y(X) += U_b T_b, computed
// with v_mfma_f64_16x16x4f64.  Schedule, storage and the tree are those of
// the single-RHS path (matvec.hip); only the inner products differ.
//
// MFMA operand layout (16 x 16 output, K = 4 per instruction), lane l:
//   A (16 x 4):  A[l % 16][l / 16]
//   B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): register v holds D[4 v + l / 16][l % 16]
// Right-hand sides are kept point-major inside the kernels (16 consecutive
// values per point), so a B fragment is 64 consecutive doubles.
#include "h2d_impl.h"

#include <algorithm>

namespace h2d {

constexpr int kR = 16;
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int32_t uni_i(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni_l(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int32_t xcd_tile_mr()
{
    const int32_t W = gridDim.x, w = blockIdx.x, xcd = w % 8, i8 = w / 8;
    const int32_t q8 = W / 8, r8 = W % 8;
    return xcd * q8 + min(xcd, r8) + i8;
}

// xs[i * 16 + r] = x[(r0 + r) * ldx + perm[i]] for r < nr, 0 beyond.
__global__ void k_gather_mr(const double* __restrict__ x, int64_t ldx, int32_t nr, const int32_t* __restrict__ perm,
                            int32_t n, double* __restrict__ xs)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * kR) return;
    const int32_t i = (int32_t)(e / kR), r = (int32_t)(e % kR);
    xs[e] = r < nr ? x[(int64_t)r * ldx + perm[i]] : 0.0;
}

// Phase A: one wave per work item (rows j0..j1 of one block's V).
// T(k x 16, row-major) = V(rows, :)^T X(rows, :), M tiles of 16 columns q.
__global__ void __launch_bounds__(256)
k_phaseA_mr(int64_t nitems, const ADesc* __restrict__ items, const double* __restrict__ V,
            const double* __restrict__ xs, double* __restrict__ tpool, double* __restrict__ ppool)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t it = (int64_t)blockIdx.x * 4 + wave;
    if (it >= nitems) return;
    const ADesc D = items[it];
    const int64_t voff = uni_l(D.voff);
    const int32_t j0 = uni_i(D.j0), j1 = uni_i(D.j1), col0 = uni_i(D.col0), k = uni_i(D.k), out = uni_i(D.out);
    double* T = out >= 0 ? tpool + (int64_t)out * kR : ppool + (int64_t)(-out - 1) * kR;
    const int li = lane % 16, lk = lane / 16;
    for (int32_t q0 = 0; q0 < k; q0 += 64) {   // up to 4 M tiles at a time
        d4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = d4{0, 0, 0, 0};
        for (int32_t j = j0; j < j1; j += 4) {
            const int32_t jj = j + lk;
            const bool rowok = jj < j1;
            const double b = rowok ? xs[(int64_t)(col0 + jj) * kR + li] : 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int32_t q = q0 + 16 * t + li;
                if (q0 + 16 * t < k) {
                    const double a = (rowok && q < k) ? V[voff + (int64_t)jj * k + q] : 0.0;
                    acc[t] = mfma(a, b, acc[t]);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t q = q0 + 16 * t + 4 * v + lk;
                if (q < k) T[(int64_t)q * kR + li] = acc[t][v];
            }
    }
}

__global__ void k_reduce_mr(int64_t nr, const RDesc* __restrict__ R, const double* __restrict__ ppool,
                            double* __restrict__ tpool)
{
    const RDesc D = R[blockIdx.x];
    for (int e = threadIdx.x; e < D.k * kR; e += blockDim.x) {
        double s = 0.0;
        for (int p = 0; p < D.nparts; ++p) s += ppool[((int64_t)D.pbeg + (int64_t)p * D.k) * kR + e];
        tpool[(int64_t)D.tout * kR + e] = s;
    }
}

// Y (rows r0 .. r0 + rows - 1 of a tile, up to 64) += A (rows x K) B (K x 16)
// where A(i, c) = Ab[c * lda + i] and B(c, r) = Bb[c * ldb + r].
__device__ __forceinline__ void mm_tile(d4 (&acc)[4], const double* __restrict__ Ab, int64_t lda, int32_t rows,
                                        const double* __restrict__ Bb, int64_t ldb, int32_t K, int lane)
{
    const int li = lane % 16, lk = lane / 16;
    for (int32_t c = 0; c < K; c += 4) {
        const int32_t cc = c + lk;
        const bool colok = cc < K;
        const double b = colok ? Bb[(int64_t)cc * ldb + li] : 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (16 * t < rows) {
                const int32_t i = 16 * t + li;
                const double a = (colok && i < rows) ? Ab[(int64_t)cc * lda + i] : 0.0;
                acc[t] = mfma(a, b, acc[t]);
            }
        }
    }
}

// Phase B1 (ancestor levels): one wave per 64-row chunk of a box at level
// kappa - 1; U tiles as in the single-RHS path.  ypart is row-major n x 16.
__global__ void __launch_bounds__(256)
k_phaseB1_mr(int32_t nitems, const int2* __restrict__ items, int tl, const int32_t* const* __restrict__ Lbegin,
             const int32_t* const* __restrict__ Lcount, const int32_t* const* __restrict__ Lparent,
             const int32_t* const* __restrict__ Lil, const BDesc* __restrict__ bil, const double* __restrict__ Up,
             const double* __restrict__ Dp, const double* __restrict__ tpool, const double* __restrict__ xs,
             double* __restrict__ ypart)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t it = xcd_tile_mr() * 4 + wave;
    if (it >= nitems) return;
    const int2 w = items[it];
    const int32_t P = uni_i(w.x), rc = uni_i(w.y);
    const int32_t p0 = uni_i(Lbegin[tl][P]), cnt = uni_i(Lcount[tl][P]);
    const int32_t rows = min(kWave, cnt - rc);
    d4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = d4{0, 0, 0, 0};
    int32_t a_box = P;
    for (int l = tl; l >= 1; --l) {
        const int32_t ab = uni_i(Lbegin[l][a_box]), ld_m = uni_i(Lcount[l][a_box]);
        const int32_t q0 = uni_i(Lil[l][a_box]), q1 = uni_i(Lil[l][a_box + 1]);
        for (int32_t q = q0; q < q1; ++q) {
            const BDesc d = bil[q];
            const int64_t off = uni_l(d.off);
            const int32_t cols = uni_i(d.cols), tsrc = uni_i(d.tsrc);
            if (cols > 0)
                mm_tile(acc, Up + off + (int64_t)cols * (p0 - ab) + rc, cnt, rows, tpool + (int64_t)tsrc * kR, kR, cols,
                        lane);
            else if (cols < 0)
                mm_tile(acc, Dp + off + (p0 - ab) + rc, ld_m, rows, xs + (int64_t)tsrc * kR, kR, -cols, lane);
        }
        a_box = uni_i(Lparent[l][a_box]);
    }
    const int li = lane % 16, lk = lane / 16;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int32_t i = 16 * t + 4 * v + lk;
            if (i < rows) ypart[(int64_t)(p0 + rc + i) * kR + li] = acc[t][v];
        }
}

// Phase B2 (leaf level): one wave per leaf box; near blocks, the leaf's
// own interaction-list blocks, plus the ancestor sums; y column-major
// (ldy) in caller order, columns r < nr.
__global__ void __launch_bounds__(256)
k_phaseB2_mr(int32_t nleaf, int kappa, const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
             const int32_t* __restrict__ il_ptr, const int32_t* __restrict__ near_ptr, const BDesc* __restrict__ bnear,
             const BDesc* __restrict__ bil, const double* __restrict__ Up, const double* __restrict__ Dp,
             const double* __restrict__ tpool, const double* __restrict__ xs, const double* __restrict__ ypart,
             const int32_t* __restrict__ perm, double* __restrict__ y, int64_t ldy, int32_t nr)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t X = xcd_tile_mr() * 4 + wave;
    if (X >= nleaf) return;
    const int32_t r0 = uni_i(begin[X]), cnt = uni_i(count[X]);
    const int32_t n0 = uni_i(near_ptr[X]), n1 = uni_i(near_ptr[X + 1]);
    const int32_t q0 = uni_i(il_ptr[X]), q1 = uni_i(il_ptr[X + 1]);
    const int li = lane % 16, lk = lane / 16;
    for (int32_t rc = 0; rc < cnt; rc += kWave) {
        const int32_t rows = min(kWave, cnt - rc);
        d4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = d4{0, 0, 0, 0};
        for (int32_t q = n0; q < n1; ++q) {
            const BDesc d = bnear[q];
            mm_tile(acc, Dp + uni_l(d.off) + rc, cnt, rows, xs + (int64_t)uni_i(d.tsrc) * kR, kR, -uni_i(d.cols), lane);
        }
        for (int32_t q = q0; q < q1; ++q) {
            const BDesc d = bil[q];
            const int64_t off = uni_l(d.off);
            const int32_t cols = uni_i(d.cols), tsrc = uni_i(d.tsrc);
            if (cols > 0) mm_tile(acc, Up + off + rc, cnt, rows, tpool + (int64_t)tsrc * kR, kR, cols, lane);
            else if (cols < 0) mm_tile(acc, Dp + off + rc, cnt, rows, xs + (int64_t)tsrc * kR, kR, -cols, lane);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t i = 16 * t + 4 * v + lk;
                if (i < rows && li < nr) {
                    const int32_t g = r0 + rc + i;
                    double s = acc[t][v];
                    if (ypart) s += ypart[(int64_t)g * kR + li];
                    y[(int64_t)li * ldy + perm[g]] = s;
                }
            }
    }
}

void launch_matvec_mr(Handle& H, const double* x, double* y, int nrhs, int64_t ld, hipStream_t s)
{
    const int32_t n = (int32_t)H.n;
    if (H.mr_cap == 0) {
        H.xs_mr.alloc((size_t)n * kR);
        H.tp_mr.alloc(std::max<int64_t>(H.t_elems, 1) * kR);
        H.pp_mr.alloc(std::max<int64_t>(H.p_elems, 1) * kR);
        H.yp_mr.alloc((size_t)n * kR);
        std::vector<const int32_t*> ptrs(4 * (kMaxLevel + 1), nullptr);
        for (int l = 0; l <= H.kappa; ++l) {
            ptrs[l] = H.lev[l].begin.p;
            ptrs[kMaxLevel + 1 + l] = H.lev[l].count.p;
            ptrs[2 * (kMaxLevel + 1) + l] = H.lev[l].parent.p;
            ptrs[3 * (kMaxLevel + 1) + l] = H.lev[l].il_ptr.p;
        }
        H.lvl_ptrs.alloc(ptrs.size());
        HIPCK(hipMemcpyAsync(H.lvl_ptrs.p, ptrs.data(), sizeof(void*) * ptrs.size(), hipMemcpyHostToDevice, s));
        H.mr_cap = kR;
    }
    const int32_t* const* Lb = H.lvl_ptrs.p;
    const int32_t* const* Lc = H.lvl_ptrs.p + (kMaxLevel + 1);
    const int32_t* const* Lp = H.lvl_ptrs.p + 2 * (kMaxLevel + 1);
    const int32_t* const* Li = H.lvl_ptrs.p + 3 * (kMaxLevel + 1);
    const int32_t nleaf = (int32_t)H.lev[H.kappa].nbox;
    for (int r0 = 0; r0 < nrhs; r0 += kR) {
        const int32_t nr = std::min(kR, nrhs - r0);
        k_gather_mr<<<(unsigned)(((int64_t)n * kR + 255) / 256), 256, 0, s>>>(x + (int64_t)r0 * ld, ld, nr, H.perm.p, n,
                                                                           H.xs_mr.p);
        if (H.n_aitems)
            k_phaseA_mr<<<(unsigned)((H.n_aitems + 3) / 4), 256, 0, s>>>(H.n_aitems, H.aitems.p, H.V64.p, H.xs_mr.p,
                                                                       H.tp_mr.p, H.pp_mr.p);
        if (H.n_ritems) k_reduce_mr<<<(unsigned)H.n_ritems, 256, 0, s>>>(H.n_ritems, H.ritems.p, H.pp_mr.p, H.tp_mr.p);
        if (H.n_b1)
            k_phaseB1_mr<<<(unsigned)((H.n_b1 + 3) / 4), 256, 0, s>>>((int32_t)H.n_b1, H.b1items.p, H.kappa - 1, Lb, Lc,
                                                                     Lp, Li, H.bil.p, H.U64.p, H.D64.p, H.tp_mr.p,
                                                                     H.xs_mr.p, H.yp_mr.p);
        k_phaseB2_mr<<<(unsigned)((nleaf + 3) / 4), 256, 0, s>>>(
            nleaf, H.kappa, H.lev[H.kappa].begin.p, H.lev[H.kappa].count.p, H.lev[H.kappa].il_ptr.p, H.near_ptr.p,
            H.bnear.p, H.bil.p, H.U64.p, H.D64.p, H.tp_mr.p, H.xs_mr.p, H.n_b1 ? H.yp_mr.p : nullptr, H.perm.p,
            y + (int64_t)r0 * ld, ld, nr);
        HIPCK(hipGetLastError());
    }
}

}  // namespace h2d
