// Algorithm 2 (MatVec) on gfx950.
//
//   gather:   xs = x(perm)                     tree order
//   phase A:  t_b = V_b^T xs(Y_b)              every low-rank block, all levels
//   reduce:   t_b = sum of partials            blocks whose V was split over waves
//   phase B:  for every row of a leaf box X, the sum over the blocks of the
//             ancestors of X of U_b(rows) t_b (or D_b(rows) xs(Y_b) for dense
//             blocks) -- the "B1" half, per slice of a box one level above
//             the leaves (half pools: per run of sibling boxes at that
//             level) -- and, in the same launch, the sum over X's dense
//             near blocks and X's own blocks -- the "B2" half, per leaf
//             chunk; the two sums go to separate arrays
//   combine:  y = the two sums (+ the FP32 diagonal term of the half
//             pools), written once in caller order.
// No atomics: every output row is owned by one wave in each half, and every
// sum is taken in a fixed order, so two runs give identical bits.
//
// Storage: U column-major m x k (a leaf box's rows are contiguous in every
// column), V row-major n x k (a wave reads whole rows: G = 64 / k rows per
// load instruction), D column-major m x n.
#include "h2d_impl.h"

#include <algorithm>
#include <cstring>
#include <cstdlib>
#include <mutex>
#include <type_traits>

namespace h2d {

struct LevelPtrs {
    const int32_t* begin[kMaxLevel + 1];
    const int32_t* count[kMaxLevel + 1];
    const int32_t* parent[kMaxLevel + 1];
    const int32_t* il_ptr[kMaxLevel + 1];
};

// Phase A streams the V values once per matvec: nontemporal loads keep
// them from evicting x, t and the descriptors from the caches.
__device__ __forceinline__ double ld_nt(const double* p) { return __builtin_nontemporal_load(p); }

// The t and x values of a block are the same for every lane of a phase-B1
// wave (all lanes walk the same columns): read through the constant address
// space they become scalar-cache loads (8 values per instruction), so the
// vector memory pipe carries only the factors.  They are written by earlier
// kernels only.
template <typename A> using ConstAS = const __attribute__((address_space(4))) A;

// Phase B reads the FP64 factors with ordinary loads (measured slightly
// faster there than nontemporal ones).
// acc += sum over c = g, g + G, ... < n of base[c ld] w[c], eight columns
// per lane loaded before any is multiplied: the loads of a chunk are in
// flight together, and a short tail is padded with zero products instead of
// running one load (and one memory latency) at a time.  The products are
// added in increasing c, as the plain loop adds them.
template <typename W>
__device__ __forceinline__ void dot_cols(double& acc, const double* base, int64_t ld, const W* w, int32_t n, int g,
                                         int G)
{
    for (int32_t c0 = 0; c0 < n; c0 += 8 * G) {
        double v[8], t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t c = c0 + u * G + g;
            v[u] = 0.0;
            t[u] = 0.0;
            if (c < n) {
                v[u] = base[(int64_t)c * ld];
                t[u] = (double)w[c];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u] * t[u];
    }
}

// Four consecutive half values at an 8-byte-aligned address: one aligned
// 8-byte load (the padded V pools).
template <typename T> __device__ __forceinline__ float4 ld4v(const T* p)
{
    const uint64_t w = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(p));
    const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
    if constexpr (std::is_same<T, __half>::value)
        return make_float4(__half2float(__ushort_as_half((unsigned short)(lo & 0xffffu))),
                           __half2float(__ushort_as_half((unsigned short)(lo >> 16))),
                           __half2float(__ushort_as_half((unsigned short)(hi & 0xffffu))),
                           __half2float(__ushort_as_half((unsigned short)(hi >> 16))));
    else
        return make_float4(__uint_as_float(lo << 16), __uint_as_float(lo & 0xffff0000u), __uint_as_float(hi << 16),
                           __uint_as_float(hi & 0xffff0000u));
}

template <typename A>
__global__ void k_gather(const double* x, const int32_t* perm, int32_t n, int64_t ldx, int64_t ldxs, int nrhs, A* xs)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t p = perm[i];
    for (int r = 0; r < nrhs; ++r) xs[(int64_t)r * ldxs + i] = (A)x[(int64_t)r * ldx + p];
}

// Wave-uniform values: loaded once per wave, then moved to scalar registers
// so that the loads they address become scalar-cache loads.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ BDesc uni(const BDesc& d) { return BDesc{uni(d.off), uni(d.cols), uni(d.tsrc)}; }

// Multiplier values (t, or x of a source box) of one block staged in a
// wave's LDS slice at a time, where lanes take different columns.
constexpr int kB2Stage = 256;

// Workgroup w -> tile index such that each XCD (workgroups are dealt
// round-robin over the 8 XCDs) walks one contiguous range of tiles, so
// neighbouring tiles, which share cache lines, share an L2.
__device__ __forceinline__ int32_t xcd_tile()
{
    const int32_t W = gridDim.x, w = blockIdx.x, xcd = w % 8, i8 = w / 8;
    const int32_t q8 = W / 8, r8 = W % 8;
    return xcd * q8 + min(xcd, r8) + i8;
}

// Phase A, grouped by source box: one workgroup per item (rows j0 .. j1 -
// 1, at most kPhaseARows, of one source box, and every low-rank block with
// that source).  The item's slice of x is staged in LDS once; the four
// waves take the blocks in turn.  For a block of rank k, lane (g, q) takes
// column q of rows g, g + G, ... (G = 64 / k): each load covers G whole
// rows, G k consecutive values, and the G sums of a column are added in a
// fixed order; ranks above 64 take 64 columns per pass.  Items are ordered
// largest first (a static longest-processing-time schedule).
__global__ void __launch_bounds__(256)
k_phaseA(const MRItem* __restrict__ items, const MRBlk* __restrict__ blks, const double* __restrict__ V,
         const double* __restrict__ xs, double* __restrict__ tpool, double* __restrict__ ppool)
{
    __shared__ double xl[kPhaseARows];
    __shared__ double red[4][kWave];
    const MRItem it = items[blockIdx.x];
    const int32_t rows = it.j1 - it.j0;
    for (int32_t j = threadIdx.x; j < rows; j += blockDim.x) xl[j] = xs[it.col0 + it.j0 + j];
    __syncthreads();
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int32_t bi = it.b0 + wave; bi < it.b1; bi += 4) {
        const MRBlk B = blks[bi];
        const int32_t k = uni(B.k), out = uni(B.out);
        const double* Vb = V + uni(B.voff) + (int64_t)it.j0 * k;
        double* o = out >= 0 ? tpool + out : ppool + (int64_t)(-out - 1) + (int64_t)it.p * k;
        if (k <= kWave) {
            const int G = kWave / k, g = lane / k, q = lane % k;
            double acc = 0.0;
            if (g < G) {
#pragma unroll 8
                for (int32_t j = g; j < rows; j += G) acc += ld_nt(Vb + (int64_t)j * k + q) * xl[j];
            }
            red[wave][lane] = acc;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            if (lane < k) {
                double sum = 0.0;
                for (int gg = 0; gg < G; ++gg) sum += red[wave][gg * k + lane];
                o[lane] = sum;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        } else {
            for (int32_t qc = 0; qc < k; qc += kWave) {
                const int32_t q = qc + lane;
                if (q < k) {
                    double acc = 0.0;
#pragma unroll 8
                    for (int32_t j = 0; j < rows; ++j) acc += ld_nt(Vb + (int64_t)j * k + q) * xl[j];
                    o[q] = acc;
                }
            }
        }
    }
}

// t = sum of a split block's partials.  One workgroup per split block; lane
// = column (a part's k values are contiguous, so each wave load is one
// coalesced row of partials); wave w sums the parts w, w + 4, ... in order
// and the four wave sums are added in wave order.
template <typename A>
__global__ void __launch_bounds__(256)
k_reduce_parts(int64_t nr, const RDesc* __restrict__ R, const A* __restrict__ ppool, A* __restrict__ tpool)
{
    __shared__ A red[4][kWave];
    const int64_t r = blockIdx.x;
    if (r >= nr) return;
    RDesc D = R[r];
    D.tout = uni(D.tout); D.k = uni(D.k); D.pbeg = uni(D.pbeg); D.nparts = uni(D.nparts);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int32_t q0 = 0; q0 < D.k; q0 += kWave) {
        const int32_t q = q0 + lane;
        A s = (A)0;
        if (q < D.k) {
#pragma unroll 8
            for (int32_t p = wave; p < D.nparts; p += 4) s += ppool[D.pbeg + (int64_t)p * D.k + q];
        }
        red[wave][lane] = s;
        __syncthreads();
        if (wave == 0 && q < D.k) tpool[D.tout + q] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        __syncthreads();
    }
}

// Phase A on the half pools, grouped by source box: one wave per item (at
// most kPhaseARows rows of a source box's wide V: the V of every low-rank
// block with that source side by side, w columns, stored in groups of 4
// rows so that 4 rows of one column are one aligned 8-byte group, each
// group of rows ws >= w columns wide).  The
// item's x rows are staged in LDS (zeros past its last row).  A lane owns
// columns and walks the item's row groups: with w <= 64, lane (g, c) takes
// column c of row groups g, g + G, ... (G = 64 / w) and the G sums of a
// column are added in a fixed order; wider items take 64 columns per pass.
// A wave load is 64 consecutive 8-byte groups (512 contiguous bytes) when
// w >= 64.  Each column's sum goes to its t entry through the source box's
// column map, or to the item's partial row.
template <typename T>
__global__ void __launch_bounds__(256)
k_phaseA_wide(int64_t nitems, const AWDesc* __restrict__ items, const int32_t* __restrict__ map,
              const T* __restrict__ V, const float* __restrict__ xs, float* __restrict__ tpool,
              float* __restrict__ ppool)
{
    __shared__ float xw[4][kPhaseARows];
    __shared__ float red[4][kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t it = (int64_t)blockIdx.x * 4 + wave;
    if (it >= nitems) return;
    const AWDesc D = items[it];
    const int64_t voff = uni(D.voff);
    const int32_t rows = uni(D.rows), w = uni(D.w), x0 = uni(D.x0), mo = uni(D.map), part = uni(D.part);
    const int32_t nq = (rows + 3) >> 2;
    float* xl = xw[wave];
    for (int32_t j = lane; j < 4 * nq; j += kWave) xl[j] = j < rows ? xs[x0 + j] : 0.f;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    auto put = [&](int32_t c, float v) {
        if (part >= 0) ppool[part + c] = v;
        else tpool[map[mo + c]] = v;
    };
    const T* Vb = V + voff;
    const int64_t rg = 4 * (int64_t)uni(D.ws);   // elements per row group
    // FP16: four running sums per lane, one per row of a group (four
    // independent chains of the mixed-precision FMA), added at the end;
    // BF16: one running sum (measured faster for each)
    auto quad = [&](float4& a, int32_t jq, int32_t c) {
        const float4 v = ld4v<T>(Vb + jq * rg + 4 * c);
        const float* xq = xl + 4 * jq;
        if constexpr (std::is_same<T, __half>::value) {
            a.x += v.x * xq[0];
            a.y += v.y * xq[1];
            a.z += v.z * xq[2];
            a.w += v.w * xq[3];
        } else {
            a.x += v.x * xq[0] + v.y * xq[1] + v.z * xq[2] + v.w * xq[3];
        }
    };
    if (w <= kWave) {
        const int G = kWave / w, g = lane / w, c = lane % w;
        float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (g < G) {
#pragma unroll 8
            for (int32_t jq = g; jq < nq; jq += G) quad(a4, jq, c);
        }
        const float a = (a4.x + a4.y) + (a4.z + a4.w);
        red[wave][lane] = a;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (lane < w) {
            float sum = 0.f;
            for (int gg = 0; gg < G; ++gg) sum += red[wave][gg * w + lane];
            put(lane, sum);
        }
        return;
    }
    for (int32_t c = lane; c < w; c += kWave) {
        float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 8
        for (int32_t jq = 0; jq < nq; ++jq) quad(a4, jq, c);
        put(c, (a4.x + a4.y) + (a4.z + a4.w));
    }
}

// t of the columns of source boxes whose phase-A rows were split: the sum
// of the partial rows.  Grid (split source boxes, ceil(max w / 64)):
// workgroup (b, g) owns columns 64 g .. 64 g + 63 of box b (one coalesced
// row of a part per wave load), its four waves take every fourth part, and
// the four wave sums are added in a fixed order.
__global__ void __launch_bounds__(256)
k_reduce_wide(int64_t nr, const AWRed* __restrict__ R, const int32_t* __restrict__ map,
              const float* __restrict__ ppool, float* __restrict__ tpool)
{
    __shared__ float part[4][kWave];
    const int64_t r = blockIdx.x;
    if (r >= nr) return;
    const AWRed D = R[r];
    if ((int32_t)blockIdx.y * kWave >= D.w) return;   // whole workgroup
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t q = blockIdx.y * kWave + lane;
    const float* base = ppool + D.pbeg + min(q, D.w - 1);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int32_t p = wave;
    for (; p + 12 < D.nparts; p += 16) {
        s0 += base[(int64_t)p * D.w];
        s1 += base[(int64_t)(p + 4) * D.w];
        s2 += base[(int64_t)(p + 8) * D.w];
        s3 += base[(int64_t)(p + 12) * D.w];
    }
    for (; p < D.nparts; p += 4) s0 += base[(int64_t)p * D.w];
    part[wave][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (wave == 0 && q < D.w) tpool[map[D.map + q]] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// Phase B1: ancestor levels.  One wave per slice of S rows (S = 16, 32 or
// 64) of a box at level kappa - 1; lane (g, r) owns row r of the slice and
// the columns g, g + G, ... (G = 64 / S) of every interaction-list block of
// that box and of each ancestor, so one load covers G columns of S
// consecutive values.  The G column-group sums are added in a fixed order.
// Smaller slices give more, shorter work items (a shorter tail when the
// items do not fill a whole number of rounds of the machine).  S0 = 0 takes
// the slice width Sr at run time: the 16- and 32-row forms use it (one code
// path for every width keeps them at the 64-row form's registers), so the
// last slice of a box, when it holds few rows, runs with more column groups.
template <int S0>
__device__ __forceinline__ void
b1_item(int32_t it, int wave, int lane, double (*red)[kWave], const int2* __restrict__ items, int tl,
        const LevelPtrs& L, const BDesc* __restrict__ bil, const double* __restrict__ Up, const double* __restrict__ Dp,
        const double* __restrict__ tpool, const double* __restrict__ xs, double* __restrict__ ypart, int Sr = 0)
{
    using cA = ConstAS<double>;
    const int2 w = items[it];
    const int32_t P = uni(w.x), rc = uni(w.y);
    const int32_t p0 = uni(L.begin[tl][P]), cnt = uni(L.count[tl][P]);
    const int S = S0 ? S0 : Sr;
    const int32_t rows = min(S, cnt - rc);
    const int G = kWave / S;
    const int g = G == 1 ? 0 : lane / S, r = G == 1 ? lane : lane % S;
    const bool act = r < rows;
    double acc = 0.0;
    int32_t a_box = P;
    for (int l = tl; l >= 1; --l) {
        const int32_t ab = uni(L.begin[l][a_box]), ld_m = uni(L.count[l][a_box]);
        const int64_t off = (int64_t)(p0 - ab + rc + r);
        const int32_t q0 = uni(L.il_ptr[l][a_box]), q1 = uni(L.il_ptr[l][a_box + 1]);
        for (int32_t q = q0; q < q1; ++q) {
            const BDesc d = uni(bil[q]);
            if (d.cols > 0) {
                // U is tiled by level-(kappa - 1) boxes: this box's tile is
                // a contiguous cnt x k column-major matrix
                const double* base = Up + d.off + (int64_t)d.cols * (p0 - ab) + rc + r;
                const cA* tv = (const cA*)(tpool + d.tsrc);
                if (act) dot_cols(acc, base, cnt, tv, d.cols, g, G);
            } else if (d.cols < 0) {
                const double* base = Dp + d.off + off;
                const cA* tv = (const cA*)(xs + d.tsrc);
                double a = 0.0;
                if (act) dot_cols(a, base, ld_m, tv, -d.cols, g, G);
                acc += a;
            }
        }
        a_box = uni(L.parent[l][a_box]);
    }
    if (G == 1) {
        if (act) ypart[p0 + rc + r] = acc;
        return;
    }
    red[wave][lane] = act ? acc : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane < rows) {
        double s = 0.0;
        for (int gg = 0; gg < G; ++gg) s += red[wave][gg * S + lane];
        ypart[p0 + rc + lane] = s;
    }
}

// Phase B2: the leaf level.  One wave per 64-row chunk of a leaf box X
// (leaves above 64 points give several items): its dense near blocks and
// its own interaction-list blocks, into the leaf-level sum.  A chunk has at
// most 64 rows;
// lane (g, r) takes row r and the columns g, g + G, ... (G = 64 / rows), so
// a load covers G consecutive columns of the column-major block.
__device__ __forceinline__ void
b2_item(int32_t X, int32_t rc, int32_t S2, int wave, int lane, double (*red)[kWave], double* tst, int kappa,
        const LevelPtrs& L, const int32_t* __restrict__ near_ptr, const BDesc* __restrict__ bnear,
        const BDesc* __restrict__ bil, const double* __restrict__ Up, const double* __restrict__ Dp,
        const double* __restrict__ tpool, const double* __restrict__ xs, double* __restrict__ yleaf)
{
    const int32_t r0 = uni(L.begin[kappa][X]), cnt = uni(L.count[kappa][X]);
    const int32_t q0 = uni(L.il_ptr[kappa][X]), q1 = uni(L.il_ptr[kappa][X + 1]);
    const int32_t n0 = uni(near_ptr[X]), n1 = uni(near_ptr[X + 1]);
    const int32_t rows = min(S2, cnt - rc);
    const int G = kWave / rows, g = lane / rows, r = lane % rows;
    const bool act = g < G;
    // one block wider than a wave: its multiplier values (t, or x of the
    // source box) are staged in this wave's LDS slice, kB2Stage at a time,
    // with one load per lane, instead of one gather load per lane and column
    // group
    auto sweep = [&](const double* base, const double* tv, int32_t nc) -> double {
        double a = 0.0;
        for (int32_t c0 = 0; c0 < nc; c0 += kB2Stage) {
            const int32_t m = min(kB2Stage, nc - c0);
            for (int32_t j = lane; j < m; j += kWave) tst[j] = tv[c0 + j];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            if (act) dot_cols(a, base + (int64_t)c0 * cnt, cnt, tst, m, g, G);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
        return a;
    };
    // the blocks in order (near blocks, then the interaction list); a block
    // of at most 64 values is staged from a register loaded while the
    // previous block's values were read, so the staging load and the block's
    // own loads share one wait
    const int32_t nn = n1 - n0, nt = nn + (q1 - q0);
    auto desc = [&](int32_t i) -> BDesc {
        if (i >= nt) return BDesc{0, 0, 0};
        return i < nn ? uni(bnear[n0 + i]) : uni(bil[q0 + i - nn]);
    };
    auto mult = [&](const BDesc& d) -> const double* { return (d.cols > 0 ? tpool : xs) + d.tsrc; };
    auto fbase = [&](const BDesc& d) -> const double* { return (d.cols > 0 ? Up : Dp) + d.off + rc + r; };
    auto first = [&](const BDesc& d, int32_t n) -> double { return n <= kWave && lane < n ? mult(d)[lane] : 0.0; };
    double acc = 0.0;
    BDesc d = desc(0);
    int32_t n = d.cols > 0 ? d.cols : -d.cols;
    double v = first(d, n);
    for (int32_t i = 0; i < nt; ++i) {
        const BDesc dn = desc(i + 1);
        const int32_t nx = dn.cols > 0 ? dn.cols : -dn.cols;
        if (n > kWave) {
            acc += sweep(fbase(d), mult(d), n);
            v = first(dn, nx);
        } else if (n > 0) {
            if (lane < n) tst[lane] = v;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            const double vn = first(dn, nx);
            double a = 0.0;
            if (act) dot_cols(a, fbase(d), cnt, tst, n, g, G);
            acc += a;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            v = vn;
        } else {
            v = first(dn, nx);
        }
        d = dn;
        n = nx;
    }
    red[wave][lane] = act ? acc : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane < rows) {
        double s = 0.0;
        for (int gg = 0; gg < G; ++gg) s += red[wave][gg * rows + lane];
        yleaf[r0 + rc + lane] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Workgroups w0 .. w0 + n - 1 of the grid -> tiles 0 .. n - 1 such that
// the workgroups each XCD receives (workgroup ids are dealt round-robin over
// the 8 XCDs) take one contiguous range of tiles.
__device__ __forceinline__ int32_t xcd_sub(int32_t w, int32_t w0, int32_t n)
{
    const int32_t x = w % 8;
    int32_t start = 0;
    for (int xx = 0; xx < x; ++xx) {
        const int32_t f = ((xx - w0) % 8 + 8) % 8;   // first local index dealt to XCD xx
        start += f < n ? (n - f + 7) / 8 : 0;
    }
    const int32_t f = ((x - w0) % 8 + 8) % 8;
    return start + (w - w0 - f) / 8;
}

// Phase B, both halves in one launch: the first nb1 workgroups do phase-B1
// items (ancestor levels, into ypart: slices of a box one level above the
// leaves), the next nb2 do phase-B2 leaf chunks (leaf level and near
// field, into yleaf).  The two halves write different
// arrays and do not depend on each other; the latency-bound leaf work is
// dispatched as the ancestor work drains, filling its tail.
template <int S>
__global__ void __launch_bounds__(256)
k_phaseB(int32_t nb1, int32_t nitems, const int2* __restrict__ items, int kappa, LevelPtrs L,
         const int32_t* __restrict__ near_ptr, const BDesc* __restrict__ bnear, const BDesc* __restrict__ bil,
         const double* __restrict__ Up, const double* __restrict__ Dp, const double* __restrict__ tpool,
         const double* __restrict__ xs, double* __restrict__ ypart, double* __restrict__ yleaf,
         const int2* __restrict__ b2items, int32_t nb2items, int32_t b2_rows)
{
    __shared__ double red[4][kWave];
    __shared__ double tst[4][kB2Stage];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t w = blockIdx.x;
    if (w < nb1) {
        const int32_t it = xcd_sub(w, 0, nb1) * 4 + wave;
        if (it >= nitems) return;
        // 16- and 32-row slices: the width is the slice's rows rounded up to
        // a power of two (at least 8), so a short last slice of a box takes
        // its columns in more lane groups; 64-row slices keep the fixed form
        // (measured: a run-time-width path for their short last slices made
        // the uniform case 9% slower)
        if constexpr (S == 64) {
            b1_item<64>(it, wave, lane, red, items, kappa - 1, L, bil, Up, Dp, tpool, xs, ypart);
        } else {
            const int2 wi = items[it];
            const int32_t rem = uni(L.count[kappa - 1][uni(wi.x)]) - uni(wi.y);
            const int Sr = min(S, rem <= 8 ? 8 : rem <= 16 ? 16 : 32);
            b1_item<0>(it, wave, lane, red, items, kappa - 1, L, bil, Up, Dp, tpool, xs, ypart, Sr);
        }
    } else {
        const int32_t it = xcd_sub(w, nb1, (int32_t)gridDim.x - nb1) * 4 + wave;
        if (it < nb2items) {
            const int2 c = b2items[it];
            b2_item(uni(c.x), uni(c.y), b2_rows, wave, lane, red, tst[wave], kappa, L, near_ptr, bnear, bil, Up, Dp, tpool,
                    xs, yleaf);
        }
    }
}

// The dot product of one row's 4-value group (half, widened to FP32) with
// 4 multiplier values.
template <typename T>
__device__ __forceinline__ float quad_dot4(uint64_t w, float t0, float t1, float t2, float t3)
{
    const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
    float v0, v1, v2, v3;
    if constexpr (std::is_same<T, __half>::value) {
        v0 = __half2float(__ushort_as_half((unsigned short)(lo & 0xffffu)));
        v1 = __half2float(__ushort_as_half((unsigned short)(lo >> 16)));
        v2 = __half2float(__ushort_as_half((unsigned short)(hi & 0xffffu)));
        v3 = __half2float(__ushort_as_half((unsigned short)(hi >> 16)));
    } else {
        v0 = __uint_as_float(lo << 16);
        v1 = __uint_as_float(lo & 0xffff0000u);
        v2 = __uint_as_float(hi << 16);
        v3 = __uint_as_float(hi & 0xffff0000u);
    }
    return v0 * t0 + v1 * t1 + v2 * t2 + v3 * t3;
}

// acc += the sum over table entries j = j0 + g, j0 + g + G, ... < j1 of the
// entry's scale times the dot product of this lane's row of the entry's
// 4-column group (at pool + 4 q + ro) with its multiplier values.  Four
// entries are loaded before any is used, so the groups of several blocks
// are in flight together, and the next four entries are fetched while
// their groups load; slots past j1 re-read entry j1 - 1 and add nothing.  kUni: G = 1, g = 0, every lane takes every entry (the entries
// and multiplier values are then wave-uniform loads).  The multiplier
// values of columns past the group's nv are taken as zero; the work
// vectors carry slack past their ends for these reads.
template <typename T, bool kUni>
__device__ __forceinline__ void qt_sweep(float& acc, const QEnt* __restrict__ qt, int32_t j0, int32_t j1, int g, int G,
                                         int64_t ro, const T* __restrict__ Up, const T* __restrict__ Dp,
                                         const float* __restrict__ tpool, const float* __restrict__ xs)
{
    constexpr int NF = 4;
    if constexpr (kUni) {
        g = 0;
        G = 1;
    }
    if (j0 >= j1) return;
    QEnt e[NF];
#pragma unroll
    for (int u = 0; u < NF; ++u) e[u] = qt[min(j0 + u * G + g, j1 - 1)];
    for (int32_t jb = j0; jb < j1; jb += NF * G) {
        uint64_t w[NF];
        float t[NF][4];
#pragma unroll
        for (int u = 0; u < NF; ++u) {
            const T* pool = e[u].src >= 0 ? Up : Dp;
            w[u] = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(pool + ((int64_t)e[u].q << 2) + ro));
        }
#pragma unroll
        for (int u = 0; u < NF; ++u) {
            const float* tb = e[u].src >= 0 ? tpool + e[u].src : xs + ~e[u].src;
#pragma unroll
            for (int c = 0; c < 4; ++c) t[u][c] = tb[c];
        }
        // the next entries are loaded while this step's groups are in flight
        // (past j1 they re-read entry j1 - 1)
        QEnt en[NF];
#pragma unroll
        for (int u = 0; u < NF; ++u) en[u] = qt[min(jb + (NF + u) * G + g, j1 - 1)];
#pragma unroll
        for (int u = 0; u < NF; ++u) {
            const int32_t nv = e[u].nv;
            const float d = quad_dot4<T>(w[u], t[u][0], nv > 1 ? t[u][1] : 0.f, nv > 2 ? t[u][2] : 0.f,
                                         nv > 3 ? t[u][3] : 0.f);
            // a slot past j1 adds d * 0 (d is computed either way, so the
            // slot's loads are not moved behind a branch)
            acc = fmaf(d, jb + u * G + g < j1 ? e[u].sc : 0.f, acc);
        }
#pragma unroll
        for (int u = 0; u < NF; ++u) e[u] = en[u];
    }
}

// Phase B on the half pools, both halves in one launch.  B1: one wave per
// 64-row slice of a box P one level above the leaves; lane r owns row r and
// walks P's table (the groups of every block of P and its ancestors); a
// slice of at most 32 rows takes the table in lane groups, as below.  B2:
// one wave per chunk of at most S2 rows of a leaf X; lane (g, r) owns row r
// and the table entries g, g + G, ... (G = 64 / rows) of X's table (near
// blocks, then X's own interaction-list blocks); the G sums of a row are
// added in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256)
k_phaseB_half(int32_t nb1, int32_t nitems, const int2* __restrict__ items, int kappa, LevelPtrs L,
              const int32_t* __restrict__ qp1, const QEnt* __restrict__ qt1, const int32_t* __restrict__ qp2,
              const QEnt* __restrict__ qt2, const T* __restrict__ Up, const T* __restrict__ Dp,
              const float* __restrict__ tpool, const float* __restrict__ xs, float* __restrict__ ypart,
              float* __restrict__ yleaf, const int2* __restrict__ b2items, int32_t nb2items, int32_t S2)
{
    __shared__ float red[4][kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t w = blockIdx.x;
    if (w < nb1) {
        const int32_t it = xcd_sub(w, 0, nb1) * 4 + wave;
        if (it >= nitems) return;
        const int2 wi = items[it];
        const int32_t P = uni(wi.x), rc = uni(wi.y);
        const int32_t p0 = uni(L.begin[kappa - 1][P]), cnt = uni(L.count[kappa - 1][P]);
        const int32_t rows = min(kWave, cnt - rc);
        const int32_t j0 = uni(qp1[P]), j1 = uni(qp1[P + 1]);
        float acc = 0.f;
        if (rows > kWave / 2) {
            qt_sweep<T, true>(acc, qt1, j0, j1, 0, 1, (int64_t)(rc + min(lane, rows - 1)) * 4, Up, Dp, tpool, xs);
            if (lane < rows) ypart[p0 + rc + lane] = acc;
            return;
        }
        // a box of at most 32 rows: lane groups take the table in turn
        const int G = kWave / rows, g = lane / rows, r = lane % rows;
        if (g < G) qt_sweep<T, false>(acc, qt1, j0, j1, g, G, (int64_t)(rc + r) * 4, Up, Dp, tpool, xs);
        red[wave][lane] = g < G ? acc : 0.f;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (lane < rows) {
            float sum = 0.f;
            for (int gg = 0; gg < G; ++gg) sum += red[wave][gg * rows + lane];
            ypart[p0 + rc + lane] = sum;
        }
        return;
    }
    const int32_t it = xcd_sub(w, nb1, (int32_t)gridDim.x - nb1) * 4 + wave;
    if (it >= nb2items) return;
    const int2 c = b2items[it];
    const int32_t X = uni(c.x), rc = uni(c.y);
    const int32_t r0 = uni(L.begin[kappa][X]), cnt = uni(L.count[kappa][X]);
    const int32_t rows = min(S2, cnt - rc);
    const int32_t j0 = uni(qp2[X]), j1 = uni(qp2[X + 1]);
    float acc = 0.f;
    if (rows > kWave / 2) {
        qt_sweep<T, true>(acc, qt2, j0, j1, 0, 1, (int64_t)(rc + min(lane, rows - 1)) * 4, Up, Dp, tpool, xs);
        if (lane < rows) yleaf[r0 + rc + lane] = acc;
        return;
    }
    const int G = kWave / rows, g = lane / rows, r = lane % rows;
    if (g < G) qt_sweep<T, false>(acc, qt2, j0, j1, g, G, (int64_t)(rc + r) * 4, Up, Dp, tpool, xs);
    red[wave][lane] = g < G ? acc : 0.f;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane < rows) {
        float sum = 0.f;
        for (int gg = 0; gg < G; ++gg) sum += red[wave][gg * rows + lane];
        yleaf[r0 + rc + lane] = sum;
    }
}

// Phase B on an adaptive tree (leaves at several levels).  One wave per
// 64-row chunk of a leaf; the chunk's rows are rounded up to S = 8, 16, 32
// or 64 and lane (g, r) owns row r and the columns g, g + G, ... (G = 64 / S)
// of every block, so small leaves still keep every lane loading.  The
// wave sums, in a fixed order, the leaf's dense near-field blocks, then
// the blocks whose target is the leaf or one of its ancestors, from the
// leaf up; the G column-group sums of a row are added in order at the end.
// U and D are plain column-major (ld = the target box's size).
__global__ void __launch_bounds__(256)
k_phaseB_adaptive(int32_t nitems, const int2* __restrict__ items, const int32_t* __restrict__ leaf_level,
                  const int32_t* __restrict__ leaf_box, LevelPtrs L, const int32_t* __restrict__ near_ptr,
                  const BDesc* __restrict__ bnear, const BDesc* __restrict__ bil, const double* __restrict__ Up,
                  const double* __restrict__ Dp, const double* __restrict__ tpool, const double* __restrict__ xs,
                  double* __restrict__ y)
{
    __shared__ double red[4][kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t it = blockIdx.x * 4 + wave;
    if (it >= nitems) return;
    const int2 w = items[it];
    const int32_t X = uni(w.x), rc = uni(w.y);
    const int lx = uni(leaf_level[X]);
    const int32_t box = uni(leaf_box[X]);
    const int32_t r0 = uni(L.begin[lx][box]), cnt = uni(L.count[lx][box]);
    const int32_t rows = min(kWave, cnt - rc);
    const int S = rows <= 8 ? 8 : rows <= 16 ? 16 : rows <= 32 ? 32 : 64, G = kWave / S;
    const int g = lane / S, r = lane % S;
    const bool act = r < rows;
    const int32_t row = r0 + rc + r;
    double acc = 0.0;
    const int32_t n0 = uni(near_ptr[X]), n1 = uni(near_ptr[X + 1]);
    for (int32_t q = n0; q < n1; ++q) {
        const BDesc d = uni(bnear[q]);
        if (!act) continue;
        const double* base = Dp + d.off + rc + r;
        const double* xv = xs + d.tsrc;
        dot_cols(acc, base, cnt, xv, -d.cols, g, G);
    }
    int32_t a = box;
    for (int l = lx; l >= 1; --l) {
        const int32_t ab = uni(L.begin[l][a]), m = uni(L.count[l][a]);
        const int32_t q0 = uni(L.il_ptr[l][a]), q1 = uni(L.il_ptr[l][a + 1]);
        for (int32_t q = q0; q < q1; ++q) {
            const BDesc d = uni(bil[q]);
            if (!act || d.cols == 0) continue;
            const int64_t roff = (int64_t)(row - ab);
            if (d.cols > 0) {
                const double* base = Up + d.off + roff;
                const double* tv = tpool + d.tsrc;
                dot_cols(acc, base, m, tv, d.cols, g, G);
            } else {
                const double* base = Dp + d.off + roff;
                const double* xv = xs + d.tsrc;
                dot_cols(acc, base, m, xv, -d.cols, g, G);
            }
        }
        a = uni(L.parent[l][a]);
    }
    red[wave][lane] = act ? acc : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane < rows) {
        double s = 0.0;
        for (int gg = 0; gg < G; ++gg) s += red[wave][gg * S + lane];
        y[r0 + rc + lane] = s;
    }
}

// y (caller order) = ypart + yleaf (+ the FP32 self diagonal times x for
// the half pools), one thread per tree row.
template <typename A, bool kHalf>
__global__ void k_combine(int32_t n, const A* __restrict__ ypart, const A* __restrict__ yleaf,
                          const int32_t* __restrict__ perm, const float* __restrict__ diag, const A* __restrict__ xs,
                          double* __restrict__ y)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    A s = yleaf[i];
    if (ypart) s += ypart[i];
    if constexpr (kHalf) s += (A)diag[i] * xs[i];
    y[perm[i]] = (double)s;
}

template <typename T>
static void upload_vec(DBuf<T>& d, const std::vector<T>& h, hipStream_t s)
{
    d.alloc(std::max<size_t>(h.size(), 1));
    if (!h.empty()) HIPCK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// The phase-A schedule, grouped by source box: the low-rank blocks in
// (source level, source box) order, each source box cut into chunks of
// a_rows rows; one item per chunk lists the blocks of its source.  A block
// whose source spans several chunks gets one partial per chunk (k values at
// partial offset + chunk k) and a reduction.  Items largest work first.
// Needs the t offsets; returns the partial values.
static int64_t build_phase_a(Handle& H, hipStream_t s)
{
    const int32_t ar = std::max(16, std::min<int32_t>(H.a_rows, kPhaseARows));
    std::vector<int64_t> idx;
    for (int64_t b = 0; b < H.n_il; ++b)
        if (H.h_il_kind[b] != kDense && H.h_il_k[b] > 0) idx.push_back(b);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        const int la = il_src_level(H, a), lb = il_src_level(H, b);
        return la != lb ? la < lb : H.h_il_src[a] < H.h_il_src[b];
    });
    std::vector<MRBlk> blks;
    std::vector<MRItem> items;
    std::vector<int64_t> work;
    std::vector<RDesc> red;
    int64_t poff = 0;
    for (size_t g0 = 0; g0 < idx.size();) {
        const int ls = il_src_level(H, idx[g0]);
        const int32_t src = H.h_il_src[idx[g0]];
        size_t g1 = g0;
        while (g1 < idx.size() && il_src_level(H, idx[g1]) == ls && H.h_il_src[idx[g1]] == src) ++g1;
        const int32_t n = H.lev[ls].h_count[src], c0 = H.lev[ls].h_begin[src];
        const int32_t parts = (n + ar - 1) / ar;
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
        for (int32_t p = 0; p < parts; ++p) {
            const int32_t j0 = p * ar, j1 = std::min(n, j0 + ar);
            items.push_back(MRItem{c0, j0, j1, b0, (int32_t)blks.size(), p});
            work.push_back((int64_t)(j1 - j0) * ksum);
        }
        g0 = g1;
    }
    if (poff > INT32_MAX) fail(H2D_EUNSUPPORTED, "phase-A partial pool above 2^31 values");
    std::vector<int64_t> ord(items.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int64_t)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return work[a] > work[b]; });
    std::vector<MRItem> sorted(items.size());
    for (size_t i = 0; i < ord.size(); ++i) sorted[i] = items[ord[i]];
    upload_vec(H.a_items, sorted, s);
    upload_vec(H.a_blks, blks, s);
    upload_vec(H.ritems, red, s);
    H.n_aitems = (int64_t)sorted.size();
    H.n_ritems = (int64_t)red.size();
    return poff;
}

// Device tables and the matvec schedule from the host block tables.
void finalize(Handle& H, hipStream_t s)
{
    const int kappa = H.kappa;
    for (int l = 0; l <= kappa; ++l) {
        Level& L = H.lev[l];
        if (L.h_il_ptr.empty()) L.h_il_ptr.assign(L.nbox + 1, 0);
        upload_vec(L.il_ptr, L.h_il_ptr, s);
    }
    upload_vec(H.near_ptr, H.h_near_ptr, s);
    const Level& LL = H.lev[kappa];
    std::vector<BDesc> bn(H.h_near_src.size());
    for (size_t q = 0; q < bn.size(); ++q) {
        int32_t y = H.h_near_src[q];
        bn[q] = BDesc{H.h_near_off[q], -LL.h_count[y], LL.h_begin[y]};
    }
    upload_vec(H.bnear, bn, s);
    const int64_t nil = H.n_il;
    std::vector<BDesc> bi(nil);
    H.h_il_toff.assign(nil, -1);
    int64_t toff = 0;
    H.max_rank = 0; H.sum_rank = 0; H.n_il_dense = 0;
    double flops = 0;
    double store_anc = 0, store_leaf = 0, t_leaf = 0;   // stored values read by the B1 / B2 halves, t values by B2
    for (int64_t b = 0; b < nil; ++b) {
        const Level& L = H.lev[H.h_il_level[b]];
        const bool leaf = H.h_il_level[b] == kappa;
        int32_t m = L.h_count[H.h_il_tgt[b]], n = L.h_count[H.h_il_src[b]], c0 = L.h_begin[H.h_il_src[b]];
        if (H.h_il_kind[b] == kDense) {
            bi[b] = BDesc{H.h_il_off[b], -n, c0};
            H.n_il_dense++;
            (leaf ? store_leaf : store_anc) += (double)m * n;
            flops += 2.0 * m * n;
            continue;
        }
        int32_t k = H.h_il_k[b];
        H.max_rank = std::max<int64_t>(H.max_rank, k);
        H.sum_rank += k;
        bi[b] = BDesc{H.h_il_off[b], k, (int32_t)toff};
        if (k == 0) continue;
        H.h_il_toff[b] = (int32_t)toff;
        (leaf ? store_leaf : store_anc) += (double)m * k;
        if (leaf) t_leaf += k;
        flops += 2.0 * k * (double)(m + n);
        toff += k;
    }
    const int64_t poff = build_phase_a(H, s);
    double near_e = 0;
    for (int64_t x = 0; x < LL.nbox; ++x)
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q)
            near_e += (double)LL.h_count[x] * LL.h_count[H.h_near_src[q]];
    flops += 2.0 * near_e;
    store_leaf += near_e;
    // phase-B1 work: 64-row chunks (multi-RHS) and b1_rows-row slices
    // (single-RHS) of the boxes one level above the leaves.  Unless set, the
    // slice rows S minimise sum over boxes of ceil(rows / S) (S + 16): the
    // slots of padded rows plus a fixed cost per item in row units (every
    // item walks its box's ancestors once).  Uniform points (boxes of a few
    // hundred points) take 64; clustered ones, whose boxes at that level
    // mostly hold a few points, take 16 (a wave then covers 4 column groups
    // of a 16-row slice instead of idling most of 64 lanes).
    if (!H.b1_rows_set && kappa >= 2) {
        const Level& T = H.lev[kappa - 1];
        int64_t best = -1;
        for (int32_t S : {64, 32, 16}) {
            int64_t cost = 0;
            for (int64_t p = 0; p < T.nbox; ++p) cost += (int64_t)((T.h_count[p] + S - 1) / S) * (S + 16);
            if (best < 0 || cost < best) {
                best = cost;
                H.b1_rows = S;
            }
        }
    }
    std::vector<int2> b1, b1s;
    const int32_t S = H.b1_rows;
    if (kappa >= 2) {
        const Level& T = H.lev[kappa - 1];
        for (int64_t p = 0; p < T.nbox; ++p) {
            for (int32_t rc = 0; rc < T.h_count[p]; rc += kWave) b1.push_back(make_int2((int32_t)p, rc));
            for (int32_t rc = 0; rc < T.h_count[p]; rc += S) b1s.push_back(make_int2((int32_t)p, rc));
        }
    }
    // phase-B2 work: b2_rows-row chunks of the leaf boxes
    std::vector<int2> b2;
    const int32_t S2 = H.b2_rows;
    for (int64_t x = 0; x < LL.nbox; ++x)
        for (int32_t rc = 0; rc < LL.h_count[x]; rc += S2) b2.push_back(make_int2((int32_t)x, rc));
    H.n_b2 = (int64_t)b2.size();
    upload_vec(H.b2items, b2, s);
    H.n_b1 = (int64_t)b1.size();
    H.n_b1s = (int64_t)b1s.size();
    upload_vec(H.b1items, b1, s);
    upload_vec(H.b1s_items, b1s, s);
    H.flops = flops;
    H.t_elems = toff; H.p_elems = poff;
    // algorithmic bytes per kernel: every stored value and vector touched once
    const double nvec = (double)H.n;
    for (int h = 0; h < 2; ++h) {
        const double sz = h ? 2.0 : 8.0, a = h ? 4.0 : 8.0;   // storage, accumulation sizes
        const double anc_t = (double)toff - t_leaf;
        H.phase_bytes[h][0] = nvec * (8 + 4 + a);                                          // x, perm -> xs
        H.phase_bytes[h][1] = (double)H.v_elems * sz + nvec * a + (double)toff * a + (double)poff * a;
        H.phase_bytes[h][2] = poff ? (double)poff * a + (double)toff * a : 0.0;           // partials -> t
        // phase B: ancestor blocks -> ypart, leaf blocks and near field -> yleaf
        H.phase_bytes[h][3] = (H.n_b1 ? store_anc * sz + anc_t * a + nvec * a : 0.0) + store_leaf * sz + t_leaf * a +
                              nvec * a;
        // combine: ypart + yleaf (+ diagonal and x for half) -> y via perm
        H.phase_bytes[h][4] = nvec * (a + 4 + 8) + (H.n_b1 ? nvec * a : 0.0) + (h ? nvec * (4 + a) : 0.0);
    }
    // one matvec: gather + A + (reduce) + B + combine (intermediate vectors counted once each way)
    for (int h = 0; h < 2; ++h) {
        double t = 0;
        for (int p = 0; p < 5; ++p) t += H.phase_bytes[h][p];
        (h ? H.alg_bytes_half : H.alg_bytes_fp64) = t;
    }
    upload_vec(H.bil, bi, s);
    H.ws_nrhs = 0;   // partial pools depend on the schedule: reallocate on next use
    H.mr_cap = 0;
    HIPCK(hipStreamSynchronize(s));
}

// Device tables and the matvec schedule of an adaptive handle: phase A as
// for a balanced tree (items per block and row range of its source box),
// phase B one item per 64-row chunk of every leaf.
void finalize_adaptive(Handle& H, hipStream_t s)
{
    const int kappa = H.kappa;
    for (int l = 0; l <= kappa; ++l) {
        Level& L = H.lev[l];
        if (L.h_il_ptr.empty()) L.h_il_ptr.assign(L.nbox + 1, 0);
        upload_vec(L.il_ptr, L.h_il_ptr, s);
    }
    upload_vec(H.near_ptr, H.h_near_ptr, s);
    upload_vec(H.leaf_level, H.h_leaf_level, s);
    upload_vec(H.leaf_box, H.h_leaf_box, s);
    const int64_t nleaf = (int64_t)H.h_leaf_level.size();
    std::vector<BDesc> bn(H.h_near_src.size());
    double store = 0, flops = 0;
    for (int64_t x = 0; x < nleaf; ++x)
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
            const int32_t y = H.h_near_src[q];
            bn[q] = BDesc{H.h_near_off[q], -H.h_leaf_count[y], H.h_leaf_begin[y]};
            store += (double)H.h_leaf_count[x] * H.h_leaf_count[y];
        }
    flops += 2.0 * store;
    upload_vec(H.bnear, bn, s);
    const int64_t nil = H.n_il;
    std::vector<BDesc> bi(nil);
    H.h_il_toff.assign(nil, -1);
    int64_t toff = 0;
    H.max_rank = 0; H.sum_rank = 0; H.n_il_dense = 0;
    for (int64_t b = 0; b < nil; ++b) {
        const Level& L = H.lev[H.h_il_level[b]];
        const Level& Ls = H.lev[il_src_level(H, b)];
        const int32_t m = L.h_count[H.h_il_tgt[b]], n = Ls.h_count[H.h_il_src[b]], c0 = Ls.h_begin[H.h_il_src[b]];
        if (H.h_il_kind[b] == kDense) {
            bi[b] = BDesc{H.h_il_off[b], -n, c0};
            H.n_il_dense++;
            store += (double)m * n;
            flops += 2.0 * m * n;
            continue;
        }
        const int32_t k = H.h_il_k[b];
        H.max_rank = std::max<int64_t>(H.max_rank, k);
        H.sum_rank += k;
        bi[b] = BDesc{H.h_il_off[b], k, (int32_t)toff};
        if (k == 0) continue;
        H.h_il_toff[b] = (int32_t)toff;
        store += (double)m * k;
        flops += 2.0 * k * (double)(m + n);
        toff += k;
    }
    const int64_t poff = build_phase_a(H, s);
    std::vector<int2> ad;
    for (int64_t x = 0; x < nleaf; ++x)
        for (int32_t rc = 0; rc < H.h_leaf_count[x]; rc += kWave) ad.push_back(make_int2((int32_t)x, rc));
    H.n_ad_items = (int64_t)ad.size();
    upload_vec(H.ad_items, ad, s);
    H.n_b1 = H.n_b1s = H.n_b2 = 0;
    H.flops = flops;
    H.t_elems = toff; H.p_elems = poff;
    const double nvec = (double)H.n;
    H.phase_bytes[0][0] = nvec * (8 + 4 + 8);
    H.phase_bytes[0][1] = (double)H.v_elems * 8 + nvec * 8 + (double)toff * 8 + (double)poff * 8;
    H.phase_bytes[0][2] = poff ? (double)poff * 8 + (double)toff * 8 : 0.0;
    H.phase_bytes[0][3] = store * 8 + (double)toff * 8 + nvec * 8;
    H.phase_bytes[0][4] = nvec * (8 + 4 + 8);
    H.alg_bytes_fp64 = 0;
    for (int p = 0; p < 5; ++p) H.alg_bytes_fp64 += H.phase_bytes[0][p];
    H.alg_bytes_half = 0;
    upload_vec(H.bil, bi, s);
    H.ws_nrhs = 0;
    H.mr_cap = 0;
    HIPCK(hipStreamSynchronize(s));
}

void ensure_workspace(Handle& H, int nrhs)
{
    if (H.ws_nrhs >= nrhs) return;
    const int64_t n = H.n;
    H.xs.alloc((size_t)n * nrhs);
    H.ypart.alloc((size_t)2 * n * nrhs);   // ancestor sums, then leaf-level sums
    H.tpool.alloc(std::max<int64_t>(H.t_elems, 1) * nrhs);
    H.ppool.alloc(std::max<int64_t>(H.p_elems, 1) * nrhs);
    if (H.prec_mask & (H2D_PREC_BIT(H2D_P_FP16) | H2D_PREC_BIT(H2D_P_BF16))) {
        // x and t carry 4 values of slack: the half phase-B walks read
        // multiplier values in fours and drop those past a block's columns
        H.xs32.alloc((size_t)n * nrhs + 4);
        H.ypart32.alloc((size_t)2 * n * nrhs);
        H.tpool32.alloc(std::max<int64_t>(H.t_elems, 1) * nrhs + 4);
        H.ppool32.alloc(std::max<int64_t>(H.p16_elems, 1) * nrhs);
    }
    H.ws_nrhs = nrhs;
}

static LevelPtrs level_ptrs(const Handle& H)
{
    LevelPtrs P{};
    for (int l = 0; l <= H.kappa; ++l) {
        P.begin[l] = H.lev[l].begin.p;
        P.count[l] = H.lev[l].count.p;
        P.parent[l] = H.lev[l].parent.p;
        P.il_ptr[l] = H.lev[l].il_ptr.p;
    }
    return P;
}

constexpr size_t kProfMax = 65536;
constexpr int kEv = 6;   // events per recorded matvec: around gather, A, reduce, B, combine

static hipEvent_t* prof_slot(Handle& H)
{
    if (!H.prof_on || H.prof_used >= kProfMax) return nullptr;
    size_t need = (H.prof_used + 1) * kEv;
    while (H.prof_ev.size() < need) {
        hipEvent_t e;
        HIPCK(hipEventCreate(&e));
        H.prof_ev.push_back(e);
    }
    return H.prof_ev.data() + H.prof_used * kEv;
}

template <typename T, typename A, bool kHalf>
static void run_one(Handle& H, const T* U, const T* V, const T* D, A* xs, A* tp, A* pp, A* yp, const double* x,
                    double* y, hipStream_t s, bool may_profile = true)
{
    const int32_t n = (int32_t)H.n;
    hipEvent_t* ev = may_profile ? prof_slot(H) : nullptr;
    if (ev) HIPCK(hipEventRecord(ev[0], s));
    k_gather<A><<<(n + 255) / 256, 256, 0, s>>>(x, H.perm.p, n, 0, 0, 1, xs);
    if (ev) HIPCK(hipEventRecord(ev[1], s));
    if constexpr (kHalf) {
        if (H.n_aw_items)
            k_phaseA_wide<T><<<(unsigned)((H.n_aw_items + 3) / 4), 256, 0, s>>>(H.n_aw_items, H.aw_items.p, H.aw_map.p, V,
                                                                               xs, tp, pp);
        if (ev) HIPCK(hipEventRecord(ev[2], s));
        if (H.n_aw_red)
            k_reduce_wide<<<dim3((unsigned)H.n_aw_red, (unsigned)((H.aw_red_maxw + kWave - 1) / kWave)), 256, 0, s>>>(
                H.n_aw_red, H.aw_red.p, H.aw_map.p, pp, tp);
    } else {
        if (H.n_aitems) k_phaseA<<<(unsigned)H.n_aitems, 256, 0, s>>>(H.a_items.p, H.a_blks.p, V, xs, tp, pp);
        if (ev) HIPCK(hipEventRecord(ev[2], s));
        if (H.n_ritems) k_reduce_parts<A><<<(unsigned)H.n_ritems, 256, 0, s>>>(H.n_ritems, H.ritems.p, pp, tp);
    }
    if (ev) HIPCK(hipEventRecord(ev[3], s));
    const LevelPtrs LP = level_ptrs(H);
    if constexpr (!kHalf) {
        if (H.adaptive) {
            double* yl = yp + n;
            if (H.n_ad_items)
                k_phaseB_adaptive<<<(unsigned)((H.n_ad_items + 3) / 4), 256, 0, s>>>(
                    (int32_t)H.n_ad_items, H.ad_items.p, H.leaf_level.p, H.leaf_box.p, LP, H.near_ptr.p, H.bnear.p,
                    H.bil.p, U, D, tp, xs, yl);
            if (ev) HIPCK(hipEventRecord(ev[4], s));
            k_combine<double, false><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, nullptr, yl, H.perm.p, nullptr, xs,
                                                                                y);
            if (ev) {
                HIPCK(hipEventRecord(ev[5], s));
                H.prof_used++;
            }
            HIPCK(hipGetLastError());
            return;
        }
    }
    A* yl = yp + n;   // the work vector holds ypart then yleaf
    int32_t ni = 0;
    if constexpr (kHalf) {
        // the half pools: table-driven walks, 64-row slices above the leaves
        ni = (int32_t)H.n_b1;
        const int32_t nb1 = (ni + 3) / 4, nb2 = (int32_t)((H.n_b2 + 3) / 4);
        k_phaseB_half<T><<<(unsigned)(nb1 + nb2), 256, 0, s>>>(nb1, ni, H.b1items.p, H.kappa, LP, H.qp1.p, H.qt1.p,
                                                                H.qp2.p, H.qt2.p, U, D, tp, xs, yp, yl, H.b2items.p,
                                                                (int32_t)H.n_b2, H.b2_rows);
    } else {
        ni = (int32_t)H.n_b1s;
        const int32_t nb1 = (ni + 3) / 4, nb2 = (int32_t)((H.n_b2 + 3) / 4);
#define H2D_PHASE_B(SR)                                                                                              \
    k_phaseB<SR><<<(unsigned)(nb1 + nb2), 256, 0, s>>>(nb1, ni, H.b1s_items.p, H.kappa, LP, H.near_ptr.p, H.bnear.p,  \
                                                      H.bil.p, U, D, tp, xs, yp, yl, H.b2items.p, (int32_t)H.n_b2,      \
                                                      H.b2_rows)
        if (H.b1_rows == 16) H2D_PHASE_B(16);
        else if (H.b1_rows == 32) H2D_PHASE_B(32);
        else H2D_PHASE_B(64);
#undef H2D_PHASE_B
    }
    if (ev) HIPCK(hipEventRecord(ev[4], s));
    k_combine<A, kHalf><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, ni ? yp : nullptr, yl, H.perm.p, H.diag32.p, xs,
                                                                   y);
    if (ev) {
        HIPCK(hipEventRecord(ev[5], s));
        H.prof_used++;
    }
    HIPCK(hipGetLastError());
}

void profile_enable(Handle& H, bool on)
{
    H.prof_on = on;
}

void profile_read(Handle& H, h2d_profile* out)
{
    std::memset(out, 0, sizeof(*out));
    out->count = (int32_t)H.prof_used;
    out->prec = H.prof_prec;
    const int h = H.prof_prec == H2D_P_FP64 ? 0 : 1;
    for (int p = 0; p < 5; ++p) out->bytes[p] = H.phase_bytes[h][p];
    if (H.prof_used) HIPCK(hipEventSynchronize(H.prof_ev[H.prof_used * kEv - 1]));
    for (size_t c = 0; c < H.prof_used; ++c)
        for (int p = 0; p < 5; ++p) {
            float ms = 0.f;
            HIPCK(hipEventElapsedTime(&ms, H.prof_ev[c * kEv + p], H.prof_ev[c * kEv + p + 1]));
            out->ms[p] += ms;
        }
    if (H.prof_used)
        for (int p = 0; p < 5; ++p) out->ms[p] /= (double)H.prof_used;
    H.prof_used = 0;
}

void launch_matvec(Handle& H, const double* x, double* y, int nrhs, int64_t ld, int prec, hipStream_t s)
{
    if (H.symmetric) {   // one factor pair per pair: its own three-walk product (FP64)
        launch_matvec_symmetric(H, x, y, nrhs, ld, s);
        return;
    }
    if (nrhs > 1 && !H.adaptive) {   // blocks of 16 right-hand sides on the matrix cores
        launch_matvec_mr(H, x, y, nrhs, ld, prec, s);
        return;
    }
    ensure_workspace(H, 1);
    H.prof_prec = prec;
    for (int r = 0; r < nrhs; ++r) {
        const double* xr = x + (int64_t)r * ld;
        double* yr = y + (int64_t)r * ld;
        if (prec == H2D_P_FP64)
            run_one<double, double, false>(H, H.U64.p, H.V64.p, H.D64.p, H.xs.p, H.tpool.p, H.ppool.p, H.ypart.p, xr,
                                           yr, s);
        else if (prec == H2D_P_FP16)
            run_one<__half, float, true>(H, H.U16.p, H.V16.p, H.D16.p, H.xs32.p, H.tpool32.p, H.ppool32.p, H.ypart32.p,
                                         xr, yr, s);
        else
            run_one<__hip_bfloat16, float, true>(H, H.Ub16.p, H.Vb16.p, H.Db16.p, H.xs32.p, H.tpool32.p, H.ppool32.p,
                                                  H.ypart32.p, xr, yr, s);
    }
}

// ---------------------------------------------------------------------
// The same single-RHS product with its work vectors (x in tree order, the
// t values, the split-block partials, the two phase-B sums) in a fixed
// device array instead of the handle's buffers, for callers that cannot
// allocate.  Each GPU the library runs on holds its own copy of the array
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress gives for the current device (the array's name is a
// host-side stand-in).  Every kernel writes each work value before it is
// read, so nothing needs clearing between calls.  Calls that overlap in
// time on one GPU share the array and race.
// ---------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)H2D_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices] = {};

// Device address of this GPU's scratch array, looked up once per device.
static char* scratch_base(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) fail(H2D_EDEVICE, "device index out of range for the fixed work space");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(H2D_EDEVICE, std::string("hipGetSymbolAddress of the fixed work space failed: ") +
                                  hipGetErrorString(e));
        }
        g_scratch[dev] = p;
    }
    return static_cast<char*>(g_scratch[dev]);
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Work-space bytes of one product of H at storage precision prec, laid out
// as xs (n), the two phase-B sums (2 n), t, partials: each 256-byte aligned.
size_t noalloc_bytes(const Handle& H, int prec)
{
    const size_t a = prec == H2D_P_FP64 ? sizeof(double) : sizeof(float);
    // x and t with 4 values of slack (the half phase-B walks read
    // multiplier values in fours)
    // (the half pools have partial rows of their own)
    const int64_t pe = prec == H2D_P_FP64 ? H.p_elems : H.p16_elems;
    return align256(a * ((size_t)H.n + 4)) + align256(a * 2 * (size_t)H.n) +
           align256(a * ((size_t)std::max<int64_t>(H.t_elems, 1) + 4)) + align256(a * (size_t)std::max<int64_t>(pe, 1));
}

void launch_matvec_noalloc(Handle& H, const double* x, double* y, int prec, hipStream_t s)
{
    int dev = 0;
    HIPCK(hipGetDevice(&dev));
    if (dev != H.device) fail(H2D_EINVAL, "the handle lives on another device than the current one");
    const size_t need = noalloc_bytes(H, prec);
    if (need > kScratchBytes)
        fail(H2D_EINVAL, "this product needs " + std::to_string(need) + " bytes of work space; the fixed array holds " +
                             std::to_string(kScratchBytes));
    char* base = scratch_base(dev);
    const size_t a = prec == H2D_P_FP64 ? sizeof(double) : sizeof(float);
    const size_t o_yp = align256(a * ((size_t)H.n + 4));
    const size_t o_tp = o_yp + align256(a * 2 * (size_t)H.n);
    const size_t o_pp = o_tp + align256(a * ((size_t)std::max<int64_t>(H.t_elems, 1) + 4));
    if (prec == H2D_P_FP64) {
        double* w = reinterpret_cast<double*>(base);
        run_one<double, double, false>(H, H.U64.p, H.V64.p, H.D64.p, w, (double*)(base + o_tp), (double*)(base + o_pp),
                                       (double*)(base + o_yp), x, y, s, false);
    } else if (prec == H2D_P_FP16) {
        run_one<__half, float, true>(H, H.U16.p, H.V16.p, H.D16.p, (float*)base, (float*)(base + o_tp),
                                     (float*)(base + o_pp), (float*)(base + o_yp), x, y, s, false);
    } else {
        run_one<__hip_bfloat16, float, true>(H, H.Ub16.p, H.Vb16.p, H.Db16.p, (float*)base, (float*)(base + o_tp),
                                              (float*)(base + o_pp), (float*)(base + o_yp), x, y, s, false);
    }
}

}  // namespace h2d
