// One factor pair per interaction-list pair (symmetric kernels), gfx950.
//
// Section 2.1 takes the interaction matrix symmetric; for a symmetric
// kernel the block of the pair (C', C) is the transpose of the block of
// (C, C').  A symmetric handle compresses only the owner block of each pair,
// the one whose target box has the smaller index: (X, Y) ~ F_X F_Y^T; the
// mirror (Y, X) ~ F_Y F_X^T uses the same two factors.  Both factors are
// stored column-major, tiled like U by the boxes one level above the leaves
// (F_Y by Y's boxes), so a wave that owns a slice of rows reads its part of
// either factor as it reads U in the ordered product.
//
// Product (no atomics; every output row is owned by one wave per pass and
// every sum is taken in a fixed order, so two runs give identical bits):
//   gather:   xs = x(perm)
//   walk 1:   per 64-row slice of a box one level above the leaves, up its
//             ancestors: for every owner block (X, Y) of the ancestor, the
//             slice's partial of the mirror's t = F_X^T xs(X)
//   reduce 1: partials -> t of the mirrors
//   walk 2:   per slice, for every mirror block (Y, X) of the ancestors:
//             y2 += F_Y t (the slice's rows), and from the same loads the
//             slice's partial of the owner's t = F_Y^T xs(Y).  In the same
//             launch one wave per leaf Y applies its self block and every
//             leaf-level pair {X < Y} (dense edge-sharing and
//             interaction-list blocks, compressed blocks) in both
//             directions from one read of the pair's data: Y's rows into
//             yown, X's rows into a slot of their own
//   reduce 2: partials -> t of the owners
//   walk 3:   per slice, y3 = y2 + sum over the owner blocks (X, Y) of
//             F_X t; in the same launch one wave per leaf adds its slots
//             to yown, in a fixed order -> yleaf
//   combine:  y = y3 + yleaf in caller order
// Above the leaf level F_X is read twice (walks 1 and 3) and F_Y once:
// 3/4 of the ordered form's factor bytes; leaf-level pairs once: 1/2.
// A dense block above the leaf level is stored once too: walk 3 reads it
// for the owner, walk 2 reads it row by row (transposed) for the mirror.
#include "h2d_impl.h"

#include <algorithm>
#include <cstring>

namespace h2d {

namespace {

constexpr int kSymS = 64;      // rows per walk slice (one per lane)
constexpr int kSymChunk = 8;   // factor columns per cross-lane partial sum
constexpr int kSymSeg = 32;    // slice partials one reduction wave sums at most

struct SymLevels {
    const int32_t* begin[kMaxLevel + 1];
    const int32_t* count[kMaxLevel + 1];
    const int32_t* parent[kMaxLevel + 1];
    const int32_t* il_ptr[kMaxLevel + 1];
    const int32_t* mid[kMaxLevel + 1];
    const int32_t* first[kMaxLevel + 1];
};

using cdouble = const __attribute__((address_space(4))) double;

__device__ __forceinline__ int32_t su(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t su(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
// acc += sum over c = g, g + G, ... < n of base[c ld] w[c], eight columns
// per lane loaded before any is multiplied (a short tail is padded with
// zero products instead of running one memory latency per column); the
// products are added in increasing c.
template <typename W>
__device__ __forceinline__ void dot8(double& acc, const double* base, int64_t ld, const W* w, int32_t n, int g, int G)
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
                t[u] = w[c];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u] * t[u];
    }
}

// A double moved between lanes by a DPP pattern (two 32-bit moves).
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, kCtrl, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), kCtrl, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over each aligned group of 8 lanes, in every lane of the group: the
// pairs (l, l ^ 1) and (l, l ^ 2) of a quad, then the two quads of the
// group (row_half_mirror pairs lane j with 7 - j).
__device__ __forceinline__ double sum8(double s)
{
    s += dpp_f64<0xB1>(s);    // quad_perm [1, 0, 3, 2]
    s += dpp_f64<0x4E>(s);    // quad_perm [2, 3, 0, 1]
    s += dpp_f64<0x141>(s);   // row_half_mirror
    return s;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// One walk item: lane r owns row r of a 64-row slice of box P one level
// above the leaves; the wave visits P and each of its ancestors and, for
// the owner blocks (kOwner) or the mirror blocks of that box's list,
// applies the block's target-side factor to its t (kApply) and/or sums the
// slice's part of F^T xs for the partner block (kReduce).  The partial sums
// go through LDS 8 columns at a time (4 KB per wave, so LDS does not cap
// the waves per CU below what the registers allow): lane (c, h) adds the 8
// products of lanes 8 h .. 8 h + 7 for column c, then three DPP steps
// finish the 64-row sum.
template <bool kApply, bool kReduce, bool kOwner>
__device__ __forceinline__ void sym_walk(int32_t it, int lane, double* red, const int2* __restrict__ items, int tl,
                                         const SymLevels& L, const SDesc* __restrict__ sd,
                                         const double* __restrict__ Fp, const double* __restrict__ Dp,
                                         const double* __restrict__ tpool, const double* __restrict__ xs,
                                         double* __restrict__ ppool, double* __restrict__ yout,
                                         const double* __restrict__ yadd)
{
    const int2 w = items[it];
    const int32_t P = su(w.x), rc = su(w.y);
    const int32_t p0 = su(L.begin[tl][P]), cnt = su(L.count[tl][P]);
    const int32_t rows = min(kSymS, cnt - rc);
    const int r = lane;
    const bool act = r < rows;
    double xr = 0.0;
    if constexpr (kReduce) xr = act ? xs[p0 + rc + r] : 0.0;
    double acc = 0.0;
    int32_t a_box = P;
    for (int l = tl; l >= 1; --l) {
        const int32_t ab = su(L.begin[l][a_box]), ld_m = su(L.count[l][a_box]);
        const int32_t q0 = su(kOwner ? L.mid[l][a_box] : L.il_ptr[l][a_box]);
        const int32_t q1 = su(kOwner ? L.il_ptr[l][a_box + 1] : L.mid[l][a_box]);
        int32_t sl = 0;
        if constexpr (kReduce) sl = it - su(L.first[l][a_box]);
        for (int32_t q = q0; q < q1; ++q) {
            const SDesc d = sd[q];
            const int64_t off = su(d.off);
            const int32_t cols = su(d.cols), tsrc = su(d.tsrc);
            if (cols > 0) {
                // this box's tile of the factor: a cnt x cols column-major matrix
                const double* base = Fp + off + (int64_t)cols * (p0 - ab) + rc + r;
                const cdouble* tv = (const cdouble*)(tpool + tsrc);
                if constexpr (!kReduce) {
                    if (act) dot8(acc, base, cnt, tv, cols, 0, 1);
                } else {
                    double* pout = ppool + su(d.part) + (int64_t)sl * cols;
                    for (int32_t c0 = 0; c0 < cols; c0 += kSymChunk) {
                        const int32_t nc = min(kSymChunk, cols - c0);
                        // the chunk's t values: one vector load, then lane
                        // reads (scalar-cache loads would share a wait
                        // counter with the LDS traffic below)
                        double tc = 0.0;
                        if constexpr (kApply) tc = lane < nc ? tpool[tsrc + c0 + lane] : 0.0;
                        double pr[kSymChunk];
#pragma unroll
                        for (int cc = 0; cc < kSymChunk; ++cc) {
                            double v = 0.0;
                            if (cc < nc && act) v = base[(int64_t)(c0 + cc) * cnt];
                            if constexpr (kApply) {
                                const uint64_t tb = __double_as_longlong(tc);
                                const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)tb, cc);
                                const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(tb >> 32), cc);
                                acc += v * __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
                            }
                            pr[cc] = v * xr;
                        }
#pragma unroll
                        for (int cc = 0; cc < kSymChunk; ++cc) red[cc * kWave + lane] = pr[cc];
                        wave_sync();
                        constexpr int kPer = kWave / kSymChunk;   // lanes per column
                        const int cc = lane / kPer, h = lane % kPer;
                        double sum = 0.0;
#pragma unroll
                        for (int i = 0; i < kSymChunk; ++i) sum += red[cc * kWave + h * kSymChunk + i];
                        static_assert(kPer == 8, "the butterfly below sums groups of 8 lanes");
                        sum = sum8(sum);
                        if (h == 0 && cc < nc) pout[c0 + cc] = sum;
                        wave_sync();
                    }
                }
            } else if (cols < 0) {
                if constexpr (kApply) {
                    const cdouble* xv = (const cdouble*)(xs + tsrc);
                    if (su(d.part) == 0) {
                        const double* base = Dp + off + (p0 - ab + rc + r);
                        if (act) dot8(acc, base, ld_m, xv, -cols, 0, 1);
                    } else {   // the owner's block, this row of the mirror is its column
                        const double* base = Dp + off + (int64_t)(p0 - ab + rc + r) * (-cols);
                        if (act) dot8(acc, base, 1, xv, -cols, 0, 1);
                    }
                }
            }
        }
        a_box = su(L.parent[l][a_box]);
    }
    if constexpr (kApply) {
        if (act) yout[p0 + rc + r] = acc + (yadd ? yadd[p0 + rc + r] : 0.0);
    }
}

// Group sum over lanes (g, i), g < G, i < m of one value per lane (lanes
// past G m hold 0); lane i < m returns the sum over g in order.
__device__ __forceinline__ double group_sum(double v, int lane, int m, int G, double* red)
{
    red[lane] = v;
    wave_sync();
    double t = 0.0;
    if (lane < m)
        for (int gg = 0; gg < G; ++gg) t += red[gg * m + lane];
    wave_sync();
    return t;
}

// One wave per leaf Y (at most 64 points): lane (g, r) owns row r of Y and
// the columns g, g + G, ... (G = 64 / |Y|) of every block applied to Y's
// rows; for X's rows the same layout with |X|.  xs of Y, and of each
// partner X in turn, sit in LDS.  Per pair {X, Y}:
//   dense D (|X| x |Y|): X's rows D xs(Y) (coalesced read) and Y's rows
//     D^T xs(X) (the same block again, from the cache);
//   low rank: t1 = F_X^T xs(X), t2 = F_Y^T xs(Y) (lane (g, q) sums rows
//     g, g + G', ... of column q, G' = 64 / k), then Y's rows F_Y t1 and
//     X's rows F_X t2 (again from the cache).
// X's rows are summed over their column groups in order into the pair's
// slot; Y's rows accumulate over all pairs and are summed once at the end.
__device__ __forceinline__ void sym_leaf(int32_t Y, int lane, double* lds, int kappa, const SymLevels& L,
                                         const int32_t* __restrict__ lp_ptr, const LPair* __restrict__ lp,
                                         const int64_t* __restrict__ self_off, const double* __restrict__ Fp,
                                         const double* __restrict__ Dp, const double* __restrict__ xs,
                                         double* __restrict__ yown, double* __restrict__ slots)
{
    double* xY = lds;                 // 64
    double* xX = lds + kWave;         // 64
    double* red = lds + 2 * kWave;    // 64
    double* red2 = lds + 3 * kWave;   // 64
    double* tv = lds + 4 * kWave;     // 128: t1, then t2 at +64
    const int32_t r0 = su(L.begin[kappa][Y]), m = su(L.count[kappa][Y]);
    const int G = kWave / m, g = lane / m, r = lane % m;
    const bool act = g < G;
    const int32_t e0 = su(lp_ptr[Y]), e1 = su(lp_ptr[Y + 1]);
    LPair nx{};
    if (e0 < e1) nx = lp[e0];
    if (lane < m) xY[lane] = xs[r0 + lane];
    wave_sync();
    double acc = 0.0;
    {
        const double* D = Dp + su(self_off[Y]) + r;
        if (act) dot8(acc, D, m, xY, m, g, G);
    }
    for (int32_t e = e0; e < e1; ++e) {
        const int64_t pa = su(nx.a), pb = su(nx.b), slot = su(nx.slot);
        const int32_t x0 = su(nx.x0), mx = su(nx.mx), k = su(nx.k);
        if (e + 1 < e1) nx = lp[e + 1];   // the next descriptor, in flight during this pair
        // X's x values, in flight while the parts that need only xs(Y) run
        const double xv = lane < mx ? xs[x0 + lane] : 0.0;
        const int Gx = kWave / mx, gx = lane / mx, ix = lane % mx;
        const bool actx = gx < Gx;
        double sx = 0.0;
        if (k < 0) {
            const double* Dr = Dp + pa + ix;
            if (actx) dot8(sx, Dr, mx, xY, m, gx, Gx);
            if (lane < mx) xX[lane] = xv;
            wave_sync();
            const double* Dc = Dp + pa + (int64_t)r * mx;
            if (act) dot8(acc, Dc, 1, xX, mx, g, G);
        } else {
            const double* FX = Fp + pa;
            const double* FY = Fp + pb;
            const int Gq = kWave / k, gq = lane / k, qq = lane % k;
            double s1 = 0.0, s2 = 0.0;
            if (gq < Gq) dot8(s2, FY + (int64_t)qq * m, 1, xY, m, gq, Gq);
            if (lane < mx) xX[lane] = xv;
            wave_sync();
            if (gq < Gq) dot8(s1, FX + (int64_t)qq * mx, 1, xX, mx, gq, Gq);
            red[lane] = s1;
            red2[lane] = s2;
            wave_sync();
            if (lane < k) {
                double a1 = 0.0, a2 = 0.0;
                for (int gg = 0; gg < Gq; ++gg) {
                    a1 += red[gg * k + lane];
                    a2 += red2[gg * k + lane];
                }
                tv[lane] = a1;
                tv[kWave + lane] = a2;
            }
            wave_sync();
            if (act) dot8(acc, FY + r, m, tv, k, g, G);
            if (actx) dot8(sx, FX + ix, mx, tv + kWave, k, gx, Gx);
        }
        const double t = group_sum(actx ? sx : 0.0, lane, mx, Gx, red);
        if (lane < mx) slots[slot + lane] = t;
    }
    const double t = group_sum(act ? acc : 0.0, lane, m, G, red);
    if (lane < m) yown[r0 + lane] = t;
}

__global__ void k_sym_gather(const double* __restrict__ x, const int32_t* __restrict__ perm, int32_t n,
                             double* __restrict__ xs)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) xs[i] = x[perm[i]];
}

// Walk 1: the mirrors' t partials from the owner factors F_X.
__global__ void __launch_bounds__(256)
k_sym_walk1(int32_t nitems, const int2* __restrict__ items, int tl, SymLevels L, const SDesc* __restrict__ sd,
            const double* __restrict__ Fp, const double* __restrict__ xs, double* __restrict__ ppool)
{
    __shared__ double lds[4][kSymChunk * kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t it = blockIdx.x * 4 + wave;
    if (it >= nitems) return;
    sym_walk<false, true, true>(it, lane, lds[wave], items, tl, L, sd, Fp, nullptr, nullptr, xs, ppool, nullptr,
                                nullptr);
}

// Walk 2: the mirrors' F_Y t into y2 and the owners' t partials.
__global__ void __launch_bounds__(256)
k_sym_walk2(int32_t nitems, const int2* __restrict__ items, int tl, SymLevels L, const SDesc* __restrict__ sd,
            const double* __restrict__ Fp, const double* __restrict__ Dp, const double* __restrict__ tpool,
            const double* __restrict__ xs, double* __restrict__ ppool, double* __restrict__ y2)
{
    __shared__ double lds[4][kSymChunk * kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t it = blockIdx.x * 4 + wave;
    if (it >= nitems) return;
    sym_walk<true, true, false>(it, lane, lds[wave], items, tl, L, sd, Fp, Dp, tpool, xs, ppool, y2, nullptr);
}

// The leaf-level pairs, one wave per leaf.
__global__ void __launch_bounds__(256)
k_sym_leaf(int32_t nleaf, int kappa, SymLevels L, const int32_t* __restrict__ lp_ptr, const LPair* __restrict__ lp,
           const int64_t* __restrict__ self_off, const double* __restrict__ Fp, const double* __restrict__ Dp,
           const double* __restrict__ xs, double* __restrict__ yown, double* __restrict__ slots)
{
    __shared__ double lds[4][6 * kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t Y = blockIdx.x * 4 + wave;
    if (Y >= nleaf) return;
    sym_leaf(Y, lane, lds[wave], kappa, L, lp_ptr, lp, self_off, Fp, Dp, xs, yown, slots);
}

// Walk 3 (first nw workgroups) and the slot sums per leaf (the rest).
__global__ void __launch_bounds__(256)
k_sym_walk3(int32_t nw, int32_t nitems, const int2* __restrict__ items, int tl, SymLevels L,
            const SDesc* __restrict__ sd, const double* __restrict__ Fp, const double* __restrict__ Dp,
            const double* __restrict__ tpool, const double* __restrict__ xs, const double* __restrict__ y2,
            double* __restrict__ y3, int32_t nleaf, int kappa, const int64_t* __restrict__ slot_base,
            const int32_t* __restrict__ nslot, const double* __restrict__ yown, const double* __restrict__ slots,
            double* __restrict__ yleaf)
{
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t w = blockIdx.x;
    if (w < nw) {
        const int32_t it = w * 4 + wave;
        if (it < nitems)
            sym_walk<true, false, true>(it, lane, nullptr, items, tl, L, sd, Fp, Dp, tpool, xs, nullptr, y3, y2);
    } else {
        const int32_t X = (w - nw) * 4 + wave;
        if (X >= nleaf) return;
        const int32_t r0 = su(L.begin[kappa][X]), mx = su(L.count[kappa][X]);
        const int64_t sb = su(slot_base[X]);
        const int32_t ns = su(nslot[X]);
        if (lane < mx) {
            double s = yown[r0 + lane];
            for (int32_t q = 0; q < ns; ++q) s += slots[sb + (int64_t)q * mx + lane];
            yleaf[r0 + lane] = s;
        }
    }
}

// Sums of consecutive k-value partials (slice-major, in the t pool):
// out = sum of the nparts rows at pbeg, one wave per descriptor.  Lane
// (g, q), G = 64 / k (k <= 64), sums column q over the rows g, g + G, ...
// and the G sums are added in order; for k > 64 lane q, q + 64, ... sums
// its columns over all rows.  Blocks with many slices are summed in two
// launches (runs of at most kSymSeg slices, then the runs), so no wave
// sums a long chain.
__global__ void __launch_bounds__(256)
k_sym_reduce(int64_t nr, const RDesc* __restrict__ R, double* __restrict__ tpool)
{
    __shared__ double red[4][kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t b = (int64_t)blockIdx.x * 4 + wave;
    if (b >= nr) return;
    const RDesc D = R[b];
    const int32_t tout = su(D.tout), k = su(D.k), pbeg = su(D.pbeg), np = su(D.nparts);
    if (k > kWave) {
        for (int q = lane; q < k; q += kWave) {
            double s = 0.0;
#pragma unroll 4
            for (int32_t i = 0; i < np; ++i) s += tpool[pbeg + (int64_t)i * k + q];
            tpool[tout + q] = s;
        }
        return;
    }
    const int G = kWave / k, g = lane / k, q = lane % k;
    double s = 0.0;
    if (g < G) {
        const double* p = tpool + pbeg + q;
#pragma unroll 4
        for (int32_t i = g; i < np; i += G) s += p[(int64_t)i * k];
    }
    red[wave][lane] = s;
    wave_sync();
    if (lane < k) {
        double a = 0.0;
        for (int gg = 0; gg < G; ++gg) a += red[wave][gg * k + lane];
        tpool[tout + lane] = a;
    }
}

__global__ void k_sym_combine(int32_t n, const double* __restrict__ y3, const double* __restrict__ yleaf,
                              const int32_t* __restrict__ perm, double* __restrict__ y)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = yleaf[i];
    if (y3) s += y3[i];
    y[perm[i]] = s;
}

template <typename T>
void up(DBuf<T>& d, const std::vector<T>& h, hipStream_t s)
{
    d.alloc(std::max<size_t>(h.size(), 1));
    if (!h.empty()) HIPCK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// index of the block (l, tgt, src) in the per-level CSR, or -1
int64_t find_block(const Handle& H, int l, int32_t tgt, int32_t src)
{
    const Level& L = H.lev[l];
    const int32_t* a = H.h_il_src.data();
    int64_t lo = L.h_il_ptr[tgt], hi = L.h_il_ptr[tgt + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (a[mid] < src) lo = mid + 1; else hi = mid;
    }
    return (lo < L.h_il_ptr[tgt + 1] && a[lo] == src) ? lo : -1;
}

// near entry (x, y) of leaf x, or -1
int64_t find_near(const Handle& H, int32_t x, int32_t y)
{
    for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q)
        if (H.h_near_src[q] == y) return q;
    return -1;
}

int64_t tiled_pos(const std::vector<int32_t>& tbeg, const std::vector<int32_t>& tcnt, bool tiled, int32_t row0,
                  int64_t m, int64_t k, int64_t i, int64_t q)
{
    if (!tiled) return q * m + i;
    const int64_t pb = tbeg[row0 + i] - row0, pc = tcnt[row0 + i];
    return k * pb + q * pc + (i - pb);
}

}  // namespace

void tile_map(const Handle& H, std::vector<int32_t>& tbeg, std::vector<int32_t>& tcnt)
{
    tbeg.assign(H.n, 0);
    tcnt.assign(H.n, 0);
    if (H.kappa < 1) return;
    const Level& T = H.lev[H.kappa - 1];
    for (int64_t p = 0; p < T.nbox; ++p)
        for (int32_t i = T.h_begin[p]; i < T.h_begin[p] + T.h_count[p]; ++i) {
            tbeg[i] = T.h_begin[p];
            tcnt[i] = T.h_count[p];
        }
}

void symmetric_partners(Handle& H)
{
    const int64_t nil = H.n_il;
    H.h_il_partner.assign(nil, -1);
    for (int64_t b = 0; b < nil; ++b) {
        const int l = H.h_il_level[b];
        const int32_t t = H.h_il_tgt[b], s = H.h_il_src[b];
        if (t == s) fail(H2D_EINVAL, "interaction-list block of a box with itself");
        if (b > 0 && H.h_il_level[b - 1] == l && H.h_il_tgt[b - 1] == t && H.h_il_src[b - 1] >= s)
            fail(H2D_EINVAL, "interaction-list sources not ascending");
        const int64_t p = find_block(H, l, s, t);
        if (p < 0) fail(H2D_EINVAL, "interaction lists are not symmetric");
        H.h_il_partner[b] = p;
    }
    const Level& LL = H.lev[H.kappa];
    for (int64_t x = 0; x < LL.nbox; ++x) {
        if (LL.h_count[x] > kSymLeafMax)
            fail(H2D_EUNSUPPORTED, "symmetric handles need leaves of at most " + std::to_string(kSymLeafMax) +
                                       " points");
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
            if (q > H.h_near_ptr[x] && H.h_near_src[q - 1] >= H.h_near_src[q])
                fail(H2D_EINVAL, "near sources not ascending");
            if (find_near(H, H.h_near_src[q], (int32_t)x) < 0) fail(H2D_EINVAL, "near lists are not symmetric");
        }
    }
}

void finalize_symmetric(Handle& H, hipStream_t s)
{
    const int kappa = H.kappa;
    const int64_t nil = H.n_il;
    const Level& LL = H.lev[kappa];
    for (int l = 0; l <= kappa; ++l) {
        Level& L = H.lev[l];
        if (L.h_il_ptr.empty()) L.h_il_ptr.assign(L.nbox + 1, 0);
        up(L.il_ptr, L.h_il_ptr, s);
    }
    up(H.near_ptr, H.h_near_ptr, s);
    // walk slices: 64-row slices of the boxes one level above the leaves
    std::vector<int2> items;
    std::vector<std::vector<int32_t>> first(kappa + 1);
    if (kappa >= 2) {
        const Level& T = H.lev[kappa - 1];
        std::vector<int32_t> box_first(T.nbox + 1);
        for (int64_t p = 0; p < T.nbox; ++p) {
            box_first[p] = (int32_t)items.size();
            for (int32_t rc = 0; rc < T.h_count[p]; rc += kSymS) items.push_back(make_int2((int32_t)p, rc));
        }
        box_first[T.nbox] = (int32_t)items.size();
        // first slice of every ancestor: the first slice of its first descendant
        for (int l = 1; l <= kappa - 1; ++l) first[l].assign(H.lev[l].nbox + 1, -1);
        for (int64_t p = T.nbox - 1; p >= 0; --p) {
            int32_t a = (int32_t)p;
            for (int l = kappa - 1; l >= 1; --l) {
                first[l][a] = box_first[p];
                a = H.lev[l].h_parent[a];
            }
        }
        for (int l = 1; l <= kappa - 1; ++l) first[l][H.lev[l].nbox] = (int32_t)items.size();
    }
    H.n_s_items = (int64_t)items.size();
    up(H.s_items, items, s);
    // owner / mirror split of every box's list
    for (int l = 0; l <= kappa; ++l) {
        const Level& L = H.lev[l];
        std::vector<int32_t> mid(std::max<int64_t>(L.nbox, 1), 0);
        for (int64_t a = 0; a < L.nbox; ++a) {
            int32_t q = L.h_il_ptr[a];
            while (q < L.h_il_ptr[a + 1] && H.h_il_src[q] < a) ++q;
            mid[a] = q;
        }
        up(H.s_mid[l], mid, s);
        if (l >= 1 && l <= kappa - 1) up(H.s_first[l], first[l], s);
        else H.s_first[l].reset();
    }
    // t offsets (every low-rank block), descriptors, partial regions
    std::vector<int32_t> toff(nil, -1);
    int64_t t_el = 0;
    H.max_rank = 0; H.sum_rank = 0; H.n_il_dense = 0;
    for (int64_t b = 0; b < nil; ++b) {
        if (H.h_il_kind[b] == kDense) { H.n_il_dense++; continue; }
        const int32_t k = H.h_il_k[b];
        H.max_rank = std::max<int64_t>(H.max_rank, k);
        H.sum_rank += k;
        if (k > 0) { toff[b] = (int32_t)t_el; t_el += k; }
    }
    H.h_il_toff = toff;
    auto nslices = [&](int l, int32_t a) -> int32_t { return first[l][a + 1] - first[l][a]; };
    std::vector<SDesc> sd(nil);
    std::vector<RDesc> r1, r2, r1b, r2b;
    int64_t poff = 0, p1 = 0, p2 = 0;
    // slice partials (past the t values), then the run sums of long partial
    // chains (past the partials): sizes first
    int64_t ptot = 0, nsegv = 0;
    for (int64_t b = 0; b < nil; ++b) {
        const int l = H.h_il_level[b];
        if (H.h_il_kind[b] == kDense || H.h_il_k[b] == 0 || l == kappa) continue;
        const int32_t ns = first[l][H.h_il_tgt[b] + 1] - first[l][H.h_il_tgt[b]];
        if (ns > 1) ptot += (int64_t)ns * H.h_il_k[b];
        if (ns > kSymSeg) nsegv += (int64_t)((ns + kSymSeg - 1) / kSymSeg) * H.h_il_k[b];
    }
    int64_t segoff = t_el + ptot;
    double anc_fx = 0, anc_fy = 0, anc_dense_own = 0, anc_dense_mir = 0, t_anc = 0;
    for (int64_t b = 0; b < nil; ++b) {
        const int l = H.h_il_level[b];
        const int32_t tg = H.h_il_tgt[b], sr = H.h_il_src[b];
        const int32_t m = H.lev[l].h_count[tg], nsrc = H.lev[l].h_count[sr];
        if (H.h_il_kind[b] == kDense) {
            sd[b] = SDesc{H.h_il_off[b], -nsrc, H.lev[l].h_begin[sr], tg > sr ? 1 : 0};
            if (l < kappa) ((tg < sr) ? anc_dense_own : anc_dense_mir) += (double)m * nsrc;
            continue;
        }
        const int32_t k = H.h_il_k[b];
        sd[b] = SDesc{H.h_il_off[b], k, std::max(toff[b], 0), 0};
        if (k == 0 || l == kappa) continue;
        const int32_t ns = nslices(l, tg);
        (tg < sr ? anc_fx : anc_fy) += (double)m * k;
        t_anc += k;
        if (ns == 1) {   // one slice: the walk writes the partner's t itself
            sd[b].part = toff[H.h_il_partner[b]];
            continue;
        }
        // partial sums of the partner's t, from this block's target-side
        // factor, in the t pool past the t values
        sd[b].part = t_el + poff;
        const int32_t tp = toff[H.h_il_partner[b]];
        std::vector<RDesc>& ra = (tg < sr) ? r1 : r2;
        std::vector<RDesc>& rb = (tg < sr) ? r1b : r2b;
        ((tg < sr) ? p1 : p2) += (int64_t)ns * k;
        if (ns <= kSymSeg) {
            ra.push_back(RDesc{tp, k, (int32_t)(t_el + poff), ns});
        } else {   // runs of kSymSeg slices into run sums (past all partials), then the runs
            const int32_t nseg = (ns + kSymSeg - 1) / kSymSeg;
            for (int32_t g = 0; g < nseg; ++g)
                ra.push_back(RDesc{(int32_t)(segoff + (int64_t)g * k), k,
                                   (int32_t)(t_el + poff + (int64_t)g * kSymSeg * k),
                                   std::min(kSymSeg, ns - g * kSymSeg)});
            rb.push_back(RDesc{tp, k, (int32_t)segoff, nseg});
            segoff += (int64_t)nseg * k;
        }
        poff += (int64_t)ns * k;
    }
    if (t_el + ptot + nsegv >= ((int64_t)1 << 31)) fail(H2D_EUNSUPPORTED, "t and partial pool exceeds 2^31 values");
    H.t_elems = t_el + ptot + nsegv;   // t values, slice partials, run sums
    H.p_elems = 0;
    up(H.sdesc, sd, s);
    {
        std::vector<RDesc>* lists[4] = {&r1, &r1b, &r2, &r2b};
        for (int i = 0; i < 4; ++i) {
            up(H.s_red[i], *lists[i], s);
            H.n_s_red[i] = (int64_t)lists[i]->size();
        }
    }
    // leaf pairs: for leaf X, its partners Y > X (near, then leaf-level IL)
    // in ascending order take its slots 0, 1, ...
    const int64_t nleaf = LL.nbox;
    std::vector<int32_t> nslot(nleaf, 0);
    std::vector<int64_t> slot_base(nleaf, 0), self_off(nleaf, 0);
    auto pair_used = [&](int64_t b) { return H.h_il_kind[b] == kDense || H.h_il_k[b] > 0; };
    for (int64_t x = 0; x < nleaf; ++x) {
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
            if (H.h_near_src[q] == x) self_off[x] = H.h_near_off[q];
            if (H.h_near_src[q] > x) nslot[x]++;
        }
        for (int32_t q = LL.h_il_ptr[x]; q < LL.h_il_ptr[x + 1]; ++q)
            if (H.h_il_src[q] > x && pair_used(q)) nslot[x]++;
    }
    int64_t sl = 0;
    for (int64_t x = 0; x < nleaf; ++x) {
        slot_base[x] = sl;
        sl += (int64_t)nslot[x] * LL.h_count[x];
    }
    H.s_slot_elems = sl;
    // slot index of pair (X, Y) within X's list
    std::vector<int32_t> next(nleaf, 0);
    std::vector<int32_t> lp_ptr(nleaf + 1, 0);
    std::vector<LPair> lps;
    double leaf_pair_vals = 0, self_vals = 0;
    // X's slots are numbered in the order of X's partners; Y visits its
    // partners X < Y in ascending order, so count the position per X first
    std::vector<std::vector<int32_t>> xlist(nleaf);
    for (int64_t x = 0; x < nleaf; ++x) {
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q)
            if (H.h_near_src[q] > x) xlist[x].push_back(-1 - q);              // near entry
        for (int32_t q = LL.h_il_ptr[x]; q < LL.h_il_ptr[x + 1]; ++q)
            if (H.h_il_src[q] > x && pair_used(q)) xlist[x].push_back(q);     // IL block
    }
    std::vector<int64_t> slot_of_near(H.h_near_src.size(), -1), slot_of_il(nil, -1);
    for (int64_t x = 0; x < nleaf; ++x)
        for (size_t i = 0; i < xlist[x].size(); ++i) {
            const int32_t v = xlist[x][i];
            const int64_t so = slot_base[x] + (int64_t)i * LL.h_count[x];
            if (v < 0) slot_of_near[-1 - v] = so; else slot_of_il[v] = so;
        }
    for (int64_t y = 0; y < nleaf; ++y) {
        lp_ptr[y] = (int32_t)lps.size();
        const int64_t my = LL.h_count[y];
        self_vals += (double)my * my;
        for (int32_t q = H.h_near_ptr[y]; q < H.h_near_ptr[y + 1]; ++q) {
            const int32_t x = H.h_near_src[q];
            if (x >= y) continue;
            const int64_t own = find_near(H, x, (int32_t)y);
            lps.push_back(LPair{H.h_near_off[own], 0, slot_of_near[own], LL.h_begin[x], LL.h_count[x], -1, 0});
            leaf_pair_vals += (double)LL.h_count[x] * my;
        }
        for (int32_t q = LL.h_il_ptr[y]; q < LL.h_il_ptr[y + 1]; ++q) {
            const int32_t x = H.h_il_src[q];
            if (x >= y) continue;
            const int64_t own = H.h_il_partner[q];
            if (!pair_used(own)) continue;
            if (H.h_il_kind[own] == kDense) {
                lps.push_back(LPair{H.h_il_off[own], 0, slot_of_il[own], LL.h_begin[x], LL.h_count[x], -1, 0});
                leaf_pair_vals += (double)LL.h_count[x] * my;
            } else {
                lps.push_back(LPair{H.h_il_off[own], H.h_il_voff[own], slot_of_il[own], LL.h_begin[x], LL.h_count[x],
                                    H.h_il_k[own], 0});
                leaf_pair_vals += (double)(LL.h_count[x] + my) * H.h_il_k[own];
            }
        }
    }
    lp_ptr[nleaf] = (int32_t)lps.size();
    up(H.s_lp_ptr, lp_ptr, s);
    up(H.s_lp, lps, s);
    up(H.s_self, self_off, s);
    up(H.s_slot_base, slot_base, s);
    up(H.s_nslot, nslot, s);
    // algorithmic bytes of one product: every stored value each time a pass
    // reads it, the vectors once per pass that touches them
    const double nv = (double)H.n, t_half = 0.5 * t_anc;   // owners and mirrors hold the same t sizes
    double fl = 0;
    for (int64_t b = 0; b < nil; ++b) {
        const int l = H.h_il_level[b];
        const double m = H.lev[l].h_count[H.h_il_tgt[b]], nn = H.lev[l].h_count[H.h_il_src[b]];
        fl += H.h_il_kind[b] == kDense ? 2.0 * m * nn : 2.0 * H.h_il_k[b] * (m + nn);
    }
    for (int64_t x = 0; x < nleaf; ++x)
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q)
            fl += 2.0 * LL.h_count[x] * LL.h_count[H.h_near_src[q]];
    H.flops = fl;
    const bool walks = kappa >= 2;
    const double slv = (double)sl;
    double* pb = H.phase_bytes[0];
    // gather: x, perm -> xs
    pb[0] = nv * (8 + 4 + 8);
    // walk 1 (F_X, xs -> partials) + reduce 1 (partials -> mirrors' t)
    pb[1] = walks ? 8 * (anc_fx + nv + (double)p1) + 8 * ((double)p1 + t_half) : 0.0;
    // walk 2 (F_Y, mirror dense blocks, mirrors' t, xs -> y2, partials) +
    // leaf pairs (self and pair data, xs -> yown, slots)
    pb[2] = (walks ? 8 * (anc_fy + anc_dense_mir + t_half + nv + (double)p2 + nv) : 0.0) +
            8 * (self_vals + leaf_pair_vals + nv + slv + nv);
    // reduce 2 (partials -> owners' t) + walk 3 (F_X, owner dense blocks,
    // owners' t, y2 -> y3) + slot sums (yown, slots -> yleaf)
    pb[3] = (walks ? 8 * ((double)p2 + t_half) + 8 * (anc_fx + anc_dense_own + t_half + nv + nv) : 0.0) +
            8 * (nv + slv + nv);
    // combine: y3, yleaf, perm -> y
    pb[4] = nv * (8 + 4 + 8) + (walks ? nv * 8 : 0.0);
    double tb = 0;
    for (int p = 0; p < 5; ++p) tb += pb[p];
    H.alg_bytes_fp64 = tb;
    H.alg_bytes_half = 0;
    H.ws_nrhs = 0;
    HIPCK(hipStreamSynchronize(s));
}

static SymLevels sym_levels(const Handle& H)
{
    SymLevels P{};
    for (int l = 0; l <= H.kappa; ++l) {
        P.begin[l] = H.lev[l].begin.p;
        P.count[l] = H.lev[l].count.p;
        P.parent[l] = H.lev[l].parent.p;
        P.il_ptr[l] = H.lev[l].il_ptr.p;
        P.mid[l] = H.s_mid[l].p;
        P.first[l] = H.s_first[l].p;
    }
    return P;
}

static hipEvent_t* sym_prof_slot(Handle& H)
{
    constexpr size_t kMax = 65536;
    if (!H.prof_on || H.prof_used >= kMax) return nullptr;
    const size_t need = (H.prof_used + 1) * 6;
    while (H.prof_ev.size() < need) {
        hipEvent_t e;
        HIPCK(hipEventCreate(&e));
        H.prof_ev.push_back(e);
    }
    return H.prof_ev.data() + H.prof_used * 6;
}

void launch_matvec_symmetric(Handle& H, const double* x, double* y, int nrhs, int64_t ld, hipStream_t s)
{
    const int32_t n = (int32_t)H.n;
    const int kappa = H.kappa;
    if (H.ws_nrhs < 1 || H.s_y.n < (size_t)(4 * n)) {
        H.xs.alloc((size_t)n);
        H.tpool.alloc(std::max<int64_t>(H.t_elems, 1));
        H.s_y.alloc((size_t)4 * n);
        H.s_slots.alloc(std::max<int64_t>(H.s_slot_elems, 1));
        H.ws_nrhs = 1;
    }
    H.prof_prec = H2D_P_FP64;
    const SymLevels L = sym_levels(H);
    double* y2 = H.s_y.p;
    double* y3 = H.s_y.p + n;
    double* yown = H.s_y.p + 2 * (int64_t)n;
    double* yleaf = H.s_y.p + 3 * (int64_t)n;
    const int32_t ni = (int32_t)H.n_s_items, nw = (ni + 3) / 4;
    const int32_t nleaf = (int32_t)H.lev[kappa].nbox, nlw = (nleaf + 3) / 4;
    const int tl = kappa - 1;
    for (int r = 0; r < nrhs; ++r) {
        const double* xr = x + (int64_t)r * ld;
        double* yr = y + (int64_t)r * ld;
        hipEvent_t* ev = sym_prof_slot(H);
        if (ev) HIPCK(hipEventRecord(ev[0], s));
        k_sym_gather<<<(n + 255) / 256, 256, 0, s>>>(xr, H.perm.p, n, H.xs.p);
        if (ev) HIPCK(hipEventRecord(ev[1], s));
        auto reduce = [&](int i) {
            if (H.n_s_red[i])
                k_sym_reduce<<<(unsigned)((H.n_s_red[i] + 3) / 4), 256, 0, s>>>(H.n_s_red[i], H.s_red[i].p, H.tpool.p);
        };
        if (ni) {
            k_sym_walk1<<<(unsigned)nw, 256, 0, s>>>(ni, H.s_items.p, tl, L, H.sdesc.p, H.U64.p, H.xs.p, H.tpool.p);
            reduce(0);
            reduce(1);
        }
        if (ev) HIPCK(hipEventRecord(ev[2], s));
        if (ni)
            k_sym_walk2<<<(unsigned)nw, 256, 0, s>>>(ni, H.s_items.p, tl, L, H.sdesc.p, H.U64.p, H.D64.p, H.tpool.p,
                                                      H.xs.p, H.tpool.p, y2);
        k_sym_leaf<<<(unsigned)nlw, 256, 0, s>>>(nleaf, kappa, L, H.s_lp_ptr.p, H.s_lp.p, H.s_self.p, H.U64.p,
                                                  H.D64.p, H.xs.p, yown, H.s_slots.p);
        if (ev) HIPCK(hipEventRecord(ev[3], s));
        if (ni) {
            reduce(2);
            reduce(3);
        }
        k_sym_walk3<<<(unsigned)(nw + nlw), 256, 0, s>>>(nw, ni, H.s_items.p, tl, L, H.sdesc.p, H.U64.p, H.D64.p,
                                                          H.tpool.p, H.xs.p, y2, y3, nleaf, kappa, H.s_slot_base.p,
                                                          H.s_nslot.p, yown, H.s_slots.p, yleaf);
        if (ev) HIPCK(hipEventRecord(ev[4], s));
        k_sym_combine<<<(n + 255) / 256, 256, 0, s>>>(n, ni ? y3 : nullptr, yleaf, H.perm.p, yr);
        if (ev) {
            HIPCK(hipEventRecord(ev[5], s));
            H.prof_used++;
        }
        HIPCK(hipGetLastError());
    }
}

void symmetrize_import(Handle& H, std::vector<double>& U, std::vector<double>& V, std::vector<double>& D)
{
    const int kappa = H.kappa;
    const int64_t nil = H.n_il;
    const Level& LL = H.lev[kappa];
    symmetric_partners(H);
    std::vector<int32_t> tbeg, tcnt;
    tile_map(H, tbeg, tcnt);
    std::vector<double> NU, ND;
    std::vector<int64_t> noff(nil, 0), nvoff(nil, 0);
    // owners first (table order), then mirrors point at them
    for (int64_t b = 0; b < nil; ++b) {
        const int l = H.h_il_level[b];
        const int32_t tg = H.h_il_tgt[b], sr = H.h_il_src[b];
        const int64_t m = H.lev[l].h_count[tg], nc = H.lev[l].h_count[sr];
        const int32_t row0 = H.lev[l].h_begin[tg], col0 = H.lev[l].h_begin[sr];
        const int64_t p = H.h_il_partner[b];
        if (H.h_il_kind[b] != H.h_il_kind[p] || H.h_il_k[b] != H.h_il_k[p])
            fail(H2D_EINVAL, "a mirror block's kind or rank differs from its owner's");
        const bool tiled = l <= kappa - 1;
        if (H.h_il_kind[b] == kDense) {
            // check against the partner (either order: both are read here)
            for (int64_t j = 0; j < nc; ++j)
                for (int64_t i = 0; i < m; ++i)
                    if (D[H.h_il_off[b] + j * m + i] != D[H.h_il_off[p] + i * nc + j])
                        fail(H2D_EINVAL, "a mirror dense block is not the transpose of its owner");
            if (tg < sr) {
                noff[b] = (int64_t)ND.size();
                ND.insert(ND.end(), D.begin() + H.h_il_off[b], D.begin() + H.h_il_off[b] + m * nc);
            } else {
                noff[b] = noff[p];
            }
            continue;
        }
        const int64_t k = H.h_il_k[b];
        if (tg > sr) {
            // mirror: U (tiled by its target Y) must equal the owner's V, its V the owner's U
            const int64_t uo = H.h_il_off[p];
            const int64_t pm = nc;   // owner's target size |X|
            for (int64_t q = 0; q < k; ++q) {
                for (int64_t i = 0; i < m; ++i)
                    if (U[H.h_il_off[b] + tiled_pos(tbeg, tcnt, tiled, row0, m, k, i, q)] != V[H.h_il_voff[p] + i * k + q])
                        fail(H2D_EINVAL, "a mirror block's U is not its owner's V");
                for (int64_t j = 0; j < pm; ++j)
                    if (V[H.h_il_voff[b] + j * k + q] != U[uo + tiled_pos(tbeg, tcnt, tiled, col0, pm, k, j, q)])
                        fail(H2D_EINVAL, "a mirror block's V is not its owner's U");
            }
            noff[b] = nvoff[p];
            nvoff[b] = noff[p];
            continue;
        }
        // owner: F_X = U (already tiled), then F_Y = V tiled by the source's boxes
        noff[b] = (int64_t)NU.size();
        NU.insert(NU.end(), U.begin() + H.h_il_off[b], U.begin() + H.h_il_off[b] + m * k);
        nvoff[b] = (int64_t)NU.size();
        const size_t o = NU.size();
        NU.resize(o + (size_t)(nc * k));
        for (int64_t j = 0; j < nc; ++j)
            for (int64_t q = 0; q < k; ++q)
                NU[o + tiled_pos(tbeg, tcnt, tiled, col0, nc, k, j, q)] = V[H.h_il_voff[b] + j * k + q];
    }
    // mirrors whose owner comes later in table order do not exist (the owner
    // has the smaller target index, hence comes first at its level)
    // near blocks: self and owners stored, mirrors share
    std::vector<int64_t> nnear(H.h_near_src.size(), 0);
    for (int64_t x = 0; x < LL.nbox; ++x)
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
            const int32_t y = H.h_near_src[q];
            const int64_t m = LL.h_count[x], nc = LL.h_count[y];
            if (y >= x) {
                nnear[q] = (int64_t)ND.size();
                ND.insert(ND.end(), D.begin() + H.h_near_off[q], D.begin() + H.h_near_off[q] + m * nc);
            } else {
                const int64_t p = find_near(H, y, (int32_t)x);
                for (int64_t j = 0; j < nc; ++j)
                    for (int64_t i = 0; i < m; ++i)
                        if (D[H.h_near_off[q] + j * m + i] != D[H.h_near_off[p] + i * nc + j])
                            fail(H2D_EINVAL, "a near block is not the transpose of its partner");
                nnear[q] = nnear[p];
            }
        }
    H.h_il_off = noff;
    H.h_il_voff = nvoff;
    H.h_near_off = nnear;
    U.swap(NU);
    V.clear();
    D.swap(ND);
}

}  // namespace h2d
