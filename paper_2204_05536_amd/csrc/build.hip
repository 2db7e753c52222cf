// Algorithm 1 (InitializeHODLR2D) on gfx950: quadtree, box tables,
// interaction lists and ACA factors, all computed on the device.
#include "h2d_impl.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <tuple>
#include <cstring>
#include <type_traits>

namespace h2d {

// ---------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------

// Spread the low 16 bits of v to the even bit positions.
__device__ __forceinline__ uint32_t spread16(uint32_t v)
{
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ __forceinline__ uint32_t compact16(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0F0F0F0Fu;
    v = (v | (v >> 4)) & 0x00FF00FFu;
    v = (v | (v >> 8)) & 0x0000FFFFu;
    return v;
}

// Morton key of cell (ix, iy): x bits at even, y bits at odd positions, so
// each base-4 digit is 2*ybit + xbit.
__device__ __forceinline__ uint32_t morton(uint32_t ix, uint32_t iy) { return spread16(ix) | (spread16(iy) << 1); }

template <typename T>
__device__ __forceinline__ int64_t lower_bound_dev(const T* a, int64_t n, T v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------
// Exclusive scan of int32 (3 phases).  Values and totals must fit int32.
// ---------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ int32_t block_excl_scan(int32_t v, int32_t* lds, int32_t* total)
{
    int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        int32_t a = (t >= d) ? lds[t - d] : 0;
        __syncthreads();
        lds[t] += a;
        __syncthreads();
    }
    int32_t incl = lds[t];
    if (total) *total = lds[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_sums(const int32_t* in, int64_t n, int32_t* sums)
{
    __shared__ int32_t lds[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    int32_t tot;
    block_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of the tile sums in place; total at sums[nb].
__global__ void k_scan_top(int32_t* sums, int64_t nb)
{
    __shared__ int32_t lds[kScanThreads];
    int32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        int64_t i = base + threadIdx.x;
        int32_t v = (i < nb) ? sums[i] : 0;
        int32_t tot;
        int32_t ex = block_excl_scan(v, lds, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void k_scan_apply(const int32_t* in, int32_t* out, int64_t n, const int32_t* sums)
{
    __shared__ int32_t lds[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int32_t ex = block_excl_scan(s, lds, nullptr) + sums[blockIdx.x];
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = ex;
        ex += v[i];
    }
}

// out[i] = sum_{j < i} in[j]; returns the total (synchronises s).
static int64_t scan_excl(const int32_t* in, int32_t* out, int64_t n, hipStream_t s)
{
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb < 1) nb = 1;
    DBuf<int32_t> sums;
    sums.alloc(nb + 1);
    k_scan_sums<<<nb, kScanThreads, 0, s>>>(in, n, sums.p);
    k_scan_top<<<1, kScanThreads, 0, s>>>(sums.p, nb);
    k_scan_apply<<<nb, kScanThreads, 0, s>>>(in, out, n, sums.p);
    HIPCK(hipGetLastError());
    int32_t tot = 0;
    HIPCK(hipMemcpyAsync(&tot, sums.p + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    return tot;
}

// ---------------------------------------------------------------------
// Box B and Morton keys
// ---------------------------------------------------------------------

// max |coordinate| as the bit pattern of a non-negative double (ordered like
// the value); bad[0] |= 1 on a non-finite coordinate.
__global__ void k_maxabs(const double* xy, int64_t n2, unsigned long long* mx, int* bad)
{
    __shared__ unsigned long long lds[256];
    unsigned long long best = 0;
    int nf = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
        double v = xy[i];
        if (!isfinite(v)) nf = 1;
        unsigned long long b = (unsigned long long)__double_as_longlong(fabs(v));
        best = b > best ? b : best;
    }
    lds[threadIdx.x] = best;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d) lds[threadIdx.x] = max(lds[threadIdx.x], lds[threadIdx.x + d]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(mx, lds[0]);
    if (nf) atomicOr(bad, 1);
}

// Cell of a coordinate at depth 16: v * 2^15 / R is exact (R is a power of
// two), so floor() gives exactly the half-open cell [lo, mid) / [mid, hi];
// the top edge v = R is clamped into the last cell.
__device__ __forceinline__ uint32_t cell16(double v, double scale)
{
    double s = floor(v * scale);
    long long c = (long long)s + 32768;
    c = c < 0 ? 0 : (c > 65535 ? 65535 : c);
    return (uint32_t)c;
}

__global__ void k_keys(const double* xy, int32_t n, double scale, uint32_t* key, int32_t* idx)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = morton(cell16(xy[2 * i], scale), cell16(xy[2 * i + 1], scale));
    idx[i] = i;
}

// ---------------------------------------------------------------------
// Stable LSD radix sort of (key, value) by `bits` low bits, 8 bits a pass.
// Tile = 256 elements, one per thread; the rank of an element inside its
// tile counts the earlier tile elements with the same digit.
// ---------------------------------------------------------------------
__global__ void k_radix_hist(const uint32_t* key, int32_t n, int shift, int32_t* hist, int32_t ntiles)
{
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int32_t e = blockIdx.x * 256 + threadIdx.x;
    if (e < n) atomicAdd(&cnt[(key[e] >> shift) & 255u], 1);
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void k_radix_scatter(const uint32_t* kin, const int32_t* vin, int32_t n, int shift, const int32_t* offs,
                                int32_t ntiles, uint32_t* kout, int32_t* vout)
{
    __shared__ int32_t dig[256];
    int32_t e = blockIdx.x * 256 + threadIdx.x;
    int32_t d = (e < n) ? (int32_t)((kin[e] >> shift) & 255u) : -1;
    dig[threadIdx.x] = d;
    __syncthreads();
    if (e >= n) return;
    int32_t r = 0;
    for (int t = 0; t < (int)threadIdx.x; ++t) r += (dig[t] == d);
    int32_t pos = offs[(int64_t)d * ntiles + blockIdx.x] + r;
    kout[pos] = kin[e];
    vout[pos] = vin[e];
}

static void radix_sort(DBuf<uint32_t>& key, DBuf<int32_t>& val, int32_t n, int bits, hipStream_t s)
{
    if (bits <= 0 || n <= 1) return;
    int32_t ntiles = (n + 255) / 256;
    DBuf<int32_t> hist, offs;
    DBuf<uint32_t> k2;
    DBuf<int32_t> v2;
    hist.alloc((size_t)ntiles * 256);
    offs.alloc((size_t)ntiles * 256);
    k2.alloc(n);
    v2.alloc(n);
    for (int shift = 0; shift < bits; shift += 8) {
        k_radix_hist<<<ntiles, 256, 0, s>>>(key.p, n, shift, hist.p, ntiles);
        scan_excl(hist.p, offs.p, (int64_t)ntiles * 256, s);
        k_radix_scatter<<<ntiles, 256, 0, s>>>(key.p, val.p, n, shift, offs.p, ntiles, k2.p, v2.p);
        HIPCK(hipGetLastError());
        std::swap(key, k2);
        std::swap(val, v2);
    }
}

// Largest number of points in one box at every depth 0..16, from keys
// sorted at depth 16.
__global__ void k_maxrun(const uint32_t* sk, int32_t n, int32_t* maxrun)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int l = 1; l <= kMaxLevel; ++l) {
        int sh = 2 * (kMaxLevel - l);
        uint32_t p = sk[i] >> sh;
        if (i > 0 && (sk[i - 1] >> sh) == p) continue;
        // end of the run: first index whose prefix exceeds p
        int64_t lo = i, hi = n;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((sk[mid] >> sh) <= p) lo = mid + 1; else hi = mid;
        }
        atomicMax(&maxrun[l], (int32_t)(lo - i));
    }
}

__global__ void k_leafkey(const uint32_t* key16, int32_t n, int sh, uint32_t* out)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = sh >= 32 ? 0u : key16[i] >> sh;   // depth 0: a single box
}

__global__ void k_gather_xy(const double* xy, const int32_t* perm, int32_t n, double* xyt)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t p = perm[i];
    xyt[2 * i] = xy[2 * p];
    xyt[2 * i + 1] = xy[2 * p + 1];
}

// Box starts of a level: flag[i] = 1 where the level prefix changes.
__global__ void k_box_flags(const uint32_t* sk, int32_t n, int sh, int32_t* flag)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || (sk[i] >> sh) != (sk[i - 1] >> sh)) ? 1 : 0;
}

__global__ void k_box_fill(const uint32_t* sk, int32_t n, int sh, const int32_t* flag, const int32_t* ex,
                           uint32_t* key, int32_t* begin)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    key[ex[i]] = sk[i] >> sh;
    begin[ex[i]] = i;
}

__global__ void k_box_count(const int32_t* begin, int32_t nbox, int32_t n, int32_t* count)
{
    int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    count[b] = ((b + 1 < nbox) ? begin[b + 1] : n) - begin[b];
}

__global__ void k_box_parent(const uint32_t* key, int32_t nbox, const uint32_t* pkey, int32_t npbox, int32_t* parent)
{
    int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    parent[b] = (int32_t)lower_bound_dev(pkey, (int64_t)npbox, key[b] >> 2);
}

// Two distinct points at the same location inside a leaf box.
__global__ void k_dups(const double* xyt, const int32_t* begin, const int32_t* count, int32_t nbox, int* found)
{
    int32_t b = blockIdx.x;
    if (b >= nbox) return;
    int32_t c = count[b], p0 = begin[b];
    for (int32_t e = threadIdx.x; e < c * c; e += blockDim.x) {
        int32_t i = e / c, j = e % c;
        if (i < j && xyt[2 * (p0 + i)] == xyt[2 * (p0 + j)] && xyt[2 * (p0 + i) + 1] == xyt[2 * (p0 + j) + 1])
            atomicOr(found, 1);
    }
}

// ---------------------------------------------------------------------
// Lists
// ---------------------------------------------------------------------

// Interaction list of box b at level l (Section 4): the clan is the
// siblings plus the children of the parent's edge sharers; keep the clan
// members that neither coincide with nor share an edge with b and hold
// points.  Sources are written in ascending key order.  out == nullptr:
// count only.
__global__ void k_il(const uint32_t* key, int32_t nbox, int level, int32_t* cnt, const int32_t* ptr, int32_t* out)
{
    int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    uint32_t k = key[b];
    int32_t x = (int32_t)compact16(k), y = (int32_t)compact16(k >> 1);
    int32_t px = x >> 1, py = y >> 1, pside = 1 << (level - 1);
    int32_t found[20];
    int nf = 0;
    const int dpx[5] = {0, -1, 1, 0, 0};
    const int dpy[5] = {0, 0, 0, -1, 1};
    for (int e = 0; e < 5; ++e) {   // parent itself (siblings) and its edge sharers
        int32_t qx = px + dpx[e], qy = py + dpy[e];
        if (qx < 0 || qy < 0 || qx >= pside || qy >= pside) continue;
        for (int d = 0; d < 4; ++d) {
            int32_t cx = 2 * qx + (d & 1), cy = 2 * qy + (d >> 1);
            int32_t ax = abs(cx - x), ay = abs(cy - y);
            if (ax + ay <= 1) continue;   // the box itself or an edge sharer
            uint32_t ck = morton((uint32_t)cx, (uint32_t)cy);
            int64_t pos = lower_bound_dev(key, (int64_t)nbox, ck);
            if (pos < nbox && key[pos] == ck) found[nf++] = (int32_t)pos;
        }
    }
    if (!out) { cnt[b] = nf; return; }
    for (int i = 1; i < nf; ++i) {   // insertion sort, at most 15 entries
        int32_t v = found[i];
        int j = i - 1;
        while (j >= 0 && found[j] > v) { found[j + 1] = found[j]; --j; }
        found[j + 1] = v;
    }
    int32_t o = ptr[b];
    for (int i = 0; i < nf; ++i) out[o + i] = found[i];
}

// Near list of leaf box b: itself and its edge sharers that hold points,
// in ascending key order.
__global__ void k_near(const uint32_t* key, int32_t nbox, int level, int32_t* cnt, const int32_t* ptr, int32_t* out)
{
    int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    uint32_t k = key[b];
    int32_t x = (int32_t)compact16(k), y = (int32_t)compact16(k >> 1), side = 1 << level;
    int32_t found[5];
    int nf = 0;
    const int dx[5] = {0, -1, 1, 0, 0};
    const int dy[5] = {0, 0, 0, -1, 1};
    for (int e = 0; e < 5; ++e) {
        int32_t cx = x + dx[e], cy = y + dy[e];
        if (cx < 0 || cy < 0 || cx >= side || cy >= side) continue;
        uint32_t ck = morton((uint32_t)cx, (uint32_t)cy);
        int64_t pos = lower_bound_dev(key, (int64_t)nbox, ck);
        if (pos < nbox && key[pos] == ck) found[nf++] = (int32_t)pos;
    }
    if (!out) { cnt[b] = nf; return; }
    for (int i = 1; i < nf; ++i) {
        int32_t v = found[i];
        int j = i - 1;
        while (j >= 0 && found[j] > v) { found[j + 1] = found[j]; --j; }
        found[j + 1] = v;
    }
    int32_t o = ptr[b];
    for (int i = 0; i < nf; ++i) out[o + i] = found[i];
}

template <typename T>
static std::vector<T> to_host(const T* d, size_t n, hipStream_t s)
{
    std::vector<T> h(n);
    if (n) HIPCK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    return h;
}

template <typename T>
static void upload(DBuf<T>& d, const std::vector<T>& h, hipStream_t s)
{
    d.alloc(h.size());
    if (!h.empty()) HIPCK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// ---------------------------------------------------------------------
// Adaptive tree (host).  A box is split exactly when it holds more than
// leaf_max points (the adaptive form of the quadtree that the end of
// Section 4 allows), so leaves sit at several levels.  Points are ordered by
// (leaf, caller index), leaves in Morton order.  Blocks come from
// descending pairs of boxes from (root, root): distinct boxes whose closed
// squares share at most one point form one compressed block; two leaves
// that share a segment, or a leaf with itself, one dense near-field block;
// any other pair gives way to the pairs of its children (only the non-leaf
// side splits when one side is a leaf).  On a balanced tree this is the
// interaction-list and near-field structure of every level.
// ---------------------------------------------------------------------
static uint32_t compact16(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0F0F0F0Fu;
    v = (v | (v >> 4)) & 0x00FF00FFu;
    v = (v | (v >> 8)) & 0x0000FFFFu;
    return v;
}

// 1 when boxes (la, ka) and (lb, kb) have at most one common point.
static bool boxes_admissible(int la, uint32_t ka, int lb, uint32_t kb)
{
    const int L = std::max(la, lb);
    const int64_t sa = (int64_t)1 << (L - la), sb = (int64_t)1 << (L - lb);
    const int64_t ax = compact16(ka) * sa, ay = compact16(ka >> 1) * sa;
    const int64_t bx = compact16(kb) * sb, by = compact16(kb >> 1) * sb;
    const int64_t wx = std::min(ax + sa, bx + sb) - std::max(ax, bx);
    const int64_t wy = std::min(ay + sa, by + sb) - std::max(ay, by);
    if (wx < 0 || wy < 0) return true;
    return wx == 0 && wy == 0;
}

void adaptive_tree_and_lists(Handle& H, const DBuf<uint32_t>& skey, const DBuf<int32_t>& sidx, hipStream_t s)
{
    const int32_t n = (int32_t)H.n;
    const int T = 256, G = (n + T - 1) / T;
    const std::vector<uint32_t> key = to_host(skey.p, n, s);
    std::vector<int32_t> idx = to_host(sidx.p, n, s);
    // levels: children of every box above leaf_max are the runs of equal
    // key prefix inside it
    for (int l = 0; l <= kMaxLevel; ++l) {
        Level& L = H.lev[l];
        L.nbox = 0;
        L.h_key.clear(); L.h_begin.clear(); L.h_count.clear(); L.h_parent.clear();
    }
    {
        Level& L0 = H.lev[0];
        L0.nbox = 1;
        L0.h_key = {0u}; L0.h_begin = {0}; L0.h_count = {n}; L0.h_parent = {-1};
    }
    int kappa = 0;
    for (int l = 0; l < kMaxLevel; ++l) {
        const Level& P = H.lev[l];
        Level& C = H.lev[l + 1];
        const int sh = 2 * (kMaxLevel - (l + 1));
        for (int64_t b = 0; b < P.nbox; ++b) {
            if (P.h_count[b] <= H.leaf_max) continue;
            const int32_t e = P.h_begin[b] + P.h_count[b];
            for (int32_t i = P.h_begin[b]; i < e;) {
                const uint32_t k = key[i] >> sh;
                int32_t j = i + 1;
                while (j < e && (key[j] >> sh) == k) ++j;
                C.h_key.push_back(k);
                C.h_begin.push_back(i);
                C.h_count.push_back(j - i);
                C.h_parent.push_back((int32_t)b);
                i = j;
            }
        }
        C.nbox = (int64_t)C.h_key.size();
        if (!C.nbox) break;
        kappa = l + 1;
    }
    for (int64_t b = 0; b < H.lev[kappa].nbox; ++b)
        if (H.lev[kappa].h_count[b] > H.leaf_max)
            fail(H2D_EDEPTH, "more than leaf_max points share a depth-16 box");
    H.kappa = kappa;
    // leaves (tree order), caller order inside each leaf
    std::vector<std::vector<int32_t>> nchild(kappa + 1);
    for (int l = 0; l <= kappa; ++l) {
        nchild[l].assign(H.lev[l].nbox, 0);
        if (l > 0)
            for (int32_t p : H.lev[l].h_parent) nchild[l - 1][p]++;
    }
    std::vector<std::vector<int32_t>> leafno(kappa + 1);
    {
        std::vector<std::pair<int32_t, std::pair<int32_t, int32_t>>> lv;   // (begin, (level, box))
        for (int l = 0; l <= kappa; ++l) {
            leafno[l].assign(H.lev[l].nbox, -1);
            for (int64_t b = 0; b < H.lev[l].nbox; ++b)
                if (!nchild[l][b]) lv.push_back({H.lev[l].h_begin[b], {l, (int32_t)b}});
        }
        std::sort(lv.begin(), lv.end());
        H.h_leaf_level.clear(); H.h_leaf_box.clear(); H.h_leaf_begin.clear(); H.h_leaf_count.clear();
        for (size_t q = 0; q < lv.size(); ++q) {
            const int l = lv[q].second.first, b = lv[q].second.second;
            leafno[l][b] = (int32_t)q;
            H.h_leaf_level.push_back(l);
            H.h_leaf_box.push_back(b);
            H.h_leaf_begin.push_back(H.lev[l].h_begin[b]);
            H.h_leaf_count.push_back(H.lev[l].h_count[b]);
            std::sort(idx.begin() + H.lev[l].h_begin[b], idx.begin() + H.lev[l].h_begin[b] + H.lev[l].h_count[b]);
        }
    }
    H.h_perm = idx;
    upload(H.perm, idx, s);
    H.xyt.alloc((size_t)2 * n);
    k_gather_xy<<<G, T, 0, s>>>(H.xy.p, H.perm.p, n, H.xyt.p);
    HIPCK(hipGetLastError());
    for (int l = 0; l <= kappa; ++l) {
        Level& L = H.lev[l];
        upload(L.key, L.h_key, s);
        upload(L.begin, L.h_begin, s);
        upload(L.count, L.h_count, s);
        upload(L.parent, L.h_parent, s);
    }
    if (H.kern.kind == H2D_K_LOG || H.kern.kind == H2D_K_INVR) {   // duplicates: two points in one leaf
        DBuf<int32_t> lb, lc;
        DBuf<int> bad;
        upload(lb, H.h_leaf_begin, s);
        upload(lc, H.h_leaf_count, s);
        bad.alloc(1);
        HIPCK(hipMemsetAsync(bad.p, 0, sizeof(int), s));
        const int32_t nl = (int32_t)H.h_leaf_begin.size();
        k_dups<<<(unsigned)nl, 256, 0, s>>>(H.xyt.p, lb.p, lc.p, nl, bad.p);
        HIPCK(hipGetLastError());
        int hbad = 0;
        HIPCK(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        if (hbad) fail(H2D_EDUP, "two distinct points coincide; the kernel is singular at r = 0");
    }
    // pair descent
    std::vector<std::vector<int32_t>> child0(kappa + 1);
    for (int l = 0; l <= kappa; ++l) {
        child0[l].assign(H.lev[l].nbox, -1);
        if (l < kappa)
            for (int64_t c = H.lev[l + 1].nbox - 1; c >= 0; --c) child0[l][H.lev[l + 1].h_parent[c]] = (int32_t)c;
    }
    struct Pair { int32_t la, a, lb, b; };
    std::vector<Pair> stack{{0, 0, 0, 0}}, il, near;
    while (!stack.empty()) {
        const Pair P = stack.back();
        stack.pop_back();
        const bool leafA = !nchild[P.la][P.a], leafB = !nchild[P.lb][P.b];
        const bool same = P.la == P.lb && P.a == P.b;
        if (!same && boxes_admissible(P.la, H.lev[P.la].h_key[P.a], P.lb, H.lev[P.lb].h_key[P.b])) {
            il.push_back(P);
            continue;
        }
        if (leafA && leafB) {
            near.push_back(P);
            continue;
        }
        const int32_t a0 = leafA ? P.a : child0[P.la][P.a], na = leafA ? 1 : nchild[P.la][P.a];
        const int32_t b0 = leafB ? P.b : child0[P.lb][P.b], nb = leafB ? 1 : nchild[P.lb][P.b];
        const int32_t la = leafA ? P.la : P.la + 1, lb = leafB ? P.lb : P.lb + 1;
        for (int32_t i = 0; i < na; ++i)
            for (int32_t j = 0; j < nb; ++j) stack.push_back({la, a0 + i, lb, b0 + j});
    }
    auto order = [](const Pair& x, const Pair& y) {
        return std::tie(x.la, x.a, x.lb, x.b) < std::tie(y.la, y.a, y.lb, y.b);
    };
    std::sort(il.begin(), il.end(), order);
    // near blocks grouped by target leaf (tree order), then (source level, source)
    std::sort(near.begin(), near.end(), [&](const Pair& x, const Pair& y) {
        const int32_t lx = leafno[x.la][x.a], ly = leafno[y.la][y.a];
        return std::tie(lx, x.lb, x.b) < std::tie(ly, y.lb, y.b);
    });
    const int32_t nleaf = (int32_t)H.h_leaf_level.size();
    H.h_near_ptr.assign(nleaf + 1, 0);
    H.h_near_src.resize(near.size());
    for (size_t q = 0; q < near.size(); ++q) {
        H.h_near_ptr[leafno[near[q].la][near[q].a] + 1]++;
        H.h_near_src[q] = leafno[near[q].lb][near[q].b];
    }
    for (int32_t x = 0; x < nleaf; ++x) H.h_near_ptr[x + 1] += H.h_near_ptr[x];
    H.n_il = (int64_t)il.size();
    H.h_il_level.resize(il.size()); H.h_il_tgt.resize(il.size());
    H.h_il_slevel.resize(il.size()); H.h_il_src.resize(il.size());
    for (size_t q = 0; q < il.size(); ++q) {
        H.h_il_level[q] = il[q].la; H.h_il_tgt[q] = il[q].a;
        H.h_il_slevel[q] = il[q].lb; H.h_il_src[q] = il[q].b;
    }
    adaptive_index(H, s);
}

void adaptive_index(Handle& H, hipStream_t s)
{
    // per-level CSR of the blocks by target box (absolute block index)
    for (int l = 0; l <= H.kappa; ++l) H.lev[l].h_il_ptr.assign(H.lev[l].nbox + 1, 0);
    for (int64_t b = 0; b < H.n_il; ++b) H.lev[H.h_il_level[b]].h_il_ptr[H.h_il_tgt[b] + 1]++;
    int64_t run = 0;
    for (int l = 0; l <= H.kappa; ++l) {
        Level& L = H.lev[l];
        L.h_il_ptr[0] = (int32_t)run;
        for (int64_t x = 0; x < L.nbox; ++x) L.h_il_ptr[x + 1] += L.h_il_ptr[x];
        run = L.h_il_ptr[L.nbox];
        upload(L.il_ptr, L.h_il_ptr, s);
    }
    upload(H.near_ptr, H.h_near_ptr, s);
    upload(H.leaf_level, H.h_leaf_level, s);
    upload(H.leaf_box, H.h_leaf_box, s);
}

void build_tree_and_lists(Handle& H, hipStream_t s)
{
    const int32_t n = (int32_t)H.n;
    const int T = 256;
    const int G = (n + T - 1) / T;
    // box B
    DBuf<unsigned long long> mx;
    DBuf<int> bad;
    mx.alloc(1);
    bad.alloc(1);
    HIPCK(hipMemsetAsync(mx.p, 0, sizeof(unsigned long long), s));
    HIPCK(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    k_maxabs<<<std::min(G, 1024), 256, 0, s>>>(H.xy.p, 2 * H.n, mx.p, bad.p);
    unsigned long long mbits = 0;
    int hbad = 0;
    HIPCK(hipMemcpyAsync(&mbits, mx.p, sizeof(mbits), hipMemcpyDeviceToHost, s));
    HIPCK(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    if (hbad) fail(H2D_EINVAL, "non-finite point coordinate");
    double m;
    std::memcpy(&m, &mbits, sizeof(m));
    double R = 1.0;
    if (m > 0.0) {
        while (R < m) R *= 2.0;
        while (R * 0.5 >= m) R *= 0.5;
    }
    H.R = R;
    // keys at depth 16, sort #1 by the full key to find kappa
    DBuf<uint32_t> key16, skey;
    DBuf<int32_t> idx, sidx;
    key16.alloc(n); idx.alloc(n); skey.alloc(n); sidx.alloc(n);
    k_keys<<<G, T, 0, s>>>(H.xy.p, n, std::ldexp(1.0, 15) / R, key16.p, idx.p);
    HIPCK(hipMemcpyAsync(skey.p, key16.p, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    HIPCK(hipMemcpyAsync(sidx.p, idx.p, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    radix_sort(skey, sidx, n, 32, s);
    if (H.adaptive) {
        adaptive_tree_and_lists(H, skey, sidx, s);
        return;
    }
    DBuf<int32_t> maxrun;
    maxrun.alloc(kMaxLevel + 1);
    HIPCK(hipMemsetAsync(maxrun.p, 0, sizeof(int32_t) * (kMaxLevel + 1), s));
    k_maxrun<<<G, T, 0, s>>>(skey.p, n, maxrun.p);
    HIPCK(hipGetLastError());
    auto hmax = to_host(maxrun.p, kMaxLevel + 1, s);
    hmax[0] = n;
    int kappa = -1;
    for (int l = 0; l <= kMaxLevel; ++l)
        if (hmax[l] <= H.leaf_max) { kappa = l; break; }
    if (kappa < 0) fail(H2D_EDEPTH, "more than leaf_max points share a depth-16 box");
    H.kappa = kappa;
    // sort #2: stable by leaf key from caller order -> perm
    DBuf<uint32_t> lkey;
    lkey.alloc(n);
    k_leafkey<<<G, T, 0, s>>>(key16.p, n, 2 * (kMaxLevel - kappa), lkey.p);
    radix_sort(lkey, idx, n, 2 * kappa, s);
    H.perm = std::move(idx);
    H.xyt.alloc((size_t)2 * n);
    k_gather_xy<<<G, T, 0, s>>>(H.xy.p, H.perm.p, n, H.xyt.p);
    H.h_perm = to_host(H.perm.p, n, s);
    // level tables
    DBuf<int32_t> flag, ex;
    flag.alloc(n); ex.alloc(n);
    for (int l = 0; l <= kappa; ++l) {
        Level& L = H.lev[l];
        int sh = 2 * (kappa - l);
        k_box_flags<<<G, T, 0, s>>>(lkey.p, n, sh, flag.p);
        int64_t nb = scan_excl(flag.p, ex.p, n, s);
        L.nbox = nb;
        L.key.alloc(nb); L.begin.alloc(nb); L.count.alloc(nb); L.parent.alloc(nb);
        k_box_fill<<<G, T, 0, s>>>(lkey.p, n, sh, flag.p, ex.p, L.key.p, L.begin.p);
        int gb = (int)((nb + T - 1) / T);
        k_box_count<<<gb, T, 0, s>>>(L.begin.p, (int32_t)nb, n, L.count.p);
        if (l > 0)
            k_box_parent<<<gb, T, 0, s>>>(L.key.p, (int32_t)nb, H.lev[l - 1].key.p, (int32_t)H.lev[l - 1].nbox,
                                          L.parent.p);
        else
            HIPCK(hipMemsetAsync(L.parent.p, 0xff, sizeof(int32_t) * nb, s));
        HIPCK(hipGetLastError());
        L.h_key = to_host(L.key.p, nb, s);
        L.h_begin = to_host(L.begin.p, nb, s);
        L.h_count = to_host(L.count.p, nb, s);
        L.h_parent = to_host(L.parent.p, nb, s);
    }
    // duplicates make log and 1/r singular
    if (H.kern.kind == H2D_K_LOG || H.kern.kind == H2D_K_INVR) {
        Level& LL = H.lev[kappa];
        HIPCK(hipMemsetAsync(bad.p, 0, sizeof(int), s));
        k_dups<<<(unsigned)LL.nbox, 256, 0, s>>>(H.xyt.p, LL.begin.p, LL.count.p, (int32_t)LL.nbox, bad.p);
        HIPCK(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        if (hbad) fail(H2D_EDUP, "two distinct points coincide; the kernel is singular at r = 0");
    }
    // near lists at the leaf level
    {
        Level& LL = H.lev[kappa];
        int32_t nb = (int32_t)LL.nbox;
        int gb = (nb + T - 1) / T;
        DBuf<int32_t> cnt, ptr, src;
        cnt.alloc(nb); ptr.alloc(nb + 1);
        k_near<<<gb, T, 0, s>>>(LL.key.p, nb, kappa, cnt.p, nullptr, nullptr);
        int64_t tot = scan_excl(cnt.p, ptr.p, nb, s);
        src.alloc(tot);
        k_near<<<gb, T, 0, s>>>(LL.key.p, nb, kappa, cnt.p, ptr.p, src.p);
        HIPCK(hipGetLastError());
        H.h_near_ptr = to_host(ptr.p, nb, s);
        H.h_near_ptr.push_back((int32_t)tot);
        H.h_near_src = to_host(src.p, tot, s);
    }
    // interaction lists per level, concatenated in (level, target, source) order
    H.h_il_level.clear(); H.h_il_tgt.clear(); H.h_il_src.clear();
    H.lev[0].h_il_ptr.assign(H.lev[0].nbox + 1, 0);
    for (int l = 1; l <= kappa; ++l) {
        Level& L = H.lev[l];
        int32_t nb = (int32_t)L.nbox;
        int gb = (nb + T - 1) / T;
        DBuf<int32_t> cnt, ptr, src;
        cnt.alloc(nb); ptr.alloc(nb + 1);
        k_il<<<gb, T, 0, s>>>(L.key.p, nb, l, cnt.p, nullptr, nullptr);
        int64_t tot = scan_excl(cnt.p, ptr.p, nb, s);
        src.alloc(tot);
        k_il<<<gb, T, 0, s>>>(L.key.p, nb, l, cnt.p, ptr.p, src.p);
        HIPCK(hipGetLastError());
        auto hp = to_host(ptr.p, nb, s);
        auto hs = to_host(src.p, tot, s);
        int64_t base = (int64_t)H.h_il_tgt.size();
        L.h_il_ptr.resize(nb + 1);
        for (int32_t b = 0; b < nb; ++b) {
            L.h_il_ptr[b] = (int32_t)(base + hp[b]);
            int32_t e = (b + 1 < nb) ? hp[b + 1] : (int32_t)tot;
            for (int32_t q = hp[b]; q < e; ++q) {
                H.h_il_level.push_back(l);
                H.h_il_tgt.push_back(b);
                H.h_il_src.push_back(hs[q]);
            }
        }
        L.h_il_ptr[nb] = (int32_t)(base + tot);
    }
    H.n_il = (int64_t)H.h_il_tgt.size();
}

// ---------------------------------------------------------------------
// Adaptive cross approximation, one workgroup per block
// ---------------------------------------------------------------------
constexpr int kAcaThreads = 256;
static_assert(kAcaThreads == 4 * kWave, "the ACA cross-term sums combine exactly 4 waves");

struct AcaJob {
    int32_t row0, m, col0, n;
    int32_t kcap, pad;
    int64_t uoff, voff, foff;   // scratch: U (m x kcap col-major), V (n x kcap col-major), flags (m + n bytes)
};

struct ArgMax { double v; int32_t i; };

// larger |value| wins; equal values: lower index wins
__device__ __forceinline__ ArgMax better(ArgMax a, ArgMax b)
{
    if (b.v > a.v || (b.v == a.v && b.i >= 0 && (a.i < 0 || b.i < a.i))) return b;
    return a;
}

__device__ ArgMax block_argmax(ArgMax a, double* lv, int32_t* li)
{
    int t = threadIdx.x;
    lv[t] = a.v; li[t] = a.i;
    __syncthreads();
    for (int d = kAcaThreads / 2; d > 0; d >>= 1) {
        if (t < d) {
            ArgMax x{lv[t], li[t]}, y{lv[t + d], li[t + d]};
            ArgMax z = better(x, y);
            lv[t] = z.v; li[t] = z.i;
        }
        __syncthreads();
    }
    ArgMax r{lv[0], li[0]};
    __syncthreads();
    return r;
}

__device__ double block_sum(double v, double* lv)
{
    int t = threadIdx.x;
    lv[t] = v;
    __syncthreads();
    for (int d = kAcaThreads / 2; d > 0; d >>= 1) {
        if (t < d) lv[t] += lv[t + d];
        __syncthreads();
    }
    double r = lv[0];
    __syncthreads();
    return r;
}

// Largest value over the workgroup (fixed order).
__device__ double block_sum_max(double v, double* lv)
{
    int t = threadIdx.x;
    lv[t] = v;
    __syncthreads();
    for (int d = kAcaThreads / 2; d > 0; d >>= 1) {
        if (t < d) lv[t] = fmax(lv[t], lv[t + d]);
        __syncthreads();
    }
    double r = lv[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Partial-pivot ACA of K(tree rows row0.., tree cols col0..).  Each step:
// residual row at pivot row i -> pivot column j* (largest |r|, lowest index
// on ties, among unused columns) -> v = r / r_j* -> residual column u at
// j* -> update |S|_F^2 -> stop when |u||v| <= tol |S|_F.  The next pivot row
// is the unused row with the largest |u|.  A zero residual row is skipped.
// The block is stored dense once k (m + n) >= m n (smaller and exact).
// kind_out: 0 low rank, 1 dense, -1 rank cap reached.
__global__ void __launch_bounds__(kAcaThreads)
k_aca(const AcaJob* jobs, const double* xyt, KernelParams kp, double tol, double* Uw, double* Vw, uint8_t* flags,
      int32_t* kind_out, int32_t* rank_out)
{
    __shared__ double lv[kAcaThreads];
    __shared__ int32_t li[kAcaThreads];
    __shared__ double row[kAcaRankCap];    // U(i, :) or V(j*, :)
    __shared__ double ab[2][kAcaRankCap];  // cross-term dot products
    __shared__ double cw[kAcaThreads / kWave][16];   // per-wave partial cross terms
    const AcaJob J = jobs[blockIdx.x];
    const int t = threadIdx.x, wave = t / kWave, lane = t % kWave;
    const int32_t m = J.m, n = J.n, kcap = J.kcap;
    double* U = Uw + J.uoff;
    double* V = Vw + J.voff;
    uint8_t* usedR = flags + J.foff;
    uint8_t* usedC = usedR + m;
    const double* P = xyt;
    for (int32_t e = t; e < m + n; e += kAcaThreads) usedR[e] = 0;
    __syncthreads();
    if (kp.kind == H2D_K_GAUSS && m > 0 && n > 0) {
        // Rows of a Gaussian block that are exactly zero: exp(-(r / c)^2)
        // is +0 in FP64 once (r / c)^2 > 746, so a row whose point lies
        // farther than c sqrt(760) from the bounding rectangle of the
        // column points has no nonzero entry.  Marking such rows used up
        // front gives the same pivots and crosses as meeting them one by
        // one (a zero residual row is only ever marked used and passed
        // over), without evaluating them.
        double bx0 = 1e300, by0 = 1e300, bx1 = -1e300, by1 = -1e300;
        for (int32_t j = t; j < n; j += kAcaThreads) {
            const double x = P[2 * (J.col0 + j)], y = P[2 * (J.col0 + j) + 1];
            bx0 = fmin(bx0, x); bx1 = fmax(bx1, x); by0 = fmin(by0, y); by1 = fmax(by1, y);
        }
        bx0 = -block_sum_max(-bx0, lv); bx1 = block_sum_max(bx1, lv);
        by0 = -block_sum_max(-by0, lv); by1 = block_sum_max(by1, lv);
        const double lim = 760.0 * kp.c * kp.c;
        for (int32_t ii = t; ii < m; ii += kAcaThreads) {
            const double px = P[2 * (J.row0 + ii)], py = P[2 * (J.row0 + ii) + 1];
            const double dx = fmax(0.0, fmax(bx0 - px, px - bx1)), dy = fmax(0.0, fmax(by0 - py, py - by1));
            if (dx * dx + dy * dy > lim) usedR[ii] = 1;
        }
        __syncthreads();
    }
    __shared__ int32_t first_nz;
    int32_t k = 0, i = 0, nusedR = 0, kind = kLowRank;
    double S2 = 0.0;
    if (m == 0 || n == 0) { if (t == 0) { kind_out[blockIdx.x] = kLowRank; rank_out[blockIdx.x] = 0; } return; }
    {
        // Before the first cross the residual row is the kernel row itself,
        // and every zero row would be tried, marked used and passed over in
        // index order.  Find the first row with a nonzero entry with the whole
        // workgroup, chunks of rows at a time, and mark the rows before it
        // used: the same pivot and the same used set, without one pass and
        // two reductions per zero row (blocks of a fast-decaying kernel can
        // be exactly zero).
        const int32_t per = max(1, min(64, 16384 / n));
        int32_t found = -1;
        for (int32_t r0 = 0; r0 < m && found < 0; r0 += per) {
            const int32_t nr = min(per, m - r0);
            if (t == 0) first_nz = INT32_MAX;
            __syncthreads();
            for (int64_t e = t; e < (int64_t)nr * n; e += kAcaThreads) {
                const int32_t ii = r0 + (int32_t)(e / n), j = (int32_t)(e % n);
                if (usedR[ii]) continue;   // known zero row
                const double v = kernel_entry(kp, P[2 * (J.row0 + ii)], P[2 * (J.row0 + ii) + 1], P[2 * (J.col0 + j)],
                                              P[2 * (J.col0 + j) + 1], J.row0 + ii == J.col0 + j);
                if (v != 0.0) atomicMin(&first_nz, ii);
            }
            __syncthreads();
            if (first_nz != INT32_MAX) found = first_nz;
            __syncthreads();
        }
        const int32_t stop = found >= 0 ? found : m;
        for (int32_t ii = t; ii < stop; ii += kAcaThreads) usedR[ii] = 1;
        __syncthreads();
        if (found < 0) {   // the block is exactly zero: rank 0
            if (t == 0) { kind_out[blockIdx.x] = kLowRank; rank_out[blockIdx.x] = 0; }
            return;
        }
        i = found;
    }
    for (;;) {
        // U(i, 0..k)
        for (int q = t; q < k; q += kAcaThreads) row[q] = U[(int64_t)q * m + i];
        if (t == 0 && !usedR[i]) usedR[i] = 1;
        __syncthreads();
        nusedR = 0;   // recount below only when needed
        const double tx = P[2 * (J.row0 + i)], ty = P[2 * (J.row0 + i) + 1];
        double* r = V + (int64_t)k * n;   // residual row stored in column k of V
        ArgMax best{-1.0, -1};
        for (int32_t j = t; j < n; j += kAcaThreads) {
            double s = kernel_entry(kp, tx, ty, P[2 * (J.col0 + j)], P[2 * (J.col0 + j) + 1],
                                    J.row0 + i == J.col0 + j);
            for (int q = 0; q < k; ++q) s -= row[q] * V[(int64_t)q * n + j];
            r[j] = s;
            if (!usedC[j]) best = better(best, ArgMax{fabs(s), j});
        }
        best = block_argmax(best, lv, li);
        const int32_t js = best.i;
        if (js < 0) break;
        const double delta = r[js];   // written by the thread owning js; visible after the barrier above
        if (delta == 0.0) {
            // zero residual row: mark it used and move to the lowest unused row
            ArgMax nxt{-1.0, -1};
            for (int32_t ii = t; ii < m; ii += kAcaThreads)
                if (!usedR[ii]) nxt = better(nxt, ArgMax{0.0, ii});
            nxt = block_argmax(nxt, lv, li);
            if (nxt.i < 0) break;
            i = nxt.i;
            continue;
        }
        for (int32_t j = t; j < n; j += kAcaThreads) r[j] = r[j] / delta;
        for (int q = t; q < k; q += kAcaThreads) row[q] = V[(int64_t)q * n + js];
        __syncthreads();
        double* u = U + (int64_t)k * m;
        const double sx = P[2 * (J.col0 + js)], sy = P[2 * (J.col0 + js) + 1];
        double uu = 0.0, vv = 0.0;
        for (int32_t ii = t; ii < m; ii += kAcaThreads) {
            double s = kernel_entry(kp, P[2 * (J.row0 + ii)], P[2 * (J.row0 + ii) + 1], sx, sy,
                                    J.row0 + ii == J.col0 + js);
            for (int q = 0; q < k; ++q) s -= U[(int64_t)q * m + ii] * row[q];
            u[ii] = s;
            uu += s * s;
        }
        for (int32_t j = t; j < n; j += kAcaThreads) vv += r[j] * r[j];
        if (t == 0) usedC[js] = 1;
        __syncthreads();
        uu = block_sum(uu, lv);
        vv = block_sum(vv, lv);
        // cross terms (U(:, q) . u) (V(:, q) . v) for q < k: every thread
        // takes rows t, t + 256, ... for 8 columns q at a time (8 loads in
        // flight; columns past k - 1 re-read column k - 1 and are dropped),
        // then shuffle sums per wave and a fixed-order sum of the 4 waves
        for (int q0 = 0; q0 < k; q0 += 8) {
            double pa[8], pb[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) { pa[c] = 0.0; pb[c] = 0.0; }
            for (int32_t ii = t; ii < m; ii += kAcaThreads) {
                const double ui = u[ii];
#pragma unroll
                for (int c = 0; c < 8; ++c) pa[c] += U[(int64_t)min(q0 + c, k - 1) * m + ii] * ui;
            }
            for (int32_t j = t; j < n; j += kAcaThreads) {
                const double vj = r[j];
#pragma unroll
                for (int c = 0; c < 8; ++c) pb[c] += V[(int64_t)min(q0 + c, k - 1) * n + j] * vj;
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                pa[c] = wave_sum(pa[c]);
                pb[c] = wave_sum(pb[c]);
            }
            if (lane == 0)
#pragma unroll
                for (int c = 0; c < 8; ++c) { cw[wave][c] = pa[c]; cw[wave][8 + c] = pb[c]; }
            __syncthreads();
            if (t < 16) {
                const double sum = (cw[0][t] + cw[1][t]) + (cw[2][t] + cw[3][t]);
                const int q = q0 + (t & 7);
                if (q < k) ab[t >> 3][q] = sum;
            }
            __syncthreads();
        }
        __syncthreads();
        double cross = 0.0;
        for (int q = 0; q < k; ++q) cross += ab[0][q] * ab[1][q];
        S2 += 2.0 * cross + uu * vv;
        ++k;
        if ((int64_t)k * (m + n) >= (int64_t)m * n) { kind = kDense; break; }
        if (sqrt(uu) * sqrt(vv) <= tol * sqrt(S2)) break;
        if (k >= kcap) { kind = -1; break; }
        ArgMax nxt{-1.0, -1};
        for (int32_t ii = t; ii < m; ii += kAcaThreads)
            if (!usedR[ii]) nxt = better(nxt, ArgMax{fabs(u[ii]), ii});
        nxt = block_argmax(nxt, lv, li);
        if (nxt.i < 0) break;
        i = nxt.i;
    }
    (void)nusedR;
    if (t == 0) { kind_out[blockIdx.x] = kind; rank_out[blockIdx.x] = k; }
}

// Copy converged factors out of the scratch: U (m x k col-major) as is,
// V transposed to row-major n x k.
// U of a block above the leaf level is stored tiled by the boxes one level
// above the leaves (the matvec's row tiles): for each such sub-box P of the
// target, in tree order, the |P| x k column-major tile U(rows of P, :).
// Element (i, q) sits at k (begin_P - row0) + q |P| + (i - (begin_P - row0)).
// tbeg / tcnt give begin_P and |P| for every tree row (null: untiled).
// V is stored row-major (n x k), except on symmetric handles (vcm), where it
// is laid out as U is, by the source box's rows starting at col0.
struct PackJob {
    int64_t su, sv;     // scratch offsets
    int64_t du, dv;     // destination offsets
    int32_t m, n, k, tiled;
    int32_t row0, col0, vcm, pad;
};

__global__ void k_pack(const PackJob* jobs, const double* Uw, const double* Vw, double* Uo, double* Vo,
                       const int32_t* tbeg, const int32_t* tcnt)
{
    const PackJob J = jobs[blockIdx.x];
    for (int64_t e = threadIdx.x; e < (int64_t)J.m * J.k; e += blockDim.x) {
        int64_t dst = e;
        if (J.tiled) {
            const int64_t q = e / J.m, i = e % J.m, gi = J.row0 + i;
            const int64_t pb = tbeg[gi] - J.row0, pc = tcnt[gi];
            dst = (int64_t)J.k * pb + q * pc + (i - pb);
        }
        Uo[J.du + dst] = Uw[J.su + e];
    }
    for (int64_t e = threadIdx.x; e < (int64_t)J.n * J.k; e += blockDim.x) {
        if (J.vcm) {
            int64_t dst = e;
            if (J.tiled) {
                const int64_t q = e / J.n, j = e % J.n, gj = J.col0 + j;
                const int64_t pb = tbeg[gj] - J.col0, pc = tcnt[gj];
                dst = (int64_t)J.k * pb + q * pc + (j - pb);
            }
            Vo[J.dv + dst] = Vw[J.sv + e];
        } else {
            int64_t j = e / J.k, q = e % J.k;
            Vo[J.dv + e] = Vw[J.sv + q * J.n + j];
        }
    }
}

// Dense blocks: D (m x n column-major) = K(rows, cols) with the diagonal
// rule where the tree indices coincide.
struct DenseJob {
    int64_t off;
    int32_t row0, m, col0, n;
};

__global__ void k_dense(const DenseJob* jobs, const double* xyt, KernelParams kp, double* D)
{
    const DenseJob J = jobs[blockIdx.x];
    for (int64_t e = threadIdx.x; e < (int64_t)J.m * J.n; e += blockDim.x) {
        int32_t j = (int32_t)(e / J.m), i = (int32_t)(e % J.m);
        D[J.off + e] = kernel_entry(kp, xyt[2 * (J.row0 + i)], xyt[2 * (J.row0 + i) + 1], xyt[2 * (J.col0 + j)],
                                    xyt[2 * (J.col0 + j) + 1], J.row0 + i == J.col0 + j);
    }
}

void build_factors(Handle& H, hipStream_t s)
{
    const int kappa = H.kappa;
    const int64_t nil = H.n_il;
    const bool sym = H.symmetric;
    if (sym) symmetric_partners(H);
    H.h_il_kind.assign(nil, kLowRank);
    H.h_il_k.assign(nil, 0);
    // blocks compressed here: all, or on a symmetric handle the owners
    // (target index below source index); mirrors take their owner's factors
    std::vector<int64_t> todo;
    todo.reserve(nil);
    for (int64_t b = 0; b < nil; ++b)
        if (!sym || H.h_il_tgt[b] < H.h_il_src[b]) todo.push_back(b);
    const int64_t ntodo = (int64_t)todo.size();
    std::vector<int32_t> m(nil), n(nil), r0(nil), c0(nil);
    for (int64_t b = 0; b < nil; ++b) {
        const Level& L = H.lev[H.h_il_level[b]];
        const Level& Ls = H.lev[il_src_level(H, b)];
        m[b] = L.h_count[H.h_il_tgt[b]];
        n[b] = Ls.h_count[H.h_il_src[b]];
        r0[b] = L.h_begin[H.h_il_tgt[b]];
        c0[b] = Ls.h_begin[H.h_il_src[b]];
    }
    // row -> (begin, size) of its box one level above the leaves
    DBuf<int32_t> tbeg, tcnt;
    {
        std::vector<int32_t> hb(H.n, 0), hc(H.n, 0);
        if (kappa >= 1) {
            const Level& T = H.lev[kappa - 1];
            for (int64_t p = 0; p < T.nbox; ++p)
                for (int32_t i = T.h_begin[p]; i < T.h_begin[p] + T.h_count[p]; ++i) { hb[i] = T.h_begin[p]; hc[i] = T.h_count[p]; }
        }
        upload(tbeg, hb, s);
        upload(tcnt, hc, s);
    }
    // scratch budget per ACA chunk
    size_t freeb = 0, totalb = 0;
    HIPCK(hipMemGetInfo(&freeb, &totalb));
    const double budget = std::max(1.0e9, std::min(16.0e9, 0.25 * (double)freeb));
    struct Chunk { int64_t b0, b1; DBuf<double> U, V; int64_t ue = 0, ve = 0; };
    std::vector<Chunk> chunks;
    int64_t b = 0;
    while (b < ntodo) {
        std::vector<AcaJob> jobs;
        int64_t uo = 0, vo = 0, fo = 0;
        double bytes = 0;
        int64_t b1 = b;
        while (b1 < ntodo) {
            const int64_t bb = todo[b1];
            int64_t mm = m[bb], nn = n[bb];
            int64_t kc = (mm * nn + mm + nn - 1) / (mm + nn);
            kc = std::min<int64_t>(kc, kAcaRankCap);
            double need = 8.0 * (double)(mm + nn) * (double)kc + (double)(mm + nn);
            if (b1 > b && (bytes + need > budget || jobs.size() >= 200000)) break;
            AcaJob J{r0[bb], m[bb], c0[bb], n[bb], (int32_t)kc, 0, uo, vo, fo};
            jobs.push_back(J);
            uo += mm * kc; vo += nn * kc; fo += mm + nn;
            bytes += need;
            ++b1;
        }
        DBuf<AcaJob> djobs;
        DBuf<double> Uw, Vw;
        DBuf<uint8_t> fl;
        DBuf<int32_t> kind, rank;
        upload(djobs, jobs, s);
        Uw.alloc(std::max<int64_t>(uo, 1)); Vw.alloc(std::max<int64_t>(vo, 1)); fl.alloc(std::max<int64_t>(fo, 1));
        kind.alloc(jobs.size()); rank.alloc(jobs.size());
        KernelParams kp = H.kern;
        k_aca<<<(unsigned)jobs.size(), kAcaThreads, 0, s>>>(djobs.p, H.xyt.p, kp, H.tol, Uw.p, Vw.p, fl.p, kind.p,
                                                              rank.p);
        HIPCK(hipGetLastError());
        auto hk = to_host(kind.p, jobs.size(), s);
        auto hr = to_host(rank.p, jobs.size(), s);
        Chunk C;
        C.b0 = b; C.b1 = b1;
        std::vector<PackJob> packs;
        for (size_t q = 0; q < jobs.size(); ++q) {
            const int64_t bb = todo[b + (int64_t)q];
            if (hk[q] < 0)
                fail(H2D_ENOCONV, "ACA reached its rank cap of " + std::to_string(kAcaRankCap) + " on a " +
                                      std::to_string(m[bb]) + " x " + std::to_string(n[bb]) + " block");
            H.h_il_kind[bb] = hk[q];
            H.h_il_k[bb] = hr[q];
            if (hk[q] == kLowRank && hr[q] > 0) {
                // U tiled by the boxes one level above the leaves (balanced
                // trees); plain column-major on an adaptive tree
                const int32_t tiled = (!H.adaptive && H.h_il_level[bb] <= kappa - 1) ? 1 : 0;
                if (sym) {   // both factors in the U pool: F_X, then F_Y
                    packs.push_back(PackJob{jobs[q].uoff, jobs[q].voff, C.ue, C.ue + (int64_t)m[bb] * hr[q], m[bb], n[bb],
                                            hr[q], tiled, r0[bb], c0[bb], 1, 0});
                    C.ue += (int64_t)(m[bb] + n[bb]) * hr[q];
                } else {
                    packs.push_back(PackJob{jobs[q].uoff, jobs[q].voff, C.ue, C.ve, m[bb], n[bb], hr[q], tiled, r0[bb], 0,
                                            0, 0});
                    C.ue += (int64_t)m[bb] * hr[q];
                    C.ve += (int64_t)n[bb] * hr[q];
                }
            }
        }
        C.U.alloc(std::max<int64_t>(C.ue, 1));
        C.V.alloc(std::max<int64_t>(C.ve, 1));
        if (!packs.empty()) {
            DBuf<PackJob> dp;
            upload(dp, packs, s);
            k_pack<<<(unsigned)packs.size(), 256, 0, s>>>(dp.p, Uw.p, Vw.p, C.U.p, sym ? C.U.p : C.V.p, tbeg.p,
                                                           tcnt.p);
            HIPCK(hipGetLastError());
            HIPCK(hipStreamSynchronize(s));
        }
        chunks.push_back(std::move(C));
        b = b1;
    }
    // final pools: U, V for low-rank blocks in table order; D for near
    // blocks (leaf order) then dense IL blocks
    H.h_il_off.assign(nil, 0);
    H.h_il_voff.assign(nil, 0);
    int64_t ue = 0, ve = 0, de = 0;
    const Level& LL = H.lev[kappa];
    int64_t nnear = (int64_t)H.h_near_src.size();
    H.h_near_off.assign(nnear, 0);
    std::vector<DenseJob> dj;
    if (sym) {
        // mirrors take the owner's kind and rank
        for (int64_t q = 0; q < nil; ++q)
            if (H.h_il_tgt[q] > H.h_il_src[q]) {
                H.h_il_kind[q] = H.h_il_kind[H.h_il_partner[q]];
                H.h_il_k[q] = H.h_il_k[H.h_il_partner[q]];
            }
    }
    if (sym) {   // self and owner near blocks stored; a mirror shares its owner's (transposed)
        for (int64_t x = 0; x < LL.nbox; ++x)
            for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
                const int32_t y = H.h_near_src[q];
                if (y < x) {
                    int32_t o = H.h_near_ptr[y];
                    while (H.h_near_src[o] != x) ++o;
                    H.h_near_off[q] = H.h_near_off[o];
                    continue;
                }
                H.h_near_off[q] = de;
                dj.push_back(DenseJob{de, LL.h_begin[x], LL.h_count[x], LL.h_begin[y], LL.h_count[y]});
                de += (int64_t)LL.h_count[x] * LL.h_count[y];
            }
    } else if (H.adaptive) {   // near CSR over leaf numbers
        const int64_t nleaf = (int64_t)H.h_leaf_begin.size();
        for (int64_t x = 0; x < nleaf; ++x)
            for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
                const int32_t y = H.h_near_src[q];
                H.h_near_off[q] = de;
                dj.push_back(DenseJob{de, H.h_leaf_begin[x], H.h_leaf_count[x], H.h_leaf_begin[y], H.h_leaf_count[y]});
                de += (int64_t)H.h_leaf_count[x] * H.h_leaf_count[y];
            }
    } else {
        for (int64_t x = 0; x < LL.nbox; ++x)
            for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
                int32_t y = H.h_near_src[q];
                H.h_near_off[q] = de;
                dj.push_back(DenseJob{de, LL.h_begin[x], LL.h_count[x], LL.h_begin[y], LL.h_count[y]});
                de += (int64_t)LL.h_count[x] * LL.h_count[y];
            }
    }
    for (int64_t q = 0; q < nil; ++q) {
        const bool mirror = sym && H.h_il_tgt[q] > H.h_il_src[q];
        if (mirror) {
            const int64_t o = H.h_il_partner[q];   // earlier in table order
            if (H.h_il_kind[q] == kDense) {
                H.h_il_off[q] = H.h_il_off[o];
            } else {
                H.h_il_off[q] = H.h_il_voff[o];
                H.h_il_voff[q] = H.h_il_off[o];
            }
            continue;
        }
        if (H.h_il_kind[q] == kDense) {
            H.h_il_off[q] = de;
            dj.push_back(DenseJob{de, r0[q], m[q], c0[q], n[q]});
            de += (int64_t)m[q] * n[q];
        } else if (sym) {
            H.h_il_off[q] = ue;
            ue += (int64_t)m[q] * H.h_il_k[q];
            H.h_il_voff[q] = ue;
            ue += (int64_t)n[q] * H.h_il_k[q];
        } else {
            H.h_il_off[q] = ue;
            H.h_il_voff[q] = ve;
            ue += (int64_t)m[q] * H.h_il_k[q];
            ve += (int64_t)n[q] * H.h_il_k[q];
        }
    }
    H.u_elems = ue; H.v_elems = ve; H.d_elems = de;
    H.U64.alloc(std::max<int64_t>(ue, 1));
    H.V64.alloc(std::max<int64_t>(ve, 1));
    H.D64.alloc(std::max<int64_t>(de, 1));
    int64_t uu = 0, vv = 0;
    for (auto& C : chunks) {
        if (C.ue) HIPCK(hipMemcpyAsync(H.U64.p + uu, C.U.p, sizeof(double) * C.ue, hipMemcpyDeviceToDevice, s));
        if (C.ve) HIPCK(hipMemcpyAsync(H.V64.p + vv, C.V.p, sizeof(double) * C.ve, hipMemcpyDeviceToDevice, s));
        uu += C.ue; vv += C.ve;
    }
    if (!dj.empty()) {
        DBuf<DenseJob> d;
        upload(d, dj, s);
        for (size_t o = 0; o < dj.size(); o += 1u << 20) {
            unsigned cnt = (unsigned)std::min<size_t>(1u << 20, dj.size() - o);
            k_dense<<<cnt, 256, 0, s>>>(d.p + o, H.xyt.p, H.kern, H.D64.p);
        }
        HIPCK(hipGetLastError());
    }
    HIPCK(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------
// Half-precision copies: per-block power-of-two scale so that FP16 cannot
// overflow; V (|v| <= 1 by construction) is stored unscaled; the diagonal
// of the self blocks is held apart in FP32 (the log kernel's diagonal N can
// exceed the FP16 range).
// ---------------------------------------------------------------------
// U and D tiles of the half pools are stored in a quad layout: a tile (the
// U of a block above the leaf level is tiled by the boxes one level above
// the leaves, as in the FP64 pool; any other block is one tile) is laid out
// as [column quads][rows][4], so the 4 values of one row in 4 consecutive
// columns form one aligned 8-byte group; the columns are padded with zeros
// to a multiple of 4, and the rows of the tiles above the leaf level to a
// multiple of 16 (so each of their column quads starts on a 128-byte line
// and a 64-row slice of one quad is four whole lines; the leaf-level tiles
// are read whole, where padding would only leave partly used lines).  Element (i, c) of a tile of p rows (p16 with the padding) sits
// at (floor(c / 4) p16 + i) 4 + c mod 4; the tiles of a k-column block
// follow one another, each k4 p16 values (k4 = k rounded up to 4).
struct HalfJob {
    int64_t src, dst;     // FP64 offset, half offset (a multiple of 64)
    int32_t m, n;         // rows, columns (the rank for U)
    int32_t tiled, self;  // U tiled as above; 1 if a self block
    int32_t row0, m16;    // first tree row of the block; tile rows of an untiled block
};

__host__ __device__ constexpr int32_t pad16(int32_t m) { return (m + 15) & ~15; }

template <typename T>
__device__ __forceinline__ T to_half(float v);
template <>
__device__ __forceinline__ __half to_half<__half>(float v) { return __float2half_rn(v); }
template <>
__device__ __forceinline__ __hip_bfloat16 to_half<__hip_bfloat16>(float v) { return __float2bfloat16(v); }

// tbeg, tcnt: per tree row, the first row and the size of its box one
// level above the leaves; tpad: per tree row, where that box's padded
// tile starts among the padded tiles of all such boxes (in rows).
template <typename T>
__global__ void k_half_q(const HalfJob* jobs, const double* src, T* dst, float* scale, float* diag,
                         const int32_t* tbeg, const int32_t* tcnt, const int64_t* tpad)
{
    __shared__ double lv[256];
    const HalfJob J = jobs[blockIdx.x];
    const int64_t cnt = (int64_t)J.m * J.n;
    double mx = 0.0;
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        bool d = J.self && (e % J.m) == (e / J.m);
        if (!d) mx = fmax(mx, fabs(src[J.src + e]));
    }
    lv[threadIdx.x] = mx;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) lv[threadIdx.x] = fmax(lv[threadIdx.x], lv[threadIdx.x + d]);
        __syncthreads();
    }
    mx = lv[0];
    int ex = 0;
    if (mx > 0.0) frexp(mx, &ex);
    // mx / sc in [0.5, 1).  The scale is stored in FP32: below its smallest
    // subnormal 2^-149 the block's values are not representable in any
    // form here and are stored as zeros (a block whose largest entry is a
    // subnormal double would otherwise give inv = inf and 0 * inf = NaN)
    ex = max(ex, -149);
    const double sc = ldexp(1.0, ex);
    const double inv = 1.0 / sc;
    if (threadIdx.x == 0) scale[blockIdx.x] = (float)sc;
    const int64_t n4 = (J.n + 3) & ~3;
    for (int64_t e = threadIdx.x; e < (int64_t)J.m * n4; e += blockDim.x) {
        const int64_t c = e / J.m, i = e % J.m;
        // the tile holding row i: its first row in the block (pb), rows (pc),
        // padded rows (p16) and start in the block's padded rows (tb)
        int64_t pb = 0, pc = J.m, p16 = J.m16, tb = 0;
        if (J.tiled) {
            pb = tbeg[J.row0 + i] - J.row0;
            pc = tcnt[J.row0 + i];
            p16 = pad16((int32_t)pc);
            tb = tpad[J.row0 + i] - tpad[J.row0];
        }
        const bool d = J.self && i == c;
        double v = 0.0;
        if (c < J.n) v = src[J.src + (J.tiled ? (int64_t)J.n * pb + c * pc + (i - pb) : c * J.m + i)];
        dst[J.dst + n4 * tb + ((c >> 2) * p16 + (i - pb)) * 4 + (c & 3)] = to_half<T>(d ? 0.0f : (float)(v * inv));
        if (d) diag[J.row0 + i] = (float)v;
    }
}

// V of one low-rank block, FP64 row-major n x k at src_off, to its place
// in its source box's wide V: element (j, q) at dst_off + (j / 4) rg + 4 q
// + j mod 4 (rg = 4 x the box's width; the pool is zeroed beforehand,
// which covers the padding rows).
struct HalfVJob {
    int64_t src_off, dst_off;
    int32_t n, k, rg, pad;
};

template <typename T>
__global__ void k_half_v(const HalfVJob* jobs, const double* src, T* dst)
{
    const HalfVJob J = jobs[blockIdx.x];
    for (int64_t e = threadIdx.x; e < (int64_t)J.n * J.k; e += blockDim.x) {
        const int32_t j = (int32_t)(e / J.k), q = (int32_t)(e % J.k);
        dst[J.dst_off + (int64_t)(j >> 2) * J.rg + 4 * q + (j & 3)] = to_half<T>((float)src[J.src_off + e]);
    }
}

// The half V pools grouped by source box: for every source box (per
// level) the V of its low-rank blocks side by side (table order, w
// columns), stored in groups of 4 rows (element (j, c) at ((j / 4) ws + c)
// 4 + j mod 4, ws = w rounded up to 16, rows padded with zeros to a
// multiple of 4).  Sets the phase-A items (at most
// kPhaseARows rows of one source box each, largest first), the column maps
// to the t pool and the reductions of split source boxes; returns the
// conversion jobs.
static std::vector<HalfVJob> wide_v_layout(Handle& H, hipStream_t s)
{
    std::vector<int64_t> order;
    for (int64_t q = 0; q < H.n_il; ++q)
        if (H.h_il_kind[q] != kDense && H.h_il_k[q] > 0) order.push_back(q);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        return H.h_il_level[a] != H.h_il_level[b] ? H.h_il_level[a] < H.h_il_level[b] : H.h_il_src[a] < H.h_il_src[b];
    });
    std::vector<HalfVJob> jobs;
    std::vector<AWDesc> items;
    std::vector<AWRed> red;
    std::vector<int32_t> map;
    int64_t vo = 0, po = 0, t_direct = 0, t_split = 0;
    for (size_t i = 0; i < order.size();) {
        size_t e = i;
        int32_t w = 0;
        while (e < order.size() && H.h_il_level[order[e]] == H.h_il_level[order[i]] &&
               H.h_il_src[order[e]] == H.h_il_src[order[i]])
            w += H.h_il_k[order[e++]];
        const int32_t ws = pad16(w);   // row-group width: every row group starts on a 128-byte line
        const Level& L = H.lev[H.h_il_level[order[i]]];
        const int32_t ny = L.h_count[H.h_il_src[order[i]]], y0 = L.h_begin[H.h_il_src[order[i]]];
        const int32_t mo = (int32_t)map.size();
        int32_t c0 = 0;
        for (size_t b = i; b < e; ++b) {
            const int64_t q = order[b];
            const int32_t k = H.h_il_k[q];
            jobs.push_back(HalfVJob{H.h_il_voff[q], vo + 4 * (int64_t)c0, ny, k, 4 * ws, 0});
            for (int32_t c = 0; c < k; ++c) map.push_back(H.h_il_toff[q] + c);
            c0 += k;
        }
        const int32_t parts = (ny + kPhaseARows - 1) / kPhaseARows;   // kPhaseARows: a multiple of 4
        for (int32_t p = 0; p < parts; ++p) {
            const int32_t j0 = p * kPhaseARows, rows = std::min(kPhaseARows, ny - j0);
            items.push_back(AWDesc{vo + (int64_t)(j0 / 4) * 4 * ws, rows, w, y0 + j0, mo,
                                   parts > 1 ? (int32_t)(po + (int64_t)p * w) : -1, ws});
        }
        if (parts > 1) {
            red.push_back(AWRed{(int32_t)po, parts, w, mo});
            po += (int64_t)parts * w;
            t_split += w;
        } else {
            t_direct += w;
        }
        vo += (int64_t)((ny + 3) / 4) * 4 * ws;
        i = e;
    }
    if (po > INT32_MAX || map.size() > (size_t)INT32_MAX)
        fail(H2D_EUNSUPPORTED, "half-precision phase-A tables above 2^31 entries");
    std::stable_sort(items.begin(), items.end(),
                     [](const AWDesc& a, const AWDesc& b) { return (int64_t)a.rows * a.w > (int64_t)b.rows * b.w; });
    H.v16_elems = vo;
    H.p16_elems = po;
    // algorithmic bytes of the half phase A (V once, x once, t and the
    // partial rows written once) and of its reduction (partial rows read,
    // t written); the library's count for the half product
    H.phase_bytes[1][1] = (double)H.v_elems * 2 + (double)H.n * 4 + (double)t_direct * 4 + (double)po * 4;
    H.phase_bytes[1][2] = po ? (double)po * 4 + (double)t_split * 4 : 0.0;
    H.alg_bytes_half = 0;
    for (int p = 0; p < 5; ++p) H.alg_bytes_half += H.phase_bytes[1][p];
    upload(H.aw_items, items, s);
    upload(H.aw_map, map, s);
    upload(H.aw_red, red, s);
    H.n_aw_items = (int64_t)items.size();
    H.n_aw_red = (int64_t)red.size();
    H.aw_red_maxw = 0;
    for (const AWRed& r : red) H.aw_red_maxw = std::max(H.aw_red_maxw, r.w);
    // the single-RHS reduction launches ceil(w / 64) workgroups per box
    // along y; the 16-RHS one takes a list of 64-value chunks (16 values per
    // column), so that no workgroup is launched empty: the first chunk of
    // every box, then the second, ... (the long reductions of the few wide
    // boxes spread over the launch)
    if ((H.aw_red_maxw + kWave - 1) / kWave > 65535)
        fail(H2D_EUNSUPPORTED, "half-precision phase-A source box wider than 2^22 columns");
    std::vector<int2> chunks;
    int32_t nch = 0;
    for (const AWRed& r : red) nch = std::max(nch, (r.w * 16 + kWave - 1) / kWave);
    for (int32_t c = 0; c < nch; ++c)
        for (size_t r = 0; r < red.size(); ++r)
            if (c * kWave < red[r].w * 16) chunks.push_back(make_int2((int32_t)r, c * kWave));
    if (chunks.size() > (size_t)INT32_MAX) fail(H2D_EUNSUPPORTED, "half-precision reduction list above 2^31 chunks");
    upload(H.aw_rchunks, chunks, s);
    H.n_aw_rchunks = (int64_t)chunks.size();
    H.ws_nrhs = 0;   // the half partial rows are sized here: reallocate on next use
    return jobs;
}

// The phase-B tables of the half pools.  Table 1, per box P one level
// above the leaves: the 4-column groups of P's tile of every block whose
// target is P or one of its ancestors, level by level from P up, blocks in
// table order.  Table 2, per leaf X: its near blocks, then its own
// interaction-list blocks.  A row slice of the box sums its table's groups
// in order.
static void build_quad_tables(Handle& H, const std::vector<int64_t>& near_off16, const std::vector<float>& sc,
                              const std::vector<int64_t>& tpad, hipStream_t s)
{
    const int kappa = H.kappa;
    std::vector<QEnt> t1, t2;
    std::vector<int32_t> p1(1, 0), p2(1, 0);
    // the groups of one tile: row 0 of its slice at e0 (elements), groups qs
    // elements apart, ncols columns whose multiplier values start at src0
    auto put = [&](std::vector<QEnt>& t, int64_t e0, int64_t qs, int32_t ncols, int32_t src0, bool dense, float scale) {
        for (int32_t u = 0; 4 * u < ncols; ++u) {
            const int64_t e = e0 + (int64_t)u * qs;
            t.push_back(QEnt{(uint32_t)(e >> 2), dense ? ~(src0 + 4 * u) : src0 + 4 * u, scale,
                             std::min(4, ncols - 4 * u)});
        }
    };
    auto close = [&](std::vector<int32_t>& p, const std::vector<QEnt>& t) {
        if (t.size() > (size_t)INT32_MAX) fail(H2D_EUNSUPPORTED, "phase-B table above 2^31 entries");
        p.push_back((int32_t)t.size());
    };
    if (kappa >= 2) {
        const Level& T = H.lev[kappa - 1];
        for (int64_t P = 0; P < T.nbox; ++P) {
            const int32_t p0 = T.h_begin[P], cnt = T.h_count[P];
            int32_t a_box = (int32_t)P;
            for (int l = kappa - 1; l >= 1; --l) {
                const Level& L = H.lev[l];
                const int32_t ab = L.h_begin[a_box], ldm = L.h_count[a_box];
                for (int32_t q = L.h_il_ptr[a_box]; q < L.h_il_ptr[a_box + 1]; ++q) {
                    if (H.h_il_kind[q] == kDense) {
                        const int32_t sb = H.h_il_src[q];
                        put(t1, H.h_il_off16[q] + (int64_t)(p0 - ab) * 4, (int64_t)pad16(ldm) * 4, L.h_count[sb],
                            L.h_begin[sb], true, sc[q]);
                    } else if (H.h_il_k[q] > 0) {
                        const int32_t k = H.h_il_k[q];
                        put(t1, H.h_il_off16[q] + (int64_t)((k + 3) & ~3) * (tpad[p0] - tpad[ab]),
                            (int64_t)pad16(cnt) * 4, k, H.h_il_toff[q], false, sc[q]);
                    }
                }
                a_box = L.h_parent[a_box];
            }
            close(p1, t1);
        }
    }
    const Level& LL = H.lev[kappa];
    for (int64_t X = 0; X < LL.nbox; ++X) {
        const int64_t qs = (int64_t)LL.h_count[X] * 4;
        for (int32_t q = H.h_near_ptr[X]; q < H.h_near_ptr[X + 1]; ++q) {
            const int32_t y = H.h_near_src[q];
            put(t2, near_off16[q], qs, LL.h_count[y], LL.h_begin[y], true, sc[H.n_il + q]);
        }
        for (int32_t q = LL.h_il_ptr[X]; q < LL.h_il_ptr[X + 1]; ++q) {
            if (H.h_il_kind[q] == kDense) {
                const int32_t sb = H.h_il_src[q];
                put(t2, H.h_il_off16[q], qs, LL.h_count[sb], LL.h_begin[sb], true, sc[q]);
            } else if (H.h_il_k[q] > 0) {
                put(t2, H.h_il_off16[q], qs, H.h_il_k[q], H.h_il_toff[q], false, sc[q]);
            }
        }
        close(p2, t2);
    }
    upload(H.qp1, p1, s);
    upload(H.qt1, t1, s);
    upload(H.qp2, p2, s);
    upload(H.qt2, t2, s);
}

void make_half_pools(Handle& H, uint32_t mask, hipStream_t s)
{
    const bool f16 = mask & H2D_PREC_BIT(H2D_P_FP16), b16 = mask & H2D_PREC_BIT(H2D_P_BF16);
    if (!f16 && !b16) return;
    const int kappa = H.kappa;
    // jobs: IL blocks (U or D) in table order, then near blocks; each pool
    // gets quad-layout offsets of its own, and the descriptors the half
    // product kernels read
    // tree row -> first row, size and padded-tile start of its box one
    // level above the leaves
    std::vector<int32_t> hb(std::max<int64_t>(H.n, 1), 0), hc(std::max<int64_t>(H.n, 1), 0);
    std::vector<int64_t> hp(std::max<int64_t>(H.n, 1), 0);
    if (kappa >= 1) {
        const Level& T = H.lev[kappa - 1];
        int64_t g = 0;
        for (int64_t p = 0; p < T.nbox; ++p) {
            for (int32_t i = T.h_begin[p]; i < T.h_begin[p] + T.h_count[p]; ++i) {
                hb[i] = T.h_begin[p];
                hc[i] = T.h_count[p];
                hp[i] = g;
            }
            g += pad16(T.h_count[p]);
        }
    }
    // padded rows of a tiled block whose rows are [r0, r0 + m)
    auto tiled_rows = [&](int32_t r0, int32_t m) -> int64_t {
        const int32_t r1 = r0 + m - 1;
        return hp[r1] + pad16(hc[r1]) - hp[r0];
    };
    std::vector<HalfJob> jobs;
    H.h_il_off16.assign(H.n_il, 0);
    int64_t uo = 0, dof = 0;
    for (int64_t q = 0; q < H.n_il; ++q) {
        const Level& L = H.lev[H.h_il_level[q]];
        const int32_t mm = L.h_count[H.h_il_tgt[q]], nn = L.h_count[H.h_il_src[q]];
        const int32_t row0 = L.h_begin[H.h_il_tgt[q]];
        if (H.h_il_kind[q] == kDense) {
            // above the leaf level the tile is read in 64-row slices: rows
            // padded to 16 (at the leaf level it is read whole: packed)
            const int32_t m16 = H.h_il_level[q] < kappa ? pad16(mm) : mm;
            H.h_il_off16[q] = dof;
            jobs.push_back(HalfJob{H.h_il_off[q], dof, mm, nn, 0, 0, row0, m16});
            dof += (int64_t)m16 * ((nn + 3) & ~3);
        } else {
            const int32_t k = H.h_il_k[q];
            const int32_t tiled = H.h_il_level[q] <= kappa - 1 ? 1 : 0;
            H.h_il_off16[q] = uo;
            jobs.push_back(HalfJob{H.h_il_off[q], uo, mm, k, tiled, 0, row0, mm});
            uo += (tiled ? tiled_rows(row0, mm) : (int64_t)mm) * ((k + 3) & ~3);
        }
    }
    const Level& LL = H.lev[kappa];
    std::vector<int64_t> near_off16(H.h_near_src.size(), 0);
    for (int64_t x = 0; x < LL.nbox; ++x)
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
            const int32_t y = H.h_near_src[q];
            near_off16[q] = dof;
            jobs.push_back(HalfJob{H.h_near_off[q], dof, LL.h_count[x], LL.h_count[y], 0, y == (int32_t)x ? 1 : 0,
                                   LL.h_begin[x], LL.h_count[x]});
            dof += (int64_t)LL.h_count[x] * ((LL.h_count[y] + 3) & ~3);
        }
    H.u16_elems = uo;
    H.d16_elems = dof;
    if (((uo + kHalfSlack) >> 2) > (int64_t)UINT32_MAX || ((dof + kHalfSlack) >> 2) > (int64_t)UINT32_MAX)
        fail(H2D_EUNSUPPORTED, "half-precision pools above 2^34 values are not supported");
    // U and D pools need per-block scales; split the jobs per pool
    std::vector<HalfJob> ujobs, djobs;
    std::vector<int64_t> uidx, didx;
    for (size_t q = 0; q < jobs.size(); ++q) {
        bool dense = (q >= (size_t)H.n_il) || H.h_il_kind[q] == kDense;
        (dense ? djobs : ujobs).push_back(jobs[q]);
        (dense ? didx : uidx).push_back((int64_t)q);
    }
    DBuf<HalfJob> du, dd;
    upload(du, ujobs, s);
    upload(dd, djobs, s);
    std::vector<HalfVJob> vjobs = wide_v_layout(H, s);
    DBuf<HalfVJob> dv;
    upload(dv, vjobs, s);
    DBuf<int32_t> tbeg, tcnt;
    DBuf<int64_t> tpad;
    upload(tbeg, hb, s);
    upload(tcnt, hc, s);
    upload(tpad, hp, s);
    DBuf<float> su, sd;
    su.alloc(std::max<size_t>(ujobs.size(), 1));
    sd.alloc(std::max<size_t>(djobs.size(), 1));
    H.diag32.alloc(H.n);
    HIPCK(hipMemsetAsync(H.diag32.p, 0, sizeof(float) * H.n, s));
    auto run = [&](auto* Up, auto* Vp, auto* Dp) {
        using T = std::remove_pointer_t<decltype(Up)>;
        for (size_t o = 0; o < ujobs.size(); o += 1u << 20) {
            unsigned c = (unsigned)std::min<size_t>(1u << 20, ujobs.size() - o);
            k_half_q<T><<<c, 256, 0, s>>>(du.p + o, H.U64.p, Up, su.p + o, H.diag32.p, tbeg.p, tcnt.p, tpad.p);
        }
        for (size_t o = 0; o < djobs.size(); o += 1u << 20) {
            unsigned c = (unsigned)std::min<size_t>(1u << 20, djobs.size() - o);
            k_half_q<T><<<c, 256, 0, s>>>(dd.p + o, H.D64.p, Dp, sd.p + o, H.diag32.p, tbeg.p, tcnt.p, tpad.p);
        }
        for (size_t o = 0; o < vjobs.size(); o += 1u << 20) {
            unsigned c = (unsigned)std::min<size_t>(1u << 20, vjobs.size() - o);
            k_half_v<T><<<c, 256, 0, s>>>(dv.p + o, H.V64.p, Vp);
        }
        HIPCK(hipGetLastError());
    };
    // every pool carries kHalfSlack zeroed elements at its end (the
    // multi-RHS tiles may read a few elements past the last block)
    auto alloc_half = [&](auto& buf, int64_t elems) {
        using T = std::remove_pointer_t<decltype(buf.p)>;
        buf.alloc((size_t)elems + kHalfSlack);
        HIPCK(hipMemsetAsync(buf.p + elems, 0, sizeof(T) * kHalfSlack, s));
    };
    // the pools are zeroed first: that fills the padding rows and columns
    auto zero_half = [&](auto& buf, int64_t elems) {
        using T = std::remove_pointer_t<decltype(buf.p)>;
        alloc_half(buf, elems);
        HIPCK(hipMemsetAsync(buf.p, 0, sizeof(T) * elems, s));
    };
    if (f16) {
        zero_half(H.U16, H.u16_elems);
        zero_half(H.V16, H.v16_elems);
        zero_half(H.D16, H.d16_elems);
        run(H.U16.p, H.V16.p, H.D16.p);
    }
    if (b16) {
        zero_half(H.Ub16, H.u16_elems);
        zero_half(H.Vb16, H.v16_elems);
        zero_half(H.Db16, H.d16_elems);
        run(H.Ub16.p, H.Vb16.p, H.Db16.p);
    }
    // one scale per IL block then per near block (table order)
    auto hsu = to_host(su.p, ujobs.size(), s);
    auto hsd = to_host(sd.p, djobs.size(), s);
    std::vector<float> sc(jobs.size(), 1.0f);
    for (size_t q = 0; q < uidx.size(); ++q) sc[uidx[q]] = hsu[q];
    for (size_t q = 0; q < didx.size(); ++q) sc[didx[q]] = hsd[q];
    upload(H.scale16, sc, s);
    build_quad_tables(H, near_off16, sc, hp, s);
    HIPCK(hipStreamSynchronize(s));
    H.prec_mask |= mask & (H2D_PREC_BIT(H2D_P_FP16) | H2D_PREC_BIT(H2D_P_BF16));
}

}  // namespace h2d
