// Algorithm 2 (MatVec) on gfx950.
//
//   gather:   xs = x(perm)                     tree order
//   phase A:  t_b = V_b^T xs(Y_b)              every low-rank block, all levels
//   reduce:   t_b = sum of partials            blocks whose V was split over waves
//   phase B:  y(X) = sum over the leaf box X's dense near blocks, and over
//             the blocks of X and of each ancestor of X, of U_b(rows of X) t_b
//             (or D_b(rows of X) xs(Y_b) for dense blocks); written once,
//             scattered back to caller order.  No atomics: every output row
//             is owned by one wave, and every sum is taken in a fixed order,
//             so two runs give identical bits.
//
// Storage: U column-major m x k (a leaf box's rows are contiguous in every
// column), V row-major n x k (a wave reads whole rows: G = 64 / k rows per
// load instruction), D column-major m x n.
#include "h2d_impl.h"

#include <algorithm>
#include <cstring>

namespace h2d {

struct LevelPtrs {
    const int32_t* begin[kMaxLevel + 1];
    const int32_t* count[kMaxLevel + 1];
    const int32_t* parent[kMaxLevel + 1];
    const int32_t* il_ptr[kMaxLevel + 1];
};

template <typename T> __device__ __forceinline__ float ldf(const T* p);
template <> __device__ __forceinline__ float ldf<__half>(const __half* p) { return __half2float(*p); }
template <> __device__ __forceinline__ float ldf<__hip_bfloat16>(const __hip_bfloat16* p) { return __bfloat162float(*p); }

template <typename T, typename A> __device__ __forceinline__ A ld(const T* p) { return (A)ldf<T>(p); }
template <> __device__ __forceinline__ double ld<double, double>(const double* p) { return *p; }

template <typename A>
__global__ void k_gather(const double* x, const int32_t* perm, int32_t n, int64_t ldx, int64_t ldxs, int nrhs, A* xs)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t p = perm[i];
    for (int r = 0; r < nrhs; ++r) xs[(int64_t)r * ldxs + i] = (A)x[(int64_t)r * ldx + p];
}

// Phase A: one wave per work item (rows j0..j1 of one block's V).
template <typename T, typename A, bool kScaled>
__global__ void __launch_bounds__(256)
k_phaseA(int64_t nitems, const ADesc* __restrict__ items, const T* __restrict__ V, const A* __restrict__ xs,
         A* __restrict__ tpool, A* __restrict__ ppool, int64_t nsplit_base, const float* __restrict__ scale)
{
    __shared__ A red[4][kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t it = (int64_t)blockIdx.x * 4 + wave;
    if (it >= nitems) return;
    const ADesc D = items[it];
    const int32_t k = D.k;
    const T* Vb = V + D.voff;
    const A* xb = xs + D.col0;
    A* out = (D.out >= 0) ? (tpool + D.out) : (ppool + (-D.out - 1));
    A sc = (A)1;
    if constexpr (kScaled) sc = (A)scale[D.pad];
    (void)nsplit_base;
    if (k <= kWave) {
        const int G = kWave / k, g = lane / k, q = lane % k;
        A acc = (A)0;
        if (g < G) {
            int32_t j = D.j0 + g;
#pragma unroll 4
            for (; j < D.j1; j += G) acc += ld<T, A>(Vb + (int64_t)j * k + q) * xb[j];
        }
        red[wave][lane] = acc;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (lane < k) {
            A s = (A)0;
            for (int gg = 0; gg < G; ++gg) s += red[wave][gg * k + lane];
            out[lane] = s * sc;
        }
    } else {
        for (int32_t qc = 0; qc < k; qc += kWave) {
            const int32_t q = qc + lane;
            if (q < k) {
                A acc = (A)0;
#pragma unroll 4
                for (int32_t j = D.j0; j < D.j1; ++j) acc += ld<T, A>(Vb + (int64_t)j * k + q) * xb[j];
                out[q] = acc * sc;
            }
        }
    }
}

template <typename A>
__global__ void k_reduce_parts(int64_t nr, const RDesc* __restrict__ R, const A* __restrict__ ppool, A* __restrict__ tpool)
{
    const int64_t r = blockIdx.x;
    if (r >= nr) return;
    const RDesc D = R[r];
    for (int q = threadIdx.x; q < D.k; q += blockDim.x) {
        A s = (A)0;
        for (int p = 0; p < D.nparts; ++p) s += ppool[D.pbeg + (int64_t)p * D.k + q];
        tpool[D.tout + q] = s;
    }
}

// Phase B: one wave per leaf box, 4 leaf boxes (consecutive in tree order)
// per workgroup; workgroups are mapped to XCDs in contiguous tile ranges so
// neighbouring boxes share an L2.
template <typename T, typename A, bool kHalf>
__global__ void __launch_bounds__(256)
k_phaseB(int32_t nleaf, int kappa, LevelPtrs L, const int32_t* __restrict__ near_ptr, const BDesc* __restrict__ bnear,
         const BDesc* __restrict__ bil, const T* __restrict__ Up, const T* __restrict__ Dp, const A* __restrict__ tpool,
         const A* __restrict__ xs, const int32_t* __restrict__ perm, double* __restrict__ y,
         const float* __restrict__ scale, const float* __restrict__ diag, int64_t n_il)
{
    __shared__ A red[4][kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    // XCD-aware tile order: hardware deals workgroups round-robin over 8 XCDs
    const int32_t W = gridDim.x, w = blockIdx.x, xcd = w % 8, i8 = w / 8;
    const int32_t q8 = W / 8, r8 = W % 8;
    const int32_t tile = xcd * q8 + min(xcd, r8) + i8;
    const int32_t X = tile * 4 + wave;
    if (X >= nleaf) return;
    const int32_t r0 = L.begin[kappa][X], cnt = L.count[kappa][X];
    for (int32_t rc = 0; rc < cnt; rc += kWave) {
        const int32_t rows = min(kWave, cnt - rc);
        const int G = kWave / rows, g = lane / rows, r = lane % rows;
        const bool act = g < G;
        A acc = (A)0;
        // dense near blocks of X (self first in key order, then edge sharers)
        for (int32_t q = near_ptr[X]; q < near_ptr[X + 1]; ++q) {
            const BDesc d = bnear[q];
            const int32_t nn = -d.cols;
            const T* base = Dp + d.off + rc + r;
            const A* tv = xs + d.tsrc;
            A a = (A)0;
            if (act) {
#pragma unroll 4
                for (int32_t j = g; j < nn; j += G) a += ld<T, A>(base + (int64_t)j * cnt) * tv[j];
            }
            if constexpr (kHalf) acc += a * (A)scale[n_il + q];
            else acc += a;
        }
        // interaction-list blocks of X and of every ancestor
        int32_t a_box = X;
        for (int l = kappa; l >= 1; --l) {
            const int32_t ab = L.begin[l][a_box], ld_m = L.count[l][a_box];
            const int32_t off = r0 - ab + rc + r;
            const int32_t q1 = L.il_ptr[l][a_box + 1];
            for (int32_t q = L.il_ptr[l][a_box]; q < q1; ++q) {
                const BDesc d = bil[q];
                if (d.cols > 0) {
                    const T* base = Up + d.off + off;
                    const A* tv = tpool + d.tsrc;
                    if (act) {
#pragma unroll 4
                        for (int32_t c = g; c < d.cols; c += G) acc += ld<T, A>(base + (int64_t)c * ld_m) * tv[c];
                    }
                } else if (d.cols < 0) {
                    const T* base = Dp + d.off + off;
                    const A* tv = xs + d.tsrc;
                    A a = (A)0;
                    if (act) {
#pragma unroll 4
                        for (int32_t j = g; j < -d.cols; j += G) a += ld<T, A>(base + (int64_t)j * ld_m) * tv[j];
                    }
                    if constexpr (kHalf) acc += a * (A)scale[q];
                    else acc += a;
                }
            }
            a_box = L.parent[l][a_box];
        }
        red[wave][lane] = act ? acc : (A)0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (lane < rows) {
            A s = (A)0;
            for (int gg = 0; gg < G; ++gg) s += red[wave][gg * rows + lane];
            const int32_t i = r0 + rc + lane;
            if constexpr (kHalf) s += (A)diag[i] * xs[i];
            y[perm[i]] = (double)s;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

template <typename T>
static void upload_vec(DBuf<T>& d, const std::vector<T>& h, hipStream_t s)
{
    d.alloc(std::max<size_t>(h.size(), 1));
    if (!h.empty()) HIPCK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
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
    std::vector<ADesc> items;
    std::vector<RDesc> red;
    H.h_il_toff.assign(nil, -1);
    int64_t toff = 0, poff = 0;
    H.max_rank = 0; H.sum_rank = 0; H.n_il_dense = 0;
    double bytes = 0, flops = 0, hbytes = 0;
    for (int64_t b = 0; b < nil; ++b) {
        const Level& L = H.lev[H.h_il_level[b]];
        int32_t m = L.h_count[H.h_il_tgt[b]], n = L.h_count[H.h_il_src[b]], c0 = L.h_begin[H.h_il_src[b]];
        if (H.h_il_kind[b] == kDense) {
            bi[b] = BDesc{H.h_il_off[b], -n, c0};
            H.n_il_dense++;
            bytes += 8.0 * m * n; hbytes += 2.0 * m * n; flops += 2.0 * m * n;
            continue;
        }
        int32_t k = H.h_il_k[b];
        H.max_rank = std::max<int64_t>(H.max_rank, k);
        H.sum_rank += k;
        bi[b] = BDesc{H.h_il_off[b], k, (int32_t)toff};
        if (k == 0) continue;
        H.h_il_toff[b] = (int32_t)toff;
        bytes += 8.0 * k * (double)(m + n); hbytes += 2.0 * k * (double)(m + n); flops += 2.0 * k * (double)(m + n);
        if (n <= kPhaseARows) {
            items.push_back(ADesc{H.h_il_voff[b], 0, n, c0, k, (int32_t)toff, (int32_t)b});
        } else {
            int32_t parts = (n + kPhaseARows - 1) / kPhaseARows;
            red.push_back(RDesc{(int32_t)toff, k, (int32_t)poff, parts});
            for (int32_t p = 0; p < parts; ++p) {
                int32_t j0 = p * kPhaseARows, j1 = std::min(n, j0 + kPhaseARows);
                items.push_back(ADesc{H.h_il_voff[b], j0, j1, c0, k, (int32_t)(-(poff + (int64_t)p * k) - 1), (int32_t)b});
            }
            poff += (int64_t)parts * k;
        }
        toff += k;
    }
    for (int64_t x = 0; x < LL.nbox; ++x)
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
            double e = (double)LL.h_count[x] * LL.h_count[H.h_near_src[q]];
            bytes += 8.0 * e; hbytes += 2.0 * e; flops += 2.0 * e;
        }
    // vectors: x read (gather), xs written and read, y written, perm read
    const double nvec = (double)H.n;
    bytes += nvec * (8 + 8 + 8 + 4);
    hbytes += nvec * (8 + 4 + 8 + 4 + 4);   // FP32 xs, FP32 diagonal
    H.alg_bytes_fp64 = bytes; H.alg_bytes_half = hbytes; H.flops = flops;
    H.t_elems = toff; H.p_elems = poff;
    // per-kernel algorithmic bytes: each operand touched once
    for (int h = 0; h < 2; ++h) {
        const double s = h ? 2.0 : 8.0, a = h ? 4.0 : 8.0;   // storage, accumulation sizes
        double vstore = 0, ustore = 0, dstore = 0;
        vstore = (double)H.v_elems * s;
        ustore = (double)H.u_elems * s;
        dstore = (double)H.d_elems * s;
        H.phase_bytes[h][0] = nvec * (8 + 4 + a);                                   // x, perm -> xs
        H.phase_bytes[h][1] = vstore + nvec * a + (double)toff * a + (double)poff * a;  // V, xs -> t / partials
        H.phase_bytes[h][2] = poff ? (double)poff * a + (double)toff * a : 0.0;        // partials -> t
        H.phase_bytes[h][3] = ustore + dstore + (double)toff * a + nvec * (a + 4 + 8) + (h ? nvec * 4 : 0.0);
    }
    upload_vec(H.bil, bi, s);
    upload_vec(H.aitems, items, s);
    upload_vec(H.ritems, red, s);
    H.n_aitems = (int64_t)items.size();
    H.n_ritems = (int64_t)red.size();
    HIPCK(hipStreamSynchronize(s));
}

void ensure_workspace(Handle& H, int nrhs)
{
    if (H.ws_nrhs >= nrhs) return;
    const int64_t n = H.n;
    H.xs.alloc((size_t)n * nrhs);
    H.tpool.alloc(std::max<int64_t>(H.t_elems, 1) * nrhs);
    H.ppool.alloc(std::max<int64_t>(H.p_elems, 1) * nrhs);
    if (H.prec_mask & (H2D_PREC_BIT(H2D_P_FP16) | H2D_PREC_BIT(H2D_P_BF16))) {
        H.xs32.alloc((size_t)n * nrhs);
        H.tpool32.alloc(std::max<int64_t>(H.t_elems, 1) * nrhs);
        H.ppool32.alloc(std::max<int64_t>(H.p_elems, 1) * nrhs);
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

// Event slot e (0..4) of the current recorded matvec, or null.
static hipEvent_t* prof_slot(Handle& H)
{
    if (!H.prof_on || H.prof_used >= kProfMax) return nullptr;
    size_t need = (H.prof_used + 1) * 5;
    while (H.prof_ev.size() < need) {
        hipEvent_t e;
        HIPCK(hipEventCreate(&e));
        H.prof_ev.push_back(e);
    }
    return H.prof_ev.data() + H.prof_used * 5;
}

template <typename T, typename A, bool kHalf>
static void run_one(Handle& H, const T* U, const T* V, const T* D, A* xs, A* tp, A* pp, const double* x, double* y,
                    hipStream_t s)
{
    const int32_t n = (int32_t)H.n;
    hipEvent_t* ev = prof_slot(H);
    if (ev) HIPCK(hipEventRecord(ev[0], s));
    k_gather<A><<<(n + 255) / 256, 256, 0, s>>>(x, H.perm.p, n, 0, 0, 1, xs);
    if (ev) HIPCK(hipEventRecord(ev[1], s));
    if (H.n_aitems)
        k_phaseA<T, A, kHalf><<<(unsigned)((H.n_aitems + 3) / 4), 256, 0, s>>>(H.n_aitems, H.aitems.p, V, xs, tp, pp, 0,
                                                                            H.scale16.p);
    if (ev) HIPCK(hipEventRecord(ev[2], s));
    if (H.n_ritems) k_reduce_parts<A><<<(unsigned)H.n_ritems, 64, 0, s>>>(H.n_ritems, H.ritems.p, pp, tp);
    if (ev) HIPCK(hipEventRecord(ev[3], s));
    const int32_t nleaf = (int32_t)H.lev[H.kappa].nbox;
    k_phaseB<T, A, kHalf><<<(unsigned)((nleaf + 3) / 4), 256, 0, s>>>(
        nleaf, H.kappa, level_ptrs(H), H.near_ptr.p, H.bnear.p, H.bil.p, U, D, tp, xs, H.perm.p, y, H.scale16.p,
        H.diag32.p, H.n_il);
    if (ev) {
        HIPCK(hipEventRecord(ev[4], s));
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
    for (int p = 0; p < 4; ++p) out->bytes[p] = H.phase_bytes[h][p];
    if (H.prof_used) HIPCK(hipEventSynchronize(H.prof_ev[H.prof_used * 5 - 1]));
    for (size_t c = 0; c < H.prof_used; ++c)
        for (int p = 0; p < 4; ++p) {
            float ms = 0.f;
            HIPCK(hipEventElapsedTime(&ms, H.prof_ev[c * 5 + p], H.prof_ev[c * 5 + p + 1]));
            out->ms[p] += ms;
        }
    if (H.prof_used)
        for (int p = 0; p < 4; ++p) out->ms[p] /= (double)H.prof_used;
    H.prof_used = 0;
}

void launch_matvec(Handle& H, const double* x, double* y, int nrhs, int64_t ld, int prec, hipStream_t s)
{
    ensure_workspace(H, 1);
    H.prof_prec = prec;
    for (int r = 0; r < nrhs; ++r) {
        const double* xr = x + (int64_t)r * ld;
        double* yr = y + (int64_t)r * ld;
        if (prec == H2D_P_FP64)
            run_one<double, double, false>(H, H.U64.p, H.V64.p, H.D64.p, H.xs.p, H.tpool.p, H.ppool.p, xr, yr, s);
        else if (prec == H2D_P_FP16)
            run_one<__half, float, true>(H, H.U16.p, H.V16.p, H.D16.p, H.xs32.p, H.tpool32.p, H.ppool32.p, xr, yr, s);
        else
            run_one<__hip_bfloat16, float, true>(H, H.Ub16.p, H.Vb16.p, H.Db16.p, H.xs32.p, H.tpool32.p, H.ppool32.p,
                                                  xr, yr, s);
    }
}

}  // namespace h2d
