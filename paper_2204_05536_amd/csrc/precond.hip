// Preconditioners for the flexible GMRES of solve.hip.
//
// Block-Jacobi: z(X) = K(X, X)^{-1} r(X) for every leaf box X, with the
// self block LU-factorised (partial pivoting) once at set-up: leaves of up
// to 64 points in LDS, larger ones (up to 1024 points, as the paper's leaves
// of 500) in place in the LU pool.
#include "h2d_impl.h"

#include <algorithm>

namespace h2d {

constexpr int kLuMax = 64;       // leaves up to this many points: LU in LDS, solve by one wave
constexpr int kLuBigMax = 1024;  // larger leaves up to this many: LU in the LU pool, solve by a workgroup

// One workgroup per leaf: LU with partial pivoting of the m x m self block
// (column-major at D + off) in LDS; stores L (unit diagonal) and U packed
// column-major, and the pivot row chosen at each step.
__global__ void __launch_bounds__(256)
k_leaf_lu(int32_t nleaf, const int32_t* __restrict__ count, const int64_t* __restrict__ self_off,
          const int64_t* __restrict__ lu_off, const double* __restrict__ D, double* __restrict__ LU,
          int32_t* __restrict__ piv, const int32_t* __restrict__ begin, int* __restrict__ singular)
{
    __shared__ double A[kLuMax][kLuMax + 1];
    __shared__ int32_t pv;
    const int32_t X = blockIdx.x;
    if (X >= nleaf) return;
    const int32_t m = count[X];
    if (m > kLuMax) return;   // k_leaf_lu_big
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const double* S = D + self_off[X];
    for (int e = t; e < m * m; e += blockDim.x) A[e % m][e / m] = S[e];
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        if (wave == 0) {
            double best = -1.0;
            int bi = -1;
            for (int i = k + lane; i < m; i += kWave) {
                const double v = fabs(A[i][k]);
                if (v > best) { best = v; bi = i; }
            }
            for (int d = 32; d > 0; d >>= 1) {
                const double ov = __shfl_xor(best, d, kWave);
                const int oi = __shfl_xor(bi, d, kWave);
                if (ov > best || (ov == best && oi >= 0 && (bi < 0 || oi < bi))) { best = ov; bi = oi; }
            }
            if (lane == 0) {
                pv = bi;
                piv[begin[X] + k] = bi;
                if (!(best > 0.0)) atomicOr(singular, 1);
            }
        }
        __syncthreads();
        const int p = pv;
        if (p != k)
            for (int j = t; j < m; j += blockDim.x) {
                const double a = A[k][j];
                A[k][j] = A[p][j];
                A[p][j] = a;
            }
        __syncthreads();
        const double d = A[k][k];
        for (int i = k + 1 + t; i < m; i += blockDim.x) A[i][k] /= d;
        __syncthreads();
        const int rem = m - k - 1;
        for (int e = t; e < rem * rem; e += blockDim.x) {
            const int i = k + 1 + e % rem, j = k + 1 + e / rem;
            A[i][j] -= A[i][k] * A[k][j];
        }
        __syncthreads();
    }
    double* O = LU + lu_off[X];
    for (int e = t; e < m * m; e += blockDim.x) O[e] = A[e % m][e / m];
}

// One workgroup per leaf of more than kLuMax points (leaves[] lists them):
// the same factorisation in place on the leaf's copy in the LU pool.  At
// step k one wave finds the pivot (largest |A(i, k)|, i >= k, the first
// such row on ties), rows k and p are swapped, the column below the
// diagonal is divided by it and the trailing block takes its rank-1
// update, a workgroup barrier between the parts.
__global__ void __launch_bounds__(256)
k_leaf_lu_big(const int32_t* __restrict__ leaves, int32_t nbig, const int32_t* __restrict__ count,
              const int64_t* __restrict__ self_off, const int64_t* __restrict__ lu_off, const double* __restrict__ D,
              double* __restrict__ LU, int32_t* __restrict__ piv, const int32_t* __restrict__ begin,
              int* __restrict__ singular)
{
    __shared__ int32_t pv;
    if ((int32_t)blockIdx.x >= nbig) return;
    const int32_t X = leaves[blockIdx.x];
    const int32_t m = count[X];
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const double* S = D + self_off[X];
    double* A = LU + lu_off[X];   // column-major: A(i, j) = A[i + j m]
    for (int64_t e = t; e < (int64_t)m * m; e += blockDim.x) A[e] = S[e];
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        const double* col = A + (int64_t)k * m;
        if (wave == 0) {
            double best = -1.0;
            int bi = -1;
            for (int i = k + lane; i < m; i += kWave) {
                const double v = fabs(col[i]);
                if (v > best) { best = v; bi = i; }
            }
            for (int d = 32; d > 0; d >>= 1) {
                const double ov = __shfl_xor(best, d, kWave);
                const int oi = __shfl_xor(bi, d, kWave);
                if (ov > best || (ov == best && oi >= 0 && (bi < 0 || oi < bi))) { best = ov; bi = oi; }
            }
            if (lane == 0) {
                pv = bi;
                piv[begin[X] + k] = bi;
                if (!(best > 0.0)) atomicOr(singular, 1);
            }
        }
        __syncthreads();
        const int p = pv;
        if (p != k)
            for (int j = t; j < m; j += blockDim.x) {
                const double a = A[k + (int64_t)j * m];
                A[k + (int64_t)j * m] = A[p + (int64_t)j * m];
                A[p + (int64_t)j * m] = a;
            }
        __syncthreads();
        const double dk = A[k + (int64_t)k * m];
        for (int i = k + 1 + t; i < m; i += blockDim.x) A[i + (int64_t)k * m] /= dk;
        __syncthreads();
        const int rem = m - k - 1;
        for (int64_t e = t; e < (int64_t)rem * rem; e += blockDim.x) {
            const int i = k + 1 + (int)(e % rem), j = k + 1 + (int)(e / rem);
            A[i + (int64_t)j * m] -= A[i + (int64_t)k * m] * A[k + (int64_t)j * m];
        }
        __syncthreads();
    }
}

// One wave per leaf: z(X) = U^{-1} L^{-1} P r(X), vectors in caller order.
__global__ void __launch_bounds__(256)
k_leaf_solve(int32_t nleaf, const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
             const int64_t* __restrict__ lu_off, const double* __restrict__ LU, const int32_t* __restrict__ piv,
             const int32_t* __restrict__ perm, const double* __restrict__ r, double* __restrict__ z)
{
    __shared__ double y[4][kLuMax];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t X = blockIdx.x * 4 + wave;
    if (X >= nleaf) return;
    const int32_t m = count[X], r0 = begin[X];
    if (m > kLuMax) return;   // k_leaf_solve_big
    const double* F = LU + lu_off[X];
    double* yw = y[wave];
    if (lane < m) yw[lane] = r[perm[r0 + lane]];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0)
        for (int k = 0; k < m; ++k) {
            const int p = piv[r0 + k];
            if (p != k) { const double a = yw[k]; yw[k] = yw[p]; yw[p] = a; }
        }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    double v = lane < m ? yw[lane] : 0.0;
    for (int k = 0; k < m; ++k) {   // unit lower triangle
        const double yk = __shfl(v, k, kWave);
        if (lane > k && lane < m) v -= F[(int64_t)k * m + lane] * yk;
    }
    for (int k = m - 1; k >= 0; --k) {   // upper triangle
        double yk = __shfl(v, k, kWave);
        yk /= F[(int64_t)k * m + k];
        if (lane == k) v = yk;
        if (lane < k) v -= F[(int64_t)k * m + lane] * yk;
    }
    if (lane < m) z[perm[r0 + lane]] = v;
}

// One workgroup per leaf of more than kLuMax points: the same solve with
// the vector in LDS, one barrier per elimination step.
__global__ void __launch_bounds__(256)
k_leaf_solve_big(const int32_t* __restrict__ leaves, int32_t nbig, const int32_t* __restrict__ begin,
                 const int32_t* __restrict__ count, const int64_t* __restrict__ lu_off, const double* __restrict__ LU,
                 const int32_t* __restrict__ piv, const int32_t* __restrict__ perm, const double* __restrict__ r,
                 double* __restrict__ z)
{
    __shared__ double y[kLuBigMax];
    if ((int32_t)blockIdx.x >= nbig) return;
    const int32_t X = leaves[blockIdx.x];
    const int32_t m = count[X], r0 = begin[X];
    const double* F = LU + lu_off[X];
    const int t = threadIdx.x;
    for (int i = t; i < m; i += blockDim.x) y[i] = r[perm[r0 + i]];
    __syncthreads();
    if (t == 0)
        for (int k = 0; k < m; ++k) {
            const int p = piv[r0 + k];
            if (p != k) { const double a = y[k]; y[k] = y[p]; y[p] = a; }
        }
    __syncthreads();
    for (int k = 0; k < m; ++k) {   // unit lower triangle
        const double yk = y[k];
        for (int i = k + 1 + t; i < m; i += blockDim.x) y[i] -= F[(int64_t)k * m + i] * yk;
        __syncthreads();
    }
    for (int k = m - 1; k >= 0; --k) {   // upper triangle
        if (t == 0) y[k] /= F[(int64_t)k * m + k];
        __syncthreads();
        const double yk = y[k];
        for (int i = t; i < k; i += blockDim.x) y[i] -= F[(int64_t)k * m + i] * yk;
        __syncthreads();
    }
    for (int i = t; i < m; i += blockDim.x) z[perm[r0 + i]] = y[i];
}

void bj_setup(Handle& H, hipStream_t s)
{
    const Level& LL = H.lev[H.kappa];
    const int32_t nleaf = (int32_t)LL.nbox;
    std::vector<int64_t> self(nleaf, -1), luo(nleaf);
    int64_t tot = 0;
    std::vector<int32_t> big;
    for (int32_t x = 0; x < nleaf; ++x) {
        if (LL.h_count[x] > kLuBigMax)
            fail(H2D_EUNSUPPORTED, "block-Jacobi needs leaf boxes of at most " + std::to_string(kLuBigMax) + " points");
        if (LL.h_count[x] > kLuMax) big.push_back(x);
        for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q)
            if (H.h_near_src[q] == x) self[x] = H.h_near_off[q];
        luo[x] = tot;
        tot += (int64_t)LL.h_count[x] * LL.h_count[x];
    }
    DBuf<int64_t> dself;
    dself.alloc(nleaf);
    HIPCK(hipMemcpyAsync(dself.p, self.data(), sizeof(int64_t) * nleaf, hipMemcpyHostToDevice, s));
    H.bj_off.alloc(nleaf);
    HIPCK(hipMemcpyAsync(H.bj_off.p, luo.data(), sizeof(int64_t) * nleaf, hipMemcpyHostToDevice, s));
    H.bj_lu.alloc(std::max<int64_t>(tot, 1));
    H.bj_piv.alloc(H.n);
    DBuf<int> sing;
    sing.alloc(1);
    HIPCK(hipMemsetAsync(sing.p, 0, sizeof(int), s));
    k_leaf_lu<<<nleaf, 256, 0, s>>>(nleaf, LL.count.p, dself.p, H.bj_off.p, H.D64.p, H.bj_lu.p, H.bj_piv.p,
                                    LL.begin.p, sing.p);
    H.bj_big.alloc(std::max<size_t>(big.size(), 1));
    H.n_bj_big = (int32_t)big.size();
    if (!big.empty()) {
        HIPCK(hipMemcpyAsync(H.bj_big.p, big.data(), sizeof(int32_t) * big.size(), hipMemcpyHostToDevice, s));
        k_leaf_lu_big<<<(unsigned)big.size(), 256, 0, s>>>(H.bj_big.p, H.n_bj_big, LL.count.p, dself.p, H.bj_off.p,
                                                            H.D64.p, H.bj_lu.p, H.bj_piv.p, LL.begin.p, sing.p);
    }
    HIPCK(hipGetLastError());
    int hs = 0;
    HIPCK(hipMemcpyAsync(&hs, sing.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    if (hs) fail(H2D_EINVAL, "a leaf self block is singular");
    H.bj_ready = true;
}

void precond_apply(Handle& H, int pc, const double* r, double* z, hipStream_t s)
{
    const Level& LL = H.lev[H.kappa];
    const int32_t nleaf = (int32_t)LL.nbox;
    if (pc == H2D_PC_BLOCK_JACOBI) {
        if (!H.bj_ready) fail(H2D_EINVAL, "block-Jacobi was not set up (h2d_bj_setup)");
        k_leaf_solve<<<(nleaf + 3) / 4, 256, 0, s>>>(nleaf, LL.begin.p, LL.count.p, H.bj_off.p, H.bj_lu.p, H.bj_piv.p,
                                                     H.perm.p, r, z);
        if (H.n_bj_big)
            k_leaf_solve_big<<<(unsigned)H.n_bj_big, 256, 0, s>>>(H.bj_big.p, H.n_bj_big, LL.begin.p, LL.count.p,
                                                                  H.bj_off.p, H.bj_lu.p, H.bj_piv.p, H.perm.p, r, z);
        HIPCK(hipGetLastError());
    } else if (pc == H2D_PC_MLP) {
        mlp_apply(H, r, z, s);
    } else {
        fail(H2D_EINVAL, "unknown preconditioner");
    }
}

}  // namespace h2d
