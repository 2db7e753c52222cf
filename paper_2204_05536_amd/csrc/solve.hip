// Restarted GMRES on the HODLR2D operator (Section 5 uses GMRES with the
// fast matvec), plus FP64 iterative refinement around a GMRES on the
// FP16/BF16 operator.
//
// Arnoldi uses classical Gram-Schmidt applied twice (two batched passes of
// dot products instead of j sequential ones); the reductions are two-stage
// with a fixed order, so results are reproducible.  The small Hessenberg
// least-squares problem (Givens rotations) is solved on the host from the
// j + 2 scalars read back per step.
#include "h2d_impl.h"

#include <chrono>
#include <cmath>

namespace h2d {

constexpr int kDotBlocks = 512;
constexpr int kDotThreads = 256;

// part[b * nv + c] = sum over block b's slice of V[c] . w  (c < nv)
__global__ void __launch_bounds__(kDotThreads)
k_dots(const double* __restrict__ V, int64_t ldv, int nv, const double* __restrict__ w, int64_t n, double* part)
{
    __shared__ double red[kDotThreads / kWave][64];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * per, i1 = min(n, i0 + per);
    for (int c0 = 0; c0 < nv; c0 += 8) {
        double acc[8];
        for (int c = 0; c < 8; ++c) acc[c] = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += kDotThreads) {
            double wi = w[i];
            for (int c = 0; c < 8; ++c)
                if (c0 + c < nv) acc[c] += V[(int64_t)(c0 + c) * ldv + i] * wi;
        }
        for (int c = 0; c < 8; ++c) {
            double v = acc[c];
            for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
            if (lane == 0) red[wave][c] = v;
        }
        __syncthreads();
        if (threadIdx.x < 8 && c0 + (int)threadIdx.x < nv) {
            double s = 0.0;
            for (int q = 0; q < kDotThreads / kWave; ++q) s += red[q][threadIdx.x];
            part[(int64_t)blockIdx.x * nv + c0 + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

__global__ void k_dots_final(const double* part, int nb, int nv, double* out)
{
    for (int c = threadIdx.x; c < nv; c += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[(int64_t)b * nv + c];
        out[c] = s;
    }
}

// w -= sum_c V[c] h[c]
__global__ void k_sub_comb(double* __restrict__ w, const double* __restrict__ V, int64_t ldv, int nv,
                           const double* __restrict__ h, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = w[i];
        for (int c = 0; c < nv; ++c) s -= V[(int64_t)c * ldv + i] * h[c];
        w[i] = s;
    }
}

// x += sum_c V[c] y[c]
__global__ void k_add_comb(double* __restrict__ x, const double* __restrict__ V, int64_t ldv, int nv,
                           const double* __restrict__ y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = x[i];
        for (int c = 0; c < nv; ++c) s += V[(int64_t)c * ldv + i] * y[c];
        x[i] = s;
    }
}

__global__ void k_scale(double* __restrict__ out, const double* __restrict__ in, double a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i] * a;
}

// out = a - b
__global__ void k_sub(double* __restrict__ out, const double* __restrict__ a, const double* __restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] - b[i];
}

// v *= 1 / |v| with |v|^2 read from device memory (no host round trip);
// a zero norm leaves v unchanged (exact breakdown, handled on the host).
__global__ void k_scale_by_norm(double* __restrict__ v, const double* __restrict__ nrm2, int64_t n)
{
    const double s2 = nrm2[0];
    if (!(s2 > 0.0)) return;
    const double a = 1.0 / sqrt(s2);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] *= a;
}

// out[0..nv) = a[0..nv) + b[0..nv) (the two Gram-Schmidt passes' coefficients)
__global__ void k_add_small(const double* __restrict__ a, const double* __restrict__ b, int nv, double* __restrict__ out)
{
    for (int c = threadIdx.x; c < nv; c += blockDim.x) out[c] = a[c] + b[c];
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

// Dot products and norms on the handle's partial-sum buffers.
struct Blas {
    hipStream_t s;
    int64_t n;
    DBuf<double>& part;
    DBuf<double>& dres;
    std::vector<double> h;
    Blas(Handle& H, hipStream_t s_, int64_t n_, int maxv) : s(s_), n(n_), part(H.gm_part), dres(H.gm_dres)
    {
        part.reserve((size_t)kDotBlocks * maxv);
        dres.reserve(4 * (size_t)maxv + 4);
        h.resize(4 * (size_t)maxv + 4);
    }
    int grid() const { return (int)std::min<int64_t>(4096, (n + 255) / 256); }
    // device result in dres[at .. at + nv), copied to host h when asked
    const double* dots(const double* V, int nv, const double* w, bool to_host, int at = 0)
    {
        k_dots<<<kDotBlocks, kDotThreads, 0, s>>>(V, n, nv, w, n, part.p);
        k_dots_final<<<1, 64, 0, s>>>(part.p, kDotBlocks, nv, dres.p + at);
        HIPCK(hipGetLastError());
        if (to_host) {
            HIPCK(hipMemcpyAsync(h.data(), dres.p + at, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
            HIPCK(hipStreamSynchronize(s));
        }
        return dres.p + at;
    }
    double nrm2(const double* w)
    {
        dots(w, 1, w, true);
        return std::sqrt(h[0]);
    }
};

struct GmresResult {
    int iters = 0;
    int restarts = 0;
    double relres = 1.0;   // true residual of the operator used, relative to |rhs|
    bool converged = false;
    int fallback_at = -1;  // Arnoldi step at which the learned preconditioner was dropped
};

// The learned preconditioner is not a fixed linear map and can be a poor
// one: when the Arnoldi residual estimate falls by less than 10% over 10
// steps with it, the cycle is closed and the solve goes on with the exact
// block-Jacobi fallback (or without a preconditioner if that was not set
// up).
constexpr int kStallSteps = 10;
constexpr double kStallRatio = 0.9;

// GMRES(restart) for A_prec x = rhs, x0 = 0, optionally right-
// preconditioned in the flexible form (z_j = M v_j kept, x += Z y).
// Convergence is judged by the true residual |rhs - A_prec x| / |rhs| <= tol
// at each restart.  An inner solve of the refinement loop (`inner`) stops
// on the Arnoldi estimate instead: the loop around it computes the true
// FP64 residual anyway, so a true residual of the half operator would be a
// product spent for nothing.
static GmresResult gmres(Handle& H, int prec, const double* rhs, double* x, double tol, int restart, int max_iter,
                         int& precond, bool inner, hipStream_t s)
{
    const int64_t n = H.n;
    const int m = restart;
    Blas B(H, s, n, m + 1);
    DBuf<double>& Vb = H.gm_V;
    DBuf<double>& Zb = H.gm_Z;
    DBuf<double>& w = H.gm_w;
    DBuf<double>& r = H.gm_r;
    DBuf<double>& yv = H.gm_y;
    Vb.reserve((size_t)n * (m + 1));
    if (precond != H2D_PC_NONE) Zb.reserve((size_t)n * m);
    w.reserve(n);
    r.reserve(n);
    yv.reserve(m + 1);
    std::vector<double> Hm((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m);
    const int grid = B.grid();
    GmresResult R;
    HIPCK(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    const double bn = B.nrm2(rhs);
    if (bn == 0.0) { R.relres = 0.0; R.converged = true; return R; }
    bool first = true;
    for (;;) {
        if (first) {
            HIPCK(hipMemcpyAsync(r.p, rhs, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        } else {
            launch_matvec(H, x, w.p, 1, n, prec, s);
            k_sub<<<grid, 256, 0, s>>>(r.p, rhs, w.p, n);
        }
        first = false;
        const double beta = B.nrm2(r.p);
        R.relres = beta / bn;
        if (R.relres <= tol) { R.converged = true; break; }
        if (R.iters >= max_iter) break;
        k_scale<<<grid, 256, 0, s>>>(Vb.p, r.p, 1.0 / beta, n);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0, j_mark = 0;
        double g_mark = beta;
        bool stalled = false;
        double hn_last = 1.0;   // norm of the last new Krylov direction (0: exact breakdown)
        for (; j < m && R.iters < max_iter; ) {
            ++R.iters;
            double* vj1 = Vb.p + (int64_t)(j + 1) * n;
            if (precond != H2D_PC_NONE) {
                double* zj = Zb.p + (int64_t)j * n;
                precond_apply(H, precond, Vb.p + (int64_t)j * n, zj, s);
                launch_matvec(H, zj, vj1, 1, n, prec, s);
            } else {
                launch_matvec(H, Vb.p + (int64_t)j * n, vj1, 1, n, prec, s);
            }
            // two passes of classical Gram-Schmidt, the norm and the
            // normalisation on the device; one read-back per step: the
            // j + 1 summed coefficients and the squared norm
            std::vector<double> hc(j + 2, 0.0);
            const int nv = j + 1, o1 = 0, o2 = nv, o3 = 2 * nv;
            const double* d1 = B.dots(Vb.p, nv, vj1, false, o1);
            k_sub_comb<<<grid, 256, 0, s>>>(vj1, Vb.p, n, nv, d1, n);
            const double* d2 = B.dots(Vb.p, nv, vj1, false, o2);
            k_sub_comb<<<grid, 256, 0, s>>>(vj1, Vb.p, n, nv, d2, n);
            double* hsum = B.dres.p + o3;
            k_add_small<<<1, 64, 0, s>>>(d1, d2, nv, hsum);
            const double* dn = B.dots(vj1, 1, vj1, false, o3 + nv);
            k_scale_by_norm<<<grid, 256, 0, s>>>(vj1, dn, n);
            HIPCK(hipGetLastError());
            HIPCK(hipMemcpyAsync(B.h.data(), hsum, sizeof(double) * (nv + 1), hipMemcpyDeviceToHost, s));
            HIPCK(hipStreamSynchronize(s));
            for (int i = 0; i <= j; ++i) hc[i] = B.h[i];
            const double hn = std::sqrt(std::max(B.h[nv], 0.0));
            hn_last = hn;
            hc[j + 1] = hn;
            double* col = Hm.data() + (size_t)j * (m + 1);
            for (int i = 0; i <= j + 1; ++i) col[i] = hc[i];
            for (int i = 0; i < j; ++i) {
                double a = col[i], c = col[i + 1];
                col[i] = cs[i] * a + sn[i] * c;
                col[i + 1] = -sn[i] * a + cs[i] * c;
            }
            double a = col[j], c = col[j + 1], d = std::sqrt(a * a + c * c);
            cs[j] = d == 0.0 ? 1.0 : a / d;
            sn[j] = d == 0.0 ? 0.0 : c / d;
            col[j] = d;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++j;
            if (std::fabs(g[j]) / bn <= tol || hn == 0.0) break;
            if (precond == H2D_PC_MLP && j - j_mark >= kStallSteps) {
                if (std::fabs(g[j]) > kStallRatio * g_mark) { stalled = true; break; }
                g_mark = std::fabs(g[j]);
                j_mark = j;
            }
        }
        for (int i = j - 1; i >= 0; --i) {
            double sum = g[i];
            for (int q = i + 1; q < j; ++q) sum -= Hm[(size_t)q * (m + 1) + i] * y[q];
            y[i] = sum / Hm[(size_t)i * (m + 1) + i];
        }
        HIPCK(hipMemcpyAsync(yv.p, y.data(), sizeof(double) * j, hipMemcpyHostToDevice, s));
        k_add_comb<<<grid, 256, 0, s>>>(x, precond != H2D_PC_NONE ? Zb.p : Vb.p, n, j, yv.p, n);
        HIPCK(hipGetLastError());
        ++R.restarts;
        if (stalled) {
            precond = H.bj_ready ? H2D_PC_BLOCK_JACOBI : H2D_PC_NONE;
            if (R.fallback_at < 0) R.fallback_at = R.iters;
        } else if (inner && (std::fabs(g[j]) / bn <= tol || hn_last == 0.0)) {
            R.relres = std::fabs(g[j]) / bn;
            R.converged = true;
            break;
        }
    }
    HIPCK(hipStreamSynchronize(s));
    return R;
}

h2d_status solve(Handle& H, const double* b, double* x, double rtol, const h2d_solve_opts& o, h2d_solve_info* info,
                 hipStream_t s)
{
    auto t0 = std::chrono::steady_clock::now();
    const int64_t n = H.n;
    h2d_solve_info I{};
    bool ok = false;
    if (o.precond == H2D_PC_BLOCK_JACOBI && !H.bj_ready) fail(H2D_EINVAL, "block-Jacobi was not set up (h2d_bj_setup)");
    if (o.precond < H2D_PC_NONE || o.precond > H2D_PC_MLP) fail(H2D_EINVAL, "unknown preconditioner");
    I.fallback_at = -1;
    int pc = o.precond;   // the learned preconditioner may hand over to block-Jacobi
    if (o.mode == H2D_SOLVE_PLAIN) {
        GmresResult R = gmres(H, H2D_P_FP64, b, x, rtol, o.restart, o.max_iter, pc, false, s);
        I.iters = R.iters; I.outer = R.restarts; I.relres = R.relres;
        I.fallback_at = R.fallback_at;
        ok = R.converged;
    } else if (o.mode == H2D_SOLVE_REFINE) {
        if (o.inner_prec != H2D_P_FP16 && o.inner_prec != H2D_P_BF16) fail(H2D_EINVAL, "inner_prec must be FP16 or BF16");
        if (!(H.prec_mask & H2D_PREC_BIT(o.inner_prec))) fail(H2D_EUNSUPPORTED, "inner precision was not built");
        if (!(o.inner_tol > 0.0 && o.inner_tol < 1.0)) fail(H2D_EINVAL, "inner_tol must be in (0, 1)");
        Blas B(H, s, n, 1);
        DBuf<double>& r = H.rf_r;
        DBuf<double>& d = H.rf_d;
        DBuf<double>& w = H.rf_w;
        r.reserve(n); d.reserve(n); w.reserve(n);
        const int grid = B.grid();
        HIPCK(hipMemsetAsync(x, 0, sizeof(double) * n, s));
        HIPCK(hipMemcpyAsync(r.p, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        const double bn = B.nrm2(b);
        double rel = bn == 0.0 ? 0.0 : 1.0;
        int outer = 0, iters = 0;
        const int max_outer = o.max_outer > 0 ? o.max_outer : 50;
        while (rel > rtol && outer < max_outer && iters < o.max_iter) {
            GmresResult R = gmres(H, o.inner_prec, r.p, d.p, o.inner_tol, o.restart, o.max_iter - iters, pc, true, s);
            if (R.fallback_at >= 0 && I.fallback_at < 0) I.fallback_at = iters + R.fallback_at;
            iters += R.iters;
            ++outer;
            k_axpy<<<grid, 256, 0, s>>>(x, d.p, 1.0, n);
            launch_matvec(H, x, w.p, 1, n, H2D_P_FP64, s);
            k_sub<<<grid, 256, 0, s>>>(r.p, b, w.p, n);
            HIPCK(hipGetLastError());
            rel = B.nrm2(r.p) / bn;
            if (R.iters == 0) break;
        }
        I.iters = iters; I.outer = outer; I.relres = rel;
        ok = rel <= rtol;
    } else {
        fail(H2D_EINVAL, "unknown solve mode");
    }
    HIPCK(hipStreamSynchronize(s));
    I.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = I;
    return ok ? H2D_OK : H2D_ENOCONV;
}

}  // namespace h2d
