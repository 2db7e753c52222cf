// C ABI of the HODLR2D library: argument checks, error reporting, handle
// lifetime, build orchestration, import / export.
#include "h2d_impl.h"

#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <memory>
#include <algorithm>
#include <utility>

namespace h2d {

static thread_local std::string g_last_error;

void fail(h2d_status code, const std::string& msg) { throw Error{code, msg}; }

static std::atomic<int64_t> g_alloc_seen{0};

bool forced_alloc_failure()
{
    const char* e = std::getenv("H2D_TEST_FAIL_ALLOC");
    if (!e || !*e) {
        g_alloc_seen.store(0);
        return false;
    }
    const long long k = std::atoll(e);
    return k >= 1 && g_alloc_seen.fetch_add(1) + 1 == k;
}

void check_hip(hipError_t e, const char* what, const char* file, int line)
{
    if (e == hipSuccess) return;
    (void)hipGetLastError();
    h2d_status code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? H2D_ENOMEM : H2D_EDEVICE;
    fail(code, std::string(what) + ": " + hipGetErrorString(e) + " (" + file + ":" + std::to_string(line) + ")");
}



template <typename F>
static h2d_status guarded(F&& f)
{
    try {
        g_last_error.clear();
        f();
        return H2D_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return H2D_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return H2D_EINVAL;
    }
}

template <typename T>
static void up(DBuf<T>& d, const std::vector<T>& h, hipStream_t s)
{
    d.alloc(std::max<size_t>(h.size(), 1));
    if (!h.empty()) HIPCK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

static void check_kernel(const h2d_kernel* k)
{
    if (!k) fail(H2D_EINVAL, "kernel is NULL");
    if (k->kind < H2D_K_LOG || k->kind > H2D_K_SEP) fail(H2D_EINVAL, "unknown kernel kind");
    if (k->diag_mode < H2D_DIAG_REPLACE || k->diag_mode > H2D_DIAG_FORMULA) fail(H2D_EINVAL, "unknown diagonal rule");
    if ((k->kind == H2D_K_MQ || k->kind == H2D_K_GAUSS || k->kind == H2D_K_PHI1 || k->kind == H2D_K_PHI2) &&
        !(k->c > 0.0))
        fail(H2D_EINVAL, "shape parameter c must be > 0");
    if (k->kind == H2D_K_PHI1 && k->c >= 1.0) fail(H2D_EINVAL, "phi_1 needs 0 < a < 1");
    if (k->kind == H2D_K_SEP && !(k->c >= 0.0 && k->c <= 64.0)) fail(H2D_EINVAL, "separable rank must be in [0, 64]");
    if ((k->kind == H2D_K_LOG || k->kind == H2D_K_INVR) && k->diag_mode != H2D_DIAG_REPLACE)
        fail(H2D_EINVAL, "log and 1/r are singular at r = 0: use the REPLACE diagonal rule");
    if (!std::isfinite(k->c) || !std::isfinite(k->diag_value)) fail(H2D_EINVAL, "non-finite kernel parameter");
}

// Symmetric sharing needs a symmetric kernel, a balanced tree and FP64
// factors only.
static void check_symmetric(int32_t kind, bool adaptive, uint32_t prec_mask)
{
    if (kind == H2D_K_SEP) fail(H2D_EUNSUPPORTED, "the separable test kernel is not symmetric");
    if (adaptive) fail(H2D_EUNSUPPORTED, "symmetric sharing needs a balanced tree");
    if (prec_mask & ~1u) fail(H2D_EUNSUPPORTED, "symmetric handles keep FP64 factors only");
}

// ---------------------------------------------------------------------
// Export / import ("H2DX" version 1)
// ---------------------------------------------------------------------
struct File {
    FILE* f = nullptr;
    explicit File(const char* path, const char* mode) : f(std::fopen(path, mode))
    {
        if (!f) fail(H2D_EINVAL, std::string("cannot open ") + path);
    }
    ~File() { if (f) std::fclose(f); }
    template <typename T>
    void w(const T* p, size_t n) { if (n && std::fwrite(p, sizeof(T), n, f) != n) fail(H2D_EINVAL, "write failed"); }
    template <typename T>
    void w1(T v) { w(&v, 1); }
    template <typename T>
    void r(T* p, size_t n) { if (n && std::fread(p, sizeof(T), n, f) != n) fail(H2D_EINVAL, "truncated file"); }
    template <typename T>
    T r1() { T v; r(&v, 1); return v; }
};

// U of blocks at levels 1..kappa-1 is stored tiled by the boxes of level
// kappa - 1 (see the pack kernel).  Convert between that layout and plain
// column-major m x k; to_tiled selects the direction.
static void retile_u(const Handle& H, int level, int64_t row0, int64_t m, int64_t k, const double* in, double* out,
                     bool to_tiled)
{
    if (H.kappa < 2 || level > H.kappa - 1) {
        std::memcpy(out, in, sizeof(double) * (size_t)(m * k));
        return;
    }
    const Level& T = H.lev[H.kappa - 1];
    auto it = std::lower_bound(T.h_begin.begin(), T.h_begin.end(), (int32_t)row0);
    for (int64_t p = it - T.h_begin.begin(); p < T.nbox && T.h_begin[p] < row0 + m; ++p) {
        const int64_t pb = T.h_begin[p] - row0, pc = T.h_count[p];
        for (int64_t q = 0; q < k; ++q)
            for (int64_t i = 0; i < pc; ++i) {
                const int64_t plain = q * m + pb + i, tiled = k * pb + q * pc + i;
                if (to_tiled) out[tiled] = in[plain];
                else out[plain] = in[tiled];
            }
    }
}

template <typename T>
static std::vector<T> dl(const T* d, size_t n)
{
    std::vector<T> h(n);
    if (n) HIPCK(hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost));
    return h;
}

static void export_handle(Handle& H, const char* path, uint32_t flags)
{
    const bool fac = flags & 1u;
    File F(path, "wb");
    F.w("H2DX", 4);
    F.w1<uint32_t>(H.adaptive ? 2u : 1u);   // version 2: adaptive tree, blocks carry their box levels
    F.w1<uint32_t>(fac ? 1u : 0u);
    F.w1<uint32_t>(0);
    F.w1<int64_t>(H.n);
    F.w1<int32_t>(H.kappa);
    F.w1<int32_t>(H.leaf_max);
    F.w1<double>(H.R);
    F.w1<double>(H.tol);
    F.w1<int32_t>(H.kern.kind);
    F.w1<int32_t>(H.kern.diag_mode);
    F.w1<double>(H.kern.c);
    F.w1<double>(H.kern.diag_value);
    auto xy = dl(H.xy.p, (size_t)(2 * H.n));
    F.w(xy.data(), xy.size());
    std::vector<int64_t> p64(H.h_perm.begin(), H.h_perm.end());
    F.w(p64.data(), p64.size());
    for (int l = 0; l <= H.kappa; ++l) {
        const Level& L = H.lev[l];
        F.w1<int64_t>(L.nbox);
        F.w(L.h_key.data(), L.h_key.size());
        std::vector<int64_t> b(L.h_begin.begin(), L.h_begin.end()), c(L.h_count.begin(), L.h_count.end()),
            p(L.h_parent.begin(), L.h_parent.end());
        F.w(b.data(), b.size());
        F.w(c.data(), c.size());
        F.w(p.data(), p.size());
    }
    const Level& LL = H.lev[H.kappa];
    std::vector<double> U, V, D;
    if (fac) { U = dl(H.U64.p, H.u_elems); V = dl(H.V64.p, H.v_elems); D = dl(H.D64.p, H.d_elems); }
    F.w1<int64_t>((int64_t)H.h_near_src.size());
    if (H.adaptive) {
        // near CSR over leaf numbers; the file names (level, box) of both leaves
        const int64_t nleaf = (int64_t)H.h_leaf_level.size();
        for (int64_t x = 0; x < nleaf; ++x)
            for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
                const int32_t y = H.h_near_src[q];
                F.w1<int32_t>(H.h_leaf_level[x]);
                F.w1<int32_t>(H.h_leaf_level[y]);
                F.w1<int64_t>(H.h_leaf_box[x]);
                F.w1<int64_t>(H.h_leaf_box[y]);
                if (fac) F.w(D.data() + H.h_near_off[q], (size_t)H.h_leaf_count[x] * H.h_leaf_count[y]);
            }
    } else {
        std::vector<double> Dt;
        for (int64_t x = 0; x < LL.nbox; ++x)
            for (int32_t q = H.h_near_ptr[x]; q < H.h_near_ptr[x + 1]; ++q) {
                const int32_t y = H.h_near_src[q];
                F.w1<int64_t>(x);
                F.w1<int64_t>(y);
                if (!fac) continue;
                const int64_t mx = LL.h_count[x], my = LL.h_count[y];
                if (H.symmetric && y < x) {   // the owner's block (rows of y), transposed
                    Dt.resize((size_t)(mx * my));
                    for (int64_t j = 0; j < my; ++j)
                        for (int64_t i = 0; i < mx; ++i) Dt[j * mx + i] = D[H.h_near_off[q] + i * my + j];
                    F.w(Dt.data(), Dt.size());
                } else {
                    F.w(D.data() + H.h_near_off[q], (size_t)(mx * my));
                }
            }
    }
    F.w1<int64_t>(H.n_il);
    std::vector<double> Vc, Uc;
    for (int64_t b = 0; b < H.n_il; ++b) {
        const Level& L = H.lev[H.h_il_level[b]];
        int64_t m = L.h_count[H.h_il_tgt[b]], n = H.lev[il_src_level(H, b)].h_count[H.h_il_src[b]], k = H.h_il_k[b];
        F.w1<int32_t>(H.h_il_level[b]);
        F.w1<int32_t>(H.h_il_kind[b]);
        if (H.adaptive) {
            F.w1<int32_t>(il_src_level(H, b));
            F.w1<int32_t>(0);
        }
        F.w1<int64_t>(H.h_il_tgt[b]);
        F.w1<int64_t>(H.h_il_src[b]);
        F.w1<int64_t>(k);
        if (!fac) continue;
        if (H.h_il_kind[b] == kDense) {
            if (H.symmetric && H.h_il_tgt[b] > H.h_il_src[b]) {
                Uc.resize((size_t)(m * n));   // the owner's block (n x m), transposed
                for (int64_t j = 0; j < n; ++j)
                    for (int64_t i = 0; i < m; ++i) Uc[j * m + i] = D[H.h_il_off[b] + i * n + j];
                F.w(Uc.data(), Uc.size());
            } else {
                F.w(D.data() + H.h_il_off[b], (size_t)(m * n));
            }
        } else if (H.symmetric) {
            // both factors in the U pool, each laid out by its own box
            const Level& Ls = H.lev[il_src_level(H, b)];
            Uc.resize((size_t)(m * k));
            retile_u(H, H.h_il_level[b], L.h_begin[H.h_il_tgt[b]], m, k, U.data() + H.h_il_off[b], Uc.data(), false);
            F.w(Uc.data(), Uc.size());
            Vc.resize((size_t)(n * k));
            retile_u(H, H.h_il_level[b], Ls.h_begin[H.h_il_src[b]], n, k, U.data() + H.h_il_voff[b], Vc.data(), false);
            F.w(Vc.data(), Vc.size());
        } else {
            Uc.resize((size_t)(m * k));
            if (H.adaptive) std::memcpy(Uc.data(), U.data() + H.h_il_off[b], sizeof(double) * Uc.size());
            else retile_u(H, H.h_il_level[b], L.h_begin[H.h_il_tgt[b]], m, k, U.data() + H.h_il_off[b], Uc.data(), false);
            F.w(Uc.data(), Uc.size());
            Vc.resize((size_t)(n * k));
            for (int64_t j = 0; j < n; ++j)
                for (int64_t q = 0; q < k; ++q) Vc[q * n + j] = V[H.h_il_voff[b] + j * k + q];
            F.w(Vc.data(), Vc.size());
        }
    }
}

static void import_handle(Handle& H, const char* path, hipStream_t s, uint32_t prec_mask)
{
    File F(path, "rb");
    char magic[4];
    F.r(magic, 4);
    if (std::memcmp(magic, "H2DX", 4) != 0) fail(H2D_EINVAL, "not an H2DX file");
    uint32_t version = F.r1<uint32_t>(), flags = F.r1<uint32_t>();
    (void)F.r1<uint32_t>();
    if (version != 1 && version != 2) fail(H2D_EINVAL, "unsupported H2DX version");
    H.adaptive = version == 2;
    if (!(flags & 1u)) fail(H2D_EINVAL, "file holds no factors");
    H.n = F.r1<int64_t>();
    H.kappa = F.r1<int32_t>();
    H.leaf_max = F.r1<int32_t>();
    H.R = F.r1<double>();
    H.tol = F.r1<double>();
    H.kern.kind = F.r1<int32_t>();
    H.kern.diag_mode = F.r1<int32_t>();
    H.kern.c = F.r1<double>();
    H.kern.diag_value = F.r1<double>();
    if (H.n < 1 || H.n >= (int64_t)1 << 31 || H.kappa < 0 || H.kappa > kMaxLevel) fail(H2D_EINVAL, "bad header");
    const int64_t n = H.n;
    std::vector<double> xy((size_t)(2 * n));
    F.r(xy.data(), xy.size());
    std::vector<int64_t> p64((size_t)n);
    F.r(p64.data(), p64.size());
    {   // perm must be a permutation of [0, n): it drives every gather and scatter
        std::vector<uint8_t> seen((size_t)n, 0);
        for (int64_t i = 0; i < n; ++i) {
            if (p64[i] < 0 || p64[i] >= n || seen[p64[i]]) fail(H2D_EINVAL, "perm is not a permutation of [0, n)");
            seen[p64[i]] = 1;
        }
    }
    H.h_perm.assign(p64.begin(), p64.end());
    for (int l = 0; l <= H.kappa; ++l) {
        Level& L = H.lev[l];
        L.nbox = F.r1<int64_t>();
        if (L.nbox < 1 || L.nbox > n) fail(H2D_EINVAL, "bad level table");
        L.h_key.resize(L.nbox);
        F.r(L.h_key.data(), L.nbox);
        std::vector<int64_t> b(L.nbox), c(L.nbox), p(L.nbox);
        F.r(b.data(), L.nbox); F.r(c.data(), L.nbox); F.r(p.data(), L.nbox);
        // the boxes of a level tile [0, n) in key order (an adaptive tree:
        // lie in [0, n) in key order without overlapping, the leaves above
        // them filling the gaps), each non-empty, and lie inside their
        // parent (key >> 2 is the parent's key)
        int64_t next = 0;
        for (int64_t x = 0; x < L.nbox; ++x) {
            const bool key_ok = (l == 0 ? L.h_key[x] == 0 : (uint64_t)L.h_key[x] < ((uint64_t)1 << (2 * l))) &&
                                (x == 0 || L.h_key[x] > L.h_key[x - 1]);
            const bool place_ok = H.adaptive ? b[x] >= next : b[x] == next;
            if (!key_ok || !place_ok || c[x] < 1 || c[x] > n - b[x]) fail(H2D_EINVAL, "bad level table");
            next = b[x] + c[x];
            if (l > 0) {
                const Level& P = H.lev[l - 1];
                if (p[x] < 0 || p[x] >= P.nbox || P.h_key[p[x]] != (L.h_key[x] >> 2) || b[x] < P.h_begin[p[x]] ||
                    b[x] + c[x] > (int64_t)P.h_begin[p[x]] + P.h_count[p[x]])
                    fail(H2D_EINVAL, "bad parent in level table");
            }
        }
        if (next != n && !(H.adaptive && l > 0)) fail(H2D_EINVAL, "level table does not cover the points");
        L.h_begin.assign(b.begin(), b.end());
        L.h_count.assign(c.begin(), c.end());
        L.h_parent.assign(p.begin(), p.end());
    }
    const Level& LL = H.lev[H.kappa];
    // adaptive trees: leaves are the boxes without children at any level,
    // numbered in tree order
    std::vector<std::vector<int32_t>> leafno(H.kappa + 1);
    if (H.adaptive) {
        std::vector<std::pair<int32_t, std::pair<int32_t, int32_t>>> lv;
        for (int l = 0; l <= H.kappa; ++l) {
            std::vector<int32_t> nch(H.lev[l].nbox, 0);
            if (l < H.kappa)
                for (int32_t p : H.lev[l + 1].h_parent) nch[p]++;
            leafno[l].assign(H.lev[l].nbox, -1);
            for (int64_t b = 0; b < H.lev[l].nbox; ++b)
                if (!nch[b]) lv.push_back({H.lev[l].h_begin[b], {l, (int32_t)b}});
        }
        std::sort(lv.begin(), lv.end());
        int64_t next = 0;
        for (size_t q = 0; q < lv.size(); ++q) {
            const int l = lv[q].second.first, b = lv[q].second.second;
            leafno[l][b] = (int32_t)q;
            H.h_leaf_level.push_back(l);
            H.h_leaf_box.push_back(b);
            H.h_leaf_begin.push_back(H.lev[l].h_begin[b]);
            H.h_leaf_count.push_back(H.lev[l].h_count[b]);
            if (H.lev[l].h_begin[b] != next) fail(H2D_EINVAL, "the leaves do not tile the points");
            next += H.lev[l].h_count[b];
        }
        if (next != n) fail(H2D_EINVAL, "the leaves do not tile the points");
        // a split box's children fill it exactly
        for (int l = 0; l < H.kappa; ++l) {
            std::vector<int64_t> filled(H.lev[l].nbox, 0);
            for (int64_t c = 0; c < H.lev[l + 1].nbox; ++c) filled[H.lev[l + 1].h_parent[c]] += H.lev[l + 1].h_count[c];
            for (int64_t b = 0; b < H.lev[l].nbox; ++b)
                if (filled[b] != 0 && filled[b] != H.lev[l].h_count[b]) fail(H2D_EINVAL, "children do not fill their box");
        }
    }
    const int64_t nleaf = H.adaptive ? (int64_t)H.h_leaf_level.size() : LL.nbox;
    // near blocks, grouped by target leaf
    int64_t nn = F.r1<int64_t>();
    std::vector<double> D;
    H.h_near_ptr.assign(nleaf + 1, 0);
    H.h_near_src.resize(nn);
    H.h_near_off.resize(nn);
    std::vector<int64_t> ntgt(nn);
    for (int64_t q = 0; q < nn; ++q) {
        int64_t t, u, mt, mu;
        if (H.adaptive) {
            const int32_t tl = F.r1<int32_t>(), sl = F.r1<int32_t>();
            const int64_t tb = F.r1<int64_t>(), sb = F.r1<int64_t>();
            if (tl < 0 || tl > H.kappa || sl < 0 || sl > H.kappa || tb < 0 || tb >= H.lev[tl].nbox || sb < 0 ||
                sb >= H.lev[sl].nbox || leafno[tl][tb] < 0 || leafno[sl][sb] < 0)
                fail(H2D_EINVAL, "bad near block");
            t = leafno[tl][tb];
            u = leafno[sl][sb];
            mt = H.h_leaf_count[t];
            mu = H.h_leaf_count[u];
        } else {
            t = F.r1<int64_t>();
            u = F.r1<int64_t>();
            if (t < 0 || t >= LL.nbox || u < 0 || u >= LL.nbox) fail(H2D_EINVAL, "bad near block");
            mt = LL.h_count[t];
            mu = LL.h_count[u];
        }
        // version 1 lists near blocks by target; version 2 in (target level,
        // target, source level, source) order, regrouped by target leaf below
        if (!H.adaptive && q > 0 && t < ntgt[q - 1]) fail(H2D_EINVAL, "near blocks not grouped by target");
        ntgt[q] = t;
        H.h_near_src[q] = (int32_t)u;
        H.h_near_off[q] = (int64_t)D.size();
        const size_t e = (size_t)mt * (size_t)mu;
        const size_t o = D.size();
        D.resize(o + e);
        F.r(D.data() + o, e);
        H.h_near_ptr[t + 1]++;
    }
    for (int64_t x = 0; x < nleaf; ++x) H.h_near_ptr[x + 1] += H.h_near_ptr[x];
    if (H.adaptive) {   // stable regrouping by target leaf (tree order)
        std::vector<int64_t> ord(nn);
        for (int64_t q = 0; q < nn; ++q) ord[q] = q;
        std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return ntgt[a] < ntgt[b]; });
        std::vector<int32_t> src2(nn);
        std::vector<int64_t> off2(nn);
        for (int64_t q = 0; q < nn; ++q) { src2[q] = H.h_near_src[ord[q]]; off2[q] = H.h_near_off[ord[q]]; }
        H.h_near_src.swap(src2);
        H.h_near_off.swap(off2);
    }
    // interaction-list blocks
    H.n_il = F.r1<int64_t>();
    const int64_t nil = H.n_il;
    H.h_il_level.resize(nil); H.h_il_kind.resize(nil); H.h_il_tgt.resize(nil); H.h_il_src.resize(nil);
    H.h_il_k.resize(nil); H.h_il_off.resize(nil); H.h_il_voff.assign(nil, 0);
    std::vector<double> U, V;
    std::vector<double> Vc;
    std::vector<std::pair<int64_t, int64_t>> pending_tile;   // (block, U offset): retiled once levels are known
    if (H.adaptive) H.h_il_slevel.resize(nil);
    for (int64_t b = 0; b < nil; ++b) {
        int32_t lv = F.r1<int32_t>(), kind = F.r1<int32_t>(), sl = lv;
        if (H.adaptive) {
            sl = F.r1<int32_t>();
            (void)F.r1<int32_t>();
            if (sl < 1 || sl > H.kappa) fail(H2D_EINVAL, "bad block source level");
            H.h_il_slevel[b] = sl;
        }
        int64_t t = F.r1<int64_t>(), u = F.r1<int64_t>(), k = F.r1<int64_t>();
        if (lv < 1 || lv > H.kappa) fail(H2D_EINVAL, "bad block level");
        const Level& L = H.lev[lv];
        const Level& Ls = H.lev[sl];
        if (t < 0 || t >= L.nbox || u < 0 || u >= Ls.nbox || k < 0) fail(H2D_EINVAL, "bad block");
        if (b > 0 && (lv < H.h_il_level[b - 1] || (lv == H.h_il_level[b - 1] && t < H.h_il_tgt[b - 1])))
            fail(H2D_EINVAL, "blocks not in (level, target) order");
        int64_t m = L.h_count[t], nc = Ls.h_count[u];
        H.h_il_level[b] = lv; H.h_il_kind[b] = kind; H.h_il_tgt[b] = (int32_t)t; H.h_il_src[b] = (int32_t)u;
        H.h_il_k[b] = (int32_t)k;
        if (kind == kDense) {
            H.h_il_off[b] = (int64_t)D.size();
            size_t o = D.size();
            D.resize(o + (size_t)(m * nc));
            F.r(D.data() + o, (size_t)(m * nc));
        } else if (kind == kLowRank) {
            if (k > std::min(m, nc)) fail(H2D_EINVAL, "rank exceeds block size");
            H.h_il_off[b] = (int64_t)U.size();
            H.h_il_voff[b] = (int64_t)V.size();
            size_t o = U.size();
            U.resize(o + (size_t)(m * k));
            F.r(U.data() + o, (size_t)(m * k));
            pending_tile.push_back({b, (int64_t)o});
            Vc.resize((size_t)(nc * k));
            F.r(Vc.data(), Vc.size());
            size_t ov = V.size();
            V.resize(ov + (size_t)(nc * k));
            for (int64_t j = 0; j < nc; ++j)
                for (int64_t q = 0; q < k; ++q) V[ov + j * k + q] = Vc[q * nc + j];
        } else {
            fail(H2D_EINVAL, "bad block kind");
        }
    }
    {
        std::vector<double> tmp;
        for (auto& pt : pending_tile) {
            const int64_t b = pt.first, o = pt.second;
            const Level& L = H.lev[H.h_il_level[b]];
            const int64_t m = L.h_count[H.h_il_tgt[b]], k = H.h_il_k[b];
            if (H.adaptive) continue;   // adaptive trees keep U plain column-major
            tmp.assign(U.begin() + o, U.begin() + o + m * k);
            retile_u(H, H.h_il_level[b], L.h_begin[H.h_il_tgt[b]], m, k, tmp.data(), U.data() + o, true);
        }
    }
    // CSR of IL blocks per level box
    for (int l = 0; l <= H.kappa; ++l) H.lev[l].h_il_ptr.assign(H.lev[l].nbox + 1, 0);
    {
        std::vector<int64_t> cnt;
        for (int64_t b = 0; b < nil; ++b) H.lev[H.h_il_level[b]].h_il_ptr[H.h_il_tgt[b] + 1]++;
        int64_t run = 0;
        for (int l = 1; l <= H.kappa; ++l) {
            Level& L = H.lev[l];
            L.h_il_ptr[0] = (int32_t)run;
            for (int64_t x = 0; x < L.nbox; ++x) L.h_il_ptr[x + 1] += L.h_il_ptr[x];
            run = L.h_il_ptr[L.nbox];
        }
    }
    if (H.symmetric) {
        if (H.adaptive) fail(H2D_EUNSUPPORTED, "symmetric sharing needs a balanced tree");
        check_symmetric(H.kern.kind, false, prec_mask);
        symmetrize_import(H, U, V, D);
    }
    // device copies (the file is checked in full before the first HIP call)
    HIPCK(hipGetDevice(&H.device));
    up(H.xy, xy, s);
    std::vector<double> xyt((size_t)(2 * n));
    for (int64_t i = 0; i < n; ++i) { xyt[2 * i] = xy[2 * H.h_perm[i]]; xyt[2 * i + 1] = xy[2 * H.h_perm[i] + 1]; }
    up(H.xyt, xyt, s);
    up(H.perm, H.h_perm, s);
    for (int l = 0; l <= H.kappa; ++l) {
        Level& L = H.lev[l];
        up(L.key, L.h_key, s);
        up(L.begin, L.h_begin, s);
        up(L.count, L.h_count, s);
        up(L.parent, L.h_parent, s);
    }
    H.u_elems = (int64_t)U.size(); H.v_elems = (int64_t)V.size(); H.d_elems = (int64_t)D.size();
    up(H.U64, U, s);
    up(H.V64, V, s);
    up(H.D64, D, s);
    HIPCK(hipStreamSynchronize(s));
}

}  // namespace h2d

using namespace h2d;

extern "C" {

struct h2d_s {
    Handle h;
};

const char* h2d_last_error(void) { return g_last_error.c_str(); }

h2d_status h2d_build(const double* xy, int64_t n, const h2d_kernel* kernel, int32_t leaf_max, double tol,
                     uint32_t prec_mask, void* stream, h2d_t* out)
{
    return guarded([&] {
        if (!out) fail(H2D_EINVAL, "out is NULL");
        *out = nullptr;
        if (!xy) fail(H2D_EINVAL, "xy is NULL");
        if (n < 1 || n >= ((int64_t)1 << 31)) fail(H2D_EINVAL, "n must be in [1, 2^31)");
        if (leaf_max < 1) fail(H2D_EINVAL, "leaf_max must be >= 1");
        if (!(tol >= 0.0) || !std::isfinite(tol)) fail(H2D_EINVAL, "tol must be finite and >= 0");
        if (prec_mask & ~(7u | H2D_BUILD_ADAPTIVE | H2D_BUILD_SYMMETRIC))
            fail(H2D_EINVAL, "unknown precision or build bits");
        const bool adaptive = (prec_mask & H2D_BUILD_ADAPTIVE) != 0;
        const bool symmetric = (prec_mask & H2D_BUILD_SYMMETRIC) != 0;
        prec_mask &= 7u;
        if (adaptive && (prec_mask & ~1u))
            fail(H2D_EUNSUPPORTED, "half-precision pools are not built for adaptive trees");
        check_kernel(kernel);
        if (symmetric) check_symmetric(kernel->kind, adaptive, prec_mask);
        hipStream_t s = (hipStream_t)stream;
        auto t0 = std::chrono::steady_clock::now();
        auto up_ = std::make_unique<h2d_s>();
        Handle& H = up_->h;
        HIPCK(hipGetDevice(&H.device));
        H.n = n; H.leaf_max = leaf_max; H.tol = tol;
        H.adaptive = adaptive;
        H.symmetric = symmetric;
        H.kern = KernelParams{kernel->kind, kernel->diag_mode, kernel->c, kernel->diag_value};
        H.xy.alloc((size_t)(2 * n));
        HIPCK(hipMemcpyAsync(H.xy.p, xy, sizeof(double) * 2 * n, hipMemcpyDefault, s));
        build_tree_and_lists(H, s);
        build_factors(H, s);
        if (adaptive) finalize_adaptive(H, s);
        else if (symmetric) finalize_symmetric(H, s);
        else finalize(H, s);
        make_half_pools(H, prec_mask, s);
        HIPCK(hipStreamSynchronize(s));
        H.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = up_.release();
    });
}

h2d_status h2d_matvec(h2d_t H, const double* x, double* y, int32_t nrhs, int64_t ld, int32_t prec, void* stream)
{
    return guarded([&] {
        if (!H || !x || !y) fail(H2D_EINVAL, "NULL argument");
        if (nrhs < 1 || ld < H->h.n) fail(H2D_EINVAL, "need nrhs >= 1 and ld >= n");
        if (prec < H2D_P_FP64 || prec > H2D_P_BF16) fail(H2D_EINVAL, "unknown precision");
        if (!(H->h.prec_mask & H2D_PREC_BIT(prec))) fail(H2D_EUNSUPPORTED, "precision was not built for this handle");
        launch_matvec(H->h, x, y, nrhs, ld, prec, (hipStream_t)stream);
    });
}

h2d_status h2d_matvec_noalloc(h2d_t H, const double* x, double* y, int32_t prec, void* stream)
{
    return guarded([&] {
        if (!H || !x || !y) fail(H2D_EINVAL, "NULL argument");
        if (prec < H2D_P_FP64 || prec > H2D_P_BF16) fail(H2D_EINVAL, "unknown precision");
        if (!(H->h.prec_mask & H2D_PREC_BIT(prec))) fail(H2D_EUNSUPPORTED, "precision was not built for this handle");
        if (H->h.symmetric) fail(H2D_EUNSUPPORTED, "symmetric handles have no fixed-array product");
        launch_matvec_noalloc(H->h, x, y, prec, (hipStream_t)stream);
    });
}

h2d_status h2d_solve(h2d_t H, const double* b, double* x, double rtol, const h2d_solve_opts* opts,
                     h2d_solve_info* info, void* stream)
{
    h2d_status st = H2D_OK;
    h2d_status g = guarded([&] {
        if (!H || !b || !x || !opts) fail(H2D_EINVAL, "NULL argument");
        if (!(rtol > 0.0)) fail(H2D_EINVAL, "rtol must be > 0");
        if (H->h.adaptive && (opts->mode != H2D_SOLVE_PLAIN || opts->precond != H2D_PC_NONE))
            fail(H2D_EUNSUPPORTED, "adaptive trees solve with plain FP64 GMRES only");
        if (H->h.symmetric && (opts->mode != H2D_SOLVE_PLAIN || opts->precond != H2D_PC_NONE))
            fail(H2D_EUNSUPPORTED, "symmetric handles solve with plain FP64 GMRES only");
        if (opts->restart < 1 || opts->max_iter < 1) fail(H2D_EINVAL, "restart and max_iter must be >= 1");
        {   // x is zeroed before b is read: the two must not overlap
            const uintptr_t b0 = (uintptr_t)b, x0 = (uintptr_t)x, len = sizeof(double) * (uintptr_t)H->h.n;
            if (b0 < x0 + len && x0 < b0 + len) fail(H2D_EINVAL, "b and x overlap");
        }
        st = solve(H->h, b, x, rtol, *opts, info, (hipStream_t)stream);
    });
    return g != H2D_OK ? g : st;
}

h2d_status h2d_info(h2d_t H, h2d_stats* s)
{
    return guarded([&] {
        if (!H || !s) fail(H2D_EINVAL, "NULL argument");
        const Handle& h = H->h;
        std::memset(s, 0, sizeof(*s));
        s->n = h.n; s->kappa = h.kappa; s->leaf_max = h.leaf_max; s->R = h.R; s->tol = h.tol;
        s->n_near = (int64_t)h.h_near_src.size(); s->n_il = h.n_il; s->n_il_dense = h.n_il_dense;
        s->max_rank = h.max_rank; s->sum_rank = h.sum_rank;
        s->u_elems = h.u_elems; s->v_elems = h.v_elems; s->d_elems = h.d_elems;
        s->alg_bytes_fp64 = h.alg_bytes_fp64; s->alg_bytes_half = h.alg_bytes_half; s->flops = h.flops;
        s->build_seconds = h.build_seconds; s->prec_mask = h.prec_mask;
    });
}

h2d_status h2d_export(h2d_t H, const char* path, uint32_t flags)
{
    return guarded([&] {
        if (!H || !path) fail(H2D_EINVAL, "NULL argument");
        export_handle(H->h, path, flags);
    });
}

h2d_status h2d_import(const char* path, uint32_t prec_mask, void* stream, h2d_t* out)
{
    return guarded([&] {
        if (!path || !out) fail(H2D_EINVAL, "NULL argument");
        *out = nullptr;
        if (prec_mask & ~(7u | H2D_BUILD_SYMMETRIC)) fail(H2D_EINVAL, "unknown precision bits");
        const bool symmetric = (prec_mask & H2D_BUILD_SYMMETRIC) != 0;
        prec_mask &= 7u;
        hipStream_t s = (hipStream_t)stream;
        auto t0 = std::chrono::steady_clock::now();
        auto up_ = std::make_unique<h2d_s>();
        Handle& H = up_->h;
        H.symmetric = symmetric;
        import_handle(H, path, s, prec_mask);
        if (H.adaptive) {
            if (prec_mask & ~1u) fail(H2D_EUNSUPPORTED, "half-precision pools are not built for adaptive trees");
            finalize_adaptive(H, s);
        } else if (symmetric) {
            finalize_symmetric(H, s);
        } else {
            finalize(H, s);
        }
        make_half_pools(H, prec_mask, s);
        HIPCK(hipStreamSynchronize(s));
        H.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = up_.release();
    });
}

h2d_status h2d_profile_enable(h2d_t H, int32_t on)
{
    return guarded([&] {
        if (!H) fail(H2D_EINVAL, "NULL handle");
        profile_enable(H->h, on != 0);
    });
}

h2d_status h2d_profile_read(h2d_t H, h2d_profile* out)
{
    return guarded([&] {
        if (!H || !out) fail(H2D_EINVAL, "NULL argument");
        profile_read(H->h, out);
    });
}

h2d_status h2d_bj_setup(h2d_t H, void* stream)
{
    return guarded([&] {
        if (!H) fail(H2D_EINVAL, "NULL handle");
        if (H->h.adaptive) fail(H2D_EUNSUPPORTED, "block-Jacobi is not built for adaptive trees");
        if (H->h.symmetric) fail(H2D_EUNSUPPORTED, "block-Jacobi is not built for symmetric handles");
        bj_setup(H->h, (hipStream_t)stream);
    });
}

h2d_status h2d_precond_apply(h2d_t H, int32_t precond, const double* r, double* z, void* stream)
{
    return guarded([&] {
        if (!H || !r || !z) fail(H2D_EINVAL, "NULL argument");
        precond_apply(H->h, precond, r, z, (hipStream_t)stream);
    });
}

h2d_status h2d_mlp_train(h2d_t H, const h2d_mlp_train_opts* opts, h2d_mlp_train_info* info, void* stream)
{
    return guarded([&] {
        if (!H || !opts) fail(H2D_EINVAL, "NULL argument");
        if (H->h.adaptive) fail(H2D_EUNSUPPORTED, "the learned preconditioner is not built for adaptive trees");
        if (H->h.symmetric) fail(H2D_EUNSUPPORTED, "the learned preconditioner is not built for symmetric handles");
        if (opts->n_solves < 1 || opts->steps < 0 || opts->batch < 1 || !(opts->lr > 0.f) ||
            (opts->target == H2D_MLP_TARGET_GLOBAL && !(opts->solve_tol > 0.0)) ||
            (opts->target != H2D_MLP_TARGET_LEAF && opts->target != H2D_MLP_TARGET_GLOBAL &&
             opts->target != H2D_MLP_TARGET_PATCH) ||
            (opts->input != H2D_MLP_INPUT_LEAF && opts->input != H2D_MLP_INPUT_PATCH) ||
            (opts->input == H2D_MLP_INPUT_PATCH && opts->target == H2D_MLP_TARGET_LEAF))
            fail(H2D_EINVAL, "bad training options");
        mlp_train(H->h, *opts, info, (hipStream_t)stream);
    });
}

h2d_status h2d_mlp_weights(h2d_t H, float* out, const float* in, double* scale, void* stream)
{
    return guarded([&] {
        if (!H) fail(H2D_EINVAL, "NULL handle");
        mlp_weights(H->h, out, in, scale, (hipStream_t)stream);
    });
}

h2d_status h2d_mlp_loss_grad(const float* W, const float* X, const float* T, const float* M, int32_t B, float* loss,
                             float* grad, void* stream)
{
    return guarded([&] {
        if (!W || !X || !T || !M || !loss || !grad || B < 1) fail(H2D_EINVAL, "bad argument");
        *loss = mlp_loss_grad(W, X, T, M, B, grad, (hipStream_t)stream);
    });
}

h2d_status h2d_autotune(h2d_t H, int32_t nrhs, void* stream, int32_t* chosen, float* ms)
{
    return guarded([&] {
        if (!H || nrhs < 1) fail(H2D_EINVAL, "bad argument");
        if (H->h.adaptive) fail(H2D_EUNSUPPORTED, "tile tuning is not built for adaptive trees");
        if (H->h.symmetric) fail(H2D_EUNSUPPORTED, "tile tuning is not built for symmetric handles");
        autotune(H->h, nrhs, (hipStream_t)stream, chosen, ms);
    });
}

h2d_status h2d_set_item_rows(h2d_t H, int32_t which, int32_t rows, void* stream)
{
    return guarded([&] {
        if (!H) fail(H2D_EINVAL, "NULL handle");
        if (H->h.adaptive) fail(H2D_EUNSUPPORTED, "tile sizes are fixed for adaptive trees");
        if (H->h.symmetric) fail(H2D_EUNSUPPORTED, "tile sizes are fixed for symmetric handles");
        if (which == H2D_TILE_A_ROWS) {
            if (rows < 16 || rows > kPhaseARows) fail(H2D_EINVAL, "phase-A item rows must lie in 16..512");
        } else if (which == H2D_TILE_MR_ROWS) {
            if (rows < 16 || rows > kMrRowsMax || rows % 16)
                fail(H2D_EINVAL, "chunk rows must be 16..512, multiple of 16");
        } else if (which == H2D_TILE_B1_ROWS) {
            if (rows != 16 && rows != 32 && rows != 64) fail(H2D_EINVAL, "phase-B1 slice rows must be 16, 32 or 64");
        } else if (which == H2D_TILE_B2_ROWS) {
            if (rows != 16 && rows != 32 && rows != 64) fail(H2D_EINVAL, "phase-B2 chunk rows must be 16, 32 or 64");
        } else {
            fail(H2D_EINVAL, "unknown tile parameter");
        }
        set_item_rows(H->h, which, rows, (hipStream_t)stream);
    });
}

struct h2d_batch_s {
    Batch* b;
};

h2d_status h2d_batch_create(h2d_t const* handles, int32_t count, int32_t nrhs, double* const* x, double* const* y,
                            const int64_t* ld, h2d_batch_t* out)
{
    return guarded([&] {
        if (!handles || !x || !y || !ld || !out || count < 1 || nrhs < 1) fail(H2D_EINVAL, "bad argument");
        *out = nullptr;
        std::vector<Handle*> hs(count);
        for (int i = 0; i < count; ++i) {
            if (!handles[i] || !x[i] || !y[i] || ld[i] < handles[i]->h.n) fail(H2D_EINVAL, "bad batch member");
            if (handles[i]->h.adaptive) fail(H2D_EUNSUPPORTED, "adaptive trees are not batched");
            if (handles[i]->h.symmetric) fail(H2D_EUNSUPPORTED, "symmetric handles are not batched");
            hs[i] = &handles[i]->h;
        }
        auto* r = new h2d_batch_s{batch_create(hs.data(), count, nrhs, x, y, ld)};
        *out = r;
    });
}

h2d_status h2d_batch_launch(h2d_batch_t B, void* stream)
{
    return guarded([&] {
        if (!B) fail(H2D_EINVAL, "NULL batch");
        batch_launch(B->b, (hipStream_t)stream);
    });
}

void h2d_batch_destroy(h2d_batch_t B)
{
    if (!B) return;
    (void)hipDeviceSynchronize();
    batch_destroy(B->b);
    delete B;
}

void h2d_destroy(h2d_t H)
{
    if (!H) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(H->h.device);
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : H->h.prof_ev) (void)hipEventDestroy(e);
    delete H;
    (void)hipSetDevice(dev);
}

}  // extern "C"
