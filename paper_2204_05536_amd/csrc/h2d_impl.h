// Internal declarations of the HODLR2D library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "../../include/h2d.h"

namespace h2d {

constexpr int kMaxLevel = 16;      // Morton keys are 2 x 16 bits
constexpr int kWave = 64;
constexpr int kAcaRankCap = 256;   // ACA scratch columns per block
constexpr int kPhaseARows = 512;   // V rows per phase-A work item (x slice staged in LDS)
constexpr int kHalfSlack = 16;     // zeroed elements after every half-precision pool
constexpr int kMrRowsMax = 512;    // multi-RHS phase-A source chunk: 512 rows x 16 x 8 bytes = 64 KiB of LDS

// Error carried from deep inside the library to the C ABI.
struct Error {
    h2d_status code;
    std::string msg;
};

[[noreturn]] void fail(h2d_status code, const std::string& msg);
// Test hook: while the environment variable H2D_TEST_FAIL_ALLOC holds k >= 1,
// the k-th device allocation (counted while the variable is set) fails as an
// out-of-memory would, so the ENOMEM paths can be exercised from the host.
bool forced_alloc_failure();
void check_hip(hipError_t e, const char* what, const char* file, int line);
#define HIPCK(x) ::h2d::check_hip((x), #x, __FILE__, __LINE__)

// Block kinds.
enum : int32_t { kLowRank = 0, kDense = 1 };

// Device buffer with RAII.
template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) { reset(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { reset(); }
    void alloc(size_t count)
    {
        reset();
        if (count == 0) return;
        if (forced_alloc_failure())
            fail(H2D_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed (forced by H2D_TEST_FAIL_ALLOC)");
        hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(H2D_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
        }
        n = count;
    }
    // keep the buffer when it already holds count elements
    void reserve(size_t count)
    {
        if (n < count) alloc(count);
    }
    void reset()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// Per-level box table (tree order).  Device arrays, host mirrors.
struct Level {
    int64_t nbox = 0;
    DBuf<uint32_t> key;       // Morton key, ascending
    DBuf<int32_t> begin;      // first point (tree order)
    DBuf<int32_t> count;      // points in the box
    DBuf<int32_t> parent;     // box index at level - 1
    DBuf<int32_t> il_ptr;     // CSR into the IL block table (nbox + 1), absolute block index
    std::vector<uint32_t> h_key;
    std::vector<int32_t> h_begin, h_count, h_parent, h_il_ptr;
};

// Phase-B block descriptor: the rows of one target box read as
// base[q * ld + r] (column-major, ld = target box size), q < |cols|.
//   cols > 0: low rank, base = U pool + off, the multiplier vector is
//             t pool + tsrc (k = cols entries)
//   cols < 0: dense, base = D pool + off, multiplier = x (tree order)
//             + tsrc (n = -cols entries)
struct BDesc {
    int64_t off;
    int32_t cols;
    int32_t tsrc;
};

// One entry of a phase-B table of the half pools: a 4-column group of one
// tile (half U and D tiles are stored as [column quads][rows][4]), as one
// row slice of a box multiplies it.  Row i of the slice's box reads the
// group's 4 values at pool + 4 q + 4 i.
//   src >= 0: low rank; U pool, multiplier values t pool + src ..
//   src < 0:  dense; D pool, multiplier values x (tree order) + ~src ..
//   sc:       the dense block's scale (1 for low rank)
//   nv:       columns of the group inside the block, 1 .. 4
struct QEnt {
    uint32_t q;
    int32_t src;
    float sc;
    int32_t nv;
};


// Phase A on the half pools, grouped by source box: rows of one source
// box's wide V (the V of all its low-rank blocks side by side, w columns,
// stored in groups of 4 rows: element (j, c) at ((j / 4) ws + c) 4 + j mod
// 4, ws = w rounded up to 16).
struct AWDesc {
    int64_t voff;     // element offset of the item's first row group
    int32_t rows, w;  // rows (at most kPhaseARows, a multiple of 4 unless last), width
    int32_t x0;       // tree index of the item's first row
    int32_t map;      // offset of the source box's column map (t index of each column)
    int32_t part;     // -1: t written through the map; else offset of the item's partial row
    int32_t ws;       // row-group width
};
// A source box whose phase-A rows were split: t[map[c]] = sum of the
// nparts partial rows (w values each, consecutive from pbeg).
struct AWRed {
    int32_t pbeg, nparts, w, map;
};

// Blocks whose phase-A work was split: t = sum of consecutive partials.
struct RDesc {
    int32_t tout;     // t pool offset
    int32_t k;
    int32_t pbeg;     // first partial offset
    int32_t nparts;   // partials, each k long, stored consecutively
};

// Phase A on the FP64 pools (single- and multi-RHS), grouped by source
// box: one work item is a row range [j0, j1) of one source box (points
// col0 + j0 .. col0 + j1 - 1 in tree order) and the blocks b0 .. b1 - 1 of
// the block list that share it; the item is chunk p of the source's rows.
struct MRItem {
    int32_t col0, j0, j1, b0, b1, p;
};
// One low-rank block of the list: V offset, rank, and where T goes
// (out >= 0: t pool offset; out < 0: partial pool offset -out - 1 of chunk 0,
// chunk p at that + p k).
struct MRBlk {
    int64_t voff;
    int32_t k, out;
    int32_t blk, pad;   // the block
};

// Static data of one instance for the table-driven multi-RHS kernels (a
// single product uses a table of one; a batch, one entry per instance).
// Device addresses are stored as integers: the kernels turn them back into
// global-memory pointers (a pointer read from memory would be a generic one
// to the compiler, with flat loads and per-lane address arithmetic).
struct MRInst {
    uint64_t U, V, D;                 // factor pools: const double*, or the FP16/BF16 pools
    uint64_t xs, tp, pp, yp, yl;      // work vectors: double*, or float* with the half pools
    uint64_t items, blks, ritems, b1items, bil, bnear;
    uint64_t near_ptr, iperm;         // const int32_t*
    uint64_t lvl;                     // const int32_t* const*: begin, count, parent, il_ptr (kMaxLevel + 1 each)
    uint64_t scale, diag;             // half pools: const float* block scales (IL blocks, then near blocks) and
                                      // self-block diagonal (tree order); unused in FP64
    uint64_t qp1, qt1, qp2, qt2;      // half pools: phase-B tables (CSR pointers, entries); unused in FP64
    uint64_t rchunks;                 // const int2*: (split block, first element) of each 64-value reduction chunk
    int32_t n, kappa, has_b1, n_il;
};
// Right-hand sides of one instance: x and y column-major, leading dimension ld.
struct MRIo {
    uint64_t x, y;
    int64_t ld;
};

// Symmetric handles (one factor pair per interaction-list pair): one
// descriptor per interaction-list block, read by the slice walks above the
// leaf level.
//   cols > 0: low rank; the block's target-side factor at U pool + off,
//             column-major and tiled by the boxes one level above the
//             leaves; tsrc: this block's t; part: partial pool offset of
//             the partner block's t (slice s of the target box at
//             part + s cols)
//   cols < 0: dense, D pool + off, multiplier xs + tsrc; part = 0: the
//             block itself, column-major (ld = target box size); part = 1:
//             a mirror, its owner's block read transposed (row-major, ld =
//             source box size)
//   cols = 0: rank 0, nothing to do
struct SDesc {
    int64_t off;
    int32_t cols, tsrc;
    int64_t part;
};
// A leaf-level pair {X, Y}, X < Y, applied in both directions from one read
// by the wave of leaf Y.  k > 0: low rank, F_X (|X| x k) at U pool + a and
// F_Y (|Y| x k) at U pool + b, column-major; k < 0: dense, D (|X| x |Y|,
// column-major) at D pool + a.  X's rows (first tree row x0, mx of them)
// of the product go to the slot pool at slot.
struct LPair {
    int64_t a, b, slot;
    int32_t x0, mx, k, pad;
};

struct KernelParams {
    int32_t kind;
    int32_t diag_mode;
    double c;
    double diag_value;
};

struct MlpState;

struct Handle {
    int device = 0;
    int64_t n = 0;
    int32_t kappa = 0, leaf_max = 0;
    double R = 1.0, tol = 0.0;
    KernelParams kern{};
    uint32_t prec_mask = 1;
    double build_seconds = 0.0;

    DBuf<double> xy;        // caller order, n x 2
    DBuf<double> xyt;       // tree order, n x 2
    DBuf<int32_t> perm;     // tree position -> caller index
    std::vector<int32_t> h_perm;
    std::vector<double> h_xy;
    Level lev[kMaxLevel + 1];

    // near field (leaf level): CSR by target leaf box
    DBuf<int32_t> near_ptr;
    std::vector<int32_t> h_near_ptr, h_near_src;
    std::vector<int64_t> h_near_off;  // D pool offsets

    // adaptive tree (leaves at several levels): leaves numbered in tree
    // order; the near CSR (near_ptr, h_near_src) is then over leaf numbers
    bool adaptive = false;
    std::vector<int32_t> h_leaf_level, h_leaf_box, h_leaf_begin, h_leaf_count;
    DBuf<int32_t> leaf_level, leaf_box;
    DBuf<int2> ad_items;         // adaptive phase-B work: (leaf, first row of a 64-row chunk)
    int64_t n_ad_items = 0;

    // interaction-list block table, (level, tgt, src) order (adaptive:
    // (target level, tgt, source level, src); h_il_slevel holds the source
    // levels, empty for a balanced tree where they equal h_il_level)
    int64_t n_il = 0;
    std::vector<int32_t> h_il_level, h_il_tgt, h_il_src, h_il_kind, h_il_k, h_il_slevel;
    std::vector<int64_t> h_il_off;    // U pool offset (low rank) or D pool offset (dense)
    std::vector<int64_t> h_il_voff;   // V pool offset (low rank)
    std::vector<int32_t> h_il_toff;   // t pool offset (low rank)

    // factor pools: FP64 offsets as in the block table; the half pools have
    // layouts and offsets of their own (below)
    int64_t u_elems = 0, v_elems = 0, d_elems = 0, t_elems = 0, p_elems = 0;
    DBuf<double> U64, V64, D64;
    DBuf<__half> U16, V16, D16;
    DBuf<__hip_bfloat16> Ub16, Vb16, Db16;
    // half U and D pools in the quad layout (every tile [column quads][rows][4],
    // columns padded to a multiple of 4, the rows of the U tiles above the
    // leaf level to a multiple of 16) at offsets of their own, and the
    // phase-B tables: per box one level above the leaves (qt1) and per leaf
    // (qt2), every 4-column group its row slices multiply, in summation order
    std::vector<int64_t> h_il_off16;
    int64_t u16_elems = 0, d16_elems = 0;
    DBuf<int32_t> qp1, qp2;
    DBuf<QEnt> qt1, qt2;
    DBuf<float> scale16;     // per-block scale of the half pools (IL blocks, then near blocks)
    DBuf<float> diag32;      // self-block diagonal (tree order) for the half pools
    int64_t max_rank = 0, sum_rank = 0, n_il_dense = 0;

    // matvec schedule
    DBuf<BDesc> bnear, bil;  // phase-B descriptors: near blocks, IL blocks
    DBuf<MRItem> a_items;       // single-RHS phase A: source-box chunks (FP64 pools)
    DBuf<MRBlk> a_blks;         // their blocks (V offset, rank, t or partial offset)
    // FP16/BF16 V pools, grouped by source box: for every source box (per
    // level) the V of its low-rank blocks side by side (w columns in table
    // order), stored in groups of 4 rows: element (j, c) of the box at
    // ((j / 4) ws + c) 4 + j mod 4 (ws = w rounded up to 16), the rows
    // padded with zeros to a multiple of 4, so 4 rows of one column are
    // one aligned 8-byte group and every row group starts on a 128-byte
    // line.
    // Phase-A items over these rows (aw_items), the column maps to the t
    // pool (aw_map), the reductions of split source boxes (aw_red) and
    // their partial rows (p16_elems values).
    int64_t v16_elems = 0, p16_elems = 0;
    DBuf<AWDesc> aw_items;
    DBuf<int32_t> aw_map;
    DBuf<AWRed> aw_red;
    DBuf<int2> aw_rchunks;     // 16 right-hand sides: (reduction, first of its w x 16 values) per 64 values
    int64_t n_aw_items = 0, n_aw_red = 0, n_aw_rchunks = 0;
    int32_t aw_red_maxw = 0;   // widest split source box (columns)
    DBuf<RDesc> ritems;
    int64_t n_aitems = 0, n_ritems = 0;
    DBuf<int2> b1items;         // multi-RHS phase-B1 work: (box at level kappa - 1, first row of a 64-row chunk)
    int64_t n_b1 = 0;
    DBuf<int2> b1s_items;       // single-RHS phase-B1 work: (box, first row of a b1_rows-row slice)
    int64_t n_b1s = 0;
    int32_t b1_rows = 64;       // 16, 32 or 64 (tuned by h2d_autotune)
    bool b1_rows_set = false;   // b1_rows set by the caller or the tuner; else chosen from the box sizes
    DBuf<int2> b2items;         // single-RHS phase-B2 work: (leaf box, first row of a b2_rows-row chunk)
    int32_t b2_rows = 64;       // 16, 32 or 64 (tuned by h2d_autotune)
    int64_t n_b2 = 0;

    // multi-RHS work (blocks of 16 right-hand sides, point-major)
    DBuf<double> xs_mr, tp_mr, pp_mr, yp_mr, yl_mr;
    DBuf<const int32_t*> lvl_ptrs;   // begin, count, parent, il_ptr per level (device copies of the pointers)
    int mr_cap = 0;
    DBuf<MRItem> mr_items;           // multi-RHS phase-A items (source-grouped)
    DBuf<MRBlk> mr_blks;
    DBuf<RDesc> mr_ritems;           // their split-block reductions
    DBuf<int2> mr_rchunks;           // (reduction, first of its k x 16 values) per 64 values
    DBuf<int32_t> iperm;             // caller index -> tree position
    int64_t n_mr_items = 0, n_mr_ritems = 0, n_mr_rchunks = 0, mr_p_elems = 0;
    std::vector<int64_t> h_mr_work;  // work of each multi-RHS phase-A item, in schedule order
    DBuf<MRInst> mr_inst;            // this handle's entry for the table-driven kernels
    // the half-pool form (FP32 work vectors; phase A on the source-grouped
    // items, phase B on the tables), set up on the first half-precision
    // multi-RHS product
    DBuf<float> xs_mr32, tp_mr32, pp_mr32, yp_mr32, yl_mr32;
    DBuf<MRInst> mr_inst16;          // [FP16, BF16]
    int mr16_cap = 0;
    int32_t mr_rows = 256;           // source rows per multi-RHS phase-A item (tuned by h2d_autotune)
    int32_t a_rows = kPhaseARows;    // rows per phase-A work item (tuned by h2d_autotune)

    // work vectors
    DBuf<double> xs, tpool, ppool, ypart;    // FP64: x in tree order, t, partials, ancestor sums
    DBuf<float> xs32, tpool32, ppool32, ypart32;
    int64_t ws_nrhs = 0;

    // preconditioners
    DBuf<double> bj_lu;        // per leaf: LU of the self block, m x m column-major
    DBuf<int32_t> bj_piv;      // per tree row: pivot row chosen at that step of its leaf
    DBuf<int64_t> bj_off;      // per leaf: offset into bj_lu
    DBuf<int32_t> bj_big;      // leaves of more than 64 points (their own LU and solve kernels)
    int32_t n_bj_big = 0;
    bool bj_ready = false;
    // solver work space, kept between solves and grown on demand: Krylov
    // basis, preconditioned directions, vectors, dot-product partials, and
    // the refinement loop's residual, correction and product
    DBuf<double> gm_V, gm_Z, gm_w, gm_r, gm_y, gm_part, gm_dres, rf_r, rf_d, rf_w;
    std::shared_ptr<MlpState> mlp;

    // symmetric sharing (one factor pair per interaction-list pair): both
    // factors of a pair in the U pool (h_il_off: the block's target side,
    // h_il_voff: its source side); a mirror block (target index > source
    // index) points at its owner's factors with the roles swapped, and a
    // mirror leaf-level dense or near block at its owner's D
    bool symmetric = false;
    std::vector<int64_t> h_il_partner;          // block (level, src, tgt) of block (level, tgt, src)
    DBuf<SDesc> sdesc;
    DBuf<int32_t> s_mid[kMaxLevel + 1];         // per box: first block of its list with src > tgt
    DBuf<int32_t> s_first[kMaxLevel + 1];       // per box (+1): its first slice item
    DBuf<int2> s_items;                         // (box one level above the leaves, first row of a 64-row slice)
    DBuf<RDesc> s_red[4];                       // partial sums: mirrors' t (first walk; runs, then run sums), owners' t (second walk; same)
    DBuf<int32_t> s_lp_ptr, s_nslot;            // per leaf: its pairs {X < leaf}; its slot count
    DBuf<LPair> s_lp;
    DBuf<int64_t> s_self, s_slot_base;          // per leaf: self block offset; first slot
    DBuf<double> s_y, s_slots;                  // work: walk sums (2 n), leaf sums (2 n); slot pool
    int64_t n_s_items = 0, n_s_red[4] = {0, 0, 0, 0}, s_slot_elems = 0;

    double alg_bytes_fp64 = 0, alg_bytes_half = 0, flops = 0;
    double phase_bytes[2][5] = {{0}};   // [FP64, half][gather, A, reduce, B, combine]

    // profiling: 6 events per recorded matvec (around its 5 kernels)
    bool prof_on = false;
    int prof_prec = 0;
    std::vector<hipEvent_t> prof_ev;
    size_t prof_used = 0;
};

// kernels.hip
void finalize(Handle& H, hipStream_t s);
void launch_matvec(Handle& H, const double* x, double* y, int nrhs, int64_t ld, int prec, hipStream_t s);
void launch_matvec_mr(Handle& H, const double* x, double* y, int nrhs, int64_t ld, int prec, hipStream_t s);
// Multi-RHS state of H (schedule, work space, instance entry), built once.
void ensure_mr(Handle& H, hipStream_t s);
MRInst mr_inst_of(const Handle& H);
// Table-driven multi-RHS product of several instances at once (each
// instance at most once): the gather, phase A, reduction, phase B and
// scatter of every instance run as one launch each.
struct MRBatchPlan {
    DBuf<MRInst> insts;
    DBuf<MRIo> io;
    DBuf<int2> wg, wa, wr, wb1, wb2;   // work lists: (instance, item)
    int32_t ng = 0, nr = 0, nb1 = 0, nb2 = 0;
    std::vector<int32_t> a_rows, a_beg, a_cnt;   // phase A: one launch per source-chunk size (LDS need)
};
void mr_plan(MRBatchPlan& P, Handle* const* hs, const MRIo* io, int count, hipStream_t s);
void mr_plan_launch(const MRBatchPlan& P, int32_t r0, int32_t nr, hipStream_t s);
void ensure_workspace(Handle& H, int nrhs);
// Single-RHS product on the fixed per-GPU work array (no allocation).
size_t noalloc_bytes(const Handle& H, int prec);
void launch_matvec_noalloc(Handle& H, const double* x, double* y, int prec, hipStream_t s);
void profile_enable(Handle& H, bool on);
void profile_read(Handle& H, h2d_profile* out);

// build.hip
void build_tree_and_lists(Handle& H, hipStream_t s);
// Adaptive tree and block lists from the points sorted by (depth-16 key,
// caller index); host code (the rest of the build runs on the device).
void adaptive_tree_and_lists(Handle& H, const DBuf<uint32_t>& skey, const DBuf<int32_t>& sidx, hipStream_t s);
// Leaf arrays and per-level block CSR of an adaptive handle from its host
// tables (build and import).
void adaptive_index(Handle& H, hipStream_t s);
void finalize_adaptive(Handle& H, hipStream_t s);
// symmetric.hip
constexpr int kSymLeafMax = 64;   // leaf points a symmetric handle allows (one wave per leaf)
void symmetric_partners(Handle& H);
void finalize_symmetric(Handle& H, hipStream_t s);
void launch_matvec_symmetric(Handle& H, const double* x, double* y, int nrhs, int64_t ld, hipStream_t s);
// Host factor arrays of an imported ordered file (U tiled, V row-major, D)
// -> the symmetric layout; EINVAL unless every mirror is the exact
// transpose of its owner.
void symmetrize_import(Handle& H, std::vector<double>& U, std::vector<double>& V, std::vector<double>& D);
// Row -> (first row, size) of its box one level above the leaves.
void tile_map(const Handle& H, std::vector<int32_t>& tbeg, std::vector<int32_t>& tcnt);
inline int32_t il_src_level(const Handle& H, int64_t b) { return H.h_il_slevel.empty() ? H.h_il_level[b] : H.h_il_slevel[b]; }
void build_factors(Handle& H, hipStream_t s);
void make_half_pools(Handle& H, uint32_t mask, hipStream_t s);

// precond.hip, mlp.hip
void bj_setup(Handle& H, hipStream_t s);
void precond_apply(Handle& H, int pc, const double* r, double* z, hipStream_t s);
void mlp_apply(Handle& H, const double* r, double* z, hipStream_t s);
void mlp_train(Handle& H, const h2d_mlp_train_opts& o, h2d_mlp_train_info* info, hipStream_t s);
void mlp_weights(Handle& H, float* out, const float* in, double* scale, hipStream_t s);
float mlp_loss_grad(const float* W, const float* X, const float* T, const float* Mk, int32_t B, float* grad,
                    hipStream_t s);

// batch.hip
struct Batch;
Batch* batch_create(Handle** hs, int count, int nrhs, double* const* x, double* const* y, const int64_t* ld);
void batch_launch(Batch* B, hipStream_t s);
void batch_destroy(Batch* B);
void autotune(Handle& H, int nrhs, hipStream_t s, int32_t* chosen, float* ms_out);
void set_item_rows(Handle& H, int which, int32_t rows, hipStream_t s);

// solve.hip
h2d_status solve(Handle& H, const double* b, double* x, double rtol, const h2d_solve_opts& o,
                 h2d_solve_info* info, hipStream_t s);

// ---------------------------------------------------------------------
// Kernel function on the device (same definitions as the public header).
// ---------------------------------------------------------------------
__device__ __forceinline__ double phi_radial(const KernelParams& k, double r)
{
    switch (k.kind) {
    case H2D_K_LOG: return log(r);
    case H2D_K_INVR: return 1.0 / r;
    case H2D_K_MQ: { double s = r / k.c; return sqrt(1.0 + s * s); }
    case H2D_K_GAUSS: { double s = r / k.c; return exp(-(s * s)); }
    case H2D_K_PHI1: {
        double a = k.c;
        if (r >= a) return log(r) / log(a);
        double rl = (r > 0.0) ? r * log(r) : 0.0;
        return (rl - 1.0) / (a * log(a) - 1.0);
    }
    case H2D_K_PHI2: { double a = k.c; return (r >= a) ? a / r : r / a; }
    default: return 0.0;
    }
}

// Entry between target point (tx, ty) and source point (sx, sy); `same`
// is true when both are the same point index (the diagonal).
__device__ __forceinline__ double kernel_entry(const KernelParams& k, double tx, double ty, double sx,
                                               double sy, bool same)
{
    if (k.kind == H2D_K_SEP) {
        double a = 1.3 * tx + 0.7 * ty, b = 0.9 * sx - 1.1 * sy, v = 0.0;
        int rank = (int)k.c;
        for (int q = 0; q < rank; ++q) v += cos(q * a) * cos(q * b);
        if (same) {
            if (k.diag_mode == H2D_DIAG_REPLACE) return k.diag_value;
            if (k.diag_mode == H2D_DIAG_ADD) return v + k.diag_value;
        }
        return v;
    }
    if (same) {
        if (k.diag_mode == H2D_DIAG_REPLACE) return k.diag_value;
        if (k.diag_mode == H2D_DIAG_ADD) return phi_radial(k, 0.0) + k.diag_value;
        return phi_radial(k, 0.0);
    }
    double dx = tx - sx, dy = ty - sy;
    return phi_radial(k, sqrt(dx * dx + dy * dy));
}

}  // namespace h2d
