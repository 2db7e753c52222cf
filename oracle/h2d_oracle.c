/*
 * HODLR2D CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 implementation of what the HODLR2D
 * method computes (arxiv 2204.05536).  It exists to check the GPU library:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or helper with the library.
 *
 * What follows the paper, and where:
 *   kernel functions ...... Section 3 (log r), Section 5.1 eq. (1/r),
 *                           Section 5.2 (phi_1, phi_2, diagonal beta); the
 *                           multiquadric and Gaussian RBFs are standard
 *                           radial functions written from their definition.
 *   box B, subdivision .... Section 3 (half-open split [-1,0) x [-1,1] and
 *                           [0,1] x [-1,1]), Section 4 (quadtree, numbering
 *                           figure), Algorithm 1 (balanced tree, leaf boxes
 *                           hold at most N_max points).
 *   E_C, V_C, W_C ......... Section 4, Definitions of edge sharing, vertex
 *                           sharing and well separated clusters.
 *   clan set, I_C ......... Section 4, Definition of the clan set and
 *                           equation (4.2) for the interaction list.
 *   leaf dense blocks ..... Algorithm 1 (self + edge-sharing blocks).
 *   ACA ................... Algorithm 1 (low rank U V^T per interaction-list
 *                           pair); the paper cites partial-pivot adaptive
 *                           cross approximation without details, the
 *                           variant used is written out in orc_aca().
 *   matvec ................ Algorithm 2 (near field, then levels 1..kappa).
 *   symmetric sharing ..... Section 2.1 (Notations: the matrix is taken
 *                           symmetric): with a symmetric kernel the block
 *                           of (C', C) is the transpose of the block of
 *                           (C, C'); in that mode only the block whose
 *                           target box has the smaller index is compressed
 *                           and its mirror is its exact transpose.
 *   GMRES ................. Section 5 (restarted GMRES on the fast matvec).
 *
 * Parity pins for every function here live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LEVEL 16

enum { OK_LOG = 0, OK_INVR = 1, OK_MQ = 2, OK_GAUSS = 3, OK_PHI1 = 4, OK_PHI2 = 5, OK_SEP = 6 };
enum { OD_REPLACE = 0, OD_ADD = 1, OD_FORMULA = 2 };
enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 2, ORC_EDUP = 4, ORC_ENOCONV = 5, ORC_EDEPTH = 7 };
enum { BK_LOWRANK = 0, BK_DENSE = 1 };

typedef struct {
    int32_t kind;       /* OK_* */
    int32_t diag_mode;  /* OD_* */
    double c;           /* shape parameter: MQ / Gauss length, phi_1/phi_2 'a', separable rank */
    double diag_value;  /* replacement or shift on the diagonal */
} orc_kernel;

/* ------------------------------------------------------------------ */
/* Kernel entries                                                       */
/* ------------------------------------------------------------------ */

/* phi(r) for the radial kernels, r > 0 (or any r for MQ/Gauss). */
static double orc_phi(const orc_kernel* k, double r)
{
    switch (k->kind) {
    case OK_LOG: return log(r);
    case OK_INVR: return 1.0 / r;
    case OK_MQ: { double s = r / k->c; return sqrt(1.0 + s * s); }
    case OK_GAUSS: { double s = r / k->c; return exp(-(s * s)); }
    case OK_PHI1: {
        double a = k->c;
        if (r >= a) return log(r) / log(a);
        /* r log r -> 0 as r -> 0 */
        double rl = (r > 0.0) ? r * log(r) : 0.0;
        return (rl - 1.0) / (a * log(a) - 1.0);
    }
    case OK_PHI2: { double a = k->c; return (r >= a) ? a / r : r / a; }
    default: return NAN;
    }
}

/* A separable (non-radial) test kernel of exact rank c:
 * K(x, y) = sum_{q < c} cos(q (1.3 x1 + 0.7 x2)) cos(q (0.9 y1 - 1.1 y2)). */
static double orc_sep(int rank, const double* x, const double* y)
{
    double a = 1.3 * x[0] + 0.7 * x[1], b = 0.9 * y[0] - 1.1 * y[1], s = 0.0;
    for (int q = 0; q < rank; ++q) s += cos(q * a) * cos(q * b);
    return s;
}

/* Entry A(i, j) of the dense kernel matrix, i and j in the caller's point
 * numbering.  The diagonal is decided by index equality. */
double orc_entry(const orc_kernel* k, const double* xy, int64_t i, int64_t j)
{
    if (k->kind == OK_SEP) {
        double v = orc_sep((int)k->c, xy + 2 * i, xy + 2 * j);
        if (i == j) {
            if (k->diag_mode == OD_REPLACE) return k->diag_value;
            if (k->diag_mode == OD_ADD) return v + k->diag_value;
        }
        return v;
    }
    if (i == j) {
        if (k->diag_mode == OD_REPLACE) return k->diag_value;
        if (k->diag_mode == OD_ADD) return orc_phi(k, 0.0) + k->diag_value;
        return orc_phi(k, 0.0);
    }
    double dx = xy[2 * i] - xy[2 * j], dy = xy[2 * i + 1] - xy[2 * j + 1];
    return orc_phi(k, sqrt(dx * dx + dy * dy));
}

void orc_entries(const orc_kernel* k, const double* xy, const int64_t* I, const int64_t* J,
                 int64_t cnt, double* out)
{
    for (int64_t t = 0; t < cnt; ++t) out[t] = orc_entry(k, xy, I[t], J[t]);
}

/* y = A x with the dense definition, O(N^2).  rows == NULL: all rows. */
void orc_dense_rows(const orc_kernel* k, const double* xy, int64_t n, const int64_t* rows,
                    int64_t nrows, const double* x, double* y)
{
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t i = rows ? rows[t] : t;
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += orc_entry(k, xy, i, j) * x[j];
        y[t] = s;
    }
}

/* ------------------------------------------------------------------ */
/* Quadtree                                                             */
/* ------------------------------------------------------------------ */

/* Half side R of the box B = [-R, R]^2: the smallest power of two that is
 * >= max |coordinate| (R = 1 for every workload of the paper). */
double orc_box_radius(const double* xy, int64_t n)
{
    double m = 0.0;
    for (int64_t i = 0; i < 2 * n; ++i) if (fabs(xy[i]) > m) m = fabs(xy[i]);
    if (!(m > 0.0)) return 1.0;
    double R = 1.0;
    while (R < m) R *= 2.0;
    while (R * 0.5 >= m) R *= 0.5;
    return R;
}

/* Cell index along one axis at level l by repeated halving: a coordinate
 * below the midpoint goes to the lower half [lo, mid), otherwise to the upper
 * half [mid, hi] (closed only at the top edge of B). */
static uint32_t orc_cell(double v, double R, int level)
{
    double lo = -R, hi = R;
    uint32_t c = 0;
    for (int l = 0; l < level; ++l) {
        double mid = 0.5 * (lo + hi);
        if (v < mid) { c = 2 * c; hi = mid; }
        else { c = 2 * c + 1; lo = mid; }
    }
    return c;
}

/* Morton key of cell (ix, iy) at level l: base-4 digits m = 2*ybit + xbit,
 * most significant digit = level 1. */
static uint32_t orc_morton(uint32_t ix, uint32_t iy, int level)
{
    uint32_t key = 0;
    for (int b = level - 1; b >= 0; --b)
        key = 4 * key + 2 * ((iy >> b) & 1u) + ((ix >> b) & 1u);
    return key;
}

static void orc_demorton(uint32_t key, int level, uint32_t* ix, uint32_t* iy)
{
    uint32_t x = 0, y = 0;
    for (int b = 0; b < level; ++b) {
        uint32_t d = (key >> (2 * b)) & 3u;
        x |= (d & 1u) << b;
        y |= (d >> 1) << b;
    }
    *ix = x; *iy = y;
}

/* The paper's box id at a level: the same base-4 digits, each mapped
 * 0->0 (bottom-left), 1->1 (bottom-right), 3->2 (top-right), 2->3 (top-left). */
uint32_t orc_paper_id(uint32_t ix, uint32_t iy, int level)
{
    uint32_t id = 0;
    for (int b = level - 1; b >= 0; --b) {
        uint32_t xb = (ix >> b) & 1u, yb = (iy >> b) & 1u, d;
        if (!yb) d = xb ? 1u : 0u;
        else d = xb ? 2u : 3u;
        id = 4 * id + d;
    }
    return id;
}

uint32_t orc_morton_key(uint32_t ix, uint32_t iy, int level) { return orc_morton(ix, iy, level); }

typedef struct { uint32_t key; int64_t idx; } orc_kv;

static int orc_kv_cmp(const void* a, const void* b)
{
    const orc_kv* x = (const orc_kv*)a;
    const orc_kv* y = (const orc_kv*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

typedef struct {
    int64_t nbox;
    uint32_t* key;    /* Morton key, ascending */
    int64_t* begin;   /* first point (tree order) */
    int64_t* count;   /* number of points */
    int64_t* parent;  /* index of the parent box at level-1 (-1 at level 0) */
    int64_t* child0;  /* first child at level+1 */
    int64_t* nchild;  /* number of children (0: the box is a leaf) */
} orc_level_t;

typedef struct {
    int32_t level, kind;     /* level of the target box */
    int32_t slevel, pad;     /* level of the source box (= level in a balanced tree) */
    int64_t tgt, src, k;     /* boxes are indices into their level's box table */
    double* U;               /* m x k column-major (kind LOWRANK) */
    double* V;               /* n x k column-major (kind LOWRANK) */
    double* D;               /* m x n column-major (kind DENSE) */
} orc_block;

typedef struct {
    int64_t n;
    int32_t leaf_max, kappa;
    double R, tol;
    orc_kernel kern;
    double* xy;              /* copy of the points, caller order */
    int64_t* perm;           /* tree position -> caller index */
    orc_level_t lev[ORC_MAX_LEVEL + 1];
    int64_t n_near, n_il;
    orc_block* near;         /* leaf level: self + edge sharers, (tgt, src) order */
    orc_block* il;           /* interaction-list blocks, (level, tgt, src) order */
    int factors;             /* 0 = structure only */
    int adaptive;            /* 1: adaptive tree (leaves at several levels) */
    int symmetric;           /* 1: the block of (s, t), t > s, is the transpose of (t, s) */
} orc_h;

static void orc_free_levels(orc_h* h)
{
    for (int l = 0; l <= ORC_MAX_LEVEL; ++l) {
        free(h->lev[l].key); free(h->lev[l].begin); free(h->lev[l].count); free(h->lev[l].parent);
        free(h->lev[l].child0); free(h->lev[l].nchild);
        memset(&h->lev[l], 0, sizeof(h->lev[l]));
    }
}

void orc_free(orc_h* h)
{
    if (!h) return;
    for (int64_t b = 0; b < h->n_near; ++b) { free(h->near[b].D); }
    for (int64_t b = 0; b < h->n_il; ++b) { free(h->il[b].U); free(h->il[b].V); free(h->il[b].D); }
    free(h->near); free(h->il);
    orc_free_levels(h);
    free(h->perm); free(h->xy);
    free(h);
}

/* Index of the box with a given key at a level, or -1 when that box holds
 * no points. */
static int64_t orc_find(const orc_level_t* L, uint32_t key)
{
    int64_t lo = 0, hi = L->nbox - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (L->key[mid] == key) return mid;
        if (L->key[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static int orc_i64_cmp(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* child0 / nchild of every box from the parent indices of the level below
 * (children of a box are consecutive there, in key order). */
static void orc_child_ranges(orc_h* h)
{
    for (int l = 0; l <= h->kappa; ++l) {
        orc_level_t* L = &h->lev[l];
        L->child0 = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L->nbox + 1));
        L->nchild = (int64_t*)calloc((size_t)(L->nbox + 1), sizeof(int64_t));
        for (int64_t b = 0; b < L->nbox; ++b) L->child0[b] = -1;
        if (l == h->kappa) continue;
        const orc_level_t* C = &h->lev[l + 1];
        for (int64_t c = 0; c < C->nbox; ++c) {
            int64_t p = C->parent[c];
            if (L->nchild[p] == 0) L->child0[p] = c;
            L->nchild[p]++;
        }
    }
}

/* Balanced quadtree (Algorithm 1): kappa is the smallest depth at which no
 * box holds more than leaf_max points.  Points are ordered by (leaf Morton
 * key, caller index); each level lists its non-empty boxes in key order. */
static int orc_tree(orc_h* h)
{
    int64_t n = h->n;
    orc_kv* kv = (orc_kv*)malloc(sizeof(orc_kv) * (size_t)(n > 0 ? n : 1));
    if (!kv) return ORC_ENOMEM;
    int kappa = -1;
    for (int l = 0; l <= ORC_MAX_LEVEL; ++l) {
        for (int64_t i = 0; i < n; ++i) {
            kv[i].key = orc_morton(orc_cell(h->xy[2 * i], h->R, l), orc_cell(h->xy[2 * i + 1], h->R, l), l);
            kv[i].idx = i;
        }
        qsort(kv, (size_t)n, sizeof(orc_kv), orc_kv_cmp);
        int64_t maxrun = 0, run = 0;
        for (int64_t i = 0; i < n; ++i) {
            run = (i > 0 && kv[i].key == kv[i - 1].key) ? run + 1 : 1;
            if (run > maxrun) maxrun = run;
        }
        if (maxrun <= h->leaf_max) { kappa = l; break; }
    }
    if (kappa < 0) { free(kv); return ORC_EDEPTH; }
    h->kappa = kappa;
    h->perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) h->perm[i] = kv[i].idx;
    /* level tables from the sorted leaf keys */
    for (int l = 0; l <= kappa; ++l) {
        orc_level_t* L = &h->lev[l];
        int shift = 2 * (kappa - l);
        int64_t nb = 0;
        for (int64_t i = 0; i < n; ++i)
            if (i == 0 || (kv[i].key >> shift) != (kv[i - 1].key >> shift)) ++nb;
        L->nbox = nb;
        L->key = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nb + 1));
        L->begin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb + 1));
        L->count = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb + 1));
        L->parent = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb + 1));
        int64_t b = -1;
        for (int64_t i = 0; i < n; ++i) {
            uint32_t kk = kv[i].key >> shift;
            if (i == 0 || kk != (kv[i - 1].key >> shift)) {
                ++b; L->key[b] = kk; L->begin[b] = i; L->count[b] = 0;
            }
            L->count[b]++;
        }
    }
    for (int l = 0; l <= kappa; ++l) {
        orc_level_t* L = &h->lev[l];
        for (int64_t b = 0; b < L->nbox; ++b)
            L->parent[b] = (l == 0) ? -1 : orc_find(&h->lev[l - 1], L->key[b] >> 2);
    }
    free(kv);
    orc_child_ranges(h);
    return ORC_OK;
}

/* Adaptive quadtree.  The paper notes (end of Section 4) that the method
 * carries over to a non-balanced, adaptive tree with small changes; the
 * reading taken here: a box is subdivided exactly when it holds more than
 * N_max points, so the leaves are the boxes of at most N_max points whose
 * parent holds more, at whatever level that happens (the same half-open
 * cells, depth at most 16).  Points are ordered by (leaf, caller index),
 * leaves in Morton order of their cells; every level lists its boxes in key
 * order.  When every box above some depth holds more than N_max points and
 * every box at it at most N_max, this is the balanced tree of Algorithm 1. */
static int orc_tree_adaptive(orc_h* h)
{
    int64_t n = h->n;
    orc_kv* kv = (orc_kv*)malloc(sizeof(orc_kv) * (size_t)(n > 0 ? n : 1));
    if (!kv) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        kv[i].key = orc_morton(orc_cell(h->xy[2 * i], h->R, ORC_MAX_LEVEL),
                               orc_cell(h->xy[2 * i + 1], h->R, ORC_MAX_LEVEL), ORC_MAX_LEVEL);
        kv[i].idx = i;
    }
    qsort(kv, (size_t)n, sizeof(orc_kv), orc_kv_cmp);
    /* level 0: the root */
    orc_level_t* L0 = &h->lev[0];
    L0->nbox = 1;
    L0->key = (uint32_t*)calloc(1, sizeof(uint32_t));
    L0->begin = (int64_t*)calloc(1, sizeof(int64_t));
    L0->count = (int64_t*)malloc(sizeof(int64_t));
    L0->parent = (int64_t*)malloc(sizeof(int64_t));
    L0->count[0] = n; L0->parent[0] = -1;
    int kappa = 0;
    for (int l = 0; l < ORC_MAX_LEVEL; ++l) {
        const orc_level_t* P = &h->lev[l];
        int shift = 2 * (ORC_MAX_LEVEL - (l + 1));
        /* children of the boxes above N_max: runs of equal level-(l+1) key */
        int64_t nb = 0;
        for (int64_t b = 0; b < P->nbox; ++b) {
            if (P->count[b] <= h->leaf_max) continue;
            for (int64_t i = P->begin[b]; i < P->begin[b] + P->count[b]; ++i)
                if (i == P->begin[b] || (kv[i].key >> shift) != (kv[i - 1].key >> shift)) ++nb;
        }
        if (nb == 0) break;
        orc_level_t* L = &h->lev[l + 1];
        L->nbox = nb;
        L->key = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)nb);
        L->begin = (int64_t*)malloc(sizeof(int64_t) * (size_t)nb);
        L->count = (int64_t*)malloc(sizeof(int64_t) * (size_t)nb);
        L->parent = (int64_t*)malloc(sizeof(int64_t) * (size_t)nb);
        int64_t c = -1;
        for (int64_t b = 0; b < P->nbox; ++b) {
            if (P->count[b] <= h->leaf_max) continue;
            for (int64_t i = P->begin[b]; i < P->begin[b] + P->count[b]; ++i) {
                uint32_t kk = kv[i].key >> shift;
                if (i == P->begin[b] || kk != (kv[i - 1].key >> shift)) {
                    ++c; L->key[c] = kk; L->begin[c] = i; L->count[c] = 0; L->parent[c] = b;
                }
                L->count[c]++;
            }
        }
        kappa = l + 1;
    }
    /* a box still above N_max at depth 16 cannot be split further */
    const orc_level_t* D = &h->lev[kappa];
    for (int64_t b = 0; b < D->nbox; ++b)
        if (D->count[b] > h->leaf_max && kappa == ORC_MAX_LEVEL) { free(kv); return ORC_EDEPTH; }
    h->kappa = kappa;
    h->perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) h->perm[i] = kv[i].idx;
    free(kv);
    orc_child_ranges(h);
    /* inside each leaf, caller order */
    for (int l = 0; l <= kappa; ++l) {
        const orc_level_t* L = &h->lev[l];
        for (int64_t b = 0; b < L->nbox; ++b)
            if (L->nchild[b] == 0)
                qsort(h->perm + L->begin[b], (size_t)L->count[b], sizeof(int64_t), orc_i64_cmp);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Neighbour sets and interaction lists (Section 4 definitions)         */
/* ------------------------------------------------------------------ */

/* Relation of two boxes at the same level: 0 same box, 1 edge sharing,
 * 2 vertex sharing, 3 well separated (no common boundary point). */
static int orc_relation(uint32_t ka, uint32_t kb, int level)
{
    uint32_t ax, ay, bx, by;
    orc_demorton(ka, level, &ax, &ay);
    orc_demorton(kb, level, &bx, &by);
    int64_t dx = (int64_t)ax - (int64_t)bx, dy = (int64_t)ay - (int64_t)by;
    if (dx < 0) dx = -dx;
    if (dy < 0) dy = -dy;
    if (dx == 0 && dy == 0) return 0;
    if (dx + dy == 1) return 1;
    if (dx == 1 && dy == 1) return 2;
    return 3;
}

/* Keys of the boxes that share an edge with box `key` (inside B). */
static int orc_edge_keys(uint32_t key, int level, uint32_t* out)
{
    uint32_t x, y, side = 1u << level;
    int c = 0;
    orc_demorton(key, level, &x, &y);
    if (x > 0) out[c++] = orc_morton(x - 1, y, level);
    if (x + 1 < side) out[c++] = orc_morton(x + 1, y, level);
    if (y > 0) out[c++] = orc_morton(x, y - 1, level);
    if (y + 1 < side) out[c++] = orc_morton(x, y + 1, level);
    return c;
}

static int orc_u32_cmp(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Interaction list of box `key` at `level` (Section 4):
 *   clan(C) = siblings(C) U children(E_parent(C)),
 *   I_C     = (clan n V_C) U (clan n W_C),
 * returned as ascending keys.  Returns the count. */
int orc_interaction_list(uint32_t key, int level, uint32_t* out)
{
    if (level < 1) return 0;
    uint32_t clan[24];
    int nc = 0;
    uint32_t pk = key >> 2;
    for (uint32_t d = 0; d < 4; ++d)
        if (4 * pk + d != key) clan[nc++] = 4 * pk + d;               /* siblings */
    uint32_t pe[4];
    int npe = orc_edge_keys(pk, level - 1, pe);                       /* E_parent */
    for (int e = 0; e < npe; ++e)
        for (uint32_t d = 0; d < 4; ++d) clan[nc++] = 4 * pe[e] + d;  /* their children */
    int c = 0;
    for (int t = 0; t < nc; ++t) {
        int rel = orc_relation(key, clan[t], level);
        if (rel == 2 || rel == 3) out[c++] = clan[t];                 /* V or W */
    }
    qsort(out, (size_t)c, sizeof(uint32_t), orc_u32_cmp);
    return c;
}

/* Edge-sharing set E_C as ascending keys (Section 4). */
int orc_edge_list(uint32_t key, int level, uint32_t* out)
{
    int c = orc_edge_keys(key, level, out);
    qsort(out, (size_t)c, sizeof(uint32_t), orc_u32_cmp);
    return c;
}

/* Classify two same-level boxes (exported for tests). */
int orc_box_relation(uint32_t ka, uint32_t kb, int level) { return orc_relation(ka, kb, level); }

/* Admissibility of two boxes of any levels (adaptive tree): their closed
 * squares, compared on the grid of the finer level, have at most one point
 * in common (a shared vertex, or none).  For boxes of one level this is
 * "vertex sharing or well separated", the compressed pairs of Section 4;
 * the same box and edge sharers are not admissible. */
int orc_admissible(int la, uint32_t ka, int lb, uint32_t kb)
{
    int L = la > lb ? la : lb;
    uint32_t ax, ay, bx, by;
    orc_demorton(ka, la, &ax, &ay);
    orc_demorton(kb, lb, &bx, &by);
    int64_t sa = (int64_t)1 << (L - la), sb = (int64_t)1 << (L - lb);
    int64_t ax0 = ax * sa, ax1 = ax0 + sa, ay0 = ay * sa, ay1 = ay0 + sa;
    int64_t bx0 = bx * sb, bx1 = bx0 + sb, by0 = by * sb, by1 = by0 + sb;
    int64_t wx = (ax1 < bx1 ? ax1 : bx1) - (ax0 > bx0 ? ax0 : bx0);
    int64_t wy = (ay1 < by1 ? ay1 : by1) - (ay0 > by0 ? ay0 : by0);
    if (wx < 0 || wy < 0) return 1;
    return wx == 0 && wy == 0;
}

static int orc_block_cmp(const void* x, const void* y)
{
    const orc_block* a = (const orc_block*)x;
    const orc_block* b = (const orc_block*)y;
    if (a->level != b->level) return a->level < b->level ? -1 : 1;
    if (a->tgt != b->tgt) return a->tgt < b->tgt ? -1 : 1;
    if (a->slevel != b->slevel) return a->slevel < b->slevel ? -1 : 1;
    if (a->src != b->src) return a->src < b->src ? -1 : 1;
    return 0;
}

typedef struct { int32_t la, lb; int64_t a, b; } orc_pair;

static void orc_push_block(orc_block** arr, int64_t* cnt, int64_t* cap, int la, int64_t a, int lb, int64_t b)
{
    if (*cnt == *cap) {
        *cap = *cap ? 2 * *cap : 1024;
        *arr = (orc_block*)realloc(*arr, sizeof(orc_block) * (size_t)*cap);
    }
    orc_block* B = &(*arr)[(*cnt)++];
    memset(B, 0, sizeof(*B));
    B->level = la; B->slevel = lb; B->tgt = a; B->src = b; B->kind = BK_DENSE;
}

/* Blocks of the adaptive tree, found by descending pairs of boxes from
 * (root, root), the pair form of the Section 4 construction: a pair of
 * distinct admissible boxes is one compressed block; a pair of leaves
 * that is not admissible (the same leaf, or leaves sharing a segment) is
 * a dense near-field block; any other pair is replaced by the pairs of
 * their children (only the non-leaf side is split when one side is a
 * leaf).  On a balanced tree this gives exactly the interaction lists of
 * every level and the self + edge-sharing leaf blocks. */
static void orc_lists_adaptive(orc_h* h)
{
    int64_t nn = 0, ncap = 0, ni = 0, icap = 0, sp = 0, scap = 1024;
    orc_pair* st = (orc_pair*)malloc(sizeof(orc_pair) * (size_t)scap);
    h->near = NULL; h->il = NULL;
    st[sp++] = (orc_pair){0, 0, 0, 0};
    while (sp > 0) {
        orc_pair P = st[--sp];
        const orc_level_t* LA = &h->lev[P.la];
        const orc_level_t* LB = &h->lev[P.lb];
        int leafA = LA->nchild[P.a] == 0, leafB = LB->nchild[P.b] == 0;
        int same = P.la == P.lb && P.a == P.b;
        if (!same && orc_admissible(P.la, LA->key[P.a], P.lb, LB->key[P.b])) {
            orc_push_block(&h->il, &ni, &icap, P.la, P.a, P.lb, P.b);
            continue;
        }
        if (leafA && leafB) {
            orc_push_block(&h->near, &nn, &ncap, P.la, P.a, P.lb, P.b);
            continue;
        }
        int64_t a0 = leafA ? P.a : LA->child0[P.a], na = leafA ? 1 : LA->nchild[P.a];
        int64_t b0 = leafB ? P.b : LB->child0[P.b], nb = leafB ? 1 : LB->nchild[P.b];
        int la = leafA ? P.la : P.la + 1, lb = leafB ? P.lb : P.lb + 1;
        for (int64_t i = 0; i < na; ++i)
            for (int64_t j = 0; j < nb; ++j) {
                if (sp == scap) { scap *= 2; st = (orc_pair*)realloc(st, sizeof(orc_pair) * (size_t)scap); }
                st[sp++] = (orc_pair){la, lb, a0 + i, b0 + j};
            }
    }
    free(st);
    if (nn) qsort(h->near, (size_t)nn, sizeof(orc_block), orc_block_cmp);
    if (ni) qsort(h->il, (size_t)ni, sizeof(orc_block), orc_block_cmp);
    for (int64_t q = 0; q < ni; ++q) h->il[q].kind = BK_LOWRANK;
    h->n_near = nn; h->n_il = ni;
    if (!h->near) h->near = (orc_block*)calloc(1, sizeof(orc_block));
    if (!h->il) h->il = (orc_block*)calloc(1, sizeof(orc_block));
}

/* ------------------------------------------------------------------ */
/* Adaptive cross approximation                                         */
/* ------------------------------------------------------------------ */

/* Partial-pivot ACA of the block A(i', j') = K(rows[i'], cols[j']).
 *
 * Each step takes the residual row at the current pivot row i, picks the
 * pivot column j* of largest |residual| among unused columns (lowest index
 * on ties), scales that row by the pivot to get v, takes the residual column
 * u at j*, and appends the cross u v^T.  The squared Frobenius norm S2 of
 * the running approximation is updated incrementally, and iteration stops
 * once |u| |v| <= tol * sqrt(S2).  The next pivot row is the unused row of
 * largest |u| (lowest index on ties).  A residual row that is identically
 * zero is skipped (its index marked used); if every row has been used the
 * approximation is exact and the loop ends.
 *
 * Storage rule: when the rank reaches min(m, n), or when k (m + n) >= m n,
 * the factors are dropped and the exact dense block is stored instead -- it
 * is then both smaller than U, V and exact.
 *
 * On return *kind is BK_LOWRANK (U: m x k, V: n x k, column-major, caller
 * frees) or BK_DENSE (*D: m x n column-major).  Returns the rank (k for
 * low rank, the ACA rank reached for dense). */
int64_t orc_aca(const orc_kernel* kern, const double* xy, const int64_t* rows, int64_t m,
                const int64_t* cols, int64_t n, double tol, int32_t* kind,
                double** Uo, double** Vo, double** Do)
{
    int64_t kmax = m < n ? m : n;
    double* U = (double*)malloc(sizeof(double) * (size_t)(m * (kmax > 0 ? kmax : 1)));
    double* V = (double*)malloc(sizeof(double) * (size_t)(n * (kmax > 0 ? kmax : 1)));
    double* r = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* u = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    char* usedR = (char*)calloc((size_t)(m > 0 ? m : 1), 1);
    char* usedC = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t k = 0, nusedR = 0, i = 0;
    double S2 = 0.0;
    int dense = 0;
    while (kmax > 0) {
        /* residual row i */
        for (int64_t j = 0; j < n; ++j) {
            double s = orc_entry(kern, xy, rows[i], cols[j]);
            for (int64_t q = 0; q < k; ++q) s -= U[q * m + i] * V[q * n + j];
            r[j] = s;
        }
        if (!usedR[i]) { usedR[i] = 1; ++nusedR; }
        int64_t js = -1;
        double best = -1.0;
        for (int64_t j = 0; j < n; ++j)
            if (!usedC[j] && fabs(r[j]) > best) { best = fabs(r[j]); js = j; }
        if (js < 0) break;
        if (r[js] == 0.0) {
            if (nusedR == m) break;
            for (i = 0; i < m && usedR[i]; ++i) {}
            continue;
        }
        double delta = r[js];
        double* v = V + k * n;
        for (int64_t j = 0; j < n; ++j) v[j] = r[j] / delta;
        for (int64_t ii = 0; ii < m; ++ii) {
            double s = orc_entry(kern, xy, rows[ii], cols[js]);
            for (int64_t q = 0; q < k; ++q) s -= U[q * m + ii] * V[q * n + js];
            u[ii] = s;
        }
        usedC[js] = 1;
        double uu = 0.0, vv = 0.0, cross = 0.0;
        for (int64_t ii = 0; ii < m; ++ii) uu += u[ii] * u[ii];
        for (int64_t j = 0; j < n; ++j) vv += v[j] * v[j];
        for (int64_t q = 0; q < k; ++q) {
            double a = 0.0, b = 0.0;
            for (int64_t ii = 0; ii < m; ++ii) a += U[q * m + ii] * u[ii];
            for (int64_t j = 0; j < n; ++j) b += V[q * n + j] * v[j];
            cross += a * b;
        }
        S2 += 2.0 * cross + uu * vv;
        memcpy(U + k * m, u, sizeof(double) * (size_t)m);
        ++k;
        if (sqrt(uu) * sqrt(vv) <= tol * sqrt(S2)) break;
        if (k == kmax) { dense = 1; break; }
        /* next pivot row */
        int64_t is = -1;
        best = -1.0;
        for (int64_t ii = 0; ii < m; ++ii)
            if (!usedR[ii] && fabs(u[ii]) > best) { best = fabs(u[ii]); is = ii; }
        if (is < 0) break;
        i = is;
    }
    if (!dense && k * (m + n) >= m * n && m * n > 0) dense = 1;
    free(r); free(u); free(usedR); free(usedC);
    if (dense) {
        double* D = (double*)malloc(sizeof(double) * (size_t)(m * n));
        for (int64_t j = 0; j < n; ++j)
            for (int64_t ii = 0; ii < m; ++ii) D[j * m + ii] = orc_entry(kern, xy, rows[ii], cols[j]);
        free(U); free(V);
        *kind = BK_DENSE; *Do = D; *Uo = NULL; *Vo = NULL;
        return k;
    }
    *kind = BK_LOWRANK; *Uo = U; *Vo = V; *Do = NULL;
    return k;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1                                                          */
/* ------------------------------------------------------------------ */

/* Index of the IL block (level, tgt, src) in the (level, tgt, src)-sorted
 * table of a balanced tree, or -1. */
static int64_t orc_find_block(const orc_h* h, int32_t level, int64_t tgt, int64_t src)
{
    int64_t lo = 0, hi = h->n_il;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        const orc_block* B = &h->il[mid];
        int less = B->level != level ? B->level < level : (B->tgt != tgt ? B->tgt < tgt : B->src < src);
        if (less) lo = mid + 1; else hi = mid;
    }
    if (lo < h->n_il && h->il[lo].level == level && h->il[lo].tgt == tgt && h->il[lo].src == src) return lo;
    return -1;
}

/* Symmetric mode: the block (level, t, s) with t > s takes the transpose of
 * the block (level, s, t): U and V swapped for low rank, D transposed for
 * dense (kind and rank from the owner). */
static int orc_mirror_block(orc_h* h, orc_block* B)
{
    int64_t o = orc_find_block(h, B->level, B->src, B->tgt);
    if (o < 0) return ORC_EINVAL;
    const orc_block* O = &h->il[o];
    int64_t m = h->lev[B->level].count[B->tgt], n = h->lev[B->level].count[B->src];
    B->kind = O->kind;
    B->k = O->k;
    if (O->kind == BK_DENSE) {
        /* owner D is n x m (rows of src) */
        B->D = (double*)malloc(sizeof(double) * (size_t)(m * n));
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) B->D[j * m + i] = O->D[i * n + j];
        return ORC_OK;
    }
    B->U = (double*)malloc(sizeof(double) * (size_t)(m * O->k > 0 ? m * O->k : 1));
    B->V = (double*)malloc(sizeof(double) * (size_t)(n * O->k > 0 ? n * O->k : 1));
    memcpy(B->U, O->V, sizeof(double) * (size_t)(m * O->k));
    memcpy(B->V, O->U, sizeof(double) * (size_t)(n * O->k));
    return ORC_OK;
}

/* Dense near-field blocks by their entries; ACA for the interaction-list
 * blocks.  Rows are the target box's points, columns the source box's, in
 * tree order (each box on its own level).  In symmetric mode the blocks
 * with tgt > src are filled last, as transposes. */
static int orc_fill_factors(orc_h* h)
{
    const orc_kernel* kern = &h->kern;
    const double* xy = h->xy;
    int64_t n = h->n;
    int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* cols = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t t = 0; t < h->n_near; ++t) {
        orc_block* B = &h->near[t];
        const orc_level_t* LT = &h->lev[B->level];
        const orc_level_t* LS = &h->lev[B->slevel];
        int64_t m = LT->count[B->tgt], nn = LS->count[B->src];
        B->D = (double*)malloc(sizeof(double) * (size_t)(m * nn));
        for (int64_t j = 0; j < nn; ++j)
            for (int64_t i = 0; i < m; ++i)
                B->D[j * m + i] = orc_entry(kern, xy, h->perm[LT->begin[B->tgt] + i], h->perm[LS->begin[B->src] + j]);
    }
    for (int64_t t = 0; t < h->n_il; ++t) {
        orc_block* B = &h->il[t];
        if (h->symmetric && B->tgt > B->src) continue;
        const orc_level_t* LT = &h->lev[B->level];
        const orc_level_t* LS = &h->lev[B->slevel];
        int64_t m = LT->count[B->tgt], nn = LS->count[B->src];
        for (int64_t i = 0; i < m; ++i) rows[i] = h->perm[LT->begin[B->tgt] + i];
        for (int64_t j = 0; j < nn; ++j) cols[j] = h->perm[LS->begin[B->src] + j];
        B->k = orc_aca(kern, xy, rows, m, cols, nn, h->tol, &B->kind, &B->U, &B->V, &B->D);
    }
    free(rows); free(cols);
    if (h->symmetric)
        for (int64_t t = 0; t < h->n_il; ++t)
            if (h->il[t].tgt > h->il[t].src && orc_mirror_block(h, &h->il[t]) != ORC_OK) return ORC_EINVAL;
    return ORC_OK;
}

static int orc_has_duplicates(const orc_h* h)
{
    /* two distinct points at distance 0 make log, 1/r, phi_1, phi_2 singular */
    if (!(h->kern.kind == OK_LOG || h->kern.kind == OK_INVR)) return 0;
    for (int l = 0; l <= h->kappa; ++l) {
        const orc_level_t* L = &h->lev[l];
        for (int64_t b = 0; b < L->nbox; ++b) {
            if (L->nchild[b] != 0) continue;   /* leaves only: they partition the points */
            for (int64_t p = L->begin[b]; p < L->begin[b] + L->count[b]; ++p)
                for (int64_t q = p + 1; q < L->begin[b] + L->count[b]; ++q) {
                    const double* a = h->xy + 2 * h->perm[p];
                    const double* c = h->xy + 2 * h->perm[q];
                    if (a[0] == c[0] && a[1] == c[1]) return 1;
                }
        }
    }
    return 0;
}

int orc_build(const double* xy, int64_t n, const orc_kernel* kern, int32_t leaf_max, double tol,
              int32_t with_factors, orc_h** out)
{
    *out = NULL;
    if (n < 1 || leaf_max < 1 || !(tol >= 0.0)) return ORC_EINVAL;
    for (int64_t i = 0; i < 2 * n; ++i) if (!isfinite(xy[i])) return ORC_EINVAL;
    orc_h* h = (orc_h*)calloc(1, sizeof(orc_h));
    h->n = n; h->leaf_max = leaf_max; h->tol = tol; h->kern = *kern;
    h->factors = with_factors & 1;
    h->adaptive = (with_factors >> 1) & 1;
    h->symmetric = (with_factors >> 2) & 1;
    /* sharing needs a symmetric kernel and same-level pairs */
    if (h->symmetric && (h->adaptive || kern->kind == OK_SEP)) { free(h->xy); free(h); return ORC_EINVAL; }
    h->xy = (double*)malloc(sizeof(double) * (size_t)(2 * n));
    memcpy(h->xy, xy, sizeof(double) * (size_t)(2 * n));
    h->R = orc_box_radius(xy, n);
    int st = h->adaptive ? orc_tree_adaptive(h) : orc_tree(h);
    if (st) { orc_free(h); return st; }
    if (orc_has_duplicates(h)) { orc_free(h); return ORC_EDUP; }
    if (h->adaptive) {
        orc_lists_adaptive(h);
        if (h->factors) orc_fill_factors(h);
        *out = h;
        return ORC_OK;
    }
    int kappa = h->kappa;
    /* near blocks at the leaf level: self, then edge sharers, in key order */
    const orc_level_t* LL = &h->lev[kappa];
    int64_t cap = 5 * LL->nbox;
    h->near = (orc_block*)calloc((size_t)(cap > 0 ? cap : 1), sizeof(orc_block));
    h->n_near = 0;
    for (int64_t b = 0; b < LL->nbox; ++b) {
        uint32_t keys[5];
        int ne = orc_edge_list(LL->key[b], kappa, keys);
        keys[ne++] = LL->key[b];
        qsort(keys, (size_t)ne, sizeof(uint32_t), orc_u32_cmp);
        for (int e = 0; e < ne; ++e) {
            int64_t s = orc_find(LL, keys[e]);
            if (s < 0) continue;
            orc_block* B = &h->near[h->n_near++];
            B->level = kappa; B->slevel = kappa; B->kind = BK_DENSE; B->tgt = b; B->src = s; B->k = 0;
        }
    }
    /* interaction-list blocks, levels 1..kappa */
    int64_t ilcap = 0;
    for (int l = 1; l <= kappa; ++l) ilcap += 15 * h->lev[l].nbox;
    h->il = (orc_block*)calloc((size_t)(ilcap > 0 ? ilcap : 1), sizeof(orc_block));
    h->n_il = 0;
    for (int l = 1; l <= kappa; ++l) {
        const orc_level_t* L = &h->lev[l];
        for (int64_t b = 0; b < L->nbox; ++b) {
            uint32_t keys[24];
            int ni = orc_interaction_list(L->key[b], l, keys);
            for (int e = 0; e < ni; ++e) {
                int64_t s = orc_find(L, keys[e]);
                if (s < 0) continue;
                orc_block* B = &h->il[h->n_il++];
                B->level = l; B->slevel = l; B->tgt = b; B->src = s;
            }
        }
    }
    if (h->factors && orc_fill_factors(h) != ORC_OK) { orc_free(h); return ORC_EINVAL; }
    *out = h;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2: b = K psi with the HODLR2D representation               */
/* ------------------------------------------------------------------ */

int orc_matvec(const orc_h* h, const double* psi, double* bout)
{
    if (!h->factors) return ORC_EINVAL;
    int64_t n = h->n;
    double* x = (double*)malloc(sizeof(double) * (size_t)n);   /* psi in tree order */
    double* b = (double*)calloc((size_t)n, sizeof(double));    /* b in tree order */
    for (int64_t i = 0; i < n; ++i) x[i] = psi[h->perm[i]];
    /* full-rank part: self and edge-sharing blocks of the leaves */
    for (int64_t t = 0; t < h->n_near; ++t) {
        const orc_block* B = &h->near[t];
        const orc_level_t* LT = &h->lev[B->level];
        const orc_level_t* LS = &h->lev[B->slevel];
        int64_t r0 = LT->begin[B->tgt], m = LT->count[B->tgt];
        int64_t c0 = LS->begin[B->src], nn = LS->count[B->src];
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < nn; ++j) s += B->D[j * m + i] * x[c0 + j];
            b[r0 + i] += s;
        }
    }
    /* low-rank part: levels 1..kappa, every box, every interaction-list box */
    double* t = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t q = 0; q < h->n_il; ++q) {
        const orc_block* B = &h->il[q];
        const orc_level_t* LT = &h->lev[B->level];
        const orc_level_t* LS = &h->lev[B->slevel];
        int64_t r0 = LT->begin[B->tgt], m = LT->count[B->tgt];
        int64_t c0 = LS->begin[B->src], nn = LS->count[B->src];
        if (B->kind == BK_DENSE) {
            for (int64_t i = 0; i < m; ++i) {
                double s = 0.0;
                for (int64_t j = 0; j < nn; ++j) s += B->D[j * m + i] * x[c0 + j];
                b[r0 + i] += s;
            }
            continue;
        }
        for (int64_t c = 0; c < B->k; ++c) {       /* t = V^T psi(Y) */
            double s = 0.0;
            for (int64_t j = 0; j < nn; ++j) s += B->V[c * nn + j] * x[c0 + j];
            t[c] = s;
        }
        for (int64_t i = 0; i < m; ++i) {          /* b(X) += U t */
            double s = 0.0;
            for (int64_t c = 0; c < B->k; ++c) s += B->U[c * m + i] * t[c];
            b[r0 + i] += s;
        }
    }
    for (int64_t i = 0; i < n; ++i) bout[h->perm[i]] = b[i];
    free(t); free(x); free(b);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Restarted GMRES on the HODLR2D operator (Section 5)                  */
/* ------------------------------------------------------------------ */

static double orc_nrm2(const double* a, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * a[i];
    return sqrt(s);
}

/* Solve A x = b with GMRES(restart), x0 = 0, modified Gram-Schmidt Arnoldi
 * and Givens rotations.  Converged when the true relative residual
 * |b - A x| / |b| <= tol (checked at every restart and at exit).
 * Returns ORC_OK or ORC_ENOCONV; *iters = total Arnoldi steps. */
int orc_gmres(const orc_h* h, const double* b, double* x, double tol, int32_t restart,
              int32_t max_iter, int32_t* iters, double* relres)
{
    int64_t n = h->n;
    int mr = restart;
    double* Vb = (double*)malloc(sizeof(double) * (size_t)(n * (mr + 1)));
    double* H = (double*)calloc((size_t)((mr + 1) * mr), sizeof(double));
    double* cs = (double*)malloc(sizeof(double) * (size_t)mr);
    double* sn = (double*)malloc(sizeof(double) * (size_t)mr);
    double* g = (double*)malloc(sizeof(double) * (size_t)(mr + 1));
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    double* r = (double*)malloc(sizeof(double) * (size_t)n);
    double bn = orc_nrm2(b, n);
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    int it = 0, status = ORC_ENOCONV;
    double rel = 1.0;
    if (bn == 0.0) { *iters = 0; *relres = 0.0; status = ORC_OK; goto done; }
    for (;;) {
        orc_matvec(h, x, w);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
        double beta = orc_nrm2(r, n);
        rel = beta / bn;
        if (rel <= tol) { status = ORC_OK; break; }
        if (it >= max_iter) break;
        for (int64_t i = 0; i < n; ++i) Vb[i] = r[i] / beta;
        for (int j = 0; j <= mr; ++j) g[j] = 0.0;
        g[0] = beta;
        int j;
        for (j = 0; j < mr && it < max_iter; ++j) {
            ++it;
            orc_matvec(h, Vb + j * n, w);
            for (int i = 0; i <= j; ++i) {
                double s = 0.0;
                for (int64_t p = 0; p < n; ++p) s += w[p] * Vb[i * n + p];
                H[j * (mr + 1) + i] = s;
                for (int64_t p = 0; p < n; ++p) w[p] -= s * Vb[i * n + p];
            }
            double hn = orc_nrm2(w, n);
            H[j * (mr + 1) + j + 1] = hn;
            if (hn != 0.0) for (int64_t p = 0; p < n; ++p) Vb[(j + 1) * n + p] = w[p] / hn;
            for (int i = 0; i < j; ++i) {
                double a = H[j * (mr + 1) + i], c = H[j * (mr + 1) + i + 1];
                H[j * (mr + 1) + i] = cs[i] * a + sn[i] * c;
                H[j * (mr + 1) + i + 1] = -sn[i] * a + cs[i] * c;
            }
            double a = H[j * (mr + 1) + j], c = H[j * (mr + 1) + j + 1];
            double d = sqrt(a * a + c * c);
            cs[j] = (d == 0.0) ? 1.0 : a / d;
            sn[j] = (d == 0.0) ? 0.0 : c / d;
            H[j * (mr + 1) + j] = d;
            H[j * (mr + 1) + j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            if (fabs(g[j + 1]) / bn <= tol || hn == 0.0) { ++j; break; }
        }
        /* back substitution and update */
        double* yv = (double*)malloc(sizeof(double) * (size_t)(j > 0 ? j : 1));
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int q = i + 1; q < j; ++q) s -= H[q * (mr + 1) + i] * yv[q];
            yv[i] = s / H[i * (mr + 1) + i];
        }
        for (int i = 0; i < j; ++i)
            for (int64_t p = 0; p < n; ++p) x[p] += yv[i] * Vb[i * n + p];
        free(yv);
    }
    *iters = it; *relres = rel;
done:
    free(Vb); free(H); free(cs); free(sn); free(g); free(w); free(r);
    return status;
}

/* ------------------------------------------------------------------ */
/* Accessors for tests                                                  */
/* ------------------------------------------------------------------ */

int32_t orc_kappa(const orc_h* h) { return h->kappa; }
double orc_R(const orc_h* h) { return h->R; }
void orc_perm(const orc_h* h, int64_t* out) { memcpy(out, h->perm, sizeof(int64_t) * (size_t)h->n); }
int64_t orc_nbox(const orc_h* h, int32_t l) { return (l >= 0 && l <= h->kappa) ? h->lev[l].nbox : 0; }
void orc_level(const orc_h* h, int32_t l, uint32_t* key, int64_t* begin, int64_t* count, int64_t* parent)
{
    const orc_level_t* L = &h->lev[l];
    memcpy(key, L->key, sizeof(uint32_t) * (size_t)L->nbox);
    memcpy(begin, L->begin, sizeof(int64_t) * (size_t)L->nbox);
    memcpy(count, L->count, sizeof(int64_t) * (size_t)L->nbox);
    memcpy(parent, L->parent, sizeof(int64_t) * (size_t)L->nbox);
}
int64_t orc_n_near(const orc_h* h) { return h->n_near; }
int64_t orc_n_il(const orc_h* h) { return h->n_il; }
void orc_near_table(const orc_h* h, int64_t* tgt, int64_t* src)
{
    for (int64_t b = 0; b < h->n_near; ++b) { tgt[b] = h->near[b].tgt; src[b] = h->near[b].src; }
}
int32_t orc_is_adaptive(const orc_h* h) { return h->adaptive; }
int32_t orc_is_symmetric(const orc_h* h) { return h->symmetric; }
/* Levels of the target and source boxes of every near and IL block. */
void orc_block_levels(const orc_h* h, int32_t* near_tl, int32_t* near_sl, int32_t* il_tl, int32_t* il_sl)
{
    for (int64_t b = 0; b < h->n_near; ++b) { near_tl[b] = h->near[b].level; near_sl[b] = h->near[b].slevel; }
    for (int64_t b = 0; b < h->n_il; ++b) { il_tl[b] = h->il[b].level; il_sl[b] = h->il[b].slevel; }
}
void orc_il_table(const orc_h* h, int32_t* level, int64_t* tgt, int64_t* src, int32_t* kind, int64_t* rank)
{
    for (int64_t b = 0; b < h->n_il; ++b) {
        level[b] = h->il[b].level; tgt[b] = h->il[b].tgt; src[b] = h->il[b].src;
        kind[b] = h->il[b].kind; rank[b] = h->il[b].k;
    }
}
/* Copy the factors of IL block b: U (m x k) and V (n x k) for low rank, or
 * D (m x n) for dense, column-major. */
void orc_il_factors(const orc_h* h, int64_t b, double* U, double* V, double* D)
{
    const orc_block* B = &h->il[b];
    int64_t m = h->lev[B->level].count[B->tgt], n = h->lev[B->slevel].count[B->src];
    if (B->kind == BK_DENSE) { if (D) memcpy(D, B->D, sizeof(double) * (size_t)(m * n)); return; }
    if (U) memcpy(U, B->U, sizeof(double) * (size_t)(m * B->k));
    if (V) memcpy(V, B->V, sizeof(double) * (size_t)(n * B->k));
}
void orc_near_factor(const orc_h* h, int64_t b, double* D)
{
    const orc_block* B = &h->near[b];
    memcpy(D, B->D, sizeof(double) * (size_t)(h->lev[B->level].count[B->tgt] * h->lev[B->slevel].count[B->src]));
}

/* ------------------------------------------------------------------ */
/* Export (binary, little-endian), the format the library's import reads */
/* ------------------------------------------------------------------ */

int orc_export(const orc_h* h, const char* path)
{
    if (!h->factors) return ORC_EINVAL;
    FILE* f = fopen(path, "wb");
    if (!f) return ORC_EINVAL;
    const char magic[4] = {'H', '2', 'D', 'X'};
    /* version 2 (adaptive trees): every block also carries the levels of its
     * boxes; flags bit 0: factors present */
    uint32_t version = h->adaptive ? 2 : 1, flags = 1, reserved = 0;
    fwrite(magic, 1, 4, f);
    fwrite(&version, 4, 1, f);
    fwrite(&flags, 4, 1, f);
    fwrite(&reserved, 4, 1, f);
    fwrite(&h->n, 8, 1, f);
    fwrite(&h->kappa, 4, 1, f);
    fwrite(&h->leaf_max, 4, 1, f);
    fwrite(&h->R, 8, 1, f);
    fwrite(&h->tol, 8, 1, f);
    fwrite(&h->kern.kind, 4, 1, f);
    fwrite(&h->kern.diag_mode, 4, 1, f);
    fwrite(&h->kern.c, 8, 1, f);
    fwrite(&h->kern.diag_value, 8, 1, f);
    fwrite(h->xy, 8, (size_t)(2 * h->n), f);
    fwrite(h->perm, 8, (size_t)h->n, f);
    for (int l = 0; l <= h->kappa; ++l) {
        const orc_level_t* L = &h->lev[l];
        fwrite(&L->nbox, 8, 1, f);
        fwrite(L->key, 4, (size_t)L->nbox, f);
        fwrite(L->begin, 8, (size_t)L->nbox, f);
        fwrite(L->count, 8, (size_t)L->nbox, f);
        fwrite(L->parent, 8, (size_t)L->nbox, f);
    }
    fwrite(&h->n_near, 8, 1, f);
    for (int64_t b = 0; b < h->n_near; ++b) {
        const orc_block* B = &h->near[b];
        if (h->adaptive) { fwrite(&B->level, 4, 1, f); fwrite(&B->slevel, 4, 1, f); }
        fwrite(&B->tgt, 8, 1, f);
        fwrite(&B->src, 8, 1, f);
        fwrite(B->D, 8, (size_t)(h->lev[B->level].count[B->tgt] * h->lev[B->slevel].count[B->src]), f);
    }
    fwrite(&h->n_il, 8, 1, f);
    for (int64_t b = 0; b < h->n_il; ++b) {
        const orc_block* B = &h->il[b];
        int64_t m = h->lev[B->level].count[B->tgt], n = h->lev[B->slevel].count[B->src];
        fwrite(&B->level, 4, 1, f);
        fwrite(&B->kind, 4, 1, f);
        if (h->adaptive) { fwrite(&B->slevel, 4, 1, f); fwrite(&B->pad, 4, 1, f); }
        fwrite(&B->tgt, 8, 1, f);
        fwrite(&B->src, 8, 1, f);
        fwrite(&B->k, 8, 1, f);
        if (B->kind == BK_DENSE) fwrite(B->D, 8, (size_t)(m * n), f);
        else {
            fwrite(B->U, 8, (size_t)(m * B->k), f);
            fwrite(B->V, 8, (size_t)(n * B->k), f);
        }
    }
    int ok = ferror(f) == 0;
    fclose(f);
    return ok ? ORC_OK : ORC_EINVAL;
}
