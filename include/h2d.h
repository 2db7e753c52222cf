/*
 * h2d.h -- C ABI of the MI355X (gfx950) HODLR2D library.
 *
 * HODLR2D (arxiv 2204.05536) represents the dense N x N kernel matrix
 * A_ij = K(x_i, x_j) of N points in the plane on a balanced quadtree:
 *   - at the leaf level, the self block and the blocks of the (at most 4)
 *     edge-sharing boxes are dense (Section 4, Algorithm 1);
 *   - at every level 1..kappa, each box interacts with the boxes of its
 *     interaction list (vertex-sharing or well-separated boxes of its clan,
 *     Section 4 definitions and eq. (4.2)) through a low-rank block U V^T
 *     obtained by adaptive cross approximation (Algorithm 1).
 * The matrix-vector product of Algorithm 2 then costs O(p N log N).
 *
 * Conventions for every entry point:
 *   - Buffers named "device" are device pointers on the current HIP device;
 *     buffers named "host" are host pointers.  The caller owns every buffer
 *     it passes; the library owns everything behind an h2d_t until
 *     h2d_destroy().
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     on it; entry points that must read results back (build, solve, info,
 *     export) synchronise that stream before returning.
 *   - Vectors are in the caller's point order (the order of `xy`).  The tree
 *     order is internal.
 *   - Errors are returned as h2d_status; h2d_last_error() gives a message
 *     for the calling thread.  No C++ exception crosses this boundary.
 *   - Calls on one handle must not overlap in time (a handle owns scratch
 *     vectors used by matvec and solve).
 */
#ifndef H2D_H
#define H2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h2d_s* h2d_t;

typedef enum {
    H2D_OK = 0,
    H2D_EINVAL = 1,       /* bad argument or non-finite input */
    H2D_ENOMEM = 2,       /* device or host allocation failed */
    H2D_EDEVICE = 3,      /* a HIP call failed */
    H2D_EDUP = 4,         /* two distinct points coincide and the kernel is singular at r = 0 */
    H2D_ENOCONV = 5,      /* solver did not reach the tolerance; ACA hit its rank cap */
    H2D_EUNSUPPORTED = 6, /* option not built in */
    H2D_EDEPTH = 7        /* quadtree deeper than 16 levels needed for leaf_max */
} h2d_status;

/* Kernel functions K(x, y) = phi(|x - y|) (plus a separable test kernel).
 *   LOG    phi = log r                      (Section 3)
 *   INVR   phi = 1 / r                      (Section 5.1)
 *   MQ     phi = sqrt(1 + (r / c)^2)        multiquadric RBF
 *   GAUSS  phi = exp(-(r / c)^2)            Gaussian RBF
 *   PHI1   phi = log r / log a (r >= a), (r log r - 1)/(a log a - 1) (r < a), a = c  (Section 5.2)
 *   PHI2   phi = a / r (r >= a), r / a (r < a), a = c                                 (Section 5.2)
 *   SEP    sum_{q < c} cos(q (1.3 x1 + 0.7 x2)) cos(q (0.9 y1 - 1.1 y2)), exact rank c (test kernel)
 * Diagonal rule (decided by index equality i == j, never by r == 0):
 *   REPLACE  A_ii = diag_value          (e.g. N for log, beta for phi_1/phi_2, 0 for 1/r)
 *   ADD      A_ii = phi(0) + diag_value (MQ, Gauss: 1 + shift)
 *   FORMULA  A_ii = K(x_i, x_i)         (only for kernels finite at r = 0) */
typedef enum {
    H2D_K_LOG = 0, H2D_K_INVR = 1, H2D_K_MQ = 2, H2D_K_GAUSS = 3,
    H2D_K_PHI1 = 4, H2D_K_PHI2 = 5, H2D_K_SEP = 6
} h2d_kind;

typedef enum { H2D_DIAG_REPLACE = 0, H2D_DIAG_ADD = 1, H2D_DIAG_FORMULA = 2 } h2d_diag;

typedef struct {
    int32_t kind;        /* h2d_kind */
    int32_t diag_mode;   /* h2d_diag */
    double c;            /* shape parameter (see above) */
    double diag_value;   /* diagonal replacement / shift */
} h2d_kernel;

/* Storage precision of U, V and the dense blocks used by a matvec. */
typedef enum { H2D_P_FP64 = 0, H2D_P_FP16 = 1, H2D_P_BF16 = 2 } h2d_prec;
#define H2D_PREC_BIT(p) (1u << (p))

/* Build flag (OR-ed into h2d_build's prec_mask): an adaptive quadtree, the
 * form the end of Section 4 says the method carries over to.  A box is
 * split exactly when it holds more than leaf_max points, so leaves sit at
 * several levels; the blocks come from descending pairs of boxes from
 * (root, root): two distinct boxes whose closed squares share at most one
 * point are one compressed (ACA) block, two leaves sharing a segment (or a
 * leaf with itself) one dense block, any other pair gives way to the pairs
 * of its children (only the non-leaf side splits when one side is a leaf).
 * On inputs where this rule stops every branch at one depth the result is
 * the balanced tree.  The tree and block lists are built by host code, the
 * factors and products on the GPU.  Adaptive handles build the FP64 pools
 * only and serve h2d_matvec (right-hand sides one at a time),
 * h2d_matvec_noalloc, plain h2d_solve, h2d_info, h2d_export (file version
 * 2) and h2d_import; the half-precision pools, preconditioners, batches and
 * tile tuning return EUNSUPPORTED. */
#define H2D_BUILD_ADAPTIVE (1u << 8)

/* Build flag (OR-ed into h2d_build's prec_mask, or h2d_import's): one
 * factor pair per interaction-list pair.  Section 2.1 takes the matrix
 * symmetric; for a symmetric kernel the block of (C', C) is the transpose
 * of the block of (C, C').  Only the block whose target box has the smaller
 * index is compressed, (X, Y) ~ F_X F_Y^T, and the mirror applies F_Y F_X^T;
 * dense and edge-sharing blocks are stored once too.  Factor
 * storage is about half the ordered form's, and the product reads the
 * factors above the leaf level 1.5 times and the leaf-level pairs once
 * (the ordered product: 2 and 2 per pair).  Needs a symmetric kernel (every
 * kind but H2D_K_SEP), the balanced tree, leaves of at most 64 points, and
 * FP64 pools only (else EUNSUPPORTED).  h2d_import with this flag takes an
 * ordered file whose mirror blocks are exact transposes of their owners
 * (the oracle's symmetric build writes such files; else EINVAL).
 * Symmetric handles serve h2d_matvec (right-hand sides one at a time),
 * plain h2d_solve, h2d_info, h2d_export (ordered, mirrors written as the
 * transposes) and h2d_profile_*; the fixed-array product, preconditioners,
 * batches and tile tuning return EUNSUPPORTED.  Profile phases of a
 * symmetric product: gather, walk 1 + its reduction, walk 2 + the leaf
 * pairs, the second reduction + walk 3 + the slot sums, combine. */
#define H2D_BUILD_SYMMETRIC (1u << 9)

/* Algorithm 1 (InitializeHODLR2D(N_max, eps)) on the GPU.
 *   xy        device, n x 2 row-major FP64 point coordinates (copied)
 *   n         number of points, 1 <= n < 2^31
 *   kernel    host, the kernel function and diagonal rule
 *   leaf_max  N_max: the tree has the smallest depth kappa (<= 16) at which
 *             no leaf box holds more than leaf_max points
 *   tol       ACA tolerance eps (relative, per block), >= 0
 *   prec_mask H2D_PREC_BIT(H2D_P_FP64) is always built; add FP16 / BF16
 *             bits to also keep half-precision copies of every factor
 *   stream    hipStream_t
 *   out       receives the handle
 * Box B = [-R, R]^2 with R the smallest power of two >= max |coordinate|;
 * cells are half-open [lo, mid) / [mid, hi] (Section 3).  Points are ordered
 * by (leaf Morton key, caller index).  Errors: EINVAL (bad sizes, non-finite
 * coordinates), EDUP, EDEPTH, ENOMEM, ENOCONV (ACA rank cap), EDEVICE. */
h2d_status h2d_build(const double* xy, int64_t n, const h2d_kernel* kernel, int32_t leaf_max,
                     double tol, uint32_t prec_mask, void* stream, h2d_t* out);

/* Algorithm 2 (MatVec(psi)): y = A_hat x for nrhs right-hand sides.
 *   x, y    device, FP64, column-major n x nrhs with leading dimension ld >= n
 *   prec    storage precision to read (must have been built); FP16/BF16
 *           accumulate in FP32 and round the result to FP64
 * nrhs > 1 runs the right-hand sides 16 at a time through matrix-core
 * (MFMA) kernels: FP64 ones on the FP64 pools, FP32 ones on the FP16/BF16
 * pools (each stored value widened to FP32 as it is loaded, right-hand
 * sides and sums in FP32); adaptive and symmetric handles run them one by
 * one.
 * Asynchronous on `stream`.  Errors: EINVAL, EUNSUPPORTED (precision not
 * built), EDEVICE. */
h2d_status h2d_matvec(h2d_t H, const double* x, double* y, int32_t nrhs, int64_t ld,
                      int32_t prec, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A_hat x
 * for one right-hand side, as h2d_matvec with nrhs = 1 (same kernels, same
 * result bit for bit), with no allocation of any kind.  Its work vectors (x
 * in tree order, the t = V^T x values, the split-block partials, the two
 * phase-B sums: about (3 n + sum of ranks + partials) values of 8 bytes for
 * FP64, 4 bytes for FP16/BF16) live in a fixed device array of
 * H2D_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.
 *   x, y    device FP64, n entries, caller order (caller-owned)
 *   prec    storage precision to read (must have been built)
 * The current device must be the one H was built on.  Errors: EINVAL (NULL
 * argument, another device, or a handle whose work vectors exceed the
 * array: the message states the bytes needed), EUNSUPPORTED, EDEVICE.
 * Calls share their GPU's array, and every kernel writes each work value
 * before reading it, so nothing carries over from one call to the next;
 * calls that overlap in time on one GPU (different streams or threads) race
 * on the array and must be serialised by the caller.  Asynchronous on
 * `stream`. */
#define H2D_NOALLOC_SCRATCH_BYTES (256u << 20)
h2d_status h2d_matvec_noalloc(h2d_t H, const double* x, double* y, int32_t prec, void* stream);

/* Solver modes for h2d_solve. */
typedef enum {
    H2D_SOLVE_PLAIN = 0,   /* restarted GMRES on the FP64 operator */
    H2D_SOLVE_REFINE = 1   /* FP64 iterative refinement around an inner GMRES
                              on the FP16/BF16 operator (inner_prec); an inner
                              solve stops on its Arnoldi residual estimate, the
                              refinement step on the true FP64 residual */
} h2d_solve_mode;

/* Right preconditioners (flexible GMRES: the preconditioned vectors are
 * kept, so a nonlinear preconditioner such as the MLP is allowed). */
typedef enum {
    H2D_PC_NONE = 0,
    H2D_PC_BLOCK_JACOBI = 1,  /* exact LU of each leaf's self block K(X, X) */
    H2D_PC_MLP = 2            /* learned per-leaf correction (h2d_mlp_train) */
} h2d_precond;

typedef struct {
    int32_t mode;          /* h2d_solve_mode */
    int32_t restart;       /* GMRES restart length (e.g. 50) */
    int32_t max_iter;      /* cap on total inner Arnoldi steps */
    int32_t inner_prec;    /* REFINE: H2D_P_FP16 or H2D_P_BF16 */
    double inner_tol;      /* REFINE: relative tolerance of each inner solve */
    int32_t max_outer;     /* REFINE: cap on refinement steps */
    int32_t precond;       /* h2d_precond, applied inside every (inner) GMRES */
} h2d_solve_opts;

typedef struct {
    int32_t iters;         /* total inner Arnoldi steps (matvecs of the inner operator) */
    int32_t outer;         /* refinement steps (REFINE) or restarts (PLAIN) */
    double relres;         /* true relative residual |b - A_hat x| / |b| in FP64 at exit */
    double seconds;        /* wall time of the call */
    int32_t fallback_at;   /* H2D_PC_MLP only: total Arnoldi step at which the learned
                              preconditioner was found stagnating (the estimated residual fell
                              by less than 10% over 10 steps) and the solve went on with
                              block-Jacobi (or none if not set up); -1 if it never did */
    int32_t pad;
} h2d_solve_info;

/* Solve A_hat x = b to relative residual rtol (GMRES as used in Section 5,
 * x0 = 0).  b, x: device FP64, n entries, caller order; they must not
 * overlap (EINVAL: x is cleared before b is read).  The convergence
 * test is always the true FP64 residual.  Returns OK or ENOCONV (x then holds
 * the last iterate and info->relres its residual).  The Krylov basis and
 * work vectors (about (2 restart + 6) n doubles with a preconditioner) are
 * allocated on the first solve and kept by the handle for the next ones. */
h2d_status h2d_solve(h2d_t H, const double* b, double* x, double rtol, const h2d_solve_opts* opts,
                     h2d_solve_info* info, void* stream);

/* Block-Jacobi set-up: LU with partial pivoting of every leaf's self block
 * (leaf boxes of at most 1024 points).  Needed before solving with
 * H2D_PC_BLOCK_JACOBI.  Errors: EUNSUPPORTED (a leaf above 1024 points, an
 * adaptive or symmetric handle), EINVAL (a singular self block). */
h2d_status h2d_bj_setup(h2d_t H, void* stream);

/* z = M r for one of the set-up preconditioners (device FP64 vectors in
 * caller order).  Asynchronous on `stream`. */
h2d_status h2d_precond_apply(h2d_t H, int32_t precond, const double* r, double* z, void* stream);

/* Learned per-leaf preconditioner (a shared MLP, 192 -> 256 -> 256 -> 64,
 * ReLU).  Input of leaf X: box-relative coordinates of its points and the
 * leaf residual normalised by |r_X| (64 slots each).  The correction on X
 * is in residual form: z_i = s |r_X| (r_i / |r_X| + out_i), with s the
 * least-squares scalar z ~ s r fitted on the training solves (so the
 * untrained network is the preconditioner s I).  Training pairs come from
 * the library's own solves for n_solves random r (every leaf gives
 * (r_X, z_X)): leaf-block solves z_X = K(X, X)^{-1} r_X (default), or FP64
 * GMRES solves A z = r.  The forward pass, backward pass and Adam steps run
 * in this library's FP32 kernels.  Weights: packed FP32 [W1 (256 x 192), b1, W2 (256 x 256), b2,
 * W3 (64 x 256), b3], row-major. */
#define H2D_MLP_PARAMS 131648

/* Network input.  LEAF: the leaf's own points and residual (192 values;
 * correction z_X = s |r_X| (r_X / |r_X| + out), H2D_MLP_PARAMS weights).
 * PATCH: the near-field patch -- the leaf and its edge-sharing leaves to the
 * left, right, below and above, 5 x 64 slots of (x offset, y offset from
 * the leaf's centre in half sides, r_i / |r_P|), 960 values -- and the
 * correction added to the block-Jacobi step: z_X = K(X, X)^{-1} r_X +
 * s |r_P| out, trained on what the target solve adds to the block-Jacobi
 * step (target PATCH: the restricted additive Schwarz step over the patch);
 * H2D_MLP_PARAMS_PATCH weights, block-Jacobi set up on the way.  A leaf-input
 * network cannot see the neighbours' residual, which is where restricted
 * Schwarz gains over block-Jacobi. */
typedef enum { H2D_MLP_INPUT_LEAF = 0, H2D_MLP_INPUT_PATCH = 1 } h2d_mlp_input;
#define H2D_MLP_PARAMS_PATCH 328256

typedef enum {
    H2D_MLP_TARGET_LEAF = 0,    /* z_X = K(X, X)^{-1} r_X: the method's leaf-block solves */
    H2D_MLP_TARGET_GLOBAL = 1,  /* z = A^{-1} r by FP64 GMRES, restricted to each leaf */
    H2D_MLP_TARGET_PATCH = 2    /* z_X = [K(P, P)^{-1} r_P]_X with P = X and its edge-sharing leaves
                                   (the leaf's near-field patch: the self and edge blocks the method
                                   stores dense), solved exactly; at most 320 patch points */
} h2d_mlp_target;

typedef struct {
    int32_t n_solves;      /* random right-hand sides used for training pairs */
    int32_t steps;         /* Adam steps */
    int32_t batch;         /* leaves per step */
    float lr;              /* Adam learning rate */
    uint64_t seed;         /* right-hand sides, initial weights, batches */
    double solve_tol;      /* GLOBAL targets: relative residual of the solves */
    int32_t target;        /* h2d_mlp_target */
    int32_t input;         /* h2d_mlp_input */
} h2d_mlp_train_opts;

typedef struct {
    double seconds_data;   /* data-generating solves */
    double seconds_train;  /* Adam steps */
    float loss_first, loss_last;
    int32_t n_samples;
    int32_t solves_converged;
    double scale;          /* fitted s (z ~ s r over the training solves) */
} h2d_mlp_train_info;

/* The network has 64 point slots per leaf: training and applying it on a
 * handle with a leaf above 64 points fail with EUNSUPPORTED (weights can
 * still be set on such a handle; the preconditioner then refuses to run). */
h2d_status h2d_mlp_train(h2d_t H, const h2d_mlp_train_opts* opts, h2d_mlp_train_info* info, void* stream);

/* Copy the MLP weights out (host, H2D_MLP_PARAMS floats, or
 * H2D_MLP_PARAMS_PATCH for a network trained with the patch input) and/or
 * set those of a leaf-input network (H2D_MLP_PARAMS floats); setting them
 * (host; marks the preconditioner ready).  `scale` (host, may be NULL)
 * receives the output scale s when reading and sets it when writing.
 * Any pointer may be NULL. */
h2d_status h2d_mlp_weights(h2d_t H, float* out, const float* in, double* scale, void* stream);

/* One forward + backward pass of the MLP on a batch, without a handle:
 * W (H2D_MLP_PARAMS), X (B x 192), T (B x 64 targets), M (B x 64 mask of
 * valid slots), grad (H2D_MLP_PARAMS): all device FP32, row-major.
 * *loss (host) = sum M (out - T)^2 / (2 sum M); grad = its gradient.
 * Synchronises `stream`. */
h2d_status h2d_mlp_loss_grad(const float* W, const float* X, const float* T, const float* M, int32_t B,
                             float* loss, float* grad, void* stream);

typedef struct {
    int64_t n;
    int32_t kappa, leaf_max;
    double R, tol;
    int64_t n_near;        /* dense leaf blocks (self + edge sharers) */
    int64_t n_il;          /* interaction-list blocks, all levels */
    int64_t n_il_dense;    /* interaction-list blocks stored dense */
    int64_t max_rank, sum_rank;
    int64_t u_elems, v_elems, d_elems;   /* stored values in U, V, dense pools */
    double alg_bytes_fp64; /* bytes one FP64 single-RHS matvec must move */
    double alg_bytes_half; /* same for FP16/BF16 storage */
    double flops;          /* 2 (sum_lowrank k (m + n) + sum_dense m n) */
    double build_seconds;
    uint32_t prec_mask;
    int32_t pad;
} h2d_stats;

/* Sizes, ranks and traffic of a built handle (host struct). */
h2d_status h2d_info(h2d_t H, h2d_stats* s);

/* Write H to `path` (little-endian, format "H2DX" version 1, the same the
 * CPU oracle writes; version 2 for an adaptive tree, where every near block
 * names (target level, source level, target box, source box) and every
 * compressed block also its source level).  flags bit 0: include the
 * factors (else structure only: tree, perm, levels, block tables with kinds
 * and ranks). */
h2d_status h2d_export(h2d_t H, const char* path, uint32_t flags);

/* Read a file written by h2d_export (with factors) or by the oracle and
 * upload it: the resulting handle applies exactly the stored operator.
 * The whole file is checked on the host before anything is uploaded: perm
 * a permutation of [0, n), every level's boxes non-empty, in ascending key
 * order, tiling [0, n) and nested in their parents, block indices, kinds,
 * ranks and order; a file that fails any check gives EINVAL. */
h2d_status h2d_import(const char* path, uint32_t prec_mask, void* stream, h2d_t* out);

/* Per-kernel timing of the matvec, for roofline reporting.
 * h2d_profile_enable(H, 1) makes every later single-RHS matvec on H record
 * HIP events around its five kernels (on the caller's stream, so the
 * timings cover exactly those kernels); h2d_profile_read() synchronises on
 * the recorded events, returns the average milliseconds and the
 * algorithmic bytes of each kernel over the recorded matvecs, and clears
 * the record.  At most 65536 matvecs are recorded between reads.
 * Kernels: 0 gather x into tree order; 1 phase A, t = V^T x for every
 * low-rank block; 2 sums of split phase-A partials; 3 phase B, U t (or
 * D x) for the blocks of levels 1..kappa-1 and, in the same launch, the
 * leaf-level blocks and near field; 4 combine, the two phase-B sums added
 * and written in caller order. */
typedef struct {
    int32_t count;         /* matvecs averaged */
    int32_t prec;          /* precision of the last recorded matvec */
    double ms[5];          /* average milliseconds per kernel */
    double bytes[5];       /* algorithmic bytes of each kernel per launch */
} h2d_profile;

h2d_status h2d_profile_enable(h2d_t H, int32_t on);
h2d_status h2d_profile_read(h2d_t H, h2d_profile* out);

/* Work-item sizes of the product kernels (h2d_set_item_rows, h2d_autotune). */
typedef enum {
    H2D_TILE_A_ROWS = 0,   /* V rows per single-RHS FP64 phase-A item: 16..512 (default 512) */
    H2D_TILE_MR_ROWS = 1,  /* source rows per multi-RHS FP64 phase-A item: 16..512, multiple of 16
                              (default 256) */
    H2D_TILE_B1_ROWS = 2,  /* rows per single-RHS FP64 phase-B1 item: 16, 32 or 64 (until set, chosen
                              from the sizes of the boxes one level above the leaves: 64 for
                              boxes of hundreds of points, 16 for boxes of a few) */
    H2D_TILE_B2_ROWS = 3   /* rows per single-RHS phase-B2 item (a chunk of a leaf box), every
                              precision: 16, 32 or 64 (default 64); chunks of fewer rows take
                              several column groups per wave, so big leaves spread over more
                              waves */
    /* The FP16/BF16 pools use fixed work items for the rest: phase A 512
     * rows of one source box, phase B1 64-row slices. */
} h2d_tile;

/* Tile tuning: times 5 FP64 products with nrhs right-hand sides for each
 * candidate and keeps the fastest for H.  nrhs == 1 tunes H2D_TILE_A_ROWS
 * over (128, 256, 512), then H2D_TILE_B1_ROWS over (16, 32, 64), then
 * H2D_TILE_B2_ROWS over (16, 32, 64); nrhs > 1 tunes H2D_TILE_MR_ROWS over
 * (128, 256, 512).  chosen (host, 3 ints, may be NULL) receives the picks
 * (0 past the first for nrhs > 1); ms (host, 9 floats, may be NULL) the
 * milliseconds per product of each candidate in that order. */
h2d_status h2d_autotune(h2d_t H, int32_t nrhs, void* stream, int32_t* chosen, float* ms);

/* Batched products: the FP64 products y_i = A_i x_i of `count` built
 * handles (nrhs right-hand sides each, x_i / y_i device column-major with
 * leading dimension ld[i]) are captured once into a HIP graph and replayed
 * by h2d_batch_launch with a single graph launch on the caller's stream.
 * With nrhs > 1 each block of 16 right-hand sides is one launch per phase
 * (gather, V^T X, reduction, U T and near field, scatter) covering every
 * instance; a handle listed more than once is served by further such
 * rounds.  With nrhs == 1 the instances' products run on parallel graph
 * branches.
 * The buffers are bound at creation (hosts arrays x, y, ld of length
 * count); the handles must outlive the batch, must not be used
 * concurrently with a launch, and must not be re-tuned (h2d_autotune,
 * h2d_set_item_rows) while the batch exists: the graph holds their
 * schedule and work-space addresses. */
/* Sets one work-item size (which: an h2d_tile value) explicitly; the
 * single-RHS schedule is rebuilt at once, the multi-RHS one at the next
 * multi-RHS product.  H2D_EINVAL outside the ranges listed at h2d_tile. */
h2d_status h2d_set_item_rows(h2d_t H, int32_t which, int32_t rows, void* stream);

typedef struct h2d_batch_s* h2d_batch_t;
h2d_status h2d_batch_create(h2d_t const* handles, int32_t count, int32_t nrhs, double* const* x, double* const* y,
                            const int64_t* ld, h2d_batch_t* out);
h2d_status h2d_batch_launch(h2d_batch_t B, void* stream);
void h2d_batch_destroy(h2d_batch_t B);

/* Free every allocation of H (NULL is a no-op). */
void h2d_destroy(h2d_t H);

/* Message describing the last error of the calling thread ("" if none). */
const char* h2d_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* H2D_H */
