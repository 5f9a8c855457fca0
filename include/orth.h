/*
 * orth.h -- C ABI of the MI355X (gfx950) block-orthogonalisation library.
 *
 * The library solves, once per block-Krylov step, the project-and-normalize
 * (PQR) problem of Dreier & Engwer, "A Hardware-aware and Stable
 * Orthogonalization Framework" (arXiv 2204.13393), eq. (1.1):
 *
 *     [Q W] = [Q U] [[I, H], [0, R]],   Q^T U = 0,  U^T U = I,
 *
 * where Q (n x k) is the basis built by earlier steps, W (n x s) the new
 * block, H = Q^T W (k x s) the projection coefficients ("P" in the paper),
 * R (s x s) the upper-triangular normaliser with positive diagonal ("N" in
 * the paper) and U (n x s) the explicit new orthonormal block.  The method
 * is TreeTSPQR (Sec. 4.1): the rows are split into leaves, every leaf
 * solves its local PQR problem with BCGS-PIP+ (CholeskyQR2, Sec. 3.1), and
 * one reduction PQR problem on the stacked leaf coefficient blocks, also
 * solved with BCGS-PIP+, yields H and R.  The basis is never stored
 * explicitly: it lives in the caller-provided workspace in the paper's
 * locally orthogonal form Q = blockdiag(Q_1..Q_p) [T_1; ...; T_p] (Sec. 4.1),
 * per-leaf local bases Q_i plus per-leaf upper-triangular tree factors T_i.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All matrices the caller passes are IEEE FP64, column-major with a
 *    leading dimension (BLAS convention): element (r, c) of an n x s matrix
 *    at ptr[c*ld + r].
 *    A contiguous torch tensor of shape (s, n) is such a matrix with ld = n.
 *  - Pointers named d_* are device pointers (HIP device memory of the
 *    current device).  The caller owns every device buffer, including the
 *    workspace; the library never allocates or frees device memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every compute entry point only enqueues work on that stream and returns
 *    without synchronising; results are valid once the stream has reached
 *    that point.
 *  - Return values: ORTH_OK or one of the error codes below.  Argument and
 *    capacity errors are detected on the host before any work is enqueued
 *    and leave the handle's state unchanged.  Numerical breakdown (a
 *    Cholesky pivot that is not positive and finite, Sec. 3.1: the textbook
 *    Cholesky is not rank revealing) is detected on the device; it is
 *    reported by orth_status, after which the handle is poisoned.
 *  - No C++ exception crosses this boundary.  Functions are not thread-safe
 *    on the same handle.
 */
#ifndef ORTH_H_
#define ORTH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orth_ctx orth_t;

enum orth_code {
    ORTH_OK = 0,
    ORTH_ERR_ARG = 1,        /* invalid argument (size, pointer, ld, alignment) */
    ORTH_ERR_CAPACITY = 2,   /* k + s would exceed k_max */
    ORTH_ERR_BREAKDOWN = 3,  /* device reported a non-positive / non-finite pivot */
    ORTH_ERR_HIP = 4,        /* a HIP runtime call failed (no device, launch error) */
    ORTH_ERR_POISONED = 5,   /* handle saw a breakdown earlier; only destroy works */
    ORTH_ERR_WORKSPACE = 6,  /* workspace missing, too small or misaligned */
    ORTH_ERR_UNSUPPORTED = 7, /* valid request the library does not implement */
    ORTH_ERR_SCRATCH = 8     /* the request needs more than the fixed scratch of
                                orth_apply_Q_noalloc */
};

/*
 * Storage form of the leaf bases.  Arithmetic is FP64 in every form; the
 * bases, tree factors, s x s factors and H, R, U are FP64.
 *   ORTH_FP64           every pass reads the FP64 leaf bases.
 *   ORTH_MIXED_SPLIT32  the leaf bases are also kept as an FP32 copy
 *                       (rounded to nearest), and the first CholeskyQR
 *                       sweep's Gram product (Sec. 3.1) runs on the FP32
 *                       matrix cores: it reads that copy (4 instead of 8
 *                       bytes per basis entry), rounds W to FP32 in
 *                       registers, accumulates in FP32 over 64 rows at a
 *                       time and in FP64 beyond, so P1 and N1 are accurate
 *                       to about 1e-7 relative.  The correction
 *                       u1 = (w - q P1) N1^{-1}, the second sweep and the
 *                       assembly of U are FP64 on the FP64 bases, so
 *                       w = q P1 + u1 N1 holds in the stored basis and the
 *                       reiteration wins the accuracy back (Sec. 3.1):
 *                       results match the FP64 form to rounding.  Leaf
 *                       bytes per step drop from 32 to 28 per basis entry
 *                       (plus 4 bytes per new entry written); the workspace
 *                       grows by 4 bytes per leaf basis entry.  The first
 *                       sweep stays stable while about 1e-7 kappa^2 << 1/2
 *                       (kappa the condition number of the projected
 *                       block); when a leaf's pivot fails in that sweep,
 *                       the step redoes its first sweep in FP64 from the
 *                       FP64 bases on the device (no host synchronisation;
 *                       counted by orth_mixed_fallbacks), so the mixed form
 *                       breaks down only where the FP64 form does.  Also
 *                       for batches: each instance keeps its own copy and
 *                       redoes only its own first sweep (counted by
 *                       orth_batch_mixed_fallbacks).
 *   ORTH_FP64_HOUSEHOLDER  the leaves run the Householder method (Sec. 2.2,
 *                       Algorithm "HH") instead of BCGS-PIP+: each leaf basis
 *                       is held as unit reflectors (column c zero above leaf
 *                       row c) with its compact-WY factor T_i (k_max x k_max
 *                       per leaf in the workspace).  A step forms Q_k^T w
 *                       (Gram, T^T M, row update), factors w~[k:] by
 *                       Householder in one workgroup per leaf, grows T from
 *                       [V v_new]^T v_new, and assembles U = Q_{k+s}[C; 0]
 *                       with a row update; the reduction level stays
 *                       BCGS-PIP+ (the paper's proposed combination, Sec.
 *                       5.2).  The leaves never break down, so a leaf whose
 *                       local block is nearly dependent is fine; the
 *                       reduction still needs u kappa^2 <= 1/2 for the
 *                       global block.  Results equal the FP64 form's to
 *                       rounding where both succeed.  Limits (else
 *                       UNSUPPORTED): every leaf at most 8192 rows for
 *                       s <= 4, 4096 for s = 8 and s = 32 (s = 32 in
 *                       8-column sub-panels), 1024 for s = 16 (the panel
 *                       is held in registers), and (k_max s + s^2) doubles
 *                       within 160 KB (the per-leaf products' LDS staging:
 *                       k_max <= 608 at s = 32).
 *                       orth_apply_Q forms Q_k [C_i; 0] per leaf through
 *                       the same compact-WY products; orth_export_local
 *                       exports the reflectors as d_Qloc.  Also for
 *                       batches (orth_batch_create).
 */
enum orth_precision {
    ORTH_FP64 = 0,
    ORTH_MIXED_SPLIT32 = 1,
    ORTH_FP64_HOUSEHOLDER = 2
};

/* Variant of the leaf and reduction subalgorithm (Sec. 3, Sec. 3.1). */
enum orth_variant {
    ORTH_PIP_PLUS = 0,       /* BCGS-PIP+ (CholeskyQR2): the default, O(eps) */
    ORTH_PIP = 1,            /* BCGS-PIP (one CholeskyQR sweep), O(eps kappa^2):
                                kept to reproduce the paper's unstable column */
    ORTH_HOUSEHOLDER = 2     /* Algorithm HH (Sec. 2.2); the reduction only
                                (orth_set_level_variants) */
};

/*
 * orth_workspace_bytes -- device workspace size for orth_create.
 * Resource management: sizes the storage of the locally orthogonal basis
 * (Sec. 4.1: per-leaf local bases Q_i and tree factors T_i, k_max columns
 * each) plus the step's scratch; no passage defines the call itself.
 *   n          rows of the basis (>= 1)
 *   s          block width, one of 1, 2, 4, 8, 16, 32
 *   k_max      largest basis width the handle will reach (multiple of s,
 *              s <= k_max, k_max + s <= 2048); a step that would pass it
 *              fails with CAPACITY
 *   leaf_rows  TSQR leaf height; 0 picks the default
 *              max(k_max, min(n, 4096)); leaves are
 *              p = max(1, n / leaf_rows) row blocks of leaf_rows rows, the
 *              last one taking the remainder; leaf_rows must be >= k_max so
 *              every local problem keeps full column rank, and <= n
 *   precision  ORTH_FP64 or ORTH_MIXED_SPLIT32
 * Returns 0 for invalid arguments.  Pure host arithmetic, no HIP call.
 */
size_t orth_workspace_bytes(int64_t n, int32_t s, int32_t k_max,
                            int32_t leaf_rows, int32_t precision);

/*
 * orth_create -- make a handle with an empty basis (k = 0).
 * Resource management: carves the workspace into the locally orthogonal
 * representation of Sec. 4.1 (an empty one: the first orth_step is the
 * tree TSQR of the start block, Sec. 4.1, as the block Arnoldi process of
 * Sec. 2 starts from the QR of its start block).
 *   d_workspace      device buffer of >= orth_workspace_bytes(...) bytes,
 *                    256-byte aligned; owned by the caller, must outlive
 *                    the handle and must not be touched while it lives
 *   stream           stream all later calls enqueue on
 *   out              receives the handle
 * Enqueues the zero fill of the tree-factor storage on `stream`.
 * Errors: ARG, WORKSPACE, UNSUPPORTED, HIP.
 */
int orth_create(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows,
                int32_t precision, void *d_workspace, size_t workspace_bytes,
                void *stream, orth_t **out);

/*
 * orth_tree_workspace_bytes / orth_create_tree -- as orth_workspace_bytes
 * and orth_create, with the reduction problem itself solved by TreeTSPQR
 * (Sec. 4.1: the reduction step is a PQR problem on an orthonormal matrix,
 * so the method can be "applied recursively"; the recursion-levels
 * experiment of Sec. 6.1): level-1 nodes take fan_in consecutive leaves,
 * level-2 nodes fan_in level-1 nodes, and so on up to one root; the last
 * node of a level takes the children that remain.  Every node solves its
 * local PQR problem on its children's stacked [[S_c, P_c], [0, N_c]] with
 * the reduction subalgorithm and passes [P_v; N_v] up; the down-sweep forms
 * each child's coefficient block C_c = [S_v,c Y~_v,c] C_v.  The basis is
 * Q = blockdiag(Q_i) B_1 ... B_L with B_l the block-diagonal matrix of
 * level-l node factors (each node stores one k_max x k_max block per child).
 *   fan_in   0 (or >= the number of leaves): the single reduction level of
 *            orth_create; otherwise >= 2
 * The workspace grows by the upper levels' factors (about 1 / (fan_in - 1)
 * of the level over the leaves).  Any leaf form; the nodes' subalgorithm is
 * the reduction variant (orth_set_level_variants, ORTH_HOUSEHOLDER
 * included).  Not with deflation (orth_set_deflation: UNSUPPORTED).  Errors
 * as orth_workspace_bytes and orth_create (fan_in < 0 or = 1: ARG).
 */
size_t orth_tree_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows,
                                 int32_t precision, int32_t fan_in);
int orth_create_tree(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t precision,
                     int32_t fan_in, void *d_workspace, size_t workspace_bytes, void *stream,
                     orth_t **out);

/*
 * Tile shapes of the leaf passes (resource management; the launch-shape
 * entries of the local-problem-size study, Sec. 6.2): how many rows of a
 * leaf one workgroup takes in the leaf Grams and in the leaf row updates,
 * and which row-update kernel runs for s >= 16.
 *   gram_rows      0 (the plan's own: 2048, halved for small problems down
 *                  to 128 while a launch has fewer workgroups than the GPU
 *                  has compute units) or a power of two in [128, 8192].
 *                  Other heights change the order in which the leaf Grams'
 *                  partial sums are added (results to rounding).
 *   update_rows    0 (the plan's own: 512, halved the same way down to 64)
 *                  or a power of two in [64, 8192]; results unchanged.
 *   update_kernel  ORTH_TILE_AUTO: LDS-staged row updates for s >= 16 where
 *                  their layout conditions hold (even leaf heights or one
 *                  leaf), register-streamed otherwise; ORTH_TILE_REGISTER:
 *                  the register-streamed kernel at every width (results
 *                  unchanged: the two kernels form the same products).
 */
typedef struct orth_tiles {
    int32_t gram_rows;
    int32_t update_rows;
    int32_t update_kernel;
} orth_tiles;

enum orth_tile_kernel {
    ORTH_TILE_AUTO = 0,
    ORTH_TILE_REGISTER = 1
};

/*
 * orth_tiles_workspace_bytes / orth_create_tiles -- as
 * orth_tree_workspace_bytes and orth_create_tree with the given tile shapes
 * (tiles may be NULL: the plan's own).  Smaller Gram tiles mean more partial
 * sums, so the workspace depends on gram_rows.  Errors as orth_create_tree;
 * invalid tile values: ARG (orth_tiles_workspace_bytes returns 0).
 */
size_t orth_tiles_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows,
                                  int32_t precision, int32_t fan_in, const orth_tiles *tiles);
int orth_create_tiles(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t precision,
                      int32_t fan_in, const orth_tiles *tiles, void *d_workspace,
                      size_t workspace_bytes, void *stream, orth_t **out);

/* orth_tiles_in_use -- the tile shapes the handle's plan resolved (heights
 * in rows, never 0).  Host state only.  Errors: ARG. */
int orth_tiles_in_use(const orth_t *h, orth_tiles *tiles);

/* orth_tree_levels -- number of reduction levels (1 for a single level) and
 * the fan-in in use (0 for a single level).  Host state only.  Resource
 * management of the Sec. 4.1 recursion, no further passage. */
int orth_tree_levels(const orth_t *h, int32_t *levels, int32_t *fan_in);

/*
 * orth_export_tree_level -- copy reduction level `level`'s stacked node
 * factors out (Sec. 4.1: each node's k x k block per child, children in
 * order; level 0 stacks the leaves' blocks, as orth_export_local's d_T)
 * into d_T, a (children * k) x k matrix, ldt >= children * k.  For tests and
 * inspection.  Enqueued on the handle's stream.  Errors: ARG, POISONED, HIP.
 */
int orth_export_tree_level(orth_t *h, int32_t level, double *d_T, int64_t ldt);

/*
 * orth_flat_workspace_bytes / orth_create_flat -- a handle that solves the
 * PQR problem (eq. (1.1)) with FlatTSPQR (Sec. 4.2, Algorithm "FlatTSPQR")
 * instead of TreeTSPQR.  The rows are cut into p = max(1, n / block_rows)
 * blocks (the last takes the rest), handled one after the other: block 1's
 * local problem is the PQR problem of its rows against its own factor F_1,
 * block i's is the PQR problem of [W_i; P_{i-1}; N_{i-1}] against F_i
 * extended by zero rows for N_{i-1}'s new coordinates; the last block's P
 * and N are the call's H and R.  The basis is the chain
 *   Q = [[F_1, 0], [0, I]] [[F_2, 0], [0, I]] ... F_p
 * (F_i spans block i's rows and the k coordinates before it), held as the
 * factors; orth_step's explicit U and orth_apply_Q run down that chain.
 *   n, s, k_max   as orth_create (FP64 only; the local subalgorithm is
 *                 orth_set_variant's, BCGS-PIP+ by default)
 *   block_rows    kmax <= block_rows <= n (no default)
 *   d_workspace, workspace_bytes, stream, out   as orth_create
 * The workspace holds every factor ((block rows + k_max) x k_max doubles,
 * padded) and a staging copy of every block's rows, about
 * 8 n (k_max + s) bytes.  The p local problems run in sequence, each on a
 * single block, so a call takes p times the latency of a leaf level: the
 * flat form suits few blocks (the paper's setting: blocks that do not fit
 * one memory level at once) where TreeTSPQR spreads the leaves over the chip.
 * Not supported on such a handle (UNSUPPORTED): orth_apply_Q_noalloc,
 * orth_export_local, orth_export_tree_level, deflation.  orth_leaf_count
 * reports (p, block_rows); orth_tree_levels reports 0 levels.
 * Errors: ARG (shapes, block_rows), UNSUPPORTED (k_max + s above the widest
 * basis), WORKSPACE, HIP.  orth_flat_workspace_bytes returns 0 for invalid
 * arguments; pure host arithmetic.
 */
size_t orth_flat_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t block_rows);
int orth_create_flat(int64_t n, int32_t s, int32_t k_max, int32_t block_rows, void *d_workspace,
                     size_t workspace_bytes, void *stream, orth_t **out);

/*
 * orth_set_variant -- choose ORTH_PIP_PLUS (default; BCGS-PIP+, Sec. 3.1)
 * or ORTH_PIP (BCGS-PIP, Sec. 3) for the following steps.  Host-side only.  Errors: ARG, POISONED, UNSUPPORTED
 * (ORTH_PIP on an ORTH_FP64_HOUSEHOLDER handle).
 */
int orth_set_variant(orth_t *h, int32_t variant);

/*
 * orth_set_level_variants -- the subalgorithm of each level separately: the
 * leaves' local problems and the reduction problem (Sec. 4.1 lets each be
 * any PQR method; the experiments of Sec. 6 vary them independently).
 * orth_set_variant(h, v) equals orth_set_level_variants(h, v, v).  The
 * leaves of an ORTH_FP64_HOUSEHOLDER handle run the Householder method:
 * their variant must stay ORTH_PIP_PLUS (else UNSUPPORTED), the reduction's
 * may be any.
 * reduction_variant = ORTH_HOUSEHOLDER: every reduction problem by
 * Algorithm HH (the stability table of Sec. 6.1 runs one method at every
 * level).  Each reduction node's basis is then held as unit reflectors over
 * its stacked rows (its children's segments of k_max rows; each call's s new
 * coordinates of a segment are zero rows of the older reflectors) with its
 * compact-WY factor, and one workgroup factors each node's panel: offered
 * when every node's rows (children x k_max; all p leaves for the single
 * level, fan_in leaves or nodes on an orth_create_tree handle) are at most
 * 8192 (s <= 4), 4096 (s = 8), 1024 (s = 16), with k_max s <= 4096, without
 * deflation, chosen before the first step or kept (a switch to or from it
 * once k > 0 is UNSUPPORTED).  The workspace of such handles holds 3 k_max^2
 * doubles per node for the factors.  R's diagonal
 * then carries the Householder signs and U's columns the same signs: (H,
 * R D, U D) with D = diag(sign R_jj) is the unique solution.
 * orth_export_local's d_T and orth_export_tree_level are UNSUPPORTED then
 * (the stored reduction factors are reflectors).
 * Host-side only.  Errors: ARG, POISONED, UNSUPPORTED.
 */
int orth_set_level_variants(orth_t *h, int32_t leaf_variant, int32_t reduction_variant);

/*
 * orth_set_deflation -- deflation at the reduction level (Sec. 3.1) for the
 * following steps: the reduction's first sweep takes the eigen
 * decomposition G - P^T P = V Lambda V^T in place of the Cholesky
 * factorisation and keeps the t eigenvalues above (delta ||W||_F)^2, i.e.
 * the directions whose residual singular value exceeds delta ||W||_F.
 *   t = s   the step is the plain one (R triangular, as without deflation);
 *   t < s   R = [Lambda~^{1/2} V~^T; 0] (kept eigenvalues in decreasing
 *           order, each eigenvector signed so that its entry of largest
 *           magnitude is positive), then the second sweep (ORTH_PIP_PLUS
 *           reduction) multiplies by its s x s factor diag(L, 0) from the
 *           left (R = N2 N1).  Columns t..s-1 of U and rows t..s-1 of R
 *           are zero, and the basis still grows by s columns (the zero
 *           ones included: a zero column of a later W is dropped again, and
 *           orth_apply_Q's coefficients for them do not matter).
 *   delta   0 turns deflation off (the default; a rank-deficient block then
 *           breaks down); 0 < delta < 1 turns it on.  The Gram matrix holds
 *           rounding errors of about 1e-16 ||W||_F^2, so delta should stay
 *           well above 1e-8 (1e-6 is a safe choice).
 * The rank of the latest step is on the device; orth_deflation_info reads
 * it.  Only ORTH_FP64_HOUSEHOLDER handles deflate: BCGS-PIP leaves break
 * down on a block that is rank deficient as a whole, since every leaf's
 * part of it is rank deficient too; and only for s <= 16 (the eigen
 * solver's width).  Host-side only.
 * Errors: ARG (delta < 0, >= 1 or NaN), POISONED, UNSUPPORTED (other forms,
 * s = 32).
 */
int orth_set_deflation(orth_t *h, double delta);

/*
 * orth_deflation_info -- synchronise the handle's stream and read the
 * deflation record (the rank t of the t < s case of eq. (1.1), Sec. 1, as
 * the truncated decomposition of Sec. 3.1 decides it).  Any output pointer may be NULL.
 *   rank     t of the latest step taken with deflation on (s before any)
 *   steps    steps so far with t < s
 *   dropped  columns dropped so far (sum of s - t)
 * Handles that cannot deflate report s, 0, 0.  Errors: ARG, HIP.
 */
int orth_deflation_info(orth_t *h, int32_t *rank, int64_t *steps, int64_t *dropped);

/*
 * orth_step -- solve the PQR problem eq. (1.1) for the new block W and grow
 * the basis by s columns (Sec. 4.1, TreeTSPQR; one step of the block
 * Arnoldi process, Sec. 2).
 *   d_W, ldw   n x s input block, ldw >= n.  May alias d_U (read before U
 *              is written in the same step).
 *   d_H, ldh   k x s output, H = Q^T W; ldh >= max(1, k).  May be NULL when
 *              k = 0 (the first step is the QR of the start block).
 *   d_R, ldr   s x s output, upper triangular with positive diagonal, zeros
 *              written below the diagonal; ldr >= s.  (A deflating step,
 *              see orth_set_deflation, writes the row-padded t x s factor.)
 *   d_U, ldu   n x s output, the explicit new orthonormal block; ldu >= n.
 * H and R may point into the caller's block Hessenberg matrix (column block
 * j: d_H at its top, d_R = d_H + k with ldh = ldr = its leading dimension).
 * On success the basis width becomes k + s (on the host at once).
 * Errors: ARG, CAPACITY, POISONED, HIP; BREAKDOWN later via orth_status.
 */
int orth_step(orth_t *h, const double *d_W, int64_t ldw,
              double *d_H, int64_t ldh, double *d_R, int64_t ldr,
              double *d_U, int64_t ldu);

/*
 * orth_apply_Q -- Y = Q C with the current basis Q (n x k), C (k x m).
 * The second-stage product "QC" of Sec. 5.1: one sweep over the tree
 * factors, then the leaf products Y_i = Q_i C_i.  Used for Ritz vectors and
 * for the explicit basis (C = I).
 *   d_C, ldc   k x m, ldc >= k;  m >= 1
 *   d_Y, ldy   n x m output, ldy >= n; must not overlap the workspace or C.
 * Errors: ARG (also for k = 0), POISONED, HIP.
 */
int orth_apply_Q(orth_t *h, const double *d_C, int64_t ldc, int32_t m,
                 double *d_Y, int64_t ldy);

/*
 * orth_apply_Q_noalloc -- orth_apply_Q for callers that cannot allocate
 * device memory at the time of the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * result and errors as orth_apply_Q (the same kernels, bit for bit); the
 * per-leaf coefficient blocks that orth_apply_Q keeps in the handle's
 * workspace live instead in a fixed 32 MiB device array inside the library
 * (one per GPU, held until the process ends).  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine) and records no
 * profiler events.
 *   Limit: one column of coefficient blocks takes ldt = p * k_max doubles
 *   (rounded up to an odd multiple of 32), twice that for an
 *   ORTH_FP64_HOUSEHOLDER handle; it must fit the 4 Mi doubles of the array,
 *   else ORTH_ERR_SCRATCH (checked before anything is enqueued).  Columns
 *   are processed in blocks of min(16, 4 Mi / that size).
 *   Every call on one GPU shares that GPU's array: calls that overlap in
 *   time on one GPU (other streams, other handles, other threads) race and
 *   must be ordered by the caller.  Nothing in the array needs to start at
 *   zero (every entry a call reads it has written first).
 * Errors: ARG (also for k = 0), POISONED, SCRATCH, HIP.
 */
int orth_apply_Q_noalloc(orth_t *h, const double *d_C, int64_t ldc, int32_t m,
                         double *d_Y, int64_t ldy);

/*
 * orth_status -- synchronise the handle's stream and read the device status
 * (breakdown: a Cholesky pivot that is not positive and finite; Sec. 3.1
 * notes that the textbook Cholesky is not rank revealing).
 *   status  receives ORTH_OK or ORTH_ERR_BREAKDOWN.  After a breakdown the
 *           handle is poisoned.
 *   info    optional (may be NULL): 4 ints {tree level (0 = leaves,
 *           1 = the reduction level over them, l + 1 = level l of a
 *           reduction tree), leaf or node index, CholeskyQR sweep (1 or 2),
 *           pivot column}.  The first failure wins; when several leaves fail in
 *           the same launch, which of them is recorded depends on the
 *           order the workgroups ran in (the breakdown itself does not).
 * Errors: ARG, HIP.
 */
int orth_status(orth_t *h, int32_t *status, int32_t *info);

/*
 * orth_mixed_fallbacks -- (the mixed form; the reiteration of Sec. 3.1
 * restores accuracy only where the first sweep did not break down)
 * synchronise the handle's stream and read how many
 * steps of the mixed form redid their first CholeskyQR sweep from the FP64
 * bases (0 for the FP64 form).  Errors: ARG, HIP.
 */
int orth_mixed_fallbacks(orth_t *h, int64_t *count);

/* orth_basis_width -- current k (host state, no synchronisation).
 * Resource management, no passage: the k of eq. (1.1) for the next step. */
int orth_basis_width(const orth_t *h, int32_t *k);

/* orth_leaf_count -- number of leaves p and the leaf height in use (the
 * local problem size of Sec. 4.1 and Sec. 6.2).  Host state only. */
int orth_leaf_count(const orth_t *h, int32_t *p, int32_t *leaf_rows);

/*
 * orth_export_local -- copy the locally orthogonal representation out, for
 * inspection and tests (Sec. 4.1): the stacked local bases
 * blockdiag(Q_1..Q_p) flattened to an n x k matrix (leaf i's rows hold Q_i)
 * into d_Qloc (ldq >= n), and the tree factors T_i (k x k, upper
 * triangular) stacked into a (p*k) x k matrix d_T (ldt >= p*k).  For an
 * ORTH_FP64_HOUSEHOLDER handle d_Qloc receives the leaf reflectors.
 * Either destination may be NULL.  Enqueued on the handle's stream.
 * Errors: ARG, POISONED, HIP.
 */
int orth_export_local(orth_t *h, double *d_Qloc, int64_t ldq,
                      double *d_T, int64_t ldt);

/*
 * orth_destroy -- release the host state.  The workspace stays owned by the
 * caller.  Always allowed, also on a poisoned handle; NULL is a no-op.
 * Resource management, no passage.
 */
int orth_destroy(orth_t *h);

/* ------------------------------------------------------------------------
 * Batched form: `count` independent bases (uneven n, s, k_max) advance one
 * orth_step together.  Each step is a fixed sequence of grouped launches,
 * one per phase over all instances (TreeTSPQR's local problems and
 * reductions are independent across instances, Sec. 4.1), with no host
 * synchronisation and no allocation, so whole runs can be captured in a
 * hipGraph.  Every instance works at k = step * s_i.  Phases are launched
 * once per block width present in the batch.
 * ------------------------------------------------------------------------ */
typedef struct orth_batch_ctx orth_batch_t;

/*
 * orth_batch_workspace_bytes -- workspace for orth_batch_create (resource
 * management: one Sec. 4.1 representation per instance).  Host arrays
 * of `count` entries: n[i], s[i], k_max[i] as for orth_workspace_bytes;
 * leaf_rows may be NULL (default height for every instance) or hold 0 for
 * the default.  The batch runs min_i(k_max[i] / s[i]) steps.  precision
 * ORTH_FP64, ORTH_MIXED_SPLIT32 or ORTH_FP64_HOUSEHOLDER, for every instance
 * (each instance within that form's limits, as for orth_workspace_bytes).
 * Returns 0 for invalid or unsupported arguments.
 */
size_t orth_batch_workspace_bytes(int32_t count, const int64_t *n, const int32_t *s,
                                  const int32_t *k_max, const int32_t *leaf_rows,
                                  int32_t precision);

/*
 * orth_batch_create -- empty bases for every instance (Sec. 4.1
 * representation, k = 0; resource management).  Copies the instance
 * descriptors and launch tables into the workspace and zero-fills the tree
 * factors on `stream`, then synchronises that stream (creation only).
 * Errors: ARG, WORKSPACE, UNSUPPORTED, HIP.
 */
int orth_batch_create(int32_t count, const int64_t *n, const int32_t *s, const int32_t *k_max,
                      const int32_t *leaf_rows, int32_t precision, void *d_workspace,
                      size_t workspace_bytes, void *stream, orth_batch_t **out);

/* orth_batch_set_variant -- ORTH_PIP_PLUS (default, Sec. 3.1) or ORTH_PIP
 * (Sec. 3) for all instances, at both levels; a batch of Householder leaves
 * takes ORTH_PIP_PLUS only (UNSUPPORTED otherwise). */
int orth_batch_set_variant(orth_batch_t *b, int32_t variant);

/*
 * orth_batch_step -- one PQR step (eq. (1.1)) for every instance, each by
 * TreeTSPQR with BCGS-PIP+ leaves and reduction (Sec. 4.1, Sec. 3.1); the
 * instances' local problems are independent (Sec. 4.1), so one launch per
 * phase serves them all.
 *   d_W     DEVICE array of `count` device pointers: instance i's new block,
 *           n_i x s_i, column-major, ld = n_i (may alias the matching d_U[i])
 *   d_U     DEVICE array: explicit new blocks, n_i x s_i, ld = n_i
 *   d_Hess  DEVICE array: instance i's K_i x K_i column-major buffer
 *           (K_i = k_max[i], ld = K_i); call j writes [H; R] (rows
 *           0 .. (j+1) s_i - 1) into its column block j (columns
 *           j s_i .. (j+1) s_i - 1), R with zeros below its diagonal
 * The pointer arrays are read by the kernels when they run, so a captured
 * graph replays with whatever they hold then.
 * Errors: ARG, CAPACITY (all steps done), POISONED, HIP; breakdown via
 * orth_batch_status.
 */
int orth_batch_step(orth_batch_t *b, const double *const *d_W, double *const *d_U,
                    double *const *d_Hess);

/*
 * orth_batch_status -- synchronise and read the batch status word (a
 * Cholesky pivot that is not positive and finite, Sec. 3.1).  info (may
 * be NULL): 5 ints {instance, level, leaf, sweep, column} of the first
 * breakdown.  After a breakdown the batch is poisoned.  Errors: ARG, HIP.
 */
int orth_batch_status(orth_batch_t *b, int32_t *status, int32_t *info);

/*
 * orth_batch_mixed_fallbacks -- (the mixed form; the reiteration of Sec. 3.1
 * restores accuracy only where the first sweep did not break down)
 * synchronise the batch's stream and read how many (instance, step) pairs
 * redid their first CholeskyQR sweep from the FP64 bases (0 for an FP64
 * batch).  Errors: ARG, HIP.
 */
int orth_batch_mixed_fallbacks(orth_batch_t *b, int64_t *count);

/* orth_batch_progress -- steps taken and the number of steps the batch
 * allows (host state; resource management, no passage). */
int orth_batch_progress(const orth_batch_t *b, int32_t *steps_done, int32_t *steps_max);

/* orth_batch_leaf_rows -- the leaf height chosen for every instance (count
 * ints): the local problem size of Sec. 4.1 / Sec. 6.2.  Host state. */
int orth_batch_leaf_rows(const orth_batch_t *b, int32_t *leaf_rows);

/* orth_batch_destroy -- release the host state (NULL is a no-op).
 * Resource management, no passage. */
int orth_batch_destroy(orth_batch_t *b);

/* ---- leaf-height autotuner -------------------------------------------------
 *
 * The local problem size is the free parameter of TreeTSPQR (Sec. 4.1): the
 * leaves stream n x k bytes whatever their height, while the reduction level
 * grows with the number of leaves p = n / leaf_rows (it holds p (k+s) rows).
 * Its best value depends on the machine and is found by measurement (the
 * local problem size study of Sec. 6.2; Sec. 5.1 ties it to the memory
 * hierarchy).
 *
 * orth_tune_leaf_rows times `steps` calls (k = 0, s, 2s, ...) on synthetic
 * blocks (uniform in [-1, 1), a fixed hash of the call index, row and column)
 * for every candidate leaf height
 *     {256, 512, ..., 65536} restricted to [k_max, n], and n itself if n <= 65536,
 * through one handle (copies = 1, orth_step) or through a batch of `copies`
 * identical instances (orth_batch_step; this saturates the GPU as a large
 * batch does).  Among candidates within 2% of the fastest the tallest is
 * written to *best_leaf_rows.  Synchronous: it waits for `stream` after
 * every call.
 *   copies        1 .. 4096
 *   d_workspace   device memory, 256-byte aligned, of at least
 *                 orth_tune_workspace_bytes(n, s, k_max, copies) bytes, owned
 *                 by the caller; its contents are overwritten.
 *   steps         calls per candidate, 1 <= steps <= k_max / s.
 *   cand_rows, cand_ms (may be NULL when max_cand = 0): arrays of max_cand
 *                 entries receiving every candidate and its time in ms for
 *                 the `steps` calls (a negative time marks a candidate whose
 *                 run broke down); *ncand (may be NULL) receives the
 *                 candidate count.
 * Errors: ARG (sizes as for orth_create, steps or copies out of range, no
 * candidate), WORKSPACE, HIP, BREAKDOWN (every candidate broke down).
 * orth_tune_workspace_bytes returns 0 for invalid sizes.
 */
size_t orth_tune_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t copies);
int orth_tune_leaf_rows(int64_t n, int32_t s, int32_t k_max, int32_t steps,
                        int32_t copies, void *d_workspace, size_t workspace_bytes,
                        void *stream, int32_t *best_leaf_rows, int32_t *cand_rows,
                        double *cand_ms, int32_t max_cand, int32_t *ncand);

/*
 * orth_tune_tree_workspace_bytes / orth_tune_tree -- the reduction tree's
 * fan-in for single handles (the recursion of Sec. 4.1; the tree fan-in
 * entry of the tuner's search space).  For the given leaf height it times
 * `steps` calls (the synthetic blocks of orth_tune_leaf_rows) through
 * orth_create_tree handles of every candidate fan-in: 0 (the single
 * reduction level), then 2, 4, 8, ... below the leaf count, and writes the
 * fastest to *best_fan_in (the single level when it is within 2% of the
 * fastest).  Synchronous.  Workspace, steps, cand_fan_in / cand_ms / ncand
 * and errors as orth_tune_leaf_rows (ARG also for leaf_rows outside
 * [k_max, n]); orth_tune_tree_workspace_bytes returns 0 for invalid sizes.
 */
size_t orth_tune_tree_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows);
int orth_tune_tree(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t steps, void *d_workspace,
                   size_t workspace_bytes, void *stream, int32_t *best_fan_in, int32_t *cand_fan_in,
                   double *cand_ms, int32_t max_cand, int32_t *ncand);

/*
 * orth_tune_tiles_workspace_bytes / orth_tune_tiles -- the tile shapes of
 * the leaf passes (orth_tiles; the rows-per-tile and kernel-variant entries
 * of the tuner's search space) for single handles of the given leaf height,
 * single reduction level.  It times `steps` calls (the synthetic blocks of
 * orth_tune_leaf_rows) through orth_create_tiles handles of every candidate:
 * the plan's own choice {0, 0, ORTH_TILE_AUTO} first, then gram_rows in
 * {1024, 2048, 4096} x update_rows in {256, 512, 1024, 2048}, each with
 * ORTH_TILE_AUTO and, for s >= 16, ORTH_TILE_REGISTER; and writes the fastest
 * to *best (the plan's own when it is within 2% of the fastest).
 * Synchronous.  Workspace, steps, cand / cand_ms / ncand and errors as
 * orth_tune_tree; orth_tune_tiles_workspace_bytes returns 0 for invalid
 * sizes.
 */
size_t orth_tune_tiles_workspace_bytes(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows);
int orth_tune_tiles(int64_t n, int32_t s, int32_t k_max, int32_t leaf_rows, int32_t steps, void *d_workspace,
                    size_t workspace_bytes, void *stream, orth_tiles *best, orth_tiles *cand, double *cand_ms,
                    int32_t max_cand, int32_t *ncand);

#ifdef __cplusplus
}
#endif

#endif /* ORTH_H_ */
