/*
 * bsmm.h -- C ABI of libbsmm.so: local block-sparse matrix multiplication
 *           on one AMD MI355X (gfx950).
 *
 * The operation is the local multiplication of DBCSR (arXiv:1705.10218,
 * Section 2): C = alpha * op(A) * op(B) + beta * C, where every matrix is
 * stored in blocked compressed-sparse-row form -- elements grouped into
 * small dense blocks whose row and column sizes follow the atomic basis --
 * and the pattern of C is not fixed in advance but produced by the product.
 * Block products whose norm product falls below a threshold are skipped
 * during the multiplication, and result blocks below it are removed after
 * it (Section 1, two-phase filtering; Section 2, on-the-fly filtering).
 *
 * Conventions used by every entry point
 *   Layout   : block rows i = 0..nbr-1 have row_blk_size[i] >= 1 rows, block
 *              columns j have col_blk_size[j] >= 1 columns.  row_ptr (int64,
 *              nbr+1 entries, row_ptr[0] = 0, non-decreasing, row_ptr[nbr] =
 *              nnzb) and col_idx (int32, nnzb entries, strictly increasing
 *              inside each block row) index the stored blocks.  Values are
 *              FP64, one block after another in CSR order, each block
 *              column-major with leading dimension = its row count.
 *   Memory   : index arrays passed to bsmm_mat_create are host memory and are
 *              copied.  values_dev is device memory on the context's device;
 *              the library borrows it (never frees it) for matrices the caller
 *              creates, and owns the values of matrices it returns.
 *   Streams  : every device operation is ordered on the context's stream
 *              (borrowed, e.g. a torch stream; NULL = the default stream).
 *              Calls that must size a result (multiply, filter) synchronise
 *              that stream internally to read the sizes back.
 *   Errors   : every call returns a status and never throws.  On a
 *              validation error the outputs are untouched.  bsmm_last_error()
 *              returns a thread-local message describing the last failure.
 *   Threads  : one context must not be used by two host threads at once.
 */
#ifndef BSMM_H
#define BSMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsmm_ctx_s *bsmm_ctx;
typedef struct bsmm_mat_s *bsmm_mat;
typedef struct bsmm_plan_s *bsmm_plan;

typedef enum {
  BSMM_OK = 0,
  BSMM_ERR_INVALID_ARG = 1,   /* null/negative argument, bad trans character   */
  BSMM_ERR_BAD_INDEX = 2,     /* malformed row_ptr / col_idx / block sizes     */
  BSMM_ERR_SHAPE = 3,         /* operand block grids or block sizes disagree   */
  BSMM_ERR_ALIAS = 4,         /* C_old values alias A or B values              */
  BSMM_ERR_OUT_OF_MEMORY = 5, /* device memory or the context budget exhausted */
  BSMM_ERR_DEVICE = 6,        /* a HIP call failed                             */
  BSMM_ERR_UNSUPPORTED = 7    /* a size beyond what the kernels handle         */
} bsmm_status;

/* Arithmetic used by the block products (the norms, the filter thresholds
 * and the stored values are FP64 in every mode).  FP32 and SPLIT need packed
 * operand copies below 2 GB (about half the FP64 values of A and of B) and
 * at most 8 distinct k block sizes; otherwise bsmm_multiply returns
 * BSMM_ERR_UNSUPPORTED. */
typedef enum {
  BSMM_COMPUTE_FP64 = 0,      /* FP64 MFMA, FP64 accumulation                  */
  BSMM_COMPUTE_FP32 = 1,      /* operands rounded to FP32, FP32 MFMA products,
                                 FP32 accumulation over a result block, then
                                 FP64 for alpha/beta, C and its norm          */
  BSMM_COMPUTE_SPLIT = 2      /* each operand split into FP32 hi + lo parts;
                                 per k-step lo*hi + hi*lo + hi*hi on FP32
                                 MFMA, accumulated across k in FP64           */
} bsmm_compute_mode;

/* Sizes and counters of one multiplication. */
typedef struct {
  int64_t c_nnzb_symbolic;  /* blocks of C before the post-filter              */
  int64_t c_nnzb;           /* blocks of C returned                            */
  int64_t c_n_values;       /* FP64 values of C returned                       */
  int64_t n_candidates;     /* block products of the symbolic pattern          */
  int64_t n_products;       /* block products that passed the on-the-fly filter*/
  double useful_flops;      /* sum over kept products of 2*m*k*n               */
  /* device time per phase in ms (only when timing is enabled, else 0)         */
  float ms_index, ms_norms, ms_symbolic, ms_stacks, ms_gemm, ms_filter, ms_total;
  /* block-GEMM path: 0 = packed operand copies (k-pair slabs, one wavefront
     per result block), 1 = 64-bit pointer walker, 2 = tile path (2x2 tiles
     of result blocks, operands staged in LDS), 3 = FP32 / split packed path,
     4 = tile path with the uniform-size kernel (every block S x S),
     5 = packed operand copies addressed per unit (as 0, the stack entries
         holding offsets from the start of their op(A) row's and op(B)
         column's packed blocks: copies of 2 GB and more)                    */
  int32_t gemm_path;
} bsmm_multiply_info;

/* Readable name of a status code (static storage). */
const char *bsmm_status_string(bsmm_status s);
/* Detail of the last failure on this host thread (static storage per thread). */
const char *bsmm_last_error(void);

/* Create a context on HIP device `device`.  `stream` is a borrowed
 * hipStream_t (NULL = default stream).  `hbm_budget_bytes` caps the device
 * memory the library itself holds (0 = no cap beyond the device). */
bsmm_status bsmm_ctx_create(int device, void *stream, size_t hbm_budget_bytes, bsmm_ctx *out);
bsmm_status bsmm_ctx_set_stream(bsmm_ctx ctx, void *stream);
/* Enable per-phase device timing in bsmm_multiply_info (adds event records). */
bsmm_status bsmm_ctx_set_timing(bsmm_ctx ctx, int enable);
bsmm_status bsmm_ctx_set_compute_mode(bsmm_ctx ctx, bsmm_compute_mode mode);
/* Kernel variant of the FP64 block GEMM for result blocks whose edges fall
 * in the size classes of m and n (classes: edges 1-8, 9-16, 17-24, 25-32):
 *   0 = default (one 16x16x4 MFMA tile when both edges are in 9..16, 4x4x4
 *       MFMA subtiles otherwise), 1 = 16x16x4 MFMA tiles, 2 = 4x4x4 MFMA
 *       subtiles, 3 = one 16x16x4 MFMA tile carrying two block products per
 *       k-slice, one in each diagonal 8x8 quadrant (both edges <= 8 only;
 *       the stacks of such blocks are padded to groups of eight products),
 *   4 = one 16x16x4 MFMA tile plus 4x4x4 MFMA subtiles along the edges
 *       beyond 16 (both edges in 9..24, one of them above 16),
 *   5 = the tile path (both edges in 17..24): one wavefront per 2x2 tile of
 *       result blocks stages the operand blocks the tile uses at each k in
 *       LDS, read straight from the stored values (no packed copies, no
 *       2 GB limit), and runs the tile's products at that k from LDS with
 *       the MFMA layout of variant 4.  When every block of op(A), op(B)
 *       and C has the same size S and a kernel for S is built (S = 23) and
 *       the tile shape is 2x2, a kernel with S fixed at compile time runs it,
 *   6 = the tile path with the general kernel only (as 5 otherwise).
 * For the class of edges 17..24 x 17..24, variant 0 selects the tile path
 * (as variant 5) when every result block of the product is in that class
 * and every contraction extent is at most 24 (else the packed-operand
 * path).  Variants 5 and 6 give bitwise the same results.
 * The variant in force when a product is planned is the one it runs with.
 * All variants give results within FP64 rounding of each other; the choice
 * only changes speed (an autotuner picks it per size class).  Applies to the
 * packed-operand path (at most 8 distinct k sizes; copies of 2 GB or more
 * are addressed per unit, see bsmm_ctx_set_packed_addressing).
 * Errors: BSMM_ERR_INVALID_ARG for edges outside 1..32, another variant,
 * variant 3 with an edge above 8, or variant 4, 5 or 6 outside its edges. */
bsmm_status bsmm_ctx_set_gemm_variant(bsmm_ctx ctx, int32_t m, int32_t n, int32_t variant);
/* Result-block tile of the tile path (variant 5): ti x tj result blocks per
 * workgroup, each of its (ti/2)(tj/2) wavefronts owning a 2 x 2 part; an
 * operand block staged in LDS serves up to tj (A) or ti (B) products.
 * Shapes: 2x2 (default: one wavefront, no barrier), 2x4, 4x2, 4x4, 4x8,
 * 8x4 (several wavefronts sharing the staged blocks, one barrier per k).  Applies to products
 * planned afterwards; results are bitwise the same for every shape (each
 * result block sums its products in ascending k).
 * Errors: BSMM_ERR_INVALID_ARG for another shape. */
bsmm_status bsmm_ctx_set_tile_shape(bsmm_ctx ctx, int32_t ti, int32_t tj);
/* Schedule of the tile path's GEMM launch (products planned afterwards):
 * xcd_chunk = consecutive tiles handed to one XCD at a time (0 = 8192; the
 * 8 XCDs take chunks in turn, so each XCD's L2 stays on neighbouring tiles).
 * Results are bitwise the same for every chunk.  persistent must be 0: a
 * persistent launch (resident workgroups taking tiles from device ticket
 * counters) is not available.
 * Errors: BSMM_ERR_INVALID_ARG for xcd_chunk outside 0..2^30,
 * BSMM_ERR_UNSUPPORTED for persistent != 0. */
bsmm_status bsmm_ctx_set_tile_schedule(bsmm_ctx ctx, int32_t persistent, int64_t xcd_chunk);
/* Addressing of the packed operand copies (FP64, products planned
 * afterwards).  The packed path reads operand blocks through 32-bit byte
 * offsets held in the stack entries.  mode 0 (default): offsets from the
 * start of each copy while both copies stay below 2 GB, else per unit;
 * mode 1: always per unit.  Per unit, the packed blocks of every row of
 * op(A) and of every column of op(B) are laid out contiguously (op(B) = B
 * takes an index transpose of B to find its columns) and an entry's offsets
 * start at its row's and column's first block, which lifts the 2 GB limit
 * of the copies (each row or column must pack below 2 GB: its edge times
 * the sum of the padded contraction extents, times 8 bytes).  Results are
 * bitwise the same in both modes: the same products are summed in the same
 * order.
 * Errors: BSMM_ERR_INVALID_ARG for another mode. */
bsmm_status bsmm_ctx_set_packed_addressing(bsmm_ctx ctx, int32_t mode);
/* Locality order of the block rows (products planned afterwards).  For a
 * square op(A) the library can derive an order of its block rows from the
 * pattern alone (recursive bisection by breadth-first-search distance; the
 * host computes it once per matrix and keeps it with the matrix): the GEMM
 * then walks the result in tiles of neighbouring rows and the row-parallel
 * kernels take rows in that order, for reuse of op(B) blocks in L2.
 * mode 0 (default): for square operands of at least 2,048 block rows;
 * mode 1: for square operands of at least 64 block rows; mode 2: never.
 * Results are bitwise the same in every mode (each result block sums its
 * products in the same order); only speed and host time change.
 * Errors: BSMM_ERR_INVALID_ARG for another mode. */
bsmm_status bsmm_ctx_set_row_order(bsmm_ctx ctx, int32_t mode);
/* Bytes of device memory the library currently holds for this context
 * (live buffers plus its cache of freed ones). */
bsmm_status bsmm_ctx_memory(bsmm_ctx ctx, size_t *held_bytes, size_t *peak_bytes);
/* Return cached free device memory to HIP. */
bsmm_status bsmm_ctx_trim(bsmm_ctx ctx);
/* Wait for all work queued on the context's stream. */
bsmm_status bsmm_ctx_synchronize(bsmm_ctx ctx);
/* Destroy the context.  Matrices created on it must be destroyed first. */
bsmm_status bsmm_ctx_destroy(bsmm_ctx ctx);

/* Create a matrix from its block sizes and block index (host arrays, copied;
 * validated: sizes >= 1, row_ptr monotone from 0 to nnzb, col_idx in range
 * and strictly increasing per row, n_values = sum of block areas) and a
 * borrowed device buffer of n_values FP64 values in the layout above.
 * values_dev may be NULL only when n_values == 0. */
bsmm_status bsmm_mat_create(bsmm_ctx ctx, int32_t nbr, int32_t nbc,
                            const int32_t *row_blk_size, const int32_t *col_blk_size,
                            int64_t nnzb, const int64_t *row_ptr, const int32_t *col_idx,
                            double *values_dev, int64_t n_values, bsmm_mat *out);
bsmm_status bsmm_mat_info(bsmm_mat m, int32_t *nbr, int32_t *nbc, int64_t *nnzb, int64_t *n_values);
/* Copy the block index to host arrays of nbr+1 and nnzb entries. */
bsmm_status bsmm_mat_get_index(bsmm_mat m, int64_t *row_ptr_host, int32_t *col_idx_host);
/* Copy the block sizes to host arrays of nbr and nbc entries. */
bsmm_status bsmm_mat_get_block_sizes(bsmm_mat m, int32_t *row_blk_size, int32_t *col_blk_size);
/* Device pointer of the values (owned or borrowed; valid while m lives). */
bsmm_status bsmm_mat_values(bsmm_mat m, double **values_dev);
/* Copy the n_values values into a device buffer, ordered on the stream. */
bsmm_status bsmm_mat_copy_values(bsmm_mat m, double *dst_dev);
/* Destroy the handle; borrowed values are left alone, owned ones freed. */
bsmm_status bsmm_mat_destroy(bsmm_mat m);

/* Frobenius norm (FP64) of every stored block, written in storage order to
 * a device array of nnzb doubles.  The norm drives both filters (Section 1;
 * Section 2, on-the-fly filtering). */
bsmm_status bsmm_block_norms(bsmm_mat m, double *norms_dev);

/* C = alpha * op(A) * op(B) + beta * C_old   (Section 2, local multiply)
 *   transa/transb : 'N' or 'T' (op(X) = X or X^T, blocks transposed too).
 *   The block column sizes of op(A) must equal the block row sizes of op(B)
 *   one by one; C_old must have op(A)'s row sizes and op(B)'s column sizes.
 *   c_old         : may be NULL iff beta == 0 and retain_sparsity == 0; with
 *                   beta == 0 its values are never read.
 *   filter_eps    : a block product A_ik B_kj is computed iff
 *                   ||A_ik||_F * ||B_kj||_F >= filter_eps, and (unless
 *                   retain_sparsity) a result block is kept iff its norm
 *                   >= filter_eps; 0 filters nothing.
 *   retain_sparsity: the pattern of C is exactly that of C_old; products
 *                   landing outside it are dropped; no post-filter.
 *   Otherwise the pattern of C is the symbolic product pattern, united with
 *   C_old's when beta != 0, minus post-filtered blocks.
 *   *c_out receives a new matrix owning its index and values.  info may be
 *   NULL.  A and B may be the same handle.  Runs asynchronously except for
 *   the size read-backs; the result is complete when the stream reaches it.
 */
bsmm_status bsmm_multiply(bsmm_ctx ctx, char transa, char transb, double alpha,
                          bsmm_mat a, bsmm_mat b, double beta, bsmm_mat c_old,
                          double filter_eps, int retain_sparsity,
                          bsmm_mat *c_out, bsmm_multiply_info *info);

/* New matrix holding the blocks of m whose Frobenius norm is >= eps
 * (the post-multiply filter of Section 1 applied on its own). */
bsmm_status bsmm_filter(bsmm_mat m, double eps, bsmm_mat *out);

/* The filter above for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops and harnesses that forbid
 * hipMalloc): the same result as bsmm_filter, bitwise, written into
 * caller-owned device buffers on m's device, ordered on the context's stream.
 * It calls no hipMalloc, hipFree or host synchronisation.
 *   row_ptr_out : nbr + 1 entries (int64), the result's block-row pointers;
 *   col_idx_out : room for nnzb(m) entries (int32); NULL allowed iff nnzb = 0;
 *   values_out  : room for n_values(m) FP64 values; NULL allowed iff
 *                 n_values = 0 -- the kept blocks in CSR order, each as stored;
 *   counts_out  : 2 entries (int64): kept blocks, kept values.
 * Its intermediates live in one fixed device array inside the library
 * (about 22 MiB on every GPU the library runs on, held until the process
 * ends), shared by every call on that GPU: calls that overlap on one GPU
 * (from any context or stream) race, so the caller must order them.
 * Errors: BSMM_ERR_INVALID_ARG (NULL buffer, eps < 0 or NaN),
 * BSMM_ERR_UNSUPPORTED for m above 262,144 block rows or 16,777,216 blocks,
 * BSMM_ERR_ALIAS when an output overlaps m's index or values; outputs are
 * untouched on every error. */
bsmm_status bsmm_filter_noalloc(bsmm_mat m, double eps, int64_t *row_ptr_out, int32_t *col_idx_out,
                                double *values_out, int64_t *counts_out);

/* ------------------------------------------------------------- plans
 * A plan splits one multiplication (same arguments as bsmm_multiply) into
 *   - bsmm_plan_create: the structural part, run once -- validation, index
 *     views, block norms, symbolic phase, stacks with the on-the-fly filter
 *     decisions taken on the values A and B have now (synchronises the
 *     stream).  It allocates no buffer of the numeric part: the result
 *     values and the workspace are either allocated by the first
 *     bsmm_plan_execute (library-owned, within the context budget, before
 *     any kernel of that call) or supplied by the caller
 *     (bsmm_plan_sizes / bsmm_plan_execute_into).  Budget: the sizes of the
 *     result pattern, and then of the stacks, are checked against the
 *     context budget as soon as the symbolic phase has produced them and
 *     before any kernel that fills them is launched; on any failure the
 *     stream is left idle and *out untouched;
 *   - bsmm_plan_execute: the numeric part -- packed operand copies and the
 *     block GEMM -- on the context's stream, asynchronous, reading the
 *     *current* values of A, B and C_old (the matrices must stay alive and
 *     keep their patterns; their value buffers may be rewritten between
 *     executions).  It launches kernels only: no host synchronisation,
 *     allocation or memset;
 *   - bsmm_plan_capture: records the numeric part once in a HIP graph on the
 *     context's stream (which must not be the default stream); from then on
 *     bsmm_plan_execute replays the graph;
 *   - bsmm_plan_result: the post filter (if filter_eps > 0 and not
 *     retain_sparsity) and a new matrix holding the last execution's result
 *     (synchronises the stream).
 * This is the repeated-multiplication case of the iterative methods of
 * Section 1 (a fixed pattern whose values change).  info (may be NULL)
 * receives the sizes, counts and the structural phase times. */
bsmm_status bsmm_plan_create(bsmm_ctx ctx, char transa, char transb, double alpha, bsmm_mat a, bsmm_mat b,
                             double beta, bsmm_mat c_old, double filter_eps, int retain_sparsity, bsmm_plan *out,
                             bsmm_multiply_info *info);
/* Sizes of a plan's numeric part, known once bsmm_plan_create returns and
 * before anything of the result is allocated: c_nnzb and c_n_values are the
 * result's blocks and FP64 values before the post-filter (upper bounds of the
 * final result), workspace_bytes the scratch of bsmm_plan_execute_into
 * (packed operand copies, result-block norms and, with a post-filter, a copy
 * of the result values for its compaction).  Any output may be NULL. */
bsmm_status bsmm_plan_sizes(bsmm_plan plan, int64_t *c_nnzb, int64_t *c_n_values, size_t *workspace_bytes);
/* Whether the plan's on-the-fly filter decisions (taken on the values A and
 * B had at bsmm_plan_create) are still those a new plan would take on their
 * current values (Section 1: the filter is part of each multiplication):
 * *holds = 1 when every candidate product is kept or dropped as before, so
 * bsmm_plan_execute gives bitwise what a fresh bsmm_multiply would; 0
 * otherwise.  First a bound from the smallest kept and largest dropped norm
 * product and the range of block-norm ratios now / then; if inconclusive,
 * every candidate is decided again and compared.  Always 1 without a filter
 * (filter_eps 0).  Synchronises the context's stream. */
bsmm_status bsmm_plan_filter_holds(bsmm_plan plan, int32_t *holds);
/* The numeric part and the post-filter in caller-owned device buffers (e.g.
 * torch tensors): c_values_dev has room for c_n_values doubles (8-byte
 * aligned), workspace_dev for workspace_bytes (256-byte aligned); neither
 * may overlap the other or the values of A, B or C_old.  *c_out receives a
 * new matrix whose index belongs to the library and whose values are
 * c_values_dev itself (borrowed: bsmm_mat_destroy leaves them alone; the
 * post-filter compacts the kept blocks to its front).  The library allocates
 * only the result's index and the post-filter's counters.  Runs eagerly (a
 * captured graph keeps the library-owned buffers); synchronises the stream
 * only to size the post-filter's result.  Same results as bsmm_plan_execute
 * followed by bsmm_plan_result, bitwise.
 * Errors: BSMM_ERR_INVALID_ARG (NULL or misaligned buffer), BSMM_ERR_ALIAS. */
bsmm_status bsmm_plan_execute_into(bsmm_plan plan, double *c_values_dev, void *workspace_dev, bsmm_mat *c_out);
bsmm_status bsmm_plan_execute(bsmm_plan plan);
bsmm_status bsmm_plan_capture(bsmm_plan plan);
bsmm_status bsmm_plan_result(bsmm_plan plan, bsmm_mat *c_out);
/* The numeric parts of n plans of one context (each plan at most once) as
 * one batch: the operand copies of every plan, then ONE block-GEMM launch
 * over the result blocks of all of them (each wavefront takes one result
 * block of one plan), so the requests' work shares the device.  Every
 * result block is computed exactly as in a launch of its own plan, so each
 * plan's result is bitwise the one it gets alone.  Plans outside the FP64
 * packed-operand path run one after another instead.  Asynchronous: the
 * launch parameters go through a ring of four pinned staging slots, and the
 * host waits only when the copy out of the slot it reuses (four batched
 * launches back) has not run yet.  The batching of stacks across independent requests is
 * what a serving loop uses (admit requests, build their plans, execute them
 * together). */
bsmm_status bsmm_plans_execute(int32_t n, bsmm_plan *plans);
/* Waits for the plan's stream, then frees it (a plan counts as a live object
 * of its context until destroyed). */
bsmm_status bsmm_plan_destroy(bsmm_plan plan);

/* Statistics of a sign iteration. */
typedef struct {
  int32_t iterations;     /* iterations run (each forms X^2)                  */
  int32_t converged;      /* 1 if the residual fell below tol                 */
  double residual;        /* ||X^2 - I||_F / sqrt(N) of the last iterate whose
                             square was formed (N = matrix dimension)         */
  int64_t nnzb;           /* blocks of the returned matrix                    */
  int64_t nnzb_max;       /* most blocks held by any iterate or 3I - X^2      */
  double useful_flops;    /* sum over all multiplications (2*m*k*n per kept
                             block product)                                   */
  float ms_total;         /* device time when timing is enabled, else 0      */
  int32_t plan_reuses;    /* multiplications that re-executed the previous
                             step's plan (same operand patterns, filter
                             decisions provably unchanged)                    */
} bsmm_sign_info;

/* Newton-Schulz iteration for the matrix sign function (Section 1, eq. (3)
 * and the iteration that follows it): X_{n+1} = 1/2 X_n (3I - X_n^2),
 * starting from x0.  x0 must be square with equal row and column block
 * sizes; the iteration converges to sign(x0) when the spectral radius of x0
 * is below 1 and no eigenvalue is 0.
 * Each iteration is two filtered multiplications on the device: T = 3I - X X
 * (beta = 3 with the block-diagonal identity as C_old, so the pattern is the
 * union) and X = 0.5 X T, both with filter_eps for the on-the-fly and post
 * filters, so the pattern of X evolves from iteration to iteration.  Once it
 * settles, each multiplication re-executes the previous iteration's plan
 * (numeric part only) when the operand patterns are the plan's and every
 * on-the-fly filter decision provably stays the same under the new block
 * norms (the smallest kept and largest dropped norm products of the plan,
 * scaled by the extreme per-block norm ratios, stay on their sides of
 * filter_eps); the results are those of planning afresh.
 * The residual ||X_n^2 - I||_F / sqrt(N) comes from T.  The loop stops after
 * max_iter iterations, or as soon as the residual of the current iterate is
 * below tol (tol <= 0: never); the current iterate is then returned as is.
 * trace_residual and trace_nnzb (each max_iter entries, or NULL) receive the
 * residual of X_n and the block count of the matrix returned after step n.
 * x0 is not modified; *x_out is a new matrix (also when max_iter = 0: a copy).
 * Errors: BSMM_ERR_SHAPE for a non-square grid or unequal row and column
 * block sizes, BSMM_ERR_INVALID_ARG for max_iter < 0 or filter_eps < 0, and
 * every error of bsmm_multiply. */
bsmm_status bsmm_sign_newton_schulz(bsmm_ctx ctx, bsmm_mat x0, int32_t max_iter, double filter_eps, double tol,
                                    bsmm_mat *x_out, bsmm_sign_info *info, double *trace_residual,
                                    int64_t *trace_nnzb);

#ifdef __cplusplus
}
#endif
#endif /* BSMM_H */
