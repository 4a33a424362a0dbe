/*
 * spmvc.h -- compressed sparse matrix-vector product and conjugate gradients
 * on AMD Instinct MI355X (gfx950).  C ABI of libspmvc.so.
 *
 * The operation is y = A x (Eq. 1, Section I) over a matrix that is stored
 * losslessly compressed with the schemes of Section V:
 *
 *   SPMVC_FMT_ELL  uncompressed ELL, one 4-byte column index and one 8-byte
 *                  value per element (the baseline of Section IV-B and the
 *                  "Original" row of Table II);
 *   SPMVC_FMT_DT   "Data Table": the value table V (unique values, ascending),
 *                  per row the column list S_i sorted by value and the
 *                  terminal indices T_i (Section V, Fig. 1);
 *   SPMVC_FMT_DIT  "Data+Index Table": columns replaced by displacements from
 *                  the diagonal, each row's displacement sequence registered in
 *                  a pattern table; a row stores only its pattern ID and T_i
 *                  (Section V, index-compression paragraph and sample code);
 *   SPMVC_FMT_DITV DIT with the element values registered in the table as
 *                  well (the further step Section V proposes at the end of
 *                  that paragraph): the registered key is the displacement
 *                  sequence together with T_i, so a row stores only its ID;
 *                  raw (non-dictionary) values stay per row as in DIT;
 *   SPMVC_FMT_BMASK the pattern table taken to one entry (the further
 *                  compression of the table Section V suggests, for matrices
 *                  with few distinct displacements): D = the ascending list of
 *                  every displacement col - row in the matrix (at most 64), and
 *                  per row a bitmask over D (bit k: an entry at column
 *                  row + D[k]; 4 bytes when |D| <= 32, else 8).  No pattern
 *                  table and no escape rows, however irregular the rows.  When
 *                  the matrix holds at most two distinct values they form V and,
 *                  with two, a second mask marks the entries holding V[1];
 *                  otherwise every value is stored per row in column order.
 *
 * Around the product: CG (cg_solve: FP64, mixed precision by iterative
 * refinement or by reliable updates, or preconditioned by one multicolor SymGS
 * sweep; cg_solve_noalloc: the FP64 CG without any allocation; cg_solve_mg:
 * preconditioned by a multigrid V-cycle, the iteration of Table I), SymGS
 * itself (spmv_symgs, spmv_color_order), and reverse Cuthill-McKee
 * reordering with the matching symmetric permutation (spmv_rcm,
 * spmv_permute; Section V, after Table II).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers unless the comment says "host".
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is ordered
 *     on that stream.  spmv, spmv_block and spmv_symgs (after its first
 *     call on a handle, which builds the coloring) are asynchronous;
 *     spmv_compress, spmv_decompress, cg_solve, cg_solve_noalloc,
 *     cg_solve_mg, spmv_color_order, spmv_rcm and spmv_permute synchronise
 *     `stream` before returning.
 *   - Every call returns an spmvc_status; no C++ exception crosses the ABI.
 *     After a failure spmvc_last_error() gives a thread-local message.
 *   - Indices: rows and columns are 0-based, < 2^31; row_ptr is int64.
 *   - The library never keeps a caller pointer beyond the call.
 */
#ifndef SPMVC_H
#define SPMVC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPMVC_OK = 0,
    SPMVC_EINVAL = -1,       /* bad argument (null pointer, size, aliasing, option)    */
    SPMVC_ENOMEM = -2,       /* device allocation failed                               */
    SPMVC_EUNSORTED = -3,    /* CSR columns not strictly ascending within a row        */
    SPMVC_ERANGE = -4,       /* row_ptr not monotone / column index out of range       */
    SPMVC_EHIP = -5,         /* HIP runtime error                                      */
    SPMVC_ENOTSPD = -6,      /* CG breakdown: p.Ap <= 0 or not finite                  */
    SPMVC_ENOCONV = -7,      /* CG reached max_iter without meeting the tolerance      */
    SPMVC_EUNSUPPORTED = -8  /* valid request this build does not handle (message says) */
} spmvc_status;

typedef enum { SPMVC_F64 = 0, SPMVC_F32 = 1 } spmvc_dtype;

typedef enum {
    SPMVC_FMT_ELL = 0,
    SPMVC_FMT_DT = 1,
    SPMVC_FMT_DIT = 2,
    SPMVC_FMT_DITV = 3,
    SPMVC_FMT_AUTO = 4, /* spmv_compress only: DIT, or ELL when DIT's stream would not be smaller */
    SPMVC_FMT_BMASK = 5 /* neighbour bitmask over the matrix's displacement list (see below)    */
} spmvc_format;

typedef struct spmvc_matrix_s *spmvc_matrix; /* opaque, owned by the library */

/* Options of spmv_compress (host struct; NULL = defaults shown). */
typedef struct {
    int32_t fmt;              /* spmvc_format, default SPMVC_FMT_DIT                      */
    int32_t k_max;            /* value-table capacity, 0..15, default 15                  */
    int32_t p_max;            /* pattern-table capacity, 1..2^31-2, default 65535         */
    int32_t min_pattern_rows; /* a pattern used by fewer rows is an escape, default 2     */
    int32_t f32_shadow;       /* also keep FP32 copies of V / raw values (FP32 spmv), def 1 */
} spmvc_compress_opts;

/*
 * Compress a CSR matrix with the steps of Section V: one pass over all
 * entries collects the distinct values into the ascending value table V; each
 * row's entries are ordered by value (S_i, ties by column); the end of every
 * value's run in that order is kept (T_i); for DIT the column indices become
 * displacements col - row whose per-row sequences go into a pattern table.
 *
 * Dictionary: a value enters V when 8*count > n_rows (it pays for its T byte
 * per row); of those the k_max most frequent are kept; V is sorted by IEEE-754
 * totalOrder on the bit pattern (-0.0 and +0.0 distinct, NaN payloads kept).
 * Entries whose value is not in V are "raw": they follow the coded entries,
 * by column, and keep their FP64 value.  T_i stores exclusive run ends.
 * Pattern IDs follow first occurrence (lowest row); for DITV a pattern is the
 * pair (displacement sequence, T_i) and the rows keep no T.  Escape rows --
 * rows longer than 255, and for DIT/DITV rows whose pattern is used by fewer than
 * min_pattern_rows rows or falls outside the p_max most frequent -- are kept
 * as plain CSR.  The encoding is deterministic.
 *
 * row_ptr [n_rows+1] int64, col_idx [nnz] int32, vals [nnz] FP64: device
 * arrays owned by the caller and read only during this call.  The CSR is
 * validated on the device: row_ptr[0] == 0, monotone, row_ptr[n_rows] == nnz
 * (else SPMVC_ERANGE); 0 <= col < n_cols (SPMVC_ERANGE); strictly ascending
 * columns per row (SPMVC_EUNSORTED).  On success *out receives a handle that
 * must be released with spmv_free.  n_rows == 0 or nnz == 0 is allowed.
 */
spmvc_status spmv_compress(int64_t n_rows, int64_t n_cols, int64_t nnz,
                           const int64_t *row_ptr, const int32_t *col_idx, const double *vals,
                           const spmvc_compress_opts *opts, void *stream, spmvc_matrix *out);

/*
 * y = A x (Eq. 1).  x: [n_cols], y: [n_rows], both of dtype `dt` (FP64 or
 * FP32), device, caller-owned; x and y must not overlap (SPMVC_EINVAL).
 * FP64: products and sums in FP64 (fused multiply-add allowed).  FP32: the
 * FP32 copies of V / raw values, FP32 x, FP32 accumulation.  Asynchronous.
 */
spmvc_status spmv(spmvc_matrix A, int32_t dt, const void *x, void *y, void *stream);

/*
 * Y = A X for nrhs right-hand sides, 1 <= nrhs <= 16.  Row-interleaved:
 * element (j, r) of X is X[j*ldx + r] (ldx >= nrhs), element (i, r) of Y is
 * Y[i*ldy + r] (ldy >= nrhs).  Each decoded matrix entry is applied to all
 * nrhs vectors.  Same dtype / aliasing rules as spmv.  Asynchronous.
 */
spmvc_status spmv_block(spmvc_matrix A, int32_t dt, int32_t nrhs, const void *X, int64_t ldx,
                        void *Y, int64_t ldy, void *stream);

/* Options of cg_solve (host struct; NULL = defaults shown). */
typedef struct {
    double rtol;         /* stop when ||r|| <= rtol * ||b||, default 1e-10                 */
    int32_t max_iter;    /* SpMV cap per (system, rhs) [FP64 mode; inner total in MIXED], 10000 */
    int32_t mode;        /* 0 = FP64 CG, 1 = mixed precision with iterative refinement,
                            2 = FP64 CG preconditioned by one SymGS sweep,
                            3 = mixed precision with reliable updates                     */
    double inner_rtol;   /* MIXED: inner FP32 solve tolerance relative to ||r||, 1e-5;     */
                         /* RELIABLE: fall of the recursive residual between replacements */
    int32_t max_outer;   /* MIXED: refinement steps cap; RELIABLE: replacements cap; 20   */
    int32_t check_every; /* iterations between host convergence checks, default 16 (PCG  */
                         /* and MG: check_every / 4, at least 1)                          */
    int32_t batched;     /* several systems or right-hand sides (FP64 mode): 0 = one solve  */
                         /* after another, 1 = all pairs advanced together by batched       */
                         /* kernels, 2 = the same with check_every iterations recorded once */
                         /* in a hipGraph and replayed (default).  Batched kernels take DIT */
                         /* matrices with at most two table values and no raw values;       */
                         /* other matrices are solved one after another.                    */
} spmvc_cg_opts;

/* Per (system, rhs) result (host struct). */
typedef struct {
    int32_t iters;           /* SpMVs inside the CG loop (MIXED, RELIABLE: FP32 iterations) */
    int32_t outer_iters;     /* MIXED: refinement steps; RELIABLE: FP32 segments; else 0   */
    int32_t status;          /* spmvc_status of this solve                                 */
    int32_t pad_;
    double relres_true;      /* ||b - A x|| / ||b|| recomputed in FP64 at exit             */
    double relres_recursive; /* last recursively updated residual norm / ||b||             */
} spmvc_cg_stat;

/*
 * Solve A_s x = b for n_sys independent systems, each with nrhs right-hand
 * sides, by unpreconditioned conjugate gradients from x0 = 0 (the CG part of
 * Table I: DotProduct, Waxpby, SpMV).  A: host array [n_sys] of handles (square
 * matrices).  b, x: host arrays [n_sys] of device pointers to row-interleaved
 * [n_rows_s][nrhs] FP64 blocks (for nrhs == 1, plain vectors); x is
 * overwritten with the solution (the last iterate on failure).  stat: host
 * array [n_sys*nrhs], index s*nrhs + r.  Each (system, rhs) pair stops at its
 * own tolerance.  Returns SPMVC_OK when every pair converged, else the first
 * failing pair's status (SPMVC_ENOTSPD, SPMVC_ENOCONV).  Blocking.
 * mode 1 (MIXED): outer FP64 residual r = b - A x, inner FP32 CG on A d = r
 * with FP64 dot products, FP64 update x += d; requires nrhs == 1, n_sys == 1.
 * mode 3 (RELIABLE): one CG run in FP32 (FP32 SpMV and vectors, FP64 dot
 * products) whose residual is replaced by the FP64 b - A x, with the FP32
 * update folded into the FP64 x, whenever the recursive residual has fallen
 * by inner_rtol since the last replacement; the search direction is kept
 * across replacements (reliable updates; the same stopping rule on the true
 * FP64 residual); requires nrhs == 1, n_sys == 1.
 * mode 2 (PCG): FP64 CG preconditioned by one multicolor symmetric
 * Gauss-Seidel sweep (z = M^-1 r: the sweep of spmv_symgs on A z = r from
 * z = 0; the coloring is built on first use) -- the iteration of Table I with
 * SymGS as the whole preconditioner; stops on ||r|| <= rtol ||b||; requires
 * nrhs == 1, n_sys == 1 and a non-zero diagonal in every row (SPMVC_EINVAL).
 */
spmvc_status cg_solve(const spmvc_matrix *A, int32_t n_sys, int32_t nrhs,
                      const double *const *b, double *const *x, const spmvc_cg_opts *opts,
                      spmvc_cg_stat *stat, void *stream);

/*
 * cg_solve's FP64 CG (mode 0, x0 = 0, the same kernels and results) for ONE
 * system with one right-hand side, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc): it calls no
 * hipMalloc, hipFree, hipHostMalloc or other allocating routine.  Its vectors,
 * reduction partials and scalars live in one static device region of the
 * library, 48.5 MiB per GPU (held from the first call on that GPU until the
 * process ends), so the system may have at most 2,097,152 rows (2^21) and the
 * handle's FP64 SpMV at most 65,536 blocks; larger systems give SPMVC_EINVAL
 * with a message.  The region keeps the previous call's contents and every
 * call clears what it needs.  Calls on one GPU share the region: calls that
 * overlap in time on one GPU (other threads, other streams) race and must be
 * serialised by the caller.
 *   A:      square matrix handle (any format).
 *   b, x:   device FP64 vectors [n_rows]; x is overwritten (the last iterate
 *           on failure); they must not overlap.
 *   opts:   rtol, max_iter, check_every as for cg_solve; mode must be 0; the
 *           other fields are ignored.  NULL = defaults.
 *   stat:   one host result, as for cg_solve.
 * Returns SPMVC_OK, SPMVC_ENOCONV, SPMVC_ENOTSPD or SPMVC_EINVAL.  Blocking.
 */
spmvc_status cg_solve_noalloc(spmvc_matrix A, const double *b, double *x, const spmvc_cg_opts *opts,
                              spmvc_cg_stat *stat, void *stream);

/*
 * Solve levels[0] x = b by FP64 CG preconditioned by one multigrid V-cycle
 * per iteration: the HPCG iteration of Table I (Section III), with the
 * V-cycle in that table's order.  On each level l above the coarsest: z = 0,
 * one multicolor SymGS sweep on A_l z = r, t = A_l z (SpMV), restriction by
 * injection r_{l+1}[i] = (r - t)[f2c[l][i]], the V-cycle on level l + 1,
 * prolongation z[f2c[l][i]] += z_{l+1}[i], one more SymGS sweep.  On the
 * coarsest level: z = 0 and one SymGS sweep.  The sweeps visit the colors
 * backward, then forward (so that the rows updated last, which keep zero
 * residual, are not the injection points of a grid hierarchy: greedy
 * coloring gives those color 0).
 *   levels:   host array [n_levels] of handles; levels[0] is the matrix of
 *             the system, each level square with a non-zero diagonal in every
 *             row, levels l >= 1 not empty and no larger than level l - 1.
 *   f2c:      host array [n_levels - 1] of device pointers; f2c[l] holds
 *             levels[l+1]'s row count entries (int32): the row of level l that
 *             coarse row i is injected from.  Entries must lie in
 *             [0, rows of level l) and be distinct: checked on the device at
 *             the start (SPMVC_EINVAL).  The caller keeps them alive for the
 *             call.  NULL when n_levels == 1.
 *   n_levels: 1..16; with 1 the preconditioner is one SymGS sweep (colors
 *             backward, then forward).
 *   b, x:     device FP64 vectors of levels[0]'s row count; x is overwritten
 *             (the last iterate on failure).
 *   opts:     rtol, max_iter and check_every as for cg_solve; the other fields
 *             are ignored.  NULL = defaults.
 *   stat:     one host result.
 * Stops on ||r|| <= rtol ||b||.  Returns SPMVC_OK, SPMVC_ENOCONV,
 * SPMVC_ENOTSPD or SPMVC_EINVAL (bad arguments, f2c or diagonal).  Blocking.
 */
spmvc_status cg_solve_mg(const spmvc_matrix *levels, const int32_t *const *f2c, int32_t n_levels,
                         const double *b, double *x, const spmvc_cg_opts *opts, spmvc_cg_stat *stat,
                         void *stream);

/*
 * Reverse Cuthill-McKee reordering (the reordering of matrix and vector that
 * Section V proposes after Table II, for locality of the x reads).
 *   n:        rows = columns; 0..2^31-1.
 *   row_ptr:  device int64 [n+1]; col_idx: device int32 [row_ptr[n]], strictly
 *             ascending within each row; the pattern must be structurally
 *             symmetric ((i, j) present iff (j, i) present); the diagonal is
 *             optional and ignored.  Checked on the device: SPMVC_ERANGE,
 *             SPMVC_EUNSORTED, SPMVC_EINVAL (not symmetric); rows longer than
 *             1024 entries give SPMVC_EUNSUPPORTED (ordering a row's entries
 *             takes O(length^2) work in one thread; the same limit holds for
 *             spmv_permute).
 *   perm:     device int32 [n], caller-owned output: perm[k] = the old index of
 *             the row numbered k.
 * Numbering: each connected component starts at the unnumbered row of least
 * (degree, index), degree = off-diagonal entries; breadth first, each level in
 * order of the least number among a row's neighbours in the level before,
 * then (degree, index); the whole sequence reversed.  Rows without
 * off-diagonal entries come first in index order (last after the reversal).
 * Cost: one pass per breadth-first level, plus one O(n) search per component
 * of two or more rows.  Blocking.
 */
spmvc_status spmv_rcm(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, int32_t *perm,
                      void *stream);

/*
 * B = P A P^T: row k of B is row perm[k] of A with each column j renamed to
 * the k' with perm[k'] == j; columns ascending.  Inputs as for spmv_rcm plus
 * vals (device f64 [nnz]) and perm (device int32 [n], a permutation of
 * 0..n-1, checked: SPMVC_EINVAL); symmetry is not required.  Outputs are
 * caller-owned device arrays out_row_ptr [n+1], out_col_idx [nnz],
 * out_vals [nnz] (values bit-identical).  Blocking.  x' = x[perm] then gives
 * B x' = (A x)[perm].
 */
spmvc_status spmv_permute(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                          const double *vals, const int32_t *perm, int64_t *out_row_ptr,
                          int32_t *out_col_idx, double *out_vals, void *stream);

/*
 * Rebuild the CSR matrix (columns ascending per row, values bit-identical)
 * into caller-owned device arrays row_ptr [n_rows+1], col_idx [nnz],
 * vals [nnz].  Blocking.  The lossless round trip of Section V.
 */
spmvc_status spmv_decompress(spmvc_matrix A, int64_t *row_ptr, int32_t *col_idx, double *vals,
                             void *stream);

/* Description of a compressed matrix (host struct filled by spmv_info). */
typedef struct {
    int32_t fmt;           /* spmvc_format                                                */
    int32_t K;             /* value-table entries                                         */
    int32_t P;             /* pattern-table entries (DIT, DITV); BMASK: |D|               */
    int32_t id_bytes;      /* width of a pattern ID (DIT): 1, 2 or 4; BMASK: mask width    */
    int32_t width;         /* ELL/DT slots per row, DIT longest pattern                   */
    int32_t max_raw;       /* most raw entries in one row                                 */
    int64_t n_rows, n_cols, nnz;
    int64_t n_escape_rows, n_escape_nnz, n_raw;
    int64_t bytes_stream;  /* bytes one FP64 spmv must read for the matrix (all arrays)   */
    int64_t bytes_ell;     /* the same matrix as FP64 ELL: 12 bytes per slot              */
    int64_t bytes_paper;   /* at the paper's widths: ELL 12/slot, DT 4*(len+K), DIT 4*(1+K),
                              DITV 4 per row */
    int32_t lds_windows;   /* x windows staged in LDS by the FP64 DIT kernel (0 = direct gather) */
    int32_t rows_per_block; /* rows per block of the FP64 spmv                             */
    double V[15];          /* the value table (first K entries)                           */
    int32_t kernel;        /* what an FP64 spmv launches: 0 direct gather, 1 DIT LDS walk, 2 DIT register,
                              3 DIT register, plane-marching, 4 BMASK with LDS windows */
    int32_t kernel_f32;    /* the same for FP32 (each dtype has its own configuration)   */
    int32_t rows_per_block_f32;
    int32_t block_split;   /* window-phased block SpMV (spmv_block mode 3): 1 when every pattern's
                              rows share their V[0]/V[1] split, so each window's entries are
                              summed per value run and scaled once; 0 = a weight per entry */
} spmvc_info;

spmvc_status spmv_info(spmvc_matrix A, spmvc_info *info /* host */);

/*
 * Internal arrays, for tests and tools: byte size of one array of the
 * encoding (which: see spmvc_array_id) in *bytes, and when dst is not NULL a
 * copy of it into the caller's device buffer dst (at least *bytes long;
 * blocking).  Layouts: ELL_VAL f64 / ELL_COL i32 / DT_S i32 are
 * [width][n_pad] column-major (n_pad = n_rows rounded up to 64, padding
 * column -1); IDS [n_pad] of id_bytes each (all-ones = escape row); T u8
 * [K][n_pad] (empty for DITV); PAT_OFF i32 [P][width] displacements, PAT_LEN
 * u8 [P]; PAT_T u8 [P][K] (DITV: the T of each pattern); RAW f64 in
 * slices of 64 rows, slice s at RAW_SLICE[s] (int64, elements), raw entry k
 * of row 64s+l at RAW[RAW_SLICE[s] + 64k + l]; ESC_ROWS i64, ESC_PTR i64
 * [n_esc+1], ESC_COL i32, ESC_VAL f64.  BMASK: BM_D i32 [|D|]; BM_MASK and
 * BM_VMASK [n_pad] of 4 or 8 bytes each (spmvc_info.id_bytes gives the width;
 * BM_VMASK empty unless K == 2); the values of a table-less BMASK matrix are
 * in RAW / RAW_SLICE, each row's in column order.
 */
typedef enum {
    SPMVC_ARR_ELL_VAL = 0, SPMVC_ARR_ELL_COL = 1, SPMVC_ARR_DT_S = 2, SPMVC_ARR_IDS = 3,
    SPMVC_ARR_T = 4, SPMVC_ARR_PAT_OFF = 5, SPMVC_ARR_PAT_LEN = 6, SPMVC_ARR_RAW = 7,
    SPMVC_ARR_RAW_SLICE = 8, SPMVC_ARR_ESC_ROWS = 9, SPMVC_ARR_ESC_PTR = 10,
    SPMVC_ARR_ESC_COL = 11, SPMVC_ARR_ESC_VAL = 12, SPMVC_ARR_V = 13, SPMVC_ARR_PAT_T = 14,
    SPMVC_ARR_BM_D = 15, SPMVC_ARR_BM_MASK = 16, SPMVC_ARR_BM_VMASK = 17
} spmvc_array_id;

spmvc_status spmv_get_array(spmvc_matrix A, int32_t which, void *dst, int64_t *bytes, void *stream);

/*
 * Kernel configuration of a handle's spmv (rows per block, LDS staging), set
 * for both dtypes (each dtype keeps its own configuration; spmv_tune sets the
 * tuned dtype's only).
 * rows_per_block: 256..4096, a multiple of 256 (0 = keep).  lds: 1 = stage x
 * windows in LDS when they fit, 2 = as 1, and where the windows are equally
 * spaced planes (stencil matrices) let each block march a row tile through
 * consecutive planes, reusing the windows it already holds; 0 = gather x
 * directly, -1 = keep.  Used by the
 * autotuner; every valid setting gives y within the same accuracy bound (the
 * kernels sum a row's products in different orders).
 */
spmvc_status spmv_set_config(spmvc_matrix A, int32_t rows_per_block, int32_t lds);

/*
 * Kernel of spmv_block (both dtypes).  Modes 3 and 2 apply to FP64 DIT
 * matrices with a value table of 1 or 2 entries (no raw values) and fall back
 * to mode 1 otherwise:
 *   3 = whole rows of the block in LDS, one x window at a time (nrhs 2, 4 or
 *       8, unpadded blocks: ldx == ldy == nrhs; 16-byte aligned; the default);
 *   2 = x windows of right-hand-side pairs in LDS (even nrhs and leading
 *       dimensions, 16-byte aligned blocks);
 *   1 = a group of lanes per row;
 *   0 = one lane per row for all right-hand sides.
 * Used by the autotuner; results agree within the accuracy bound.
 * SPMVC_EINVAL for other values or a null handle.
 */
spmvc_status spmv_set_block_mode(spmvc_matrix A, int32_t mode);

/*
 * Autotuner: times each candidate kernel configuration of `A` for dtype `dt`
 * and `nrhs` (spmv when nrhs == 1, else spmv_block) on scratch vectors, keeps
 * the fastest in the handle as that dtype's configuration and reports it (host
 * outputs, may be NULL).  nrhs == 1: rows per block and LDS mode (0 direct,
 * 1 windows, 2 plane-marching).  nrhs > 1: *best_lds reports the block kernel
 * (the mode of spmv_set_block_mode).
 * Results are cached per (arch, format, n_rows, P, K, dtype, nrhs) in the JSON
 * file named by $SPMVC_TUNE_CACHE when set.  Blocking.
 */
spmvc_status spmv_tune(spmvc_matrix A, int32_t dt, int32_t nrhs, void *stream,
                       int32_t *best_rows_per_block, int32_t *best_lds, double *best_us);

/*
 * The SpMV configuration the last batched cg_solve in this process chose
 * (host outputs): *form 0 = window-phased (whole right-hand-side rows of one x
 * window at a time in LDS), 1 = lane groups with two right-hand sides per
 * lane, 2 = lane groups with one per lane; *chunk = consecutive row tiles
 * handed to one XCD; *us_per_spmv = its time per batched SpMV at tuning.
 * A batched solve times every applicable (form, chunk in {8, 32, 128}) on its
 * own batch before iterating and keeps the fastest; the choice is cached per
 * batch shape (systems, rows, tiles, nrhs, longest pattern), so repeated
 * solves of one batch sum in the same order.  The environment variable
 * SPMVC_BATCHED_SPMV="form,chunk" fixes the configuration instead (a form
 * that does not apply falls back to the next).  *form = -1 before any
 * batched solve; *form = -2 when the last cg_solve that asked for batched
 * kernels (batched 1 or 2, several systems or right-hand sides) solved its
 * pairs one after another instead, because a matrix is outside what the
 * batched kernels take (see spmvc_cg_opts.batched).
 */
spmvc_status spmvc_batched_config(int32_t *form, int32_t *chunk, double *us_per_spmv);

/*
 * Symmetric Gauss-Seidel, the other kernel of the HPCG iteration (Section
 * III, Table I: SymGS beside SpMV), over the compressed matrix: `sweeps`
 * times, the rows are updated with x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii,
 * color by color -- colors 0..C-1, then C-1..0 -- where the rows of a color
 * share no entry, so each color is one parallel step.  The coloring is greedy
 * in row order over the pattern of A + A^T (each row takes the smallest color
 * no lower-numbered neighbour holds; the 27-point stencil gets its 8 parity
 * classes).  FP64; b [n_rows] and x [n_rows] are device arrays, x is read as
 * the initial guess and overwritten; they must not overlap.  Any format.
 * The first call on a handle builds the coloring (blocking, O(nnz) on the
 * host from the decompressed matrix) and must not run concurrently with other
 * calls on that handle; later calls are asynchronous on `stream`.
 * SPMVC_EINVAL: null argument, sweeps < 0, overlap, a non-square matrix or a
 * row without a non-zero diagonal entry.
 */
spmvc_status spmv_symgs(spmvc_matrix A, const double *b, double *x, int32_t sweeps, void *stream);

/*
 * The coloring spmv_symgs uses: *n_colors (host) and, when color is not NULL,
 * the color of every row into color [n_rows] int32 (device).  Builds the
 * coloring on first use, as spmv_symgs does.  Blocking.
 */
spmvc_status spmv_colors(spmvc_matrix A, int32_t *n_colors, int32_t *color, void *stream);

/*
 * The matrix in the color order of its SymGS coloring: B = P A P^T, where P
 * lists the rows color by color (colors ascending, each color's rows
 * ascending), so that each color is one contiguous range of B's rows.  B is a
 * new handle (release with spmv_free), compressed with A's options; its
 * coloring is the one induced from A's (spmv_colors on B gives color c to rows
 * n_0 + ... + n_{c-1} .. n_0 + ... + n_c - 1), not a coloring of B's own, so
 * spmv_symgs on B with b' = b[perm], x' = x[perm] performs the same updates as
 * on A and returns x' = x[perm] (up to the order of each row's sum).  With
 * every color contiguous, a sweep's color steps read b and write x with
 * coalesced accesses.  perm: device int32 [n], caller-owned output (may be NULL):
 * perm[k] = the row of A that is row k of B.  A must be square with a non-zero
 * diagonal in every row (SPMVC_EINVAL); SPMVC_EUNSUPPORTED when B cannot be
 * compressed in A's format (e.g. BMASK with more than 64 displacements after
 * the reordering).  Blocking.  (On the 27-point stencil the sweep gains little
 * from the contiguous colors -- each color step is bound by its chain of
 * dependent loads -- while B's SpMV loses the few dense x windows of A's
 * natural order, so cg_solve keeps A's order.)
 */
spmvc_status spmv_color_order(spmvc_matrix A, spmvc_matrix *B, int32_t *perm, void *stream);

/*
 * Device memory of the library (handle arrays, solver vectors, scratch):
 * from now on allocated with alloc_fn(bytes, stream, ctx) and released with
 * free_fn(ptr, stream, ctx) -- e.g. a framework's caching allocator -- instead
 * of hipMalloc / hipFree.  `stream` is passed as NULL (the null stream): the
 * memory must be usable on any stream once alloc_fn returns, and the library
 * frees a buffer only after the work that used it has finished on its stream
 * (spmv_compress, cg_solve and spmv_colors synchronise; handle arrays are
 * freed by spmv_free, after which the caller must not have work in flight
 * on the handle).  alloc_fn returning NULL gives SPMVC_ENOMEM.  Buffers keep
 * the allocator that made them and are returned to it, so the hooks may be
 * changed at any time; both NULL restores hipMalloc / hipFree.  alloc_fn and
 * free_fn must both be set or both be NULL (else SPMVC_EINVAL).  Process-wide.
 */
spmvc_status spmvc_set_allocator(void *(*alloc_fn)(size_t bytes, void *stream, void *ctx),
                                 void (*free_fn)(void *ptr, void *stream, void *ctx), void *ctx);

/*
 * Debug aid.  A library built with -DSPMVC_CHECK (the package's build with
 * check=True: libspmvc_check.so) bounds-checks every gathered column and
 * every LDS index in its SpMV, block SpMV, batched and SymGS kernels; an
 * index out of range is recorded and the access redirected in bounds, so a
 * wrong index is reported here rather than read out of bounds.  *count
 * (host): nonzero when a kernel met an index out of range since the last
 * call (then reset; it counts the kernel sources that did, not the
 * accesses); waits for the device first.  *checked (host): 1 in a checked
 * build, else 0 (and *count is always 0).
 */
spmvc_status spmvc_check_violations(int64_t *count, int32_t *checked);

/*
 * Debug aid, checked builds only: one kernel passes the index i against the
 * range [0, n) through the kernels' bounds check (and nothing else), so that
 * a test can see that an index out of range is recorded and reported by
 * spmvc_check_violations.  Blocking (on stream).  The release library
 * returns SPMVC_EUNSUPPORTED.
 */
spmvc_status spmvc_check_probe(int64_t i, int64_t n, void *stream);

void spmv_free(spmvc_matrix A);

const char *spmvc_status_string(int32_t status);
const char *spmvc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPMVC_H */
