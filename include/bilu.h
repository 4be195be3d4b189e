/*
 * bilu.h -- C ABI of the MI355X (gfx950) decoupled block-wise ILU(k)
 * preconditioner and the Krylov solves it is applied in.
 *
 * Method: Yang, Liu, Zhong, Chen, "Decoupled Block-Wise ILU(k)
 * Preconditioner on GPU" (arXiv:1703.01325).  The calls follow the paper's
 * statement of the problem (Algorithm 5, Eq 5, Algorithm 7):
 *
 *   bilu_analyze          symbolic ILU(k) on the point-wise view of the block
 *                         pattern (Algorithm 3, Eq 1-2) and level sets for
 *                         the sweeps (Eq 4, Algorithm 6)              [host]
 *   bilu_factor_numeric   backfill A into the ILU(k) pattern and block ILU(0)
 *                         on it (Algorithm 5 steps 3-5, Algorithm 4)  [GPU]
 *   bilu_factor_diag      U = D U' (Eq 5), factors laid out for the sweeps
 *   bilu_apply            z = (L D U')^{-1} r (Eq 6, Algorithm 7)     [GPU]
 *   bilu_spmv             y = A x (or A^T x), block CSR               [GPU]
 *   bilu_solve            right-preconditioned BiCGSTAB / GMRES(m)    [GPU]
 *   bilu_grad_A           dL/dA = -lambda x^T on A's block pattern    [GPU]
 *
 * Common conventions
 * ------------------
 * - Indices are int32, 0-based.  A block pattern is block-CSR: Ap[nb+1] row
 *   starts, Aj[nnzb] block columns, strictly ascending within a block row,
 *   the diagonal block present in every row (Section 2.1).  A stored block
 *   is an entry of the pattern whatever its values.
 * - Block values: nnzb * bs * bs doubles, each bs x bs block stored column
 *   by column (Section 2.1), blocks in Aj order: element (r, c) of block e
 *   is Ax[e*bs*bs + c*bs + r].
 * - Vectors: device doubles, nb*bs rows by nrhs columns, row-major
 *   (element (i, j) at v[i*nrhs + j]).
 * - Pointers named *_dev or documented as device pointers are device memory
 *   owned by the caller; the library reads/writes them only during the call
 *   (stream-ordered).  Host arrays passed in are borrowed for the call and
 *   copied.  Host views returned by bilu_get_* are owned by the context and
 *   stay valid until bilu_destroy.
 * - Every GPU call is enqueued on `stream` and returns without waiting,
 *   except bilu_factor_numeric (reads back the singular-pivot flag) and
 *   bilu_solve (returns host-side convergence information); both
 *   synchronise `stream`.
 * - Errors are returned, never thrown; a negative status means the call did
 *   nothing useful, a positive one is a numerical outcome.  One context is
 *   used by one host thread / stream at a time.
 */
#ifndef BILU_H
#define BILU_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BILU_OK = 0,
    BILU_ERR_ARG = -1,          /* bad argument (null pointer, size, block size)   */
    BILU_ERR_ALLOC = -2,        /* host or device allocation failed                */
    BILU_ERR_HIP = -3,          /* a HIP runtime call failed                       */
    BILU_ERR_MISSING_DIAG = -4, /* a block row does not store its diagonal block   */
    BILU_ERR_PATTERN = -5,      /* unsorted / duplicate / out-of-range columns     */
    BILU_ERR_TIMEOUT = -6,      /* a sweep's bounded wait expired (results invalid)*/
    BILU_ERR_STATE = -7,        /* call order violated (e.g. apply before factor)  */
    BILU_SINGULAR_PIVOT = 1,    /* a pivot block is singular or not finite         */
    BILU_NOT_CONVERGED = 2,     /* maxit reached above the tolerance               */
    BILU_BREAKDOWN = 3,         /* BiCGSTAB rho, <r^,v> or omega became zero       */
    BILU_NONFINITE = 4          /* NaN / Inf met in the iteration                  */
} bilu_status;

/* Sweeps of the preconditioner and of its transpose (Eq 4 levels each). */
typedef enum {
    BILU_SWEEP_L = 0,   /* L y = r, forward                                 */
    BILU_SWEEP_U = 1,   /* U' x = D^{-1} y, backward                        */
    BILU_SWEEP_UT = 2,  /* U'^T w = r, forward   (transposed application)   */
    BILU_SWEEP_LT = 3   /* L^T s = D^{-T} w, backward                       */
} bilu_sweep;

typedef enum { BILU_FACTORS_FP64 = 0, BILU_FACTORS_FP32 = 1 } bilu_precision;
typedef enum { BILU_BICGSTAB = 0, BILU_GMRES = 1, BILU_ORTHOMIN = 2 } bilu_method;

/* bilu_analyze flags */
#define BILU_WANT_TRANSPOSE 1   /* also build U'^T / L^T sweeps and A^T SpMV */
#define BILU_DEVICE_SYMBOLIC 2  /* symbolic phase and level sets on the current GPU
                                   (bilu_symbolic_device / bilu_levels_device), results
                                   copied back; the same pattern and levels as the host */

typedef struct bilu_ctx bilu_ctx;

/* Sizes of an analysed pattern (filled by bilu_get_info). */
typedef struct {
    int nb, bs, k;
    int64_t nnzb_A;       /* stored blocks of A                    */
    int64_t nnzb_P;       /* blocks of the ILU(k) pattern P        */
    int64_t nnzb_L;       /* strictly lower blocks of P            */
    int64_t nnzb_U;       /* strictly upper blocks of P            */
    int nlev[4];          /* levels per sweep (0 if not built)     */
    int rows_per_chunk;   /* block rows per wavefront in the sweeps */
    int64_t sweep_slots[4]; /* padded block slots of each sweep layout */
    int tile_rows;        /* block rows per tile of the tiled sweeps (0: not chosen yet) */
    int tile_group;       /* tiles per workgroup of the tiled sweeps (1: one wavefront
                             per tile; see BILU_TUNE_TILE_GROUP)                         */
    int lds_ring[4];      /* per tiled sweep: chunks whose rows a wavefront keeps in LDS
                             (0: the whole tile; > 0 when every in-tile dependency is
                             fewer than that many chunks back, single-tile layouts only) */
    int tile_block[4];    /* per tiled sweep: ny + 256*nz when its tiles are blocks of
                             ny x nz grid lines (BILU_TUNE_TILE_BLOCK), else 0       */
    int line_sweep[2];    /* L, U' sweeps: ny + 256*nz when they run as line sweeps
                             (BILU_TUNE_LINE_SWEEP), else 0                          */
} bilu_info;

typedef struct {
    int method;      /* bilu_method                                         */
    int restart;     /* GMRES(m) restart length (ignored by BiCGSTAB)       */
    double rtol;     /* stop when ||b - A x||_2 <= rtol ||b||_2 (true res.) */
    int maxit;       /* BiCGSTAB steps / total GMRES Arnoldi steps           */
} bilu_solve_opts;

typedef struct {
    int status;      /* bilu_status of this right-hand side              */
    int iters;       /* BiCGSTAB steps or GMRES Arnoldi steps taken        */
    double relres;   /* true relative residual ||b - A x|| / ||b|| at exit */
    int restarts;    /* BiCGSTAB: restarts from the true residual, taken when
                        the recurrence residual passed the test but the
                        true one did not; GMRES: restart cycles completed   */
    int reserved;
} bilu_rhs_info;

/*
 * Symbolic phase (Algorithm 5 steps 1-2: Algorithm 3 with Eq 1-2) and the
 * level sets of Eq 4, then the layouts of the sweeps.  On the host (needs no
 * GPU) unless flags has BILU_DEVICE_SYMBOLIC.
 *   nb, bs   block rows (>= 1) and block size (1..32).  Sizes 1..8 have
 *            block-row sweep and SpMV kernels; 9..32 (the large blocks of
 *            Section 3, Table 2) factor by blocks, sweep at point
 *            granularity (bilu_apply_point) and take one right-hand side,
 *            FP64 factors, no transposed solve, no batch, no autotune, no
 *            bilu_apply_noalloc (BILU_ERR_ARG there)
 *   Ap, Aj   host block-CSR pattern of A (borrowed, copied)
 *   k        fill level (>= 0); entries with level <= k are kept
 *   flags    BILU_WANT_TRANSPOSE and/or BILU_DEVICE_SYMBOLIC, or 0
 *   out      receives a new context (free with bilu_destroy)
 * Errors: BILU_ERR_ARG, BILU_ERR_PATTERN, BILU_ERR_MISSING_DIAG,
 * BILU_ERR_ALLOC (with BILU_DEVICE_SYMBOLIC also those of
 * bilu_symbolic_device / bilu_levels_device).  Device memory is allocated on
 * first factorisation.
 */
bilu_status bilu_analyze(int nb, int bs, const int32_t* Ap, const int32_t* Aj, int k,
                         int flags, bilu_ctx** out);

/* Host views of the ILU(k) pattern P (block-CSR, ascending columns) and the
 * level of fill of each kept entry (Eq 1-2).  Owned by the context. */
bilu_status bilu_get_pattern(const bilu_ctx* ctx, int64_t* nnzb, const int32_t** Pp,
                             const int32_t** Pj, const int32_t** lev);

/* Host views of the level sets of one sweep (Eq 4, Algorithm 6): 0-based
 * levels, level_ptr[nlev+1], level_rows[nb] with rows ascending inside a
 * level.  BILU_ERR_STATE if the sweep was not built. */
bilu_status bilu_get_levels(const bilu_ctx* ctx, int sweep, int* nlev,
                            const int32_t** level_ptr, const int32_t** level_rows);

bilu_status bilu_get_info(const bilu_ctx* ctx, bilu_info* info);

/*
 * Symbolic phase on the GPU (Algorithm 3 with Eq 1-2): the ILU(k) pattern P
 * and the level of fill of every kept entry, identical to bilu_analyze's
 * (bilu_get_pattern).  Each row is searched independently: (i, j) is kept
 * with level l when the shortest path from i to j in the graph of A whose
 * inner vertices all lie below min(i, j) has l + 1 edges, which gives the
 * levels of Eq 1-2's row-by-row recurrence.
 *   nb       block rows (>= 1)
 *   Ap, Aj   device block-CSR pattern of A (Ap[nb+1], Aj[Ap[nb]]), columns
 *            strictly ascending per row, diagonal present (checked)
 *   k        fill level, 0..250
 *   Pp       device [nb+1]: receives the row pointers of P
 *   Pj, lev  device [cap] each: receive the columns (ascending per row) and
 *            levels of P; both NULL with cap = 0 to query the size
 *   nnzb     host: receives the number of entries of P
 *   stream   hipStream_t (NULL: the default stream); the call returns once
 *            the results are complete
 * Buffers are the caller's; the call allocates and frees device scratch.
 * Errors: BILU_ERR_ARG (bad argument, or cap < *nnzb: Pp and *nnzb are
 * still set), BILU_ERR_PATTERN, BILU_ERR_MISSING_DIAG, BILU_ERR_ALLOC (a
 * row's search reaches more than 768 distinct block columns, or P exceeds
 * 2^31 - 1 entries), BILU_ERR_HIP.
 */
bilu_status bilu_symbolic_device(int nb, const int32_t* Ap, const int32_t* Aj, int k, int32_t* Pp,
                                 int32_t* Pj, int32_t* lev, int64_t cap, int64_t* nnzb, void* stream);

/*
 * Level sets of one sweep on the GPU (Eq 4, Algorithm 6): the level of a row
 * is one more than the deepest row it reads, 0 for a row that reads none;
 * identical to bilu_get_levels for the same pattern.
 *   nb           block rows
 *   Pp, Pj       device pattern of P (ascending columns, diagonal present)
 *   sweep        bilu_sweep (L and U' read the rows of P below / above the
 *                diagonal; U'^T and L^T the columns)
 *   lvl          device [nb]: receives the level of every row
 *   level_ptr    device [nb+1]: receives level_ptr[0..nlev]
 *   level_rows   device [nb]: receives the rows ordered by level, ascending
 *                inside a level
 *   nlev         host: receives the number of levels
 *   stream       as for bilu_symbolic_device; the call returns once done
 * Errors: BILU_ERR_ARG, BILU_ERR_ALLOC, BILU_ERR_HIP, BILU_ERR_TIMEOUT (a
 * bounded wait expired: the pattern is not one of P's forms).
 */
bilu_status bilu_levels_device(int nb, const int32_t* Pp, const int32_t* Pj, int sweep, int32_t* lvl,
                               int32_t* level_ptr, int32_t* level_rows, int* nlev, void* stream);

/* Host-only self-check of the sweep layouts: every row appears once per
 * sweep, every index is in range, every dependency sits in a strictly
 * earlier chunk of the schedule (the persistent sweeps rely on this to
 * drain) and matches the pattern.  BILU_OK or BILU_ERR_STATE. */
bilu_status bilu_validate(const bilu_ctx* ctx);

/*
 * Factorisation phase (Algorithm 5 steps 3-5, Algorithm 4) on the GPU:
 * copies A's blocks into P (zero blocks at fill positions) and runs block
 * ILU(0) on P, block rows scheduled by the L level sets, each pivot block
 * inverted explicitly in FP64 (Gauss-Jordan, partial pivoting inside the
 * block).  Ax_dev: device values of A (layout above).  Synchronises
 * `stream`.  Returns BILU_SINGULAR_PIVOT with *bad_row (may be NULL) set to
 * the smallest block row whose pivot block is singular or not finite.
 */
bilu_status bilu_factor_numeric(bilu_ctx* ctx, const double* Ax_dev, hipStream_t stream,
                                int* bad_row);

/*
 * Diagonal factorisation U = D U' (Eq 5): D^{-1} is the block diagonal of
 * pivot inverses, U'_ij = D_i^{-1} U_ij.  Lays L, D^{-1} and U' out for the
 * level-scheduled sweeps, stored as FP64 or rounded (nearest-even) to FP32
 * (precision = bilu_precision).  Must follow bilu_factor_numeric.  The first
 * call (and the first after a change of precision or layout) allocates the
 * laid-out factors; later factorisations of the same matrix structure reuse
 * them.
 */
bilu_status bilu_factor_diag(bilu_ctx* ctx, int precision, hipStream_t stream);

/*
 * Copies the FP64 factors in pattern order to caller device buffers:
 * F_dev[nnzb_P*bs*bs] holds L at strictly lower positions, U' at strictly
 * upper positions and the identity at diagonal positions; Dinv_dev[nb*bs*bs]
 * holds D^{-1}.  Either pointer may be NULL.  The sweeps read their own
 * layouts, so F is formed from the factorisation (on `stream`) the first time
 * it is asked for after bilu_factor_diag.
 */
bilu_status bilu_get_factors(const bilu_ctx* ctx, double* F_dev, double* Dinv_dev,
                             hipStream_t stream);

/* Same, for the FP32 factors the sweeps read when precision was FP32. */
bilu_status bilu_get_factors_f32(bilu_ctx* ctx, float* F_dev, float* Dinv_dev,
                                 hipStream_t stream);

/*
 * z = M^{-1} r with M = L D U' (Eq 6, Algorithm 7): forward L sweep, D^{-1}
 * fused into the backward U' sweep.  r, z: device vectors (nb*bs x nrhs,
 * nrhs >= 1); z may not alias r.  Accumulation is FP64 whatever the factor
 * precision.  BILU_ERR_TIMEOUT if a sweep's bounded wait expired.
 */
bilu_status bilu_apply(bilu_ctx* ctx, const double* r, double* z, int nrhs,
                       hipStream_t stream);

/*
 * z = M^{-1} r through the point-granularity mechanism of Section 2.4 and
 * Algorithm 6: the split factors are expanded to point matrices (unit-
 * diagonal L and U', point row I*b + r holding row r of the blocks of block
 * row I) and swept point row by point row, level by level, with D^{-1}
 * applied by blocks between the two sweeps.  Point levels equal the block
 * levels (every point of a block row has its block row's level), and each
 * point row sums its products in the order the block sweeps use, so the
 * result is the one bilu_apply gives.  One right-hand side, not transposed.
 * The point context is analysed on the first call (host, pattern of
 * nnz(P)*b entries about) and its values expanded from the factors after each
 * factorisation (device, allocates the point matrices).  Factors must exist
 * (bilu_factor_diag), else BILU_ERR_STATE; BILU_ERR_TIMEOUT if a sweep's
 * bounded wait expired.
 */
bilu_status bilu_apply_point(bilu_ctx* ctx, const double* r, double* z, hipStream_t stream);

/*
 * bilu_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result bits as bilu_apply, with the
 * intermediate vector and the sweeps' counters in a fixed 32 MiB scratch
 * array of the library (one per device, held until the process ends); calls
 * no hipMalloc, hipFree or allocating routine.  nb*bs*nrhs doubles must fit
 * in 32 MiB - 256 bytes, else BILU_ERR_ARG.  The layouts must already hold
 * the current factors (they do after bilu_factor_diag for nrhs = 1, or after
 * one bilu_apply with the same nrhs), else BILU_ERR_STATE, as when the
 * current device is not the context's.  Every call on a device shares its
 * scratch: calls that overlap on one device (other streams, other contexts)
 * race.  An expired bounded wait is reported as for bilu_apply (bilu_check,
 * the solvers).
 */
bilu_status bilu_apply_noalloc(bilu_ctx* ctx, const double* r, double* z, int nrhs,
                               hipStream_t stream);

/* z = M^{-T} r = L^{-T} D^{-T} U'^{-T} r (needs BILU_WANT_TRANSPOSE). */
bilu_status bilu_apply_transpose(bilu_ctx* ctx, const double* r, double* z, int nrhs,
                                 hipStream_t stream);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1, needs
 * BILU_WANT_TRANSPOSE); Ax_dev as in bilu_factor_numeric; y may not alias x. */
bilu_status bilu_spmv(bilu_ctx* ctx, const double* Ax_dev, const double* x, double* y,
                      int nrhs, int transpose, hipStream_t stream);

/*
 * Solves A x = b (transpose = 0) or A^T x = b (transpose = 1) for nrhs
 * independent right-hand sides with right-preconditioned BiCGSTAB,
 * GMRES(m) (opts->restart = m, one right-hand side) or ORTHOMIN(k), the
 * reservoir simulators' method named in the paper's introduction
 * (opts->restart = k kept directions, 0..16, one right-hand side), x0 = 0,
 * FP64 vectors and reductions on the GPU.  Exit test on the true residual
 * ||b - A x||_2 <= rtol ||b||_2.  info[nrhs] (host) receives per-RHS
 * results; the return value is the worst of them.  Synchronises `stream`.
 */
bilu_status bilu_solve(bilu_ctx* ctx, const double* Ax_dev, const double* b, double* x,
                       int nrhs, const bilu_solve_opts* opts, bilu_rhs_info* info,
                       int transpose, hipStream_t stream);

/* dAx_dev[e*bs*bs + c*bs + r] = -lambda[i*bs + r] * x[j*bs + c] for every
 * stored block e = (i, j) of A: the gradient of a loss with respect to A for
 * x = A^{-1} b, given the adjoint lambda = A^{-T} dL/dx (single RHS). */
bilu_status bilu_grad_A(bilu_ctx* ctx, const double* lambda, const double* x, double* dAx_dev,
                        hipStream_t stream);

/* Launch tuning knobs (bilu_tune).  None changes any result bit. */
enum {
    BILU_TUNE_SWEEP_MODE = 0, /* 0: one launch per level; 1: one persistent launch per
                                 sweep over level chunks; 2: one persistent launch per
                                 sweep over row tiles, one wavefront per (tile,
                                 right-hand side) (default)                          */
    BILU_TUNE_TILE_ROWS = 1,  /* block rows per tile in mode 2 (capped so a tile's
                                 values fit 64 KiB of LDS); 0 = chosen by a host
                                 simulation of the tiled schedule (default)          */
    BILU_TUNE_BLOCKS = 3,     /* persistent grid in workgroups, 0 = automatic        */
    BILU_TUNE_RHS_TILE = 4,   /* right-hand-side columns per pass of the level-chunk
                                 sweeps and the SpMV when nrhs > 1: 1, 4 or 8;
                                 0 (default): 8 for the sweeps, and one SpMV pass
                                 with lanes over all columns                         */
    BILU_TUNE_FUSE_SPMV = 5,  /* 1: inside bilu_solve, each U' sweep of an application
                                 followed by an SpMV of its output runs with that
                                 SpMV in one launch (row tiles, one right-hand side,
                                 not transposed, tiles not grouped); 0 (default):
                                 separate launches                                   */
    BILU_TUNE_TILE_BLOCK = 7, /* mode 2 on a pattern in natural grid order (block rows
                                 in lines of nx, lines in planes): value ny + 256*nz
                                 makes every tile a block of ny x nz grid lines (all
                                 of their block rows), one wavefront per tile, so
                                 dependencies between neighbouring lines and planes
                                 stay inside a tile; 0 (default): row-range tiles.
                                 Falls back to row-range tiles where the pattern has
                                 no grid lines or the blocks cannot be ordered        */
    BILU_TUNE_LINE_SWEEP = 8, /* mode 2, one right-hand side, on a 7-point ILU(0)
                                 pattern in natural grid order: value ny + 256*nz runs
                                 the L and U' sweeps as line sweeps, one wavefront per
                                 block of ny x nz grid lines (ny*nz <= 64/bs) computing
                                 one diagonal of its block per step; 0 (default): off.
                                 Other patterns keep the tiled sweeps               */
    BILU_TUNE_HELPER = 9,     /* mode 2, one right-hand side: run each tile (or tile
                                 group member) with a helper wavefront in its
                                 workgroup that reads the values of other tiles and
                                 hands them over through LDS, so the tile's own
                                 loads are prefetches only.  0 (default): automatic,
                                 helpers for ungrouped tiles whose rows load six or
                                 more dependency slots ahead; 1: always (tile groups
                                 of at most 2 tiles; larger groups run without);
                                 2: never.
                                 bilu_autotune times both                           */
    BILU_TUNE_SPMV_STREAM = 10, /* A x with one right-hand side, b <= 3: 1 stages each
                                 wavefront's run of A through LDS with nontemporal
                                 whole-wavefront loads, the rows in contiguous
                                 ranges per XCD (A fetched once, x kept in L2);
                                 2: direct loads; 0 (default): staged from 2^19
                                 block rows up.  Same bits either way              */
    BILU_TUNE_RHS_PAIRS = 11, /* mode 2, an even number R >= 2 of right-hand sides on
                                 single tiles: two columns per wavefront (16-byte
                                 vector accesses, each factor block loaded once for
                                 both) where the doubled LDS fits, b <= 5 and at
                                 most 18 dependency values per lane are kept.
                                 0 (default): from 16 columns up; 1: never;
                                 2: from 2 columns up.  Same bits                  */
    BILU_TUNE_FACTOR = 13,    /* numeric factorisation: 0 (default) one persistent
                                 launch, a wavefront per row (8 rows per workgroup,
                                 4, 2 or 1 where rows need more LDS), rows waiting
                                 for their pivot rows' finished blocks instead of
                                 whole levels, where each row's blocks, pivot
                                 inverses, lists and one pivot's update blocks fit
                                 96 KiB (block sizes 1-8); 1: one launch per L
                                 level; 2 / 3: the persistent launch with 16 (where
                                 the LDS allows) / at most 4 rows per workgroup.
                                 Same bits                                          */
    BILU_TUNE_SPLIT_DINV = 12, /* one right-hand side, mode 2: form
                                 D^{-1} y by blocks ahead of the U' sweep and run that
                                 sweep unfused (2), or fuse D^{-1} into it (1);
                                 0 (default): split where U' rows keep six or more
                                 dependency slots in registers.  Same bits           */
    BILU_TUNE_SPIN_LIMIT = 14, /* polls a bounded wait of the persistent kernels
                                 makes before it gives up (the call then returns
                                 BILU_ERR_TIMEOUT, its results invalid); 0: the
                                 default, 2^24.  For tests of that error path       */
    BILU_TUNE_TILE_GROUP = 6  /* mode 2: up to this many tiles (1..4) run as the
                                 wavefronts of one workgroup, handing rows to each
                                 other through its LDS instead of global memory; a
                                 group takes tiles a fixed tile distance apart (the
                                 most frequent one between dependent rows: on a grid,
                                 the same tile of consecutive planes).  Smaller groups
                                 are used where the device's LDS or the ticket order
                                 forbids larger ones.  0 = chosen with the tile size
                                 by the host simulation (default)                    */
};
bilu_status bilu_tune(bilu_ctx* ctx, int param, int value);

typedef struct {
    int sweep_mode;     /* chosen BILU_TUNE_SWEEP_MODE                          */
    int tile_rows;      /* chosen rows per wavefront tile (mode 2)              */
    int rhs_tile;       /* chosen right-hand-side columns per pass              */
    int candidates;     /* configurations timed                                 */
    double apply_us;    /* median bilu_apply time of the chosen configuration   */
    double default_us;  /* the same for the configuration in force on entry     */
    int tile_group;     /* chosen tiles per workgroup (mode 2)                  */
} bilu_tune_result;

/* Autotuner: times bilu_apply with nrhs columns (device scratch input, 2
 * warm-ups + median of 5, HIP events on `stream`) for candidate launch
 * configurations and keeps the fastest (the one in force on entry if none
 * beats it).  Candidates: nrhs = 1, the row tiles of the four (tile size,
 * group size) pairs with the shortest simulated schedules, the best
 * ungrouped tile size, and the level-chunk form; nrhs > 1, the row tiles of
 * the simulated choice, grouped and not, and the level-chunk form with 1, 4
 * and 8 columns per pass.  Needs the factors
 * (after bilu_factor_diag); results of later calls are bit-identical to
 * those before it.  Synchronises `stream`. */
bilu_status bilu_autotune(bilu_ctx* ctx, int nrhs, hipStream_t stream, bilu_tune_result* out);

/* Synchronises `stream` and reports (then clears) a timeout recorded by any
 * sweep since the last check: BILU_ERR_TIMEOUT, else BILU_OK. */
bilu_status bilu_check(bilu_ctx* ctx, hipStream_t stream);

/* Kernel classes timed by bilu_timing. */
enum {
    BILU_K_SWEEP_L = 0, BILU_K_SWEEP_U = 1, BILU_K_SWEEP_UT = 2, BILU_K_SWEEP_LT = 3,
    BILU_K_SPMV = 4, BILU_K_FACTOR = 5, BILU_K_SPLIT = 6,
    BILU_K_SWEEP_U_SPMV = 7,    /* U' sweep with the SpMV of its output (solvers) */
    BILU_K_COUNT = 8
};

typedef struct {
    int64_t launches;   /* timed launches (a whole factorisation counts once) */
    double total_ms;    /* summed HIP-event time between their start and end  */
} bilu_kernel_time;

/* enable = 1 clears the counters and starts recording a HIP event pair on
 * the launch stream around every sweep launch, SpMV launch, numeric
 * factorisation and split; enable = 0 stops recording. */
bilu_status bilu_timing(bilu_ctx* ctx, int enable);

/* Synchronises `stream` and returns the accumulated times in
 * out[BILU_K_COUNT] (host array). */
bilu_status bilu_timing_read(bilu_ctx* ctx, hipStream_t stream, bilu_kernel_time* out);

void bilu_destroy(bilu_ctx* ctx);
const char* bilu_status_string(int status);

/* ======================================================================
 * Batches of independent systems of uneven sizes and block sizes.
 *
 * Every member is the method above on its own (Algorithm 5 for the
 * factors, Algorithm 7 for the application, the Krylov loop as in
 * bilu_solve); a batch runs the members side by side so that one sweep
 * launch, one SpMV launch and one launch per vector step serve every
 * member: the sweep launches take (member, level chunk) items from one
 * work queue, merged level by level across members.
 *
 * Batch vectors (r, z, x, y, b) are the members' vectors laid end to end,
 * member s owning unknowns [off[s], off[s+1]) with
 * off[s+1] - off[s] = nb_s * bs_s (bilu_batch_offsets); one right-hand side
 * per member.
 * ====================================================================== */
typedef struct bilu_batch bilu_batch;

typedef struct {
    int nb;              /* block rows                                     */
    int bs;              /* block size, 1..8                               */
    const int32_t* Ap;   /* block CSR structure (host, borrowed for the    */
    const int32_t* Aj;   /* call), same rules as bilu_analyze              */
} bilu_sys_desc;

/* Host analysis (Algorithm 3, Eq 4) of every member with fill level k.
 * Errors as bilu_analyze; *bad_sys (if given) names the first failing
 * member, else -1. */
bilu_status bilu_batch_create(int nsys, const bilu_sys_desc* sys, int k, bilu_batch** out,
                              int* bad_sys);

/* Host view of the vector offsets off[nsys+1] (batch-owned) and the total
 * number of unknowns off[nsys]. */
bilu_status bilu_batch_offsets(const bilu_batch* batch, const int64_t** off, int64_t* n);

/* Numeric factorisation and split of every member (Algorithm 4, Eq 5):
 * Ax_dev[s] is member s's device value array (laid out as for
 * bilu_factor_numeric); the array of pointers is host memory, borrowed for
 * the call, and the value arrays must stay valid and unchanged for later
 * bilu_batch_spmv / bilu_batch_solve calls, which read them.  Factors are
 * stored in `precision`.  On BILU_SINGULAR_PIVOT, *bad_sys and *bad_row name
 * the member and its block row.  Synchronises `stream`. */
bilu_status bilu_batch_factor(bilu_batch* batch, const double* const* Ax_dev, int precision,
                              hipStream_t stream, int* bad_sys, int* bad_row);

/* z = M_s^{-1} r for every member in one L-sweep launch and one U'-sweep
 * launch; r, z are batch vectors on the device, z may not alias r. */
bilu_status bilu_batch_apply(bilu_batch* batch, const double* r, double* z, hipStream_t stream);

/* y = A_s x for every member in one launch. */
bilu_status bilu_batch_spmv(bilu_batch* batch, const double* x, double* y, hipStream_t stream);

/* BiCGSTAB (opts->method must be BILU_BICGSTAB) on every member at once,
 * x0 = 0, with the member's own scalars and its own exit test
 * ||b_s - A_s x_s||_2 <= rtol ||b_s||_2; a member that has converged (or
 * failed) is frozen while the others go on.  info[nsys] (host) receives
 * per-member results; the return value is the worst of them.  Synchronises
 * `stream`. */
bilu_status bilu_batch_solve(bilu_batch* batch, const double* b, double* x, const bilu_solve_opts* opts,
                             bilu_rhs_info* info, hipStream_t stream);

/* Device-timed choice of the members' row-tile sizes for the batch sweeps:
 * every member's tiles are rebuilt with its default tile rows times a
 * common scale (0.25, 0.5, 1, 2, 4; at least one chunk, at most 64 KiB of
 * LDS per tile), the batch apply + SpMV pair is timed with HIP events on
 * `stream` (three pairs after one untimed), and the fastest scale is kept.
 * Results of apply, SpMV and solve do not depend on the choice.  Requires
 * factors (bilu_batch_factor); allocates three batch vectors for the time of
 * the call.  BILU_ERR_TIMEOUT if a timed sweep hit its spin limit. */
typedef struct bilu_batch_tune_info {
    double tile_scale;   /* chosen scale of the members' tile rows              */
    double pair_us;      /* apply + SpMV over the batch with it, microseconds   */
    double default_us;   /* the same with the tiles in force before the call    */
    int candidates;      /* scales timed besides the one in force               */
    int reserved;
} bilu_batch_tune_info;
bilu_status bilu_batch_autotune(bilu_batch* batch, hipStream_t stream, bilu_batch_tune_info* info);

/* Member s as a single-system context (owned by the batch: do not destroy),
 * e.g. for bilu_get_factors. */
bilu_status bilu_batch_member(bilu_batch* batch, int s, bilu_ctx** ctx);

void bilu_batch_destroy(bilu_batch* batch);

#ifdef __cplusplus
}
#endif
#endif /* BILU_H */
