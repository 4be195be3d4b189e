/*
 * bilu_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 reference implementation of the
 * decoupled block-wise ILU(k) preconditioner of Yang, Liu, Zhong and Chen,
 * "Decoupled Block-Wise ILU(k) Preconditioner on GPU" (arXiv:1703.01325),
 * together with the Krylov loops it is applied in.  Only the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU library never links, includes or calls anything in this directory,
 * and this file uses nothing from the GPU library.
 *
 * Conventions (Section 2.1): block-CSR with 0-based int32 indices, sorted
 * unique column indices per block row, every block stored densely and
 * column by column, element (r, c) of block e at X[e*b*b + c*b + r].
 *
 * Readings of points the paper leaves open are listed where they are used.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_PATTERN (-5)
#define ORC_ERR_MISSING_DIAG (-4)
#define ORC_ERR_ALLOC (-2)
#define ORC_SINGULAR 1
#define ORC_NOT_CONVERGED 2
#define ORC_BREAKDOWN 3

/* Largest block size: the large blocks of Section 3 (Table 2 uses b = 25)
 * fit; the blocks live on the stack in the factorisation and the solves. */
#define ORC_MAX_B 32

/* ------------------------------------------------------------------------ */
/* Pattern store in the spirit of imatcsr_t (Section 2.1, Fig. 3): row      */
/* lengths plus one separately allocated column array per row, so a row can */
/* be edited without moving the rest of the matrix.                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    int *nz;      /* number of kept entries per row            */
    int **cols;   /* cols[i][0..nz[i]) ascending               */
    int **lev;    /* level of fill of each kept entry (Eq 1-2) */
} orc_pattern;

static void pattern_free(orc_pattern *P)
{
    if (!P) return;
    for (int i = 0; i < P->n; i++) {
        free(P->cols ? P->cols[i] : NULL);
        free(P->lev ? P->lev[i] : NULL);
    }
    free(P->cols);
    free(P->lev);
    free(P->nz);
    free(P);
}

/* Checks a block pattern: row pointers monotone, columns in range, strictly
 * ascending in each row, diagonal present. */
int orc_check_pattern(int n, const int *Ap, const int *Aj)
{
    if (n < 0 || Ap[0] != 0) return ORC_ERR_PATTERN;
    for (int i = 0; i < n; i++) {
        if (Ap[i + 1] < Ap[i]) return ORC_ERR_PATTERN;
        int has_diag = 0;
        for (int e = Ap[i]; e < Ap[i + 1]; e++) {
            if (Aj[e] < 0 || Aj[e] >= n) return ORC_ERR_PATTERN;
            if (e > Ap[i] && Aj[e] <= Aj[e - 1]) return ORC_ERR_PATTERN;
            if (Aj[e] == i) has_diag = 1;
        }
        if (!has_diag) return ORC_ERR_MISSING_DIAG;
    }
    return ORC_OK;
}

/*
 * Symbolic phase, Algorithm 3 with the level rule of Eq 1 and Eq 2.
 *
 * The block matrix is first viewed as a point-wise matrix whose entries are
 * the stored blocks (Section 2.3, first step of Algorithm 5): Ap/Aj are used
 * directly, and a stored block counts as an entry whatever its values.
 *
 * For each row i, in increasing order:
 *   - every stored (i, j) starts at level 0, everything else at infinity
 *     (Eq 1);
 *   - the lower columns p < i are visited in increasing order, including
 *     fill entries created earlier in the same row, and only those whose
 *     current level is <= k are used as pivots;
 *   - for every kept entry (p, j) of row p with j > p the level of (i, j)
 *     becomes min(lev(i,j), lev(i,p) + lev(p,j) + 1) (Eq 2);
 *   - when all pivots are done, entries with level > k are removed and the
 *     rest is kept (readings: "keep lev <= k", the removal test applies to
 *     every column of the row once the row is finished).
 * Dropped entries of earlier rows never feed Eq 2: any sum through one of
 * them already exceeds k.
 */
int orc_symbolic(int n, const int *Ap, const int *Aj, int k, orc_pattern **out)
{
    int st = orc_check_pattern(n, Ap, Aj);
    if (st != ORC_OK) return st;
    if (k < 0) return ORC_ERR_PATTERN;
    const int INF = 0x3fffffff;
    orc_pattern *P = (orc_pattern *)calloc(1, sizeof(orc_pattern));
    if (!P) return ORC_ERR_ALLOC;
    P->n = n;
    P->nz = (int *)calloc((size_t)n + 1, sizeof(int));
    P->cols = (int **)calloc((size_t)n + 1, sizeof(int *));
    P->lev = (int **)calloc((size_t)n + 1, sizeof(int *));
    int *levrow = (int *)malloc(((size_t)n + 1) * sizeof(int)); /* dense level of row i */
    int *touched = (int *)malloc(((size_t)n + 1) * sizeof(int)); /* columns with finite level */
    int *lower = (int *)malloc(((size_t)n + 1) * sizeof(int));   /* sorted lower columns    */
    if (!P->nz || !P->cols || !P->lev || !levrow || !touched || !lower) {
        free(levrow); free(touched); free(lower); pattern_free(P);
        return ORC_ERR_ALLOC;
    }
    for (int j = 0; j < n; j++) levrow[j] = INF;

    for (int i = 0; i < n; i++) {
        int ntouched = 0, nlower = 0;
        for (int e = Ap[i]; e < Ap[i + 1]; e++) {
            int j = Aj[e];
            levrow[j] = 0;
            touched[ntouched++] = j;
            if (j < i) lower[nlower++] = j;   /* already ascending */
        }
        /* Visit lower columns in ascending order; the list grows as fill
         * appears, and a new column is always inserted after the current
         * position because it exceeds the current pivot p. */
        for (int t = 0; t < nlower; t++) {
            int p = lower[t];
            int lip = levrow[p];
            if (lip > k) continue;
            for (int q = 0; q < P->nz[p]; q++) {
                int j = P->cols[p][q];
                if (j <= p) continue;
                int cand = lip + P->lev[p][q] + 1;
                if (levrow[j] == INF) {
                    touched[ntouched++] = j;
                    levrow[j] = cand;
                    if (j < i) {
                        /* insertion into the sorted tail lower[t+1..] */
                        int pos = nlower;
                        while (pos > t + 1 && lower[pos - 1] > j) {
                            lower[pos] = lower[pos - 1];
                            pos--;
                        }
                        lower[pos] = j;
                        nlower++;
                    }
                } else if (cand < levrow[j]) {
                    levrow[j] = cand;
                }
            }
        }
        /* Keep the entries with level <= k, sorted by column. */
        int keep = 0;
        for (int t = 0; t < ntouched; t++)
            if (levrow[touched[t]] <= k) keep++;
        P->nz[i] = keep;
        P->cols[i] = (int *)malloc((size_t)(keep > 0 ? keep : 1) * sizeof(int));
        P->lev[i] = (int *)malloc((size_t)(keep > 0 ? keep : 1) * sizeof(int));
        if (!P->cols[i] || !P->lev[i]) {
            free(levrow); free(touched); free(lower); pattern_free(P);
            return ORC_ERR_ALLOC;
        }
        int m = 0;
        for (int t = 0; t < ntouched; t++) {
            int j = touched[t];
            if (levrow[j] <= k) {
                /* insertion sort: rows are short */
                int pos = m;
                while (pos > 0 && P->cols[i][pos - 1] > j) {
                    P->cols[i][pos] = P->cols[i][pos - 1];
                    P->lev[i][pos] = P->lev[i][pos - 1];
                    pos--;
                }
                P->cols[i][pos] = j;
                P->lev[i][pos] = levrow[j];
                m++;
            }
        }
        for (int t = 0; t < ntouched; t++) levrow[touched[t]] = INF;
    }
    free(levrow);
    free(touched);
    free(lower);
    *out = P;
    return ORC_OK;
}

long long orc_pattern_nnz(const orc_pattern *P)
{
    long long s = 0;
    for (int i = 0; i < P->n; i++) s += P->nz[i];
    return s;
}

void orc_pattern_export(const orc_pattern *P, int *Pp, int *Pj, int *lev)
{
    Pp[0] = 0;
    for (int i = 0; i < P->n; i++) {
        for (int q = 0; q < P->nz[i]; q++) {
            Pj[Pp[i] + q] = P->cols[i][q];
            if (lev) lev[Pp[i] + q] = P->lev[i][q];
        }
        Pp[i + 1] = Pp[i] + P->nz[i];
    }
}

void orc_pattern_free(orc_pattern *P) { pattern_free(P); }

/*
 * Level of every row for a level-scheduled sweep (Eq 4, Algorithm 6):
 * l(i) = 1 + max l(j) over the entries the row depends on, with an empty
 * max taken as 0.  Returned 0-based (l(i) - 1).  which:
 *   0  L   sweep, forward : depends on j < i with (i, j) in P
 *   1  U'  sweep, backward: depends on j > i with (i, j) in P
 *   2  U'^T sweep, forward: row j depends on i < j with (i, j) in P
 *   3  L^T sweep, backward: row p depends on i > p with (i, p) in P
 * Returns the number of levels.
 */
int orc_levels(int n, const int *Pp, const int *Pj, int which, int *lvl)
{
    int nlev = 0;
    for (int i = 0; i < n; i++) lvl[i] = 0;
    if (which == 0) {
        for (int i = 0; i < n; i++) {
            int m = 0;
            for (int e = Pp[i]; e < Pp[i + 1]; e++)
                if (Pj[e] < i && lvl[Pj[e]] + 1 > m) m = lvl[Pj[e]] + 1;
            lvl[i] = m;
        }
    } else if (which == 1) {
        for (int i = n - 1; i >= 0; i--) {
            int m = 0;
            for (int e = Pp[i]; e < Pp[i + 1]; e++)
                if (Pj[e] > i && lvl[Pj[e]] + 1 > m) m = lvl[Pj[e]] + 1;
            lvl[i] = m;
        }
    } else if (which == 2) {
        /* the level of row i is final once every i' < i has been pushed */
        for (int i = 0; i < n; i++)
            for (int e = Pp[i]; e < Pp[i + 1]; e++)
                if (Pj[e] > i && lvl[i] + 1 > lvl[Pj[e]]) lvl[Pj[e]] = lvl[i] + 1;
    } else {
        for (int i = n - 1; i >= 0; i--)
            for (int e = Pp[i]; e < Pp[i + 1]; e++)
                if (Pj[e] < i && lvl[i] + 1 > lvl[Pj[e]]) lvl[Pj[e]] = lvl[i] + 1;
    }
    for (int i = 0; i < n; i++)
        if (lvl[i] + 1 > nlev) nlev = lvl[i] + 1;
    return nlev;
}

/* Level sets: level_ptr[nlev+1], level_rows[n], rows ascending in a level. */
void orc_level_sets(int n, const int *lvl, int nlev, int *level_ptr, int *level_rows)
{
    for (int l = 0; l <= nlev; l++) level_ptr[l] = 0;
    for (int i = 0; i < n; i++) level_ptr[lvl[i] + 1]++;
    for (int l = 0; l < nlev; l++) level_ptr[l + 1] += level_ptr[l];
    int *fill = (int *)malloc(((size_t)nlev + 1) * sizeof(int));
    for (int l = 0; l < nlev; l++) fill[l] = level_ptr[l];
    for (int i = 0; i < n; i++) level_rows[fill[lvl[i]]++] = i;
    free(fill);
}

/* ------------------------------------------------------------------------ */
/* Dense b x b block helpers (column-major).                                */
/* ------------------------------------------------------------------------ */

/* C = A * B */
static void blk_mul(int b, const double *A, const double *B, double *C)
{
    for (int c = 0; c < b; c++)
        for (int r = 0; r < b; r++) {
            double s = 0.0;
            for (int t = 0; t < b; t++) s += A[t * b + r] * B[c * b + t];
            C[c * b + r] = s;
        }
}

/* C -= A * B */
static void blk_mul_sub(int b, const double *A, const double *B, double *C)
{
    for (int c = 0; c < b; c++)
        for (int r = 0; r < b; r++) {
            double s = 0.0;
            for (int t = 0; t < b; t++) s += A[t * b + r] * B[c * b + t];
            C[c * b + r] -= s;
        }
}

/* Explicit inverse of a b x b block by Gauss-Jordan elimination with partial
 * (row) pivoting inside the block.  Reading: the paper asks for the inverse
 * of the pivot block (Algorithm 4) and applies D^{-1} as a matrix-vector
 * product (Algorithm 7), so the inverse is formed explicitly, in FP64.
 * Returns 0, or 1 if a pivot is zero or not finite. */
static int blk_inv(int b, const double *A, double *Ainv)
{
    double W[ORC_MAX_B * 2 * ORC_MAX_B];   /* augmented [A | I], row-major */
    int w = 2 * b;
    for (int r = 0; r < b; r++)
        for (int c = 0; c < b; c++) {
            W[r * w + c] = A[c * b + r];
            W[r * w + b + c] = (r == c) ? 1.0 : 0.0;
        }
    for (int col = 0; col < b; col++) {
        int piv = col;
        double best = fabs(W[col * w + col]);
        for (int r = col + 1; r < b; r++)
            if (fabs(W[r * w + col]) > best) { best = fabs(W[r * w + col]); piv = r; }
        if (!(best > 0.0) || !isfinite(best)) return 1;
        if (piv != col)
            for (int c = 0; c < w; c++) {
                double t = W[col * w + c]; W[col * w + c] = W[piv * w + c]; W[piv * w + c] = t;
            }
        double d = W[col * w + col];
        for (int c = 0; c < w; c++) W[col * w + c] /= d;
        for (int r = 0; r < b; r++) {
            if (r == col) continue;
            double f = W[r * w + col];
            if (f == 0.0) continue;
            for (int c = 0; c < w; c++) W[r * w + c] -= f * W[col * w + c];
        }
    }
    for (int r = 0; r < b; r++)
        for (int c = 0; c < b; c++) Ainv[c * b + r] = W[r * w + b + c];
    return 0;
}

static int find_col(const int *Pj, int lo, int hi, int j)
{
    for (int e = lo; e < hi; e++)
        if (Pj[e] == j) return e;
    return -1;
}

/*
 * Factorisation phase, Algorithm 5 steps 3-5 and Algorithm 4.
 *
 * A' is the pattern P (from the symbolic phase) holding A's blocks where A
 * stores them and zero blocks at the fill positions.  Then block ILU(0) on
 * A', block rows in increasing order:
 *     for each p < i with (i, p) in P, ascending:
 *         A'_ip <- A'_ip * inv(A'_pp)
 *         for each j > p with (i, j) in P and (p, j) in P:
 *             A'_ij <- A'_ij - A'_ip * A'_pj
 * When row i is finished its diagonal block is U_ii and its inverse is
 * formed (used by later rows as inv(A'_pp) and by Eq 5 as D^{-1}).
 * On return LU holds L (strictly lower blocks, unit diagonal implied) and
 * U (upper blocks with the diagonal) on P, and Dinv[i] = inv(U_ii).
 * Returns 0, ORC_ERR_PATTERN if A has a block outside P, or ORC_SINGULAR
 * with *bad_row set.
 */
int orc_factor(int n, int b, const int *Ap, const int *Aj, const double *Ax,
               const int *Pp, const int *Pj, double *LU, double *Dinv, int *bad_row)
{
    const int bb = b * b;
    if (b < 1 || b > ORC_MAX_B) return ORC_ERR_PATTERN;
    /* Backfill: copy A's blocks into their positions in P, zeros elsewhere. */
    memset(LU, 0, (size_t)Pp[n] * bb * sizeof(double));
    for (int i = 0; i < n; i++)
        for (int e = Ap[i]; e < Ap[i + 1]; e++) {
            int pos = find_col(Pj, Pp[i], Pp[i + 1], Aj[e]);
            if (pos < 0) return ORC_ERR_PATTERN;
            memcpy(LU + (size_t)pos * bb, Ax + (size_t)e * bb, bb * sizeof(double));
        }
    double T[ORC_MAX_B * ORC_MAX_B];
    for (int i = 0; i < n; i++) {
        for (int e = Pp[i]; e < Pp[i + 1]; e++) {
            int p = Pj[e];
            if (p >= i) break;
            double *Aip = LU + (size_t)e * bb;
            blk_mul(b, Aip, Dinv + (size_t)p * bb, T);
            memcpy(Aip, T, bb * sizeof(double));
            for (int f = e + 1; f < Pp[i + 1]; f++) {
                int j = Pj[f];
                int pj = find_col(Pj, Pp[p], Pp[p + 1], j);
                if (pj < 0) continue;
                blk_mul_sub(b, Aip, LU + (size_t)pj * bb, LU + (size_t)f * bb);
            }
        }
        int d = find_col(Pj, Pp[i], Pp[i + 1], i);
        if (d < 0) return ORC_ERR_MISSING_DIAG;
        if (blk_inv(b, LU + (size_t)d * bb, Dinv + (size_t)i * bb)) {
            if (bad_row) *bad_row = i;
            return ORC_SINGULAR;
        }
    }
    return ORC_OK;
}

/*
 * Diagonal factorisation U = D (D^{-1} U) = D U' (Eq 5).
 * F receives, on the pattern P: L at the strictly lower positions, U' =
 * D_i^{-1} U_ij at the strictly upper positions and the identity at the
 * diagonal positions (both L and U' have identity diagonal blocks).
 */
void orc_split(int n, int b, const int *Pp, const int *Pj, const double *LU,
               const double *Dinv, double *F)
{
    const int bb = b * b;
    for (int i = 0; i < n; i++)
        for (int e = Pp[i]; e < Pp[i + 1]; e++) {
            int j = Pj[e];
            double *Fe = F + (size_t)e * bb;
            if (j < i) {
                memcpy(Fe, LU + (size_t)e * bb, bb * sizeof(double));
            } else if (j == i) {
                for (int t = 0; t < bb; t++) Fe[t] = 0.0;
                for (int r = 0; r < b; r++) Fe[r * b + r] = 1.0;
            } else {
                blk_mul(b, Dinv + (size_t)i * bb, LU + (size_t)e * bb, Fe);
            }
        }
}

/* The factors as the preconditioner reads them: FP64, or FP32 copies. */
typedef struct {
    int n, b;
    const int *Pp, *Pj;
    const double *F, *Dinv;   /* used when F32 == NULL */
    const float *F32, *Dinv32;
} orc_precond;

static double fval(const orc_precond *M, size_t idx)
{
    return M->F32 ? (double)M->F32[idx] : M->F[idx];
}

static double dval(const orc_precond *M, size_t idx)
{
    return M->Dinv32 ? (double)M->Dinv32[idx] : M->Dinv[idx];
}

/*
 * Preconditioner application M^{-1} r with M = L D U' (Eq 6, Algorithm 7):
 *     L y = r      forward, rows ascending   y_i = r_i - sum_{j<i} L_ij y_j
 *     z = D^{-1} y blockwise                  z_i = D_i^{-1} y_i
 *     U' x = z     backward, rows descending x_i = z_i - sum_{j>i} U'_ij x_j
 * Row order is the sequential order; a level schedule (Eq 4) computes the
 * same rows from the same finished values.
 */
static void precond_apply(const orc_precond *M, const double *r, double *x)
{
    const int n = M->n, b = M->b, bb = b * b;
    double *y = (double *)malloc((size_t)n * b * sizeof(double));
    double acc[ORC_MAX_B];
    for (int i = 0; i < n; i++) {
        for (int rr = 0; rr < b; rr++) acc[rr] = r[(size_t)i * b + rr];
        for (int e = M->Pp[i]; e < M->Pp[i + 1]; e++) {
            int j = M->Pj[e];
            if (j >= i) break;
            for (int c = 0; c < b; c++)
                for (int rr = 0; rr < b; rr++)
                    acc[rr] -= fval(M, (size_t)e * bb + c * b + rr) * y[(size_t)j * b + c];
        }
        for (int rr = 0; rr < b; rr++) y[(size_t)i * b + rr] = acc[rr];
    }
    for (int i = n - 1; i >= 0; i--) {
        for (int rr = 0; rr < b; rr++) {
            double s = 0.0;
            for (int c = 0; c < b; c++)
                s += dval(M, (size_t)i * bb + c * b + rr) * y[(size_t)i * b + c];
            acc[rr] = s;
        }
        for (int e = M->Pp[i]; e < M->Pp[i + 1]; e++) {
            int j = M->Pj[e];
            if (j <= i) continue;
            for (int c = 0; c < b; c++)
                for (int rr = 0; rr < b; rr++)
                    acc[rr] -= fval(M, (size_t)e * bb + c * b + rr) * x[(size_t)j * b + c];
        }
        for (int rr = 0; rr < b; rr++) x[(size_t)i * b + rr] = acc[rr];
    }
    free(y);
}

/*
 * Transposed application M^{-T} r = L^{-T} D^{-T} U'^{-T} r:
 *     U'^T w = r   forward  (U'^T is unit lower triangular)
 *     v_i = (D_i^{-1})^T w_i
 *     L^T s = v    backward (L^T is unit upper triangular)
 * Written column-oriented: once an unknown is final its contribution is
 * pushed into the unknowns that depend on it.
 */
static void precond_apply_t(const orc_precond *M, const double *r, double *s)
{
    const int n = M->n, b = M->b, bb = b * b;
    double *w = (double *)malloc((size_t)n * b * sizeof(double));
    memcpy(w, r, (size_t)n * b * sizeof(double));
    for (int i = 0; i < n; i++) {           /* w_i is final here */
        for (int e = M->Pp[i]; e < M->Pp[i + 1]; e++) {
            int j = M->Pj[e];
            if (j <= i) continue;
            /* w_j -= (U'_ij)^T w_i */
            for (int c = 0; c < b; c++) {
                double t = 0.0;
                for (int rr = 0; rr < b; rr++)
                    t += fval(M, (size_t)e * bb + c * b + rr) * w[(size_t)i * b + rr];
                w[(size_t)j * b + c] -= t;
            }
        }
    }
    for (int i = 0; i < n; i++)
        for (int c = 0; c < b; c++) {
            double t = 0.0;
            for (int rr = 0; rr < b; rr++)
                t += dval(M, (size_t)i * bb + c * b + rr) * w[(size_t)i * b + rr];
            s[(size_t)i * b + c] = t;
        }
    for (int i = n - 1; i >= 0; i--) {      /* s_i is final here */
        for (int e = M->Pp[i]; e < M->Pp[i + 1]; e++) {
            int p = M->Pj[e];
            if (p >= i) break;
            /* s_p -= (L_ip)^T s_i */
            for (int c = 0; c < b; c++) {
                double t = 0.0;
                for (int rr = 0; rr < b; rr++)
                    t += fval(M, (size_t)e * bb + c * b + rr) * s[(size_t)i * b + rr];
                s[(size_t)p * b + c] -= t;
            }
        }
    }
    free(w);
}

void orc_apply(int n, int b, const int *Pp, const int *Pj, const double *F,
               const double *Dinv, const double *r, double *z)
{
    orc_precond M = {n, b, Pp, Pj, F, Dinv, NULL, NULL};
    precond_apply(&M, r, z);
}

void orc_apply_t(int n, int b, const int *Pp, const int *Pj, const double *F,
                 const double *Dinv, const double *r, double *z)
{
    orc_precond M = {n, b, Pp, Pj, F, Dinv, NULL, NULL};
    precond_apply_t(&M, r, z);
}

/* Apply with FP32-stored factors: every factor element is widened to FP64
 * before it is multiplied; vectors and sums stay FP64. */
void orc_apply_f32(int n, int b, const int *Pp, const int *Pj, const float *F,
                   const float *Dinv, const double *r, double *z)
{
    orc_precond M = {n, b, Pp, Pj, NULL, NULL, F, Dinv};
    precond_apply(&M, r, z);
}

/* Round FP64 factors to FP32, round-to-nearest-even (C's conversion). */
void orc_round_f32(long long count, const double *src, float *dst)
{
    for (long long t = 0; t < count; t++) dst[t] = (float)src[t];
}

/* y = A x on the block pattern of A. */
void orc_spmv(int n, int b, const int *Ap, const int *Aj, const double *Ax,
              const double *x, double *y)
{
    const int bb = b * b;
    for (int i = 0; i < n; i++)
        for (int rr = 0; rr < b; rr++) {
            double s = 0.0;
            for (int e = Ap[i]; e < Ap[i + 1]; e++) {
                int j = Aj[e];
                for (int c = 0; c < b; c++)
                    s += Ax[(size_t)e * bb + c * b + rr] * x[(size_t)j * b + c];
            }
            y[(size_t)i * b + rr] = s;
        }
}

/* y = A^T x. */
void orc_spmv_t(int n, int b, const int *Ap, const int *Aj, const double *Ax,
                const double *x, double *y)
{
    const int bb = b * b;
    memset(y, 0, (size_t)n * b * sizeof(double));
    for (int i = 0; i < n; i++)
        for (int e = Ap[i]; e < Ap[i + 1]; e++) {
            int j = Aj[e];
            for (int c = 0; c < b; c++) {
                double s = 0.0;
                for (int rr = 0; rr < b; rr++)
                    s += Ax[(size_t)e * bb + c * b + rr] * x[(size_t)i * b + rr];
                y[(size_t)j * b + c] += s;
            }
        }
}

/* ------------------------------------------------------------------------ */
/* Krylov loops                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n, b;
    const int *Ap, *Aj;
    const double *Ax;
    orc_precond M;
    int transpose;
} orc_system;

static void op_A(const orc_system *S, const double *x, double *y)
{
    if (S->transpose) orc_spmv_t(S->n, S->b, S->Ap, S->Aj, S->Ax, x, y);
    else orc_spmv(S->n, S->b, S->Ap, S->Aj, S->Ax, x, y);
}

static void op_M(const orc_system *S, const double *r, double *z)
{
    if (S->transpose) precond_apply_t(&S->M, r, z);
    else precond_apply(&S->M, r, z);
}

static double dot(long long N, const double *a, const double *c)
{
    double s = 0.0;
    for (long long t = 0; t < N; t++) s += a[t] * c[t];
    return s;
}

static double true_residual(const orc_system *S, const double *bvec, const double *x,
                            double *work)
{
    long long N = (long long)S->n * S->b;
    op_A(S, x, work);
    for (long long t = 0; t < N; t++) work[t] = bvec[t] - work[t];
    return sqrt(dot(N, work, work));
}

/*
 * Right-preconditioned BiCGSTAB (van der Vorst), x0 = 0, r^ = r0.  One
 * iteration is one full step (two preconditioner applications).  The exit
 * test is the true residual ||b - A x||_2 <= rtol ||b||_2: whenever the
 * recurrence residual passes the test the true residual is recomputed; if it
 * fails, the iteration restarts from r = b - A x with r^ = r.
 * Returns 0, ORC_NOT_CONVERGED or ORC_BREAKDOWN (rho = 0, <r^,v> = 0, or
 * omega = 0).
 */
/* Number of true-residual restarts taken by the last BiCGSTAB solve (a
 * counter for the tests; it does not enter the arithmetic). */
static int last_restarts = 0;
int orc_last_restarts(void) { return last_restarts; }

static int bicgstab(const orc_system *S, const double *bvec, double *x, double rtol,
                    int maxit, int *iters, double *relres)
{
    long long N = (long long)S->n * S->b;
    size_t sz = (size_t)N * sizeof(double);
    double *r = malloc(sz), *rh = malloc(sz), *p = malloc(sz), *v = malloc(sz);
    double *ph = malloc(sz), *s = malloc(sz), *sh = malloc(sz), *t = malloc(sz);
    double *w = malloc(sz);
    int status = ORC_NOT_CONVERGED, it = 0;
    double bnorm = sqrt(dot(N, bvec, bvec));
    memset(x, 0, sz);
    memcpy(r, bvec, sz);
    memcpy(rh, r, sz);
    double rho_old = 1.0, alpha = 1.0, omega = 1.0, rres = bnorm;
    int fresh = 1;
    last_restarts = 0;
    if (bnorm == 0.0) { status = ORC_OK; rres = 0.0; goto done; }
    for (it = 1; it <= maxit; it++) {
        double rho = dot(N, rh, r);
        if (rho == 0.0) { status = ORC_BREAKDOWN; break; }
        if (fresh) {
            memcpy(p, r, sz);
            fresh = 0;
        } else {
            double beta = (rho / rho_old) * (alpha / omega);
            for (long long q = 0; q < N; q++) p[q] = r[q] + beta * (p[q] - omega * v[q]);
        }
        op_M(S, p, ph);
        op_A(S, ph, v);
        double rv = dot(N, rh, v);
        if (rv == 0.0) { status = ORC_BREAKDOWN; break; }
        alpha = rho / rv;
        for (long long q = 0; q < N; q++) s[q] = r[q] - alpha * v[q];
        double snorm = sqrt(dot(N, s, s));
        if (snorm <= rtol * bnorm) {
            for (long long q = 0; q < N; q++) x[q] += alpha * ph[q];
            rres = true_residual(S, bvec, x, w);
            if (rres <= rtol * bnorm) { status = ORC_OK; break; }
            memcpy(r, w, sz);
            memcpy(rh, r, sz);
            fresh = 1;
            last_restarts++;
            rho_old = rho;
            continue;
        }
        op_M(S, s, sh);
        op_A(S, sh, t);
        double tt = dot(N, t, t);
        if (tt == 0.0) { status = ORC_BREAKDOWN; break; }
        omega = dot(N, t, s) / tt;
        for (long long q = 0; q < N; q++) {
            x[q] += alpha * ph[q] + omega * sh[q];
            r[q] = s[q] - omega * t[q];
        }
        rho_old = rho;
        if (omega == 0.0) { status = ORC_BREAKDOWN; break; }
        double rnorm = sqrt(dot(N, r, r));
        if (rnorm <= rtol * bnorm) {
            rres = true_residual(S, bvec, x, w);
            if (rres <= rtol * bnorm) { status = ORC_OK; break; }
            memcpy(r, w, sz);
            memcpy(rh, r, sz);
            fresh = 1;
            last_restarts++;
        }
    }
    if (it > maxit) it = maxit;
    if (status != ORC_OK) rres = true_residual(S, bvec, x, w);
done:
    *iters = it;
    *relres = bnorm > 0.0 ? rres / bnorm : 0.0;
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t); free(w);
    return status;
}

/*
 * Restarted right-preconditioned GMRES(m): Arnoldi with modified
 * Gram-Schmidt, Givens rotations on the Hessenberg matrix, x += M^{-1} V y at
 * the end of each cycle, then the true-residual exit test.  maxit bounds the
 * total number of Arnoldi steps, which is what *iters reports.
 */
static int gmres(const orc_system *S, const double *bvec, double *x, double rtol,
                 int restart, int maxit, int *iters, double *relres)
{
    long long N = (long long)S->n * S->b;
    size_t sz = (size_t)N * sizeof(double);
    int m = restart;
    double *V = malloc(sz * (size_t)(m + 1));
    double *H = calloc((size_t)(m + 1) * m, sizeof(double)); /* H[i*m + j] */
    double *cs = calloc((size_t)m, sizeof(double)), *sn = calloc((size_t)m, sizeof(double));
    double *g = calloc((size_t)m + 1, sizeof(double)), *y = calloc((size_t)m, sizeof(double));
    double *w = malloc(sz), *z = malloc(sz), *u = malloc(sz);
    int status = ORC_NOT_CONVERGED, total = 0;
    double bnorm = sqrt(dot(N, bvec, bvec)), rres = bnorm;
    memset(x, 0, sz);
    if (bnorm == 0.0) { status = ORC_OK; rres = 0.0; goto done; }
    while (1) {
        rres = true_residual(S, bvec, x, w);
        if (rres <= rtol * bnorm) { status = ORC_OK; break; }
        if (total >= maxit) break;
        double beta = rres;
        for (long long q = 0; q < N; q++) V[q] = w[q] / beta;
        for (int i = 0; i <= m; i++) g[i] = 0.0;
        g[0] = beta;
        int jend = 0;
        for (int j = 0; j < m; j++) {
            op_M(S, V + (size_t)j * N, z);
            op_A(S, z, w);
            for (int i = 0; i <= j; i++) {
                double h = dot(N, w, V + (size_t)i * N);
                H[i * m + j] = h;
                for (long long q = 0; q < N; q++) w[q] -= h * V[(size_t)i * N + q];
            }
            double hn = sqrt(dot(N, w, w));
            H[(j + 1) * m + j] = hn;
            if (hn != 0.0)
                for (long long q = 0; q < N; q++) V[(size_t)(j + 1) * N + q] = w[q] / hn;
            for (int i = 0; i < j; i++) {
                double a = H[i * m + j], c2 = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c2;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c2;
            }
            double a = H[j * m + j], c2 = H[(j + 1) * m + j];
            double rr = hypot(a, c2);
            if (rr == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = a / rr; sn[j] = c2 / rr; }
            H[j * m + j] = cs[j] * a + sn[j] * c2;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            total++;
            jend = j + 1;
            if (fabs(g[j + 1]) <= rtol * bnorm || total >= maxit || hn == 0.0) break;
        }
        for (int i = jend - 1; i >= 0; i--) {
            double s = g[i];
            for (int c = i + 1; c < jend; c++) s -= H[i * m + c] * y[c];
            if (H[i * m + i] == 0.0) { status = ORC_BREAKDOWN; goto done_res; }
            y[i] = s / H[i * m + i];
        }
        memset(u, 0, sz);
        for (int i = 0; i < jend; i++)
            for (long long q = 0; q < N; q++) u[q] += y[i] * V[(size_t)i * N + q];
        op_M(S, u, z);
        for (long long q = 0; q < N; q++) x[q] += z[q];
    }
    goto done;
done_res:
    rres = true_residual(S, bvec, x, w);
done:
    *iters = total;
    *relres = bnorm > 0.0 ? rres / bnorm : 0.0;
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(w); free(z); free(u);
    return status;
}

/*
 * Right-preconditioned ORTHOMIN(k) (Vinsome's method, named in the paper's
 * introduction as the reservoir simulators' Krylov solver), x0 = 0.  Each
 * iteration takes the preconditioned residual z = M^{-1} r as a new search
 * direction p with Ap = A z, makes Ap orthogonal to the A-images q_i of the
 * last k kept directions, beta_i = -(A z, q_i) / (q_i, q_i) (every beta_i
 * from the unmodified A z; the kept q_i are mutually orthogonal),
 * p = z + sum_i beta_i p_i and q = A z + sum_i beta_i q_i (kept directions
 * from the oldest to the newest), then minimises the residual along p:
 * alpha = (r, q) / (q, q), x += alpha p, r -= alpha q.  Exit on the true
 * residual as in BiCGSTAB; when the recurrence residual passes but the true
 * one does not, r = b - A x and the kept directions are dropped.  k = 0
 * is the minimal-residual iteration.  Returns 0, ORC_NOT_CONVERGED or
 * ORC_BREAKDOWN ((q, q) = 0).
 */
static int orthomin(const orc_system *S, const double *bvec, double *x, double rtol, int k,
                    int maxit, int *iters, double *relres)
{
    long long N = (long long)S->n * S->b;
    size_t sz = (size_t)N * sizeof(double);
    int K1 = k + 1;
    double *P = malloc(sz * (size_t)K1), *Q = malloc(sz * (size_t)K1);
    double *qq = calloc((size_t)K1, sizeof(double)), *beta = calloc((size_t)K1, sizeof(double));
    double *r = malloc(sz), *w = malloc(sz);
    int status = ORC_NOT_CONVERGED, it = 0, count = 0;
    double bnorm = sqrt(dot(N, bvec, bvec)), rres = bnorm;
    memset(x, 0, sz);
    memcpy(r, bvec, sz);
    last_restarts = 0;
    if (bnorm == 0.0) { status = ORC_OK; rres = 0.0; goto done; }
    for (it = 1; it <= maxit; it++) {
        int s = (it - 1) % K1;
        double *p = P + (size_t)s * N, *q = Q + (size_t)s * N;
        op_M(S, r, p);
        op_A(S, p, q);
        /* kept directions: the count slots before s, oldest first */
        for (int i = 0; i < count; i++) {
            int si = ((s - count + i) % K1 + K1) % K1;
            beta[i] = -dot(N, q, Q + (size_t)si * N) / qq[si];
        }
        for (int i = 0; i < count; i++) {
            int si = ((s - count + i) % K1 + K1) % K1;
            const double *pi = P + (size_t)si * N, *qi = Q + (size_t)si * N;
            for (long long t = 0; t < N; t++) {
                p[t] += beta[i] * pi[t];
                q[t] += beta[i] * qi[t];
            }
        }
        qq[s] = dot(N, q, q);
        if (qq[s] == 0.0) { status = ORC_BREAKDOWN; break; }
        double alpha = dot(N, r, q) / qq[s];
        for (long long t = 0; t < N; t++) {
            x[t] += alpha * p[t];
            r[t] -= alpha * q[t];
        }
        count = count < k ? count + 1 : k;
        double rnorm = sqrt(dot(N, r, r));
        if (rnorm <= rtol * bnorm) {
            rres = true_residual(S, bvec, x, w);
            if (rres <= rtol * bnorm) { status = ORC_OK; break; }
            memcpy(r, w, sz);
            count = 0;
            last_restarts++;
        }
    }
    if (it > maxit) it = maxit;
    if (status != ORC_OK) rres = true_residual(S, bvec, x, w);
done:
    *iters = it;
    *relres = bnorm > 0.0 ? rres / bnorm : 0.0;
    free(P); free(Q); free(qq); free(beta); free(r); free(w);
    return status;
}

/* method 0 = BiCGSTAB, 1 = GMRES(restart), 2 = ORTHOMIN(k = restart).
 * F32/Dinv32 non-NULL selects the FP32-stored factors.  transpose = 1 solves
 * A^T x = b with M^{-T}. */
int orc_solve(int n, int b, const int *Ap, const int *Aj, const double *Ax,
              const int *Pp, const int *Pj, const double *F, const double *Dinv,
              const float *F32, const float *Dinv32, const double *bvec, double *x,
              int method, int restart, double rtol, int maxit, int transpose,
              int *iters, double *relres)
{
    orc_system S;
    S.n = n; S.b = b; S.Ap = Ap; S.Aj = Aj; S.Ax = Ax; S.transpose = transpose;
    S.M.n = n; S.M.b = b; S.M.Pp = Pp; S.M.Pj = Pj;
    S.M.F = F; S.M.Dinv = Dinv; S.M.F32 = F32; S.M.Dinv32 = Dinv32;
    if (method == 1) return gmres(&S, bvec, x, rtol, restart, maxit, iters, relres);
    if (method == 2) return orthomin(&S, bvec, x, rtol, restart, maxit, iters, relres);
    return bicgstab(&S, bvec, x, rtol, maxit, iters, relres);
}

/* Gradient of a loss with respect to the stored blocks of A for x = A^{-1} b:
 * dL/dA_ij = -lambda_i x_j^T on A's own block pattern, lambda = A^{-T} g. */
void orc_grad_A(int n, int b, const int *Ap, const int *Aj, const double *lambda,
                const double *x, double *dAx)
{
    const int bb = b * b;
    for (int i = 0; i < n; i++)
        for (int e = Ap[i]; e < Ap[i + 1]; e++) {
            int j = Aj[e];
            for (int c = 0; c < b; c++)
                for (int rr = 0; rr < b; rr++)
                    dAx[(size_t)e * bb + c * b + rr] = -lambda[(size_t)i * b + rr] * x[(size_t)j * b + c];
        }
}
