/*
 * oracle.c -- plain, slow, obviously correct CPU oracle for M-HDC SpMV.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * Source: Fukaya, Ishida, Miura, Iwashita, Nakashima, "Accelerating the SpMV
 * kernel on standard CPUs by exploiting the partially diagonal structures",
 * arXiv:2105.04937.
 *
 * Conventions (all taken from the paper):
 *   - zero-based indices, CSR with row_ptr[n] = nnz            (Sec. 3.1-3.2)
 *   - FP64 values, INT32 indices                                (Sec. 6.1.2)
 *   - a diagonal offset is used as x[i + off], so off = j - i   (Figs. 4, 5)
 *
 * Readings where the paper is silent or inconsistent (each one is listed in
 * the design notes of the repository):
 *   R1 offset sign: off = j - i (the text defines i - j, but every figure and
 *      kernel indexes x[i + off] and Fig. 4's offsets only fit j - i).
 *   R2 selection compares (double)count / (double)rows >= theta with a
 *      correctly rounded IEEE division ("≥" as in the formulas of Secs. 3.4
 *      and 4.3; the prose says "larger than").
 *   R3 denominator: HDC divides by n (Sec. 3.4); M-HDC divides by the number
 *      of rows of the block, which is bl for every full block (Sec. 4.3); the
 *      last block may be shorter when bl does not divide n.
 *   R4 only stored entries whose value compares != 0.0 count as nonzeros and
 *      may enter the DIA part; stored zeros stay in the CSR remainder.  DIA
 *      padding is +0.0.  A candidate diagonal needs at least one nonzero.
 *   R5 diagonals of one block are kept in ascending offset order (Figs. 4,
 *      7, 15).
 *   R6 M-HDC values are segment-local: the value of row i on the k-th partial
 *      diagonal of block ib sits at dia_val[k*bl + (i - ib*bl)] (Fig. 15
 *      stores bl values per partial diagonal).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.  With
 * -ffp-contract=off every "s += a * b" below is one rounded multiply followed
 * by one rounded add, in the order written.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ENOMEM (-1)
#define ORC_EARG (-2)

/* ------------------------------------------------------------------------ */
/* CSR SpMV (Sec. 3.2, Fig. 3): y_i = sum over k in [row_ptr[i], row_ptr[i+1])
 * of val[k] * x[col_ind[k]], accumulated from s = 0 in ascending k and then
 * stored.  Rows are independent, so the OpenMP split over rows does not change
 * any result bit.  nthreads <= 0 leaves the thread count to OpenMP. */
void orc_csr_spmv(int32_t n, const int32_t *row_ptr, const int32_t *col_ind,
                  const double *val, const double *x, double *y,
                  int32_t nthreads)
{
    if (nthreads <= 0) {
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; i++) {
            double s = 0.0;
            for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; k++)
                s += val[k] * x[col_ind[k]];
            y[i] = s;
        }
    } else {
#pragma omp parallel for schedule(static) num_threads(nthreads)
        for (int32_t i = 0; i < n; i++) {
            double s = 0.0;
            for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; k++)
                s += val[k] * x[col_ind[k]];
            y[i] = s;
        }
    }
}

/* The same definition applied to nrhs right-hand sides stored column by
 * column: column r of X starts at X + r*ldx, column r of Y at Y + r*ldy. */
void orc_csr_spmm(int32_t n, const int32_t *row_ptr, const int32_t *col_ind,
                  const double *val, int32_t nrhs, const double *X, int64_t ldx,
                  double *Y, int64_t ldy, int32_t nthreads)
{
    for (int32_t r = 0; r < nrhs; r++)
        orc_csr_spmv(n, row_ptr, col_ind, val, X + (int64_t)r * ldx,
                     Y + (int64_t)r * ldy, nthreads);
}

/* (|A||x|)_i = sum_k |val[k]| * |x[col_ind[k]]|: the scale of the error
 * bound used to compare two summation orders of the same row. */
void orc_csr_absmv(int32_t n, const int32_t *row_ptr, const int32_t *col_ind,
                   const double *val, const double *x, double *y)
{
    for (int32_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
            double a = val[k] < 0 ? -val[k] : val[k];
            double b = x[col_ind[k]] < 0 ? -x[col_ind[k]] : x[col_ind[k]];
            s += a * b;
        }
        y[i] = s;
    }
}

/* Dense matrix-vector product y = A x with A row-major n x n, summed in
 * ascending column order; the brute-force definition of SpMV (Sec. 3.1). */
void orc_dense_matvec(int32_t n, const double *A, const double *x, double *y)
{
    for (int32_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int32_t j = 0; j < n; j++)
            s += A[(int64_t)i * n + j] * x[j];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
static int cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

/* Selection rule of Sec. 4.3 (and of Sec. 3.4 with the whole matrix as one
 * block): keep a diagonal with cnt nonzeros out of `rows` rows iff
 * cnt / rows >= theta, with cnt >= 1 (a diagonal line is nonzero only if it
 * holds a nonzero, Sec. 3.3). */
static int selected(int64_t cnt, int64_t rows, double theta)
{
    return cnt >= 1 && ((double)cnt / (double)rows) >= theta;
}

/*
 * M-HDC reference converter (Sec. 4.3, Figs. 14-15).
 *
 * Rows are cut into n_blk = ceil(n / bl) blocks; block ib holds rows
 * [ib*bl, min(n, (ib+1)*bl)).  For every block:
 *   1. collect the offsets d = j - i of its nonzero entries,
 *   2. sort them and count each distinct d: that count is N~(d, ib),
 *   3. keep d iff N~(d, ib) / rows_ib >= theta (ascending order),
 *   4. put every nonzero on a kept diagonal into its segment slot and every
 *      other stored entry into the CSR remainder, row by row in column order.
 *
 * Output arrays (any may be NULL to only count):
 *   dia_ptr[n_blk+1], dia_off[K], dia_val[K*bl] (segment-local, +0.0 pad),
 *   rem_ptr[n+1], rem_col[R], rem_val[R].
 * *out_K and *out_R receive the numbers of kept partial diagonals and of
 * remainder entries.  Returns ORC_OK, ORC_EARG or ORC_ENOMEM.
 */
int orc_mhdc_convert(int32_t n, const int32_t *row_ptr, const int32_t *col_ind,
                     const double *val, int32_t bl, double theta,
                     int32_t *dia_ptr, int32_t *dia_off, double *dia_val,
                     int32_t *rem_ptr, int32_t *rem_col, double *rem_val,
                     int64_t *out_K, int64_t *out_R)
{
    if (n < 0 || bl < 1)
        return ORC_EARG;
    int64_t n_blk = n == 0 ? 0 : ((int64_t)n + bl - 1) / bl;

    int64_t max_m = 0;
    for (int64_t ib = 0; ib < n_blk; ib++) {
        int64_t r0 = ib * bl, r1 = r0 + bl < n ? r0 + bl : n;
        int64_t m = (int64_t)row_ptr[r1] - row_ptr[r0];
        if (m > max_m)
            max_m = m;
    }
    int32_t *offs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(max_m + 1));
    int32_t *sel = (int32_t *)malloc(sizeof(int32_t) * (size_t)(max_m + 1));
    if (!offs || !sel) {
        free(offs);
        free(sel);
        return ORC_ENOMEM;
    }

    int64_t K = 0, R = 0;
    if (rem_ptr && n >= 0)
        rem_ptr[0] = 0;
    for (int64_t ib = 0; ib < n_blk; ib++) {
        int64_t r0 = ib * bl, r1 = r0 + bl < n ? r0 + bl : n;
        int64_t rows = r1 - r0;

        /* steps 1-2: offsets of the nonzeros, sorted */
        int64_t m = 0;
        for (int64_t i = r0; i < r1; i++)
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++)
                if (val[k] != 0.0)
                    offs[m++] = col_ind[k] - (int32_t)i;
        qsort(offs, (size_t)m, sizeof(int32_t), cmp_i32);

        /* step 3: runs of equal offsets are the counts N~(d, ib) */
        int64_t nsel = 0;
        for (int64_t a = 0; a < m;) {
            int64_t b = a;
            while (b < m && offs[b] == offs[a])
                b++;
            if (selected(b - a, rows, theta))
                sel[nsel++] = offs[a];
            a = b;
        }
        if (dia_ptr)
            dia_ptr[ib] = (int32_t)K;
        if (dia_off)
            for (int64_t t = 0; t < nsel; t++)
                dia_off[K + t] = sel[t];
        if (dia_val)
            for (int64_t s = 0; s < nsel * (int64_t)bl; s++)
                dia_val[K * (int64_t)bl + s] = 0.0;

        /* step 4: scatter */
        for (int64_t i = r0; i < r1; i++) {
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
                int32_t d = col_ind[k] - (int32_t)i;
                int32_t *hit = NULL;
                if (val[k] != 0.0 && nsel > 0)
                    hit = (int32_t *)bsearch(&d, sel, (size_t)nsel,
                                             sizeof(int32_t), cmp_i32);
                if (hit) {
                    int64_t t = hit - sel;
                    if (dia_val)
                        dia_val[(K + t) * (int64_t)bl + (i - r0)] = val[k];
                } else {
                    if (rem_col)
                        rem_col[R] = col_ind[k];
                    if (rem_val)
                        rem_val[R] = val[k];
                    R++;
                }
            }
            if (rem_ptr)
                rem_ptr[i + 1] = (int32_t)R;
        }
        K += nsel;
    }
    if (dia_ptr)
        dia_ptr[n_blk] = (int32_t)K;
    free(offs);
    free(sel);
    *out_K = K;
    *out_R = R;
    return ORC_OK;
}

/*
 * HDC reference converter (Sec. 3.4, Figs. 6-7): one global DIA part plus a
 * CSR part.  N(d) counts the nonzeros of diagonal d over the whole matrix and
 * d is kept iff N(d) / n >= theta.  Kept values are stored per diagonal over
 * all n rows: dia_val[k*n + i] = a(i, i + off_k), +0.0 where the row has no
 * entry (including the out-of-range corners, as in Fig. 7).
 * Outputs: dia_off[K], dia_val[K*n], rem_ptr[n+1], rem_col[R], rem_val[R];
 * any may be NULL to only count.
 */
int orc_hdc_convert(int32_t n, const int32_t *row_ptr, const int32_t *col_ind,
                    const double *val, double theta, int32_t *dia_off,
                    double *dia_val, int32_t *rem_ptr, int32_t *rem_col,
                    double *rem_val, int64_t *out_K, int64_t *out_R)
{
    if (n < 0)
        return ORC_EARG;
    int64_t span = n == 0 ? 1 : 2 * (int64_t)n - 1; /* d in [-(n-1), n-1] */
    int64_t *cnt = (int64_t *)calloc((size_t)span, sizeof(int64_t));
    int32_t *kidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)span);
    if (!cnt || !kidx) {
        free(cnt);
        free(kidx);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++)
            if (val[k] != 0.0)
                cnt[(int64_t)col_ind[k] - i + (n - 1)]++;

    int64_t K = 0;
    for (int64_t q = 0; q < span; q++) {
        if (n > 0 && selected(cnt[q], n, theta)) {
            if (dia_off)
                dia_off[K] = (int32_t)(q - (n - 1));
            kidx[q] = (int32_t)K++;
        } else {
            kidx[q] = -1;
        }
    }
    if (dia_val)
        for (int64_t s = 0; s < K * (int64_t)n; s++)
            dia_val[s] = 0.0;

    int64_t R = 0;
    if (rem_ptr)
        rem_ptr[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
            int64_t q = (int64_t)col_ind[k] - i + (n - 1);
            if (val[k] != 0.0 && kidx[q] >= 0) {
                if (dia_val)
                    dia_val[(int64_t)kidx[q] * n + i] = val[k];
            } else {
                if (rem_col)
                    rem_col[R] = col_ind[k];
                if (rem_val)
                    rem_val[R] = val[k];
                R++;
            }
        }
        if (rem_ptr)
            rem_ptr[i + 1] = (int32_t)R;
    }
    free(cnt);
    free(kidx);
    *out_K = K;
    *out_R = R;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* M-HDC kernel semantics (Sec. 4.3, Fig. 16) on the arrays above, executed
 * sequentially: per block, the remainder rows first (y_i = s), then each
 * partial diagonal of the block in ascending k, clamped to the rows whose
 * column i + off lies in [0, n). */
void orc_mhdc_spmv(int32_t n, int32_t bl, const int32_t *dia_ptr,
                   const int32_t *dia_off, const double *dia_val,
                   const int32_t *rem_ptr, const int32_t *rem_col,
                   const double *rem_val, const double *x, double *y)
{
    int64_t n_blk = n == 0 ? 0 : ((int64_t)n + bl - 1) / bl;
    for (int64_t ib = 0; ib < n_blk; ib++) {
        int64_t r0 = ib * bl, r1 = r0 + bl < n ? r0 + bl : n;
        for (int64_t i = r0; i < r1; i++) {
            double s = 0.0;
            for (int64_t k = rem_ptr[i]; k < rem_ptr[i + 1]; k++)
                s += rem_val[k] * x[rem_col[k]];
            y[i] = s;
        }
        for (int64_t k = dia_ptr[ib]; k < dia_ptr[ib + 1]; k++) {
            int64_t off = dia_off[k];
            int64_t is = r0 > -off ? r0 : -off;
            int64_t ie = r1 < n - off ? r1 : n - off;
            for (int64_t i = is; i < ie; i++)
                y[i] += dia_val[k * (int64_t)bl + (i - r0)] * x[i + off];
        }
    }
}

/* HDC kernel semantics (Sec. 3.4, Fig. 8): the CSR part writes y, then every
 * global diagonal adds its products over rows [max(0,-off), min(n, n-off)). */
void orc_hdc_spmv(int32_t n, int32_t K, const int32_t *dia_off,
                  const double *dia_val, const int32_t *rem_ptr,
                  const int32_t *rem_col, const double *rem_val,
                  const double *x, double *y)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t k = rem_ptr[i]; k < rem_ptr[i + 1]; k++)
            s += rem_val[k] * x[rem_col[k]];
        y[i] = s;
    }
    for (int64_t k = 0; k < K; k++) {
        int64_t off = dia_off[k];
        int64_t is = 0 > -off ? 0 : -off;
        int64_t ie = n < n - off ? n : n - off;
        for (int64_t i = is; i < ie; i++)
            y[i] += dia_val[k * (int64_t)n + i] * x[i + off];
    }
}

/* ------------------------------------------------------------------------ */
/*
 * Decoder M-HDC -> CSR: row i of block ib is the merge, by column, of its
 * remainder entries (already in column order) and of the nonzero slots
 * (value != 0.0) of the block's partial diagonals whose column i + off lies
 * in [0, n).  Offsets ascend within a block, so those columns ascend too.
 * out_ptr[n+1]; out_col and out_val need room for every emitted entry.
 */
int orc_mhdc_to_csr(int32_t n, int32_t bl, const int32_t *dia_ptr,
                    const int32_t *dia_off, const double *dia_val,
                    const int32_t *rem_ptr, const int32_t *rem_col,
                    const double *rem_val, int32_t *out_ptr, int32_t *out_col,
                    double *out_val)
{
    int64_t e = 0;
    out_ptr[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t ib = i / bl, r0 = ib * bl;
        int64_t k = dia_ptr[ib], kend = dia_ptr[ib + 1];
        int64_t q = rem_ptr[i], qend = rem_ptr[i + 1];
        for (;;) {
            /* next nonzero in-range diagonal slot */
            while (k < kend) {
                int64_t j = i + dia_off[k];
                if (j >= 0 && j < n &&
                    dia_val[k * (int64_t)bl + (i - r0)] != 0.0)
                    break;
                k++;
            }
            int have_d = k < kend, have_r = q < qend;
            if (!have_d && !have_r)
                break;
            int take_d;
            if (have_d && have_r) {
                int64_t jd = i + dia_off[k];
                if (jd == rem_col[q])
                    return ORC_EARG; /* one position stored twice */
                take_d = jd < rem_col[q];
            } else {
                take_d = have_d;
            }
            if (take_d) {
                out_col[e] = (int32_t)(i + dia_off[k]);
                out_val[e] = dia_val[k * (int64_t)bl + (i - r0)];
                k++;
            } else {
                out_col[e] = rem_col[q];
                out_val[e] = rem_val[q];
                q++;
            }
            e++;
        }
        out_ptr[i + 1] = (int32_t)e;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Memory benchmark kernels of Sec. 6.2 (Figs. 19-20), sequential loops. */
void orc_stream_direct(int64_t N, const double *A, const double *B, double *C)
{
    for (int64_t i = 0; i < N; i++)
        C[i] += A[i] * B[i];
}

void orc_stream_indirect(int64_t N, const double *A, const double *B,
                         const int32_t *I, double *C)
{
    for (int64_t i = 0; i < N; i++)
        if (I[i] >= 0 && I[i] < N)  /* an index outside [0, N) leaves C[i] */
            C[i] += A[i] * B[I[i]];
}
