/*
 * mhdc.h -- C-ABI of libmhdc.so: FP64 sparse matrix-vector multiplication
 * y = A x in the M-HDC format on AMD Instinct MI355X (gfx950).
 *
 * Method: Fukaya, Ishida, Miura, Iwashita, Nakashima, "Accelerating the SpMV
 * kernel on standard CPUs by exploiting the partially diagonal structures",
 * arXiv:2105.04937.
 *
 * Formats (all zero-based, FP64 values, INT32 indices, Sec. 3.1 and 6.1.2):
 *   CSR    rowptr[n+1] (rowptr[0] = 0, rowptr[n] = nnz), colind[nnz],
 *          val[nnz]; columns strictly increasing within a row (Sec. 3.2).
 *   HDC    diagonals d = j - i with N(d)/n >= theta stored DIA-style over
 *          all n rows, the other entries in a CSR part (Sec. 3.4).
 *   M-HDC  rows cut into blocks of n_b rows; in block ib the partial
 *          diagonals with N~(d,ib)/rows_ib >= theta are stored as n_b-long
 *          value segments keyed by offset, the rest in a CSR remainder
 *          (Sec. 4.3).  rows_ib = min(n_b, n - ib*n_b).
 *
 * Conventions shared by every entry point:
 *   - Every array argument is a DEVICE pointer on the current HIP device
 *     unless stated otherwise.  The caller keeps ownership of its arrays;
 *     a handle owns copies of what it needs and frees them in *_destroy.
 *   - *_from_csr is synchronous (it returns when the handle is complete).
 *     *_spmv / *_spmm are asynchronous on the given stream (0 = the null
 *     stream) and overwrite y (they do not accumulate).  x and y must not
 *     overlap.  A handle is read-only after creation, so spmv calls on one
 *     handle may run concurrently on several streams; *_destroy requires
 *     that no work using the handle is still in flight.
 *   - Functions returning int give MHDC_OK (0) or a negative MHDC_ERR_*
 *     code; functions returning a handle give NULL on failure.  In both
 *     cases the code and a message are kept per host thread
 *     (mhdc_last_error, mhdc_last_error_message).
 *   - Entries whose stored value compares equal to 0.0 (+0.0 or -0.0) never
 *     count as nonzeros and always stay in the CSR part; DIA padding is
 *     +0.0.  Results are promised for finite x (a padded 0 * Inf is NaN).
 *   - The threshold test is (double)count / (double)rows >= theta in IEEE
 *     FP64 with a correctly rounded division; a candidate diagonal needs at
 *     least one nonzero (Sec. 3.3).  Offsets are d = j - i (the figures and
 *     kernels of the paper index x[i + offset]).
 */
#ifndef MHDC_H
#define MHDC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
enum {
    MHDC_OK = 0,
    MHDC_ERR_INVALID_ARG = -1,   /* bad size, NULL pointer, theta/n_b range */
    MHDC_ERR_BAD_CSR = -2,       /* rowptr not monotone, rowptr[0] != 0,
                                    column out of range, unsorted or
                                    duplicate columns */
    MHDC_ERR_OOM = -3,           /* device allocation failed or too large */
    MHDC_ERR_HIP = -4,           /* a HIP runtime call failed */
    MHDC_ERR_SIZE = -5,          /* a count does not fit the index types */
    MHDC_ERR_NOT_SUPPORTED = -6  /* option outside the compiled variants */
};

/* Code of the last failure on the calling host thread (MHDC_OK if none). */
int mhdc_last_error(void);
/* Human-readable message of that failure (static storage, thread-local). */
const char *mhdc_last_error_message(void);
/* Name of an error code. */
const char *mhdc_error_string(int code);

/* ------------------------------------------------------------ handles */
typedef struct mhdc_s *mhdc_handle;
typedef struct hdc_s *hdc_handle;
typedef struct csr_s *csr_handle;

/* Sizes and model figures of a handle.  bytes_alg is what one spmv must
 * move at the least with the format's layout (every stored array element
 * read once, x read once, y written once):
 *   M-HDC  4*(n_blk+1) + 4*K + 8*S + (R > 0 ? 4*(n+1) : 0) + 12*R + 16*n
 *   HDC    4*K + 8*S + (R > 0 ? 4*(n+1) : 0) + 12*R + 16*n  (S = K*n; the
 *          layout of Fig. 7 has no block pointer)
 *   CSR    4*(n+1) + 12*nnz + 16*n
 * (the library's remainder bit mask is not counted: the format does not
 * need it).  bytes_paper is the paper's
 * volume V = V_A + V_x + V_y with v_x = 1 (Eqs. 24/34 of Sec. 5.3):
 *   12*R + 4*n + 8*S + 8*n + 8*n.  alpha and beta are the filling rate and
 * CSR rate of Eqs. 23/33, rp_est the relative performance over CSR of
 * Eq. 28 (1 + Eq. 28) with v_x = 1. */
typedef struct {
    int32_t kind;        /* 0 = M-HDC, 1 = HDC, 2 = CSR */
    int32_t n;
    int64_t nnz;         /* stored entries of the input CSR */
    int32_t n_b;         /* rows per block (n for HDC, 0 for CSR) */
    double theta;
    int64_t n_blk;       /* number of row blocks */
    int64_t K;           /* kept (partial) diagonals */
    int64_t S;           /* DIA slots = K * n_b */
    int64_t R;           /* entries in the CSR part / remainder */
    double alpha, beta;
    double bytes_alg, bytes_paper, rp_est;
    int32_t rows_per_lane, wg_size, xcd_remap, csr_mode, rhs_group; /* launch shape */
    double row_repeat;   /* share of the CSR part's nonempty rows whose column
                            offsets (col - row) repeat the previous row's, in
                            length and order; 0 for an empty CSR part */
    double lone_per_row; /* CSR-part entries per row (over all n rows) with no
                            column within 16 of theirs in the CSR part of
                            either of the two previous rows (rows before the
                            first hold none); 0 for an empty CSR part */
} mhdc_info;

/* Launch shape of the SpMV kernel.  rows_per_lane in {1, 2, 4} (4 only for
 * k = 1): rows each lane owns (spaced one wavefront apart); wg_size in
 * {64, 256};
 * xcd_remap (0..64) places row tiles on the 8 XCDs: 0 = dispatch order
 * (tile w on XCD w mod 8), 1 = each XCD walks one contiguous eighth of the
 * tiles, C >= 2 = runs of C consecutive tiles per XCD, the XCDs taking the
 * runs in turn (tile t + 8*C*j shares tile t's L2); csr_mode selects how
 * the CSR part of a tile is processed: 1 = each staging lane multiplies its
 * entries by the gathered x and stages the rounded products in LDS, 2 =
 * values and columns are staged and each lane gathers x for its own rows,
 * 0 = 1 for one right-hand side and 2 for several; rhs_group in {0, 1, 2,
 * 4, 8, 16}:
 * right-hand sides processed per pass over a tile (0 = all, up to 16; a
 * further pass reads the tile's share of A again from the caches).  Every
 * variant gives the same bits.  A new handle starts with {1, 256, C, c, 0}
 * for n >= 2^20 rows, C in 8..16 chosen at conversion so that the x rows a
 * tile reads through its farthest diagonal mostly lie in tiles on its own
 * XCD (16 without a DIA part; 16 for the 7-point 256^3 stencil, 9 for the
 * 27-point 192^3 one) ({2, 256, 8, 0, 0} when it averages under 4 stored
 * entries per row and n_b is a multiple of 128 or the whole matrix) and
 * {1, 64, 0, c, 0} below, where c = 2 for a handle without DIA part (CSR,
 * or K = 0) whose row_repeat (mhdc_info) is at least 0.5, else 0.  Set
 * before use, not while spmv calls on the handle are in flight. */
typedef struct {
    int32_t rows_per_lane;
    int32_t wg_size;
    int32_t xcd_remap;
    int32_t csr_mode;
    int32_t rhs_group;
} mhdc_launch;

/* M-HDC conversion (Sec. 4.3, Figs. 14-15), all steps in HIP kernels:
 * CSR validation, per-block census of nonzeros per offset, selection with
 * the threshold rule, ascending order per block, scans of the per-block
 * diagonal counts (dia_ptr) and per-row remainder counts, and the scatter
 * into segment-local slots dia_val[k*n_b + (i - ib*n_b)].
 * n >= 0; rowptr has n+1 entries; n_b >= 1; 0 <= threshold <= 1.
 * Fails with BAD_CSR on malformed input, SIZE if nnz > 2^31 - 4097 (the
 * kernels number a tile's entries in int32 chunks of up to 2048), OOM if the
 * DIA part (8 * K * n_b bytes) does not fit. */
mhdc_handle mhdc_from_csr(int32_t n, const int32_t *rowptr,
                          const int32_t *colind, const double *val,
                          int32_t n_b, double threshold);

/* y = A x with the M-HDC kernel (Sec. 4.3, Fig. 16): per row block the
 * CSR-remainder rows, then the block's partial diagonals, each y element
 * written once.  x and y hold n doubles. */
int mhdc_spmv(mhdc_handle h, const double *x, double *y, hipStream_t stream);

/* Y = A X for k right-hand sides, 1 <= k <= 16, A read once per launch.
 * Column r of X starts at X + r*ldx (ldx >= n), likewise Y with ldy. */
int mhdc_spmm(mhdc_handle h, const double *X, int64_t ldx, double *Y,
              int64_t ldy, int32_t k, hipStream_t stream);

/* Y = A X for 1 <= k <= 16 right-hand sides stored row by row: element
 * (i, r) of X at X[i*ldx + r] (ldx >= k), likewise Y with ldy >= k.  Same
 * bits in every column as mhdc_spmm.  Each remainder entry reads one row of
 * X (k contiguous doubles) and each diagonal a contiguous span of rows,
 * where column-major X costs one cache line per column.  The handle's
 * csr_mode (mhdc_launch) picks the CSR-part variant: 1 = staged products
 * (independent gathers; scattered columns), 2 = staged values and columns
 * with each lane gathering for its own rows (rows that repeat their
 * neighbours' offsets, such as stencils), 0 = 2 when row_repeat >= 0.5,
 * the CSR part holds at most 6 entries per row (R <= 6n) or 5 <= k <= 8,
 * else 1.
 * rows_per_lane and rhs_group do not apply.  Each lane carries
 * adjacent columns; X and Y 16-byte aligned with even ldx and ldy let it
 * move them with 16-byte loads and stores (the fast case; otherwise 8-byte
 * accesses, same bits).  k = 1 with ldx = ldy = 1 (a plain vector) runs
 * the single-column kernel of mhdc_spmv.  Asynchronous. */
int mhdc_spmm_rowmajor(mhdc_handle h, const double *X, int64_t ldx, double *Y,
                       int64_t ldy, int32_t k, hipStream_t stream);

/* Y = A X for column-major X and Y exactly as mhdc_spmm (same arguments,
 * same checks, same bits), given a workspace that lets it take the
 * row-major kernel: route 2 transposes X into the workspace (a row-major
 * copy, element (i, r) at ws[i*k' + r], k' = k rounded up to even; 256 rows
 * per workgroup through LDS), then runs the kernel of mhdc_spmm_rowmajor on
 * the copy, storing Y by column; route 1 is mhdc_spmm (ws unused); route 0
 * takes the route mhdc_spmm_ws_route names.  The detour moves 2*n*k'
 * doubles more and pays where the CSR part gathers scattered columns: each
 * such gather then reads one row of X instead of one cache line per
 * column.
 * ws: device memory of at least mhdc_spmm_workspace_bytes(h, k) bytes,
 * 256-byte aligned, overlapping neither X nor Y (INVALID_ARG otherwise,
 * when route 2 is taken); owned by the caller, who keeps it alive until
 * the work queued on the stream has finished; calls that share one
 * workspace must not overlap in time (different streams race).  Allocates
 * nothing.  Asynchronous: two launches on route 2. */
int mhdc_spmm_ws(mhdc_handle h, const double *X, int64_t ldx, double *Y,
                 int64_t ldy, int32_t k, int32_t route, void *ws,
                 size_t ws_bytes, hipStream_t stream);
/* Workspace bytes of mhdc_spmm_ws for k right-hand sides (1..16):
 * 8*n*k', the row-major copy of X. */
int mhdc_spmm_workspace_bytes(mhdc_handle h, int32_t k, size_t *bytes);
/* The route mhdc_spmm_ws takes for route 0 and k right-hand sides:
 * 2 when k >= 2 and k * lone_per_row (mhdc_info) >= 2, else 1.  A lone
 * entry's gather from column-major X touches one cache line per column
 * that no neighbouring row shares; the row-major copy serves all k
 * columns from one line. */
int mhdc_spmm_ws_route(mhdc_handle h, int32_t k, int32_t *route);

/* Decode back to CSR on the device: rowptr[n+1], colind[nnz], val[nnz]
 * (nnz from mhdc_get_info).  Row i merges, by column, its remainder entries
 * and the nonzero slots of its block's partial diagonals; for canonical CSR
 * input this is the identity, bit for bit.  Synchronous. */
int mhdc_to_csr(mhdc_handle h, int32_t *rowptr, int32_t *colind, double *val);

/* Copy the handle's arrays into caller buffers (device pointers, any may be
 * NULL): dia_ptr[n_blk+1], dia_off[K], dia_val[S], rem_ptr[n+1],
 * rem_col[R], rem_val[R].  Synchronous. */
int mhdc_export(mhdc_handle h, int32_t *dia_ptr, int32_t *dia_off,
                double *dia_val, int32_t *rem_ptr, int32_t *rem_col,
                double *rem_val);

int mhdc_get_info(mhdc_handle h, mhdc_info *out);
int mhdc_set_launch(mhdc_handle h, const mhdc_launch *cfg);
void mhdc_destroy(mhdc_handle h);

/* HDC (Sec. 3.4, Figs. 6-8): global census N(d) over the whole matrix,
 * d kept iff N(d)/n >= threshold, DIA values dia_val[k*n + i].  The spmv
 * kernel is the cache-blocked B-HDC kernel (Sec. 4.2, Fig. 13): the format
 * is M-HDC with a single block of n rows, which the paper notes selects the
 * same diagonals (Sec. 6.4.2). */
hdc_handle hdc_from_csr(int32_t n, const int32_t *rowptr,
                        const int32_t *colind, const double *val,
                        double threshold);
int hdc_spmv(hdc_handle h, const double *x, double *y, hipStream_t stream);
/* The HDC kernel without cache blocking (Fig. 8; Fig. 5's DIA kernel when
 * the CSR part is empty): y is set to the CSR part's product, then every
 * diagonal is added in a pass of its own over y, in ascending offset order
 * (Sec. 4.1: y and x move once per diagonal).  Same bits as hdc_spmv; kept
 * as the baseline of the paper's stencil study (Sec. 6.3).  x and y hold
 * n doubles and must not overlap.  Asynchronous: 1 + K launches. */
int hdc_spmv_unblocked(hdc_handle h, const double *x, double *y,
                       hipStream_t stream);
int hdc_spmm(hdc_handle h, const double *X, int64_t ldx, double *Y,
             int64_t ldy, int32_t k, hipStream_t stream);
/* Row-major right-hand sides as in mhdc_spmm_rowmajor. */
int hdc_spmm_rowmajor(hdc_handle h, const double *X, int64_t ldx, double *Y,
                      int64_t ldy, int32_t k, hipStream_t stream);
/* Column-major right-hand sides through a workspace as in mhdc_spmm_ws. */
int hdc_spmm_ws(hdc_handle h, const double *X, int64_t ldx, double *Y,
                int64_t ldy, int32_t k, int32_t route, void *ws,
                size_t ws_bytes, hipStream_t stream);
int hdc_spmm_workspace_bytes(hdc_handle h, int32_t k, size_t *bytes);
int hdc_spmm_ws_route(hdc_handle h, int32_t k, int32_t *route);
int hdc_export(hdc_handle h, int32_t *dia_off, double *dia_val,
               int32_t *rem_ptr, int32_t *rem_col, double *rem_val);
int hdc_get_info(hdc_handle h, mhdc_info *out);
int hdc_set_launch(hdc_handle h, const mhdc_launch *cfg);
void hdc_destroy(hdc_handle h);

/* Plain CSR baseline (Sec. 3.2, Fig. 3): the handle holds a validated copy
 * of the CSR arrays; spmv stages each tile's entries through LDS with
 * coalesced loads and sums every row in ascending column order. */
csr_handle csr_from_csr(int32_t n, const int32_t *rowptr,
                        const int32_t *colind, const double *val);
int csr_spmv(csr_handle h, const double *x, double *y, hipStream_t stream);
int csr_spmm(csr_handle h, const double *X, int64_t ldx, double *Y,
             int64_t ldy, int32_t k, hipStream_t stream);
/* Row-major right-hand sides as in mhdc_spmm_rowmajor. */
int csr_spmm_rowmajor(csr_handle h, const double *X, int64_t ldx, double *Y,
                      int64_t ldy, int32_t k, hipStream_t stream);
/* Column-major right-hand sides through a workspace as in mhdc_spmm_ws. */
int csr_spmm_ws(csr_handle h, const double *X, int64_t ldx, double *Y,
                int64_t ldy, int32_t k, int32_t route, void *ws,
                size_t ws_bytes, hipStream_t stream);
int csr_spmm_workspace_bytes(csr_handle h, int32_t k, size_t *bytes);
int csr_spmm_ws_route(csr_handle h, int32_t k, int32_t *route);
int csr_get_info(csr_handle h, mhdc_info *out);
int csr_set_launch(csr_handle h, const mhdc_launch *cfg);
void csr_destroy(csr_handle h);

/* -------------------------------------------------- memory benchmark */
/* The two memory benchmark kernels of Sec. 6.2 (Figs. 19-20):
 * direct C[i] += A[i]*B[i] (32 bytes per element) and indirect
 * C[i] += A[i]*B[I[i]] (36 bytes per element), the product rounded before
 * the add.  All arrays hold N elements; an index I[i] outside [0, N) leaves
 * C[i] unchanged.  Asynchronous. */
int mhdc_stream_direct(int64_t N, const double *A, const double *B,
                       double *C, hipStream_t stream);
int mhdc_stream_indirect(int64_t N, const double *A, const double *B,
                         const int32_t *I, double *C, hipStream_t stream);

/* ---------------------------------------------- batched persistent launch */
/* Many M-HDC products in one launch.  Not in the paper; it addresses the
 * under-filled machine the paper reports when a matrix has too few row
 * blocks for the threads (Secs. 6.4.2-6.4.3, matrix #17).  All tiles of
 * all items form one sequence (items with more right-hand sides first, so
 * the launch ends on its cheapest tiles); a persistent grid of (CUs x
 * resident workgroups) takes tiles until none is left.  Each item's tiles
 * go to one XCD (items dealt by descending bytes to the least-loaded XCD),
 * so the tiles sharing an item's x rows share an L2; each XCD takes its
 * tiles from a counter of its own and then other XCDs' tiles once its own
 * have run out.  Each
 * tile writes only its own rows, so item i's result is bit-identical to
 * mhdc_spmm(mats[i], X[i], ldx[i], Y[i], ldy[i], nrhs[i]).
 *
 * mats[count]: M-HDC handles (not owned; must outlive the batch).
 * nrhs[count]: right-hand sides per item, 1..16.
 * X[count], Y[count]: HOST arrays of DEVICE pointers, column-major blocks
 * with leading dimensions ldx[i], ldy[i] >= n_i (NULL ldx/ldy = n_i).
 * wg_size: 64 or 256 lanes per workgroup (mhdc_batch_tune picks).
 * Y blocks must not overlap any X block.
 * One batch runs on one stream at a time: every launch of a batch (run or
 * graph_launch) takes tiles from the batch's device counters, so two
 * launches of the same batch in flight together on different streams race
 * and give undefined results.  Launches ordered on one stream are safe;
 * for concurrent streams create one batch per stream (handles may be
 * shared).  SIZE if the tiles of all items exceed 2^31 - 2^20.
 *
 * X/Y are bound at create (and bind) time rather than passed to run: a
 * captured graph replays the same kernel arguments, and the descriptor
 * table it reads is the one place the pointers can change between replays. */
typedef struct mhdc_batch_s *mhdc_batch;
typedef struct {
    int32_t count, wg_size;
    int64_t total_tiles;
    int32_t grid;          /* persistent workgroups per launch */
    double flops;          /* sum of 2 * nnz_i * nrhs_i */
    double bytes_alg;      /* sum of algorithmic bytes (A once, X once, Y once) */
} mhdc_batch_info;

mhdc_batch mhdc_batch_create(int32_t count, const mhdc_handle *mats,
                             const int32_t *nrhs, const double *const *X,
                             const int64_t *ldx, double *const *Y,
                             const int64_t *ldy, int32_t wg_size);
/* As mhdc_batch_create for right-hand sides stored row by row: X[i] holds
 * n_i rows of nrhs[i] values, row r at X[i] + r*ldx[i] with ldx[i] >=
 * nrhs[i] (NULL ldx/ldy = nrhs[i]), as in mhdc_spmm_rowmajor; item i's
 * result is bit-identical to mhdc_spmm_rowmajor(mats[i], X[i], ldx[i],
 * Y[i], ldy[i], nrhs[i]).  The layout is the batch's for its lifetime
 * (mhdc_batch_bind takes pointers of the same layout). */
mhdc_batch mhdc_batch_create_rowmajor(int32_t count, const mhdc_handle *mats,
                                      const int32_t *nrhs,
                                      const double *const *X, const int64_t *ldx,
                                      double *const *Y, const int64_t *ldy,
                                      int32_t wg_size);
/* Replace the X/Y pointers (synchronous; waits for work in flight).  A
 * captured graph reads the table from device memory and sees the change.
 * On failure the batch keeps its previous binding and stays runnable. */
int mhdc_batch_bind(mhdc_batch b, const double *const *X, const int64_t *ldx,
                    double *const *Y, const int64_t *ldy);
/* Enqueue counter reset + persistent kernel on `stream` (asynchronous). */
int mhdc_batch_run(mhdc_batch b, hipStream_t stream);
/* First call captures the reset + persistent kernel into a HIP graph (on an
 * internal stream, no memset node); every call launches that graph on
 * `stream`.  Asynchronous. */
int mhdc_batch_graph_launch(mhdc_batch b, hipStream_t stream);
/* Change the workgroup size (64 or 256; synchronous).  The descriptor table
 * is rebuilt for the new tile size; on failure nothing changes. */
int mhdc_batch_set_wg(mhdc_batch b, int32_t wg_size);
int mhdc_batch_get_info(mhdc_batch b, mhdc_batch_info *out);
void mhdc_batch_destroy(mhdc_batch b);

/* ------------------------------------------------------------ autotuner */
typedef struct {
    int32_t n_b;           /* chosen rows per block */
    mhdc_launch launch;    /* chosen launch shape */
    float us;              /* its mean time per call, microseconds */
    int32_t tried;         /* (n_b, shape) pairs timed */
} mhdc_tune_result;

/* Convert for every candidate n_b (threshold fixed), time spmm with nrhs
 * right-hand sides for each launch shape on `stream` with HIP events, and
 * return the fastest handle (launch shape set) or NULL on error.  The
 * paper gives only a policy range for bl (Sec. 6.4.3); this measures it.
 * Synchronous; allocates and frees its own x/y scratch. */
mhdc_handle mhdc_autotune(int32_t n, const int32_t *rowptr,
                          const int32_t *colind, const double *val,
                          double threshold, int32_t nrhs,
                          const int32_t *nb_candidates, int32_t n_candidates,
                          hipStream_t stream, mhdc_tune_result *out);
/* Mean time of one mhdc_spmv(h, x, y) in microseconds: HIP events around
 * back-to-back launches issued from C on `stream` (the count grows until
 * the window is >= 0.2 ms; best of 4 windows, after 2 warm-up calls), so
 * host-side call overhead does not enter.  Overwrites y.  Synchronous. */
int mhdc_time_spmv(mhdc_handle h, const double *x, double *y, hipStream_t stream,
                   float *us);
/* Time the batch under wg_size 64 and 256, keep the faster.  Runs the
 * batch, so the bound Y blocks are overwritten.  Synchronous. */
int mhdc_batch_tune(mhdc_batch b, hipStream_t stream, int32_t *best_wg,
                    float *best_us);

/* ----------------------------------------------------- learned selector */
/* The paper fixes neither theta nor bl: it proposes a policy (50 <~ bl <~
 * 500, theta = 0.6; Sec. 6.4.3) and leaves the decision open (Sec. 7).  A
 * small network proposes (theta, n_b) from a census of the matrix; the
 * paper's byte model (V = V_A + V_x + V_y, Eqs. 24/34) judges the proposal
 * against the policy (theta = 0.6, n_b = 256), which is also the fallback.
 *
 * Features: 66 floats.  f[b], b < 64 = (sum over block ib, offset d in bin
 * b of N~(d,ib)^2 / rows_ib) / nnz with N~ counted at block size 256 (Sec.
 * 4.3's count) and bin b = 32 for d = 0, 33 + min(floor(log2 d), 30) for
 * d > 0, 31 - min(floor(log2 -d), 31) for d < 0; f[64] = log2(n)/32,
 * f[65] = log2(nnz)/32.  `feat` is a device array of 66 floats.
 * Synchronous. */
int mhdc_features(int32_t n, const int32_t *rowptr, const int32_t *colind,
                  const double *val, float *feat, hipStream_t stream);

/* Network: 66 -> 128 -> 128 -> 2, ReLU hidden layers, FP32.  Parameters
 * (MHDC_MLP_PARAMS floats) in the order W1 (128x66), b1, W2 (128x128), b2,
 * W3 (2x128), b3, row-major.  Output o = (theta, log2 n_b).
 * Scorer (not in the paper): the same network with 40 outputs, one per
 * point of the sweep grid of Sec. 6.4.1 (theta = 0.5 + 0.1 i, i < 5, n_b =
 * 2^(5+j), j < 8, output 8 i + j), each an estimate of that point's log
 * time ratio log(t / t_best); MHDC_MLP_SCORER_PARAMS floats, W3 40x128 and
 * b3 of 40.  The decision is the point of the smallest estimate.  Every
 * entry point below takes either kind; out arrays hold B x
 * mhdc_mlp_outputs(m) floats. */
#define MHDC_MLP_PARAMS 25346
#define MHDC_MLP_SCORER_PARAMS 30248
typedef struct mhdc_mlp_s *mhdc_mlp;
/* params_host: HOST array of initial parameters (the caller draws them). */
mhdc_mlp mhdc_mlp_create(const float *params_host);
/* A scorer from MHDC_MLP_SCORER_PARAMS host floats. */
mhdc_mlp mhdc_mlp_create_scorer(const float *params_host);
/* Outputs per row: 2, or 40 for a scorer (0 and INVALID_ARG for NULL). */
int32_t mhdc_mlp_outputs(mhdc_mlp m);
/* Copy the current parameters to a HOST array (synchronous; 25346 or
 * 30248 floats by kind). */
int mhdc_mlp_get_params(mhdc_mlp m, float *params_host);
/* out[B][2] (scorer: [B][40]) = network(X[B][66]); device arrays;
 * asynchronous on stream. */
int mhdc_mlp_forward(mhdc_mlp m, const float *X, int32_t B, float *out,
                     hipStream_t stream);
/* The forward pass of mhdc_mlp_forward for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels in the same order, so
 * out holds the same bits, but the two hidden layers live in a fixed 2 MB
 * device array of the library (one per GPU, kept until the process ends)
 * and nothing is allocated, freed or synchronised.  1 <= B <= 2048 (SIZE
 * beyond).  X[B][66] and out[B][outputs] are caller device arrays.  Calls on one
 * GPU share that array: two calls that overlap in time on the same GPU
 * (different streams, or different host threads) race and give undefined
 * results; order them on one stream.  Asynchronous on stream. */
int mhdc_mlp_forward_noalloc(mhdc_mlp m, const float *X, int32_t B, float *out,
                             hipStream_t stream);
/* loss = sum_r (w0 (o_r0 - T_r0)^2 + w1 (o_r1 - T_r1)^2) / B and its
 * gradient (MHDC_MLP_PARAMS floats, parameter order) by backpropagation;
 * device arrays; asynchronous on stream.  2-output networks only
 * (NOT_SUPPORTED for a scorer; so is mhdc_mlp_train). */
int mhdc_mlp_loss_grad(mhdc_mlp m, const float *X, const float *T, int32_t B,
                       float w0, float w1, float *loss, float *grad,
                       hipStream_t stream);
/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, rate lr) on
 * minibatches of B rows: step s uses rows order[s*B .. s*B+B) of X[N][66]
 * and targets T[N][2] (device arrays; the caller draws the order).  Every
 * order entry is checked to lie in [0, N) before training (INVALID_ARG
 * otherwise).
 * loss_hist[s] receives each step's loss.  One step is captured once as a
 * HIP graph and replayed.  Synchronous. */
int mhdc_mlp_train(mhdc_mlp m, const float *X, const float *T, int32_t N,
                   const int32_t *order, int64_t steps, int32_t B, float lr,
                   float w0, float w1, float *loss_hist, hipStream_t stream);
/* Grid loss (not in the paper; it scores a proposal by what the paper's
 * sweep of Sec. 6.4.1 measures): G[B][40] holds per row the measured log
 * time ratios log(t / t_best) at theta = 0.5 + 0.1 i (i < 5), n_b =
 * 2^(5+j) (j < 8), at G[r][8 i + j].  Output o_r = (theta, log2 n_b) is
 * scored by the bilinear interpolation of the four grid values around it
 * (the cell above a point on an inner grid line), and outside the grid's
 * box by the value at the clamped point plus |theta - clamp| + |log2 n_b -
 * clamp|; loss = sum_r score_r / B and its gradient (MHDC_MLP_PARAMS
 * floats).  For a scorer, whose outputs o_r[k] estimate G[r][k], the loss
 * is instead sum_r sum_k w_rk (o_r[k] - G[r][k])^2 / (40 B) with w =
 * exp(-G / 0.1) + 0.05 (the near-best points weigh most), gradient
 * MHDC_MLP_SCORER_PARAMS floats.  Device arrays; asynchronous on stream. */
int mhdc_mlp_grid_loss_grad(mhdc_mlp m, const float *X, const float *G, int32_t B,
                            float *loss, float *grad, hipStream_t stream);
/* As mhdc_mlp_train with the grid loss: G[N][40] as above replaces the
 * targets.  The Adam state and step count carry over from earlier training
 * calls on the network.  Synchronous. */
int mhdc_mlp_train_grid(mhdc_mlp m, const float *X, const float *G, int32_t N,
                        const int32_t *order, int64_t steps, int32_t B, float lr,
                        float *loss_hist, hipStream_t stream);
/* Decisions for B feature rows: theta[r] = round(10 clip(o_r0, 0.5, 0.9))/10
 * (the theta grid of Sec. 6.4.1), n_b[r] = 2^clip(round(o_r1), 5, 12),
 * ok[r] = 0 (and the policy 0.6 / 256) for a non-finite output.  A scorer
 * takes the grid point k of its smallest output (the first of equal ones):
 * theta 0.5 + 0.1 (k / 8), n_b 2^(5 + k % 8); ok = 0 and the policy if any
 * output is not finite.  Device arrays; asynchronous on stream. */
int mhdc_mlp_decide(mhdc_mlp m, const float *X, int32_t B, double *theta,
                    int32_t *n_b, int32_t *ok, hipStream_t stream);
void mhdc_mlp_destroy(mhdc_mlp m);

typedef struct {
    double theta;          /* chosen threshold */
    int32_t n_b;           /* chosen rows per block */
    int32_t used_rule;     /* 1 if the policy (0.6, 256) was used */
    double theta_net;      /* the network's proposal (theta snapped to 0.1) */
    int32_t n_b_net;
    int32_t net_ok;        /* 0 if the network gave a non-finite output */
    double bytes_net;      /* model volume V of the proposal */
    double bytes_rule;     /* model volume V of the policy */
    /* The byte model's verdict on the chosen layout against plain CSR
     * (Sec. 5.3), the question of whether to use M-HDC at all (Sec. 7): */
    double rp_est;         /* V_CSR / V of the choice (1 + Eq. 28, v_x = 1) */
    double alpha, beta;    /* filling rate and CSR rate of the choice (Eq. 33) */
    int32_t csr_cheaper;   /* 1 if V_CSR < V, i.e. alpha < 1/(1+b) = 2/3
                              (Eqs. 31-32): plain CSR moves fewer bytes */
    int32_t reserved;
} mhdc_select_result;

/* The judge of mhdc_select, exposed so that offline evaluations apply the
 * same rule: 1 if a proposal whose model volume is v_proposal is kept
 * against the policy's v_policy (v_proposal <= (1 + tolerance) v_policy),
 * else 0.  Host-only; needs no GPU. */
int mhdc_judge_keep(double v_proposal, double v_policy, double tolerance);

/* The candidates mhdc_select_refine times besides the decision (theta,
 * n_b): n_b halved and doubled, theta -+ 0.1, the policy (0.6, 256) and
 * (theta, 4096), each kept only inside the grid of Sec. 6.4.1 (theta in
 * 0.5 .. 0.9, n_b in 32 .. 4096) and only once, the decision itself left
 * out.  Writes up to `cap` pairs and returns how many there are (at most
 * 6).  Host-only; needs no GPU. */
int32_t mhdc_refine_candidates(double theta, int32_t n_b, double *theta_out,
                               int32_t *n_b_out, int32_t cap);

/* Choose (theta, n_b) and convert.  model = NULL uses the policy.  The
 * proposal is kept unless its V exceeds (1 + tolerance) x the policy's V.
 * Returns the M-HDC handle of the choice, NULL on error.  Synchronous. */
mhdc_handle mhdc_select(int32_t n, const int32_t *rowptr,
                        const int32_t *colind, const double *val,
                        mhdc_mlp model, double tolerance,
                        mhdc_select_result *out);

/* mhdc_select's choice refined by measurement (the paper leaves the
 * choice open, Sec. 7; its sweep grid is that of Sec. 6.4.1): the choice,
 * its grid neighbours (n_b halved and doubled within [32, 4096], theta
 * -+ 0.1 within [0.5, 0.9]), the policy (0.6, 256) and the choice's theta
 * with n_b = 4096 are converted and timed with mhdc_time_spmv on `stream`
 * (internal x and y), and the fastest handle is returned; out->theta /
 * n_b / used_rule describe it, the other fields are mhdc_select's.  Up to
 * six conversions beyond mhdc_select's own.  Synchronous; NULL on error
 * (nothing leaks). */
mhdc_handle mhdc_select_refine(int32_t n, const int32_t *rowptr,
                               const int32_t *colind, const double *val,
                               mhdc_mlp model, double tolerance,
                               hipStream_t stream, mhdc_select_result *out);

/* ------------------------------------------------------ failure injection */
/* Test hook: the countdown-th device allocation made by the library from now
 * on fails with MHDC_ERR_OOM (0 disables).  Lets a host-side test drive every
 * error path of a conversion and check that nothing leaks.  Process-wide. */
int mhdc_debug_fail_alloc(int32_t countdown);

#ifdef __cplusplus
}
#endif
#endif /* MHDC_H */
