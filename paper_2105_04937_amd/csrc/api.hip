// api.hip -- the extern "C" entry points of libmhdc.so (declared in
// include/mhdc.h): argument checks, handle lifetime, error state, and the
// per-handle size/model figures.  All arithmetic runs in the kernels of
// converter.hip, scan.hip and spmv.hip.
#include "internal.h"

#include <atomic>
#include <cmath>
#include <new>

namespace mhdc {

namespace {
thread_local int t_code = MHDC_OK;
thread_local std::string t_msg;
std::atomic<int32_t> g_fail_countdown{0};
}  // namespace

int32_t xcd_run(int32_t far_offset, int32_t tile_rows)
{
    // A tile's rows [t*T, t*T + T) read x through the diagonal at +D in tiles
    // t + D/T and t + D/T + 1 (rows weighted by how much of the window each
    // holds); with runs of C tiles per XCD, tile u sits on XCD (u / C) mod 8.
    // Score each C whose runs hold 2048 to 4096 rows (8..16 tiles of 256
    // rows, 4..8 of 512) by the share of those rows on the tile's own XCD
    // over one round of 8*C tiles; ties go to the longer run (near
    // neighbours in the same L2).  192^3 27-point stencil (D = N^2 + N + 1 =
    // 37,057, T = 256): C = 9 (144 tiles = 16 runs), 442 against 460 us at
    // C = 16 for one right-hand side; 256^3 7-point (D = 65,536): C = 16,
    // or 8 for 512-row tiles.
    const int32_t c_hi = tile_rows > 0 && 4096 / tile_rows >= 2 ? 4096 / tile_rows : 2;
    const int32_t c_lo = c_hi / 2;
    if (far_offset <= 0 || tile_rows <= 0)
        return c_hi;
    const int64_t d0 = far_offset / tile_rows, part = far_offset % tile_rows;
    int32_t best = c_hi;
    int64_t best_score = -1;
    for (int32_t c = c_hi; c >= c_lo; c--) {
        int64_t score = 0;  // rows on the own XCD, summed over one round
        for (int64_t t = 0; t < 8 * c; t++) {
            const int64_t x = (t / c) % 8;
            if ((t + d0) / c % 8 == x)
                score += tile_rows - part;
            if (part && (t + d0 + 1) / c % 8 == x)
                score += part;
        }
        // compare shares (score / (8c)) without division
        if (best_score < 0 || score * 8 * best > best_score * 8 * c) {
            best = c;
            best_score = score;
        }
    }
    return best;
}

mhdc_launch default_launch(int32_t n, int32_t n_b, int64_t nnz, double row_repeat,
                           int32_t far_offset)
{
    // Large matrices: 256-lane workgroups, runs of 8-16 consecutive tiles
    // per XCD (xcd_run): a tile's neighbours, whose x entries it also reads
    // through the near diagonals, then share its L2, and the run length puts
    // the tiles its farthest diagonals reach there too (one contiguous eighth
    // per XCD, xcd_remap = 1, is 5% slower).  One row per lane, or two where rows are
    // short (under 4 stored entries on average: a 256-row tile of the banded
    // 3-point matrix moves too little per workgroup and runs 33% slower than
    // a 512-row one); two rows per lane keep the wave-uniform diagonal path
    // only when n_b is a multiple of 128 (or the matrix one block).  On the
    // 256^3 heptadiagonal and the 192^3 partially diagonal cases the default
    // is within 4% of the best of 7 shapes for every n_b tried.
    // Small matrices: 64-lane workgroups so that the 256 CUs get work.
    // With one row per lane, a CSR part whose rows mostly repeat the previous
    // row's column offsets (stencils) stages values and columns and lets
    // each lane gather x for its own rows (csr_mode 2): the wavefront's
    // gathers then hit neighbouring elements (256^3 7-point CSR: 338 us
    // against 361 us with staged products; on rows of mixed structure the
    // staged products are faster, 545 against 596 us on the 192^3 partially
    // diagonal CSR).
    const int32_t mode1 = row_repeat >= 0.5 ? 2 : 0;
    if ((int64_t)n >= 256LL * 2 * 2048) {
        const bool short_rows = nnz > 0 && nnz < 4LL * n;
        const bool v2_uniform = n_b <= 0 || n_b >= n || n_b % 128 == 0;
        if (short_rows && v2_uniform)
            return mhdc_launch{2, 256, 8, 0, 0};
        return mhdc_launch{1, 256, xcd_run(far_offset, 256), mode1, 0};
    }
    return mhdc_launch{1, 64, 0, mode1, 0};
}

namespace {

void fill_info(const BdcMatrix &m, mhdc_info *o)
{
    o->kind = m.kind;
    o->n = m.n;
    o->nnz = m.nnz;
    o->n_b = m.kind == KIND_CSR ? 0 : m.n_b;
    o->theta = m.theta;
    o->n_blk = m.n_blk;
    o->K = m.K;
    o->S = m.S;
    o->R = m.R;
    const double n = m.n, nnz = (double)m.nnz, R = (double)m.R, S = (double)m.S;
    o->beta = nnz > 0 ? R / nnz : 0.0;
    o->alpha = S > 0 ? (nnz - R) / S : 1.0;
    o->bytes_alg = format_bytes(m) + 16.0 * n;
    o->bytes_paper = m.kind == KIND_CSR ? 12.0 * nnz + 4.0 * n + 16.0 * n
                                        : 12.0 * R + 4.0 * n + 8.0 * S + 16.0 * n;
    const double v_csr = 12.0 * nnz + 4.0 * n + 16.0 * n;
    o->rp_est = o->bytes_paper > 0 ? v_csr / o->bytes_paper : 1.0;
    o->rows_per_lane = m.launch.rows_per_lane;
    o->wg_size = m.launch.wg_size;
    o->xcd_remap = m.launch.xcd_remap;
    o->csr_mode = m.launch.csr_mode;
    o->rhs_group = m.launch.rhs_group;
    o->row_repeat = m.row_repeat;
    o->lone_per_row = m.lone_per_row;
}

int check_theta_nb(int32_t n, int32_t n_b, double theta, bool need_nb)
{
    if (n < 0)
        return set_error(MHDC_ERR_INVALID_ARG, "n must be >= 0");
    if (need_nb && n_b < 1)
        return set_error(MHDC_ERR_INVALID_ARG, "n_b must be >= 1");
    if (!(theta >= 0.0 && theta <= 1.0))
        return set_error(MHDC_ERR_INVALID_ARG, "threshold must lie in [0, 1]");
    return MHDC_OK;
}

template <class H>
H *make_handle(int kind, int32_t n, int32_t n_b, double theta)
{
    H *h = new (std::nothrow) H;
    if (!h) {
        set_error(MHDC_ERR_OOM, "host allocation of the handle failed");
        return nullptr;
    }
    h->m.kind = kind;
    h->m.n = n;
    h->m.n_b = n_b;
    h->m.theta = theta;
    h->m.launch = default_launch(n, n_b, 0, 0.0, 0);
    (void)hipGetDevice(&h->m.device);
    return h;
}

template <class H>
H *finish(H *h, int rc)
{
    if (rc) {
        free_matrix(h->m);
        delete h;
        return nullptr;
    }
    // the staging choice by row repetition is made for handles without a
    // DIA part: next to partial diagonals the remainder is small, and with
    // it the staged products measured faster on the selector's matrices
    h->m.launch = default_launch(h->m.n, h->m.n_b, h->m.nnz, h->m.K > 0 ? 0.0 : h->m.row_repeat,
                                 h->m.far_offset);
    h->m.dflt = h->m.launch;
    return h;
}

int copy_out(void *dst, const void *src, size_t bytes)
{
    if (!dst || bytes == 0)
        return MHDC_OK;
    MHDC_HIP_CHECK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToDevice));
    return MHDC_OK;
}

int set_launch(BdcMatrix &m, const mhdc_launch *cfg)
{
    if (!cfg)
        return set_error(MHDC_ERR_INVALID_ARG, "cfg is NULL");
    int rc = check_launch(*cfg);
    if (rc)
        return rc;
    m.launch = *cfg;
    return MHDC_OK;
}

}  // namespace

int set_error(int code, const std::string &msg)
{
    t_code = code;
    t_msg = msg;
    return code;
}

void clear_error()
{
    t_code = MHDC_OK;
    t_msg.clear();
}

int dmalloc(void **p, size_t bytes, const char *what)
{
    *p = nullptr;
    if (bytes == 0)
        return MHDC_OK;
    int32_t c = g_fail_countdown.load();
    if (c > 0 && g_fail_countdown.fetch_sub(1) == 1)
        return set_error(MHDC_ERR_OOM, std::string("injected allocation failure: ") + what);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(MHDC_ERR_OOM, std::string("hipMalloc of ") + what + " (" +
                                           std::to_string(bytes) + " bytes) failed: " +
                                           hipGetErrorString(e));
    }
    return MHDC_OK;
}

void dfree(void *p)
{
    if (p)
        (void)hipFree(p);
}

}  // namespace mhdc

using namespace mhdc;

extern "C" {

int mhdc_last_error(void) { return t_code; }
const char *mhdc_last_error_message(void) { return t_msg.c_str(); }

const char *mhdc_error_string(int code)
{
    switch (code) {
    case MHDC_OK: return "MHDC_OK";
    case MHDC_ERR_INVALID_ARG: return "MHDC_ERR_INVALID_ARG";
    case MHDC_ERR_BAD_CSR: return "MHDC_ERR_BAD_CSR";
    case MHDC_ERR_OOM: return "MHDC_ERR_OOM";
    case MHDC_ERR_HIP: return "MHDC_ERR_HIP";
    case MHDC_ERR_SIZE: return "MHDC_ERR_SIZE";
    case MHDC_ERR_NOT_SUPPORTED: return "MHDC_ERR_NOT_SUPPORTED";
    }
    return "unknown";
}

int mhdc_debug_fail_alloc(int32_t countdown)
{
    g_fail_countdown.store(countdown > 0 ? countdown : 0);
    return MHDC_OK;
}

// ------------------------------------------------------------------ M-HDC
mhdc_handle mhdc_from_csr(int32_t n, const int32_t *rowptr, const int32_t *colind,
                          const double *val, int32_t n_b, double threshold)
{
    clear_error();
    if (check_theta_nb(n, n_b, threshold, true))
        return nullptr;
    mhdc_s *h = make_handle<mhdc_s>(KIND_MHDC, n, n_b, threshold);
    if (!h)
        return nullptr;
    return finish(h, build_blocked(h->m, rowptr, colind, val));
}

int mhdc_spmv(mhdc_handle h, const double *x, double *y, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmv(h->m, x, h->m.n, y, h->m.n, 1, stream);
}

int mhdc_spmm(mhdc_handle h, const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t k,
              hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmv(h->m, X, ldx, Y, ldy, k, stream);
}

int mhdc_spmm_rowmajor(mhdc_handle h, const double *X, int64_t ldx, double *Y, int64_t ldy,
                       int32_t k, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmm_rm(h->m, X, ldx, Y, ldy, k, stream);
}

int mhdc_spmm_ws(mhdc_handle h, const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t k,
                int32_t route, void *ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmm_ws(h->m, X, ldx, Y, ldy, k, route, ws, ws_bytes, stream);
}

int mhdc_spmm_workspace_bytes(mhdc_handle h, int32_t k, size_t *bytes)
{
    clear_error();
    if (!h || !bytes)
        return set_error(MHDC_ERR_INVALID_ARG, "handle or bytes is NULL");
    if (k < 1 || k > 16)
        return set_error(MHDC_ERR_INVALID_ARG, "k must be in [1, 16]");
    *bytes = spmm_ws_bytes(h->m, k);
    return MHDC_OK;
}

int mhdc_spmm_ws_route(mhdc_handle h, int32_t k, int32_t *route)
{
    clear_error();
    if (!h || !route)
        return set_error(MHDC_ERR_INVALID_ARG, "handle or route is NULL");
    if (k < 1 || k > 16)
        return set_error(MHDC_ERR_INVALID_ARG, "k must be in [1, 16]");
    *route = spmm_ws_prefers_rm(h->m, k) ? 2 : 1;
    return MHDC_OK;
}

int mhdc_to_csr(mhdc_handle h, int32_t *rowptr, int32_t *colind, double *val)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return decode_to_csr(h->m, rowptr, colind, val);
}

int mhdc_export(mhdc_handle h, int32_t *dia_ptr, int32_t *dia_off, double *dia_val,
                int32_t *rem_ptr, int32_t *rem_col, double *rem_val)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    const BdcMatrix &m = h->m;
    int rc;
    if ((rc = copy_out(dia_ptr, m.dia_ptr, sizeof(int32_t) * (size_t)(m.n_blk + 1))))
        return rc;
    if ((rc = copy_out(dia_off, m.dia_off, sizeof(int32_t) * (size_t)m.K)))
        return rc;
    if ((rc = copy_out(dia_val, m.dia_val, sizeof(double) * (size_t)m.S)))
        return rc;
    if ((rc = copy_out(rem_ptr, m.rem_ptr, sizeof(int32_t) * (size_t)(m.n + 1))))
        return rc;
    if ((rc = copy_out(rem_col, m.rem_col, sizeof(int32_t) * (size_t)m.R)))
        return rc;
    return copy_out(rem_val, m.rem_val, sizeof(double) * (size_t)m.R);
}

int mhdc_get_info(mhdc_handle h, mhdc_info *out)
{
    clear_error();
    if (!h || !out)
        return set_error(MHDC_ERR_INVALID_ARG, "handle or out is NULL");
    fill_info(h->m, out);
    return MHDC_OK;
}

int mhdc_set_launch(mhdc_handle h, const mhdc_launch *cfg)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return set_launch(h->m, cfg);
}

void mhdc_destroy(mhdc_handle h)
{
    if (!h)
        return;
    free_matrix(h->m);
    delete h;
}

// ------------------------------------------------------------------ HDC
hdc_handle hdc_from_csr(int32_t n, const int32_t *rowptr, const int32_t *colind,
                        const double *val, double threshold)
{
    clear_error();
    if (check_theta_nb(n, 1, threshold, false))
        return nullptr;
    hdc_s *h = make_handle<hdc_s>(KIND_HDC, n, n > 0 ? n : 1, threshold);
    if (!h)
        return nullptr;
    return finish(h, build_blocked(h->m, rowptr, colind, val));
}

int hdc_spmv(hdc_handle h, const double *x, double *y, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmv(h->m, x, h->m.n, y, h->m.n, 1, stream);
}

int hdc_spmm(hdc_handle h, const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t k,
             hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmv(h->m, X, ldx, Y, ldy, k, stream);
}

int hdc_spmm_rowmajor(hdc_handle h, const double *X, int64_t ldx, double *Y, int64_t ldy,
                       int32_t k, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmm_rm(h->m, X, ldx, Y, ldy, k, stream);
}

int hdc_spmm_ws(hdc_handle h, const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t k,
               int32_t route, void *ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmm_ws(h->m, X, ldx, Y, ldy, k, route, ws, ws_bytes, stream);
}

int hdc_spmm_workspace_bytes(hdc_handle h, int32_t k, size_t *bytes)
{
    clear_error();
    if (!h || !bytes)
        return set_error(MHDC_ERR_INVALID_ARG, "handle or bytes is NULL");
    if (k < 1 || k > 16)
        return set_error(MHDC_ERR_INVALID_ARG, "k must be in [1, 16]");
    *bytes = spmm_ws_bytes(h->m, k);
    return MHDC_OK;
}

int hdc_spmm_ws_route(hdc_handle h, int32_t k, int32_t *route)
{
    clear_error();
    if (!h || !route)
        return set_error(MHDC_ERR_INVALID_ARG, "handle or route is NULL");
    if (k < 1 || k > 16)
        return set_error(MHDC_ERR_INVALID_ARG, "k must be in [1, 16]");
    *route = spmm_ws_prefers_rm(h->m, k) ? 2 : 1;
    return MHDC_OK;
}

int hdc_export(hdc_handle h, int32_t *dia_off, double *dia_val, int32_t *rem_ptr,
               int32_t *rem_col, double *rem_val)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    const BdcMatrix &m = h->m;
    int rc;
    if ((rc = copy_out(dia_off, m.dia_off, sizeof(int32_t) * (size_t)m.K)))
        return rc;
    if ((rc = copy_out(dia_val, m.dia_val, sizeof(double) * (size_t)m.S)))
        return rc;
    if ((rc = copy_out(rem_ptr, m.rem_ptr, sizeof(int32_t) * (size_t)(m.n + 1))))
        return rc;
    if ((rc = copy_out(rem_col, m.rem_col, sizeof(int32_t) * (size_t)m.R)))
        return rc;
    return copy_out(rem_val, m.rem_val, sizeof(double) * (size_t)m.R);
}

int hdc_get_info(hdc_handle h, mhdc_info *out)
{
    clear_error();
    if (!h || !out)
        return set_error(MHDC_ERR_INVALID_ARG, "handle or out is NULL");
    fill_info(h->m, out);
    return MHDC_OK;
}

int hdc_set_launch(hdc_handle h, const mhdc_launch *cfg)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return set_launch(h->m, cfg);
}

void hdc_destroy(hdc_handle h)
{
    if (!h)
        return;
    free_matrix(h->m);
    delete h;
}

// ------------------------------------------------------------------ CSR
csr_handle csr_from_csr(int32_t n, const int32_t *rowptr, const int32_t *colind,
                        const double *val)
{
    clear_error();
    if (check_theta_nb(n, 1, 0.0, false))
        return nullptr;
    csr_s *h = make_handle<csr_s>(KIND_CSR, n, 0, 0.0);
    if (!h)
        return nullptr;
    return finish(h, build_csr(h->m, rowptr, colind, val));
}

int csr_spmv(csr_handle h, const double *x, double *y, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmv(h->m, x, h->m.n, y, h->m.n, 1, stream);
}

int csr_spmm(csr_handle h, const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t k,
             hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmv(h->m, X, ldx, Y, ldy, k, stream);
}

int csr_spmm_rowmajor(csr_handle h, const double *X, int64_t ldx, double *Y, int64_t ldy,
                       int32_t k, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmm_rm(h->m, X, ldx, Y, ldy, k, stream);
}

int csr_spmm_ws(csr_handle h, const double *X, int64_t ldx, double *Y, int64_t ldy, int32_t k,
               int32_t route, void *ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return launch_spmm_ws(h->m, X, ldx, Y, ldy, k, route, ws, ws_bytes, stream);
}

int csr_spmm_workspace_bytes(csr_handle h, int32_t k, size_t *bytes)
{
    clear_error();
    if (!h || !bytes)
        return set_error(MHDC_ERR_INVALID_ARG, "handle or bytes is NULL");
    if (k < 1 || k > 16)
        return set_error(MHDC_ERR_INVALID_ARG, "k must be in [1, 16]");
    *bytes = spmm_ws_bytes(h->m, k);
    return MHDC_OK;
}

int csr_spmm_ws_route(csr_handle h, int32_t k, int32_t *route)
{
    clear_error();
    if (!h || !route)
        return set_error(MHDC_ERR_INVALID_ARG, "handle or route is NULL");
    if (k < 1 || k > 16)
        return set_error(MHDC_ERR_INVALID_ARG, "k must be in [1, 16]");
    *route = spmm_ws_prefers_rm(h->m, k) ? 2 : 1;
    return MHDC_OK;
}

int csr_get_info(csr_handle h, mhdc_info *out)
{
    clear_error();
    if (!h || !out)
        return set_error(MHDC_ERR_INVALID_ARG, "handle or out is NULL");
    fill_info(h->m, out);
    return MHDC_OK;
}

int csr_set_launch(csr_handle h, const mhdc_launch *cfg)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    return set_launch(h->m, cfg);
}

void csr_destroy(csr_handle h)
{
    if (!h)
        return;
    free_matrix(h->m);
    delete h;
}

}  // extern "C"
