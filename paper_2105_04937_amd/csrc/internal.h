// internal.h -- shared declarations of libmhdc (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/mhdc.h"

namespace mhdc {

enum Kind : int32_t { KIND_MHDC = 0, KIND_HDC = 1, KIND_CSR = 2 };

// Row-blocked DIA part plus CSR remainder.  M-HDC uses n_b rows per block;
// HDC is the one-block case (n_b = n); CSR has no DIA part (K = 0) and its
// remainder is the whole matrix.
struct BdcMatrix {
    int32_t kind = KIND_MHDC;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t n_b = 1;
    double theta = 0.0;
    int64_t n_blk = 0;
    int64_t K = 0, S = 0, R = 0;
    int32_t *dia_ptr = nullptr;  // [n_blk+1]
    int32_t *dia_off = nullptr;  // [K]
    double *dia_val = nullptr;   // [S]
    int32_t *rem_ptr = nullptr;  // [n+1]
    int32_t *rem_col = nullptr;  // [R]
    double *rem_val = nullptr;   // [R]
    // Blocked kinds with R > 0: bit g of word g/32 is set when rows
    // [64g, 64g+64) hold remainder entries (ceil(n/2048) words).  A tile
    // tests its bits in this small, cache-resident array instead of
    // fetching rem_ptr from HBM before it can start on its diagonals.
    uint32_t *rem_mask = nullptr;
    // Share of the CSR part's nonempty rows whose column offsets repeat the
    // previous row's (0 when the CSR part is empty); picks the CSR mode.
    double row_repeat = 0.0;
    // CSR-part entries per row with no column within 16 of theirs in the
    // two previous rows (0 when the CSR part is empty): gathers that share
    // no cache line with the neighbouring rows'; picks the route of
    // column-major products given a workspace.
    double lone_per_row = 0.0;
    // Largest |offset| of the DIA part's diagonals (0 without a DIA part):
    // how far a tile's x rows lie from its own rows; picks the XCD run length.
    int32_t far_offset = 0;
    int device = 0;
    mhdc_launch launch{2, 256, 0, 0, 0};
    // the launch the conversion chose (launch differs once the caller or
    // the autotuner sets one)
    mhdc_launch dflt{2, 256, 0, 0, 0};
};

// Words of BdcMatrix::rem_mask for n rows (one bit per 64 rows).
inline int64_t rem_mask_words(int64_t n) { return (n + 2047) / 2048; }

// Largest accepted nnz.  The SpMV kernels walk a tile's CSR entries in
// chunks of up to 2048 with int32 entry numbers (chunk end = start + chunk),
// so entry numbers must stay 4096 below INT32_MAX.
constexpr int64_t MAX_NNZ = (int64_t)INT32_MAX - 4096;

// Bytes of the format's own arrays that one product reads (Figs. 2, 7, 15):
// block pointer (M-HDC only: the HDC layout of Fig. 7 has none), offsets,
// DIA slots, and the CSR part (its row pointer only when it has entries).
// The remainder bit mask is an index of this library, not of the format,
// and is not counted.  Every term is an integer below 2^53: the sum is exact.
inline double format_bytes(const BdcMatrix &m)
{
    const double n = m.n;
    if (m.kind == KIND_CSR)
        return 4.0 * (n + 1) + 12.0 * (double)m.nnz;
    const double blk_ptr = m.kind == KIND_HDC ? 0.0 : 4.0 * ((double)m.n_blk + 1);
    return blk_ptr + 4.0 * (double)m.K + 8.0 * (double)m.S + (m.R > 0 ? 4.0 * (n + 1) : 0.0) +
           12.0 * (double)m.R;
}

// Thread-local error state.
int set_error(int code, const std::string &msg);
void clear_error();

// Device memory helpers that record errors.
int dmalloc(void **p, size_t bytes, const char *what);
void dfree(void *p);

#define MHDC_HIP_CHECK(call)                                                  \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            return ::mhdc::set_error(MHDC_ERR_HIP,                            \
                                     std::string(#call " failed: ") +         \
                                         hipGetErrorString(e_));              \
    } while (0)

// converter.hip
int validate_csr(int32_t n, const int32_t *rowptr, const int32_t *colind,
                 const double *val, int64_t *nnz_out);
int build_blocked(BdcMatrix &m, const int32_t *rowptr, const int32_t *colind,
                  const double *val);  // M-HDC (m.kind = MHDC) or HDC
int build_csr(BdcMatrix &m, const int32_t *rowptr, const int32_t *colind,
              const double *val);
int decode_to_csr(const BdcMatrix &m, int32_t *rowptr, int32_t *colind,
                  double *val);
void free_matrix(BdcMatrix &m);

// spmv.hip
struct SpmvArgs;
SpmvArgs make_args(const BdcMatrix &m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                   int32_t k, int32_t v);
int kc_for(int k);
bool row_gather(int32_t csr_mode, int kc);
int check_operands(const BdcMatrix &m, const double *X, int64_t ldx, const double *Y,
                   int64_t ldy, int32_t k);
// y = the CSR part's product alone (zero rows where the part is empty), one
// right-hand side: the first pass of the unblocked HDC kernel.
int launch_rem_part(const BdcMatrix &m, const double *x, double *y, hipStream_t stream);
int launch_spmv(const BdcMatrix &m, const double *X, int64_t ldx, double *Y,
                int64_t ldy, int32_t k, hipStream_t stream);
int check_launch(const mhdc_launch &cfg);
// Row-major right-hand sides (element (i, r) at X[i*ldx + r], ldx >= k).
int check_operands_rm(const BdcMatrix &m, const double *X, int64_t ldx, const double *Y,
                      int64_t ldy, int32_t k);
// Two adjacent columns per lane (16-byte loads and stores) in the row-major
// kernel: X and Y 16-byte aligned, even leading dimensions.  Same bits.
bool rm_pairs(const double *X, int64_t ldx, const double *Y, int64_t ldy);
int rm_columns(int32_t k);  // accumulator width of the row-major kernel (2..16)
// Row-major CSR part by row gathers (csr_mode 2, or csr_mode 0 and rows that
// mostly repeat their neighbours' column offsets, a CSR part of at most 6
// entries per row, or an accumulator width kc of 8) rather than staged
// products.
bool rm_row_gather(const BdcMatrix &m, int kc);
int launch_spmm_rm(const BdcMatrix &m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                   int32_t k, hipStream_t stream);
// Column-major right-hand sides with a caller workspace: route 1 = the
// column-major kernel, 2 = transposed into the workspace, the row-major
// kernel, transposed back (same bits), 0 = 2 where spmm_ws_prefers_rm.
size_t spmm_ws_bytes(const BdcMatrix &m, int32_t k);
bool spmm_ws_prefers_rm(const BdcMatrix &m, int32_t k);
int launch_spmm_ws(const BdcMatrix &m, const double *X, int64_t ldx, double *Y, int64_t ldy,
                   int32_t k, int32_t route, void *ws, size_t ws_bytes, hipStream_t stream);

// scan.hip: exclusive prefix sum of cnt[0..N) into out[0..N] (out[N] =
// total), all int32 on the device; total also returned on the host.
int exclusive_scan_i32(const int32_t *cnt, int32_t *out, int64_t N,
                       int64_t *total, hipStream_t stream);

// api.hip: handle creation shared with the autotuner
mhdc_launch default_launch(int32_t n, int32_t n_b, int64_t nnz, double row_repeat,
                           int32_t far_offset);
// Run length (tiles per XCD run, runs of 2048..4096 rows: 8..16 tiles of
// 256 rows) that keeps the x rows a tile reads through its farthest
// diagonals in the tile's own XCD (the longest without a DIA part).
int32_t xcd_run(int32_t far_offset, int32_t tile_rows);

}  // namespace mhdc

// The opaque handle types of the C-ABI: each wraps one BdcMatrix.
struct mhdc_s {
    mhdc::BdcMatrix m;
};
struct hdc_s {
    mhdc::BdcMatrix m;
};
struct csr_s {
    mhdc::BdcMatrix m;
};
