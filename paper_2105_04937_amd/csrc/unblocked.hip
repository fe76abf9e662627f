// unblocked.hip -- the HDC kernel without cache blocking (Fig. 8; the DIA
// kernel of Fig. 5 when the CSR part is empty), kept as the baseline the
// paper's cache blocking is measured against (Secs. 4.1, 6.3).
//
// y is first set to the CSR part's product, then each diagonal is added in a
// pass of its own over y in ascending offset order, so every element of y
// (and the shifted x) is read once per diagonal.  Within a row this is the
// same sequence of rounded products and additions as the blocked kernel,
// so the two give the same bits.
#include "internal.h"

namespace mhdc {
namespace {

constexpr int UB_WG = 256;

// One diagonal of the global DIA part (values val_k[0..n)): rows whose
// column i + off lies in [0, n) (the is/ie range of Fig. 5) add their term.
__global__ __launch_bounds__(UB_WG) void k_dia_pass(int32_t n, const int32_t *__restrict__ off_k,
                                                    const double *__restrict__ val_k,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ y)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * UB_WG + threadIdx.x;
    if (i >= n)
        return;
    const int64_t j = i + (int64_t)off_k[0];
    if (j < 0 || j >= n)
        return;
    y[i] = __dadd_rn(y[i], __dmul_rn(__builtin_nontemporal_load(val_k + i), x[j]));
}

}  // namespace
}  // namespace mhdc

using namespace mhdc;

extern "C" int hdc_spmv_unblocked(hdc_handle h, const double *x, double *y, hipStream_t stream)
{
    clear_error();
    if (!h)
        return set_error(MHDC_ERR_INVALID_ARG, "handle is NULL");
    const BdcMatrix &m = h->m;
    int rc = launch_rem_part(m, x, y, stream);
    if (rc || m.n == 0)
        return rc;
    const unsigned grid = (unsigned)(((int64_t)m.n + UB_WG - 1) / UB_WG);
    for (int64_t k = 0; k < m.K; k++)
        k_dia_pass<<<grid, UB_WG, 0, stream>>>(m.n, m.dia_off + k, m.dia_val + k * (int64_t)m.n,
                                               x, y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string("diagonal pass launch: ") + hipGetErrorString(e));
    return MHDC_OK;
}
