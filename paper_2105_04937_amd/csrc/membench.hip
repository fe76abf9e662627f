// membench.hip -- the memory benchmark kernels of Sec. 6.2 (Figs. 19-20),
// used to calibrate achievable HBM bandwidth and the hardware byte counters.
#include "internal.h"

namespace mhdc {
namespace {

__global__ __launch_bounds__(256) void k_stream_direct(int64_t N, const double *__restrict__ A,
                                                       const double *__restrict__ B,
                                                       double *__restrict__ C)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * 256)
        C[i] += A[i] * B[i];
}

__global__ __launch_bounds__(256) void k_stream_indirect(int64_t N, const double *__restrict__ A,
                                                         const double *__restrict__ B,
                                                         const int32_t *__restrict__ I,
                                                         double *__restrict__ C)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * 256)
        C[i] += A[i] * B[I[i]];
}

unsigned stream_grid(int64_t N)
{
    int64_t g = (N + 255) / 256;
    if (g > 256 * 64)
        g = 256 * 64;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace
}  // namespace mhdc

using namespace mhdc;

extern "C" int mhdc_stream_direct(int64_t N, const double *A, const double *B, double *C,
                                  hipStream_t stream)
{
    clear_error();
    if (N < 0 || (N > 0 && (!A || !B || !C)))
        return set_error(MHDC_ERR_INVALID_ARG, "bad stream_direct arguments");
    if (N == 0)
        return MHDC_OK;
    k_stream_direct<<<stream_grid(N), 256, 0, stream>>>(N, A, B, C);
    MHDC_HIP_CHECK(hipGetLastError());
    return MHDC_OK;
}

extern "C" int mhdc_stream_indirect(int64_t N, const double *A, const double *B,
                                    const int32_t *I, double *C, hipStream_t stream)
{
    clear_error();
    if (N < 0 || (N > 0 && (!A || !B || !I || !C)))
        return set_error(MHDC_ERR_INVALID_ARG, "bad stream_indirect arguments");
    if (N == 0)
        return MHDC_OK;
    k_stream_indirect<<<stream_grid(N), 256, 0, stream>>>(N, A, B, I, C);
    MHDC_HIP_CHECK(hipGetLastError());
    return MHDC_OK;
}
