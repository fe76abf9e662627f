// autotune.hip -- empirical choice of block size and launch shape.
//
// mhdc_autotune converts one CSR matrix for every candidate n_b, times
// the SpMV/SpMM for every launch shape with HIP events on the caller's
// stream, and returns the fastest handle (the others are freed).  The paper
// leaves the choice of bl open beyond a policy range (50 <~ bl <~ 500 with
// theta = 0.6, Sec. 6.4.3); here the choice is measured.
// mhdc_batch_tune times a batch under each workgroup size and keeps the
// faster one.
#include "internal.h"

#include <cstring>
#include <vector>

using namespace mhdc;

namespace {

__global__ __launch_bounds__(256) void k_fill_const(double *p, int64_t count, double v)
{
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < count;
         s += (int64_t)gridDim.x * 256)
        p[s] = v;
}

// Mean time in microseconds of `reps` back-to-back calls after 2 warm-ups;
// reps grows until the timed window is at least ~200 us.
template <class F>
int time_us(F &&call, hipStream_t s, float *out)
{
    hipEvent_t e0, e1;
    MHDC_HIP_CHECK(hipEventCreate(&e0));
    MHDC_HIP_CHECK(hipEventCreate(&e1));
    int rc = MHDC_OK;
    float best = 1e30f;
    int reps = 3;
    for (int w = 0; w < 2 && !rc; w++)
        rc = call();
    for (int round = 0; round < 4 && !rc; round++) {
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && !rc; r++)
            rc = call();
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = set_error(MHDC_ERR_HIP, "event synchronize failed");
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const float us = 1000.0f * ms / reps;
        if (us < best)
            best = us;
        if (ms < 0.2f && reps < 4096)
            reps *= 4;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *out = best;
    return rc;
}

}  // namespace

extern "C" {

mhdc_handle mhdc_autotune(int32_t n, const int32_t *rowptr, const int32_t *colind,
                          const double *val, double threshold, int32_t nrhs,
                          const int32_t *nb_candidates, int32_t n_candidates,
                          hipStream_t stream, mhdc_tune_result *out)
{
    clear_error();
    if (n < 1 || nrhs < 1 || nrhs > 16 || !nb_candidates || n_candidates < 1) {
        set_error(MHDC_ERR_INVALID_ARG, "n >= 1, nrhs in [1,16] and >= 1 candidate required");
        return nullptr;
    }
    double *X = nullptr, *Y = nullptr;
    if (dmalloc((void **)&X, sizeof(double) * (size_t)n * nrhs, "tuning x") ||
        dmalloc((void **)&Y, sizeof(double) * (size_t)n * nrhs, "tuning y")) {
        dfree(X);
        return nullptr;
    }
    k_fill_const<<<256, 256, 0, stream>>>(X, (int64_t)n * nrhs, 0.5);

    // launch shapes (rows per lane, lanes, XCD remap, CSR-part variant,
    // right-hand sides per pass)
    static const mhdc_launch shapes[] = {
        {1, 64, 0, 0, 0},  {1, 256, 0, 0, 0}, {2, 256, 0, 0, 0}, {4, 256, 0, 0, 0},
        {2, 256, 1, 0, 0}, {2, 256, 8, 0, 0}, {1, 256, 16, 0, 0}, {1, 256, 0, 1, 0},
        {1, 256, 0, 2, 0}, {2, 256, 0, 2, 0}, {1, 256, 0, 0, 4}, {2, 256, 0, 0, 4}};
    mhdc_handle best = nullptr;
    mhdc_tune_result res{};
    res.us = 1e30f;
    int rc = MHDC_OK;
    for (int32_t c = 0; c < n_candidates && !rc; c++) {
        mhdc_handle h = mhdc_from_csr(n, rowptr, colind, val, nb_candidates[c], threshold);
        if (!h) {
            rc = mhdc_last_error();
            break;
        }
        bool keep = false;
        // the handle's own default first (its XCD runs fit the matrix's
        // farthest diagonals), then the fixed shapes
        mhdc_launch cands[1 + sizeof(shapes) / sizeof(shapes[0])];
        int n_cand = 0;
        cands[n_cand++] = h->m.launch;
        for (const mhdc_launch &shp : shapes)
            if (memcmp(&shp, &h->m.launch, sizeof(shp)) != 0)
                cands[n_cand++] = shp;
        for (int ci = 0; ci < n_cand && !rc; ci++) {
            const mhdc_launch &shp = cands[ci];
            if ((shp.rows_per_lane == 4 && nrhs > 1) || (shp.rhs_group && shp.rhs_group >= nrhs))
                continue;
            h->m.launch = shp;
            float us = 0;
            rc = time_us([&] { return launch_spmv(h->m, X, n, Y, n, nrhs, stream); }, stream, &us);
            if (rc)
                break;
            res.tried++;
            if (us < res.us) {
                res.us = us;
                res.n_b = nb_candidates[c];
                res.launch = shp;
                keep = true;
            }
        }
        if (keep) {
            if (best)
                mhdc_destroy(best);
            best = h;
            best->m.launch = res.launch;
        } else {
            mhdc_destroy(h);
        }
    }
    (void)hipStreamSynchronize(stream);
    dfree(X);
    dfree(Y);
    if (rc) {
        if (best)
            mhdc_destroy(best);
        set_error(rc, std::string("autotune: ") + mhdc_last_error_message());
        return nullptr;
    }
    if (out)
        *out = res;
    return best;
}

int mhdc_time_spmv(mhdc_handle h, const double *x, double *y, hipStream_t stream, float *us)
{
    clear_error();
    if (!h || !us)
        return set_error(MHDC_ERR_INVALID_ARG, "handle and us are required");
    return time_us([&] { return launch_spmv(h->m, x, h->m.n, y, h->m.n, 1, stream); }, stream,
                   us);
}

int mhdc_batch_tune(mhdc_batch b, hipStream_t stream, int32_t *best_wg, float *best_us)
{
    clear_error();
    if (!b)
        return set_error(MHDC_ERR_INVALID_ARG, "batch is NULL");
    int32_t wgs[2] = {64, 256};
    float t[2] = {0, 0};
    for (int i = 0; i < 2; i++) {
        int rc = mhdc_batch_set_wg(b, wgs[i]);
        if (!rc)
            rc = time_us([&] { return mhdc_batch_run(b, stream); }, stream, &t[i]);
        if (rc)
            return rc;
    }
    const int pick = t[0] <= t[1] ? 0 : 1;
    int rc = mhdc_batch_set_wg(b, wgs[pick]);
    if (rc)
        return rc;
    if (best_wg)
        *best_wg = wgs[pick];
    if (best_us)
        *best_us = t[pick];
    return MHDC_OK;
}

}  // extern "C"
