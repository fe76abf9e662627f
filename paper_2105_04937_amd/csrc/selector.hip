// selector.hip -- learned choice of (theta, n_b) for M-HDC.
//
// The paper fixes neither parameter; it gives a policy (50 <~ bl <~ 500,
// theta = 0.6) and notes that the CSR rate, computable in advance, drives
// performance (Sec. 6.4.3), and leaves open how to decide M-HDC's use
// (Sec. 7).  Here a small network reads a census of the matrix and proposes
// (theta, n_b); the paper's byte model (V of Eqs. 24/34, the basis of the
// relative performance of Eq. 28) judges the proposal against the policy
// and the policy is the fallback.
//
// Features (66, FP32): census of nonzeros per (block, offset) at probe
// block size 256 (the N~(d, ib) of Sec. 4.3); per offset bin b (sign and
// floor(log2|d|)) f[b] = sum N~^2 / rows_ib / nnz, then log2(n)/32 and
// log2(nnz)/32.  The sums are exact 64-bit integers split into full blocks
// and the last block, finished in FP64.
//
// Network: 66 -> 128 -> 128 -> 2, ReLU hidden layers, FP32 parameters in
// one vector (W1 128x66, b1, W2 128x128, b2, W3 2x128, b3, row-major).
// Scorer: the same network with 40 outputs (W3 40x128, b3), one per point
// of the (theta, n_b) sweep grid, each an estimate of that point's log
// time ratio; the decision is the point of the smallest estimate.
// Every reduction (over inputs in the forward pass, over the minibatch in
// the weight gradients) runs in a fixed order in one thread, so training is
// deterministic.  One training step (minibatch gather, forward, loss,
// backward, Adam, step counter) is captured once as a HIP graph and
// replayed; the step counter lives in device memory.  The layers are tiny
// (at most 128x128 per sample); each launch is latency-bound, not a job
// for the matrix cores.
#include "census.h"
#include "internal.h"

#include <cmath>
#include <mutex>
#include <new>
#include <vector>

namespace mhdc {
namespace {

constexpr int N_BINS = 64, N_IN = 66, HID = 128, N_OUT = 2, PROBE_NB = 256;
// the (theta, log2 n_b) sweep grid of the grid loss: theta = 0.5 + 0.1 i
// (i < 5), n_b = 2^(5 + j) (j < 8)
constexpr int GRID_TH = 5, GRID_NB = 8, N_GRID = GRID_TH * GRID_NB;
constexpr int P_W1 = 0;
constexpr int P_B1 = P_W1 + HID * N_IN;
constexpr int P_W2 = P_B1 + HID;
constexpr int P_B2 = P_W2 + HID * HID;
constexpr int P_W3 = P_B2 + HID;
constexpr int P_B3 = P_W3 + N_OUT * HID;
constexpr int N_PARAMS = P_B3 + N_OUT;
static_assert(N_PARAMS == 25346, "parameter layout");
// offsets of b3 and parameter counts for n_out outputs
constexpr int p_b3(int n_out) { return P_W3 + n_out * HID; }
constexpr int n_params(int n_out) { return p_b3(n_out) + n_out; }
static_assert(n_params(N_GRID) == 30248, "scorer parameter layout");
// scorer loss weight exp(-g / SCORE_TEMP) + SCORE_FLOOR per grid point
constexpr float SCORE_TEMP = 0.1f, SCORE_FLOOR = 0.05f;
constexpr int TW = 256;

inline unsigned blocks_for(int64_t items) { return (unsigned)((items + TW - 1) / TW); }

// ------------------------------------------------------------- features
__device__ inline int offset_bin(int32_t d)
{
    if (d == 0)
        return 32;
    const uint32_t a = d > 0 ? (uint32_t)d : (uint32_t)(-(int64_t)d);
    const int k = 31 - __clz(a);
    return d > 0 ? 33 + min(k, 30) : 31 - min(k, 31);
}

__global__ __launch_bounds__(CENSUS_WG) void k_feat_census(
    int32_t n, int64_t n_blk, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ colind, const double *__restrict__ val, int32_t *gkeys,
    int32_t *gcnts, unsigned long long *sums)
{
    __shared__ int32_t s_keys[CENSUS_LDS_SLOTS];
    __shared__ int32_t s_cnts[CENSUS_LDS_SLOTS];
    __shared__ unsigned long long s_sum[2 * N_BINS];  // [0,64) full blocks, [64,128) last
    for (int t = threadIdx.x; t < 2 * N_BINS; t += CENSUS_WG)
        s_sum[t] = 0;
    for (int64_t ib = blockIdx.x; ib < n_blk; ib += gridDim.x) {
        const int64_t r0 = ib * PROBE_NB, r1 = min((int64_t)n, r0 + PROBE_NB);
        int32_t *keys, *cnts;
        const uint32_t cap = census_block(r0, r1, rowptr[r0], rowptr[r1], rowptr, colind, val,
                                          s_keys, s_cnts, CENSUS_LDS_SLOTS, gkeys, gcnts,
                                          &keys, &cnts);
        const int base = ib == n_blk - 1 ? N_BINS : 0;
        for (uint32_t s = threadIdx.x; s < cap; s += CENSUS_WG) {
            const int32_t key = keys[s];
            if (key != EMPTY_KEY) {
                const unsigned long long c = (unsigned long long)cnts[s];
                atomicAdd(&s_sum[base + offset_bin(key)], c * c);
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < 2 * N_BINS; t += CENSUS_WG)
        if (s_sum[t])
            atomicAdd(&sums[t], s_sum[t]);
}

__global__ void k_feat_finish(int32_t n, int64_t nnz, int64_t n_blk,
                              const unsigned long long *__restrict__ sums, float *feat)
{
    const int b = threadIdx.x;
    const double rows_last = (double)(n - (n_blk - 1) * PROBE_NB);
    if (b < N_BINS) {
        double f = 0.0;
        if (nnz > 0)
            f = ((double)sums[b] / (double)PROBE_NB + (double)sums[N_BINS + b] / rows_last) /
                (double)nnz;
        feat[b] = (float)f;
    } else if (b == N_BINS) {
        feat[b] = (float)(log2((double)n) / 32.0);
    } else if (b == N_BINS + 1) {
        feat[b] = nnz > 0 ? (float)(log2((double)nnz) / 32.0) : 0.0f;
    }
}

// ------------------------------------------------------------- network
// out[r][j] = act(b[j] + sum_i W[j][i] * in[r][i]), i ascending
__global__ __launch_bounds__(TW) void k_dense_fwd(const float *__restrict__ in, int in_dim,
                                                  const float *__restrict__ W,
                                                  const float *__restrict__ b, int out_dim,
                                                  float *__restrict__ out, int B, int relu)
{
    const int idx = blockIdx.x * TW + threadIdx.x;
    if (idx >= B * out_dim)
        return;
    const int r = idx / out_dim, j = idx - r * out_dim;
    const float *w = W + (int64_t)j * in_dim;
    const float *x = in + (int64_t)r * in_dim;
    float s = b[j];
    for (int i = 0; i < in_dim; i++)
        s += w[i] * x[i];
    out[idx] = relu ? fmaxf(s, 0.0f) : s;
}

// loss = sum_r sum_o w_o (out - T)^2 / B (fixed-order tree), d_out = 2 w (out - T) / B.
// One workgroup.  loss_at: destination of the loss; with step != nullptr the
// loss goes to loss_at[*local_step].
__global__ __launch_bounds__(TW) void k_loss_grad(const float *__restrict__ out,
                                                  const float *__restrict__ T, int B, float w0,
                                                  float w1, float *__restrict__ d_out,
                                                  float *loss_at, const int32_t *local_step)
{
    __shared__ float part[TW];
    float acc = 0.0f;
    for (int idx = threadIdx.x; idx < B * N_OUT; idx += TW) {
        const float w = (idx % N_OUT) == 0 ? w0 : w1;
        const float d = out[idx] - T[idx];
        d_out[idx] = 2.0f * w * d / (float)B;
        acc += w * d * d;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = TW / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float *dst = loss_at + (local_step ? *local_step : 0);
        *dst = part[0] / (float)B;
    }
}

// gW[j][i] = sum_r d_out[r][j] * in[r][i];  gb[j] = sum_r d_out[r][j]
__global__ __launch_bounds__(TW) void k_dense_bwd_w(const float *__restrict__ d_out,
                                                    const float *__restrict__ in, int B,
                                                    int in_dim, int out_dim,
                                                    float *__restrict__ gW,
                                                    float *__restrict__ gb)
{
    const int idx = blockIdx.x * TW + threadIdx.x;
    if (idx >= out_dim * (in_dim + 1))
        return;
    const int j = idx / (in_dim + 1), i = idx - j * (in_dim + 1);
    float s = 0.0f;
    if (i < in_dim) {
        for (int r = 0; r < B; r++)
            s += d_out[(int64_t)r * out_dim + j] * in[(int64_t)r * in_dim + i];
        gW[(int64_t)j * in_dim + i] = s;
    } else {
        for (int r = 0; r < B; r++)
            s += d_out[(int64_t)r * out_dim + j];
        gb[j] = s;
    }
}

// d_in[r][i] = (sum_j d_out[r][j] W[j][i]) * [h[r][i] > 0]   (h = ReLU output)
__global__ __launch_bounds__(TW) void k_dense_bwd_x(const float *__restrict__ d_out,
                                                    const float *__restrict__ W,
                                                    const float *__restrict__ h, int B,
                                                    int in_dim, int out_dim,
                                                    float *__restrict__ d_in)
{
    const int idx = blockIdx.x * TW + threadIdx.x;
    if (idx >= B * in_dim)
        return;
    const int r = idx / in_dim, i = idx - r * in_dim;
    float s = 0.0f;
    for (int j = 0; j < out_dim; j++)
        s += d_out[(int64_t)r * out_dim + j] * W[(int64_t)j * in_dim + i];
    d_in[idx] = h[idx] > 0.0f ? s : 0.0f;
}

// Adam at step t = *step + 1 (Kingma & Ba, bias-corrected moments)
__global__ __launch_bounds__(TW) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                             float *__restrict__ m, float *__restrict__ v,
                                             int P, float lr, float b1, float b2, float eps,
                                             const int32_t *step)
{
    const int idx = blockIdx.x * TW + threadIdx.x;
    if (idx >= P)
        return;
    const float t = (float)(*step + 1);
    const float mi = b1 * m[idx] + (1.0f - b1) * g[idx];
    const float vi = b2 * v[idx] + (1.0f - b2) * g[idx] * g[idx];
    m[idx] = mi;
    v[idx] = vi;
    const float mh = mi / (1.0f - powf(b1, t));
    const float vh = vi / (1.0f - powf(b2, t));
    p[idx] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_steps_inc(int32_t *step, int32_t *local_step)
{
    *step += 1;
    *local_step += 1;
}

__global__ void k_zero_i32(int32_t *p) { *p = 0; }

// x = 0.5 (timing input of the refinement; the values do not change the
// kernel's work)
__global__ __launch_bounds__(TW) void k_fill_half(double *x, int32_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * TW + threadIdx.x; i < n; i += (int64_t)gridDim.x * TW)
        x[i] = 0.5;
}

// bad = 1 if an entry of order[0..count) is outside [0, N)
__global__ __launch_bounds__(TW) void k_check_order(const int32_t *__restrict__ order, int64_t count,
                                                    int32_t N, int32_t *bad)
{
    for (int64_t i = (int64_t)blockIdx.x * TW + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * TW)
        if (order[i] < 0 || order[i] >= N)
            *bad = 1;
}

// rows order[local_step*B + r] of X and of the targets T (tdim values per
// row: N_OUT target outputs, or N_GRID grid values) -> minibatch buffers
__global__ __launch_bounds__(TW) void k_gather(const float *__restrict__ X,
                                               const float *__restrict__ T, int tdim,
                                               const int32_t *__restrict__ order,
                                               const int32_t *local_step, int B,
                                               float *__restrict__ Xb, float *__restrict__ Tb)
{
    const int idx = blockIdx.x * TW + threadIdx.x;
    if (idx >= B * (N_IN + tdim))
        return;
    const int r = idx / (N_IN + tdim), c = idx - r * (N_IN + tdim);
    const int64_t src = order[(int64_t)(*local_step) * B + r];
    if (c < N_IN)
        Xb[(int64_t)r * N_IN + c] = X[src * N_IN + c];
    else
        Tb[(int64_t)r * tdim + (c - N_IN)] = T[src * tdim + (c - N_IN)];
}

// Grid loss: each output row o = (theta, log2 n_b) read as a point of the
// sweep grid and scored by the grid values G (the measured log time ratios)
// interpolated bilinearly from the four surrounding points; outside the
// grid's box the value at the clamped point plus the distance to the box.
// loss = sum_r value_r / B (fixed-order tree), d_out = d value / d o / B.
// One workgroup.
__global__ __launch_bounds__(TW) void k_grid_loss_grad(const float *__restrict__ out,
                                                       const float *__restrict__ G, int B,
                                                       float *__restrict__ d_out,
                                                       float *loss_at, const int32_t *local_step)
{
    __shared__ float part[TW];
    float acc = 0.0f;
    for (int r = threadIdx.x; r < B; r += TW) {
        const float o0 = out[2 * r], o1 = out[2 * r + 1];
        const float t = fminf(fmaxf(o0, 0.5f), 0.9f), l = fminf(fmaxf(o1, 5.0f), 12.0f);
        const float u = (t - 0.5f) / 0.1f, v = l - 5.0f;
        const int i = min((int)floorf(u), GRID_TH - 2), j = min((int)floorf(v), GRID_NB - 2);
        const float fu = u - (float)i, fv = v - (float)j;
        const float *g = G + (int64_t)r * N_GRID;
        const float g00 = g[i * GRID_NB + j], g10 = g[(i + 1) * GRID_NB + j];
        const float g01 = g[i * GRID_NB + j + 1], g11 = g[(i + 1) * GRID_NB + j + 1];
        const float val = (1.0f - fu) * (1.0f - fv) * g00 + fu * (1.0f - fv) * g10 +
                          (1.0f - fu) * fv * g01 + fu * fv * g11;
        const float du = (1.0f - fv) * (g10 - g00) + fv * (g11 - g01);
        const float dv = (1.0f - fu) * (g01 - g00) + fu * (g11 - g10);
        const float d0 = o0 < 0.5f ? -1.0f : (o0 > 0.9f ? 1.0f : du / 0.1f);
        const float d1 = o1 < 5.0f ? -1.0f : (o1 > 12.0f ? 1.0f : dv);
        d_out[2 * r] = d0 / (float)B;
        d_out[2 * r + 1] = d1 / (float)B;
        acc += val + fabsf(o0 - t) + fabsf(o1 - l);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = TW / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float *dst = loss_at + (local_step ? *local_step : 0);
        *dst = part[0] / (float)B;
    }
}

// Scorer loss: out and G are [B][N_GRID] (estimates and measured log time
// ratios, theta outer); loss = sum w (out - G)^2 / (N_GRID B) with w =
// exp(-G / SCORE_TEMP) + SCORE_FLOOR (fixed-order tree), d_out = 2 w (out -
// G) / (N_GRID B).  One workgroup.
__global__ __launch_bounds__(TW) void k_score_loss_grad(const float *__restrict__ out,
                                                        const float *__restrict__ G, int B,
                                                        float *__restrict__ d_out,
                                                        float *loss_at, const int32_t *local_step)
{
    __shared__ float part[TW];
    const float norm = (float)(N_GRID * B);
    float acc = 0.0f;
    for (int idx = threadIdx.x; idx < B * N_GRID; idx += TW) {
        const float g = G[idx];
        const float w = expf(-g / SCORE_TEMP) + SCORE_FLOOR;
        const float d = out[idx] - g;
        d_out[idx] = 2.0f * w * d / norm;
        acc += w * d * d;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = TW / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float *dst = loss_at + (local_step ? *local_step : 0);
        *dst = part[0] / norm;
    }
}

// (theta, n_b) from each scorer output row: the grid point k of the
// smallest estimate (the first of equal ones), theta = 0.5 + 0.1 (k / 8),
// n_b = 2^(5 + k % 8); ok = 0 for a row with a non-finite estimate (then
// theta = 0.6, n_b = 256).
__global__ void k_decode_scores(const float *__restrict__ out, int B, double *theta, int32_t *nb,
                                int32_t *ok)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B)
        return;
    const float *o = out + (int64_t)r * N_GRID;
    bool fin = true;
    int k = 0;
    for (int i = 0; i < N_GRID; i++) {
        fin = fin && isfinite(o[i]);
        if (o[i] < o[k])
            k = i;
    }
    ok[r] = fin ? 1 : 0;
    const int i = fin ? k / GRID_NB : 1, j = fin ? k % GRID_NB : 3;
    theta[r] = (double)(5 + i) / 10.0;
    nb[r] = 1 << (5 + j);
}

// (theta, n_b) from each network output row: theta = round(10 clip(o0, .5,
// .9))/10 (the paper's theta grid, Sec. 6.4.1), n_b = 2^clip(round(o1), 5,
// 12); ok = 0 for non-finite outputs (then theta = 0.6, n_b = 256).
__global__ void k_decode(const float *__restrict__ out, int B, double *theta, int32_t *nb,
                         int32_t *ok)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B)
        return;
    const float o0 = out[2 * r], o1 = out[2 * r + 1];
    const bool fin = isfinite(o0) && isfinite(o1);
    ok[r] = fin ? 1 : 0;
    const double c = fin ? fmin(fmax((double)o0, 0.5), 0.9) : 0.6;
    theta[r] = rint(c * 10.0) / 10.0;
    const float l = fin ? fminf(fmaxf(rintf(o1), 5.0f), 12.0f) : 8.0f;
    nb[r] = 1 << (int)l;
}

// Most candidates mhdc_refine_candidates can return.
constexpr int32_t MAX_REFINE = 6;

// The byte model's verdict on a chosen handle against plain CSR: its V_CSR /
// V (Eq. 28), alpha, beta, and whether CSR moves fewer bytes -- exactly when
// 3 (nnz - R) < 2 S, i.e. alpha < 2/3 (Eqs. 31-32), decided in integers.
void set_verdict(mhdc_handle h, mhdc_select_result *res)
{
    mhdc_info inf{};
    if (mhdc_get_info(h, &inf) != MHDC_OK)
        return;
    res->rp_est = inf.rp_est;
    res->alpha = inf.alpha;
    res->beta = inf.beta;
    res->csr_cheaper = inf.S > 0 && 3 * (inf.nnz - inf.R) < 2 * inf.S ? 1 : 0;
}

// Hidden activations of the forward pass that allocates nothing
// (mhdc_mlp_forward_noalloc): two layers of at most NOALLOC_MAX_B rows of
// HID floats, 2 MB in all.  Each GPU the library runs on holds its own copy
// until the process ends.  Host code never passes this name to a kernel (on
// the host it is a stand-in, not a device address): it looks the address up
// per device with hipGetSymbolAddress and passes that.
constexpr int NOALLOC_MAX_B = 2048;
static __device__ __align__(256) float scratch[2 * NOALLOC_MAX_B * HID];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int noalloc_scratch(float **out)
{
    int dev = 0;
    MHDC_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(MHDC_ERR_HIP, std::string("scratch address lookup: ") +
                                               hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[dev];
    return MHDC_OK;
}

}  // namespace
}  // namespace mhdc

using namespace mhdc;

struct mhdc_mlp_s {
    int32_t n_out = N_OUT;  // 2 (theta, log2 n_b) or N_GRID (scorer)
    int32_t n_par = N_PARAMS;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    int32_t *step = nullptr, *local_step = nullptr;
    int32_t cap = 0;  // minibatch capacity of the buffers below
    float *Xb = nullptr, *Tb = nullptr, *h1 = nullptr, *h2 = nullptr, *out = nullptr;
    float *d_out = nullptr, *d_h2 = nullptr, *d_h1 = nullptr, *loss = nullptr;
};

namespace {

void free_buffers(mhdc_mlp_s *M)
{
    for (float *q : {M->Xb, M->Tb, M->h1, M->h2, M->out, M->d_out, M->d_h2, M->d_h1})
        dfree(q);
    M->Xb = M->Tb = M->h1 = M->h2 = M->out = M->d_out = M->d_h2 = M->d_h1 = nullptr;
    M->cap = 0;
}

int ensure_buffers(mhdc_mlp_s *M, int32_t B)
{
    if (B <= M->cap)
        return MHDC_OK;
    free_buffers(M);
    int rc;
    const size_t f = sizeof(float);
    if ((rc = dmalloc((void **)&M->Xb, f * B * N_IN, "mlp Xb")) ||
        (rc = dmalloc((void **)&M->Tb, f * B * N_GRID, "mlp Tb")) ||
        (rc = dmalloc((void **)&M->h1, f * B * HID, "mlp h1")) ||
        (rc = dmalloc((void **)&M->h2, f * B * HID, "mlp h2")) ||
        (rc = dmalloc((void **)&M->out, f * B * M->n_out, "mlp out")) ||
        (rc = dmalloc((void **)&M->d_out, f * B * M->n_out, "mlp d_out")) ||
        (rc = dmalloc((void **)&M->d_h2, f * B * HID, "mlp d_h2")) ||
        (rc = dmalloc((void **)&M->d_h1, f * B * HID, "mlp d_h1"))) {
        free_buffers(M);
        return rc;
    }
    M->cap = B;
    return MHDC_OK;
}

void enqueue_forward(mhdc_mlp_s *M, const float *X, int B, hipStream_t s)
{
    k_dense_fwd<<<blocks_for(B * HID), TW, 0, s>>>(X, N_IN, M->p + P_W1, M->p + P_B1, HID, M->h1, B, 1);
    k_dense_fwd<<<blocks_for(B * HID), TW, 0, s>>>(M->h1, HID, M->p + P_W2, M->p + P_B2, HID, M->h2, B, 1);
    k_dense_fwd<<<blocks_for(B * M->n_out), TW, 0, s>>>(M->h2, HID, M->p + P_W3, M->p + p_b3(M->n_out), M->n_out, M->out, B, 0);
}

void enqueue_backward(mhdc_mlp_s *M, const float *X, int B, hipStream_t s)
{
    const int no = M->n_out;
    k_dense_bwd_w<<<blocks_for(no * (HID + 1)), TW, 0, s>>>(M->d_out, M->h2, B, HID, no, M->g + P_W3, M->g + p_b3(no));
    k_dense_bwd_x<<<blocks_for(B * HID), TW, 0, s>>>(M->d_out, M->p + P_W3, M->h2, B, HID, no, M->d_h2);
    k_dense_bwd_w<<<blocks_for(HID * (HID + 1)), TW, 0, s>>>(M->d_h2, M->h1, B, HID, HID, M->g + P_W2, M->g + P_B2);
    k_dense_bwd_x<<<blocks_for(B * HID), TW, 0, s>>>(M->d_h2, M->p + P_W2, M->h1, B, HID, HID, M->d_h1);
    k_dense_bwd_w<<<blocks_for(HID * (N_IN + 1)), TW, 0, s>>>(M->d_h1, X, B, N_IN, HID, M->g + P_W1, M->g + P_B1);
}

int launch_ok(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return MHDC_OK;
}

}  // namespace

extern "C" {

int mhdc_features(int32_t n, const int32_t *rowptr, const int32_t *colind, const double *val,
                  float *feat, hipStream_t stream)
{
    clear_error();
    if (n < 1 || !feat)
        return set_error(MHDC_ERR_INVALID_ARG, "n >= 1 and a feature buffer are required");
    (void)hipStreamSynchronize(stream);
    int64_t nnz = 0;
    int rc = validate_csr(n, rowptr, colind, val, &nnz);
    if (rc)
        return rc;
    const int64_t n_blk = ((int64_t)n + PROBE_NB - 1) / PROBE_NB;
    unsigned long long *sums = nullptr;
    int32_t *gkeys = nullptr, *gcnts = nullptr;
    if ((rc = dmalloc((void **)&sums, sizeof(unsigned long long) * 2 * N_BINS, "feature sums")))
        return rc;
    // the census needs the global table only for blocks of >= 8192 entries;
    // find the largest block from a host copy of the row pointer
    int64_t maxm = 0;
    std::vector<int32_t> hrp((size_t)n + 1);
    hipError_t e = hipMemcpy(hrp.data(), rowptr, sizeof(int32_t) * ((size_t)n + 1),
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        dfree(sums);
        return set_error(MHDC_ERR_HIP, std::string("features: ") + hipGetErrorString(e));
    }
    for (int64_t ib = 0; ib < n_blk; ib++) {
        const int64_t r1 = std::min<int64_t>(n, (ib + 1) * PROBE_NB);
        maxm = std::max<int64_t>(maxm, hrp[r1] - hrp[ib * PROBE_NB]);
    }
    if (maxm >= CENSUS_LDS_SLOTS) {
        const size_t nz = (size_t)std::max<int64_t>(nnz, 1);
        if ((rc = dmalloc((void **)&gkeys, sizeof(int32_t) * 2 * nz, "feature table")) ||
            (rc = dmalloc((void **)&gcnts, sizeof(int32_t) * 2 * nz, "feature table"))) {
            dfree(sums);
            dfree(gkeys);
            return rc;
        }
    }
    (void)hipMemsetAsync(sums, 0, sizeof(unsigned long long) * 2 * N_BINS, stream);
    const unsigned grid = (unsigned)std::min<int64_t>(n_blk, 2048);
    k_feat_census<<<grid, CENSUS_WG, 0, stream>>>(n, n_blk, rowptr, colind, val, gkeys, gcnts,
                                                   sums);
    k_feat_finish<<<1, 128, 0, stream>>>(n, nnz, n_blk, sums, feat);
    rc = launch_ok("features");
    if (hipStreamSynchronize(stream) != hipSuccess && !rc)
        rc = set_error(MHDC_ERR_HIP, "features: synchronize failed");
    dfree(sums);
    dfree(gkeys);
    dfree(gcnts);
    return rc;
}

}  // extern "C"

namespace {

mhdc_mlp create_impl(const float *params_host, int32_t n_out)
{
    clear_error();
    if (!params_host) {
        set_error(MHDC_ERR_INVALID_ARG, "initial parameters are required");
        return nullptr;
    }
    mhdc_mlp_s *M = new (std::nothrow) mhdc_mlp_s;
    if (!M) {
        set_error(MHDC_ERR_OOM, "host allocation of the network failed");
        return nullptr;
    }
    M->n_out = n_out;
    M->n_par = n_params(n_out);
    const size_t pb = sizeof(float) * M->n_par;
    int rc;
    if ((rc = dmalloc((void **)&M->p, pb, "mlp params")) ||
        (rc = dmalloc((void **)&M->g, pb, "mlp grads")) ||
        (rc = dmalloc((void **)&M->m, pb, "mlp adam m")) ||
        (rc = dmalloc((void **)&M->v, pb, "mlp adam v")) ||
        (rc = dmalloc((void **)&M->step, 2 * sizeof(int32_t), "mlp step"))) {
        mhdc_mlp_destroy(M);
        return nullptr;
    }
    M->local_step = M->step + 1;
    if (hipMemcpy(M->p, params_host, pb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(M->g, 0, pb) != hipSuccess || hipMemset(M->m, 0, pb) != hipSuccess ||
        hipMemset(M->v, 0, pb) != hipSuccess ||
        hipMemset(M->step, 0, 2 * sizeof(int32_t)) != hipSuccess) {
        set_error(MHDC_ERR_HIP, "initialising the network failed");
        mhdc_mlp_destroy(M);
        return nullptr;
    }
    return M;
}

}  // namespace

extern "C" {

mhdc_mlp mhdc_mlp_create(const float *params_host) { return create_impl(params_host, N_OUT); }

mhdc_mlp mhdc_mlp_create_scorer(const float *params_host)
{
    return create_impl(params_host, N_GRID);
}

int32_t mhdc_mlp_outputs(mhdc_mlp M)
{
    clear_error();
    if (!M) {
        set_error(MHDC_ERR_INVALID_ARG, "network is NULL");
        return 0;
    }
    return M->n_out;
}

int mhdc_mlp_get_params(mhdc_mlp M, float *params_host)
{
    clear_error();
    if (!M || !params_host)
        return set_error(MHDC_ERR_INVALID_ARG, "network or buffer is NULL");
    MHDC_HIP_CHECK(hipDeviceSynchronize());
    MHDC_HIP_CHECK(hipMemcpy(params_host, M->p, sizeof(float) * M->n_par, hipMemcpyDeviceToHost));
    return MHDC_OK;
}

int mhdc_mlp_forward(mhdc_mlp M, const float *X, int32_t B, float *out, hipStream_t stream)
{
    clear_error();
    if (!M || !X || !out || B < 1)
        return set_error(MHDC_ERR_INVALID_ARG, "network, X, out and B >= 1 required");
    MHDC_HIP_CHECK(hipStreamSynchronize(stream));
    int rc = ensure_buffers(M, B);
    if (rc)
        return rc;
    enqueue_forward(M, X, B, stream);
    MHDC_HIP_CHECK(hipMemcpyAsync(out, M->out, sizeof(float) * B * M->n_out,
                                  hipMemcpyDeviceToDevice, stream));
    return launch_ok("mlp forward");
}

int mhdc_mlp_forward_noalloc(mhdc_mlp M, const float *X, int32_t B, float *out,
                             hipStream_t stream)
{
    clear_error();
    if (!M || !X || !out || B < 1)
        return set_error(MHDC_ERR_INVALID_ARG, "network, X, out and B >= 1 required");
    if (B > NOALLOC_MAX_B)
        return set_error(MHDC_ERR_SIZE,
                         "B exceeds 2048 rows, the scratch size of the allocation-free forward pass");
    float *s = nullptr;
    int rc = noalloc_scratch(&s);
    if (rc)
        return rc;
    float *h1 = s, *h2 = s + (size_t)NOALLOC_MAX_B * HID;
    // the kernels and their order are those of mhdc_mlp_forward, so the
    // outputs are the same bits; the last layer writes `out` directly
    k_dense_fwd<<<blocks_for(B * HID), TW, 0, stream>>>(X, N_IN, M->p + P_W1, M->p + P_B1, HID, h1, B, 1);
    k_dense_fwd<<<blocks_for(B * HID), TW, 0, stream>>>(h1, HID, M->p + P_W2, M->p + P_B2, HID, h2, B, 1);
    k_dense_fwd<<<blocks_for(B * M->n_out), TW, 0, stream>>>(h2, HID, M->p + P_W3, M->p + p_b3(M->n_out), M->n_out, out, B, 0);
    return launch_ok("mlp forward (no allocation)");
}

int mhdc_mlp_loss_grad(mhdc_mlp M, const float *X, const float *T, int32_t B, float w0,
                       float w1, float *loss, float *grad, hipStream_t stream)
{
    clear_error();
    if (!M || !X || !T || !loss || !grad || B < 1)
        return set_error(MHDC_ERR_INVALID_ARG, "network, X, T, loss, grad and B >= 1 required");
    if (M->n_out != N_OUT)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "the squared error to targets is for 2-output networks");
    MHDC_HIP_CHECK(hipStreamSynchronize(stream));
    int rc = ensure_buffers(M, B);
    if (rc)
        return rc;
    enqueue_forward(M, X, B, stream);
    k_loss_grad<<<1, TW, 0, stream>>>(M->out, T, B, w0, w1, M->d_out, loss, nullptr);
    enqueue_backward(M, X, B, stream);
    MHDC_HIP_CHECK(hipMemcpyAsync(grad, M->g, sizeof(float) * M->n_par, hipMemcpyDeviceToDevice,
                                  stream));
    return launch_ok("mlp loss/grad");
}

}  // extern "C"

namespace {

// Training shared by the losses: grid = false, T holds N_OUT target
// outputs per row and the loss is the weighted squared error; grid = true,
// T holds the N_GRID grid values per row and the loss is the grid loss (a
// 2-output network) or the scorer loss (a scorer).
int train_impl(mhdc_mlp M, const float *X, const float *T, int32_t N, const int32_t *order,
               int64_t steps, int32_t B, float lr, float w0, float w1, float *loss_hist,
               hipStream_t stream, bool grid)
{
    if (!M || !X || !T || !order || !loss_hist || N < 1 || B < 1 || steps < 1)
        return set_error(MHDC_ERR_INVALID_ARG, "bad training arguments");
    if (steps * (int64_t)B > INT32_MAX)
        return set_error(MHDC_ERR_SIZE, "steps * B exceeds the order index range");
    if (!grid && M->n_out != N_OUT)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "the squared error to targets is for 2-output networks");
    MHDC_HIP_CHECK(hipStreamSynchronize(stream));
    int rc = ensure_buffers(M, B);
    if (rc)
        return rc;
    {
        // every minibatch row index must name a row of X/T
        int32_t *bad = nullptr;
        if ((rc = dmalloc((void **)&bad, sizeof(int32_t), "order check flag")))
            return rc;
        const int64_t count = steps * (int64_t)B;
        k_zero_i32<<<1, 1, 0, stream>>>(bad);
        const int64_t blocks = (count + TW - 1) / TW;
        k_check_order<<<(unsigned)(blocks < 4096 ? blocks : 4096), TW, 0, stream>>>(order, count, N,
                                                                                   bad);
        int32_t h = 0;
        hipError_t e = hipMemcpyAsync(&h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(stream);
        dfree(bad);
        if (e != hipSuccess)
            return set_error(MHDC_ERR_HIP, std::string("mlp train: ") + hipGetErrorString(e));
        if (h)
            return set_error(MHDC_ERR_INVALID_ARG, "order holds a row index outside [0, N)");
    }
    // capture one step: gather, forward, loss, backward, Adam, counters
    hipStream_t cs = nullptr;
    MHDC_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    k_zero_i32<<<1, 1, 0, cs>>>(M->local_step);
    hipError_t e = hipStreamSynchronize(cs);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess)
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const int tdim = grid ? N_GRID : N_OUT;
        k_gather<<<blocks_for(B * (N_IN + tdim)), TW, 0, cs>>>(X, T, tdim, order, M->local_step, B,
                                                              M->Xb, M->Tb);
        enqueue_forward(M, M->Xb, B, cs);
        if (grid && M->n_out == N_GRID)
            k_score_loss_grad<<<1, TW, 0, cs>>>(M->out, M->Tb, B, M->d_out, loss_hist,
                                                M->local_step);
        else if (grid)
            k_grid_loss_grad<<<1, TW, 0, cs>>>(M->out, M->Tb, B, M->d_out, loss_hist,
                                               M->local_step);
        else
            k_loss_grad<<<1, TW, 0, cs>>>(M->out, M->Tb, B, w0, w1, M->d_out, loss_hist,
                                          M->local_step);
        enqueue_backward(M, M->Xb, B, cs);
        k_adam<<<blocks_for(M->n_par), TW, 0, cs>>>(M->p, M->g, M->m, M->v, M->n_par, lr, 0.9f, 0.999f, 1e-8f, M->step);
        k_steps_inc<<<1, 1, 0, cs>>>(M->step, M->local_step);
        e = hipStreamEndCapture(cs, &graph);
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) {
        for (int64_t t = 0; t < steps && e == hipSuccess; t++)
            e = hipGraphLaunch(exec, cs);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(cs);
    if (exec)
        (void)hipGraphExecDestroy(exec);
    if (graph)
        (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string("mlp train: ") + hipGetErrorString(e));
    return MHDC_OK;
}

}  // namespace

extern "C" {

int mhdc_mlp_train(mhdc_mlp M, const float *X, const float *T, int32_t N, const int32_t *order,
                   int64_t steps, int32_t B, float lr, float w0, float w1, float *loss_hist,
                   hipStream_t stream)
{
    clear_error();
    return train_impl(M, X, T, N, order, steps, B, lr, w0, w1, loss_hist, stream, false);
}

int mhdc_mlp_train_grid(mhdc_mlp M, const float *X, const float *G, int32_t N,
                        const int32_t *order, int64_t steps, int32_t B, float lr,
                        float *loss_hist, hipStream_t stream)
{
    clear_error();
    return train_impl(M, X, G, N, order, steps, B, lr, 0.0f, 0.0f, loss_hist, stream, true);
}

int mhdc_mlp_grid_loss_grad(mhdc_mlp M, const float *X, const float *G, int32_t B, float *loss,
                            float *grad, hipStream_t stream)
{
    clear_error();
    if (!M || !X || !G || !loss || !grad || B < 1)
        return set_error(MHDC_ERR_INVALID_ARG, "network, X, G, loss, grad and B >= 1 required");
    MHDC_HIP_CHECK(hipStreamSynchronize(stream));
    int rc = ensure_buffers(M, B);
    if (rc)
        return rc;
    enqueue_forward(M, X, B, stream);
    if (M->n_out == N_GRID)
        k_score_loss_grad<<<1, TW, 0, stream>>>(M->out, G, B, M->d_out, loss, nullptr);
    else
        k_grid_loss_grad<<<1, TW, 0, stream>>>(M->out, G, B, M->d_out, loss, nullptr);
    enqueue_backward(M, X, B, stream);
    MHDC_HIP_CHECK(hipMemcpyAsync(grad, M->g, sizeof(float) * M->n_par, hipMemcpyDeviceToDevice,
                                  stream));
    return launch_ok("mlp grid loss/grad");
}

int mhdc_mlp_decide(mhdc_mlp M, const float *X, int32_t B, double *theta, int32_t *n_b,
                    int32_t *ok, hipStream_t stream)
{
    clear_error();
    if (!M || !X || !theta || !n_b || !ok || B < 1)
        return set_error(MHDC_ERR_INVALID_ARG, "network, X, outputs and B >= 1 required");
    MHDC_HIP_CHECK(hipStreamSynchronize(stream));
    int rc = ensure_buffers(M, B);
    if (rc)
        return rc;
    enqueue_forward(M, X, B, stream);
    if (M->n_out == N_GRID)
        k_decode_scores<<<blocks_for(B), TW, 0, stream>>>(M->out, B, theta, n_b, ok);
    else
        k_decode<<<blocks_for(B), TW, 0, stream>>>(M->out, B, theta, n_b, ok);
    return launch_ok("mlp decide");
}

void mhdc_mlp_destroy(mhdc_mlp M)
{
    if (!M)
        return;
    free_buffers(M);
    dfree(M->p);
    dfree(M->g);
    dfree(M->m);
    dfree(M->v);
    dfree(M->step);
    delete M;
}

mhdc_handle mhdc_select(int32_t n, const int32_t *rowptr, const int32_t *colind,
                        const double *val, mhdc_mlp model, double tolerance,
                        mhdc_select_result *out)
{
    clear_error();
    const double rule_theta = 0.6;
    const int32_t rule_nb = 256;
    mhdc_select_result res{};
    res.theta = rule_theta;
    res.n_b = rule_nb;
    res.used_rule = 1;
    mhdc_handle net = nullptr;
    if (model) {
        float *feat = nullptr, *o = nullptr;
        double *th = nullptr;
        int32_t *nbok = nullptr;
        int rc = dmalloc((void **)&feat, sizeof(float) * N_IN, "select features");
        if (!rc)
            rc = dmalloc((void **)&o, sizeof(float) * model->n_out, "select out");
        if (!rc)
            rc = dmalloc((void **)&th, sizeof(double), "select theta");
        if (!rc)
            rc = dmalloc((void **)&nbok, 2 * sizeof(int32_t), "select nb");
        if (!rc)
            rc = mhdc_features(n, rowptr, colind, val, feat, 0);
        if (!rc)
            rc = mhdc_mlp_forward(model, feat, 1, o, 0);
        double h_th = 0.6;
        int32_t h_nbok[2] = {0, 0};
        if (!rc) {
            if (model->n_out == N_GRID)
                k_decode_scores<<<1, 1>>>(o, 1, th, nbok, nbok + 1);
            else
                k_decode<<<1, 1>>>(o, 1, th, nbok, nbok + 1);
            if (hipMemcpy(&h_th, th, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(h_nbok, nbok, sizeof(h_nbok), hipMemcpyDeviceToHost) != hipSuccess)
                rc = set_error(MHDC_ERR_HIP, "select: reading the decision failed");
        }
        dfree(feat);
        dfree(o);
        dfree(th);
        dfree(nbok);
        if (rc)
            return nullptr;
        res.theta_net = h_th;
        res.n_b_net = h_nbok[0];
        res.net_ok = h_nbok[1];
        if (res.net_ok) {
            net = mhdc_from_csr(n, rowptr, colind, val, res.n_b_net, res.theta_net);
            if (!net)
                return nullptr;
        }
    }
    mhdc_handle rule = mhdc_from_csr(n, rowptr, colind, val, rule_nb, rule_theta);
    if (!rule) {
        if (net)
            mhdc_destroy(net);
        return nullptr;
    }
    mhdc_info ir{}, in{};
    (void)mhdc_get_info(rule, &ir);
    res.bytes_rule = ir.bytes_paper;
    mhdc_handle pick = rule;
    if (net) {
        (void)mhdc_get_info(net, &in);
        res.bytes_net = in.bytes_paper;
        // the paper's byte model judges: keep the network's choice unless
        // it is predicted to move more than (1 + tolerance) x the policy's
        if (mhdc_judge_keep(in.bytes_paper, ir.bytes_paper, tolerance)) {
            pick = net;
            res.theta = res.theta_net;
            res.n_b = res.n_b_net;
            res.used_rule = 0;
        }
    }
    if (pick != rule)
        mhdc_destroy(rule);
    if (net && pick != net)
        mhdc_destroy(net);
    set_verdict(pick, &res);
    if (out)
        *out = res;
    return pick;
}

mhdc_handle mhdc_select_refine(int32_t n, const int32_t *rowptr, const int32_t *colind,
                               const double *val, mhdc_mlp model, double tolerance,
                               hipStream_t stream, mhdc_select_result *out)
{
    clear_error();
    mhdc_select_result res{};
    mhdc_handle best = mhdc_select(n, rowptr, colind, val, model, tolerance, &res);
    if (!best)
        return nullptr;
    if (n < 1) {
        if (out)
            *out = res;
        return best;
    }
    // the decision's neighbours on the grid of Sec. 6.4.1 (theta in 0.1
    // steps within [0.5, 0.9], n_b a power of two in [32, 4096]), the
    // policy and the largest block size
    struct Cand {
        double theta;
        int32_t n_b;
    };
    std::vector<Cand> cand;
    {
        double th[MAX_REFINE];
        int32_t nb[MAX_REFINE];
        const int32_t nc = mhdc_refine_candidates(res.theta, res.n_b, th, nb, MAX_REFINE);
        for (int32_t c = 0; c < nc; c++)
            cand.push_back({th[c], nb[c]});
    }
    double *x = nullptr, *y = nullptr;
    int rc = dmalloc((void **)&x, sizeof(double) * (size_t)n, "refine x");
    if (!rc)
        rc = dmalloc((void **)&y, sizeof(double) * (size_t)n, "refine y");
    if (!rc) {
        k_fill_half<<<blocks_for(n < (1 << 22) ? n : (1 << 22)), TW, 0, stream>>>(x, n);
        rc = launch_ok("refine fill");
    }
    float t_best = 0.0f;
    if (!rc)
        rc = mhdc_time_spmv(best, x, y, stream, &t_best);
    for (size_t c = 0; c < cand.size() && !rc; c++) {
        mhdc_handle h = mhdc_from_csr(n, rowptr, colind, val, cand[c].n_b, cand[c].theta);
        if (!h) {
            rc = mhdc_last_error();
            break;
        }
        float t = 0.0f;
        rc = mhdc_time_spmv(h, x, y, stream, &t);
        if (!rc && t < t_best) {
            mhdc_destroy(best);
            best = h;
            t_best = t;
            res.theta = cand[c].theta;
            res.n_b = cand[c].n_b;
            res.used_rule = std::fabs(cand[c].theta - 0.6) < 1e-9 && cand[c].n_b == 256;
        } else {
            mhdc_destroy(h);
        }
    }
    dfree(x);
    dfree(y);
    if (rc) {
        const std::string msg = mhdc_last_error_message();
        mhdc_destroy(best);
        set_error(rc, "select refine: " + msg);
        return nullptr;
    }
    set_verdict(best, &res);
    if (out)
        *out = res;
    return best;
}

int mhdc_judge_keep(double v_proposal, double v_policy, double tolerance)
{
    return v_proposal <= (1.0 + tolerance) * v_policy ? 1 : 0;
}

int32_t mhdc_refine_candidates(double theta, int32_t n_b, double *theta_out, int32_t *n_b_out,
                               int32_t cap)
{
    double th[MAX_REFINE];
    int32_t nb[MAX_REFINE];
    int32_t cnt = 0;
    auto add = [&](double t, int64_t b) {
        t = std::round(t * 10.0) / 10.0;
        if (t < 0.5 - 1e-9 || t > 0.9 + 1e-9 || b < 32 || b > 4096)
            return;
        if (std::fabs(t - theta) < 1e-9 && b == n_b)
            return;
        for (int32_t c = 0; c < cnt; c++)
            if (std::fabs(th[c] - t) < 1e-9 && nb[c] == b)
                return;
        th[cnt] = t;
        nb[cnt] = (int32_t)b;
        cnt++;
    };
    add(theta, n_b / 2);
    add(theta, (int64_t)n_b * 2);
    add(theta - 0.1, n_b);
    add(theta + 0.1, n_b);
    add(0.6, 256);
    // the largest block of the grid: on matrices of a few 1e5 rows (10-30 us
    // products) the fewest, longest segments often win by 5-20 %, far from
    // the network's choice
    add(theta, 4096);
    for (int32_t c = 0; c < cnt && c < cap; c++) {
        if (theta_out)
            theta_out[c] = th[c];
        if (n_b_out)
            n_b_out[c] = nb[c];
    }
    return cnt;
}

}  // extern "C"
