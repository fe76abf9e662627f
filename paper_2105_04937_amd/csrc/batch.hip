// batch.hip -- many M-HDC / HDC / CSR products in one persistent launch.
//
// A batch holds up to thousands of (matrix, right-hand-side block) items of
// uneven sizes.  The tiles of all items are dealt to the XCDs item by item;
// a persistent grid sized to the machine (CUs x resident workgroups) takes
// tiles from per-XCD atomic counters until every XCD's list is exhausted, so
// small matrices never leave CUs idle the way one launch per matrix does.
// Each tile writes only its own rows (no floating-point atomics): the result
// of every item is bit-identical to its single-matrix launch.
//
// The counters are cleared by a one-wavefront kernel launched just before
// the persistent kernel (no memset node, so the pair can be captured in a
// HIP graph and replayed).  Descriptors live in device memory, so rebinding X/Y
// pointers takes effect in later replays without re-capture.
#include "internal.h"
#include "spmv_tile.h"
#include "spmv_tile_rm.h"

#include <algorithm>
#include <new>
#include <vector>

namespace mhdc {
namespace {

struct BatchItem {
    SpmvArgs a;
    int64_t tile_begin;  // first global tile number of this item
    int32_t kc;          // accumulator width class (1, 2, 4, 8, 16)
    int32_t rg;          // CSR part: stage values/columns (1) or products (0)
    int32_t user;        // the item's index in the caller's arrays
};

// LDS bytes of the CSR-part variants batch_tile() can run at this width.
template <int WG, int KC>
constexpr int lds_of()
{
    return KC > 1 ? TileShape<WG, KC, true>::LDS_BYTES
                  : std::max(TileShape<WG, KC, false>::LDS_BYTES, TileShape<WG, KC, true>::LDS_BYTES);
}

// Right-hand sides per pass over a tile in the persistent kernel (larger
// items take several passes).  One pass of up to 16 measured faster than
// passes of 4 despite the larger register budget: every further pass reads
// the tile's share of A again.
constexpr int BATCH_MAX_KC = 16;

template <int WG>
constexpr int batch_lds_doubles()
{
    int m = 8;
    m = std::max(m, lds_of<WG, 1>());
    m = std::max(m, lds_of<WG, 2>());
    m = std::max(m, lds_of<WG, 4>());
    m = std::max(m, lds_of<WG, 8>());
    m = std::max(m, lds_of<WG, 16>());
    return (m + 7) / 8;
}

// One right-hand side: either CSR-part variant; several: values/columns
// staged (the product variant's LDS grows with the number of columns).
template <int WG, int KC>
__device__ inline void batch_tile(const BatchItem &it, int64_t local, double *lds)
{
    if constexpr (KC > 1) {
        spmv_tile<WG, 1, KC, true, true, true, 1>(it.a, local, lds);
    } else {
        if (it.rg)
            spmv_tile<WG, 1, KC, true, true, true>(it.a, local, lds);
        else
            spmv_tile<WG, 1, KC, true, true, false>(it.a, local, lds);
    }
}

// Row-major right-hand sides: the row-slot tile routine at the item's width.
template <int WG, int KC>
__device__ inline void batch_tile_rm(const BatchItem &it, int64_t local, double *lds)
{
    if (it.rg)
        spmv_tile_rm<WG, KC, true, true, true>(it.a, local, lds);
    else
        spmv_tile_rm<WG, KC, true, true, false>(it.a, local, lds);
}

// Every item's tiles go to one XCD: the items are dealt to the 8 XCDs,
// largest algorithmic bytes first, each to the XCD with the least so far
// (the host's schedule, below), so the tiles that share an item's x rows --
// its neighbours through the near diagonals and the planes its far
// diagonals reach -- are processed under one L2.  The schedule lists each
// XCD's tiles as (item slot << 32 | local tile) in a device array after the
// XCDs' start indices; each XCD has a tile counter of its own
// (BATCH_CTR_STRIDE ints apart).  Persistent workgroup w runs on XCD w mod 8
// (a launch's workgroups are dispatched to the XCDs in turn) and takes its
// XCD's entries in order; a workgroup whose XCD has run out takes the next
// XCD's, until all eight have run out.  Reading the entry also names the
// item, so no search over the items is needed.
constexpr int BATCH_XCDS = 8, BATCH_CTR_STRIDE = 32;
// schedule layout: starts[0..8] at [0, 9), entries from index SCHED_HEAD
constexpr int SCHED_HEAD = 16;

__global__ void k_batch_reset(int32_t *counter)
{
    if (threadIdx.x < BATCH_XCDS)
        counter[threadIdx.x * BATCH_CTR_STRIDE] = 0;
}

// Next schedule entry for this workgroup (uniform), or -1 when every XCD has
// run out.  *x is the XCD whose entries the workgroup is taking; x0 its own;
// s_start holds the XCDs' start indices.  Each counter only grows, and a
// workgroup moves past an XCD at its first exhausted answer, so every
// workgroup reaches -1.
__device__ inline int64_t batch_take(int32_t *counter, const int64_t *__restrict__ sched,
                                     const int64_t *s_start, int x0, int *x, int64_t *s_tile)
{
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t i = s_start[*x] + atomicAdd(&counter[*x * BATCH_CTR_STRIDE], 1);
            *s_tile = i < s_start[*x + 1] ? sched[SCHED_HEAD + i] : -1;
        }
        __syncthreads();
        const int64_t e = *s_tile;
        __syncthreads();
        if (e >= 0)
            return e;
        *x = (*x + 1) & (BATCH_XCDS - 1);
        if (*x == x0)
            return -1;
    }
}

// The XCDs' start indices of the schedule, staged in LDS once per workgroup.
__device__ inline void batch_load_starts(const int64_t *__restrict__ sched, int64_t *s_start)
{
    if (threadIdx.x <= BATCH_XCDS)
        s_start[threadIdx.x] = sched[threadIdx.x];
    __syncthreads();
}

// Four waves per SIMD (at most 128 VGPRs): uncapped, the compiler took 132
// and the machine held three 256-lane workgroups per CU, which measured 6%
// slower on a 64-matrix batch.
template <int WG>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_batch(const BatchItem *__restrict__ items,
                                              const int64_t *__restrict__ sched, int32_t *counter)
{
    __shared__ double s_prod[batch_lds_doubles<WG>()];
    __shared__ int64_t s_tile;
    __shared__ int64_t s_start[BATCH_XCDS + 1];
    batch_load_starts(sched, s_start);
    const int x0 = blockIdx.x & (BATCH_XCDS - 1);
    int x = x0;
    for (;;) {
        const int64_t e = batch_take(counter, sched, s_start, x0, &x, &s_tile);
        if (e < 0)
            break;
        const BatchItem &it = items[e >> 32];
        const int64_t local = e & 0xffffffffLL;
        switch (it.kc) {
        case 1: batch_tile<WG, 1>(it, local, s_prod); break;
        case 2: batch_tile<WG, 2>(it, local, s_prod); break;
        case 4: batch_tile<WG, 4>(it, local, s_prod); break;
        case 8: batch_tile<WG, 8>(it, local, s_prod); break;
        default: batch_tile<WG, 16>(it, local, s_prod); break;
        }
    }
}

// The persistent loop for a batch whose right-hand sides are stored row by
// row.  Kernels of their own: the tile routine keeps KC/2 rows per lane in
// registers and would not fit the column-major kernel's register cap.
template <int WG>
__device__ inline void batch_rm_loop(const BatchItem *__restrict__ items,
                                     const int64_t *__restrict__ sched, int32_t *counter)
{
    __shared__ double s_prod[(TileShapeRm<WG, 2>::LDS_BYTES + 7) / 8];
    static_assert(TileShapeRm<WG, 2>::LDS_BYTES == TileShapeRm<WG, 16>::LDS_BYTES,
                  "one LDS size for every width");
    __shared__ int64_t s_tile;
    __shared__ int64_t s_start[BATCH_XCDS + 1];
    batch_load_starts(sched, s_start);
    const int x0 = blockIdx.x & (BATCH_XCDS - 1);
    int x = x0;
    for (;;) {
        const int64_t e = batch_take(counter, sched, s_start, x0, &x, &s_tile);
        if (e < 0)
            break;
        const BatchItem &it = items[e >> 32];
        const int64_t local = e & 0xffffffffLL;
        switch (it.kc) {
        case 2: batch_tile_rm<WG, 2>(it, local, s_prod); break;
        case 4: batch_tile_rm<WG, 4>(it, local, s_prod); break;
        case 8: batch_tile_rm<WG, 8>(it, local, s_prod); break;
        default: batch_tile_rm<WG, 16>(it, local, s_prod); break;
        }
    }
}

// 64 lanes: one wave per SIMD (LDS-bound).
__global__ __launch_bounds__(64) void k_batch_rm64(const BatchItem *__restrict__ items,
                                                   const int64_t *__restrict__ sched,
                                                   int32_t *counter)
{
    batch_rm_loop<64>(items, sched, counter);
}

// 256 lanes: held to three waves per SIMD (at most 168 VGPRs, no spills;
// uncapped the compiler took 170 and only two fitted).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_batch_rm256(
    const BatchItem *__restrict__ items, const int64_t *__restrict__ sched, int32_t *counter)
{
    batch_rm_loop<256>(items, sched, counter);
}

}  // namespace
}  // namespace mhdc

using namespace mhdc;

struct mhdc_batch_s {
    int32_t count = 0;
    int32_t wg = 256;
    int64_t total_tiles = 0;
    int32_t grid = 0;
    std::vector<const BdcMatrix *> mats;
    std::vector<int32_t> nrhs;
    std::vector<BatchItem> host_items;
    BatchItem *d_items = nullptr;
    int32_t *d_counter = nullptr;
    int64_t *d_sched = nullptr;  // XCD starts, then (slot << 32 | local tile) entries
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double flops = 0, bytes_alg = 0;
    int32_t rowmajor = 0;  // right-hand sides stored row by row
};

namespace {

const void *batch_kernel(int wg, int rowmajor)
{
    if (rowmajor)
        return wg == 64 ? reinterpret_cast<const void *>(k_batch_rm64)
                        : reinterpret_cast<const void *>(k_batch_rm256);
    return wg == 64 ? reinterpret_cast<const void *>(k_batch<64>)
                    : reinterpret_cast<const void *>(k_batch<256>);
}

int batch_grid(int wg, int rowmajor, int64_t total_tiles, int32_t *grid)
{
    int dev = 0, cus = 0, per_cu = 0;
    MHDC_HIP_CHECK(hipGetDevice(&dev));
    MHDC_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MHDC_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, batch_kernel(wg, rowmajor), wg, 0));
    int64_t g = (int64_t)cus * std::max(per_cu, 1);
    if (g > total_tiles)
        g = total_tiles;
    *grid = (int32_t)std::max<int64_t>(g, 1);
    return MHDC_OK;
}

// Largest tile count of a batch: a per-XCD int32 counter runs past its
// XCD's last tile by up to one increment per persistent workgroup (at most
// 256 CUs x 32 resident workgroups).
constexpr int64_t BATCH_MAX_TILES = (int64_t)INT32_MAX - (1LL << 20);

void drop_graph(mhdc_batch_s *b);

// The XCD schedule (see batch_take): items dealt to the XCDs by descending
// work (algorithmic bytes), each to the least-loaded XCD (the first on
// ties); each XCD's entries list its items' tiles in slot order.
void build_schedule(const std::vector<int64_t> &tiles_of, const std::vector<double> &work,
                    std::vector<int64_t> *sched)
{
    const int32_t count = (int32_t)tiles_of.size();
    std::vector<int32_t> by_work(count);
    for (int32_t i = 0; i < count; i++)
        by_work[i] = i;
    std::stable_sort(by_work.begin(), by_work.end(),
                     [&](int32_t a, int32_t c) { return work[a] > work[c]; });
    std::vector<int32_t> xcd_of(count, 0);
    double load[BATCH_XCDS] = {};
    for (int32_t slot : by_work) {
        int x = 0;
        for (int y = 1; y < BATCH_XCDS; y++)
            if (load[y] < load[x])
                x = y;
        xcd_of[slot] = x;
        load[x] += work[slot];
    }
    int64_t total = 0;
    for (int64_t t : tiles_of)
        total += t;
    sched->assign((size_t)(SCHED_HEAD + total), 0);
    int64_t pos = 0;
    for (int x = 0; x < BATCH_XCDS; x++) {
        (*sched)[x] = pos;
        for (int32_t slot = 0; slot < count; slot++)
            if (xcd_of[slot] == x)
                for (int64_t l = 0; l < tiles_of[slot]; l++)
                    (*sched)[SCHED_HEAD + pos++] = ((int64_t)slot << 32) | l;
    }
    (*sched)[BATCH_XCDS] = pos;
}

// Build the descriptor table for an X/Y binding and workgroup size, upload
// it, and only then take it over into the batch: a failure leaves the batch
// with its previous binding, workgroup size and grid, still runnable.  The
// XCD schedule depends on the workgroup size only (the items' tiles and
// bytes): it is rebuilt into a new buffer when that changes, and kept
// otherwise.
int upload_items(mhdc_batch_s *b, int32_t wg, const double *const *X, const int64_t *ldx,
                 double *const *Y, const int64_t *ldy)
{
    // Tiles are numbered item by item, the items with the most right-hand
    // sides first (then the longest): the persistent grid then ends on the
    // cheapest tiles, which shortens the tail where workgroups run out of
    // work.  Each item still writes only its own Y.
    std::vector<int32_t> order(b->count);
    for (int32_t i = 0; i < b->count; i++)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        if (b->nrhs[x] != b->nrhs[y])
            return b->nrhs[x] > b->nrhs[y];
        return b->mats[x]->n > b->mats[y]->n;
    });
    std::vector<BatchItem> items(b->count, BatchItem{});
    std::vector<int64_t> tiles_of(b->count);
    std::vector<double> work(b->count);
    int64_t tiles = 0;
    double flops = 0, bytes = 0;
    for (int32_t slot = 0; slot < b->count; slot++) {
        const int32_t i = order[slot];
        const BdcMatrix &m = *b->mats[i];
        const int32_t k = b->nrhs[i];
        const int64_t dflt = b->rowmajor ? k : m.n;
        const int64_t lx = ldx ? ldx[i] : dflt, ly = ldy ? ldy[i] : dflt;
        int rc = b->rowmajor ? check_operands_rm(m, X[i], lx, Y[i], ly, k)
                             : check_operands(m, X[i], lx, Y[i], ly, k);
        if (rc)
            return rc;
        BatchItem &it = items[slot];
        it.user = i;
        it.a = make_args(m, X[i], lx, Y[i], ly, k, 1);
        it.kc = b->rowmajor ? rm_columns(k) : kc_for(k < BATCH_MAX_KC ? k : BATCH_MAX_KC);
        it.rg = (b->rowmajor ? rm_row_gather(m, it.kc) : row_gather(m.launch.csr_mode, it.kc)) ? 1 : 0;
        it.a.pairs = b->rowmajor && rm_pairs(X[i], lx, Y[i], ly) ? 1 : 0;
        it.tile_begin = tiles;
        tiles_of[slot] = ((int64_t)m.n + wg - 1) / wg;
        tiles += tiles_of[slot];
        flops += 2.0 * (double)m.nnz * k;
        work[slot] = format_bytes(m) + 16.0 * (double)m.n * k;
        bytes += work[slot];
    }
    if (tiles > BATCH_MAX_TILES)
        return set_error(MHDC_ERR_SIZE, "too many tiles in the batch");
    int32_t grid = 0;
    int rc = batch_grid(wg, b->rowmajor, tiles, &grid);
    if (rc)
        return rc;
    int64_t *nd = nullptr;
    if (!(b->d_sched && wg == b->wg && tiles == b->total_tiles)) {
        std::vector<int64_t> sched;
        build_schedule(tiles_of, work, &sched);
        if ((rc = dmalloc((void **)&nd, sizeof(int64_t) * sched.size(), "batch schedule")))
            return rc;
        if (hipMemcpy(nd, sched.data(), sizeof(int64_t) * sched.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
            dfree(nd);
            return set_error(MHDC_ERR_HIP, "batch schedule upload failed");
        }
    }
    if (hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * b->count,
                  hipMemcpyHostToDevice) != hipSuccess) {
        dfree(nd);
        return set_error(MHDC_ERR_HIP, "batch descriptor upload failed");
    }
    if (nd) {
        // a captured graph holds the old schedule's address
        drop_graph(b);
        dfree(b->d_sched);
        b->d_sched = nd;
    }
    b->host_items.swap(items);
    b->wg = wg;
    b->total_tiles = tiles;
    b->grid = grid;
    b->flops = flops;
    b->bytes_alg = bytes;
    return MHDC_OK;
}

int enqueue(mhdc_batch_s *b, hipStream_t s)
{
    if (b->total_tiles == 0)
        return MHDC_OK;
    k_batch_reset<<<1, 64, 0, s>>>(b->d_counter);
    if (b->rowmajor && b->wg == 64)
        k_batch_rm64<<<b->grid, 64, 0, s>>>(b->d_items, b->d_sched, b->d_counter);
    else if (b->rowmajor)
        k_batch_rm256<<<b->grid, 256, 0, s>>>(b->d_items, b->d_sched, b->d_counter);
    else if (b->wg == 64)
        k_batch<64><<<b->grid, 64, 0, s>>>(b->d_items, b->d_sched, b->d_counter);
    else
        k_batch<256><<<b->grid, 256, 0, s>>>(b->d_items, b->d_sched, b->d_counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(MHDC_ERR_HIP, std::string("batch launch: ") + hipGetErrorString(e));
    return MHDC_OK;
}

mhdc_batch batch_create(int32_t count, const mhdc_handle *mats, const int32_t *nrhs,
                        const double *const *X, const int64_t *ldx, double *const *Y,
                        const int64_t *ldy, int32_t wg_size, int32_t rowmajor);

}  // namespace

namespace {

void drop_graph(mhdc_batch_s *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace

extern "C" {

mhdc_batch mhdc_batch_create(int32_t count, const mhdc_handle *mats, const int32_t *nrhs,
                             const double *const *X, const int64_t *ldx, double *const *Y,
                             const int64_t *ldy, int32_t wg_size)
{
    return batch_create(count, mats, nrhs, X, ldx, Y, ldy, wg_size, 0);
}

mhdc_batch mhdc_batch_create_rowmajor(int32_t count, const mhdc_handle *mats,
                                      const int32_t *nrhs, const double *const *X,
                                      const int64_t *ldx, double *const *Y, const int64_t *ldy,
                                      int32_t wg_size)
{
    return batch_create(count, mats, nrhs, X, ldx, Y, ldy, wg_size, 1);
}

}  // extern "C"

namespace {

mhdc_batch batch_create(int32_t count, const mhdc_handle *mats, const int32_t *nrhs,
                        const double *const *X, const int64_t *ldx, double *const *Y,
                        const int64_t *ldy, int32_t wg_size, int32_t rowmajor)
{
    clear_error();
    if (count < 1 || !mats || !nrhs || !X || !Y) {
        set_error(MHDC_ERR_INVALID_ARG, "count >= 1 and non-NULL mats, nrhs, X, Y required");
        return nullptr;
    }
    if (wg_size != 64 && wg_size != 256) {
        set_error(MHDC_ERR_NOT_SUPPORTED, "wg_size must be 64 or 256");
        return nullptr;
    }
    mhdc_batch_s *b = new (std::nothrow) mhdc_batch_s;
    if (!b) {
        set_error(MHDC_ERR_OOM, "host allocation of the batch failed");
        return nullptr;
    }
    b->count = count;
    b->wg = wg_size;
    b->rowmajor = rowmajor;
    for (int32_t i = 0; i < count; i++) {
        if (!mats[i] || nrhs[i] < 1 || nrhs[i] > 16) {
            set_error(MHDC_ERR_INVALID_ARG, "matrix handle NULL or nrhs outside [1, 16]");
            delete b;
            return nullptr;
        }
        b->mats.push_back(&mats[i]->m);
        b->nrhs.push_back(nrhs[i]);
    }
    int rc = dmalloc((void **)&b->d_items, sizeof(BatchItem) * (size_t)count, "batch items");
    if (!rc)
        rc = dmalloc((void **)&b->d_counter, sizeof(int32_t) * BATCH_XCDS * BATCH_CTR_STRIDE,
                     "batch counters");
    if (!rc)
        rc = upload_items(b, wg_size, X, ldx, Y, ldy);
    if (rc) {
        dfree(b->d_items);
        dfree(b->d_counter);
        dfree(b->d_sched);
        delete b;
        return nullptr;
    }
    return b;
}

}  // namespace

extern "C" {

int mhdc_batch_bind(mhdc_batch b, const double *const *X, const int64_t *ldx, double *const *Y,
                    const int64_t *ldy)
{
    clear_error();
    if (!b || !X || !Y)
        return set_error(MHDC_ERR_INVALID_ARG, "batch, X and Y must be non-NULL");
    MHDC_HIP_CHECK(hipDeviceSynchronize());  // replays in flight read the table
    const int32_t grid0 = b->grid;
    int rc = upload_items(b, b->wg, X, ldx, Y, ldy);
    if (!rc && b->grid != grid0)
        drop_graph(b);
    return rc;
}

int mhdc_batch_run(mhdc_batch b, hipStream_t stream)
{
    clear_error();
    if (!b)
        return set_error(MHDC_ERR_INVALID_ARG, "batch is NULL");
    return enqueue(b, stream);
}

int mhdc_batch_graph_launch(mhdc_batch b, hipStream_t stream)
{
    clear_error();
    if (!b)
        return set_error(MHDC_ERR_INVALID_ARG, "batch is NULL");
    if (!b->exec) {
        hipStream_t cs = nullptr;
        MHDC_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        int rc = e == hipSuccess ? enqueue(b, cs)
                                 : set_error(MHDC_ERR_HIP, std::string("begin capture: ") +
                                                               hipGetErrorString(e));
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (rc)
            return rc;
        if (e2 != hipSuccess)
            return set_error(MHDC_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e2));
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(b);
            return set_error(MHDC_ERR_HIP, std::string("graph instantiate: ") +
                                               hipGetErrorString(e));
        }
    }
    MHDC_HIP_CHECK(hipGraphLaunch(b->exec, stream));
    return MHDC_OK;
}

int mhdc_batch_set_wg(mhdc_batch b, int32_t wg_size)
{
    clear_error();
    if (!b)
        return set_error(MHDC_ERR_INVALID_ARG, "batch is NULL");
    if (wg_size != 64 && wg_size != 256)
        return set_error(MHDC_ERR_NOT_SUPPORTED, "wg_size must be 64 or 256");
    if (wg_size == b->wg)
        return MHDC_OK;
    MHDC_HIP_CHECK(hipDeviceSynchronize());
    std::vector<const double *> X(b->count);
    std::vector<double *> Y(b->count);
    std::vector<int64_t> lx(b->count), ly(b->count);
    for (const BatchItem &it : b->host_items) {
        X[it.user] = it.a.X;
        Y[it.user] = it.a.Y;
        lx[it.user] = it.a.ldx;
        ly[it.user] = it.a.ldy;
    }
    int rc = upload_items(b, wg_size, X.data(), lx.data(), Y.data(), ly.data());
    if (!rc)
        drop_graph(b);
    return rc;
}

int mhdc_batch_get_info(mhdc_batch b, mhdc_batch_info *out)
{
    clear_error();
    if (!b || !out)
        return set_error(MHDC_ERR_INVALID_ARG, "batch or out is NULL");
    out->count = b->count;
    out->wg_size = b->wg;
    out->total_tiles = b->total_tiles;
    out->grid = b->grid;
    out->flops = b->flops;
    out->bytes_alg = b->bytes_alg;
    return MHDC_OK;
}

void mhdc_batch_destroy(mhdc_batch b)
{
    if (!b)
        return;
    drop_graph(b);
    dfree(b->d_items);
    dfree(b->d_counter);
    dfree(b->d_sched);
    delete b;
}

}  // extern "C"
