// batched.hip -- many parameter sets in one persistent launch (the paper runs one work item per
// parameter set concurrently, Sec. 2; here a set is an ensemble of trajectories).
//
// The parameter, trajectory-count, step-count and window tables are device arrays, and the call
// only enqueues kernels, so a whole sweep can be captured into a graph and replayed. The plan is
// built on the device, in stream order:
//   1. k_batch_prepare  (one thread per set): check the set's values, compute its FP32 constants,
//                       tile and work-item counts; a bad set raises the status word;
//   2. k_batch_rank     (one thread per set): the set's place in longest-first order (more steps
//                       first, equal step counts in index order);
//   3. k_batch_scan     (one block): tile offsets in set order, work-item offsets in rank order,
//                       totals, the capacity check, the queue head and the item count;
//   4. k_batch_items    (one thread per set): the set's work items at its offset.
// Then a grid sized to the device's residency runs waves that each take the next item from an
// atomic counter until the list is empty. Every item starts from the set's initial condition
// (Philox domain 1), integrates to the set's window start, snapshots the position, integrates to
// the end and leaves per-tile FP64 partials in the set's slots; one block per set then adds the
// tiles in order. A set therefore gives the same bits as abp_integrate with set_id = its index,
// id0 = 0, and a window of the same length (the constants come from the same make_coef). When the
// status word is raised, the integration does nothing and the finalize writes NaN and zero counts.
//
// Workspace layout (abp_batched_workspace_bytes; cap = tiles the workspace holds):
//   SetRow rows[n_sets] | u32 order[n_sets] | i64 item_off[n_sets] | Ctl | u32 hist[n_sets][n_bins]
//   | Item items[cap] | double part[cap][2]
#include <algorithm>

#include "reduce.hpp"

namespace abp {

struct SetRow {
    Coef k;
    uint32_t pad;
    int64_t n_steps;
    int64_t win_begin;
    int64_t n_traj;
    int64_t first_tile;  // offset of the set's tiles in the partial array
};

struct Item {
    uint32_t set;
    uint32_t tile0;  // first local tile of the item
};

// Control words of one call, cleared by the host-side enqueue before the plan runs.
struct Ctl {
    uint32_t head;     // next work item
    int32_t status;    // ABP_OK, or the error the plan found (max over the codes raised)
    uint32_t n_items;  // items in the list
    uint32_t pad;
};

struct BatchArgs {
    const SetRow *rows;
    const Item *items;
    Ctl *ctl;
    double *part;
    uint32_t *hist;
    int32_t n_bins;
    uint32_t k0, k1;  // Philox key
};

struct BatchLayout {
    size_t rows, order, item_off, ctl, hist, items, part, total;
};

inline BatchLayout batch_layout(int32_t n_sets, int64_t cap, int32_t n_bins)
{
    BatchLayout L;
    L.rows = 0;
    L.order = align_up(L.rows + sizeof(SetRow) * (size_t)n_sets, 256);
    L.item_off = align_up(L.order + sizeof(uint32_t) * (size_t)n_sets, 256);
    L.ctl = align_up(L.item_off + sizeof(int64_t) * (size_t)n_sets, 256);
    L.hist = align_up(L.ctl + sizeof(Ctl), 256);
    L.items = align_up(L.hist + sizeof(uint32_t) * (size_t)n_sets * (size_t)n_bins, 256);
    L.part = align_up(L.items + sizeof(Item) * (size_t)cap, 256);
    L.total = align_up(L.part + 2 * sizeof(double) * (size_t)cap, 256);
    return L;
}

// Tiles of one sweep: item and tile indices, and the queue head (which passes the item count by at
// most the number of waves), stay within 32 bits.
constexpr int64_t kMaxTiles = 0x7FFFFFFFll;

// Tiles a workspace of ws_bytes holds for n_sets sets and n_bins bins (-1 if not even the
// per-set part fits): the largest cap with batch_layout(n_sets, cap, n_bins).total <= ws_bytes.
inline int64_t batch_capacity(int32_t n_sets, int32_t n_bins, size_t ws_bytes)
{
    const size_t fixed = batch_layout(n_sets, 0, n_bins).total;
    if (ws_bytes < fixed)
        return -1;
    const size_t per_tile = sizeof(Item) + 2 * sizeof(double);
    int64_t lo = (int64_t)((ws_bytes - fixed) / per_tile);  // an upper bound; step down to fit
    while (lo > 0 && batch_layout(n_sets, lo, n_bins).total > ws_bytes)
        --lo;
    return std::min<int64_t>(lo, kMaxTiles);
}

// The checks abp_integrate applies to a single set, for set k of the tables.
__device__ __forceinline__ int32_t set_status(const abp_params &p, int32_t n_traj, int64_t S,
                                              int64_t W, double dt)
{
    if (!params_ok(p) || !coef_ok(make_coef(p, dt)))
        return ABP_E_ARG;
    if (n_traj < 1 || S < 1 || S > kMaxStepIndex || W < 1 || W > S)
        return ABP_E_ARG;
    return ABP_OK;
}

__global__ __launch_bounds__(256) void k_batch_prepare(int32_t n_sets, const abp_params *params,
                                                       const int32_t *ntraj, const int64_t *nsteps,
                                                       const int64_t *window, double dt,
                                                       SetRow *rows, Ctl *ctl)
{
    const int32_t k = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n_sets)
        return;
    const abp_params p = params[k];
    const int64_t S = nsteps[k];
    const int64_t W = window ? window[k] : S / 2;
    const int32_t st = set_status(p, ntraj[k], S, W, dt);
    if (st != ABP_OK)
        atomicMax(&ctl->status, st);
    SetRow r;
    r.k = make_coef(p, dt);
    r.pad = 0;
    r.n_steps = S;
    r.win_begin = S - W;
    r.n_traj = ntraj[k];
    r.first_tile = 0;  // k_batch_scan
    rows[k] = r;
}

// order[rank] = set, rank = #{j : S_j > S_k} + #{j < k : S_j == S_k}, with the step counts
// staged through LDS 256 at a time.
__global__ __launch_bounds__(256) void k_batch_rank(int32_t n_sets, const SetRow *rows,
                                                    uint32_t *order)
{
    __shared__ int64_t tile[256];
    const int32_t k = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    const int64_t Sk = k < n_sets ? rows[k].n_steps : 0;
    uint32_t rank = 0;
    for (int32_t j0 = 0; j0 < n_sets; j0 += 256) {
        __syncthreads();
        if (j0 + (int32_t)threadIdx.x < n_sets)
            tile[threadIdx.x] = rows[j0 + threadIdx.x].n_steps;
        __syncthreads();
        const int32_t m = std::min(256, n_sets - j0);
        for (int32_t t = 0; t < m; ++t) {
            const int64_t Sj = tile[t];
            rank += (Sj > Sk) | ((Sj == Sk) & (j0 + t < k));
        }
    }
    if (k < n_sets)
        order[rank] = (uint32_t)k;
}

constexpr int kScanThreads = 1024;

// Exclusive prefix sum of one value per thread over a kScanThreads block (fixed order); returns
// the thread's offset and leaves the block total in `total`.
__device__ __forceinline__ int64_t block_scan(int64_t x, int64_t &total)
{
    __shared__ int64_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += y;
    }
    if (lane == 63)
        wsum[w] = incl;
    __syncthreads();
    int64_t before = 0;
    total = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
        if (i < w)
            before += wsum[i];
        total += wsum[i];
    }
    __syncthreads();  // wsum is reused by the next call
    return before + incl - x;
}

// One block: tile offsets in set order into rows[k].first_tile, item offsets in rank order into
// item_off[k]; the tile total against the capacity; the queue head and the item count.
__global__ __launch_bounds__(kScanThreads) void k_batch_scan(int32_t n_sets, int32_t ppl,
                                                             int64_t cap, SetRow *rows,
                                                             const uint32_t *order,
                                                             int64_t *item_off, Ctl *ctl)
{
    int64_t tiles_before = 0, items_before = 0;
    for (int32_t c = 0; c < n_sets; c += kScanThreads) {
        const int32_t k = c + (int32_t)threadIdx.x;
        int64_t tiles = 0, items = 0;
        uint32_t s = 0;
        if (k < n_sets) {
            tiles = (rows[k].n_traj + 63) / 64;
            s = order[k];  // the set at rank k
            items = ((rows[s].n_traj + 63) / 64 + ppl - 1) / ppl;
        }
        int64_t t_total, i_total;
        const int64_t t_off = block_scan(tiles, t_total);
        const int64_t i_off = block_scan(items, i_total);
        if (k < n_sets) {
            rows[k].first_tile = tiles_before + t_off;
            item_off[s] = items_before + i_off;
        }
        tiles_before += t_total;
        items_before += i_total;
    }
    if (threadIdx.x == 0) {
        if (tiles_before > cap)
            atomicMax(&ctl->status, (int32_t)ABP_E_WORKSPACE);
        ctl->head = 0;
        ctl->n_items = (uint32_t)std::min<int64_t>(items_before, kMaxTiles);
    }
}

__global__ __launch_bounds__(256) void k_batch_items(int32_t n_sets, int32_t ppl,
                                                     const SetRow *rows, const int64_t *item_off,
                                                     const Ctl *ctl, Item *items)
{
    const int32_t k = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n_sets || ctl->status != ABP_OK)
        return;  // with the status raised the offsets may lie past the workspace
    const uint32_t tiles = (uint32_t)((rows[k].n_traj + 63) / 64);
    Item *out = items + item_off[k];
    uint32_t i = 0;
    for (uint32_t t = 0; t < tiles; t += (uint32_t)ppl)
        out[i++] = Item{(uint32_t)k, t};
}

template <int SCHEME, int PPL, int UNROLL>
__global__ __launch_bounds__(256) void k_batched(BatchArgs a)
{
    const int lane = threadIdx.x & 63;
    if (a.ctl->status != ABP_OK)
        return;
    const uint32_t n_items = a.ctl->n_items;
    for (;;) {
        uint32_t taken = 0;
        if (lane == 0)
            taken = atomicAdd(&a.ctl->head, 1u);
        const uint32_t idx = __builtin_amdgcn_readfirstlane(taken);
        if (idx >= n_items)
            break;  // the counter only grows, so every wave leaves once the list is used up
        const Item it = a.items[idx];
        const SetRow row = a.rows[it.set];
        const Stream s{a.k0, a.k1, it.set};

        Particle p[PPL];
        uint32_t pid[PPL];
        bool live[PPL];
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int64_t i = (int64_t)(it.tile0 + q) * 64 + lane;
            live[q] = i < row.n_traj;
            pid[q] = (uint32_t)i;
            const Philox4 r = philox4x32_10(0u, pid[q], it.set, kDomainInit, a.k0, a.k1);
            p[q].cell = 0;
            p[q].xf = (float)(r.w[0] >> 8) * 0x1p-24f;
            p[q].v = p[q].e = 0.0f;
            p[q].lx = p[q].lv = p[q].le = 0.0f;
        }
        int64_t step = 0;
        double xs[PPL], xe[PPL];
        advance<SCHEME, PPL, UNROLL>(row.k, s, pid, p, step, row.win_begin);
#pragma unroll
        for (int q = 0; q < PPL; ++q)
            xs[q] = position64(p[q].cell, p[q].xf, p[q].lx);
        advance<SCHEME, PPL, UNROLL>(row.k, s, pid, p, step, row.n_steps);
#pragma unroll
        for (int q = 0; q < PPL; ++q)
            xe[q] = position64(p[q].cell, p[q].xf, p[q].lx);
        reduce_tiles<PPL>(xe, xs, live, it.tile0, row.n_traj, lane, a.n_bins,
                          a.part + 2 * row.first_tile,
                          a.hist + (size_t)it.set * (size_t)(a.n_bins > 0 ? a.n_bins : 0));
    }
}

// One block of kFinalizeThreads per set; block 0 also reports the status.
__global__ __launch_bounds__(kFinalizeThreads) void k_batched_finalize(const SetRow *rows,
                                                                       const Ctl *ctl,
                                                                       const double *part,
                                                                       const uint32_t *hist32,
                                                                       int32_t n_bins, double dt,
                                                                       double *out,
                                                                       uint64_t *hist64,
                                                                       int32_t *status)
{
    const uint32_t k = blockIdx.x;
    const int32_t st = ctl->status;
    if (k == 0 && threadIdx.x == 0 && status)
        *status = st;
    if (st != ABP_OK) {
        if (threadIdx.x < 2)
            out[2 * (size_t)k + threadIdx.x] = __builtin_nan("");
        for (int b = threadIdx.x; b < n_bins; b += kFinalizeThreads)
            hist64[(size_t)k * n_bins + b] = 0;
        return;
    }
    const SetRow &row = rows[k];
    const double wtime = (double)(row.n_steps - row.win_begin) * dt;
    finalize_set(part + 2 * row.first_tile, (row.n_traj + 63) / 64, row.n_traj, wtime,
                 out + 2 * (size_t)k);
    for (int b = threadIdx.x; b < n_bins; b += kFinalizeThreads)
        hist64[(size_t)k * n_bins + b] = hist32[(size_t)k * n_bins + b];
}

template <int SCHEME, int PPL, int UNROLL>
static void launch_batched(const BatchArgs &a, int block, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_batched<SCHEME, PPL, UNROLL>), dim3(grid), dim3(block), 0, st, a);
}

template <int SCHEME, int PPL>
static void dispatch_loop(const BatchArgs &a, const Shape &sh, int grid, hipStream_t st)
{
    switch (sh.loop()) {
    case 1: launch_batched<SCHEME, PPL, 1>(a, sh.block, grid, st); break;
    case 2: launch_batched<SCHEME, PPL, 2>(a, sh.block, grid, st); break;
    default: launch_batched<SCHEME, PPL, kAhead>(a, sh.block, grid, st); break;
    }
}

template <int SCHEME>
static void dispatch_batched(const BatchArgs &a, const Shape &sh, int grid, hipStream_t st)
{
    if (sh.ppl == 1)
        dispatch_loop<SCHEME, 1>(a, sh, grid, st);
    else
        dispatch_loop<SCHEME, 2>(a, sh, grid, st);
}

constexpr Shape kDefaultBatched = {256, 1, 1, 8, 0};
constexpr int32_t kMaxSets = 1 << 20;

}  // namespace abp

using namespace abp;

extern "C" size_t abp_batched_workspace_bytes(int32_t n_sets, int64_t n_tiles, int32_t n_bins)
{
    if (n_sets < 1 || n_sets > kMaxSets || n_tiles < n_sets || n_tiles > kMaxTiles ||
        !bins_ok(n_bins))
        return 0;
    return batch_layout(n_sets, n_tiles, n_bins).total;
}

extern "C" abp_status abp_integrate_batched(int32_t n_sets, const abp_params *d_params,
                                            const int32_t *d_ntraj, const int64_t *d_nsteps,
                                            const int64_t *d_window, const abp_batch *cfg,
                                            const abp_tuning *tune, void *d_ws, size_t ws_bytes,
                                            double *d_out, uint64_t *d_hist, int32_t *d_status,
                                            void *stream)
{
    if (n_sets < 1 || n_sets > kMaxSets || !cfg || !d_params || !d_ntraj || !d_nsteps ||
        !aligned(d_params, 8) || !aligned(d_ntraj, 4) || !aligned(d_nsteps, 8) ||
        !aligned(d_window, 8) || !aligned(d_status, 4))
        return ABP_E_ARG;
    if (!(cfg->dt > 0.0) || !is_finite(cfg->dt) || !bins_ok(cfg->n_bins) ||
        (cfg->scheme != ABP_EM && cfg->scheme != ABP_HEUN))
        return ABP_E_ARG;
    if (!d_ws || !aligned(d_ws, 256) || !d_out || !aligned(d_out, 8) ||
        (cfg->n_bins > 0 && (!d_hist || !aligned(d_hist, 8))))
        return ABP_E_ARG;
    Shape sh;
    if (!resolve_tuning(tune, kDefaultBatched, sh))
        return ABP_E_ARG;
    const int64_t cap = batch_capacity(n_sets, cfg->n_bins, ws_bytes);
    if (cap < n_sets)  // every set has at least one tile
        return ABP_E_WORKSPACE;
    if (abp_status st = check_device())
        return st;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return ABP_E_HIP;

    const BatchLayout L = batch_layout(n_sets, cap, cfg->n_bins);
    char *ws = reinterpret_cast<char *>(d_ws);
    SetRow *rows = reinterpret_cast<SetRow *>(ws + L.rows);
    uint32_t *order = reinterpret_cast<uint32_t *>(ws + L.order);
    int64_t *item_off = reinterpret_cast<int64_t *>(ws + L.item_off);
    Ctl *ctl = reinterpret_cast<Ctl *>(ws + L.ctl);
    Item *items = reinterpret_cast<Item *>(ws + L.items);
    hipStream_t st = as_stream(stream);
    const unsigned set_blocks = (unsigned)((n_sets + 255) / 256);

    fill_u32(reinterpret_cast<uint32_t *>(ctl), sizeof(Ctl) / sizeof(uint32_t), st);
    if (cfg->n_bins > 0)
        fill_u32(reinterpret_cast<uint32_t *>(ws + L.hist), (int64_t)n_sets * cfg->n_bins, st);
    hipLaunchKernelGGL(k_batch_prepare, dim3(set_blocks), dim3(256), 0, st, n_sets, d_params,
                       d_ntraj, d_nsteps, d_window, cfg->dt, rows, ctl);
    hipLaunchKernelGGL(k_batch_rank, dim3(set_blocks), dim3(256), 0, st, n_sets, rows, order);
    hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(kScanThreads), 0, st, n_sets, sh.ppl, cap,
                       rows, order, item_off, ctl);
    hipLaunchKernelGGL(k_batch_items, dim3(set_blocks), dim3(256), 0, st, n_sets, sh.ppl, rows,
                       item_off, ctl, items);
    if (hipGetLastError() != hipSuccess)
        return ABP_E_HIP;

    BatchArgs a{};
    a.rows = rows;
    a.items = items;
    a.ctl = ctl;
    a.part = reinterpret_cast<double *>(ws + L.part);
    a.hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    a.n_bins = cfg->n_bins;
    const Stream ks = make_stream(cfg->seed, 0);
    a.k0 = ks.k0;
    a.k1 = ks.k1;
    // a persistent grid at the requested residency; waves beyond the list leave at once
    const int waves_per_block = sh.block / 64;
    const int64_t grid = std::max<int64_t>(1, (int64_t)cus * 4 * sh.waves_per_simd /
                                                  waves_per_block);
    resolve_lookahead(sh, grid * waves_per_block);
    if (cfg->scheme == ABP_EM)
        dispatch_batched<0>(a, sh, (int)grid, st);
    else
        dispatch_batched<1>(a, sh, (int)grid, st);
    if (hipGetLastError() != hipSuccess)
        return ABP_E_HIP;
    hipLaunchKernelGGL(k_batched_finalize, dim3((unsigned)n_sets), dim3(kFinalizeThreads), 0, st,
                       a.rows, a.ctl, a.part, a.hist, cfg->n_bins, cfg->dt, d_out, d_hist,
                       d_status);
    return launch_status();
}
