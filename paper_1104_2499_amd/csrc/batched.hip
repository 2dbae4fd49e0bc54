// batched.hip -- many parameter sets in one persistent launch (the paper runs one work item per
// parameter set concurrently, Sec. 2; here a set is an ensemble of trajectories).
//
// The host cuts every set into work items of PPL 64-particle tiles, sorts the items by step count
// (longest first, so the shortest items fill the tail), and stages per-set constants and the item
// list in the workspace. A grid sized to the device's residency runs waves that each take the
// next item from an atomic counter until the list is empty. Every item starts from the set's
// initial condition (Philox domain 1), integrates to the set's window start, snapshots the
// position, integrates to the end and leaves per-tile FP64 partials in the set's slots; one wave
// per set then adds the tiles in order. A set therefore gives the same bits as abp_integrate with
// set_id = its index, id0 = 0, and a window of the same length.
//
// Workspace layout (abp_batched_workspace_bytes):
//   SetRow rows[n_sets] | Item items[n_tiles_total] | u32 head | double part[n_tiles_total][2] |
//   u32 hist[n_sets][n_bins]
#include <algorithm>
#include <vector>

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

struct BatchArgs {
    const SetRow *rows;
    const Item *items;
    uint32_t *head;
    double *part;
    uint32_t *hist;
    uint32_t n_items;
    int32_t n_bins;
    uint32_t k0, k1;  // Philox key
};

struct BatchLayout {
    size_t rows, items, head, part, hist, total;
};

inline BatchLayout batch_layout(int32_t n_sets, int64_t tiles, int32_t n_bins)
{
    BatchLayout L;
    L.rows = 0;
    L.items = align_up(L.rows + sizeof(SetRow) * (size_t)n_sets, 256);
    L.head = align_up(L.items + sizeof(Item) * (size_t)tiles, 256);
    L.part = align_up(L.head + sizeof(uint32_t), 256);
    L.hist = align_up(L.part + 2 * sizeof(double) * (size_t)tiles, 256);
    L.total = align_up(L.hist + sizeof(uint32_t) * (size_t)n_sets * (size_t)n_bins, 256);
    return L;
}

template <int SCHEME, int PPL, int UNROLL>
__global__ __launch_bounds__(256) void k_batched(BatchArgs a)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        uint32_t taken = 0;
        if (lane == 0)
            taken = atomicAdd(a.head, 1u);
        const uint32_t idx = __builtin_amdgcn_readfirstlane(taken);
        if (idx >= a.n_items)
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

// One block of kFinalizeThreads per set.
__global__ __launch_bounds__(kFinalizeThreads) void k_batched_finalize(const SetRow *rows,
                                                                       const double *part,
                                                                       const uint32_t *hist32,
                                                                       int32_t n_bins, double dt,
                                                                       double *out,
                                                                       uint64_t *hist64)
{
    const uint32_t k = blockIdx.x;
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

template <int SCHEME>
static void dispatch_batched(const BatchArgs &a, const Shape &sh, int grid, hipStream_t st)
{
    if (sh.ppl == 1) {
        if (sh.unroll == 1)
            launch_batched<SCHEME, 1, 1>(a, sh.block, grid, st);
        else
            launch_batched<SCHEME, 1, 2>(a, sh.block, grid, st);
    } else {
        if (sh.unroll == 1)
            launch_batched<SCHEME, 2, 1>(a, sh.block, grid, st);
        else
            launch_batched<SCHEME, 2, 2>(a, sh.block, grid, st);
    }
}

constexpr Shape kDefaultBatched = {256, 1, 1, 8};

static bool batch_sizes(int32_t n_sets, const int32_t *h_ntraj, int64_t &tiles)
{
    if (n_sets < 1 || !h_ntraj)
        return false;
    tiles = 0;
    for (int32_t k = 0; k < n_sets; ++k) {
        if (h_ntraj[k] < 1)
            return false;
        tiles += (h_ntraj[k] + 63) / 64;
    }
    return tiles <= 0xFFFFFFFFll;
}

}  // namespace abp

using namespace abp;

extern "C" size_t abp_batched_workspace_bytes(int32_t n_sets, const int32_t *h_ntraj,
                                              int32_t n_bins)
{
    int64_t tiles = 0;
    if (!batch_sizes(n_sets, h_ntraj, tiles) || !bins_ok(n_bins))
        return 0;
    return batch_layout(n_sets, tiles, n_bins).total;
}

extern "C" abp_status abp_integrate_batched(int32_t n_sets, const abp_params *h_params,
                                            const int32_t *h_ntraj, const int64_t *h_nsteps,
                                            const int64_t *h_window, const abp_batch *cfg,
                                            const abp_tuning *tune, void *d_ws, size_t ws_bytes,
                                            double *d_out, uint64_t *d_hist, void *stream)
{
    int64_t tiles = 0;
    if (!h_params || !h_nsteps || !cfg || !batch_sizes(n_sets, h_ntraj, tiles))
        return ABP_E_ARG;
    if (!(cfg->dt > 0.0) || !is_finite(cfg->dt) || !bins_ok(cfg->n_bins) ||
        (cfg->scheme != ABP_EM && cfg->scheme != ABP_HEUN))
        return ABP_E_ARG;
    if (!d_ws || !aligned(d_ws, 256) || !d_out || !aligned(d_out, 8) ||
        (cfg->n_bins > 0 && (!d_hist || !aligned(d_hist, 8))))
        return ABP_E_ARG;
    for (int32_t k = 0; k < n_sets; ++k) {
        const int64_t S = h_nsteps[k];
        const int64_t W = h_window ? h_window[k] : S / 2;
        if (!params_ok(h_params[k]) || !coef_ok(make_coef(h_params[k], cfg->dt)) || S < 1 ||
            S > kMaxStepIndex || W < 1 || W > S)
            return ABP_E_ARG;
    }
    Shape sh;
    if (!resolve_tuning(tune, kDefaultBatched, sh))
        return ABP_E_ARG;
    const BatchLayout L = batch_layout(n_sets, tiles, cfg->n_bins);
    if (ws_bytes < L.total)
        return ABP_E_WORKSPACE;
    if (abp_status st = check_device())
        return st;

    // per-set constants, tile offsets and the work list (longest first)
    std::vector<SetRow> rows((size_t)n_sets);
    std::vector<Item> items;
    items.reserve((size_t)tiles);
    int64_t first = 0;
    for (int32_t k = 0; k < n_sets; ++k) {
        SetRow &r = rows[(size_t)k];
        std::memset(&r, 0, sizeof r);
        r.k = make_coef(h_params[k], cfg->dt);
        r.n_steps = h_nsteps[k];
        r.win_begin = r.n_steps - (h_window ? h_window[k] : r.n_steps / 2);
        r.n_traj = h_ntraj[k];
        r.first_tile = first;
        const uint32_t set_tiles = (uint32_t)((h_ntraj[k] + 63) / 64);
        for (uint32_t t = 0; t < set_tiles; t += (uint32_t)sh.ppl)
            items.push_back(Item{(uint32_t)k, t});
        first += set_tiles;
    }
    std::stable_sort(items.begin(), items.end(), [&](const Item &x, const Item &y) {
        return rows[x.set].n_steps > rows[y.set].n_steps;
    });

    hipStream_t st = as_stream(stream);
    char *ws = reinterpret_cast<char *>(d_ws);
    WaitOnExit wait{st, true};  // rows and items are read by the copies below
    if (hipMemcpyAsync(ws + L.rows, rows.data(), sizeof(SetRow) * rows.size(),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(ws + L.items, items.data(), sizeof(Item) * items.size(),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return ABP_E_HIP;
    fill_u32(reinterpret_cast<uint32_t *>(ws + L.head), 1, st);
    if (cfg->n_bins > 0)
        fill_u32(reinterpret_cast<uint32_t *>(ws + L.hist), (int64_t)n_sets * cfg->n_bins, st);

    BatchArgs a{};
    a.rows = reinterpret_cast<const SetRow *>(ws + L.rows);
    a.items = reinterpret_cast<const Item *>(ws + L.items);
    a.head = reinterpret_cast<uint32_t *>(ws + L.head);
    a.part = reinterpret_cast<double *>(ws + L.part);
    a.hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    a.n_items = (uint32_t)items.size();
    a.n_bins = cfg->n_bins;
    const Stream ks = make_stream(cfg->seed, 0);
    a.k0 = ks.k0;
    a.k1 = ks.k1;

    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return ABP_E_HIP;
    const int waves_per_block = sh.block / 64;
    int64_t grid = (int64_t)cus * 4 * sh.waves_per_simd / waves_per_block;
    const int64_t needed = ((int64_t)items.size() + waves_per_block - 1) / waves_per_block;
    grid = std::max<int64_t>(1, std::min(grid, needed));
    if (cfg->scheme == ABP_EM)
        dispatch_batched<0>(a, sh, (int)grid, st);
    else
        dispatch_batched<1>(a, sh, (int)grid, st);
    if (hipGetLastError() != hipSuccess)
        return ABP_E_HIP;
    hipLaunchKernelGGL(k_batched_finalize, dim3((unsigned)n_sets), dim3(kFinalizeThreads), 0, st, a.rows, a.part,
                       a.hist, cfg->n_bins, cfg->dt, d_out, d_hist);
    if (hipGetLastError() != hipSuccess)
        return ABP_E_HIP;
    // the staged tables live in pageable host memory owned by this call
    wait.armed = false;
    return hipStreamSynchronize(st) == hipSuccess ? ABP_OK : ABP_E_HIP;
}
