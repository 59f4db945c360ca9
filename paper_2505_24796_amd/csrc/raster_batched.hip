// Multi-view forward rasterisation in one persistent launch (serving many
// cameras of one scene per frame; TC-GS paper Sec. 4 per tile).
//
// Every (view, tile) pair of the frame is one work item.  The items live in
// eight queues, one per XCD: queue q holds, view after view, the tiles of
// the bands of two tile rows with band index = q mod 8 (the same band-to-XCD
// assignment the one-view launch uses), so neighbouring tiles, which share
// most of their splats, are rendered under one L2.  A workgroup (4 waves,
// 256 pixels) takes items from its own XCD's queue with an atomic counter
// and, once that queue is empty, from the other seven in turn; it exits when
// all eight are empty, so every workgroup finishes and the launch drains
// without any wait.  A single-queue mode (row-major tiles, view after view)
// is kept for the tuner.
//
// Each tile is rendered by raster_tile_mfma, the per-tile body of the
// one-view kernel, so a view's image is bit-identical to gs_rasterize_fwd's.
// Optionally the launch stamps, per view, the device wall clock at which the
// view's last tile finished (per-view latency inside a batched frame).
#include <vector>

#include "raster_tile.h"

namespace {

constexpr int MAX_VIEWS = 64;
constexpr int NQ = 8;

struct PlanHead {
    int32_t nviews;
    uint32_t qsize[NQ + 1];  // items per XCD queue; [NQ]: the single queue
    uint32_t pad[6];
};
static_assert(sizeof(PlanHead) == 64, "plan head is 64 bytes");

// Device plan: head, then per view the raster arguments, then the queue
// bases qbase[q][v] = first item of view v in queue q (q = NQ: single queue)
// and ntiles[v].
struct PlanView {
    RasterArgs a;
};

__host__ __device__ inline size_t plan_views_off() { return sizeof(PlanHead); }
__host__ __device__ inline size_t plan_qbase_off(int nv) { return plan_views_off() + (size_t)nv * sizeof(PlanView); }
__host__ __device__ inline size_t plan_ntiles_off(int nv) { return plan_qbase_off(nv) + (size_t)(NQ + 1) * nv * 4; }
inline size_t plan_bytes(int nv) { return (plan_ntiles_off(nv) + (size_t)nv * 4 + 255) / 256 * 256; }

// Workspace words: [0, NQ] queue heads, [16, 16 + nviews) tiles finished
// per view.
constexpr int WS_DONE = 16;
inline size_t ws_words(int nv) { return (size_t)WS_DONE + nv; }

__global__ __launch_bounds__(256) void k_batch_init(uint32_t *__restrict__ ws, int nwords) {
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) ws[i] = 0u;
}

__global__ void k_clock_stamp(unsigned long long *dst) {
    if (threadIdx.x == 0) *dst = (unsigned long long)wall_clock64();
}

// Tile of item j of a view inside XCD queue q: bands of two tile rows, band
// q, q + 8, q + 16, ... of the view, row-major inside a band.
__device__ __forceinline__ int band_tile(uint32_t j, int q, int gx) {
    const uint32_t band = 2u * (uint32_t)gx;
    const uint32_t slot = j / band, within = j - slot * band;
    return (int)((q + NQ * slot) * band + within);
}

template <int VAR, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_raster_batched(
    const uint8_t *__restrict__ plan, uint32_t *__restrict__ ws, unsigned long long *__restrict__ clk,
    int xcd_queues) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[Stage<VAR, NB>::BYTES];
    __shared__ TileShared sh;
    __shared__ uint32_t s_qbase[(NQ + 1) * MAX_VIEWS];
    __shared__ uint32_t s_ntiles[MAX_VIEWS];
    __shared__ int s_view, s_tile;
    const PlanHead *head = (const PlanHead *)plan;
    const PlanView *views = (const PlanView *)(plan + plan_views_off());
    const int nv = head->nviews;
    {
        const uint32_t *qb = (const uint32_t *)(plan + plan_qbase_off(nv));
        const uint32_t *nt = (const uint32_t *)(plan + plan_ntiles_off(nv));
        for (int i = threadIdx.x; i < (NQ + 1) * nv; i += 256) s_qbase[i] = qb[i];
        for (int i = threadIdx.x; i < nv; i += 256) s_ntiles[i] = nt[i];
    }
    const int nq = xcd_queues ? NQ : 1;
    const int q0 = xcd_queues ? (int)(blockIdx.x & (NQ - 1)) : NQ;
    int prev = -1;  // view of this workgroup's last tile (thread 0)
    for (int qi = 0; qi < nq; ++qi) {
        const int q = xcd_queues ? (q0 + qi) & (NQ - 1) : NQ;
        const uint32_t qsize = head->qsize[q];
        for (;;) {
            // every wave has finished the previous tile and read s_view/s_tile
            __syncthreads();
            if (threadIdx.x == 0) {
                if (prev >= 0) {
                    const uint32_t d = atomicAdd(ws + WS_DONE + prev, 1u);
                    if (clk && d + 1u == s_ntiles[prev])
                        clk[prev] = (unsigned long long)wall_clock64();
                    prev = -1;
                }
                const uint32_t item = atomicAdd(ws + q, 1u);
                int v = -1, t = 0;
                if (item < qsize) {
                    // last view whose share of queue q starts at or before item
                    const uint32_t *qb = s_qbase + q * nv;
                    int lo = 0, hi = nv;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (qb[mid] <= item) lo = mid;
                        else hi = mid;
                    }
                    v = lo;
                    const uint32_t j = item - qb[v];
                    t = q < NQ ? band_tile(j, q, views[v].a.gx) : (int)j;
                    prev = v;
                }
                s_view = v;
                s_tile = t;
            }
            __syncthreads();
            const int v = __builtin_amdgcn_readfirstlane(s_view);
            const int t = __builtin_amdgcn_readfirstlane(s_tile);
            if (v < 0) break;
            raster_tile_mfma<VAR, false, NB>(views[v].a, t, stage, sh);
        }
    }
}

template <int VAR, int NB>
void launch_batched(int grid, const uint8_t *plan, uint32_t *ws, unsigned long long *clk, int xcd,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_raster_batched<VAR, NB>), dim3(grid), dim3(256), 0, s, plan, ws, clk, xcd);
}

template <int VAR>
void launch_batched_nb(int nb, int grid, const uint8_t *plan, uint32_t *ws, unsigned long long *clk,
                       int xcd, hipStream_t s) {
    switch (nb) {
    case 64: launch_batched<VAR, 64>(grid, plan, ws, clk, xcd, s); break;
    case 128: launch_batched<VAR, 128>(grid, plan, ws, clk, xcd, s); break;
    default: launch_batched<VAR, 256>(grid, plan, ws, clk, xcd, s); break;
    }
}

int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n;
}

}  // namespace

extern "C" size_t gs_batch_plan_bytes(int32_t nviews) {
    if (nviews <= 0 || nviews > MAX_VIEWS) return 0;
    return plan_bytes(nviews);
}

extern "C" size_t gs_batch_workspace_bytes(int32_t nviews) {
    if (nviews <= 0 || nviews > MAX_VIEWS) return 0;
    return ws_words(nviews) * 4;
}

extern "C" gs_status gs_batch_plan_write(int32_t nviews, const gs_view *views, void *plan,
                                         size_t plan_bytes_) {
    if (nviews <= 0 || nviews > MAX_VIEWS || !views || !plan || !gs::aligned(plan, 256))
        return GS_ERR_INVALID_ARG;
    if (plan_bytes_ < plan_bytes(nviews)) return GS_ERR_CAPACITY;
    std::vector<uint8_t> host(plan_bytes(nviews), 0);
    PlanHead *head = (PlanHead *)host.data();
    PlanView *pv = (PlanView *)(host.data() + plan_views_off());
    uint32_t *qbase = (uint32_t *)(host.data() + plan_qbase_off(nviews));
    uint32_t *ntl = (uint32_t *)(host.data() + plan_ntiles_off(nviews));
    head->nviews = nviews;
    uint64_t qtot[NQ + 1] = {};
    for (int v = 0; v < nviews; ++v) {
        const gs_view &g = views[v];
        const void *ptrs[] = {g.tile_ranges, g.sorted_ids, g.means2d, g.conics, g.log_opacities,
                              g.rgb, g.out_rgb, g.out_T, g.out_ncontrib};
        if (!valid_inputs(g.width, g.height, ptrs, 9) || !gs::aligned(g.means2d, 8))
            return GS_ERR_INVALID_ARG;
        RasterArgs &a = pv[v].a;
        a.chunk_rows = 2;
        a.W = g.width;
        a.H = g.height;
        a.gx = gs::grid_x(g.width);
        a.gy = gs::grid_y(g.height);
        a.ranges = g.tile_ranges;
        a.ids = g.sorted_ids;
        a.means2d = (const float2 *)g.means2d;
        a.conics = g.conics;
        a.lno = g.log_opacities;
        a.rgb = g.rgb;
        a.bg0 = g.background[0];
        a.bg1 = g.background[1];
        a.bg2 = g.background[2];
        a.out_rgb = g.out_rgb;
        a.out_T = g.out_T;
        a.out_nc = g.out_ncontrib;
        a.counters = nullptr;
        const uint32_t nt = (uint32_t)a.gx * (uint32_t)a.gy;
        ntl[v] = nt;
        // tiles per XCD queue: bands of two rows, band b -> queue b mod 8
        uint32_t cnt[NQ] = {};
        for (int b = 0; 2 * b < a.gy; ++b)
            cnt[b % NQ] += (uint32_t)a.gx * (2 * b + 1 < a.gy ? 2u : 1u);
        for (int q = 0; q < NQ; ++q) {
            qbase[q * nviews + v] = (uint32_t)qtot[q];
            qtot[q] += cnt[q];
        }
        qbase[NQ * nviews + v] = (uint32_t)qtot[NQ];
        qtot[NQ] += nt;
    }
    if (qtot[NQ] >= 0x80000000ull) return GS_ERR_INVALID_ARG;
    for (int q = 0; q <= NQ; ++q) head->qsize[q] = (uint32_t)qtot[q];
    if (hipMemcpy(plan, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
        return GS_ERR_HIP;
    return GS_OK;
}

extern "C" gs_status gs_rasterize_fwd_batched(int32_t nviews, const void *plan, int32_t precision,
                                              const gs_batch_tune *tune, void *workspace,
                                              size_t workspace_bytes, uint64_t *d_view_clock,
                                              void *stream) {
    if (nviews <= 0 || nviews > MAX_VIEWS || !plan || !gs::aligned(plan, 256) || !workspace ||
        !gs::aligned(workspace, 4))
        return GS_ERR_INVALID_ARG;
    if (d_view_clock && !gs::aligned(d_view_clock, 8)) return GS_ERR_INVALID_ARG;
    if (workspace_bytes < ws_words(nviews) * 4) return GS_ERR_CAPACITY;
    if (precision < GS_PREC_FP32 || precision > GS_PREC_BF16_G2L_SPLIT) return GS_ERR_INVALID_ARG;
    if (precision < GS_PREC_FP16_GLOBAL) return GS_ERR_UNSUPPORTED;
    gs_batch_tune t = tune ? *tune : gs_batch_tune{256, 5, 1};
    if ((t.batch != 64 && t.batch != 128 && t.batch != 256) || t.blocks_per_cu < 1 ||
        t.blocks_per_cu > 16 || (t.xcd_queues != 0 && t.xcd_queues != 1))
        return GS_ERR_INVALID_ARG;
    const int cus = device_cus();
    if (cus <= 0) return GS_ERR_HIP;
    // a multiple of 8 keeps workgroup b on XCD b mod 8 for every b
    const int grid = (cus * t.blocks_per_cu + NQ - 1) / NQ * NQ;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *ws = (uint32_t *)workspace;
    const uint8_t *pl = (const uint8_t *)plan;
    auto *clk = (unsigned long long *)d_view_clock;
    hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(256), 0, s, ws, (int)ws_words(nviews));
    switch (precision) {
    case GS_PREC_FP16_GLOBAL: launch_batched_nb<VAR_F16_GLOBAL>(t.batch, grid, pl, ws, clk, t.xcd_queues, s); break;
    case GS_PREC_FP16_G2L: launch_batched_nb<VAR_F16_G2L>(t.batch, grid, pl, ws, clk, t.xcd_queues, s); break;
    case GS_PREC_FP16_G2L_SPLIT: launch_batched_nb<VAR_F16_SPLIT>(t.batch, grid, pl, ws, clk, t.xcd_queues, s); break;
    case GS_PREC_BF16_G2L_SPLIT: launch_batched_nb<VAR_BF16_SPLIT>(t.batch, grid, pl, ws, clk, t.xcd_queues, s); break;
    }
    return gs::launch_status();
}

extern "C" gs_status gs_clock_stamp(uint64_t *d_dst, void *stream) {
    if (!d_dst || !gs::aligned(d_dst, 8)) return GS_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_clock_stamp, dim3(1), dim3(64), 0, (hipStream_t)stream,
                       (unsigned long long *)d_dst);
    return gs::launch_status();
}

extern "C" gs_status gs_wall_clock_khz(int32_t *khz) {
    if (!khz) return GS_ERR_INVALID_ARG;
    int dev = 0, r = 0;
    if (hipGetDevice(&dev) != hipSuccess) return GS_ERR_HIP;
    if (hipDeviceGetAttribute(&r, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return GS_ERR_HIP;
    *khz = r;
    return GS_OK;
}
