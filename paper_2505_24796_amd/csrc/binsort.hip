// Binning and sorting (TC-GS paper, Sec. 3.1 "Sorting"): per-tile splat
// lists ordered by depth, then Gaussian id.
//
// Instead of one radix sort of N 64-bit (tile | depth) keys, the stage
//   1. sorts the P Gaussians by depth (stable LSD radix, 4 x 8-bit passes on
//      an order-preserving image of the float bits; ties keep id order),
//   2. scans the per-Gaussian tile counts in that order and emits the splats
//      (tile, id) in depth order,
//   3. sorts the N splats by tile only (stable LSD radix, ceil(bits/8)
//      passes over ceil(log2 ntiles) bits), which keeps depth order within a
//      tile, and
//   4. finds each tile's [start, end).
// This touches every splat 2 x (8 + 8) bytes per tile pass instead of
// 6 passes x 24 bytes, and every stage is bound by HBM bandwidth.
#include "common.h"

namespace {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;  // keys per block
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int WAVES = SORT_THREADS / 64;
constexpr int WAVE_ITEMS = SORT_TILE / WAVES;          // 1024 per wave
constexpr int WAVE_CHUNKS = WAVE_ITEMS / 64;           // 16 chunks of 64

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Number of valid elements of a pass: static, or the device splat count
// (zero when it exceeds the capacity, so an overflowing frame does nothing).
struct Count {
    uint32_t n_static;
    const uint32_t *n_dev;
    uint32_t cap;
    __device__ __forceinline__ uint32_t get() const {
        if (!n_dev) return n_static;
        uint32_t n = *n_dev;
        return n > cap ? 0u : n;
    }
};

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of u32 values (u64 running totals so that an
// overflowing splat count is detected instead of wrapping).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t &excl, uint64_t *lds4) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t inc = wave_incl_scan_u64(v);
    if (lane == 63) lds4[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        uint64_t s = lds4[i];
        if (i < w) off += s;
        tot += s;
    }
    excl = off + inc - v;
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(SORT_THREADS) void k_scan_reduce(const uint32_t *__restrict__ in,
                                                              uint32_t n,
                                                              uint64_t *__restrict__ part) {
    __shared__ uint64_t lds4[WAVES];
    size_t base = (size_t)blockIdx.x * SORT_TILE + (size_t)threadIdx.x * SORT_ITEMS;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k)
        if (base + k < n) s += in[base + k];
    uint64_t ex;
    uint64_t tot = block_excl_scan(s, ex, lds4);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block partials in place; writes the
// grand total (saturated to u32) to *total when total is non-null.
__global__ __launch_bounds__(1024) void k_scan_partials(uint64_t *__restrict__ part, uint32_t nparts,
                                                        uint32_t *__restrict__ total) {
    __shared__ uint64_t lds16[16];
    uint64_t carry = 0;
    for (uint32_t base = 0; base < nparts; base += 1024) {
        uint32_t i = base + threadIdx.x;
        uint64_t v = i < nparts ? part[i] : 0;
        uint64_t ex;
        uint64_t tot = block_excl_scan(v, ex, lds16);
        if (i < nparts) part[i] = carry + ex;
        carry += tot;
    }
    if (total && threadIdx.x == 0) *total = carry > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)carry;
}

__global__ __launch_bounds__(SORT_THREADS) void k_scan_down(const uint32_t *in, uint32_t *out,
                                                            uint32_t n,
                                                            const uint64_t *__restrict__ part) {
    __shared__ uint64_t lds4[WAVES];
    size_t base = (size_t)blockIdx.x * SORT_TILE + (size_t)threadIdx.x * SORT_ITEMS;
    uint32_t v[SORT_ITEMS];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint64_t ex;
    block_excl_scan(s, ex, lds4);
    uint64_t run = part[blockIdx.x] + ex;
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        if (base + k < n) out[base + k] = (uint32_t)run;
        run += v[k];
    }
}

struct ScanPlan {
    uint32_t n, blocks;
};

gs_status device_scan(const uint32_t *in, uint32_t *out, uint32_t n, uint64_t *part,
                      uint32_t *total, hipStream_t s) {
    uint32_t blocks = (n + SORT_TILE - 1) / SORT_TILE;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3(blocks), dim3(SORT_THREADS), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, part, blocks, total);
    hipLaunchKernelGGL(k_scan_down, dim3(blocks), dim3(SORT_THREADS), 0, s, in, out, n,
                       (const uint64_t *)part);
    return gs::launch_status();
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort pass (8-bit digit) of u32 keys with u32 values.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint32_t *__restrict__ keys,
                                                             Count cnt, int shift,
                                                             uint32_t *__restrict__ hist,
                                                             uint32_t nblocks) {
    __shared__ uint32_t h[RADIX];
    uint32_t n = cnt.get();
    h[threadIdx.x] = 0;
    __syncthreads();
    size_t base = (size_t)blockIdx.x * SORT_TILE;
    if (base < n) {
#pragma unroll
        for (int k = 0; k < SORT_ITEMS; ++k) {
            size_t i = base + (size_t)k * SORT_THREADS + threadIdx.x;
            if (i < n) atomicAdd(&h[(keys[i] >> shift) & (RADIX - 1)], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, Count cnt, int shift, const uint32_t *__restrict__ hist_scan,
    uint32_t nblocks) {
    __shared__ uint32_t wcnt[WAVES][RADIX];
    __shared__ uint32_t gbase[RADIX];
    uint32_t n = cnt.get();
    size_t base = (size_t)blockIdx.x * SORT_TILE;
    if (base >= n) return;  // whole block idle: uniform exit
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < WAVES; ++i) wcnt[i][threadIdx.x] = 0;
    gbase[threadIdx.x] = hist_scan[(size_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();

    uint32_t key[WAVE_CHUNKS], val[WAVE_CHUNKS], pos[WAVE_CHUNKS];
    size_t wbase = base + (size_t)w * WAVE_ITEMS;
#pragma unroll
    for (int c = 0; c < WAVE_CHUNKS; ++c) {
        size_t i = wbase + (size_t)c * 64 + lane;
        bool ok = i < n;
        key[c] = ok ? kin[i] : 0u;
        val[c] = ok ? vin[i] : 0u;
        uint32_t d = (key[c] >> shift) & (RADIX - 1);
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = gs::lanes_below(peers);
        uint32_t before = ok ? wcnt[w][d] : 0u;
        pos[c] = before + rank;
        if (ok && rank == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        uint32_t d = threadIdx.x, off = 0;
#pragma unroll
        for (int i = 0; i < WAVES; ++i) {
            uint32_t t = wcnt[i][d];
            wcnt[i][d] = off;
            off += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < WAVE_CHUNKS; ++c) {
        size_t i = wbase + (size_t)c * 64 + lane;
        if (i < n) {
            uint32_t d = (key[c] >> shift) & (RADIX - 1);
            uint32_t dst = gbase[d] + wcnt[w][d] + pos[c];
            kout[dst] = key[c];
            vout[dst] = val[c];
        }
    }
}

struct SortBufs {
    uint32_t *k[2], *v[2];
};

// Sorts on bits [0, bits) with ceil(bits/8) passes; returns the index of the
// buffer pair holding the result.
int radix_sort(SortBufs b, Count cnt, uint32_t max_n, int bits, uint32_t *hist, uint64_t *part,
               hipStream_t s) {
    uint32_t nblocks = (max_n + SORT_TILE - 1) / SORT_TILE;
    if (nblocks == 0) nblocks = 1;
    int cur = 0;
    for (int shift = 0; shift < bits; shift += RADIX_BITS) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(SORT_THREADS), 0, s, b.k[cur], cnt,
                           shift, hist, nblocks);
        device_scan(hist, hist, RADIX * nblocks, part, nullptr, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(SORT_THREADS), 0, s, b.k[cur],
                           b.v[cur], b.k[cur ^ 1], b.v[cur ^ 1], cnt, shift, hist, nblocks);
        cur ^= 1;
    }
    return cur;
}

// ---------------------------------------------------------------------------
// Stage kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t depth_key(float d) {
    uint32_t f = __float_as_uint(d);
    if (f == 0x80000000u) f = 0u;  // -0 equals +0
    return (f & 0x80000000u) ? ~f : (f | 0x80000000u);
}

__device__ __forceinline__ int splat_count(const float2 *means2d, const int *radii,
                                           const float *depths, int i, int W, int H, int gx,
                                           int &tx0, int &tx1, int &ty0, int &ty1) {
    float d = depths[i];
    if (!isfinite(d)) return 0;
    float2 m = means2d[i];
    return gs::tile_rect(m.x, m.y, radii[i], W, H, gx, tx0, tx1, ty0, ty1);
}

__global__ __launch_bounds__(256) void k_depth_keys(int P, const float2 *__restrict__ means2d,
                                                    const int *__restrict__ radii,
                                                    const float *__restrict__ depths, int W, int H,
                                                    int gx, uint32_t *__restrict__ keys,
                                                    uint32_t *__restrict__ ids) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    int a, b, c, d;
    int n = splat_count(means2d, radii, depths, i, W, H, gx, a, b, c, d);
    keys[i] = n > 0 ? depth_key(depths[i]) : 0xFFFFFFFFu;
    ids[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_counts(int P, const uint32_t *__restrict__ order,
                                                const float2 *__restrict__ means2d,
                                                const int *__restrict__ radii,
                                                const float *__restrict__ depths, int W, int H,
                                                int gx, uint32_t *__restrict__ cnt) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P) return;
    int a, b, c, d;
    cnt[j] = (uint32_t)splat_count(means2d, radii, depths, (int)order[j], W, H, gx, a, b, c, d);
}

__global__ __launch_bounds__(256) void k_emit(int P, const uint32_t *__restrict__ order,
                                              const uint32_t *__restrict__ offs,
                                              const float2 *__restrict__ means2d,
                                              const int *__restrict__ radii,
                                              const float *__restrict__ depths, int W, int H,
                                              int gx, const uint32_t *__restrict__ n_splats,
                                              uint32_t cap, uint32_t *__restrict__ tkey,
                                              uint32_t *__restrict__ tid) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P) return;
    if (*n_splats > cap) return;  // overflow: nothing is written
    uint32_t g = order[j];
    int tx0, tx1, ty0, ty1;
    int n = splat_count(means2d, radii, depths, (int)g, W, H, gx, tx0, tx1, ty0, ty1);
    if (n == 0) return;
    uint32_t o = offs[j];
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            tkey[o] = (uint32_t)(ty * gx + tx);
            tid[o] = g;
            ++o;
        }
}

__global__ __launch_bounds__(256) void k_ranges_zero(uint32_t *__restrict__ ranges, int n2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n2) ranges[i] = 0u;
}

__global__ __launch_bounds__(256) void k_ranges(const uint32_t *__restrict__ tkey, Count cnt,
                                                uint32_t *__restrict__ ranges) {
    uint32_t n = cnt.get();
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t t = tkey[i];
    if (i == 0 || tkey[i - 1] != t) ranges[2 * t] = i;
    if (i == n - 1 || tkey[i + 1] != t) ranges[2 * t + 1] = i + 1;
}

// Workspace carve-up (every region 256-byte aligned).
struct Layout {
    size_t dkey0, dkey1, did0, did1, cnt, tkey0, tkey1, tid, hist, part, total;
};

Layout layout(uint32_t P, uint32_t cap) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + (bytes ? bytes : 4), 256);
        return o;
    };
    uint32_t maxn = P > cap ? P : cap;
    uint32_t nblocks = (maxn + SORT_TILE - 1) / SORT_TILE + 1;
    size_t hist_n = (size_t)RADIX * nblocks;
    size_t parts = (hist_n + SORT_TILE - 1) / SORT_TILE + (P + SORT_TILE - 1) / SORT_TILE + 2;
    L.dkey0 = take(4ull * P);
    L.dkey1 = take(4ull * P);
    L.did0 = take(4ull * P);
    L.did1 = take(4ull * P);
    L.cnt = take(4ull * P);
    L.tkey0 = take(4ull * cap);
    L.tkey1 = take(4ull * cap);
    L.tid = take(4ull * cap);
    L.hist = take(4ull * hist_n);
    L.part = take(8ull * parts);
    L.total = off;
    return L;
}

int ceil_log2(uint32_t x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

}  // namespace

extern "C" size_t gs_bin_sort_workspace_bytes(int32_t P, uint32_t capacity, int32_t width,
                                              int32_t height) {
    if (P < 0 || width <= 0 || height <= 0 || width > GS_MAX_DIM || height > GS_MAX_DIM) return 0;
    return layout((uint32_t)P, capacity).total;
}

extern "C" gs_status gs_bin_sort(int32_t P, const float *means2d, const int32_t *radii,
                                 const float *depths, int32_t width, int32_t height,
                                 uint32_t capacity, void *workspace, size_t workspace_bytes,
                                 uint32_t *sorted_ids, uint32_t *tile_ranges,
                                 uint32_t *d_num_splats, void *stream) {
    if (P < 0 || width <= 0 || height <= 0 || width > GS_MAX_DIM || height > GS_MAX_DIM)
        return GS_ERR_INVALID_ARG;
    if (!tile_ranges || !d_num_splats || !workspace || !gs::aligned(workspace, 256) ||
        !gs::aligned(tile_ranges, 4) || !gs::aligned(d_num_splats, 4))
        return GS_ERR_INVALID_ARG;
    if (P > 0 && (!means2d || !radii || !depths || !gs::aligned(means2d, 8) ||
                  !gs::aligned(radii, 4) || !gs::aligned(depths, 4)))
        return GS_ERR_INVALID_ARG;
    if (capacity >= 0x80000000u) return GS_ERR_INVALID_ARG;
    if (capacity > 0 && (!sorted_ids || !gs::aligned(sorted_ids, 4))) return GS_ERR_INVALID_ARG;
    Layout L = layout((uint32_t)P, capacity);
    if (workspace_bytes < L.total) return GS_ERR_CAPACITY;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    auto U = [&](size_t o) { return (uint32_t *)(ws + o); };
    uint64_t *part = (uint64_t *)(ws + L.part);
    int gx = gs::grid_x(width), gy = gs::grid_y(height);
    int ntiles = gx * gy;

    hipLaunchKernelGGL(k_ranges_zero, dim3((2 * ntiles + 255) / 256), dim3(256), 0, s, tile_ranges,
                       2 * ntiles);
    if (P == 0) {
        // N = 0
        hipLaunchKernelGGL(k_ranges_zero, dim3(1), dim3(256), 0, s, d_num_splats, 1);
        return gs::launch_status();
    }
    const float2 *m2 = (const float2 *)means2d;
    int pblocks = (P + 255) / 256;
    // 1. depth order of the Gaussians
    hipLaunchKernelGGL(k_depth_keys, dim3(pblocks), dim3(256), 0, s, P, m2, radii, depths, width,
                       height, gx, U(L.dkey0), U(L.did0));
    SortBufs db{{U(L.dkey0), U(L.dkey1)}, {U(L.did0), U(L.did1)}};
    int dcur = radix_sort(db, Count{(uint32_t)P, nullptr, 0}, (uint32_t)P, 32, U(L.hist), part, s);
    const uint32_t *order = db.v[dcur];
    // 2. counts in depth order, scan, emit
    hipLaunchKernelGGL(k_counts, dim3(pblocks), dim3(256), 0, s, P, order, m2, radii, depths, width,
                       height, gx, U(L.cnt));
    device_scan(U(L.cnt), U(L.cnt), (uint32_t)P, part, d_num_splats, s);
    int tbits = ceil_log2((uint32_t)ntiles);
    if (tbits == 0) tbits = 1;
    int npass = (tbits + RADIX_BITS - 1) / RADIX_BITS;
    // ids are emitted into the buffer that the last tile pass does NOT write,
    // so the sorted ids land in sorted_ids.
    uint32_t *emit_ids = (npass % 2 == 0) ? sorted_ids : U(L.tid);
    uint32_t *other_ids = (npass % 2 == 0) ? U(L.tid) : sorted_ids;
    if (capacity == 0) {
        emit_ids = other_ids = U(L.tid);  // nothing fits; kernels see N > 0 = overflow
    }
    hipLaunchKernelGGL(k_emit, dim3(pblocks), dim3(256), 0, s, P, order, U(L.cnt), m2, radii,
                       depths, width, height, gx, d_num_splats, capacity, U(L.tkey0), emit_ids);
    // 3. stable sort by tile
    SortBufs tb{{U(L.tkey0), U(L.tkey1)}, {emit_ids, other_ids}};
    Count nc{0u, d_num_splats, capacity};
    int tcur = radix_sort(tb, nc, capacity, tbits, U(L.hist), part, s);
    // 4. ranges
    uint32_t rblocks = (capacity + 255) / 256;
    if (rblocks == 0) rblocks = 1;
    hipLaunchKernelGGL(k_ranges, dim3(rblocks), dim3(256), 0, s, tb.k[tcur], nc, tile_ranges);
    return gs::launch_status();
}
