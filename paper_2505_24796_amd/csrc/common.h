// Shared device/host helpers of libgsmfma (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

#define GS_TILE 16
#define GS_TILE_PIX 256
#define GS_MAX_DIM 16384
// Centres with |coordinate| >= 2^22 are not binned; radii are clamped to 2^22.
#define GS_COORD_LIMIT 4194304.0f
#define GS_RADIUS_LIMIT 4194304

namespace gs {

__host__ __device__ inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline int grid_x(int W) { return (W + GS_TILE - 1) / GS_TILE; }
inline int grid_y(int H) { return (H + GS_TILE - 1) / GS_TILE; }

inline gs_status launch_status() {
    return hipGetLastError() == hipSuccess ? GS_OK : GS_ERR_HIP;
}

// Inclusive tile rectangle met by the pixel box [floor(m) - r, floor(m) + r]
// (clamped to the image).  Returns the tile count, 0 when nothing is covered.
// All arithmetic is exact: floor of a float is exact, |floor(m)| < 2^22 and
// r <= 2^22 keep every integer below 2^23.
__device__ __forceinline__ int tile_rect(float mx, float my, int r, int W, int H, int gx,
                                         int &tx0, int &tx1, int &ty0, int &ty1) {
    if (r <= 0 || !(fabsf(mx) < GS_COORD_LIMIT) || !(fabsf(my) < GS_COORD_LIMIT)) return 0;
    r = min(r, GS_RADIUS_LIMIT);
    int fx = (int)floorf(mx), fy = (int)floorf(my);
    int x0 = fx - r, x1 = fx + r, y0 = fy - r, y1 = fy + r;
    if (x1 < 0 || y1 < 0 || x0 > W - 1 || y0 > H - 1) return 0;
    x0 = max(x0, 0);
    y0 = max(y0, 0);
    x1 = min(x1, W - 1);
    y1 = min(y1, H - 1);
    tx0 = x0 / GS_TILE;
    tx1 = x1 / GS_TILE;
    ty0 = y0 / GS_TILE;
    ty1 = y1 / GS_TILE;
    (void)gx;
    return (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
}

// Popcount of the bits of `mask` held by lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Tile visited by workgroup `b` of a launch over the gx x gy tiles.
// Workgroups are dispatched to the 8 XCDs round-robin (b -> XCD b mod 8),
// and each XCD has its own L2.  The row-major tile sequence is cut into
// 8 m chunks of c consecutive tiles (about `rows` tile rows each, 1 or 2:
// m = ceil(ceil(gy / rows) / 8) rounds of 8), and chunk k is served by XCD
// k mod 8.
// A Gaussian that spans neighbouring tiles is then mostly fetched into one
// XCD's L2, every XCD gets a spread of light and heavy image regions, and
// every XCD gets the same number of tiles (whole two-row bands would give
// some XCDs a band more than others: 1200 against 960 tiles at 1920x1080).
// Returns -1 for padding workgroups.
__host__ __device__ inline void xcd_chunks(int gx, int gy, int rows, int &m, int &c) {
    const int nbands = (gy + rows - 1) / rows;
    m = (nbands + 7) / 8;
    const int ntiles = gx * gy;
    c = (ntiles + 8 * m - 1) / (8 * m);
}
__host__ __device__ inline int xcd_grid_blocks(int gx, int gy, int rows = 2) {
    int m, c;
    xcd_chunks(gx, gy, rows, m, c);
    return 8 * m * c;
}
__device__ __forceinline__ int xcd_tile(int b, int gx, int gy, int rows = 2) {
    int m, c;
    xcd_chunks(gx, gy, rows, m, c);
    const int xcd = b & 7, j = b >> 3;
    const int t = ((j / c) * 8 + xcd) * c + j % c;
    return t < gx * gy ? t : -1;
}

}  // namespace gs
