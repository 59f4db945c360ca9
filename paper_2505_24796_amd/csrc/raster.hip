// Conditional alpha-blending per 16x16 tile (TC-GS paper, Sec. 3.1,
// Algorithm 1) in two forms:
//
//  * k_raster_fp32: Algorithm 1 literally on the vector ALUs, one pixel per
//    lane, the tile's splats staged through LDS 256 at a time.  With EARLY the
//    1/255 test is made on the exponent before exp (EarlyCull, Sec. 4.1).
//
//  * k_raster_mfma: the exponent matrix B = U^T V (Frag2Mat, Sec. 4.2) of
//    256 pixels x 32 splats on the matrix cores, in tile-local coordinates
//    (G2L, Sec. 4.3), then EarlyCull and blending on the vector ALUs; the
//    per-tile body is raster_tile_mfma (raster_tile.h).
#include "raster_tile.h"


namespace {

// ---------------------------------------------------------------------------
// Plain FP32 kernel
// ---------------------------------------------------------------------------
// Without NC the last composited position is not tracked (out_ncontrib NULL).
template <bool EARLY, bool COUNT, bool NC = true>
__global__ __launch_bounds__(256) void k_raster_fp32(RasterArgs a) {
    __shared__ float2 s_mu[BATCH];
    __shared__ float4 s_co[BATCH];  // s11, s12, s22, o (ln o with EARLY)
    __shared__ float4 s_rgb[BATCH];
    int tile = gs::xcd_tile(blockIdx.x, a.gx, a.gy, a.chunk_rows);
    if (tile < 0) return;
    int tx = tile % a.gx, ty = tile / a.gx;
    int px = tx * GS_TILE + (threadIdx.x & 15), py = ty * GS_TILE + (threadIdx.x >> 4);
    bool done = !(px < a.W && py < a.H);
    uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    float fx = (float)px, fy = (float)py;
    float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    uint32_t last = 0, nb = 0, nc = 0, nt = 0;
    for (uint32_t b0 = start; b0 < end; b0 += BATCH) {
        if (__syncthreads_count(done) == BATCH) break;
        uint32_t k = b0 + threadIdx.x;
        if (k < end) {
            uint32_t id = a.ids[k];
            s_mu[threadIdx.x] = a.means2d[id];
            const float lno = a.lno[id];
            const Float3 c3 = *(const Float3 *)(a.conics + 3 * (size_t)id);
            const Float3 k3 = *(const Float3 *)(a.rgb + 3 * (size_t)id);
            s_co[threadIdx.x] = make_float4(c3.x, c3.y, c3.z, EARLY ? lno : __expf(lno));
            s_rgb[threadIdx.x] = make_float4(k3.x, k3.y, k3.z, 0.f);
        }
        __syncthreads();
        int cnt = (int)min((uint32_t)BATCH, end - b0);
        if (EARLY) {
            // EarlyCull at wave level: the exponent beta = ln o - q/2 is
            // tested against -ln 255 first; the exp and the blend run only
            // for splats that survive at some pixel of the wave (a uniform
            // branch on the ballot), masked per lane; a wave whose pixels
            // have all stopped leaves the round
            for (int j = 0; j < cnt; ++j) {
                const bool alive = !done;
                float2 m = s_mu[j];
                float4 c = s_co[j];
                float dx = m.x - fx, dy = m.y - fy;
                float power = -0.5f * (c.x * dx * dx + c.z * dy * dy) - c.y * dx * dy;
                float beta = c.w + power;
                const bool culled = beta < CULL_LN;
                const bool keep = alive && !culled;
                if (COUNT) nc += (alive && culled) ? 1u : 0u;
                if (__ballot(keep) == 0) {
                    if (__ballot(alive) == 0) break;
                    continue;
                }
                float alpha = fminf(ALPHA_MAX, __expf(beta));
                float test = fmaf(-alpha, T, T);
                const bool stop = keep && test < T_MIN;
                const bool blend = keep && !stop;
                if (stop) {
                    done = true;
                    if (COUNT) nt = 1;
                }
                if (blend) {
                    float w = alpha * T;
                    float4 col = s_rgb[j];
                    C0 = fmaf(col.x, w, C0);
                    C1 = fmaf(col.y, w, C1);
                    C2 = fmaf(col.z, w, C2);
                    T = test;
                    if (NC) last = b0 - start + (uint32_t)j + 1u;
                    if (COUNT) ++nb;
                }
            }
        } else if (!done) {
            // Algorithm 1 as written, per lane: alpha = o exp(-q/2), then the
            // 1/255 test
            for (int j = 0; j < cnt; ++j) {
                float2 m = s_mu[j];
                float4 c = s_co[j];
                float dx = m.x - fx, dy = m.y - fy;
                float power = -0.5f * (c.x * dx * dx + c.z * dy * dy) - c.y * dx * dy;
                float alpha = fminf(ALPHA_MAX, c.w * __expf(power));
                if (alpha < CULL_ALPHA) {
                    if (COUNT) ++nc;
                    continue;
                }
                float test = fmaf(-alpha, T, T);
                if (test < T_MIN) {
                    done = true;
                    if (COUNT) nt = 1;
                    break;
                }
                float w = alpha * T;
                float4 col = s_rgb[j];
                C0 = fmaf(col.x, w, C0);
                C1 = fmaf(col.y, w, C1);
                C2 = fmaf(col.z, w, C2);
                T = test;
                if (NC) last = b0 - start + (uint32_t)j + 1u;
                if (COUNT) ++nb;
            }
        }
    }
    write_pixel(a, px, py, C0, C1, C2, T, last);
    if (COUNT) add_counters(a.counters, nb, nc, nt);
}


// At least 5 resident waves per SIMD (the compiler then fits the kernel in
// <= 80 VGPRs, i.e. 6 waves): the blend's exp / LDS / gather latencies are
// hidden by other waves rather than by instruction-level parallelism.  NB
// splats are gathered and staged per round (64, 128 or 256; the default
// launch takes 128, the tuned one what an autotuner picked).
constexpr int DEFAULT_NB = 128;
template <int VAR, bool COUNT, int NB, bool NC = true, bool CULL = true>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_raster_mfma(RasterArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[Stage<VAR, NB>::BYTES];
    __shared__ TileShared sh;
    const int tile = gs::xcd_tile(blockIdx.x, a.gx, a.gy, a.chunk_rows);
    if (tile < 0) return;
    raster_tile_mfma<VAR, COUNT, NB, NC, CULL>(a, tile, stage, sh);
}

// Diagnostic: exponents of the first `count` splats of one tile.
template <int VAR>
__global__ __launch_bounds__(256) void k_beta_dump(RasterArgs a, int tile, int count, float *out) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[Stage<VAR>::BYTES];
    const int tx = tile % a.gx, ty = tile / a.gx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int qx = (wave & 1) * 8, qy = (wave >> 1) * 8;
    const float ox = VarTraits<VAR>::LOCAL ? tx * GS_TILE + 7.5f : 0.0f;
    const float oy = VarTraits<VAR>::LOCAL ? ty * GS_TILE + 7.5f : 0.0f;
    UOperand u0, u1;
    {
        int j = lane & 31, slice = lane >> 5;
        float bx = (float)(tx * GS_TILE + qx + (j & 7)) - ox;
        float by0 = (float)(ty * GS_TILE + qy + (j >> 3)) - oy;
        u0 = make_u<VAR>(bx, by0, slice);
        u1 = make_u<VAR>(bx, by0 + 4.0f, slice);
    }
    const int pix = (qy + (lane >> 3)) * GS_TILE + qx + (lane & 7);
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const uint32_t n = end - start;
    for (int b0 = 0; b0 < count; b0 += BATCH) {
        uint32_t k = start + b0 + threadIdx.x;
        bool valid = (uint32_t)(b0 + threadIdx.x) < n;
        uint32_t id = valid ? a.ids[k] : 0u;
        __syncthreads();
        stage_splat<VAR>(stage, threadIdx.x, gather(a, id, valid), ox, oy, b0 + threadIdx.x);
        __syncthreads();
        for (int sidx = 0; sidx < BATCH / SUB && b0 + sidx * SUB < count; ++sidx) {
            float lo[16], hi[16];
            exponents<VAR>(stage + sidx * SUB * VarTraits<VAR>::ROW1,
                           stage + Stage<VAR>::A1 + sidx * SUB * VarTraits<VAR>::ROW2, u0, u1, lane,
                           lo, hi);
#pragma unroll
            for (int g = 0; g < 32; ++g) {
                int row = b0 + sidx * SUB + g;
                if (row < count) {
                    float v = g < 16 ? lo[g] : hi[g - 16];
                    out[(size_t)row * GS_TILE_PIX + pix] = (uint32_t)row < n ? v : __builtin_nanf("");
                }
            }
        }
    }
}

// Counting launches (diagnostics) always take the default batch and track
// the last composited position; they already stage and visit every listed
// splat (to count its fragments), so CULL does not apply to them.
template <int VAR, bool NC, bool CULL>
void launch_mfma_nb(const RasterArgs &a, int blocks, int nb, hipStream_t s) {
    switch (nb) {
    case 64: hipLaunchKernelGGL((k_raster_mfma<VAR, false, 64, NC, CULL>), dim3(blocks), dim3(256), 0, s, a); break;
    case 256: hipLaunchKernelGGL((k_raster_mfma<VAR, false, 256, NC, CULL>), dim3(blocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_raster_mfma<VAR, false, 128, NC, CULL>), dim3(blocks), dim3(256), 0, s, a); break;
    }
}
template <int VAR, bool CULL = true>
void launch_mfma(const RasterArgs &a, int blocks, bool count, int nb, hipStream_t s) {
    if (count)
        hipLaunchKernelGGL((k_raster_mfma<VAR, true, DEFAULT_NB>), dim3(blocks), dim3(256), 0, s, a);
    else if (a.out_nc)
        launch_mfma_nb<VAR, true, CULL>(a, blocks, nb, s);
    else
        launch_mfma_nb<VAR, false, CULL>(a, blocks, nb, s);
}

}  // namespace

extern "C" gs_status gs_rasterize_fwd_tuned(int32_t width, int32_t height,
                                            const uint32_t *tile_ranges, const uint32_t *sorted_ids,
                                            const float *means2d, const float *conics,
                                            const float *log_opacities, const float *rgb,
                                            const float *background, int32_t precision,
                                            const gs_raster_tune *tune, float *out_rgb,
                                            float *out_T, uint32_t *out_ncontrib,
                                            uint64_t *d_counters, void *stream) {
    const void *ptrs[] = {tile_ranges, sorted_ids, means2d, conics, log_opacities, rgb, out_rgb, out_T};
    if (!valid_inputs(width, height, ptrs, 8) || !gs::aligned(means2d, 8)) return GS_ERR_INVALID_ARG;
    if (out_ncontrib && !gs::aligned(out_ncontrib, 4)) return GS_ERR_INVALID_ARG;
    if (d_counters && !gs::aligned(d_counters, 8)) return GS_ERR_INVALID_ARG;
    if (precision < GS_PREC_FP32 || precision > GS_PREC_FP16_G2L_SPLIT_NOCULL) return GS_ERR_INVALID_ARG;
    const int nb = tune ? tune->batch : DEFAULT_NB;
    const int rows = tune ? tune->chunk_rows : 2;
    if (!(nb == 64 || nb == 128 || nb == 256) || !(rows == 1 || rows == 2)) return GS_ERR_INVALID_ARG;
    RasterArgs a;
    a.chunk_rows = rows;
    a.W = width;
    a.H = height;
    a.gx = gs::grid_x(width);
    a.gy = gs::grid_y(height);
    a.ranges = tile_ranges;
    a.ids = sorted_ids;
    a.means2d = (const float2 *)means2d;
    a.conics = conics;
    a.lno = log_opacities;
    a.rgb = rgb;
    a.bg0 = background ? background[0] : 0.f;
    a.bg1 = background ? background[1] : 0.f;
    a.bg2 = background ? background[2] : 0.f;
    a.out_rgb = out_rgb;
    a.out_T = out_T;
    a.out_nc = out_ncontrib;
    a.counters = (unsigned long long *)d_counters;
    hipStream_t s = (hipStream_t)stream;
    int blocks = gs::xcd_grid_blocks(a.gx, a.gy, rows);
    bool cnt = d_counters != nullptr;
    switch (precision) {
    case GS_PREC_FP32:
        if (cnt) hipLaunchKernelGGL((k_raster_fp32<false, true>), dim3(blocks), dim3(256), 0, s, a);
        else if (out_ncontrib) hipLaunchKernelGGL((k_raster_fp32<false, false>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_raster_fp32<false, false, false>), dim3(blocks), dim3(256), 0, s, a);
        break;
    case GS_PREC_FP32_EARLYCULL:
        if (cnt) hipLaunchKernelGGL((k_raster_fp32<true, true>), dim3(blocks), dim3(256), 0, s, a);
        else if (out_ncontrib) hipLaunchKernelGGL((k_raster_fp32<true, false>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_raster_fp32<true, false, false>), dim3(blocks), dim3(256), 0, s, a);
        break;
    case GS_PREC_FP16_GLOBAL: launch_mfma<VAR_F16_GLOBAL>(a, blocks, cnt, nb, s); break;
    case GS_PREC_FP16_G2L: launch_mfma<VAR_F16_G2L>(a, blocks, cnt, nb, s); break;
    case GS_PREC_FP16_G2L_SPLIT: launch_mfma<VAR_F16_SPLIT>(a, blocks, cnt, nb, s); break;
    case GS_PREC_BF16_G2L_SPLIT: launch_mfma<VAR_BF16_SPLIT>(a, blocks, cnt, nb, s); break;
    case GS_PREC_FP16_G2L_SPLIT_NOCULL: launch_mfma<VAR_F16_SPLIT, false>(a, blocks, cnt, nb, s); break;
    }
    return gs::launch_status();
}

extern "C" gs_status gs_rasterize_fwd(int32_t width, int32_t height, const uint32_t *tile_ranges,
                                      const uint32_t *sorted_ids, const float *means2d,
                                      const float *conics, const float *log_opacities,
                                      const float *rgb, const float *background, int32_t precision,
                                      float *out_rgb, float *out_T, uint32_t *out_ncontrib,
                                      uint64_t *d_counters, void *stream) {
    return gs_rasterize_fwd_tuned(width, height, tile_ranges, sorted_ids, means2d, conics,
                                  log_opacities, rgb, background, precision, nullptr, out_rgb,
                                  out_T, out_ncontrib, d_counters, stream);
}

extern "C" gs_status gs_rasterize_beta(int32_t width, int32_t height, int32_t tile,
                                       const uint32_t *tile_ranges, const uint32_t *sorted_ids,
                                       const float *means2d, const float *conics,
                                       const float *log_opacities, int32_t precision, int32_t count,
                                       float *out_beta, void *stream) {
    const void *ptrs[] = {tile_ranges, sorted_ids, means2d, conics, log_opacities, out_beta};
    if (!valid_inputs(width, height, ptrs, 6) || !gs::aligned(means2d, 8)) return GS_ERR_INVALID_ARG;
    int ntiles = gs::grid_x(width) * gs::grid_y(height);
    if (tile < 0 || tile >= ntiles || count <= 0) return GS_ERR_INVALID_ARG;
    if (precision < GS_PREC_FP16_GLOBAL || precision > GS_PREC_BF16_G2L_SPLIT) return GS_ERR_INVALID_ARG;
    RasterArgs a{};
    a.chunk_rows = 2;
    a.W = width;
    a.H = height;
    a.gx = gs::grid_x(width);
    a.gy = gs::grid_y(height);
    a.ranges = tile_ranges;
    a.ids = sorted_ids;
    a.means2d = (const float2 *)means2d;
    a.conics = conics;
    a.lno = log_opacities;
    a.rgb = log_opacities;  // colours are not needed; any valid pointer
    hipStream_t s = (hipStream_t)stream;
    switch (precision) {
    case GS_PREC_FP16_GLOBAL: hipLaunchKernelGGL(k_beta_dump<VAR_F16_GLOBAL>, dim3(1), dim3(256), 0, s, a, tile, count, out_beta); break;
    case GS_PREC_FP16_G2L: hipLaunchKernelGGL(k_beta_dump<VAR_F16_G2L>, dim3(1), dim3(256), 0, s, a, tile, count, out_beta); break;
    case GS_PREC_FP16_G2L_SPLIT: hipLaunchKernelGGL(k_beta_dump<VAR_F16_SPLIT>, dim3(1), dim3(256), 0, s, a, tile, count, out_beta); break;
    case GS_PREC_BF16_G2L_SPLIT: hipLaunchKernelGGL(k_beta_dump<VAR_BF16_SPLIT>, dim3(1), dim3(256), 0, s, a, tile, count, out_beta); break;
    }
    return gs::launch_status();
}

extern "C" const char *gs_status_string(int status) {
    switch (status) {
    case GS_OK: return "GS_OK";
    case GS_ERR_INVALID_ARG: return "GS_ERR_INVALID_ARG";
    case GS_ERR_UNSUPPORTED: return "GS_ERR_UNSUPPORTED";
    case GS_ERR_HIP: return "GS_ERR_HIP";
    case GS_ERR_CAPACITY: return "GS_ERR_CAPACITY";
    case GS_ERR_NOT_IMPLEMENTED: return "GS_ERR_NOT_IMPLEMENTED";
    default: return "GS_ERR_UNKNOWN";
    }
}

extern "C" int gs_version(void) { return 202; }
