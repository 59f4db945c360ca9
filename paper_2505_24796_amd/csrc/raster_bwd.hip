// Backward of the tile alpha-blending (TC-GS paper, Sec. 3.1, Algorithm 1):
// gradients of a loss with respect to means2D, conics, opacities and colours
// given dL/dC per pixel, by reverse traversal of each pixel's blended
// fragments with the transmittance recovered by division (T_k = T_{k+1} /
// (1 - a_k), well conditioned because a <= 0.99) instead of stored.
//
// For the blended fragments k of a pixel,
//   C_out = sum_k c_k a_k T_k + T_final bg,
//   dC_out/dc_k = a_k T_k,
//   dC_out/da_k = T_k (c_k - B_k),  B_{k-1} = a_k c_k + (1 - a_k) B_k,
//   B_last = bg,
// and a = min(0.99, exp(beta)), beta = ln o - 1/2 d^T S d (Sec. 4.1), so
// dL/dbeta = a dL/da (zero where the clamp is active), dbeta/do = 1/o,
// dbeta/dmu' = -S d, dbeta/d(s11, s12, s22) = -1/2 (dx^2, 2 dx dy, dy^2),
// d = mu' - p.
//
// The fragments are re-evaluated with exactly the forward's arithmetic (the
// same expression for the FP32 paths, the same staged V rows, per-tile cull
// and matrix-core products for the FP16/BF16 paths), so every cull and
// termination decision agrees with the forward.  Per splat, the 256 pixel
// contributions are summed with DPP wave reductions, across the 4 waves in
// LDS, and added to the gradient arrays with one atomic per value per tile.
#include "raster_common.h"

namespace {

constexpr int NGRAD = 9;  // dmu(2), dconic(3), dopacity, dcolour(3)

// Sum over the 64 lanes with DPP (result in lane 63).  All lanes must be
// active.
__device__ __forceinline__ float wave_sum(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));  // quad [1,0,3,2]
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));  // quad [2,3,0,1]
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false)); // row_half_mirror
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false)); // row_mirror
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xA, 0xF, false)); // row_bcast:15
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xC, 0xF, false)); // row_bcast:31
    return x;
}

struct BwdArgs {
    RasterArgs f;  // forward inputs (out_* unused)
    const float *out_T;
    const uint32_t *out_nc;
    const float *dimg;
    float *g_mu, *g_conic, *g_opac, *g_rgb;
};

// Per-lane state of the reverse traversal.
struct PixState {
    float T, B0, B1, B2, d0, d1, d2;
    uint32_t nc;
};

__device__ __forceinline__ PixState load_pixel(const BwdArgs &a, int px, int py) {
    PixState s;
    if (px < a.f.W && py < a.f.H) {
        size_t pi = (size_t)py * a.f.W + px, hw = (size_t)a.f.W * a.f.H;
        s.T = a.out_T[pi];
        s.nc = a.out_nc[pi];
        s.d0 = a.dimg[pi];
        s.d1 = a.dimg[hw + pi];
        s.d2 = a.dimg[2 * hw + pi];
    } else {
        s.T = 1.0f;
        s.nc = 0;
        s.d0 = s.d1 = s.d2 = 0.0f;
    }
    s.B0 = a.f.bg0;
    s.B1 = a.f.bg1;
    s.B2 = a.f.bg2;
    return s;
}

// Sums of eight per-lane values over the wave, transposed: on return lane L
// holds the wave total of v[4 b3 + 2 b4 + b5], (b3, b4, b5) = bits 3..5 of L.
// Each exchange step halves the values a lane carries: v_permlane32_swap
// pairs lanes L and L ^ 32 (lower half keeps the even member of each pair),
// v_permlane16_swap pairs L and L ^ 16, a DPP row rotate by 8 pairs L and
// L ^ 8; the last three steps sum over the 8 lanes of equal bits 3..5.
// 18 instructions for 8 sums instead of 8 x 12.
__device__ __forceinline__ float wave_sum8_transposed(const float v[8]) {
    const int lane = threadIdx.x & 63;
    float w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * j]),
                                                        __float_as_uint(v[2 * j + 1]), false, false);
        w[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);  // v[2j + b5]
    }
    float x[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w[2 * j]),
                                                        __float_as_uint(w[2 * j + 1]), false, false);
        x[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);  // v[4j + 2 b4 + b5]
    }
    const bool b3 = (lane >> 3) & 1;
    const float keep = b3 ? x[1] : x[0], send = b3 ? x[0] : x[1];
    float y = keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), 0x128, 0xF,
                                                                0xF, false));  // row_ror:8 = L ^ 8
    y += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), 0xB1, 0xF, 0xF, false));
    y += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), 0x4E, 0xF, 0xF, false));
    y += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), 0x141, 0xF, 0xF, false));
    return y;
}

// One fragment's contribution (zero unless `bl`), reduced over the wave and
// added to s_grad[NGRAD] by lane 63; updates the lane's T and B when `bl`.
// dL/dbeta = a dL/da, or 0 where the 0.99 clamp is active.
__device__ __forceinline__ void fragment_grad(PixState &ps, bool bl, float alpha, bool clamped,
                                              float4 col, float mx, float my, float s11, float s12,
                                              float s22, float inv_o, float fx, float fy,
                                              float *s_grad) {
    float g[NGRAD];
    // T before this fragment (1 - alpha >= 0.01: a reciprocal-based divide
    // of ~1 ulp is ample for the gradient)
    float Tk = __fdividef(ps.T, 1.0f - alpha);
    float da = ps.d0 * (col.x - ps.B0) + ps.d1 * (col.y - ps.B1) + ps.d2 * (col.z - ps.B2);
    da *= Tk;
    // lanes that do not blend this fragment contribute zero
    const float wT = bl ? alpha * Tk : 0.0f;
    const float dbeta = (clamped || !bl) ? 0.0f : da * alpha;
    float dx = mx - fx, dy = my - fy;
    g[0] = -dbeta * (s11 * dx + s12 * dy);
    g[1] = -dbeta * (s12 * dx + s22 * dy);
    g[2] = -0.5f * dbeta * dx * dx;
    g[3] = -dbeta * dx * dy;
    g[4] = -0.5f * dbeta * dy * dy;
    g[5] = dbeta * inv_o;  // dbeta/do = 1/o
    g[6] = ps.d0 * wT;
    g[7] = ps.d1 * wT;
    g[8] = ps.d2 * wT;
    if (bl) {
        ps.B0 = alpha * col.x + (1.0f - alpha) * ps.B0;
        ps.B1 = alpha * col.y + (1.0f - alpha) * ps.B1;
        ps.B2 = alpha * col.z + (1.0f - alpha) * ps.B2;
        ps.T = Tk;
    }
    const int lane = threadIdx.x & 63;
    const float t8 = wave_sum8_transposed(g);
    const float t9 = wave_sum(g[8]);
    if ((lane & 7) == 0) {
        // lane 8q holds the total of gradient 4 (q & 1) + 2 ((q >> 1) & 1) + (q >> 2)
        const int q = lane >> 3;
        atomicAdd(&s_grad[4 * (q & 1) + 2 * ((q >> 1) & 1) + (q >> 2)], t8);
    }
    if (lane == 63) atomicAdd(&s_grad[8], t9);
}

// Device-memory float adds (the gradient arrays are ordinary device
// allocations, so the hardware float atomics apply).
__device__ __forceinline__ void gadd(float *p, float v) {
    if (v != 0.f) unsafeAtomicAdd(p, v);
}

__device__ __forceinline__ void flush_grads(const BwdArgs &a, const float *gr, uint32_t id) {
    gadd(&a.g_mu[2 * id], gr[0]);
    gadd(&a.g_mu[2 * id + 1], gr[1]);
    gadd(&a.g_conic[3 * id], gr[2]);
    gadd(&a.g_conic[3 * id + 1], gr[3]);
    gadd(&a.g_conic[3 * id + 2], gr[4]);
    gadd(&a.g_opac[id], gr[5]);
    gadd(&a.g_rgb[3 * id], gr[6]);
    gadd(&a.g_rgb[3 * id + 1], gr[7]);
    gadd(&a.g_rgb[3 * id + 2], gr[8]);
}

// Largest n_contrib of the tile (the reverse traversal starts there).
__device__ __forceinline__ uint32_t tile_max_nc(uint32_t nc, uint32_t *s_max) {
    if (threadIdx.x == 0) *s_max = 0u;
    __syncthreads();
    uint32_t m = nc;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(s_max, m);
    __syncthreads();
    return *s_max;
}

// ---------------------------------------------------------------------------
// FP32 paths: the fragment is re-evaluated exactly as k_raster_fp32 does.
// ---------------------------------------------------------------------------
template <bool EARLY>
__global__ __launch_bounds__(256) void k_raster_bwd_fp32(BwdArgs a) {
    __shared__ float2 s_mu[BATCH];
    __shared__ float4 s_co[BATCH];   // s11, s12, s22, o (or ln o with EARLY)
    __shared__ float4 s_rgb[BATCH];  // r, g, b, o
    __shared__ uint32_t s_id[BATCH];
    __shared__ float s_grad[BATCH][NGRAD];
    __shared__ uint32_t s_max;
    int tile = gs::xcd_tile(blockIdx.x, a.f.gx, a.f.gy);
    if (tile < 0) return;
    const int tx = tile % a.f.gx, ty = tile / a.f.gx;
    const int px = tx * GS_TILE + (threadIdx.x & 15), py = ty * GS_TILE + (threadIdx.x >> 4);
    const bool inside = px < a.f.W && py < a.f.H;
    const float fx = (float)px, fy = (float)py;
    PixState ps = load_pixel(a, px, py);
    const uint32_t last = tile_max_nc(ps.nc, &s_max);
    const uint32_t start = a.f.ranges[2 * tile], end = a.f.ranges[2 * tile + 1];
    const uint32_t nscan = min(end - start, last);
    const int nb = (int)((nscan + BATCH - 1) / BATCH);
    for (int b = nb - 1; b >= 0; --b) {
        __syncthreads();
        const uint32_t j0 = (uint32_t)b * BATCH;
        const uint32_t cnt = min((uint32_t)BATCH, nscan - j0);
        if (threadIdx.x < cnt) {
            uint32_t id = a.f.ids[start + j0 + threadIdx.x];
            s_mu[threadIdx.x] = a.f.means2d[id];
            const float lno = a.f.lno[id];
            const Float3 c3 = *(const Float3 *)(a.f.conics + 3 * (size_t)id);
            const Float3 k3 = *(const Float3 *)(a.f.rgb + 3 * (size_t)id);
            // the forward's staging exactly: ln o, or o = exp(ln o)
            s_co[threadIdx.x] = make_float4(c3.x, c3.y, c3.z, EARLY ? lno : __expf(lno));
            s_rgb[threadIdx.x] = make_float4(k3.x, k3.y, k3.z, __expf(-lno));
            s_id[threadIdx.x] = id;
        }
#pragma unroll
        for (int k = 0; k < NGRAD; ++k) s_grad[threadIdx.x][k] = 0.0f;
        __syncthreads();
        for (int j = (int)cnt - 1; j >= 0; --j) {
            const uint32_t pos = j0 + (uint32_t)j + 1u;
            const float2 m = s_mu[j];
            const float4 c = s_co[j];
            const float dx = m.x - fx, dy = m.y - fy;
            const float power = -0.5f * (c.x * dx * dx + c.z * dy * dy) - c.y * dx * dy;
            float araw, alpha;
            bool kept;
            if (EARLY) {
                float beta = c.w + power;
                kept = !(beta < CULL_LN);
                araw = __expf(beta);
            } else {
                araw = c.w * __expf(power);
                kept = !(fminf(ALPHA_MAX, araw) < CULL_ALPHA);
            }
            alpha = fminf(ALPHA_MAX, araw);
            const bool bl = inside && kept && pos <= ps.nc;
            if (__ballot(bl) != 0ull) {
                const float4 col = s_rgb[j];
                fragment_grad(ps, bl, alpha, araw > ALPHA_MAX, col, m.x, m.y, c.x, c.y, c.z, col.w,
                              fx, fy, s_grad[j]);
            }
        }
        __syncthreads();
        if (threadIdx.x < cnt) flush_grads(a, s_grad[threadIdx.x], s_id[threadIdx.x]);
    }
}

// ---------------------------------------------------------------------------
// Matrix-core paths: the same staging (per-tile cull, compaction, V rows) and
// the same products as k_raster_mfma, walked in reverse.
// At least 5 waves per SIMD (86 VGPRs for the FP16 split; 4 waves at the
// 120 the compiler otherwise takes were 3 % slower).
// ---------------------------------------------------------------------------
template <int VAR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_raster_bwd_mfma(BwdArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[Stage<VAR>::BYTES];
    __shared__ float4 s_p0[BATCH];   // mu'x, mu'y, s11, s12
    __shared__ float4 s_p1[BATCH];   // s22, 1/o, id, -
    __shared__ float s_grad[BATCH][NGRAD];
    __shared__ int s_wcnt[4];
    __shared__ uint32_t s_max;
    int tile = gs::xcd_tile(blockIdx.x, a.f.gx, a.f.gy);
    if (tile < 0) return;
    const int tx = tile % a.f.gx, ty = tile / a.f.gx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int qx = (wave & 1) * 8, qy = (wave >> 1) * 8;
    const int px = tx * GS_TILE + qx + (lane & 7), py = ty * GS_TILE + qy + (lane >> 3);
    const float fx = (float)px, fy = (float)py;
    const float ox = VarTraits<VAR>::LOCAL ? tx * GS_TILE + 7.5f : 0.0f;
    const float oy = VarTraits<VAR>::LOCAL ? ty * GS_TILE + 7.5f : 0.0f;
    const float bx0 = (float)(tx * GS_TILE), by0 = (float)(ty * GS_TILE);
    UOperand u0, u1;
    {
        int j = lane & 31, slice = lane >> 5;
        float bx = (float)(tx * GS_TILE + qx + (j & 7)) - ox;
        float by = (float)(ty * GS_TILE + qy + (j >> 3)) - oy;
        u0 = make_u<VAR>(bx, by, slice);
        u1 = make_u<VAR>(bx, by + 4.0f, slice);
    }
    const bool inside = px < a.f.W && py < a.f.H;
    const float thr = inside ? CULL_LOG2 : __builtin_inff();
    PixState ps = load_pixel(a, px, py);
    const uint32_t last = tile_max_nc(ps.nc, &s_max);
    const uint32_t start = a.f.ranges[2 * tile], end = a.f.ranges[2 * tile + 1];
    const uint32_t nscan = min(end - start, last);
    const int nb = (int)((nscan + BATCH - 1) / BATCH);
    const float4 *rgbs = (const float4 *)(stage + Stage<VAR>::A1 + Stage<VAR>::A2);
    // the splat ids of each batch are loaded one round ahead (one register;
    // gathering the whole next batch ahead measured no better)
    uint32_t id_next = 0u;
    if (nb > 0) {
        const uint32_t q = (uint32_t)(nb - 1) * BATCH + threadIdx.x;
        id_next = q < nscan ? a.f.ids[start + q] : 0u;
    }
    for (int b = nb - 1; b >= 0; --b) {
        // splats of batch b (only positions up to the tile's last blended one
        // can contribute; the staging of the rest matches the forward's)
        const bool in_scan = (uint32_t)b * BATCH + threadIdx.x < nscan;
        const uint32_t my_id = id_next;
        SplatRegs cur = gather(a.f, my_id, in_scan);
        if (b > 0) {
            const uint32_t q = (uint32_t)(b - 1) * BATCH + threadIdx.x;
            id_next = q < nscan ? a.f.ids[start + q] : 0u;
        }
        const bool keep = tile_alive(cur, bx0, by0);
        const uint64_t kmask = __ballot(keep);
        __syncthreads();  // previous batch fully consumed
        if (lane == 0) s_wcnt[wave] = __popcll(kmask);
#pragma unroll
        for (int k = 0; k < NGRAD; ++k) s_grad[threadIdx.x][k] = 0.0f;
        __syncthreads();
        int wofs = 0, total = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int c = s_wcnt[i];
            wofs += i < wave ? c : 0;
            total += c;
        }
        if (keep) {
            const int jj = wofs + (int)gs::lanes_below(kmask);
            stage_splat<VAR>(stage, jj, cur, ox, oy, (uint32_t)b * BATCH + threadIdx.x);
            s_p0[jj] = make_float4(cur.mu.x, cur.mu.y, cur.s11, cur.s12);
            s_p1[jj] = make_float4(cur.s22, __expf(-cur.lno), __uint_as_float(my_id), 0.0f);
        }
        __syncthreads();
        const int nsub = (total + SUB - 1) / SUB;
        for (int sidx = nsub - 1; sidx >= 0; --sidx) {
            float lo[16], hi[16];
            exponents<VAR>(stage + sidx * SUB * VarTraits<VAR>::ROW1,
                           stage + Stage<VAR>::A1 + sidx * SUB * VarTraits<VAR>::ROW2, u0, u1, lane,
                           lo, hi);
            const uint32_t scount = min((uint32_t)SUB, (uint32_t)total - (uint32_t)sidx * SUB);
            const uint32_t valid = scount >= 32u ? 0xFFFFFFFFu : ((1u << scount) - 1u);
#pragma unroll
            for (int g = SUB - 1; g >= 0; --g) {
                if (!((valid >> g) & 1u)) continue;
                const int j = sidx * SUB + g;
                const float beta = g < 16 ? lo[g] : hi[g - 16];
                const float4 col = rgbs[j];
                const uint32_t pos = __float_as_uint(col.w);  // 1-based list position
                const bool bl = beta >= thr && pos <= ps.nc;
                if (__ballot(bl) != 0ull) {
                    const float araw = __builtin_amdgcn_exp2f(beta);
                    const float4 p0 = s_p0[j], p1 = s_p1[j];
                    fragment_grad(ps, bl, fminf(ALPHA_MAX, araw), araw > ALPHA_MAX, col, p0.x, p0.y,
                                  p0.z, p0.w, p1.x, p1.y, fx, fy, s_grad[j]);
                }
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < total)
            flush_grads(a, s_grad[threadIdx.x], __float_as_uint(s_p1[threadIdx.x].z));
    }
}

}  // namespace

extern "C" gs_status gs_rasterize_bwd(int32_t width, int32_t height, const uint32_t *tile_ranges,
                                      const uint32_t *sorted_ids, const float *means2d,
                                      const float *conics, const float *log_opacities,
                                      const float *rgb, const float *background, int32_t precision,
                                      const float *out_T, const uint32_t *out_ncontrib,
                                      const float *dL_dimg, float *dL_dmeans2d,
                                      float *dL_dconics, float *dL_dopacities, float *dL_drgb,
                                      void *stream) {
    const void *ptrs[] = {tile_ranges, sorted_ids, means2d, conics, log_opacities, rgb, out_T,
                          out_ncontrib, dL_dimg, dL_dmeans2d, dL_dconics, dL_dopacities, dL_drgb};
    if (!valid_inputs(width, height, ptrs, 13) || !gs::aligned(means2d, 8)) return GS_ERR_INVALID_ARG;
    if (precision < GS_PREC_FP32 || precision > GS_PREC_BF16_G2L_SPLIT) return GS_ERR_INVALID_ARG;
    BwdArgs a{};
    a.f.chunk_rows = 2;
    a.f.W = width;
    a.f.H = height;
    a.f.gx = gs::grid_x(width);
    a.f.gy = gs::grid_y(height);
    a.f.ranges = tile_ranges;
    a.f.ids = sorted_ids;
    a.f.means2d = (const float2 *)means2d;
    a.f.conics = conics;
    a.f.lno = log_opacities;
    a.f.rgb = rgb;
    a.f.bg0 = background ? background[0] : 0.f;
    a.f.bg1 = background ? background[1] : 0.f;
    a.f.bg2 = background ? background[2] : 0.f;
    a.out_T = out_T;
    a.out_nc = out_ncontrib;
    a.dimg = dL_dimg;
    a.g_mu = dL_dmeans2d;
    a.g_conic = dL_dconics;
    a.g_opac = dL_dopacities;
    a.g_rgb = dL_drgb;
    hipStream_t s = (hipStream_t)stream;
    int blocks = gs::xcd_grid_blocks(a.f.gx, a.f.gy);
    switch (precision) {
    case GS_PREC_FP32: hipLaunchKernelGGL(k_raster_bwd_fp32<false>, dim3(blocks), dim3(256), 0, s, a); break;
    case GS_PREC_FP32_EARLYCULL: hipLaunchKernelGGL(k_raster_bwd_fp32<true>, dim3(blocks), dim3(256), 0, s, a); break;
    case GS_PREC_FP16_GLOBAL: hipLaunchKernelGGL(k_raster_bwd_mfma<VAR_F16_GLOBAL>, dim3(blocks), dim3(256), 0, s, a); break;
    case GS_PREC_FP16_G2L: hipLaunchKernelGGL(k_raster_bwd_mfma<VAR_F16_G2L>, dim3(blocks), dim3(256), 0, s, a); break;
    case GS_PREC_FP16_G2L_SPLIT: hipLaunchKernelGGL(k_raster_bwd_mfma<VAR_F16_SPLIT>, dim3(blocks), dim3(256), 0, s, a); break;
    case GS_PREC_BF16_G2L_SPLIT: hipLaunchKernelGGL(k_raster_bwd_mfma<VAR_BF16_SPLIT>, dim3(blocks), dim3(256), 0, s, a); break;
    }
    return gs::launch_status();
}
