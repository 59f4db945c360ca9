// One 16x16 tile of the matrix-core forward rasteriser (TC-GS paper, Sec. 4:
// Frag2Mat in G2L local coordinates with EarlyCull, blending by Sec. 3.1
// Algorithm 1).  Shared by the one-view kernel (one workgroup per tile) and
// the persistent multi-view kernel (workgroups pull (view, tile) items).
//
// MFMA layout (v_mfma_f32_32x32x{8,16}): rows = 32 splats (operand A = V),
// columns = 32 pixels (operand B = U), FP32 accumulators.  A wave owns one
// 8x8 pixel quadrant of the tile = two 32-pixel column groups, so each
// 32-splat sub-batch costs two MFMAs.  Output lane l of group G holds column
// l%32 and 16 of the 32 rows; rows are assigned to splats so that after one
// v_permlane32_swap per accumulator pair every lane holds the exponents of
// ITS OWN pixel for all 32 splats in depth order: register r of the first
// accumulator = splat r, of the second = splat 16 + r.  Blending then runs
// per lane with no LDS round trip for B.
//
// EarlyCull on SIMD: a splat is visited only if ballot(beta >= -log2 255) is
// non-zero over the wave's 64 pixels; the exp and the blend run only then.
// The coefficients are pre-scaled by log2(e) so alpha = 2^beta (v_exp_f32).
#pragma once

#include "raster_common.h"

namespace {

// LDS a tile needs besides the splat stage.
struct TileShared {
    int wcnt[4];
    int wdone[4];
};

// Renders tile `tile` of view `a` with a workgroup of 256 threads (4 waves).
// NB splats (64, 128 or 256) are gathered and staged per round; every thread
// of the workgroup must call this with the same arguments.  Touches only
// `stage` and `sh` in LDS; the caller separates two calls with a barrier.
// Without NC the position of each pixel's last composited splat is not
// tracked (one vector instruction less per visited splat; for callers that
// do not ask for it).  Without CULL (the EarlyCull-off cell of the paper's
// EarlyCull x Frag2Mat ablation, Sec. 5.3, Table 5) every listed splat is
// staged and visited: no per-tile cull, and the exp and blend run for every
// splat; the per-lane threshold still decides what each pixel composites.
template <int VAR, bool COUNT, int NB, bool NC = true, bool CULL = true>
__device__ __forceinline__ void raster_tile_mfma(const RasterArgs &a, int tile, uint8_t *stage,
                                                 TileShared &sh) {
    static_assert(NB == 64 || NB == 128 || NB == 256, "batch of 64, 128 or 256 splats");
    const int tx = tile % a.gx, ty = tile / a.gx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int qx = (wave & 1) * 8, qy = (wave >> 1) * 8;
    const int px = tx * GS_TILE + qx + (lane & 7), py = ty * GS_TILE + qy + (lane >> 3);
    // frame origin: the tile centre (G2L) or the image origin
    const float ox = VarTraits<VAR>::LOCAL ? tx * GS_TILE + 7.5f : 0.0f;
    const float oy = VarTraits<VAR>::LOCAL ? ty * GS_TILE + 7.5f : 0.0f;
    const float bx0 = (float)(tx * GS_TILE), by0 = (float)(ty * GS_TILE);
    // operand B: column j = lane%32 of group G is pixel (qx + j%8, qy + 4G + j/8)
    UOperand u0, u1;
    {
        int j = lane & 31, slice = lane >> 5;
        float bx = (float)(tx * GS_TILE + qx + (j & 7)) - ox;
        float by = (float)(ty * GS_TILE + qy + (j >> 3)) - oy;
        u0 = make_u<VAR>(bx, by, slice);
        u1 = make_u<VAR>(bx, by + 4.0f, slice);
    }
    // per-lane cull threshold; +inf marks a finished (or out-of-image) pixel
    float thr = (px < a.W && py < a.H) ? CULL_LOG2 : __builtin_inff();
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const uint32_t n = end - start;
    const uint32_t nbatch = (n + NB - 1) / NB;
    float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    uint32_t last = 0, nb = 0, ncl = 0, nt = 0;
    // threads beyond NB take no splat
    const bool gatherer = NB == 256 || (int)threadIdx.x < NB;

    // software pipeline: the geometry (mean, conic, ln o) of batch b+1 and
    // the id of batch b+2 are in flight while batch b is blended; a splat's
    // colour is fetched only once the per-tile cull has kept it
    uint32_t k0 = start + threadIdx.x;
    uint32_t id_cur = gatherer && k0 < end ? a.ids[k0] : 0u;
    SplatRegs cur = gather<false>(a, id_cur, gatherer && k0 < end);
    uint32_t k1 = k0 + NB;
    uint32_t id_next = gatherer && k1 < end ? a.ids[k1] : 0u;

    for (uint32_t b = 0; b < nbatch; ++b) {
        // 1. which splats of the batch can contribute to this tile at all
        // (counting mode keeps every splat so culled fragments are counted
        // per pixel in list order)
        const bool keep = COUNT || !CULL ? cur.valid : tile_alive(cur, bx0, by0);
        // the colours of the kept splats only (most listed splats are culled
        // here); the loads are in flight across the barrier below
        if (keep) load_rgb(a, cur);
        const uint64_t kmask = __ballot(keep);
        const bool wave_done = __ballot(thr != __builtin_inff()) == 0ull;
        if (lane == 0) {
            sh.wcnt[wave] = __popcll(kmask);
            sh.wdone[wave] = wave_done;
        }
        __syncthreads();  // (A) also: every wave has finished the previous batch
        if (sh.wdone[0] & sh.wdone[1] & sh.wdone[2] & sh.wdone[3]) break;
        int wofs = 0, total = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int c = sh.wcnt[i];
            wofs += i < wave ? c : 0;
            total += c;
        }
        // 2. compacted staging of the kept splats (depth order preserved)
        if (keep)
            stage_splat<VAR, NB>(stage, wofs + (int)gs::lanes_below(kmask), cur, ox, oy,
                                 b * NB + threadIdx.x);
        {
            uint32_t kn = start + (b + 1) * NB + threadIdx.x;
            cur = gather<false>(a, id_next, gatherer && kn < end);
            uint32_t kn2 = kn + NB;
            id_next = gatherer && kn2 < end ? a.ids[kn2] : 0u;
        }
        __syncthreads();  // (B) staging visible
        if (wave_done || total == 0) continue;
        const uint32_t nsub = ((uint32_t)total + SUB - 1) / SUB;
        const float4 *rgbs = (const float4 *)(stage + Stage<VAR, NB>::A1 + Stage<VAR, NB>::A2);
        for (uint32_t sidx = 0; sidx < nsub; ++sidx) {
            float lo[16], hi[16];
            exponents<VAR>(stage + sidx * SUB * VarTraits<VAR>::ROW1,
                           stage + Stage<VAR, NB>::A1 + sidx * SUB * VarTraits<VAR>::ROW2, u0, u1,
                           lane, lo, hi);
            const uint32_t scount = min((uint32_t)SUB, (uint32_t)total - sidx * SUB);
            const float4 *cols = rgbs + sidx * SUB;
            // Front-to-back over the 32 splats.  `thr` is the lane's cull
            // threshold, +inf once the pixel has terminated, so one compare
            // both culls and masks finished pixels; a splat is visited only
            // if some lane of the wave survives it (EarlyCull at wave level).
            // The body is branch-free per lane: non-surviving lanes compute
            // but commit nothing.
            const uint32_t valid = scount >= 32u ? 0xFFFFFFFFu : ((1u << scount) - 1u);
#pragma unroll
            for (int g = 0; g < SUB; ++g) {
                if (!((valid >> g) & 1u)) break;
                const float beta = g < 16 ? lo[g] : hi[g - 16];
                const bool sv = beta >= thr;
                if (COUNT) ncl += (thr != __builtin_inff() && !sv) ? 1u : 0u;
                if (COUNT || !CULL || __ballot(sv) != 0ull) {
                    const float4 col = cols[g];
                    const float alpha = fminf(ALPHA_MAX, __builtin_amdgcn_exp2f(beta));
                    const float test = fmaf(-alpha, T, T);
                    // one compare decides both outcomes (test is finite)
                    const bool live = test >= T_MIN;
                    const bool blend = sv && live, stop = sv && !live;
                    // the weight alpha T as the drop in transmittance: zero
                    // for lanes that do not blend, and the weights and the
                    // final T sum to exactly 1
                    const float Tn = blend ? test : T;
                    const float w = T - Tn;
                    C0 = fmaf(col.x, w, C0);
                    C1 = fmaf(col.y, w, C1);
                    C2 = fmaf(col.z, w, C2);
                    T = Tn;
                    if (NC) last = blend ? __float_as_uint(col.w) : last;
                    thr = stop ? __builtin_inff() : thr;
                    if (COUNT) {
                        nb += blend ? 1u : 0u;
                        nt += stop ? 1u : 0u;
                    }
                }
            }
            if (__ballot(thr != __builtin_inff()) == 0ull) break;
        }
    }
    write_pixel(a, px, py, C0, C1, C2, T, last);
    if (COUNT) add_counters(a.counters, nb, ncl, nt);
}

}  // namespace
