// Device-side pieces shared by the forward and backward rasterisers
// (tile alpha-blending, TC-GS paper Sec. 3.1 Algorithm 1 and Sec. 4):
// constants of Algorithm 1, the matrix-core operand layouts (Frag2Mat,
// Sec. 4.2, in G2L local coordinates, Sec. 4.3), splat staging with the
// exact per-tile cull, and output helpers.
#pragma once

#include "common.h"

namespace {

constexpr float ALPHA_MAX = 0.99f;
constexpr float T_MIN = 1e-4f;
constexpr float CULL_ALPHA = 1.0f / 255.0f;
constexpr float LOG2E = 1.4426950408889634f;
constexpr float CULL_LN = -5.541263545158426f;   // -ln 255
constexpr float CULL_LOG2 = -7.994353436858858f; // -log2 255
constexpr int BATCH = 256;                       // splats staged per LDS round
constexpr int SUB = 32;                          // splats per MFMA

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

struct RasterArgs {
    int W, H, gx, gy;
    int chunk_rows;  // tile rows per XCD chunk (1 or 2), see gs::xcd_tile
    const uint32_t *ranges;
    const uint32_t *ids;
    const float2 *means2d;
    const float *conics;
    const float *lno;  // ln o per Gaussian
    const float *rgb;
    float bg0, bg1, bg2;
    float *out_rgb;
    float *out_T;
    uint32_t *out_nc;
    unsigned long long *counters;
};

__device__ __forceinline__ void add_counters(unsigned long long *c, uint32_t nb, uint32_t nc,
                                             uint32_t nt) {
    // wave-reduce then one atomic per wave
    unsigned long long b = nb, cl = nc, t = nt;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        b += __shfl_xor(b, d, 64);
        cl += __shfl_xor(cl, d, 64);
        t += __shfl_xor(t, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(c + 0, b);
        atomicAdd(c + 1, cl);
        atomicAdd(c + 2, t);
        atomicAdd(c + 3, b + cl + t);
    }
}

__device__ __forceinline__ void write_pixel(const RasterArgs &a, int px, int py, float C0, float C1,
                                            float C2, float T, uint32_t last) {
    if (px < a.W && py < a.H) {
        size_t pi = (size_t)py * a.W + px, hw = (size_t)a.W * a.H;
        a.out_rgb[pi] = fmaf(T, a.bg0, C0);
        a.out_rgb[hw + pi] = fmaf(T, a.bg1, C1);
        a.out_rgb[2 * hw + pi] = fmaf(T, a.bg2, C2);
        a.out_T[pi] = T;
        if (a.out_nc) a.out_nc[pi] = last;
    }
}


// ---------------------------------------------------------------------------
// Matrix-core kernel
// ---------------------------------------------------------------------------
enum Variant { VAR_F16_GLOBAL = 0, VAR_F16_G2L = 1, VAR_F16_SPLIT = 2, VAR_BF16_SPLIT = 3 };

template <int VAR> struct VarTraits;
// K = 8: [v0/3 x3, v1..v5] against [1 x3, dx, dy, dx^2, dxdy, dy^2]
template <> struct VarTraits<VAR_F16_GLOBAL> { static constexpr int ROW1 = 16, ROW2 = 0; static constexpr bool LOCAL = false; };
template <> struct VarTraits<VAR_F16_G2L> { static constexpr int ROW1 = 16, ROW2 = 0; static constexpr bool LOCAL = true; };
// K = 16: [hi(6), 0, 0 | lo(6), 0, 0] against [256 u(6), 0, 0 | u(6), 0, 0],
// hi = fp16(v / 256), lo = fp16(v - 256 hi)
template <> struct VarTraits<VAR_F16_SPLIT> { static constexpr int ROW1 = 32, ROW2 = 0; static constexpr bool LOCAL = true; };
// K = 16 + 8: [hi(6),0,0 | mid(6),0,0] then [lo0..3 | lo4, lo5, 0, 0]
template <> struct VarTraits<VAR_BF16_SPLIT> { static constexpr int ROW1 = 32, ROW2 = 16; static constexpr bool LOCAL = true; };

// Row of the 32x32 MFMA that holds splat j of a sub-batch: output register
// r of lanes 0-31 holds row 8(r/4) + r%4, of lanes 32-63 row 8(r/4)+4+r%4.
__device__ __forceinline__ int row_of_splat(int j) {
    int h = j >> 4, r = j & 15;
    return 8 * (r >> 2) + 4 * h + (r & 3);
}

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    __bf16 b = (__bf16)x;
    return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ float bf16_val(float x) { return (float)(__bf16)x; }

// a*b + c*d, rounded once more than a single product: the rounding error
// of c*d is recovered exactly with an FMA and added back, so the result is
// accurate to a few ulps of itself even when the two products cancel.
__device__ __forceinline__ float dot2_acc(float a, float b, float c, float d) {
    const float p = c * d;
    const float e = fmaf(c, d, -p);
    return fmaf(a, b, p) + e;
}

// Write the operand-A row of one splat.  Coefficients (Sec. 4.2) in the frame
// with origin (ox, oy), scaled by log2(e):
//   v0 = log2e (ln o - 1/2 dmu^T S dmu), v1 = log2e (s11 dx + s12 dy),
//   v2 = log2e (s12 dx + s22 dy), v3 = -1/2 log2e s11, v4 = -log2e s12,
//   v5 = -1/2 log2e s22,  dmu = mu' - origin.
// They are computed once per splat and tile, so they are evaluated with
// care: dmu^T S dmu as s11 (dx + (s12/s11) dy)^2 + (det S / s11) dy^2, two
// non-negative terms with det S = s11 s22 - s12^2 from Kahan's FMA scheme,
// and v1, v2 with dot2_acc.  The plain expansion loses to cancellation all
// the digits of near-degenerate (needle-like) splats, whose terms are far
// larger than their sum; these forms keep the error near the size of the
// result.
template <int VAR>
__device__ __forceinline__ void build_row(bool valid, float2 mu, float s11, float s12, float s22,
                                          float lno, float ox, float oy, uint8_t *row1, uint8_t *row2) {
    float v[6];
    if (valid) {
        const float dx = mu.x - ox, dy = mu.y - oy;
        const float w = s12 * s12;
        const float det = fmaf(s11, s22, -w) - fmaf(s12, s12, -w);
        const float r11 = 1.0f / s11;
        const float t = fmaf(s12 * r11, dy, dx);
        const float q = fmaf(s11 * t, t, (det * r11) * dy * dy);
        v[0] = LOG2E * fmaf(-0.5f, q, lno);
        v[1] = LOG2E * dot2_acc(s11, dx, s12, dy);
        v[2] = LOG2E * dot2_acc(s12, dx, s22, dy);
        v[3] = -0.5f * LOG2E * s11;
        v[4] = -LOG2E * s12;
        v[5] = -0.5f * LOG2E * s22;
    } else {
        v[0] = -__builtin_inff();
        v[1] = v[2] = v[3] = v[4] = v[5] = 0.0f;
    }
    if (VAR == VAR_F16_GLOBAL || VAR == VAR_F16_G2L) {
        _Float16 w0 = (_Float16)(v[0] * (1.0f / 3.0f));
        half8_t r = {w0, w0, w0, (_Float16)v[1], (_Float16)v[2], (_Float16)v[3], (_Float16)v[4],
                     (_Float16)v[5]};
        *(half8_t *)row1 = r;
    } else if (VAR == VAR_F16_SPLIT) {
        // hi holds v / 256 (its pixel features are 256 u, exact in FP16), so
        // coefficients up to 256 x 65504 stay finite: the exponent at the
        // tile centre of a needle-thin splat crossing the tile can be far
        // below -65504 while pixels on its axis still blend
        half8_t hi, lo;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            _Float16 h = (_Float16)(v[i] * (1.0f / 256.0f));
            hi[i] = h;
            lo[i] = valid ? (_Float16)(v[i] - 256.0f * (float)h) : (_Float16)0.0f;
        }
        hi[6] = hi[7] = lo[6] = lo[7] = (_Float16)0.0f;
        *(half8_t *)row1 = hi;
        *(half8_t *)(row1 + 16) = lo;
    } else {
        uint16_t hb[8], mb[8], lb[4 + 4];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            float h = bf16_val(v[i]);
            float rem = valid ? v[i] - h : 0.0f;
            float m = bf16_val(rem);
            float rem2 = valid ? rem - m : 0.0f;
            hb[i] = bf16_bits(v[i]);
            mb[i] = bf16_bits(rem);
            lb[i] = bf16_bits(rem2);
        }
        hb[6] = hb[7] = mb[6] = mb[7] = lb[6] = lb[7] = 0;
        uint4 w1 = make_uint4(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16), hb[4] | (hb[5] << 16), 0u);
        uint4 w2 = make_uint4(mb[0] | (mb[1] << 16), mb[2] | (mb[3] << 16), mb[4] | (mb[5] << 16), 0u);
        uint4 w3 = make_uint4(lb[0] | (lb[1] << 16), lb[2] | (lb[3] << 16), lb[4] | (lb[5] << 16), 0u);
        *(uint4 *)row1 = w1;
        *(uint4 *)(row1 + 16) = w2;
        *(uint4 *)row2 = w3;
    }
}

// Operand B (pixel features) of one lane for column group G.
struct UOperand {
    half4_t k8;
    half8_t k16;
    bf16x8_t b16;
    short4_t b8;
};

template <int VAR>
__device__ __forceinline__ UOperand make_u(float ux, float uy, int slice) {
    UOperand u;
    float f[6] = {1.0f, ux, uy, ux * ux, ux * uy, uy * uy};
    if (VAR == VAR_F16_GLOBAL || VAR == VAR_F16_G2L) {
        float e[8] = {1.0f, 1.0f, 1.0f, f[1], f[2], f[3], f[4], f[5]};
#pragma unroll
        for (int i = 0; i < 4; ++i) u.k8[i] = (_Float16)e[4 * slice + i];
    } else if (VAR == VAR_F16_SPLIT) {
        // K 0-7 (slice 0) meet the hi row, K 8-15 (slice 1) the lo row
        const float sc = slice == 0 ? 256.0f : 1.0f;
#pragma unroll
        for (int i = 0; i < 6; ++i) u.k16[i] = (_Float16)(sc * f[i]);
        u.k16[6] = u.k16[7] = (_Float16)0.0f;
    } else {
#pragma unroll
        for (int i = 0; i < 6; ++i) u.b16[i] = (__bf16)f[i];
        u.b16[6] = u.b16[7] = (__bf16)0.0f;
        float e[8] = {f[0], f[1], f[2], f[3], f[4], f[5], 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < 4; ++i) u.b8[i] = (short)bf16_bits(e[4 * slice + i]);
    }
    return u;
}

// B for the two column groups of this lane's wave quadrant -> exponents of
// this lane's own pixel for 32 splats (log2 units): lo[r] = splat r,
// hi[r] = splat 16 + r.
template <int VAR>
__device__ __forceinline__ void exponents(const uint8_t *a1, const uint8_t *a2, const UOperand &u0,
                                          const UOperand &u1, int lane, float lo[16], float hi[16]) {
    f32x16_t acc0 = {}, acc1 = {};
    int row = lane & 31, slice = lane >> 5;
    if (VAR == VAR_F16_GLOBAL || VAR == VAR_F16_G2L) {
        half4_t av = *(const half4_t *)(a1 + row * 16 + slice * 8);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x8f16(av, u0.k8, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x8f16(av, u1.k8, acc1, 0, 0, 0);
    } else if (VAR == VAR_F16_SPLIT) {
        half8_t av = *(const half8_t *)(a1 + row * 32 + slice * 16);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, u0.k16, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, u1.k16, acc1, 0, 0, 0);
    } else {
        bf16x8_t av = *(const bf16x8_t *)(a1 + row * 32 + slice * 16);
        short4_t aw = *(const short4_t *)(a2 + row * 16 + slice * 8);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, u0.b16, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, u1.b16, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(aw, u0.b8, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(aw, u1.b8, acc1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc0[r]), __float_as_uint(acc1[r]),
                                                   false, false);
        lo[r] = __uint_as_float(sw[0]);
        hi[r] = __uint_as_float(sw[1]);
    }
}

// LDS footprint of one staged batch of NB splats.
template <int VAR, int NB = BATCH> struct Stage {
    static constexpr int A1 = NB * VarTraits<VAR>::ROW1;
    static constexpr int A2 = NB * VarTraits<VAR>::ROW2;
    static constexpr int RGB = NB * 16;
    static constexpr int BYTES = A1 + A2 + RGB;
};

struct SplatRegs {
    float2 mu;
    float s11, s12, s22, lno, r, g, b;
    bool valid;
    uint32_t id;
};

// Three consecutive floats read with one 12-byte load (the arrays are only
// 4-byte aligned per Gaussian; gfx950 loads dword-aligned dwordx3).
struct __attribute__((aligned(4))) Float3 {
    float x, y, z;
};

// One splat's parameters: four loads (mean, conic, ln o, colour) rather
// than one per float, so a wave's gather touches each array's lines once.
// Without RGB the colour is left to load_rgb, so that a caller can fetch it
// only for the splats its per-tile cull keeps.
template <bool RGB = true>
__device__ __forceinline__ SplatRegs gather(const RasterArgs &a, uint32_t id, bool valid) {
    SplatRegs s;
    s.valid = valid;
    s.id = id;
    if (valid) {
        s.mu = a.means2d[id];
        const Float3 c = *(const Float3 *)(a.conics + 3 * (size_t)id);
        s.s11 = c.x;
        s.s12 = c.y;
        s.s22 = c.z;
        s.lno = a.lno[id];
        if (RGB) {
            const Float3 k = *(const Float3 *)(a.rgb + 3 * (size_t)id);
            s.r = k.x;
            s.g = k.y;
            s.b = k.z;
        } else {
            s.r = s.g = s.b = 0.f;
        }
    } else {
        s.mu = make_float2(0.f, 0.f);
        s.s11 = s.s12 = s.s22 = 0.f;
        s.lno = 0.f;
        s.r = s.g = s.b = 0.f;
    }
    return s;
}

// The colour of a splat gathered without it (gather<false>).
__device__ __forceinline__ void load_rgb(const RasterArgs &a, SplatRegs &s) {
    const Float3 k = *(const Float3 *)(a.rgb + 3 * (size_t)s.id);
    s.r = k.x;
    s.g = k.y;
    s.b = k.z;
}

template <int VAR, int NB = BATCH>
__device__ __forceinline__ void stage_splat(uint8_t *stage, int j, const SplatRegs &s, float ox,
                                            float oy, uint32_t list_pos) {
    int sub = j / SUB, row = row_of_splat(j % SUB);
    uint8_t *row1 = stage + sub * SUB * VarTraits<VAR>::ROW1 + row * VarTraits<VAR>::ROW1;
    uint8_t *row2 = stage + Stage<VAR, NB>::A1 + sub * SUB * VarTraits<VAR>::ROW2 + row * VarTraits<VAR>::ROW2;
    build_row<VAR>(s.valid, s.mu, s.s11, s.s12, s.s22, s.lno, ox, oy, row1, row2);
    float4 *rgb = (float4 *)(stage + Stage<VAR, NB>::A1 + Stage<VAR, NB>::A2);
    // w: 1-based position of the splat in the tile list (for n_contrib)
    rgb[j] = make_float4(s.r, s.g, s.b, __uint_as_float(list_pos + 1u));
}

// Can the splat reach the 1/255 threshold anywhere in the pixel box
// [x0, x0 + 15] x [y0, y0 + 15]?  Exact minimum of the convex form
// q/2 = 1/2 d^T S d over the box (zero if the centre is inside, otherwise the
// smaller of the minima along the vertical and the horizontal edge on the
// centre's side, each a clamped 1D minimisation), compared
// with ln o + ln 255 with a margin that covers FP32 rounding of the bound.
// A splat that fails the test is culled at every pixel of the tile, so
// dropping it changes no output of the exact computation.
__device__ __forceinline__ bool tile_alive(const SplatRegs &s, float x0, float y0) {
    if (!s.valid) return false;
    const float x1 = x0 + (GS_TILE - 1), y1 = y0 + (GS_TILE - 1);
    const float a = s.s11, b = s.s12, c = s.s22;
    const float mx = s.mu.x, my = s.mu.y;
    float fmin = 0.0f, fabs_terms = 0.0f;
    if (!(mx >= x0 && mx <= x1 && my >= y0 && my <= y1)) {
        fmin = __builtin_inff();
        // Each edge's minimiser -b dx / c (or -b dy / a) through one hardware
        // reciprocal per coefficient: it only picks the point where the form
        // is evaluated, and at the minimum the form is flat, so its 1-ulp
        // error moves f by far less than the margin below.
        const float nb_c = -b * __builtin_amdgcn_rcpf(c), nb_a = -b * __builtin_amdgcn_rcpf(a);
        // The form is convex with its minimum at the mean, outside the box,
        // so its minimum over the box lies on an edge whose half-plane the
        // mean violates: from a boundary point on no such edge, a step
        // toward the mean stays in the box and lowers the form.  The mean
        // violates at most one vertical and one horizontal edge, those on
        // its side, so those two are evaluated; where the mean lies within
        // the box's x (or y) span, the edge taken there is not violated and
        // only adds a value above the minimum.
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            float dx, dy;
            if (e == 0) {
                dx = (mx < x0 ? x0 : x1) - mx;
                dy = fminf(fmaxf(nb_c * dx, y0 - my), y1 - my);
            } else {
                dy = (my < y0 ? y0 : y1) - my;
                dx = fminf(fmaxf(nb_a * dy, x0 - mx), x1 - mx);
            }
            float t0 = a * dx * dx, t1 = 2.0f * b * dx * dy, t2 = c * dy * dy;
            float f = 0.5f * (t0 + t1 + t2);
            if (f < fmin) {
                fmin = f;
                fabs_terms = 0.5f * (fabsf(t0) + fabsf(t1) + fabsf(t2));
            }
        }
    }
    float margin = 1e-3f * (1.0f + fmin) + 1e-5f * fabs_terms;
    return s.lno - fmin >= CULL_LN - margin;
}

inline bool valid_inputs(int32_t width, int32_t height, const void *const *p, int n) {
    if (width <= 0 || height <= 0 || width > GS_MAX_DIM || height > GS_MAX_DIM) return false;
    for (int i = 0; i < n; ++i)
        if (!p[i] || !gs::aligned(p[i], 4)) return false;
    return true;
}

}  // namespace
