// Preprocess: projection of 3D Gaussians to screen space (TC-GS paper,
// Sec. 3.1 "Preprocess": mu' = W mu, Sigma' = J W Sigma W^T J^T), conic
// inversion, radius and tile count.  One thread per Gaussian; the stage is
// bound by HBM bandwidth (240 input bytes per Gaussian, 192 of them SH).
#include "common.h"

// No floating-point contraction in this file: every product and sum below is
// rounded as written, so the one-camera and the multi-camera kernels, which
// share these functions, give bit-identical results (fused multiply-adds are
// spelled out with fmaf where they are wanted).
#pragma clang fp contract(off)

namespace {

struct CamParams {
    float R[9], t[3];
    float fx, fy, cx, cy;
    int W, H, gx;
    float near_z, limx, limy, lowpass;
    float cpos[3];
};

// Real spherical harmonics up to degree 3 with the Condon-Shortley phase,
// orthonormal on the unit sphere, as polynomials in the unit direction
// (x, y, z); coefficient index l*l + l + m.  Constants are the closed forms
// K = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the polynomial factors.
__device__ __forceinline__ void load_sh(const float4 *sh4, float k[48]) {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        float4 v = sh4[i];
        k[4 * i] = v.x;
        k[4 * i + 1] = v.y;
        k[4 * i + 2] = v.z;
        k[4 * i + 3] = v.w;
    }
}

// Colour max(0, sum_i Y_i(x, y, z) k[3i + ch] + 1/2) of coefficients k[16][3]
// up to degree `deg`.
__device__ __forceinline__ void sh_colour(const float k[48], int deg, float x, float y, float z,
                                          float out[3]) {
    const float C0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
    const float C1 = 0.48860251190291992f;   // sqrt(3 / (4 pi))
    float Y[16];
    Y[0] = C0;
    Y[1] = -C1 * y;
    Y[2] = C1 * z;
    Y[3] = -C1 * x;
    float xx = x * x, yy = y * y, zz = z * z, xy = x * y, yz = y * z, xz = x * z;
    Y[4] = 1.0925484305920792f * xy;                    // sqrt(15/(4pi))
    Y[5] = -1.0925484305920792f * yz;
    Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy); // sqrt(5/(16pi))
    Y[7] = -1.0925484305920792f * xz;
    Y[8] = 0.54627421529603959f * (xx - yy);            // sqrt(15/(16pi))
    Y[9] = -0.59004358992664352f * y * (3.0f * xx - yy);  // sqrt(35/(32pi))
    Y[10] = 2.8906114426405538f * xy * z;                 // sqrt(105/(4pi))
    Y[11] = -0.45704579946446572f * y * (4.0f * zz - xx - yy);  // sqrt(21/(32pi))
    Y[12] = 0.37317633259011540f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);  // sqrt(7/(16pi))
    Y[13] = -0.45704579946446572f * x * (4.0f * zz - xx - yy);
    Y[14] = 1.4453057213202769f * z * (xx - yy);          // sqrt(105/(16pi))
    Y[15] = -0.59004358992664352f * x * (xx - 3.0f * yy);
    int n = (deg + 1) * (deg + 1);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i < n) acc = fmaf(Y[i], k[3 * i + ch], acc);
        acc += 0.5f;
        out[ch] = fmaxf(acc, 0.0f);
    }
}

// Conic and radius of Sigma' = [[a, b], [b, c]].  The determinant and the
// inverse switch to FP64 when FP32 would lose more than ~10 bits to
// cancellation (det < 2^-10 * a * c); products of floats are exact in FP64.
__device__ __forceinline__ bool conic_radius(float a, float b, float c, float3 &conic, int &radius) {
    float det = a * c - b * b;
    float con0, con1, con2;
    if (det < 0.0009765625f * a * c) {
        double dd = (double)a * (double)c - (double)b * (double)b;
        if (!(dd > 0.0) || !isfinite(dd)) return false;
        double inv = 1.0 / dd;
        con0 = (float)(c * inv);
        con1 = (float)(-b * inv);
        con2 = (float)(a * inv);
        det = (float)dd;
    } else {
        if (!(det > 0.0f) || !isfinite(det)) return false;
        float inv = 1.0f / det;
        con0 = c * inv;
        con1 = -b * inv;
        con2 = a * inv;
    }
    float mid = 0.5f * (a + c);
    float lmax = mid + sqrtf(fmaxf(0.1f, mid * mid - det));
    float r3 = ceilf(3.0f * sqrtf(lmax));
    if (!(r3 >= 1.0f)) return false;
    radius = r3 > (float)GS_RADIUS_LIMIT ? GS_RADIUS_LIMIT : (int)r3;
    conic = make_float3(con0, con1, con2);
    return true;
}

// View-independent part of a 3D Gaussian: mean, squared scales and the
// rotation matrix of its normalised quaternion (w, x, y, z).
struct Gauss3 {
    float mx, my, mz;
    float ss[3];
    float Rq[9];
};

__device__ __forceinline__ Gauss3 load_gauss(int i, const float *__restrict__ means,
                                             const float *__restrict__ scales,
                                             const float4 *__restrict__ quats) {
    Gauss3 g;
    g.mx = means[3 * i];
    g.my = means[3 * i + 1];
    g.mz = means[3 * i + 2];
    float4 q = quats[i];
    float qn = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
    float w = q.x * qn, x = q.y * qn, y = q.z * qn, z = q.w * qn;
    g.Rq[0] = 1.f - 2.f * (y * y + z * z);
    g.Rq[1] = 2.f * (x * y - w * z);
    g.Rq[2] = 2.f * (x * z + w * y);
    g.Rq[3] = 2.f * (x * y + w * z);
    g.Rq[4] = 1.f - 2.f * (x * x + z * z);
    g.Rq[5] = 2.f * (y * z - w * x);
    g.Rq[6] = 2.f * (x * z - w * y);
    g.Rq[7] = 2.f * (y * z + w * x);
    g.Rq[8] = 1.f - 2.f * (x * x + y * y);
    float s0 = scales[3 * i], s1 = scales[3 * i + 1], s2 = scales[3 * i + 2];
    g.ss[0] = s0 * s0;
    g.ss[1] = s1 * s1;
    g.ss[2] = s2 * s2;
    return g;
}

// Screen-space footprint of one Gaussian in one camera.  nt = 0 means not
// rendered (behind near_z, degenerate Sigma', or no tile covered); then the
// other fields are zero.
struct Footprint {
    float2 m2;
    float3 con;
    float depth;
    int r;
    uint32_t nt;
};

__device__ __forceinline__ Footprint project(const Gauss3 &g, const CamParams &cam) {
    Footprint f;
    f.m2 = make_float2(0.f, 0.f);
    f.con = make_float3(0.f, 0.f, 0.f);
    f.depth = 0.f;
    f.r = 0;
    f.nt = 0;
    float tx = cam.R[0] * g.mx + cam.R[1] * g.my + cam.R[2] * g.mz + cam.t[0];
    float ty = cam.R[3] * g.mx + cam.R[4] * g.my + cam.R[5] * g.mz + cam.t[1];
    float tz = cam.R[6] * g.mx + cam.R[7] * g.my + cam.R[8] * g.mz + cam.t[2];
    if (!(tz > cam.near_z)) return f;
    // A = (J Wrot) Rq; Sigma' = A diag(s^2) A^T
    float inv_z = 1.0f / tz;
    float xr = fminf(fmaxf(tx * inv_z, -cam.limx), cam.limx);
    float yr = fminf(fmaxf(ty * inv_z, -cam.limy), cam.limy);
    float J00 = cam.fx * inv_z, J02 = -cam.fx * xr * inv_z;
    float J11 = cam.fy * inv_z, J12 = -cam.fy * yr * inv_z;
    float M[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        M[0][c] = J00 * cam.R[c] + J02 * cam.R[6 + c];
        M[1][c] = J11 * cam.R[3 + c] + J12 * cam.R[6 + c];
    }
    float A[2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            A[a][c] = M[a][0] * g.Rq[c] + M[a][1] * g.Rq[3 + c] + M[a][2] * g.Rq[6 + c];
    float ca = cam.lowpass, cb = 0.f, cc = cam.lowpass;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ca = fmaf(A[0][k] * g.ss[k], A[0][k], ca);
        cb = fmaf(A[0][k] * g.ss[k], A[1][k], cb);
        cc = fmaf(A[1][k] * g.ss[k], A[1][k], cc);
    }
    float2 m2 = make_float2(cam.fx * tx * inv_z + cam.cx, cam.fy * ty * inv_z + cam.cy);
    float3 con;
    int r = 0;
    uint32_t nt = 0;
    if (conic_radius(ca, cb, cc, con, r)) {
        int tx0, tx1, ty0, ty1;
        nt = (uint32_t)gs::tile_rect(m2.x, m2.y, r, cam.W, cam.H, cam.gx, tx0, tx1, ty0, ty1);
    }
    if (nt == 0) return f;
    f.m2 = m2;
    f.con = con;
    f.depth = tz;
    f.r = r;
    f.nt = nt;
    return f;
}

__device__ __forceinline__ void view_dir(const Gauss3 &g, const CamParams &cam, float &x, float &y,
                                         float &z) {
    float dx = g.mx - cam.cpos[0], dy = g.my - cam.cpos[1], dz = g.mz - cam.cpos[2];
    float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
    x = dx * dn;
    y = dy * dn;
    z = dz * dn;
}

__device__ __forceinline__ void store_footprint(size_t i, const Footprint &f,
                                                float2 *__restrict__ means2d,
                                                float *__restrict__ conics,
                                                float *__restrict__ depths, int *__restrict__ radii,
                                                uint32_t *__restrict__ tiles_touched) {
    means2d[i] = f.m2;
    conics[3 * i] = f.con.x;
    conics[3 * i + 1] = f.con.y;
    conics[3 * i + 2] = f.con.z;
    depths[i] = f.depth;
    radii[i] = f.r;
    tiles_touched[i] = f.nt;
}

// ln o, the form in which opacity enters the exponent (Sec. 4.1); -inf for
// o = 0.  Computed once per Gaussian here rather than per splat and tile.
__device__ __forceinline__ float log_opacity(float o) { return logf(o); }

__device__ __forceinline__ void store_rgb(size_t i, const float col[3], float *__restrict__ rgb) {
    rgb[3 * i] = col[0];
    rgb[3 * i + 1] = col[1];
    rgb[3 * i + 2] = col[2];
}

__global__ __launch_bounds__(256) void k_preprocess_3d(int P, const float *__restrict__ means,
                                                       const float *__restrict__ scales,
                                                       const float4 *__restrict__ quats,
                                                       const float *__restrict__ opac,
                                                       const float4 *__restrict__ sh, int sh_deg,
                                                       CamParams cam, float2 *__restrict__ means2d,
                                                       float *__restrict__ conics,
                                                       float *__restrict__ lno,
                                                       float *__restrict__ depths,
                                                       int *__restrict__ radii,
                                                       float *__restrict__ rgb,
                                                       uint32_t *__restrict__ tiles_touched) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const Gauss3 g = load_gauss(i, means, scales, quats);
    const Footprint f = project(g, cam);
    float col[3] = {0.f, 0.f, 0.f};
    if (f.nt) {
        // the SH coefficients (192 of the 236 input bytes) are read only for
        // Gaussians that are drawn
        float k[48];
        load_sh(sh + (size_t)i * 12, k);
        float x, y, z;
        view_dir(g, cam, x, y, z);
        sh_colour(k, sh_deg, x, y, z, col);
    }
    store_footprint(i, f, means2d, conics, depths, radii, tiles_touched);
    store_rgb(i, col, rgb);
    lno[i] = log_opacity(opac[i]);
}

// Up to MV_CHUNK cameras per launch, passed by value.
constexpr int MV_CHUNK = 16;
struct CamChunk {
    CamParams c[MV_CHUNK];
};

// Several cameras per thread: the Gaussian (and its SH coefficients, if some
// camera draws it) is read once; outputs are view-major with stride P.
__global__ __launch_bounds__(256) void k_preprocess_mv(int P, const float *__restrict__ means,
                                                       const float *__restrict__ scales,
                                                       const float4 *__restrict__ quats,
                                                       const float *__restrict__ opac,
                                                       const float4 *__restrict__ sh, int sh_deg,
                                                       CamChunk cams, int v0, int nv,
                                                       float2 *__restrict__ means2d,
                                                       float *__restrict__ conics,
                                                       float *__restrict__ lno,
                                                       float *__restrict__ depths,
                                                       int *__restrict__ radii,
                                                       float *__restrict__ rgb,
                                                       uint32_t *__restrict__ tiles_touched) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const Gauss3 g = load_gauss(i, means, scales, quats);
    if (v0 == 0) lno[i] = log_opacity(opac[i]);
    uint32_t drawn = 0;
    const float zero[3] = {0.f, 0.f, 0.f};
    for (int c = 0; c < nv; ++c) {
        const Footprint f = project(g, cams.c[c]);
        const size_t o = (size_t)(v0 + c) * (size_t)P + (size_t)i;
        store_footprint(o, f, means2d, conics, depths, radii, tiles_touched);
        if (f.nt) drawn |= 1u << c;
        else store_rgb(o, zero, rgb);
    }
    if (drawn) {
        float k[48];
        load_sh(sh + (size_t)i * 12, k);
        for (int c = 0; c < nv; ++c) {
            if (!((drawn >> c) & 1u)) continue;
            float x, y, z, col[3];
            view_dir(g, cams.c[c], x, y, z);
            sh_colour(k, sh_deg, x, y, z, col);
            store_rgb((size_t)(v0 + c) * (size_t)P + (size_t)i, col, rgb);
        }
    }
}

__global__ __launch_bounds__(256) void k_preprocess_2d(int P, const float2 *__restrict__ means2d,
                                                       const float *__restrict__ cov2d,
                                                       const float *__restrict__ opac, int W, int H,
                                                       int gx, float *__restrict__ conics,
                                                       float *__restrict__ lno,
                                                       int *__restrict__ radii,
                                                       uint32_t *__restrict__ tiles_touched) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    float2 m = means2d[i];
    float3 con = make_float3(0.f, 0.f, 0.f);
    int r = 0;
    uint32_t nt = 0;
    if (conic_radius(cov2d[3 * i], cov2d[3 * i + 1], cov2d[3 * i + 2], con, r)) {
        int tx0, tx1, ty0, ty1;
        nt = (uint32_t)gs::tile_rect(m.x, m.y, r, W, H, gx, tx0, tx1, ty0, ty1);
    }
    if (nt == 0) {
        r = 0;
        con = make_float3(0.f, 0.f, 0.f);
    }
    conics[3 * i] = con.x;
    conics[3 * i + 1] = con.y;
    conics[3 * i + 2] = con.z;
    radii[i] = r;
    tiles_touched[i] = nt;
    lno[i] = log_opacity(opac[i]);
}

CamParams cam_params(const gs_camera &cam) {
    CamParams cp;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) cp.R[3 * r + c] = cam.viewmat[4 * r + c];
        cp.t[r] = cam.viewmat[4 * r + 3];
    }
    cp.fx = cam.fx;
    cp.fy = cam.fy;
    cp.cx = cam.cx;
    cp.cy = cam.cy;
    cp.W = cam.width;
    cp.H = cam.height;
    cp.gx = gs::grid_x(cam.width);
    cp.near_z = cam.near_z;
    cp.limx = cam.frustum_guard * (0.5f * cam.width / cam.fx);
    cp.limy = cam.frustum_guard * (0.5f * cam.height / cam.fy);
    cp.lowpass = cam.lowpass;
    for (int k = 0; k < 3; ++k) cp.cpos[k] = cam.campos[k];
    return cp;
}

bool camera_ok(const gs_camera &cam) {
    if (cam.width <= 0 || cam.height <= 0 || cam.width > GS_MAX_DIM || cam.height > GS_MAX_DIM)
        return false;
    return cam.fx > 0.f && cam.fy > 0.f;
}

}  // namespace

extern "C" gs_status gs_preprocess(int32_t P, const float *means3d, const float *scales,
                                   const float *quats, const float *opacities, const float *sh,
                                   int32_t sh_degree, const gs_camera *cam, float *means2d,
                                   float *conics, float *log_opacities, float *depths,
                                   int32_t *radii, float *rgb, uint32_t *tiles_touched,
                                   void *stream) {
    if (P < 0 || !cam || sh_degree < 0 || sh_degree > 3 || !camera_ok(*cam)) return GS_ERR_INVALID_ARG;
    if (P == 0) return GS_OK;
    const void *ptrs[] = {means3d, scales, quats, opacities, sh, means2d, conics, log_opacities,
                          depths, radii, rgb, tiles_touched};
    for (const void *p : ptrs)
        if (!p || !gs::aligned(p, 4)) return GS_ERR_INVALID_ARG;
    if (!gs::aligned(quats, 16) || !gs::aligned(sh, 16) || !gs::aligned(means2d, 8))
        return GS_ERR_INVALID_ARG;
    CamParams cp = cam_params(*cam);
    hipStream_t s = (hipStream_t)stream;
    int blocks = (P + 255) / 256;
    hipLaunchKernelGGL(k_preprocess_3d, dim3(blocks), dim3(256), 0, s, P, means3d, scales,
                       (const float4 *)quats, opacities, (const float4 *)sh, sh_degree, cp,
                       (float2 *)means2d, conics, log_opacities, depths, radii, rgb, tiles_touched);
    return gs::launch_status();
}

extern "C" gs_status gs_preprocess_multiview(int32_t P, const float *means3d, const float *scales,
                                             const float *quats, const float *opacities,
                                             const float *sh, int32_t sh_degree, int32_t nviews,
                                             const gs_camera *cams, float *means2d, float *conics,
                                             float *log_opacities, float *depths, int32_t *radii,
                                             float *rgb, uint32_t *tiles_touched, void *stream) {
    if (P < 0 || !cams || sh_degree < 0 || sh_degree > 3 || nviews < 1 || nviews > 64)
        return GS_ERR_INVALID_ARG;
    for (int v = 0; v < nviews; ++v)
        if (!camera_ok(cams[v])) return GS_ERR_INVALID_ARG;
    if (P == 0) return GS_OK;
    const void *ptrs[] = {means3d, scales, quats, opacities, sh, means2d, conics, log_opacities,
                          depths, radii, rgb, tiles_touched};
    for (const void *p : ptrs)
        if (!p || !gs::aligned(p, 4)) return GS_ERR_INVALID_ARG;
    if (!gs::aligned(quats, 16) || !gs::aligned(sh, 16) || !gs::aligned(means2d, 8))
        return GS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    int blocks = (P + 255) / 256;
    for (int v0 = 0; v0 < nviews; v0 += MV_CHUNK) {
        const int nv = nviews - v0 < MV_CHUNK ? nviews - v0 : MV_CHUNK;
        CamChunk ch{};
        for (int c = 0; c < nv; ++c) ch.c[c] = cam_params(cams[v0 + c]);
        hipLaunchKernelGGL(k_preprocess_mv, dim3(blocks), dim3(256), 0, s, P, means3d, scales,
                           (const float4 *)quats, opacities, (const float4 *)sh, sh_degree, ch, v0,
                           nv, (float2 *)means2d, conics, log_opacities, depths, radii, rgb,
                           tiles_touched);
    }
    return gs::launch_status();
}

extern "C" gs_status gs_preprocess_2d(int32_t P, const float *means2d, const float *cov2d,
                                      const float *opacities, int32_t width, int32_t height,
                                      float *conics, float *log_opacities, int32_t *radii,
                                      uint32_t *tiles_touched, void *stream) {
    if (P < 0 || width <= 0 || height <= 0 || width > GS_MAX_DIM || height > GS_MAX_DIM)
        return GS_ERR_INVALID_ARG;
    if (P == 0) return GS_OK;
    const void *ptrs[] = {means2d, cov2d, opacities, conics, log_opacities, radii, tiles_touched};
    for (const void *p : ptrs)
        if (!p || !gs::aligned(p, 4)) return GS_ERR_INVALID_ARG;
    if (!gs::aligned(means2d, 8)) return GS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    int blocks = (P + 255) / 256;
    hipLaunchKernelGGL(k_preprocess_2d, dim3(blocks), dim3(256), 0, s, P, (const float2 *)means2d,
                       cov2d, opacities, width, height, gs::grid_x(width), conics, log_opacities,
                       radii, tiles_touched);
    return gs::launch_status();
}
