// Preprocess: projection of 3D Gaussians to screen space (TC-GS paper,
// Sec. 3.1 "Preprocess": mu' = W mu, Sigma' = J W Sigma W^T J^T), conic
// inversion, radius and tile count.  One thread per Gaussian; the stage is
// bound by HBM bandwidth (236 input bytes per Gaussian, 192 of them SH).
#include "common.h"

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
__device__ __forceinline__ void sh_colour(const float4 *sh4, int deg, float x, float y, float z,
                                          float out[3]) {
    // unpack [16][3] floats from 12 float4
    float k[48];
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        float4 v = sh4[i];
        k[4 * i] = v.x;
        k[4 * i + 1] = v.y;
        k[4 * i + 2] = v.z;
        k[4 * i + 3] = v.w;
    }
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

__global__ __launch_bounds__(256) void k_preprocess_3d(int P, const float *__restrict__ means,
                                                       const float *__restrict__ scales,
                                                       const float4 *__restrict__ quats,
                                                       const float4 *__restrict__ sh, int sh_deg,
                                                       CamParams cam, float2 *__restrict__ means2d,
                                                       float *__restrict__ conics,
                                                       float *__restrict__ depths,
                                                       int *__restrict__ radii,
                                                       float *__restrict__ rgb,
                                                       uint32_t *__restrict__ tiles_touched) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    float tx = cam.R[0] * mx + cam.R[1] * my + cam.R[2] * mz + cam.t[0];
    float ty = cam.R[3] * mx + cam.R[4] * my + cam.R[5] * mz + cam.t[1];
    float tz = cam.R[6] * mx + cam.R[7] * my + cam.R[8] * mz + cam.t[2];
    int r = 0;
    uint32_t nt = 0;
    float2 m2 = make_float2(0.f, 0.f);
    float3 con = make_float3(0.f, 0.f, 0.f);
    float col[3] = {0.f, 0.f, 0.f};
    if (tz > cam.near_z) {
        float4 q = quats[i];
        float qn = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
        float w = q.x * qn, x = q.y * qn, y = q.z * qn, z = q.w * qn;
        float Rq[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                       2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                       2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
        float s0 = scales[3 * i], s1 = scales[3 * i + 1], s2 = scales[3 * i + 2];
        float ss[3] = {s0 * s0, s1 * s1, s2 * s2};
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
                A[a][c] = M[a][0] * Rq[c] + M[a][1] * Rq[3 + c] + M[a][2] * Rq[6 + c];
        float ca = cam.lowpass, cb = 0.f, cc = cam.lowpass;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ca = fmaf(A[0][k] * ss[k], A[0][k], ca);
            cb = fmaf(A[0][k] * ss[k], A[1][k], cb);
            cc = fmaf(A[1][k] * ss[k], A[1][k], cc);
        }
        m2 = make_float2(cam.fx * tx * inv_z + cam.cx, cam.fy * ty * inv_z + cam.cy);
        if (conic_radius(ca, cb, cc, con, r)) {
            int tx0, tx1, ty0, ty1;
            nt = (uint32_t)gs::tile_rect(m2.x, m2.y, r, cam.W, cam.H, cam.gx, tx0, tx1, ty0, ty1);
        }
        if (nt == 0) {
            r = 0;
            m2 = make_float2(0.f, 0.f);
            con = make_float3(0.f, 0.f, 0.f);
        } else {
            float dx = mx - cam.cpos[0], dy = my - cam.cpos[1], dz = mz - cam.cpos[2];
            float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
            sh_colour(sh + (size_t)i * 12, sh_deg, dx * dn, dy * dn, dz * dn, col);
        }
    }
    means2d[i] = m2;
    conics[3 * i] = con.x;
    conics[3 * i + 1] = con.y;
    conics[3 * i + 2] = con.z;
    depths[i] = nt ? tz : 0.0f;
    radii[i] = r;
    rgb[3 * i] = col[0];
    rgb[3 * i + 1] = col[1];
    rgb[3 * i + 2] = col[2];
    tiles_touched[i] = nt;
}

__global__ __launch_bounds__(256) void k_preprocess_2d(int P, const float2 *__restrict__ means2d,
                                                       const float *__restrict__ cov2d, int W, int H,
                                                       int gx, float *__restrict__ conics,
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
}

}  // namespace

extern "C" gs_status gs_preprocess(int32_t P, const float *means3d, const float *scales,
                                   const float *quats, const float *sh, int32_t sh_degree,
                                   const gs_camera *cam, float *means2d, float *conics,
                                   float *depths, int32_t *radii, float *rgb,
                                   uint32_t *tiles_touched, void *stream) {
    if (P < 0 || !cam || sh_degree < 0 || sh_degree > 3) return GS_ERR_INVALID_ARG;
    if (cam->width <= 0 || cam->height <= 0 || cam->width > GS_MAX_DIM || cam->height > GS_MAX_DIM)
        return GS_ERR_INVALID_ARG;
    if (!(cam->fx > 0.f) || !(cam->fy > 0.f)) return GS_ERR_INVALID_ARG;
    if (P == 0) return GS_OK;
    const void *ptrs[] = {means3d, scales, quats, sh, means2d, conics, depths, radii, rgb, tiles_touched};
    for (const void *p : ptrs)
        if (!p || !gs::aligned(p, 4)) return GS_ERR_INVALID_ARG;
    if (!gs::aligned(quats, 16) || !gs::aligned(sh, 16) || !gs::aligned(means2d, 8))
        return GS_ERR_INVALID_ARG;
    CamParams cp;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) cp.R[3 * r + c] = cam->viewmat[4 * r + c];
        cp.t[r] = cam->viewmat[4 * r + 3];
    }
    cp.fx = cam->fx;
    cp.fy = cam->fy;
    cp.cx = cam->cx;
    cp.cy = cam->cy;
    cp.W = cam->width;
    cp.H = cam->height;
    cp.gx = gs::grid_x(cam->width);
    cp.near_z = cam->near_z;
    cp.limx = cam->frustum_guard * (0.5f * cam->width / cam->fx);
    cp.limy = cam->frustum_guard * (0.5f * cam->height / cam->fy);
    cp.lowpass = cam->lowpass;
    for (int k = 0; k < 3; ++k) cp.cpos[k] = cam->campos[k];
    hipStream_t s = (hipStream_t)stream;
    int blocks = (P + 255) / 256;
    hipLaunchKernelGGL(k_preprocess_3d, dim3(blocks), dim3(256), 0, s, P, means3d, scales,
                       (const float4 *)quats, (const float4 *)sh, sh_degree, cp, (float2 *)means2d,
                       conics, depths, radii, rgb, tiles_touched);
    return gs::launch_status();
}

extern "C" gs_status gs_preprocess_2d(int32_t P, const float *means2d, const float *cov2d,
                                      int32_t width, int32_t height, float *conics,
                                      int32_t *radii, uint32_t *tiles_touched, void *stream) {
    if (P < 0 || width <= 0 || height <= 0 || width > GS_MAX_DIM || height > GS_MAX_DIM)
        return GS_ERR_INVALID_ARG;
    if (P == 0) return GS_OK;
    const void *ptrs[] = {means2d, cov2d, conics, radii, tiles_touched};
    for (const void *p : ptrs)
        if (!p || !gs::aligned(p, 4)) return GS_ERR_INVALID_ARG;
    if (!gs::aligned(means2d, 8)) return GS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    int blocks = (P + 255) / 256;
    hipLaunchKernelGGL(k_preprocess_2d, dim3(blocks), dim3(256), 0, s, P, (const float2 *)means2d,
                       cov2d, width, height, gs::grid_x(width), conics, radii, tiles_touched);
    return gs::launch_status();
}
