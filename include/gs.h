/*
 * gs.h -- C ABI of libgsmfma, a tile-based Gaussian-splatting rasteriser for
 * AMD Instinct MI355X (gfx950).
 *
 * The library implements the forward rendering path of 3D Gaussian Splatting
 * as described in Sec. 3.1 of the TC-GS paper (arXiv 2505.24796): preprocess
 * (projection of 3D Gaussians to 2D), sorting (per-tile depth-ordered splat
 * lists) and conditional alpha-blending (Algorithm 1), with the alpha
 * computation optionally recast as a matrix product on the matrix cores
 * (EarlyCull, Frag2Mat and G2L, Sec. 4.1-4.3).
 *
 * General conventions (all entry points):
 *   - Every pointer argument except `cam`, `background` and explicit host
 *     pointers is a DEVICE pointer, owned by the caller; the library never
 *     allocates, frees or retains it.  Device pointers must be 4-byte aligned
 *     (16-byte for `sh`, `workspace`); misalignment returns GS_ERR_INVALID_ARG.
 *   - All work is enqueued on `stream` (a hipStream_t; NULL means the default
 *     stream) and is asynchronous: a GS_OK return means the work was queued.
 *   - Host-side argument errors return immediately and enqueue nothing.
 *   - Images are at most 16384 x 16384; tiles are 16 x 16 pixels, tile
 *     (tx, ty) has index ty * ceil(W/16) + tx.  Pixel (x, y) has image-plane
 *     coordinate (x, y).
 *   - Per-Gaussian arrays are indexed by Gaussian id in [0, P).
 *   - No exceptions cross the ABI.  The functions keep no global state apart
 *     from a lazily initialised, thread-safe cache of device properties.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARG = 1,      /* null/misaligned pointer, bad size or enum */
    GS_ERR_UNSUPPORTED = 2,      /* valid request this build does not serve   */
    GS_ERR_HIP = 3,              /* a HIP runtime call failed                 */
    GS_ERR_CAPACITY = 4,         /* workspace smaller than required           */
    GS_ERR_NOT_IMPLEMENTED = 5
} gs_status;

/* How the rasteriser computes the exponent of each pixel-Gaussian pair.
 *   FP32            Algorithm 1 literally: alpha = o exp(-q/2) per pair on the
 *                   vector ALUs, then the 1/255 test (Sec. 3.1).
 *   FP32_EARLYCULL  beta = ln o - q/2 on the vector ALUs, cull on beta before
 *                   any exp (Sec. 4.1).
 *   FP16_GLOBAL     Frag2Mat (Sec. 4.2) on FP16 matrix cores in image
 *                   coordinates, K = 8 layout (Sec. 5.1).  Negative control:
 *                   the quadratic pixel terms lose precision or overflow.
 *   FP16_G2L        Frag2Mat + G2L local tile coordinates (Sec. 4.3), FP16,
 *                   K = 8 layout with v0/3 three times (Sec. 5.1).
 *   FP16_G2L_SPLIT  as FP16_G2L, with each coefficient split into FP16 high
 *                   and low parts in the spare K slots (K = 16).
 *   BF16_G2L_SPLIT  BF16 with a three-way high/mid/low split (K = 24 of 32).
 * All matrix-core variants accumulate in FP32 and apply EarlyCull. */
typedef enum {
    GS_PREC_FP32 = 0,
    GS_PREC_FP32_EARLYCULL = 1,
    GS_PREC_FP16_GLOBAL = 2,
    GS_PREC_FP16_G2L = 3,
    GS_PREC_FP16_G2L_SPLIT = 4,
    GS_PREC_BF16_G2L_SPLIT = 5
} gs_precision;

/* Pinhole camera (OpenCV axes: x right, y down, z forward). */
typedef struct {
    float viewmat[16];    /* world -> camera, row-major 4x4 [R t; 0 1]          */
    float fx, fy, cx, cy; /* focal lengths and principal point, pixels          */
    int32_t width, height;
    float near_z;         /* Gaussians with view depth <= near_z are dropped    */
    float frustum_guard;  /* x/z, y/z clamped to guard*tan(fov/2) inside J      */
    float lowpass;        /* added to both diagonal entries of Sigma' (px^2)    */
    float campos[3];      /* camera centre in world coordinates (SH direction)  */
} gs_camera;

/* Returns a static, human-readable name for a gs_status value. */
const char *gs_status_string(int status);

/* Library ABI version (major * 100 + minor). */
int gs_version(void);

/*
 * gs_preprocess -- project P 3D Gaussians (Sec. 3.1, "Preprocess":
 * mu' = W mu, Sigma' = J W Sigma W^T J^T).
 *   means3d  [P][3]  world-space means            scales [P][3] per-axis std
 *   quats    [P][4]  rotation (w, x, y, z), normalised internally
 *   sh       [P][16][3] real SH coefficients (Condon-Shortley phase), degree
 *            sh_degree in 0..3 (coefficients beyond the degree are ignored)
 * Outputs, per Gaussian:
 *   means2d [P][2] pixel-space centre; conics [P][3] = (s11, s12, s22) of
 *   Sigma'^-1; depths [P] view-space z; radii [P] = ceil(3 sqrt(lambda_max))
 *   (0 = dropped: behind near_z, det(Sigma') <= 0, or touching no tile);
 *   rgb [P][3] = max(0, SH(view direction) + 0.5); tiles_touched [P].
 * The 2x2 determinant and inverse run in FP64 when FP32 would cancel.
 * Errors: GS_ERR_INVALID_ARG for P < 0, null pointers (when P > 0), bad
 * camera size or sh_degree; GS_ERR_HIP if the launch fails.
 */
gs_status gs_preprocess(int32_t P, const float *means3d, const float *scales, const float *quats,
                        const float *sh, int32_t sh_degree, const gs_camera *cam,
                        float *means2d, float *conics, float *depths, int32_t *radii,
                        float *rgb, uint32_t *tiles_touched, void *stream);

/*
 * gs_preprocess_2d -- pre-projected Gaussians: Sigma' = (a, b, c) given as
 * cov2d [P][3] (no dilation).  Writes conics, radii and tiles_touched as
 * gs_preprocess does.  Errors as gs_preprocess.
 */
gs_status gs_preprocess_2d(int32_t P, const float *means2d, const float *cov2d, int32_t width,
                           int32_t height, float *conics, int32_t *radii, uint32_t *tiles_touched,
                           void *stream);

/*
 * Workspace bytes gs_bin_sort needs for P Gaussians, room for `capacity`
 * splats and a width x height image.  Returns 0 for invalid sizes.
 */
size_t gs_bin_sort_workspace_bytes(int32_t P, uint32_t capacity, int32_t width, int32_t height);

/*
 * gs_bin_sort -- build the per-tile, depth-ordered splat lists (Sec. 3.1,
 * "Sorting").  A Gaussian with centre mu' and radius r > 0 covers every tile
 * met by the pixel box [floor(mu'x) - r, floor(mu'x) + r] x [floor(mu'y) - r,
 * floor(mu'y) + r] (clamped to the image; centres with |coordinate| >= 2^22
 * are skipped).  Within a tile, splats are ordered by depth ascending, then
 * Gaussian id ascending (a stable order; -0.0 equals +0.0; Gaussians with a
 * non-finite depth are skipped).
 *   sorted_ids [capacity]   Gaussian id of each splat, tile-major
 *   tile_ranges [ntiles][2] [start, end) into sorted_ids per tile
 *   d_num_splats [1]        device word receiving N, the total splat count
 * The count N is data-dependent and stays on the device.  If N > capacity the
 * lists are not built, every tile range is empty (the frame renders as
 * background) and *d_num_splats still receives N, so the caller can read it
 * after synchronising and retry with a larger capacity.
 * capacity must be below 2^31.
 * Errors: GS_ERR_INVALID_ARG for bad sizes or pointers; GS_ERR_CAPACITY if
 * workspace_bytes < gs_bin_sort_workspace_bytes(...); GS_ERR_HIP.
 */
gs_status gs_bin_sort(int32_t P, const float *means2d, const int32_t *radii, const float *depths,
                      int32_t width, int32_t height, uint32_t capacity, void *workspace,
                      size_t workspace_bytes, uint32_t *sorted_ids, uint32_t *tile_ranges,
                      uint32_t *d_num_splats, void *stream);

/*
 * gs_rasterize_fwd -- conditional alpha-blending (Algorithm 1) per 16x16
 * tile.  For each pixel, front to back over its tile's list:
 *   alpha = min(0.99, o exp(beta)), beta = ln o - 1/2 d^T Sigma'^-1 d,
 *   d = mu' - p; skip the pair when alpha < 1/255 (equivalently beta <
 *   -ln 255, Sec. 4.1); stop the pixel, without compositing, when
 *   T - alpha T < 1e-4; otherwise C += c alpha T and T -= alpha T.
 * How beta is computed is selected by `precision` (gs_precision).
 *   means2d [P][2], conics [P][3], opacities [P] in (0, 1], rgb [P][3]
 *   background  HOST pointer to 3 floats composited as C + T * bg (NULL = 0)
 *   out_rgb [3][H][W] planar colour; out_T [H][W] final transmittance;
 *   out_ncontrib [H][W] 1-based position in the tile list of the last
 *   composited splat (0 if none).
 *   d_counters  NULL, or device uint64[4] that the call ADDS fragment counts
 *   to: {blended, culled, terminating, pairs = the three summed}; counting
 *   slows the kernel and is meant for diagnostics only.
 * Errors: GS_ERR_INVALID_ARG for bad sizes, pointers or precision; GS_ERR_HIP.
 */
gs_status gs_rasterize_fwd(int32_t width, int32_t height, const uint32_t *tile_ranges,
                           const uint32_t *sorted_ids, const float *means2d, const float *conics,
                           const float *opacities, const float *rgb, const float *background,
                           int32_t precision, float *out_rgb, float *out_T, uint32_t *out_ncontrib,
                           uint64_t *d_counters, void *stream);

/*
 * gs_rasterize_bwd -- gradients of a loss through gs_rasterize_fwd (the
 * backward of Algorithm 1).  Given dL_dimg = dL/dC [3][H][W] (planar, the
 * same layout as out_rgb) and the forward's out_T and out_ncontrib, walks
 * each pixel's blended fragments in reverse, recovering the transmittance by
 * division, and ADDS to (caller zeroes):
 *   dL_dmeans2d [P][2], dL_dconics [P][3] (d/d(s11, s12, s22)),
 *   dL_dopacities [P], dL_drgb [P][3].
 * The derivative is that of alpha = min(0.99, o exp(beta)) with the clamp's
 * zero slope where it is active; culled and skipped fragments contribute
 * nothing.  `precision` must be the one the forward used: fragments are
 * re-evaluated with the same arithmetic so every cull and termination
 * decision agrees with the forward.  Results are summed with atomics, so the
 * last bits may differ between runs.
 * Errors: GS_ERR_INVALID_ARG for bad sizes, pointers or precision; GS_ERR_HIP.
 */
gs_status gs_rasterize_bwd(int32_t width, int32_t height, const uint32_t *tile_ranges,
                           const uint32_t *sorted_ids, const float *means2d, const float *conics,
                           const float *opacities, const float *rgb, const float *background,
                           int32_t precision, const float *out_T, const uint32_t *out_ncontrib,
                           const float *dL_dimg, float *dL_dmeans2d, float *dL_dconics,
                           float *dL_dopacities, float *dL_drgb, void *stream);

/*
 * gs_rasterize_beta -- diagnostic: the exponent matrix B = U^T V (Sec. 4.2,
 * eq. MM) of one tile, exactly as the matrix-core path of gs_rasterize_fwd
 * computes it for `precision` (one of the FP16/BF16 variants), in log2
 * units (beta * log2 e).  Covers the first `count` splats of the tile's
 * list.  out_beta [count][256] (row = splat, column = pixel 16*y + x within
 * the tile) must hold count * 256 floats.  Errors: GS_ERR_INVALID_ARG.
 */
gs_status gs_rasterize_beta(int32_t width, int32_t height, int32_t tile, const uint32_t *tile_ranges,
                            const uint32_t *sorted_ids, const float *means2d, const float *conics,
                            const float *opacities, int32_t precision, int32_t count,
                            float *out_beta, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
