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
 * Opacity crosses the boundary as its natural logarithm: preprocess turns
 * each opacity o into ln o once per Gaussian, and the rasterisers and the
 * precise binning take ln o, since the exponent the rasteriser evaluates is
 * beta = ln o - 1/2 d^T Sigma'^-1 d (Sec. 4.1) and no per-tile logarithm is
 * then needed.
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
 *     from a lazily initialised, thread-safe cache of device properties and
 *     the per-device scratch array of gs_bin_sort_noalloc.
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
 *   FP16_G2L_SPLIT_NOCULL  ablation only (Sec. 5.3, Table 5: Frag2Mat with
 *                   G2L, EarlyCull off): FP16_G2L_SPLIT's exponents, but
 *                   every listed splat is staged (no per-tile cull) and the
 *                   exp and blend run for every one of them.  The image is
 *                   that of FP16_G2L_SPLIT's counting launch (d_counters set),
 *                   which also keeps every splat.  gs_rasterize_fwd(_tuned)
 *                   only; the backward and the batched rasteriser reject it.
 * All other matrix-core variants accumulate in FP32 and apply EarlyCull. */
typedef enum {
    GS_PREC_FP32 = 0,
    GS_PREC_FP32_EARLYCULL = 1,
    GS_PREC_FP16_GLOBAL = 2,
    GS_PREC_FP16_G2L = 3,
    GS_PREC_FP16_G2L_SPLIT = 4,
    GS_PREC_BF16_G2L_SPLIT = 5,
    GS_PREC_FP16_G2L_SPLIT_NOCULL = 6
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

/* Library ABI version (major * 100 + minor); 200 = opacity as ln o; 201 =
 * gs_rasterize_fwd(_tuned) also accepts out_ncontrib = NULL; 202 = the
 * GS_PREC_FP16_G2L_SPLIT_NOCULL ablation variant. */
int gs_version(void);

/*
 * gs_preprocess -- project P 3D Gaussians (Sec. 3.1, "Preprocess":
 * mu' = W mu, Sigma' = J W Sigma W^T J^T).
 *   means3d  [P][3]  world-space means            scales [P][3] per-axis std
 *   quats    [P][4]  rotation (w, x, y, z), normalised internally
 *   opacities [P]    o in [0, 1]
 *   sh       [P][16][3] real SH coefficients (Condon-Shortley phase), degree
 *            sh_degree in 0..3 (coefficients beyond the degree are ignored)
 * Outputs, per Gaussian:
 *   means2d [P][2] pixel-space centre; conics [P][3] = (s11, s12, s22) of
 *   Sigma'^-1; log_opacities [P] = ln o (-inf for o = 0; written for every
 *   Gaussian); depths [P] view-space z; radii [P] = ceil(3 sqrt(lambda_max))
 *   (0 = dropped: behind near_z, det(Sigma') <= 0, or touching no tile);
 *   rgb [P][3] = max(0, SH(view direction) + 0.5); tiles_touched [P].
 * The 2x2 determinant and inverse run in FP64 when FP32 would cancel.
 * Errors: GS_ERR_INVALID_ARG for P < 0, null pointers (when P > 0), bad
 * camera size or sh_degree; GS_ERR_HIP if the launch fails.
 */
gs_status gs_preprocess(int32_t P, const float *means3d, const float *scales, const float *quats,
                        const float *opacities, const float *sh, int32_t sh_degree,
                        const gs_camera *cam, float *means2d, float *conics,
                        float *log_opacities, float *depths, int32_t *radii, float *rgb,
                        uint32_t *tiles_touched, void *stream);

/*
 * gs_preprocess_2d -- pre-projected Gaussians: Sigma' = (a, b, c) given as
 * cov2d [P][3] (no dilation), opacities [P] in [0, 1].  Writes conics,
 * log_opacities, radii and tiles_touched as gs_preprocess does.  Errors as
 * gs_preprocess.
 */
gs_status gs_preprocess_2d(int32_t P, const float *means2d, const float *cov2d,
                           const float *opacities, int32_t width, int32_t height, float *conics,
                           float *log_opacities, int32_t *radii, uint32_t *tiles_touched,
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
 * after synchronising and retry with a larger capacity.  *d_num_splats is
 * thus also the call's device-side status: N <= capacity means the lists are
 * complete, N > capacity means they overflowed (no separate status word).
 * capacity must be below 2^31.
 * Errors: GS_ERR_INVALID_ARG for bad sizes or pointers; GS_ERR_CAPACITY if
 * workspace_bytes < gs_bin_sort_workspace_bytes(...); GS_ERR_HIP.
 */
gs_status gs_bin_sort(int32_t P, const float *means2d, const int32_t *radii, const float *depths,
                      int32_t width, int32_t height, uint32_t capacity, void *workspace,
                      size_t workspace_bytes, uint32_t *sorted_ids, uint32_t *tile_ranges,
                      uint32_t *d_num_splats, void *stream);

/* Size of the device scratch array gs_bin_sort_noalloc works in (128 MiB:
 * room for gs_bin_sort_workspace_bytes() of, e.g., 1M Gaussians with up to
 * 7.2M splats, the 1920x1080 frame of a 1M-Gaussian scene). */
#define GS_NOALLOC_SCRATCH_BYTES (128u << 20)

/*
 * gs_bin_sort_noalloc -- gs_bin_sort without a workspace argument, for
 * callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The lists, counts
 * and overflow behaviour are exactly gs_bin_sort's.  The workspace is a
 * file-scope device array of GS_NOALLOC_SCRATCH_BYTES bytes that each GPU the
 * library runs on holds until the process ends; its device address is looked
 * up on the first call on a device (the only call that does more than
 * enqueue work), and no call allocates or frees memory.  Every call on one
 * GPU shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (several streams or threads at once) race, so order them
 * on one stream.  Nothing in the array needs to start at zero.
 * Errors: as gs_bin_sort; GS_ERR_CAPACITY if gs_bin_sort_workspace_bytes(P,
 * capacity, width, height) exceeds GS_NOALLOC_SCRATCH_BYTES (nothing is
 * enqueued); GS_ERR_HIP if the array's address cannot be found.
 */
gs_status gs_bin_sort_noalloc(int32_t P, const float *means2d, const int32_t *radii,
                              const float *depths, int32_t width, int32_t height,
                              uint32_t capacity, uint32_t *sorted_ids, uint32_t *tile_ranges,
                              uint32_t *d_num_splats, void *stream);

/* Workspace bytes gs_bin_sort_precise needs (0 for invalid sizes). */
size_t gs_bin_sort_precise_workspace_bytes(int32_t P, uint32_t capacity, int32_t width,
                                           int32_t height);

/*
 * gs_bin_sort_precise -- gs_bin_sort with a precise Gaussian-tile
 * intersection (the tighter binning of the pipelines TC-GS composes with,
 * Sec. 2.1, Tables 3 and 4): of the tiles the 3-sigma rectangle covers, a
 * Gaussian is listed only on those whose pixel box [16 tx, min(16 tx + 15,
 * W - 1)] x [same in y] holds a point where its raw opacity
 * o exp(-1/2 d^T S d) reaches the 1/255 culling threshold of Algorithm 1
 * (S = conic, d = point - mean).  Every dropped fragment is culled at each
 * pixel of its tile, so the rendered image is that of gs_bin_sort's lists;
 * fewer splats are sorted and visited.  Per tile row the kept tiles form one
 * contiguous run, found from the ellipse's chord in FP32 (determinant from
 * exact FP64 products) with every bound enlarged beyond its rounding: the
 * threshold 2 (ln o + ln 255) by a relative 4e-6 plus 4e-5, the ellipse's
 * vertical extent and half-widths by a relative 1e-6, the row's band and run
 * by 4e-6 (extent + |centre|) + 1e-4 px.  Rounding can thus keep a boundary
 * tile, never drop one.
 *   conics [P][3] (s11, s12, s22) and log_opacities [P] (ln o) as for
 *   gs_rasterize_fwd;
 *   everything else exactly as gs_bin_sort (order within a tile, capacity
 *   and overflow behaviour, d_num_splats).
 * Errors: as gs_bin_sort; GS_ERR_CAPACITY if workspace_bytes <
 * gs_bin_sort_precise_workspace_bytes(...).
 */
gs_status gs_bin_sort_precise(int32_t P, const float *means2d, const int32_t *radii,
                              const float *depths, const float *conics,
                              const float *log_opacities,
                              int32_t width, int32_t height, uint32_t capacity, void *workspace,
                              size_t workspace_bytes, uint32_t *sorted_ids, uint32_t *tile_ranges,
                              uint32_t *d_num_splats, void *stream);

/* Views one gs_bin_sort_multiview call can serve. */
#define GS_MAX_BIN_VIEWS 64

/* Workspace bytes gs_bin_sort_multiview needs (0 for invalid sizes). */
size_t gs_bin_sort_multiview_workspace_bytes(int32_t nviews, int32_t P, uint32_t capacity,
                                             const int32_t *widths, const int32_t *heights,
                                             int32_t precise);

/*
 * gs_bin_sort_multiview -- the per-tile lists of `nviews` views of one scene
 * (Sec. 3.1 "Sorting" per view) in one call: every stage runs once over all
 * (Gaussian, view) pairs instead of once per view.  The lists of each view
 * are exactly those gs_bin_sort (precise = 0) or gs_bin_sort_precise
 * (precise != 0) builds for that view alone; they are stored view after
 * view in one id array.
 *   nviews in [1, GS_MAX_BIN_VIEWS]; widths[v], heights[v] HOST arrays;
 *   means2d [nviews][P][2], radii [nviews][P], depths [nviews][P] and, when
 *   precise, conics [nviews][P][3] (as gs_preprocess_multiview writes them)
 *   and log_opacities [P] (ln o, shared by the views);
 *   sorted_ids [capacity]     Gaussian ids (0..P-1) of every view's lists
 *   tile_ranges [T][2]         T = sum over views of ceil(w/16) ceil(h/16);
 *                              view v's tiles come after those of views < v,
 *                              each view's in row-major order; [start, end)
 *                              index sorted_ids directly, so view v's
 *                              tile_ranges slice and the whole sorted_ids
 *                              array are what gs_rasterize_fwd (or a
 *                              gs_view) takes for that view
 *   d_num_splats [1]           total splat count N (device)
 *   d_view_splats [nviews]     per-view splat counts (device; may be NULL)
 * If N > capacity no list is built (every range empty); the counts are still
 * written, so the caller can size the next call.  nviews * P must be below
 * 2^31.  Errors: as gs_bin_sort, plus GS_ERR_INVALID_ARG for a bad view count
 * or size and GS_ERR_CAPACITY if workspace_bytes is below
 * gs_bin_sort_multiview_workspace_bytes(...).
 */
gs_status gs_bin_sort_multiview(int32_t nviews, int32_t P, const int32_t *widths,
                                const int32_t *heights, const float *means2d,
                                const int32_t *radii, const float *depths, const float *conics,
                                const float *log_opacities, int32_t precise, uint32_t capacity,
                                void *workspace, size_t workspace_bytes, uint32_t *sorted_ids,
                                uint32_t *tile_ranges, uint32_t *d_num_splats,
                                uint32_t *d_view_splats, void *stream);

/*
 * gs_rasterize_fwd -- conditional alpha-blending (Algorithm 1) per 16x16
 * tile.  For each pixel, front to back over its tile's list:
 *   alpha = min(0.99, o exp(beta)), beta = ln o - 1/2 d^T Sigma'^-1 d,
 *   d = mu' - p; skip the pair when alpha < 1/255 (equivalently beta <
 *   -ln 255, Sec. 4.1); stop the pixel, without compositing, when
 *   T - alpha T < 1e-4; otherwise C += c alpha T and T -= alpha T.
 * How beta is computed is selected by `precision` (gs_precision).
 *   means2d [P][2], conics [P][3], log_opacities [P] = ln o (o in [0, 1],
 *   as gs_preprocess writes it), rgb [P][3]
 *   background  HOST pointer to 3 floats composited as C + T * bg (NULL = 0)
 *   out_rgb [3][H][W] planar colour; out_T [H][W] final transmittance;
 *   out_ncontrib [H][W] 1-based position in the tile list of the last
 *   composited splat (0 if none); NULL = not written, and the kernels then
 *   skip that bookkeeping (gs_rasterize_bwd needs it: pass it when the
 *   frame will be differentiated).
 *   d_counters  NULL, or device uint64[4] that the call ADDS fragment counts
 *   to: {blended, culled, terminating, pairs = the three summed}; counting
 *   slows the kernel and is meant for diagnostics only.
 * Errors: GS_ERR_INVALID_ARG for bad sizes, pointers or precision; GS_ERR_HIP.
 */
gs_status gs_rasterize_fwd(int32_t width, int32_t height, const uint32_t *tile_ranges,
                           const uint32_t *sorted_ids, const float *means2d, const float *conics,
                           const float *log_opacities, const float *rgb, const float *background,
                           int32_t precision, float *out_rgb, float *out_T, uint32_t *out_ncontrib,
                           uint64_t *d_counters, void *stream);

/* Launch shape of the one-view rasteriser (chosen by an autotuner).
 *   batch       splats gathered and staged per round by the matrix-core
 *               kernels: 64, 128 or 256 (the FP32 kernels stage 256)
 *   chunk_rows  tile rows per XCD chunk: the row-major tiles are cut into
 *               chunks of about this many rows (1 or 2), chunk k served by
 *               XCD k mod 8, every XCD the same number of tiles */
typedef struct {
    int32_t batch;
    int32_t chunk_rows;
} gs_raster_tune;

/*
 * gs_rasterize_fwd_tuned -- gs_rasterize_fwd with an explicit launch shape
 * (tune: HOST pointer, NULL = {128, 2}, the shape gs_rasterize_fwd uses).
 * Every shape renders bit-identical outputs; only the time differs.
 * Counting launches (d_counters) use batch 128.  Errors: as
 * gs_rasterize_fwd, plus GS_ERR_INVALID_ARG for a shape outside the listed
 * values.
 */
gs_status gs_rasterize_fwd_tuned(int32_t width, int32_t height, const uint32_t *tile_ranges,
                                 const uint32_t *sorted_ids, const float *means2d,
                                 const float *conics, const float *log_opacities, const float *rgb,
                                 const float *background, int32_t precision,
                                 const gs_raster_tune *tune, float *out_rgb, float *out_T,
                                 uint32_t *out_ncontrib, uint64_t *d_counters, void *stream);

/*
 * gs_rasterize_bwd -- gradients of a loss through gs_rasterize_fwd (the
 * backward of Algorithm 1).  Given dL_dimg = dL/dC [3][H][W] (planar, the
 * same layout as out_rgb) and the forward's out_T and out_ncontrib, walks
 * each pixel's blended fragments in reverse, recovering the transmittance by
 * division, and ADDS to (caller zeroes):
 *   dL_dmeans2d [P][2], dL_dconics [P][3] (d/d(s11, s12, s22)),
 *   dL_dopacities [P] (d/do, o = exp(log_opacities)), dL_drgb [P][3].
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
                           const float *log_opacities, const float *rgb, const float *background,
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
                            const float *log_opacities, int32_t precision, int32_t count,
                            float *out_beta, void *stream);

/*
 * gs_preprocess_multiview -- gs_preprocess for `nviews` cameras of one scene
 * in one pass: each Gaussian's means3d, scales, quats and (if it is visible
 * in some view) sh are read once and projected into every camera.  `cams`
 * is a HOST array of nviews cameras (1 <= nviews <= 64).  Every output is
 * view-major with a stride of P entries: view v's means2d start at
 * means2d + 2 * v * P, conics at conics + 3 * v * P, depths/radii/
 * tiles_touched at + v * P, rgb at rgb + 3 * v * P; each view's slice is
 * what gs_preprocess with that camera writes.  log_opacities [P] (ln o, view
 * independent) is written once.
 * Errors: as gs_preprocess, plus GS_ERR_INVALID_ARG for nviews out of range.
 */
gs_status gs_preprocess_multiview(int32_t P, const float *means3d, const float *scales,
                                  const float *quats, const float *opacities, const float *sh,
                                  int32_t sh_degree, int32_t nviews, const gs_camera *cams,
                                  float *means2d, float *conics, float *log_opacities,
                                  float *depths, int32_t *radii, float *rgb,
                                  uint32_t *tiles_touched, void *stream);

/* One view of a batched frame: its image size, its own gs_bin_sort lists,
 * its gs_preprocess outputs and its output images, laid out exactly as for
 * gs_rasterize_fwd.  All pointers are DEVICE pointers. */
typedef struct {
    int32_t width, height;
    const uint32_t *tile_ranges; /* [ntiles][2]                              */
    const uint32_t *sorted_ids;  /* tile-major splat list of this view       */
    const float *means2d;        /* [P][2]                                   */
    const float *conics;         /* [P][3]                                   */
    const float *log_opacities;  /* [P] ln o                                 */
    const float *rgb;            /* [P][3]                                   */
    float background[3];         /* composited as C + T * bg                 */
    float *out_rgb;              /* [3][H][W]                                */
    float *out_T;                /* [H][W]                                   */
    uint32_t *out_ncontrib;      /* [H][W]                                   */
} gs_view;

/* Launch shape of gs_rasterize_fwd_batched (chosen by an autotuner).
 *   batch          splats gathered and staged per round: 64, 128 or 256
 *   blocks_per_cu  persistent workgroups per compute unit, 1..16 (the grid
 *                  is the CU count times this, rounded up to a multiple of 8)
 *   xcd_queues     1: eight work queues, one per XCD, holding bands of two
 *                  tile rows (band b -> queue b mod 8), with stealing once a
 *                  queue is empty; 0: one queue of row-major tiles */
typedef struct {
    int32_t batch;
    int32_t blocks_per_cu;
    int32_t xcd_queues;
} gs_batch_tune;

/* Bytes of the device plan for nviews views (0 if nviews is not 1..64). */
size_t gs_batch_plan_bytes(int32_t nviews);

/* Bytes of the device workspace gs_rasterize_fwd_batched needs (queue heads
 * and per-view tile counters; 0 if nviews is not 1..64). */
size_t gs_batch_workspace_bytes(int32_t nviews);

/*
 * gs_batch_plan_write -- build the device plan of a batched frame from a
 * HOST array of nviews gs_view and copy it to `plan` (device, 256-byte
 * aligned, gs_batch_plan_bytes(nviews) bytes).  SYNCHRONOUS (a blocking
 * host-to-device copy): call it once at set-up, outside stream capture; the
 * plan stays valid while the buffers it names do.
 * Errors: GS_ERR_INVALID_ARG (bad view or pointer), GS_ERR_CAPACITY (plan
 * too small), GS_ERR_HIP.
 */
gs_status gs_batch_plan_write(int32_t nviews, const gs_view *views, void *plan, size_t plan_bytes);

/*
 * gs_rasterize_fwd_batched -- gs_rasterize_fwd for every view of a plan in
 * ONE persistent launch (after a one-workgroup launch that clears the
 * workspace).  Workgroups take (view, tile) items from device work queues
 * until all are empty; each tile is rendered exactly as gs_rasterize_fwd
 * renders it, so every view's outputs are bit-identical to a one-view call.
 * Only the matrix-core precisions are served (GS_ERR_UNSUPPORTED for FP32).
 *   tune        HOST pointer, NULL = {256, 5, 1}
 *   workspace   device, gs_batch_workspace_bytes(nviews) bytes; a call
 *               overwrites it, so two calls in flight need two workspaces
 *   d_view_clock NULL, or device uint64[nviews] receiving, per view, the
 *               device wall clock (gs_wall_clock_khz ticks) at which its
 *               last tile finished
 * The call enqueues no memset and no host synchronisation, so it can be
 * captured in a hipGraph.
 * Errors: GS_ERR_INVALID_ARG, GS_ERR_CAPACITY (workspace), GS_ERR_UNSUPPORTED,
 * GS_ERR_HIP.
 */
gs_status gs_rasterize_fwd_batched(int32_t nviews, const void *plan, int32_t precision,
                                   const gs_batch_tune *tune, void *workspace,
                                   size_t workspace_bytes, uint64_t *d_view_clock, void *stream);

/* Enqueue a write of the device wall clock to *d_dst (device uint64). */
gs_status gs_clock_stamp(uint64_t *d_dst, void *stream);

/* Frequency of the device wall clock in kHz (host call, current device). */
gs_status gs_wall_clock_khz(int32_t *khz);

/*
 * gs_peak_probe -- diagnostic: enqueue one peak-rate probe of the device, for
 * roofline fractions stated against measured rather than assumed rates.
 * blocks workgroups of 256 threads each run `iters` rounds of independent
 * operations (timed by the caller with events on `stream`):
 *   kind 0  v_exp_f32 (x <- 2^-x), 8 per lane per round;
 *   kind 1  v_fma_f32 (2 flop), 8 per lane per round;
 *   kind 2  v_mfma_f32_32x32x16_f16 (32768 flop per wave instruction), 4 per
 *           wave per round.
 * d_out [blocks * 256] floats receives one value per thread (keeps the work
 * live).  Errors: GS_ERR_INVALID_ARG (kind, iters < 1, blocks outside
 * 1..2^20, null or misaligned d_out), GS_ERR_HIP.
 */
gs_status gs_peak_probe(int32_t kind, int32_t iters, int32_t blocks, float *d_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
