/*
 * gs_oracle.c -- FP64 CPU oracle for tile-based Gaussian splatting.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, deliberately unoptimised
 * implementation of what the GPU rasterisation path computes.  It is loaded
 * only by the test suite, the smoke check and the benchmark's CPU-baseline
 * leg; the product library never links, loads or calls it, and the two share
 * no code (no headers, helpers, tables or constants).
 *
 * What it follows (citations are to the TC-GS paper, arXiv 2505.24796):
 *   - 3D Gaussian density and the preprocessing projection
 *     mu' = W mu, Sigma' = J W Sigma W^T J^T            (Sec. 3.1, "Preprocess")
 *   - tiles, splats and per-tile depth order             (Sec. 3.1, "Sorting")
 *   - conditional alpha-blending                         (Sec. 3.1, Algorithm 1,
 *                                                          eqs. alpha_raw, vanilla
 *                                                          pruning, alpha-blending)
 *   - fragment categories culled / blended / skipped     (Sec. 3.2, Table 2)
 *   - exponent form beta = ln o - 1/2 d^T S d            (Sec. 4.1, EarlyCull)
 *   - Frag2Mat coefficients v0..v5 and B = U^T V         (Sec. 4.2)
 *   - G2L local coordinates about the tile centre        (Sec. 4.3)
 *   - K = 8 padding (v0/3 three times)                   (Sec. 5.1, Implementation)
 *
 * Readings where the paper is silent (all stated again in the design notes):
 *   - alpha is clamped to at most 0.99; culling is strict (alpha < 1/255);
 *     termination follows Algorithm 1: test T - alpha*T < 1e-4 before
 *     compositing, and stop without compositing that fragment.
 *   - pixel (x, y) has coordinate (x, y); the tile centre of tile (tx, ty) is
 *     (16 tx + 7.5, 16 ty + 7.5).
 *   - coverage: a Gaussian with centre mu' and integer radius r covers the
 *     pixel-index box [floor(mu'x) - r, floor(mu'x) + r] x [same in y], and
 *     every tile that box meets (clamped to the image).  r = ceil(3 sqrt(lmax))
 *     with lmax the larger eigenvalue of Sigma' (floored as below), clamped to
 *     2^22; a Gaussian whose centre has |coordinate| >= 2^22 is not binned.
 *   - order inside a tile: depth ascending, then Gaussian index ascending.
 *   - colour of a 3D Gaussian: real spherical harmonics (Condon-Shortley
 *     phase, orthonormal) up to degree 3 at the unit direction from the camera
 *     centre to the mean, plus 0.5, clamped below at 0.
 *   - projection: OpenCV pinhole, near plane 0.2 (Gaussians with view depth
 *     <= near are dropped), tx/tz and ty/tz clamped to 1.3 tan(fov/2) inside
 *     J, low-pass dilation Sigma' += 0.3 I, eigenvalue term floored at 0.1.
 *
 * Pins: Algorithm 1, binning and the emulated exponent are pinned by closed
 * forms, invariants, brute force and library routines in the tests.  The 3D
 * projection conventions above are readings of the 3DGS pipeline the paper
 * builds on (it prints no projection example); how this file implements each
 * of them is pinned by a route that shares nothing with the code below:
 * R(q) by rotations built from Hamilton products and a closed-form rotation
 * about a world axis, the SH basis function by function by Rodrigues'
 * formula for the associated Legendre functions plus the addition theorem,
 * Sigma' by finite-difference Jacobians of the pinhole map (at the clamped
 * point outside the guard band), and the optical axis and isotropic size by
 * closed forms.
 *
 * Everything here is double precision except where a function emulates the
 * rounding of a reduced-precision format on purpose (the *_emu modes), which
 * is spelled out at the rounding function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TILE 16
#define ORC_COORD_LIMIT 4194304.0 /* 2^22 */

/* ------------------------------------------------------------------------ */
/* Rounding to a binary floating-point format, round-to-nearest-even.       */
/* p = significand bits including the implicit one, emin = exponent of the  */
/* smallest normal, maxval = largest finite value.  Values below the normal */
/* range use the fixed subnormal spacing 2^(emin - p + 1).  Results whose   */
/* magnitude exceeds maxval after rounding become +-infinity.               */
/* fp16: p = 11, emin = -14, max 65504.  bf16: p = 8, emin = -126.          */
/* ------------------------------------------------------------------------ */
double orc_round_format(double x, int p, int emin, double maxval)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);            /* |x| in [2^(e-1), 2^e) */
    int lead = e - 1;
    if (lead < emin) lead = emin;
    double ulp = ldexp(1.0, lead - (p - 1));
    double y = nearbyint(x / ulp) * ulp; /* default mode: nearest, ties to even */
    if (fabs(y) > maxval) return copysign(INFINITY, x);
    return y;
}

static double rnd_h(double x) { return orc_round_format(x, 11, -14, 65504.0); }
static double rnd_b(double x) { return orc_round_format(x, 8, -126, ldexp(255.0, 120)); }

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics.                                                */
/* Y_lm for m > 0: sqrt2 K_lm cos(m phi) P_l^m(cos theta)                   */
/*          m < 0: sqrt2 K_l|m| sin(|m| phi) P_l^|m|(cos theta)             */
/*          m = 0: K_l0 P_l(cos theta)                                      */
/* K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), P_l^m with the Condon-Shortley */
/* phase, from the standard three-term recurrence in l.                     */
/* Output index l*l + l + m.                                                */
/* ------------------------------------------------------------------------ */
static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

static double assoc_legendre(int l, int m, double x)
{
    /* P_m^m = (-1)^m (2m-1)!! (1-x^2)^(m/2) */
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * s;
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm; /* P_{m+1}^m */
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

void orc_sh_basis(int deg, const double *dir, double *out)
{
    double n = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double x = dir[0] / n, y = dir[1] / n, z = dir[2] / n;
    double phi = atan2(y, x);
    for (int l = 0; l <= deg; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double P = assoc_legendre(l, am, z);
            double v;
            if (m > 0) v = sqrt(2.0) * K * cos(am * phi) * P;
            else if (m < 0) v = sqrt(2.0) * K * sin(am * phi) * P;
            else v = K * P;
            out[l * l + l + m] = v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Coverage rule (shared definition, independently implemented on the GPU). */
/* Writes the inclusive tile rectangle; returns the number of tiles.        */
/* ------------------------------------------------------------------------ */
static int64_t tile_rect(double mx, double my, int r, int W, int H, int *tx0, int *tx1,
                         int *ty0, int *ty1)
{
    if (r <= 0 || !isfinite(mx) || !isfinite(my)) return 0;
    if (fabs(mx) >= ORC_COORD_LIMIT || fabs(my) >= ORC_COORD_LIMIT) return 0;
    if (r > (int)ORC_COORD_LIMIT) r = (int)ORC_COORD_LIMIT;
    double fx = floor(mx), fy = floor(my);
    double x0 = fx - r, x1 = fx + r, y0 = fy - r, y1 = fy + r;
    if (x1 < 0 || y1 < 0 || x0 > W - 1 || y0 > H - 1) return 0;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > W - 1) x1 = W - 1;
    if (y1 > H - 1) y1 = H - 1;
    *tx0 = (int)x0 / ORC_TILE;
    *tx1 = (int)x1 / ORC_TILE;
    *ty0 = (int)y0 / ORC_TILE;
    *ty1 = (int)y1 / ORC_TILE;
    return (int64_t)(*tx1 - *tx0 + 1) * (*ty1 - *ty0 + 1);
}

/* Conic (inverse 2D covariance) and radius from Sigma' = [[a, b], [b, c]].
 * Returns 0 when the Gaussian is dropped (det <= 0 or not finite).
 * rad_dist receives the distance of 3 sqrt(lmax) to the nearest integer, so a
 * caller can tell which radii sit on a ceil boundary. */
static int conic_radius(double a, double b, double c, double *conic, int *radius,
                        double *rad_dist)
{
    double det = a * c - b * b;
    if (!(det > 0.0) || !isfinite(det)) return 0;
    conic[0] = c / det;
    conic[1] = -b / det;
    conic[2] = a / det;
    double mid = 0.5 * (a + c);
    double lmax = mid + sqrt(fmax(0.1, mid * mid - det));
    double r3 = 3.0 * sqrt(lmax);
    if (rad_dist) *rad_dist = fabs(r3 - nearbyint(r3));
    double rc = ceil(r3);
    if (rc > ORC_COORD_LIMIT) rc = ORC_COORD_LIMIT;
    *radius = (int)rc;
    return *radius > 0;
}

/* ------------------------------------------------------------------------ */
/* Preprocess, 3D scene (Sec. 3.1 "Preprocess").                            */
/* cam: viewmat[16] row-major world->camera, fx, fy, cx, cy, W, H, near,    */
/*      guard, lowpass, campos[3]  (28 doubles).                            */
/* Dropped Gaussians get radius 0 and tiles_touched 0.                      */
/* ------------------------------------------------------------------------ */
void orc_preprocess_3d(int P, const float *means, const float *scales, const float *quats,
                       const float *sh, int sh_deg, const double *cam,
                       double *means2d, double *cov2d, double *conics, double *depths,
                       int32_t *radii, double *rgb, int32_t *tiles_touched, double *rad_dist)
{
    const double *V = cam;
    double fx = cam[16], fy = cam[17], cx = cam[18], cy = cam[19];
    int W = (int)cam[20], H = (int)cam[21];
    double near_z = cam[22], guard = cam[23], lowpass = cam[24];
    const double *cpos = cam + 25;
    double limx = guard * (0.5 * W / fx), limy = guard * (0.5 * H / fy);
    int nsh = (sh_deg + 1) * (sh_deg + 1);

#pragma omp parallel for schedule(static)
    for (int i = 0; i < P; ++i) {
        radii[i] = 0;
        tiles_touched[i] = 0;
        means2d[2 * i] = means2d[2 * i + 1] = 0.0;
        depths[i] = 0.0;
        for (int k = 0; k < 3; ++k) conics[3 * i + k] = cov2d[3 * i + k] = rgb[3 * i + k] = 0.0;
        rad_dist[i] = 1.0;

        double m[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
        double t[3];
        for (int r = 0; r < 3; ++r) t[r] = V[4 * r] * m[0] + V[4 * r + 1] * m[1] + V[4 * r + 2] * m[2] + V[4 * r + 3];
        if (!(t[2] > near_z)) continue;

        /* R(q) for q = (w, x, y, z) normalised */
        double qw = quats[4 * i], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
        double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        double R[3][3] = {
            {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
            {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
            {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
        double s[3] = {scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]};
        /* Sigma = R diag(s^2) R^T */
        double Sig[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += R[a][k] * s[k] * s[k] * R[b][k];
                Sig[a][b] = acc;
            }
        /* J W: J = d(pixel)/d(camera point) at the clamped point */
        double tz = t[2];
        double xr = t[0] / tz, yr = t[1] / tz;
        if (xr < -limx) xr = -limx;
        if (xr > limx) xr = limx;
        if (yr < -limy) yr = -limy;
        if (yr > limy) yr = limy;
        double J[2][3] = {{fx / tz, 0.0, -fx * xr / tz}, {0.0, fy / tz, -fy * yr / tz}};
        double M[2][3]; /* J * Wrot */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += J[a][k] * V[4 * k + b];
                M[a][b] = acc;
            }
        double C2[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc += M[a][k] * Sig[k][l] * M[b][l];
                C2[a][b] = acc;
            }
        double ca = C2[0][0] + lowpass, cb = C2[0][1], cc = C2[1][1] + lowpass;
        double mx = fx * t[0] / tz + cx, my = fy * t[1] / tz + cy;
        double conic[3];
        int r;
        double rd;
        if (!conic_radius(ca, cb, cc, conic, &r, &rd)) continue;
        int tx0, tx1, ty0, ty1;
        int64_t nt = tile_rect(mx, my, r, W, H, &tx0, &tx1, &ty0, &ty1);
        if (nt == 0) continue;

        means2d[2 * i] = mx;
        means2d[2 * i + 1] = my;
        cov2d[3 * i] = ca; cov2d[3 * i + 1] = cb; cov2d[3 * i + 2] = cc;
        for (int k = 0; k < 3; ++k) conics[3 * i + k] = conic[k];
        depths[i] = tz;
        radii[i] = r;
        tiles_touched[i] = (int32_t)nt;
        rad_dist[i] = rd;

        /* colour: SH at the direction camera centre -> mean */
        double dir[3] = {m[0] - cpos[0], m[1] - cpos[1], m[2] - cpos[2]};
        double Y[16];
        orc_sh_basis(sh_deg, dir, Y);
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int k = 0; k < nsh; ++k) acc += Y[k] * sh[(size_t)i * 48 + 3 * k + ch];
            acc += 0.5;
            rgb[3 * i + ch] = acc < 0.0 ? 0.0 : acc;
        }
    }
}

/* Preprocess, pre-projected 2D Gaussians: covariance (a, b, c) given, no dilation. */
void orc_preprocess_2d(int P, const float *means2d, const float *cov2d, int W, int H,
                       double *conics, int32_t *radii, int32_t *tiles_touched, double *rad_dist)
{
    for (int i = 0; i < P; ++i) {
        radii[i] = 0;
        tiles_touched[i] = 0;
        rad_dist[i] = 1.0;
        conics[3 * i] = conics[3 * i + 1] = conics[3 * i + 2] = 0.0;
        double conic[3];
        int r;
        double rd;
        if (!conic_radius(cov2d[3 * i], cov2d[3 * i + 1], cov2d[3 * i + 2], conic, &r, &rd)) continue;
        int tx0, tx1, ty0, ty1;
        int64_t nt = tile_rect(means2d[2 * i], means2d[2 * i + 1], r, W, H, &tx0, &tx1, &ty0, &ty1);
        if (nt == 0) continue;
        for (int k = 0; k < 3; ++k) conics[3 * i + k] = conic[k];
        radii[i] = r;
        tiles_touched[i] = (int32_t)nt;
        rad_dist[i] = rd;
    }
}

/* ------------------------------------------------------------------------ */
/* Binning (Sec. 3.1 "Sorting"): every (tile, Gaussian) splat, ordered by   */
/* tile, then depth, then Gaussian index.  Inputs are the float32 values    */
/* the GPU sees; all decisions are exact on them.                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t tile;
    float depth;
    int32_t id;
} splat_t;

static int splat_cmp(const void *pa, const void *pb)
{
    const splat_t *a = (const splat_t *)pa, *b = (const splat_t *)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->depth != b->depth) return a->depth < b->depth ? -1 : 1;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return 0;
}

/* Precise Gaussian-tile intersection (the tighter binning of the pipelines
 * TC-GS composes with, Sec. 2.1, Tables 3 and 4): keep a tile of the 3-sigma
 * rectangle only if the raw opacity o exp(-q/2), q = d^T S d, d = p - mu',
 * reaches the culling threshold 1/255 of Algorithm 1 somewhere in the
 * tile's pixel box [16 tx, min(16 tx + 15, W - 1)] x [same in y] (the
 * convex hull of its pixel coordinates).  A tile that fails is culled at
 * each of its pixels, so dropping it changes no output.
 * The largest o exp(-q/2) over the box is at the box minimum of the convex
 * form q: zero if mu' is inside; otherwise on an edge, where q restricted to
 * the edge is a 1D quadratic minimised at its vertex clamped to the edge. */
static double box_min_q(double mx, double my, const double *S, double X0, double X1, double Y0,
                        double Y1)
{
    double a = S[0], b = S[1], c = S[2];
    if (mx >= X0 && mx <= X1 && my >= Y0 && my <= Y1) return 0.0;
    double best = INFINITY;
    for (int e = 0; e < 4; ++e) {
        double dx, dy;
        if (e < 2) {              /* vertical edge x = X0 or X1 */
            dx = (e == 0 ? X0 : X1) - mx;
            dy = -b * dx / c;
            if (dy < Y0 - my) dy = Y0 - my;
            if (dy > Y1 - my) dy = Y1 - my;
        } else {                  /* horizontal edge y = Y0 or Y1 */
            dy = (e == 2 ? Y0 : Y1) - my;
            dx = -b * dy / a;
            if (dx < X0 - mx) dx = X0 - mx;
            if (dx > X1 - mx) dx = X1 - mx;
        }
        double q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
        if (q < best) best = q;
    }
    return best;
}

static int tile_reaches_cull(double mx, double my, const double *S, double o, int tx, int ty,
                             int W, int H)
{
    double X0 = ORC_TILE * tx, Y0 = ORC_TILE * ty;
    double X1 = X0 + ORC_TILE - 1, Y1 = Y0 + ORC_TILE - 1;
    if (X1 > W - 1) X1 = W - 1;
    if (Y1 > H - 1) Y1 = H - 1;
    double q = box_min_q(mx, my, S, X0, X1, Y0, Y1);
    return o * exp(-0.5 * q) >= 1.0 / 255.0;
}

/* Slack of the precise test for one (Gaussian, tile): ln o - qmin/2 + ln 255
 * (>= 0: kept).  For tests that compare near-threshold decisions. */
double orc_tile_slack(double mx, double my, const double *S, double o, int tx, int ty, int W, int H)
{
    double X0 = ORC_TILE * tx, Y0 = ORC_TILE * ty;
    double X1 = X0 + ORC_TILE - 1, Y1 = Y0 + ORC_TILE - 1;
    if (X1 > W - 1) X1 = W - 1;
    if (Y1 > H - 1) Y1 = H - 1;
    return log(o) - 0.5 * box_min_q(mx, my, S, X0, X1, Y0, Y1) + log(255.0);
}

/* Does Gaussian i cover tile (tx, ty)?  3-sigma rectangle rule, plus the
 * precise test when conics/opac are given. */
static int covers(const float *means2d, const double *conics, const double *opac, int i, int tx,
                  int ty, int W, int H)
{
    if (!conics) return 1;
    return tile_reaches_cull(means2d[2 * i], means2d[2 * i + 1], conics + 3 * i, opac[i], tx, ty,
                             W, H);
}

/* Returns N (total splats).  Writes min(N, capacity) sorted ids and, when
 * N <= capacity, ranges[2*tile] = start, ranges[2*tile+1] = end.  With
 * conics (s11, s12, s22 per Gaussian) and opac non-NULL, a rectangle tile is
 * kept only if it passes the precise intersection test above. */
int64_t orc_bin(int P, const float *means2d, const int32_t *radii, const float *depths,
                int W, int H, uint32_t *ranges, uint32_t *ids, int64_t capacity,
                const double *conics, const double *opac)
{
    int gx = (W + ORC_TILE - 1) / ORC_TILE, gy = (H + ORC_TILE - 1) / ORC_TILE;
    int ntiles = gx * gy;
    int64_t N = 0;
    for (int i = 0; i < P; ++i) {
        int tx0, tx1, ty0, ty1;
        if (!isfinite(depths[i])) continue;
        if (!tile_rect(means2d[2 * i], means2d[2 * i + 1], radii[i], W, H, &tx0, &tx1, &ty0, &ty1)) continue;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx)
                N += covers(means2d, conics, opac, i, tx, ty, W, H);
    }
    for (int t = 0; t < 2 * ntiles; ++t) ranges[t] = 0;
    if (N == 0 || capacity <= 0) return N;
    splat_t *sp = (splat_t *)malloc((size_t)N * sizeof(splat_t));
    if (!sp) return -1;
    int64_t k = 0;
    for (int i = 0; i < P; ++i) {
        int tx0, tx1, ty0, ty1;
        if (!isfinite(depths[i])) continue;
        if (!tile_rect(means2d[2 * i], means2d[2 * i + 1], radii[i], W, H, &tx0, &tx1, &ty0, &ty1)) continue;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                if (!covers(means2d, conics, opac, i, tx, ty, W, H)) continue;
                sp[k].tile = ty * gx + tx;
                sp[k].depth = depths[i] == 0.0f ? 0.0f : depths[i]; /* -0 equals +0 */
                sp[k].id = i;
                ++k;
            }
    }
    qsort(sp, (size_t)N, sizeof(splat_t), splat_cmp);
    int64_t lim = N < capacity ? N : capacity;
    for (int64_t j = 0; j < lim; ++j) ids[j] = (uint32_t)sp[j].id;
    if (N <= capacity) {
        for (int64_t j = 0; j < N; ++j) {
            int t = sp[j].tile;
            if (j == 0 || sp[j - 1].tile != t) ranges[2 * t] = (uint32_t)j;
            if (j == N - 1 || sp[j + 1].tile != t) ranges[2 * t + 1] = (uint32_t)(j + 1);
        }
    }
    free(sp);
    return N;
}

/* Binning restricted to a list of tiles (for sampled checks of very large
 * frames): the same rule and order as orc_bin, but only splats on the listed
 * tiles are kept.  ranges[2*j], ranges[2*j+1] delimit the list of tile_list[j]
 * in ids.  Returns the number of kept splats (writes at most capacity ids). */
int64_t orc_bin_tiles(int P, const float *means2d, const int32_t *radii, const float *depths,
                      int W, int H, int ntl, const int32_t *tile_list, uint32_t *ranges,
                      uint32_t *ids, int64_t capacity, const double *conics, const double *opac)
{
    int gx = (W + ORC_TILE - 1) / ORC_TILE, gy = (H + ORC_TILE - 1) / ORC_TILE;
    int ntiles = gx * gy;
    int32_t *slot = (int32_t *)malloc((size_t)ntiles * sizeof(int32_t));
    if (!slot) return -1;
    for (int t = 0; t < ntiles; ++t) slot[t] = -1;
    for (int j = 0; j < ntl; ++j) slot[tile_list[j]] = j;
    int64_t cap = 1024, k = 0;
    splat_t *sp = (splat_t *)malloc((size_t)cap * sizeof(splat_t));
    if (!sp) { free(slot); return -1; }
    for (int i = 0; i < P; ++i) {
        int tx0, tx1, ty0, ty1;
        if (!isfinite(depths[i])) continue;
        if (!tile_rect(means2d[2 * i], means2d[2 * i + 1], radii[i], W, H, &tx0, &tx1, &ty0, &ty1)) continue;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                int j = slot[ty * gx + tx];
                if (j < 0) continue;
                if (!covers(means2d, conics, opac, i, tx, ty, W, H)) continue;
                if (k == cap) {
                    cap *= 2;
                    splat_t *n2 = (splat_t *)realloc(sp, (size_t)cap * sizeof(splat_t));
                    if (!n2) { free(sp); free(slot); return -1; }
                    sp = n2;
                }
                sp[k].tile = j;  /* position in tile_list, so the lists come out in list order */
                sp[k].depth = depths[i] == 0.0f ? 0.0f : depths[i];
                sp[k].id = i;
                ++k;
            }
    }
    qsort(sp, (size_t)k, sizeof(splat_t), splat_cmp);
    for (int j = 0; j < 2 * ntl; ++j) ranges[j] = 0;
    int64_t lim = k < capacity ? k : capacity;
    for (int64_t m = 0; m < lim; ++m) ids[m] = (uint32_t)sp[m].id;
    for (int64_t m = 0; m < k; ++m) {
        int j = sp[m].tile;
        if (m == 0 || sp[m - 1].tile != j) ranges[2 * j] = (uint32_t)m;
        if (m == k - 1 || sp[m + 1].tile != j) ranges[2 * j + 1] = (uint32_t)(m + 1);
    }
    free(sp);
    free(slot);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Exponent modes.                                                          */
/*  0 DEFINITION: alpha = o exp(-q/2), q = d^T S d, d = mu' - p (Alg. 1).   */
/*  Emulation modes evaluate beta = u^T v (Sec. 4.2) with the coefficient   */
/*  vector scaled by log2(e) and alpha = 2^beta, rounding v (and u) to the  */
/*  stated format exactly as a reduced-precision matrix unit would see it;  */
/*  the dot product itself is exact (double):                               */
/*  1 FP16, global coordinates, K = 8 layout (Sec. 5.1)                     */
/*  2 FP16, local coordinates (Sec. 4.3), K = 8 layout                      */
/*  3 FP16, local, v split into hi (v/256, met by 256 u) + lo FP16 parts    */
/*  4 BF16, local, v split into hi + mid + lo BF16 parts                    */
/* ------------------------------------------------------------------------ */
enum { MODE_DEF = 0, MODE_F16_GLOBAL = 1, MODE_F16_G2L = 2, MODE_F16_SPLIT = 3, MODE_BF16_SPLIT = 4 };

static const double LOG2E = 1.4426950408889634074;

/* Frag2Mat coefficients (Sec. 4.2) in a frame whose origin is `org`. */
static void frag2mat_v(const double *mu, const double *S, double lno, const double *org, double *v)
{
    double dx = mu[0] - org[0], dy = mu[1] - org[1];
    v[0] = lno - 0.5 * (S[0] * dx * dx + 2.0 * S[1] * dx * dy + S[2] * dy * dy);
    v[1] = S[0] * dx + S[1] * dy;
    v[2] = S[1] * dx + S[2] * dy;
    v[3] = -0.5 * S[0];
    v[4] = -S[1];
    v[5] = -0.5 * S[2];
}

/* Emulated exponent in log2 units for pixel p of tile with centre tc. */
double orc_beta_emulated(int mode, const double *mu, const double *S, double opac,
                         const double *p, const double *tc)
{
    double zero[2] = {0.0, 0.0};
    const double *org = (mode == MODE_F16_GLOBAL) ? zero : tc;
    double v[6];
    frag2mat_v(mu, S, log(opac), org, v);
    for (int i = 0; i < 6; ++i) v[i] *= LOG2E;
    double px = p[0] - org[0], py = p[1] - org[1];
    double u[6] = {1.0, px, py, px * px, px * py, py * py};
    double beta = 0.0;
    if (mode == MODE_F16_GLOBAL || mode == MODE_F16_G2L) {
        /* K = 8: v0/3 three times against three copies of the constant 1 */
        double w0 = rnd_h(v[0] / 3.0);
        beta = 3.0 * w0;
        for (int i = 1; i < 6; ++i) beta += rnd_h(u[i]) * rnd_h(v[i]);
    } else if (mode == MODE_F16_SPLIT) {
        /* hi part stored as v/256 in FP16 (met by 256 u), lo = v - 256 hi */
        for (int i = 0; i < 6; ++i) {
            double hi = 256.0 * rnd_h(v[i] / 256.0);
            double lo = rnd_h(v[i] - hi);
            beta += rnd_h(u[i]) * hi + rnd_h(u[i]) * lo;
        }
    } else if (mode == MODE_BF16_SPLIT) {
        for (int i = 0; i < 6; ++i) {
            double hi = rnd_b(v[i]);
            double mid = rnd_b(v[i] - hi);
            double lo = rnd_b(v[i] - hi - mid);
            double ub = rnd_b(u[i]);
            beta += ub * hi + ub * mid + ub * lo;
        }
    }
    return beta;
}

/* Per-pixel outputs of Algorithm 1. */
typedef struct {
    double C[3];
    double T;
    int32_t n_contrib; /* 1-based position (in the tile list) of the last blended fragment */
    int32_t n_proc;    /* non-skipped fragments: blended + culled + terminating */
    int32_t f_blend, f_cull;
    int32_t term;      /* 1 when the pixel stopped at a fragment (T - aT < 1e-4) */
    int32_t n_amb;     /* decisions within delta of a threshold */
    double sens;       /* sum over composited fragments of alpha T * (1/2 sum of |terms| of q) */
} pix_out_t;

typedef struct {
    const uint32_t *ranges, *ids;
    const double *means2d, *conics, *opac, *rgb;
    int W, H, mode;
    double dc, dr, dt;
} scene_ref_t;

/* Algorithm 1 for one pixel.  flip_mask: the j-th (j < 4) near-threshold
 * decision met along the way is inverted when bit j is set.  */
static void render_pixel(const scene_ref_t *s, int x, int y, unsigned flip_mask, pix_out_t *o)
{
    int gx = (s->W + ORC_TILE - 1) / ORC_TILE;
    int tx = x / ORC_TILE, ty = y / ORC_TILE, tile = ty * gx + tx;
    uint32_t start = s->ranges[2 * tile], end = s->ranges[2 * tile + 1];
    double p[2] = {(double)x, (double)y};
    double tc[2] = {ORC_TILE * tx + 0.5 * (ORC_TILE - 1), ORC_TILE * ty + 0.5 * (ORC_TILE - 1)};
    const double cull_ln = -log(255.0);
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    int nb = 0, nc = 0, term = 0, last = 0, namb = 0, nflag = 0;
    double sens = 0.0;
    for (uint32_t k = start; k < end; ++k) {
        uint32_t g = s->ids[k];
        const double *mu = s->means2d + 2 * g, *S = s->conics + 3 * g;
        double o = s->opac[g];
        double alpha, margin, band = s->dc, terms = 0.0;
        int cull;
        if (s->mode == MODE_DEF) {
            double dx = mu[0] - p[0], dy = mu[1] - p[1];
            double q = S[0] * dx * dx + 2.0 * S[1] * dx * dy + S[2] * dy * dy;
            alpha = o * exp(-0.5 * q);
            cull = alpha < 1.0 / 255.0;
            margin = (log(o) - 0.5 * q) - cull_ln;        /* distance in ln(alpha) */
            /* a reduced-precision evaluation errs relative to the size of the
             * quadratic form's terms, not of q itself */
            terms = 0.5 * (fabs(S[0]) * dx * dx + 2.0 * fabs(S[1] * dx * dy) + fabs(S[2]) * dy * dy);
            band += s->dr * terms;
        } else {
            /* EarlyCull (Sec. 4.1): the test on the exponent, here in log2 units */
            double b2 = orc_beta_emulated(s->mode, mu, S, o, p, tc);
            alpha = exp2(b2);
            cull = b2 < cull_ln * LOG2E;
            margin = (b2 - cull_ln * LOG2E) / LOG2E;
        }
        if (alpha > 0.99) alpha = 0.99;
        if (fabs(margin) < band) {
            ++namb;
            if (nflag < 4 && ((flip_mask >> nflag) & 1u)) cull = !cull;
            ++nflag;
        }
        if (cull) { ++nc; continue; }
        double test = T - alpha * T;
        int stop = test < 1e-4;
        if (fabs(test - 1e-4) < s->dt * 1e-4) {
            ++namb;
            if (nflag < 4 && ((flip_mask >> nflag) & 1u)) stop = !stop;
            ++nflag;
        }
        if (stop) { term = 1; break; }
        const double *c = s->rgb + 3 * g;
        for (int ch = 0; ch < 3; ++ch) C[ch] += c[ch] * alpha * T;
        /* First-order size of the result's response to errors in the
         * exponents: an error e_k in fragment k's exponent moves C by at most
         * alpha_k T_k (|c_k| + max |c|) |e_k| and T_final by at most
         * alpha_k T_k |e_k| (the fragments behind k carry at most T_{k+1}).
         * An evaluation that errs by rho times the size of q/2's terms moves
         * C by at most 2 max|c| rho sens and T by rho sens. */
        sens += alpha * T * terms;
        T = test;
        ++nb;
        last = (int)(k - start) + 1;
    }
    for (int ch = 0; ch < 3; ++ch) o->C[ch] = C[ch];
    o->T = T;
    o->n_contrib = last;
    o->n_proc = nb + nc + term;
    o->f_blend = nb;
    o->f_cull = nc;
    o->term = term;
    o->n_amb = namb;
    o->sens = sens;
}

/* Render the image (or only the listed tiles when ntl > 0).  Planar colour
 * out_rgb[3][H][W] with the background composited as C + T*bg. */
void orc_render(int W, int H, const uint32_t *ranges, const uint32_t *ids,
                const double *means2d, const double *conics, const double *opac,
                const double *rgb, const double *bg, int mode, double delta_c, double delta_r,
                double delta_t, int ntl, const int32_t *tile_list,
                double *out_rgb, double *out_T, int32_t *n_contrib, int32_t *n_proc,
                int32_t *f_blend, int32_t *f_cull, int32_t *term, int32_t *n_amb, double *sens)
{
    scene_ref_t s = {ranges, ids, means2d, conics, opac, rgb, W, H, mode, delta_c, delta_r, delta_t};
    int gx = (W + ORC_TILE - 1) / ORC_TILE, gy = (H + ORC_TILE - 1) / ORC_TILE;
    int nt = ntl > 0 ? ntl : gx * gy;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < nt; ++j) {
        int tile = ntl > 0 ? tile_list[j] : j;
        int tx = tile % gx, ty = tile / gx;
        for (int yy = 0; yy < ORC_TILE; ++yy)
            for (int xx = 0; xx < ORC_TILE; ++xx) {
                int x = tx * ORC_TILE + xx, y = ty * ORC_TILE + yy;
                if (x >= W || y >= H) continue;
                pix_out_t o;
                render_pixel(&s, x, y, 0u, &o);
                size_t pi = (size_t)y * W + x;
                for (int ch = 0; ch < 3; ++ch) out_rgb[(size_t)ch * W * H + pi] = o.C[ch] + o.T * bg[ch];
                out_T[pi] = o.T;
                n_contrib[pi] = o.n_contrib;
                n_proc[pi] = o.n_proc;
                f_blend[pi] = o.f_blend;
                f_cull[pi] = o.f_cull;
                term[pi] = o.term;
                n_amb[pi] = o.n_amb;
                if (sens) sens[pi] = o.sens;
            }
    }
}

/* Admissible alternatives for the listed pixels: for every combination of
 * inverting the first four near-threshold decisions (16 combinations) the
 * resulting colour (with background) and T are written to
 * alt_rgb[(j*16 + m)*3 + ch], alt_T[j*16 + m]. */
void orc_render_alternatives(int W, int H, const uint32_t *ranges, const uint32_t *ids,
                             const double *means2d, const double *conics, const double *opac,
                             const double *rgb, const double *bg, int mode, double delta_c,
                             double delta_r, double delta_t, int npix, const int32_t *pix_xy,
                             double *alt_rgb, double *alt_T)
{
    scene_ref_t s = {ranges, ids, means2d, conics, opac, rgb, W, H, mode, delta_c, delta_r, delta_t};
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < npix; ++j) {
        for (unsigned m = 0; m < 16; ++m) {
            pix_out_t o;
            render_pixel(&s, pix_xy[2 * j], pix_xy[2 * j + 1], m, &o);
            for (int ch = 0; ch < 3; ++ch) alt_rgb[((size_t)j * 16 + m) * 3 + ch] = o.C[ch] + o.T * bg[ch];
            alt_T[(size_t)j * 16 + m] = o.T;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Gradients (definition mode).  For a loss L with dL/dC given per pixel    */
/* (planar [3][H][W]), the derivative of Algorithm 1's output              */
/*   C_out = sum_k c_k a_k T_k + T_final bg,  T_{k+1} = T_k (1 - a_k)       */
/* over the blended fragments k of a pixel, with respect to each            */
/* fragment's a_k and c_k:                                                  */
/*   dC_out/dc_k = a_k T_k                                                  */
/*   dC_out/da_k = T_k (c_k - B_k),  B_k = (sum_{i>k} c_i a_i T_i +         */
/*                 T_final bg) / T_{k+1}                                    */
/* and a_k = o exp(-q/2) unless clamped at 0.99 (zero derivative there):    */
/*   da/do = exp(-q/2), da/dq = -a/2, dq/dmu = 2 S (mu - p),                */
/*   dq/d(s11, s12, s22) = (dx^2, 2 dx dy, dy^2).                           */
/* Culled and skipped fragments contribute nothing.  Accumulates into the   */
/* gradient arrays (caller zeroes).  Pixels are visited in order, so the    */
/* sums are deterministic.                                                  */
/* ------------------------------------------------------------------------ */
void orc_render_backward(int W, int H, const uint32_t *ranges, const uint32_t *ids,
                         const double *means2d, const double *conics, const double *opac,
                         const double *rgb, const double *bg, const double *dL_dC,
                         double *g_means2d, double *g_conics, double *g_opac, double *g_rgb)
{
    int gx = (W + ORC_TILE - 1) / ORC_TILE;
    size_t HW = (size_t)W * H;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int tile = (y / ORC_TILE) * gx + x / ORC_TILE;
            uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
            size_t pi = (size_t)y * W + x;
            double dC[3] = {dL_dC[pi], dL_dC[HW + pi], dL_dC[2 * HW + pi]};
            /* forward pass of this pixel, recording its blended fragments */
            int nbl = 0, cap = 64;
            uint32_t *kk = (uint32_t *)malloc((size_t)cap * sizeof(uint32_t));
            double *aa = (double *)malloc((size_t)cap * sizeof(double));
            double *tt = (double *)malloc((size_t)cap * sizeof(double));
            int *cl = (int *)malloc((size_t)cap * sizeof(int));
            double T = 1.0;
            for (uint32_t k = start; k < end; ++k) {
                uint32_t g = ids[k];
                const double *mu = means2d + 2 * g, *S = conics + 3 * g;
                double dx = mu[0] - x, dy = mu[1] - y;
                double q = S[0] * dx * dx + 2.0 * S[1] * dx * dy + S[2] * dy * dy;
                double a = opac[g] * exp(-0.5 * q);
                int clamped = a > 0.99;
                if (clamped) a = 0.99;
                if (a < 1.0 / 255.0) continue;
                double test = T - a * T;
                if (test < 1e-4) break;
                if (nbl == cap) {
                    cap *= 2;
                    kk = (uint32_t *)realloc(kk, (size_t)cap * sizeof(uint32_t));
                    aa = (double *)realloc(aa, (size_t)cap * sizeof(double));
                    tt = (double *)realloc(tt, (size_t)cap * sizeof(double));
                    cl = (int *)realloc(cl, (size_t)cap * sizeof(int));
                }
                kk[nbl] = g;
                aa[nbl] = a;
                tt[nbl] = T;
                cl[nbl] = clamped;
                ++nbl;
                T = test;
            }
            /* reverse traversal */
            double B[3] = {bg[0], bg[1], bg[2]};
            for (int j = nbl - 1; j >= 0; --j) {
                uint32_t g = kk[j];
                double a = aa[j], Tk = tt[j];
                const double *c = rgb + 3 * g;
                double da = 0.0;
                for (int ch = 0; ch < 3; ++ch) {
                    da += dC[ch] * Tk * (c[ch] - B[ch]);
                    g_rgb[3 * g + ch] += dC[ch] * a * Tk;
                    B[ch] = a * c[ch] + (1.0 - a) * B[ch];
                }
                if (cl[j]) continue;
                const double *mu = means2d + 2 * g, *S = conics + 3 * g;
                double dx = mu[0] - x, dy = mu[1] - y;
                double q = S[0] * dx * dx + 2.0 * S[1] * dx * dy + S[2] * dy * dy;
                g_opac[g] += da * exp(-0.5 * q);
                double dq = da * (-0.5 * a);
                g_means2d[2 * g] += dq * 2.0 * (S[0] * dx + S[1] * dy);
                g_means2d[2 * g + 1] += dq * 2.0 * (S[1] * dx + S[2] * dy);
                g_conics[3 * g] += dq * dx * dx;
                g_conics[3 * g + 1] += dq * 2.0 * dx * dy;
                g_conics[3 * g + 2] += dq * dy * dy;
            }
            free(kk);
            free(aa);
            free(tt);
            free(cl);
        }
}

/* Set the number of OpenMP threads of later parallel loops (timing only). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of OpenMP threads the parallel loops use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
