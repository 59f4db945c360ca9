"""Shared helpers of the GPU parity tests: device transfers, the oracle
comparison (admissible-set comparator for the FP32 path, statistics for the
reduced-precision paths) and image metrics."""
import numpy as np
import torch

import oracle

DELTA_C = 1e-5   # |ln alpha + ln 255| below this counts as a near-threshold cull decision
DELTA_T = 1e-3   # |T(1-a)/1e-4 - 1| below this counts as a near-threshold termination
DELTA_R = 1e-6   # plus this fraction of the quadratic form's term magnitudes (FP32: ~16 ulp)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def psnr(x, ref):
    mse = float(np.mean((x - ref) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def fp32_check(W, H, ranges, ids, means2d, conics, opac, rgb, gpu_rgb, gpu_T, tol=1e-4,
               tiles=None, bg=(0.0, 0.0, 0.0)):
    """FP32 path vs FP64 oracle: every pixel must be within its tolerance of
    some admissible result (decisions within delta of a threshold may go
    either way).  The tolerance is `tol` plus the FP32 evaluation error of
    Algorithm 1's exponent: an exponent computed from the conic's raw terms
    errs by up to ~DELTA_R times half their summed magnitude, which moves the
    colour by at most 2 max|c| DELTA_R sens and T by DELTA_R sens (the
    oracle's first-order bound, pinned on the CPU).  For well-conditioned
    splats the added term is far below `tol`; for near-degenerate needles,
    whose terms are large and cancel, it is what FP32 can do.  Returns a
    stats dict."""
    ref = oracle.render(W, H, ranges, ids, means2d, conics, opac, rgb, bg=bg,
                        delta_c=DELTA_C, delta_t=DELTA_T, delta_r=DELTA_R, tiles=tiles)
    mask = ~np.isnan(ref["T"])
    cm = max(float(np.abs(rgb).max()) if len(rgb) else 0.0, float(np.abs(bg).max()))
    sens = np.where(mask, ref["sens"], 0.0)
    tolC = tol + 2.0 * cm * DELTA_R * sens
    tolT = tol + DELTA_R * sens
    err = np.abs(gpu_rgb - ref["rgb"]).max(axis=0)
    errT = np.abs(gpu_T - ref["T"])
    amb = ref["n_amb"] > 0
    bad = mask & ((err > tolC) | (errT > tolT))
    hard = bad & ~amb
    assert not hard.any(), (f"{hard.sum()} unambiguous pixels off by up to {err[hard].max():.3e} "
                            f"(tolerance there {tolC[hard].min():.3e})")
    ys, xs = np.nonzero(bad & amb)
    if len(ys):
        alt, altT = oracle.render_alternatives(W, H, ranges, ids, means2d, conics, opac, rgb,
                                               np.stack([xs, ys], 1), bg=bg, delta_c=DELTA_C,
                                               delta_t=DELTA_T, delta_r=DELTA_R)
        for j, (x, y) in enumerate(zip(xs, ys)):
            e = np.abs(alt[j] - gpu_rgb[:, y, x]).max(axis=1)
            eT = np.abs(altT[j] - gpu_T[y, x])
            assert np.any((e <= tolC[y, x]) & (eT <= tolT[y, x])), (x, y, e.min())
    good = mask & ~bad
    return dict(max_abs=float(err[good].max()) if good.any() else 0.0,
                n_pix=int(mask.sum()), n_amb=int((mask & amb).sum()), n_flip=int(len(ys)),
                n_wide=int(np.sum(mask & (tolC > 2 * tol))), ref=ref)


def quality(gpu_rgb, ref_rgb, mask=None):
    """Reduced-precision statistics vs the FP64 oracle."""
    if mask is None:
        mask = np.ones(gpu_rgb.shape[1:], bool)
    d = np.abs(gpu_rgb - ref_rgb).max(axis=0)[mask]
    return dict(psnr=psnr(gpu_rgb[:, mask], ref_rgb[:, mask]), max_abs=float(d.max()),
                rms=float(np.sqrt(np.mean((gpu_rgb[:, mask] - ref_rgb[:, mask]) ** 2))),
                frac_2_255=float(np.mean(d <= 2.0 / 255.0)))
