"""GPU parity of the whole path against the FP64 oracle's own chain, the
near-degenerate conic branch, and degenerate inputs.

* Whole chain (Sec. 3.1 pipeline): the GPU renders a 3D scene through its
  FP32 preprocess, its bin/sort and each rasteriser; the oracle renders the
  same scene through ITS OWN FP64 preprocess and binning and Algorithm 1.
  No GPU intermediate enters the reference, so the comparison states the
  error of the whole path against FP64.
* Near-degenerate 2D covariances (det < 2^-10 ac): the GPU takes the
  determinant and inverse in FP64; conics must match the oracle's to FP32
  rounding and the image must pass the usual bars.
* Degenerate inputs: opacity exactly 0 and 1, non-finite means, covariances,
  scales and quaternions.
"""
import sys

import numpy as np
import pytest

import oracle
import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_24796_amd as gs  # noqa: E402
from gpu_helpers import dev, fp32_check, host, quality  # noqa: E402

PRECS = ["fp32", "fp32_earlycull", "fp16_g2l_split", "bf16_g2l_split", "fp16_g2l"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gs_cam(c):
    return gs.make_camera(c.viewmat, c.fx, c.fy, c.cx, c.cy, c.width, c.height, campos=c.campos)


def chain_stats(img, ref, mask=None):
    q = quality(img, ref, mask)
    m = np.ones(img.shape[1:], bool) if mask is None else mask
    d = np.abs(img - ref).max(axis=0)[m]
    q["frac_1e-4"] = float(np.mean(d <= 1e-4))
    return q


def check_chain(prec, q):
    """Bars of the whole path against the FP64 chain.  Every precision: PSNR
    >= 50 dB and >= 99.9 % of pixels within 2/255 (FP32 preprocess rounding,
    ceil boundaries of the radius and depth-order ties make the whole-chain
    result differ from FP64 by more than the raster stage alone does); the
    FP32 raster additionally keeps >= 99 % of pixels within 1e-4.  The paper's
    K = 8 layout is held to the PSNR bar only (its per-pixel agreement is
    checked against its own rounding emulation elsewhere)."""
    assert q["psnr"] >= 50.0, (prec, q)
    if prec != "fp16_g2l":
        assert q["frac_2_255"] >= 0.999, (prec, q)
    if prec.startswith("fp32"):
        assert q["frac_1e-4"] >= 0.99, (prec, q)


def oracle_chain(sc, cam, tiles=None):
    """The FP64 chain: oracle preprocess, oracle binning of its own 2D
    footprint (means and depths rounded to float32 only for the binning
    rule's integer decisions and the sort key), Algorithm 1 in FP64."""
    o = oracle.preprocess_3d(sc, cam)
    W, H = cam.width, cam.height
    m32, d32 = o["means2d"].astype(np.float32), o["depths"].astype(np.float32)
    if tiles is None:
        ranges, ids = oracle.bin_splats(m32, o["radii"], d32, W, H)
        full = ranges
    else:
        gx, gy = oracle.grid(W, H)
        r_t, ids = oracle.bin_tiles(m32, o["radii"], d32, W, H, tiles)
        full = np.zeros((gx * gy, 2), np.uint32)
        full[tiles] = r_t
    ref = oracle.render(W, H, full, ids, o["means2d"], o["conics"], sc.opacities, o["rgb"],
                        tiles=tiles)
    return o, ref


@pytest.mark.parametrize("W,H,P,seed,pose", [(480, 270, 100_000, 4321, 0), (333, 250, 60_000, 77, 3)])
def test_whole_chain_3d_vs_fp64_chain(W, H, P, seed, pose):
    say(f"whole chain 3D P={P} {W}x{H} pose {pose}")
    sc = scenegen.scene_3d(P, seed)
    cam = scenegen.orbit_camera(pose, 8, W, H)
    o, ref = oracle_chain(sc, cam)
    pre = gs.preprocess(dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacities), dev(sc.sh),
                        gs_cam(cam))
    bs = gs.bin_sort(pre["means2d"], pre["radii"], pre["depths"], W, H)
    rad_g = host(pre["radii"])
    vis_g, vis_o = rad_g > 0, o["radii"] > 0
    say(f"  drawn: GPU {vis_g.sum()}, oracle {vis_o.sum()}, differing {np.sum(vis_g != vis_o)}; "
        f"splats GPU {bs.n_splats()}")
    assert np.mean(vis_g == vis_o) > 0.999
    opac = pre["log_opacities"]
    for prec in PRECS:
        r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, pre["means2d"], pre["conics"], opac,
                             pre["rgb"], prec)
        img, T = host(r.rgb), host(r.T)
        assert np.isfinite(img).all() and T.min() >= 1e-4 and T.max() <= 1.0
        q = chain_stats(img, ref["rgb"])
        say(f"  {prec}: PSNR {q['psnr']:.1f} dB, max|err| {q['max_abs']:.2e}, rms {q['rms']:.2e}, "
            f"within 1e-4 {q['frac_1e-4']:.5f}, within 2/255 {q['frac_2_255']:.6f}")
        check_chain(prec, q)


def test_near_degenerate_conic_takes_fp64_branch():
    """Needle-like splats at ~45 degrees (covariance ratio 1e4..9e4): the
    FP32 determinant ac - b^2 cancels (det < 2^-10 ac), so the GPU forms it
    and the inverse in FP64.  Conics equal the oracle's FP64 conics to FP32
    rounding; a well-conditioned half of the scene takes the FP32 branch and
    is checked the same way; the images of the FP32 path and of the FP16 and
    BF16 split variants meet the raster bars (the paper's K = 8 layout
    overflows FP16 on these splats, shown below).  The FP32
    raster evaluates Algorithm 1's exponent from the conic's raw terms, which
    for these needles are large and cancel: its per-pixel tolerance adds the
    first-order effect of that evaluation error (see fp32_check)."""
    W, H = 256, 200
    nd = scenegen.scene_2d_needles(1500, W, H, seed=41)
    ok = scenegen.scene_2d(1500, W, H, seed=42)
    cat = lambda a, b: np.concatenate([a, b])
    m2, cov = cat(nd.means2d, ok.means2d), cat(nd.cov2d, ok.cov2d)
    opac, rgb, dep = cat(nd.opacities, ok.opacities), cat(nd.rgb, ok.rgb), cat(nd.depths, ok.depths)
    a, b, c = cov[:, 0], cov[:, 1], cov[:, 2]
    # the branch test of the kernel, evaluated with the same FP32 roundings
    det32 = a * c - b * b
    branch = det32 < np.float32(2.0 ** -10) * a * c
    say(f"near-degenerate: {branch.sum()} of {len(a)} take the FP64 branch")
    assert branch[:1500].all() and not branch[1500:].any()
    pre = gs.preprocess_2d(dev(m2), dev(cov), dev(opac), W, H)
    o = oracle.preprocess_2d(m2, cov, W, H)
    rad = host(pre["radii"])
    same = rad == o["radii"]
    assert np.all(same | (o["rad_dist"] < 1e-4))
    vis = same & (rad > 0)
    assert vis[:1500].sum() > 1000
    cg = host(pre["conics"]).astype(np.float64)
    rel = np.abs(cg - o["conics"]) / np.abs(o["conics"]).max(axis=1, keepdims=True)
    say(f"  conic max rel err: FP64 branch {rel[vis & branch].max():.2e}, "
        f"FP32 branch {rel[vis & ~branch].max():.2e}")
    assert rel[vis & branch].max() < 2e-7
    assert rel[vis & ~branch].max() < 2e-5
    # what the FP32 formula would have given for the needles: far off
    inv32 = c / det32
    bad32 = np.abs(inv32 - o["conics"][:, 0]) / np.abs(o["conics"]).max(axis=1)
    say(f"  (an FP32 determinant would be off by up to {bad32[vis & branch].max():.1e})")
    ranges, ids = oracle.bin_splats(m2, rad, dep, W, H)
    bs = gs.bin_sort(dev(m2), pre["radii"], dev(dep), W, H)
    N = bs.n_splats()
    assert N == len(ids) and np.array_equal(host(bs.sorted_ids)[:N].astype(np.uint32), ids)
    results = {}
    for prec in PRECS:
        r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, dev(m2), pre["conics"],
                             pre["log_opacities"], dev(rgb), prec)
        img = host(r.rgb)
        if prec.startswith("fp32"):
            st = fp32_check(W, H, ranges, ids, m2, cg, opac, rgb, img, host(r.T))
            say(f"  {prec}: max|err| {st['max_abs']:.2e}, ambiguous {st['n_amb']}, flips {st['n_flip']}, "
                f"pixels whose FP32 exponent bound exceeds 1e-4: {st['n_wide']}")
        else:
            ref = oracle.render(W, H, ranges, ids, m2, cg, opac, rgb)
            results[prec] = q = quality(img, ref["rgb"])
            say(f"  {prec}: PSNR {q['psnr']:.1f} dB, max|err| {q['max_abs']:.2e}, "
                f"within 2/255 {q['frac_2_255']:.6f}")
    # The paper's K = 8 layout stores v0/3 and v1..v5 in plain FP16: at the
    # centre of a tile that a needle crosses off-centre, q/2 runs to 1e5 and
    # more, beyond FP16's 65504, so the row overflows and the splat is lost
    # at pixels on its axis.  The hi/lo split stores v/256 in its high part
    # (range 256 x 65504) and BF16 has FP32's range: those two meet the bars.
    assert results["fp16_g2l"]["psnr"] < 50.0
    for prec in ("fp16_g2l_split", "bf16_g2l_split"):
        q = results[prec]
        assert q["psnr"] >= 50.0, (prec, q)
        assert q["frac_2_255"] >= 0.999, (prec, q)


def test_degenerate_inputs_2d():
    """Opacity exactly 0 (never drawn: alpha = 0 < 1/255) and exactly 1
    (alpha clamped to 0.99 at the centre); non-finite means and covariances,
    and covariances that are not positive definite, get radius 0 and no
    splats.  Lists equal the oracle's and images pass the raster bars."""
    W, H = 200, 150
    sc = scenegen.scene_2d(1200, W, H, seed=43)
    m2, cov, opac = sc.means2d.copy(), sc.cov2d.copy(), sc.opacities.copy()
    nan, inf = np.float32("nan"), np.float32("inf")
    opac[0::10] = 0.0
    opac[1::10] = 1.0
    m2[2::40, 0] = nan
    m2[3::40, 1] = inf
    m2[4::40, 0] = -inf
    cov[5::40, 0] = nan
    cov[6::40, 1] = inf
    cov[7::40, 2] = -1.0          # indefinite
    cov[8::40] = [4.0, 2.0, 1.0]  # singular (det = 0)
    cov[9::40, :] = inf
    pre = gs.preprocess_2d(dev(m2), dev(cov), dev(opac), W, H)
    o = oracle.preprocess_2d(m2, cov, W, H)
    rad = host(pre["radii"])
    lno = host(pre["log_opacities"])
    assert np.all(lno[opac == 0] == -np.inf) and np.all(lno[opac == 1] == 0.0)
    bad = np.zeros(sc.P, bool)
    for k in range(2, 10):
        bad[k::40] = True
    say(f"degenerate 2D: {bad.sum()} invalid, opacity 0 x{np.sum(opac == 0)}, 1 x{np.sum(opac == 1)}")
    assert (rad[bad] == 0).all() and (o["radii"][bad] == 0).all()
    assert (host(pre["tiles_touched"])[bad] == 0).all()
    same = rad == o["radii"]
    assert np.all(same | (o["rad_dist"] < 1e-4))
    ranges, ids = oracle.bin_splats(m2, rad, sc.depths, W, H)
    bs = gs.bin_sort(dev(m2), pre["radii"], dev(sc.depths), W, H)
    N = bs.n_splats()
    assert N == len(ids) and np.array_equal(host(bs.sorted_ids)[:N].astype(np.uint32), ids)
    assert not np.isin(ids, np.nonzero(bad)[0]).any()
    cg = host(pre["conics"]).astype(np.float64)
    ref = oracle.render(W, H, ranges, ids, m2, cg, opac, sc.rgb)
    for prec in PRECS:
        r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, dev(m2), pre["conics"],
                             pre["log_opacities"], dev(sc.rgb), prec, count=True)
        img, T = host(r.rgb), host(r.T)
        assert np.isfinite(img).all() and T.min() >= 1e-4 and T.max() <= 1.0
        if prec.startswith("fp32"):
            st = fp32_check(W, H, ranges, ids, m2, cg, opac, sc.rgb, img, T)
            say(f"  {prec}: max|err| {st['max_abs']:.2e}")
        else:
            q = quality(img, ref["rgb"])
            say(f"  {prec}: PSNR {q['psnr']:.1f} dB, within 2/255 {q['frac_2_255']:.6f}")
            assert q["psnr"] >= 50.0
            if prec != "fp16_g2l":
                assert q["frac_2_255"] >= 0.999
    # a scene of opacity-0 Gaussians only renders the background everywhere
    z = gs.preprocess_2d(dev(m2), dev(cov), dev(np.zeros_like(opac)), W, H)["log_opacities"]
    r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, dev(m2), pre["conics"], z, dev(sc.rgb),
                         "fp16_g2l_split", background=(0.25, 0.5, 0.75))
    img = host(r.rgb)
    assert np.all(img[0] == 0.25) and np.all(img[1] == 0.5) and np.all(img[2] == 0.75)
    assert np.all(host(r.T) == 1.0) and np.all(host(r.n_contrib) == 0)


def test_degenerate_inputs_3d():
    """3D Gaussians with a non-finite mean, scale or quaternion, a zero
    quaternion, or opacity 0 / 1: the invalid ones are dropped by both the
    GPU and the oracle preprocess, and the whole chain still matches."""
    W, H = 320, 200
    sc = scenegen.scene_3d(40_000, 44)
    nan, inf = np.float32("nan"), np.float32("inf")
    sc.means[0::97, 0] = nan
    sc.means[1::97, 2] = inf
    sc.scales[2::97, 1] = nan
    sc.scales[3::97, 0] = inf
    sc.quats[4::97] = 0.0
    sc.quats[5::97, 2] = nan
    sc.opacities[6::13] = 0.0
    sc.opacities[7::13] = 1.0
    bad = np.zeros(sc.P, bool)
    for k in range(6):
        bad[k::97] = True
    cam = scenegen.orbit_camera(1, 8, W, H)
    o, ref = oracle_chain(sc, cam)
    pre = gs.preprocess(dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacities), dev(sc.sh),
                        gs_cam(cam))
    rad = host(pre["radii"])
    assert (rad[bad] == 0).all() and (o["radii"][bad] == 0).all()
    assert np.isfinite(host(pre["means2d"])).all() and np.isfinite(host(pre["conics"])).all()
    assert np.isfinite(host(pre["rgb"])).all()
    bs = gs.bin_sort(pre["means2d"], pre["radii"], pre["depths"], W, H)
    opac = pre["log_opacities"]
    for prec in ("fp32", "fp16_g2l_split", "bf16_g2l_split"):
        r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, pre["means2d"], pre["conics"], opac,
                             pre["rgb"], prec)
        q = chain_stats(host(r.rgb), ref["rgb"])
        say(f"  {prec}: PSNR {q['psnr']:.1f} dB, max|err| {q['max_abs']:.2e}, "
            f"within 2/255 {q['frac_2_255']:.6f}")
        check_chain(prec, q)
