"""Backward (gradients through the rasteriser) against the FP64 oracle's
analytic gradients, which are themselves pinned by finite differences."""
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
from gpu_helpers import dev, host  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def grad_check(name, got, ref, rel=1e-3, frac=0.995):
    """Per-element |got - ref| <= rel * (|ref| + scale), scale = RMS of ref;
    at least `frac` of the elements pass (the rest sit on pixels whose
    near-threshold decisions differ between FP32 and FP64) and the relative
    L2 error of the whole array is below 10 * rel."""
    got, ref = np.asarray(got, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    scale = np.sqrt(np.mean(ref ** 2)) + 1e-30
    ok = np.abs(got - ref) <= rel * (np.abs(ref) + scale)
    l2 = np.linalg.norm(got - ref) / (np.linalg.norm(ref) + 1e-30)
    say(f"  {name}: pass {ok.mean():.5f}, rel L2 {l2:.2e}")
    assert ok.mean() >= frac and l2 <= 10 * rel, (name, ok.mean(), l2)


@pytest.mark.parametrize("prec", ["fp32", "fp32_earlycull", "fp16_g2l_split", "bf16_g2l_split"])
@pytest.mark.parametrize("W,H,P,seed", [(64, 64, 200, 1014), (250, 190, 3000, 7)])
def test_backward_vs_oracle(prec, W, H, P, seed):
    say(f"backward {prec} {W}x{H} P={P}")
    sc = scenegen.scene_2d(P, W, H, seed, s_min=1.0 if P == 200 else 0.5, s_max=6.0 if P == 200 else 8.0)
    m2, cv, op, col = dev(sc.means2d), dev(sc.cov2d), dev(sc.opacities), dev(sc.rgb)
    pre = gs.preprocess_2d(m2, cv, op, W, H)
    lno = pre["log_opacities"]
    ranges, ids = oracle.bin_splats(sc.means2d, host(pre["radii"]), sc.depths, W, H)
    rg = dev(ranges.astype(np.int32))
    idg = dev(ids.astype(np.int32))
    bg = (0.2, 0.1, 0.3)
    r = gs.rasterize_fwd(W, H, rg, idg, m2, pre["conics"], lno, col, prec, background=bg)
    w = np.random.default_rng(seed).normal(0, 1, (3, H, W)).astype(np.float32)
    g = gs.rasterize_bwd(W, H, rg, idg, m2, pre["conics"], lno, col, r.T, r.n_contrib, dev(w), prec,
                         background=bg)
    conics = host(pre["conics"]).astype(np.float64)
    ref = oracle.render_backward(W, H, ranges, ids, sc.means2d, conics, sc.opacities, sc.rgb, w, bg=bg)
    rel = 1e-3 if prec.startswith("fp32") else 3e-3
    for k in ("means2d", "conics", "opacities", "rgb"):
        grad_check(k, host(g[k]), ref[k], rel=rel)


def test_autograd_function_and_l1_loss():
    """RasterizeFn gives the same gradients as the explicit call, through an
    L1 loss against a target image (the training-step loss)."""
    W, H = 128, 96
    sc = scenegen.scene_2d(800, W, H, 21)
    m2, cv = dev(sc.means2d), dev(sc.cov2d)
    pre = gs.preprocess_2d(m2, cv, dev(sc.opacities), W, H)
    lno = pre["log_opacities"]
    bs = gs.bin_sort(m2, pre["radii"], dev(sc.depths), W, H)
    target = torch.rand(3, H, W, device="cuda")
    params = [m2.clone().requires_grad_(), pre["conics"].clone().requires_grad_(),
              dev(sc.opacities).requires_grad_(), dev(sc.rgb).requires_grad_()]
    img = gs.RasterizeFn.apply(*params, lno, bs.ranges, bs.sorted_ids, W, H, "fp16_g2l_split")
    loss = (img - target).abs().mean()
    loss.backward()
    dimg = (torch.sign(img.detach() - target) / img.numel()).contiguous()
    m, c, _, k = [p.detach() for p in params]
    r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, m, c, lno, k, "fp16_g2l_split")
    g = gs.rasterize_bwd(W, H, bs.ranges, bs.sorted_ids, m, c, lno, k, r.T, r.n_contrib, dimg,
                         "fp16_g2l_split")
    for p, k in zip(params, ("means2d", "conics", "opacities", "rgb")):
        a, b = host(p.grad), host(g[k])
        assert np.allclose(a, b, rtol=1e-4, atol=1e-7 * np.abs(b).max()), k


def test_backward_fullsize_sampled_tiles():
    """1600x1064, 1M Gaussians (the training-step configuration), forward in
    FP16 split: dL/dC is non-zero only on sampled tiles, so every Gaussian's
    gradient comes from those tiles and the FP64 oracle evaluates just them."""
    cfg = scenegen.CONFIGS["train_1600x1064_1M"]
    W, H = cfg["width"], cfg["height"]
    gx, gy = (W + 15) // 16, (H + 15) // 16
    sc = scenegen.make_scene(cfg)
    cam_np = scenegen.make_camera(cfg)
    cam = gs.make_camera(cam_np.viewmat, cam_np.fx, cam_np.fy, cam_np.cx, cam_np.cy, W, H,
                         campos=cam_np.campos)
    pre = gs.preprocess(dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacities), dev(sc.sh), cam)
    bs = gs.bin_sort(pre["means2d"], pre["radii"], pre["depths"], W, H)
    op = pre["log_opacities"]
    prec = "fp16_g2l_split"
    r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, pre["means2d"], pre["conics"], op, pre["rgb"], prec)
    ranges_g = host(bs.ranges).astype(np.int64)
    counts = ranges_g[:, 1] - ranges_g[:, 0]
    tiles = np.unique(np.concatenate([np.argsort(-counts)[:4],
                                      np.random.default_rng(0).choice(gx * gy, 12, replace=False),
                                      [gx * gy - 1]])).astype(np.int32)
    w = np.zeros((3, H, W), np.float32)
    rnd = np.random.default_rng(1).normal(0, 1, (3, H, W)).astype(np.float32)
    for t in tiles:
        ty, tx = divmod(int(t), gx)
        w[:, 16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = rnd[:, 16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16]
    g = gs.rasterize_bwd(W, H, bs.ranges, bs.sorted_ids, pre["means2d"], pre["conics"], op, pre["rgb"],
                         r.T, r.n_contrib, dev(w), prec)
    m2, conics, rgb = host(pre["means2d"]), host(pre["conics"]).astype(np.float64), host(pre["rgb"])
    r_o, i_o = oracle.bin_tiles(m2, host(pre["radii"]), host(pre["depths"]), W, H, tiles)
    full_r = np.zeros((gx * gy, 2), np.uint32)
    full_r[tiles] = r_o
    ref = oracle.render_backward(W, H, full_r, i_o, m2, conics, sc.opacities, rgb, w)
    for k in ("means2d", "conics", "opacities", "rgb"):
        grad_check(k, host(g[k]), ref[k], rel=3e-3)
