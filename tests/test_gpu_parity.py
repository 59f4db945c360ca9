"""GPU parity: every stage of the HIP path against the FP64 oracle on the
same seeded inputs (through the C ABI via the ctypes binding)."""
import math
import sys

import numpy as np
import pytest

import oracle
import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU machines too, but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_24796_amd as gs  # noqa: E402
from gpu_helpers import dev, fp32_check, host, psnr, quality  # noqa: E402

MFMA_PRECS = ["fp16_g2l", "fp16_g2l_split", "bf16_g2l_split", "fp16_g2l_split_nocull"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def scene2d_inputs(W, H, P, seed, **kw):
    sc = scenegen.scene_2d(P, W, H, seed, **kw)
    return sc, dict(means2d=dev(sc.means2d), cov2d=dev(sc.cov2d), opac=dev(sc.opacities),
                    rgb=dev(sc.rgb), depths=dev(sc.depths))


def oracle_lists(means2d, radii, depths, W, H):
    ranges, ids = oracle.bin_splats(means2d, radii, depths, W, H)
    return ranges, ids


def upload_lists(ranges, ids):
    return dev(ranges.astype(np.int32)), dev(ids.astype(np.int32) if ids.size else np.zeros(1, np.int32))


# ---------------------------------------------------------------- preprocess
@pytest.mark.parametrize("W,H", [(256, 256), (250, 190)])
def test_preprocess_2d_parity(W, H):
    say(f"preprocess_2d {W}x{H}")
    sc, d = scene2d_inputs(W, H, 2000, 1001)
    g = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    o = oracle.preprocess_2d(sc.means2d, sc.cov2d, W, H)
    r_g = host(g["radii"])
    same = r_g == o["radii"]
    # radii may differ only where 3 sqrt(lambda) sits on an integer (FP32 vs FP64)
    assert np.all(same | (o["rad_dist"] < 1e-4))
    assert np.all(host(g["tiles_touched"])[same] == o["tiles_touched"][same])
    vis = same & (o["radii"] > 0)
    np.testing.assert_allclose(host(g["conics"])[vis], o["conics"][vis], rtol=2e-5, atol=1e-7)
    # ln o for every Gaussian, to FP32 rounding (opacity crosses as ln o)
    np.testing.assert_allclose(host(g["log_opacities"]), np.log(sc.opacities.astype(np.float64)),
                               rtol=3e-7, atol=1e-7)


def test_preprocess_3d_parity():
    say("preprocess_3d 50k @ 640x360")
    sc = scenegen.scene_3d(50_000, 1234)
    cam = scenegen.orbit_camera(1, 7, 640, 360)
    c = gs.make_camera(cam.viewmat, cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height,
                       campos=cam.campos)
    g = gs.preprocess(dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacities), dev(sc.sh), c)
    o = oracle.preprocess_3d(sc, cam)
    r_g = host(g["radii"])
    same = r_g == o["radii"]
    assert np.mean(same) > 0.999
    assert np.all(same | (o["rad_dist"] < 1e-3) | (r_g == 0) | (o["radii"] == 0))
    vis = same & (o["radii"] > 0)
    assert vis.sum() > 1000
    np.testing.assert_allclose(host(g["means2d"])[vis], o["means2d"][vis], rtol=1e-5, atol=1e-3)
    np.testing.assert_allclose(host(g["depths"])[vis], o["depths"][vis], rtol=1e-5)
    cg, co = host(g["conics"])[vis], o["conics"][vis]
    scale = np.abs(co).max(axis=1, keepdims=True)
    assert np.max(np.abs(cg - co) / scale) < 2e-3
    np.testing.assert_allclose(host(g["rgb"])[vis], o["rgb"][vis], atol=2e-5)
    np.testing.assert_allclose(host(g["log_opacities"]), np.log(sc.opacities.astype(np.float64)),
                               rtol=3e-7, atol=1e-7)


# ---------------------------------------------------------------- bin / sort
@pytest.mark.parametrize("W,H,P,seed", [(256, 256, 2000, 1001), (250, 190, 3000, 7),
                                        (1000, 520, 20000, 8), (4100, 40, 5000, 9)])
def test_bin_sort_exact(W, H, P, seed):
    say(f"bin_sort {W}x{H} P={P}")
    sc, d = scene2d_inputs(W, H, P, seed)
    depths = sc.depths.copy()
    depths[::5] = 7.0          # ties are broken by id
    depths[1::97] = -0.0       # -0 equals +0
    depths[2::97] = 0.0
    depths[3::101] = np.nan    # skipped
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    radii = host(pre["radii"])
    bs = gs.bin_sort(d["means2d"], pre["radii"], dev(depths), W, H)
    ranges_o, ids_o = oracle.bin_splats(sc.means2d, radii, depths, W, H)
    N = bs.n_splats()
    assert N == len(ids_o)
    assert np.array_equal(host(bs.ranges).astype(np.uint32), ranges_o)
    assert np.array_equal(host(bs.sorted_ids)[:N].astype(np.uint32), ids_o)


def test_bin_sort_overflow_and_empty():
    say("bin_sort overflow / empty")
    W, H = 128, 96
    sc, d = scene2d_inputs(W, H, 500, 3)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    full = gs.bin_sort(d["means2d"], pre["radii"], d["depths"], W, H)
    N = full.n_splats()
    assert N > 10
    small = gs.BinSorter(500, N - 1, W, H)
    small(d["means2d"], pre["radii"], d["depths"])
    assert small.n_splats() == N                      # count still reported
    assert int(host(small.ranges).max()) == 0         # nothing built
    exact = gs.BinSorter(500, N, W, H)
    exact(d["means2d"], pre["radii"], d["depths"])
    assert np.array_equal(host(exact.ranges), host(full.ranges))
    # P = 0
    z = gs.BinSorter(0, 16, W, H)
    e = torch.empty(0, 2, device="cuda")
    z(e, torch.empty(0, dtype=torch.int32, device="cuda"), torch.empty(0, device="cuda"))
    assert z.n_splats() == 0 and int(host(z.ranges).max()) == 0
    # all radii zero
    zr = torch.zeros(500, dtype=torch.int32, device="cuda")
    b2 = gs.BinSorter(500, 16, W, H)
    b2(d["means2d"], zr, d["depths"])
    assert b2.n_splats() == 0 and int(host(b2.ranges).max()) == 0


def test_bin_sort_first_pass_histogram_both_ways():
    """A one-view call counts the first tile pass's digits during the
    expansion when 256 counts per 2048-slot window fit in its capacity, and
    runs a histogram kernel otherwise: both give the oracle's lists."""
    W, H = 96, 64
    sc, d = scene2d_inputs(W, H, 40, 12)  # ~190 splats
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    ranges_o, ids_o = oracle.bin_splats(sc.means2d, host(pre["radii"]), sc.depths, W, H)
    N = len(ids_o)
    say(f"bin_sort first-pass histogram, N={N}")
    assert 0 < N < 256, N  # capacity N: the histogram kernel
    for cap in (N, 256, 4096 + 7):
        bs = gs.BinSorter(40, cap, W, H)
        bs(d["means2d"], pre["radii"], d["depths"])
        assert bs.n_splats() == N
        assert np.array_equal(host(bs.ranges).astype(np.uint32), ranges_o), cap
        assert np.array_equal(host(bs.sorted_ids)[:N].astype(np.uint32), ids_o), cap


@pytest.mark.parametrize("W", [4096, 4160])
def test_bin_sort_tile_key_width(W):
    """A one-view call carries tile keys as 16-bit words up to 65536 tiles
    (4096 x 4096 is exactly 65536, the largest key 65535) and as 32-bit
    words beyond (4160 x 4160: 67600 tiles); both give the oracle's lists."""
    sc, d = scene2d_inputs(W, W, 20000, 41, s_min=0.5, s_max=6.0)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, W)
    radii = host(pre["radii"])
    ranges_o, ids_o = oracle.bin_splats(sc.means2d, radii, sc.depths, W, W)
    say(f"bin_sort {W}x{W}: {(W // 16) ** 2} tiles, N={len(ids_o)}")
    bs = gs.bin_sort(d["means2d"], pre["radii"], d["depths"], W, W)
    N = bs.n_splats()
    assert N == len(ids_o)
    assert np.array_equal(host(bs.ranges).astype(np.uint32), ranges_o)
    assert np.array_equal(host(bs.sorted_ids)[:N].astype(np.uint32), ids_o)


def test_bin_sort_expansion_staged_and_unstaged_windows():
    """The one-view expansion stages up to 1025 Gaussians of a 2048-slot
    window in LDS and reads the global arrays for windows with more (their
    Gaussians average under two splats).  Near tiny Gaussians (one or two
    tiles each) before far large ones in depth order give windows of both
    kinds; both must give the oracle's lists."""
    W, H = 512, 512
    tiny = scenegen.scene_2d(12000, W, H, 31, s_min=0.1, s_max=0.4)
    big = scenegen.scene_2d(1500, W, H, 32, s_min=4.0, s_max=30.0)
    m2 = np.concatenate([tiny.means2d, big.means2d])
    cov = np.concatenate([tiny.cov2d, big.cov2d])
    opac = np.concatenate([tiny.opacities, big.opacities])
    depths = np.concatenate([1.0 + 9.0 * (tiny.depths - 1.0) / 99.0,
                             50.0 + 50.0 * (big.depths - 1.0) / 99.0]).astype(np.float32)
    P = len(depths)
    pre = gs.preprocess_2d(dev(m2), dev(cov), dev(opac), W, H)
    radii = host(pre["radii"])
    ranges_o, ids_o = oracle.bin_splats(m2, radii, depths, W, H)
    # Gaussians per 2048-slot window in the emission (depth) order
    cnt = np.bincount(ids_o.astype(np.int64), minlength=P)
    order = [g for g in np.lexsort((np.arange(P), depths)) if cnt[g] > 0]
    ends = np.cumsum(cnt[order])
    starts = ends - cnt[order]
    nwin = (int(ends[-1]) + 2047) // 2048
    per_win = [int(np.sum((starts < 2048 * (w + 1)) & (ends > 2048 * w))) for w in range(nwin)]
    say(f"bin_sort staged/unstaged windows: N={len(ids_o)}, Gaussians per window "
        f"{min(per_win)}..{max(per_win)}")
    assert min(per_win) <= 1025 < max(per_win)
    bs = gs.bin_sort(dev(m2), pre["radii"], dev(depths), W, H)
    N = bs.n_splats()
    assert N == len(ids_o)
    assert np.array_equal(host(bs.ranges).astype(np.uint32), ranges_o)
    assert np.array_equal(host(bs.sorted_ids)[:N].astype(np.uint32), ids_o)


# ---------------------------------------------------------------- raster FP32
@pytest.mark.parametrize("prec", ["fp32", "fp32_earlycull"])
@pytest.mark.parametrize("W,H,P,seed", [(256, 256, 2000, 1001), (250, 190, 3000, 7)])
def test_raster_fp32_parity(prec, W, H, P, seed):
    say(f"raster {prec} {W}x{H}")
    sc, d = scene2d_inputs(W, H, P, seed)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    conics = host(pre["conics"]).astype(np.float64)
    ranges, ids = oracle_lists(sc.means2d, host(pre["radii"]), sc.depths, W, H)
    rg, idg = upload_lists(ranges, ids)
    bg = (0.1, 0.2, 0.3)
    r = gs.rasterize_fwd(W, H, rg, idg, d["means2d"], pre["conics"], pre["log_opacities"], d["rgb"], prec,
                         background=bg)
    st = fp32_check(W, H, ranges, ids, sc.means2d, conics, sc.opacities, sc.rgb, host(r.rgb),
                    host(r.T), bg=bg)
    say(f"  max|err| vs FP64 = {st['max_abs']:.2e}  ambiguous px {st['n_amb']}  flips {st['n_flip']}")
    ref = st["ref"]
    nc = host(r.n_contrib)
    amb = ref["n_amb"] > 0
    assert np.array_equal(nc[~amb], ref["n_contrib"][~amb])


def test_raster_counters_match_oracle():
    say("raster counters")
    W, H = 256, 256
    sc, d = scene2d_inputs(W, H, 2000, 1001)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    ranges, ids = oracle_lists(sc.means2d, host(pre["radii"]), sc.depths, W, H)
    rg, idg = upload_lists(ranges, ids)
    ref = oracle.render(W, H, ranges, ids, sc.means2d, host(pre["conics"]), sc.opacities, sc.rgb)
    want = np.array([ref["f_blend"].sum(), ref["f_cull"].sum(), ref["term"].sum()])
    for prec in ["fp32", "fp32_earlycull"] + MFMA_PRECS:
        r = gs.rasterize_fwd(W, H, rg, idg, d["means2d"], pre["conics"], pre["log_opacities"], d["rgb"], prec,
                             count=True)
        got = host(r.counters)
        say(f"  {prec}: blend {got[0]} cull {got[1]} term {got[2]} (oracle {want.tolist()})")
        assert got[3] == got[:3].sum()
        rel = np.abs(got[:3] - want) / np.maximum(want, 1)
        assert np.all(rel < (1e-4 if prec.startswith("fp32") else 2e-3)), (prec, got, want)


# ---------------------------------------------------------------- raster MFMA
@pytest.mark.parametrize("prec", MFMA_PRECS)
@pytest.mark.parametrize("W,H,P,seed", [(256, 256, 2000, 1001), (250, 190, 3000, 7)])
def test_raster_mfma_quality(prec, W, H, P, seed):
    say(f"raster {prec} {W}x{H}")
    sc, d = scene2d_inputs(W, H, P, seed)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    ranges, ids = oracle_lists(sc.means2d, host(pre["radii"]), sc.depths, W, H)
    rg, idg = upload_lists(ranges, ids)
    r = gs.rasterize_fwd(W, H, rg, idg, d["means2d"], pre["conics"], pre["log_opacities"], d["rgb"], prec)
    ref = oracle.render(W, H, ranges, ids, sc.means2d, host(pre["conics"]), sc.opacities, sc.rgb)
    q = quality(host(r.rgb), ref["rgb"])
    say(f"  PSNR {q['psnr']:.1f} dB  max {q['max_abs']:.2e}  within 2/255 {q['frac_2_255']:.5f}")
    check_mfma_quality(prec, q, host(r.rgb), W, H, ranges, ids, sc.means2d, host(pre["conics"]),
                       sc.opacities, sc.rgb)


def check_mfma_quality(prec, q, img, W, H, ranges, ids, means2d, conics, opac, rgb):
    """Split variants meet the full bar against the FP64 definition (>= 50 dB
    and >= 99.9% of pixels within 2/255).  The paper's own K = 8 FP16 layout
    meets the PSNR bar only; its per-pixel agreement is checked against the
    oracle's emulation of that layout's rounding instead."""
    assert q["psnr"] >= 50.0
    if prec == "fp16_g2l":
        emu = oracle.render(W, H, ranges, ids, means2d, conics, opac, rgb, mode=oracle.MODE_F16_G2L)
        qe = quality(img, emu["rgb"])
        say(f"  vs emulated K8 rounding: PSNR {qe['psnr']:.1f} dB within 2/255 {qe['frac_2_255']:.5f}")
        assert qe["psnr"] >= 60.0 and qe["frac_2_255"] >= 0.999
    else:
        assert q["frac_2_255"] >= 0.999


def test_raster_without_earlycull_equals_counting_launch():
    """The EarlyCull-off ablation variant stages and visits every listed
    splat, as the FP16 split's counting launch does to count fragments, so
    the two composite exactly the same fragments: colour, transmittance and
    n_contrib bit for bit, at every launch shape."""
    W, H = 250, 190
    sc, d = scene2d_inputs(W, H, 3000, 7)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    bs = gs.bin_sort(d["means2d"], pre["radii"], d["depths"], W, H)
    ref = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"],
                           pre["log_opacities"], d["rgb"], "fp16_g2l_split", count=True)
    want = (host(ref.rgb), host(ref.T), host(ref.n_contrib))
    for tune in (None, gs.make_raster_tune(64, 1), gs.make_raster_tune(256, 2)):
        rz = gs.Rasterizer(W, H)
        rz(bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"], pre["log_opacities"], d["rgb"],
           "fp16_g2l_split_nocull", tune=tune)
        got = (host(rz.rgb), host(rz.T), host(rz.n_contrib))
        for k in range(3):
            assert np.array_equal(got[k], want[k]), (tune, k)
    say("fp16_g2l_split_nocull equals the counting launch")


def test_raster_fp16_global_is_negative_control():
    """Without G2L the FP16 quadratic pixel terms destroy the image (the
    paper's FP16-without-local-coordinates ablation)."""
    W, H = 256, 256
    sc, d = scene2d_inputs(W, H, 2000, 1001)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    ranges, ids = oracle_lists(sc.means2d, host(pre["radii"]), sc.depths, W, H)
    rg, idg = upload_lists(ranges, ids)
    r = gs.rasterize_fwd(W, H, rg, idg, d["means2d"], pre["conics"], pre["log_opacities"], d["rgb"], "fp16_global")
    ref = oracle.render(W, H, ranges, ids, sc.means2d, host(pre["conics"]), sc.opacities, sc.rgb)
    p = psnr(host(r.rgb), ref["rgb"])
    say(f"fp16_global PSNR {p:.1f} dB")
    assert p < 35.0


UNIT = {oracle.MODE_F16_G2L: 2.0 ** -11, oracle.MODE_F16_SPLIT: 2.0 ** -22,
        oracle.MODE_BF16_SPLIT: 2.0 ** -24, oracle.MODE_F16_GLOBAL: 2.0 ** -11}


@pytest.mark.parametrize("prec,mode", [("fp16_g2l", oracle.MODE_F16_G2L),
                                       ("fp16_g2l_split", oracle.MODE_F16_SPLIT),
                                       ("bf16_g2l_split", oracle.MODE_BF16_SPLIT),
                                       ("fp16_global", oracle.MODE_F16_GLOBAL)])
def test_beta_matches_emulation(prec, mode):
    """The exponent matrix B from the matrix cores (a) lies within the
    rounding-error bound of the exact exponent (Appendix A, refined for exact
    local u and RNE) for the local variants, and (b) equals the oracle's
    emulation of the same rounding to FP32-accumulation accuracy, except
    where FP32 rounding of a coefficient moved it across an FP16/BF16
    rounding boundary (rare)."""
    say(f"beta dump {prec}")
    W, H = 256, 256
    sc, d = scene2d_inputs(W, H, 2000, 1001)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    ranges, ids = oracle_lists(sc.means2d, host(pre["radii"]), sc.depths, W, H)
    rg, idg = upload_lists(ranges, ids)
    conics = host(pre["conics"]).astype(np.float64)
    gx = 16
    checked = close = 0
    L2E = 1.0 / math.log(2.0)
    for tile in (0, 17, 120, 255):
        s, e = ranges[tile]
        cnt = int(min(e - s, 64))
        if cnt == 0:
            continue
        B = host(gs.rasterize_beta(W, H, tile, rg, idg, d["means2d"], pre["conics"], pre["log_opacities"],
                                   prec, cnt))
        tx, ty = tile % gx, tile // gx
        tc = np.array([16 * tx + 7.5, 16 * ty + 7.5])
        org = np.zeros(2) if mode == oracle.MODE_F16_GLOBAL else tc
        for j in range(cnt):
            gid = ids[s + j]
            mu = sc.means2d[gid].astype(np.float64)
            S = conics[gid]
            o = float(sc.opacities[gid])
            dx, dy = mu - org
            v = np.array([math.log(o) - 0.5 * (S[0] * dx * dx + 2 * S[1] * dx * dy + S[2] * dy * dy),
                          S[0] * dx + S[1] * dy, S[1] * dx + S[2] * dy, -0.5 * S[0], -S[1],
                          -0.5 * S[2]]) * L2E
            for pix in range(0, 256, 5):
                p = np.array([16 * tx + pix % 16, 16 * ty + pix // 16], float)
                px, py = p - org
                u = np.array([1, px, py, px * px, px * py, py * py])
                suv = float(np.abs(u * v).sum())
                got = float(B[j, pix])
                emu = oracle.beta_emulated(mode, mu, S, o, p, tc)
                acc = 40 * 2.0 ** -24 * suv + 2.0 ** -24 * 8
                if mode != oracle.MODE_F16_GLOBAL:
                    d_ = mu - p
                    exact = (math.log(o) - 0.5 * (S[0] * d_[0] ** 2 + 2 * S[1] * d_[0] * d_[1] +
                                                  S[2] * d_[1] ** 2)) * L2E
                    bound = UNIT[mode] * suv * (3 if mode == oracle.MODE_F16_G2L else 1) + acc + \
                        2.0 ** -25 * 2 * float(np.abs(u).sum())
                    assert abs(got - exact) <= bound, (prec, tile, j, pix, got, exact, bound)
                    checked += 1
                    close += abs(got - emu) <= acc
                elif np.isfinite(emu) and np.isfinite(got):
                    checked += 1
                    close += abs(got - emu) <= acc + 1e-3 * abs(emu)
    say(f"  checked {checked}, matching emulation {close}")
    assert checked > 500
    assert close >= 0.99 * checked


def test_translation_invariance_g2l():
    """G2L: shifting every centre by whole tiles shifts the image bit-exactly
    (centres on a 2^-8 grid so the shift is exact in FP32)."""
    W, H = 256, 256
    P = 600
    g = np.random.default_rng(77)
    mu = np.round(g.uniform(48, 112, (P, 2)) * 256) / 256
    sc = scenegen.scene_2d(P, W, H, 5, s_max=4.0)
    shift = np.array([64.0, 48.0])
    outs = {}
    for prec in ("fp16_g2l", "fp16_g2l_split", "bf16_g2l_split", "fp16_global"):
        imgs = []
        for off in (np.zeros(2), shift):
            m = (mu + off).astype(np.float32)
            pre = gs.preprocess_2d(dev(m), dev(sc.cov2d), dev(sc.opacities), W, H)
            ranges, ids = oracle_lists(m, host(pre["radii"]), sc.depths, W, H)
            rg, idg = upload_lists(ranges, ids)
            r = gs.rasterize_fwd(W, H, rg, idg, dev(m), pre["conics"], pre["log_opacities"], dev(sc.rgb), prec)
            imgs.append(host(r.rgb).copy())
        a = imgs[0][:, 0:160, 0:176]
        b = imgs[1][:, 48:208, 64:240]
        outs[prec] = np.array_equal(a, b)
    say(f"translation exact: {outs}")
    assert outs["fp16_g2l"] and outs["fp16_g2l_split"] and outs["bf16_g2l_split"]
    assert not outs["fp16_global"]


def test_determinism_and_empty_tiles():
    W, H = 250, 190
    sc, d = scene2d_inputs(W, H, 300, 12, s_max=3.0)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    bs = gs.bin_sort(d["means2d"], pre["radii"], d["depths"], W, H)
    ranges = host(bs.ranges)
    assert (ranges[:, 1] == ranges[:, 0]).any()  # some tiles are empty
    for prec in ["fp32", "fp32_earlycull"] + MFMA_PRECS:
        imgs = []
        for _ in range(3):
            r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"],
                                 pre["log_opacities"], d["rgb"], prec, background=(0.5, 0.25, 1.0))
            imgs.append((host(r.rgb).copy(), host(r.T).copy(), host(r.n_contrib).copy()))
        for k in range(3):
            assert np.array_equal(imgs[0][k], imgs[1][k]) and np.array_equal(imgs[0][k], imgs[2][k])
        empty = np.nonzero(ranges[:, 1] == ranges[:, 0])[0][0]
        ty, tx = divmod(int(empty), (W + 15) // 16)
        blk = imgs[0][0][:, 16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16]
        assert np.all(blk[0] == 0.5) and np.all(blk[1] == 0.25) and np.all(blk[2] == 1.0)


def test_end_to_end_3d_small():
    """Projection -> bin/sort -> raster on a 3D scene, every stage checked."""
    say("end-to-end 3D 100k @ 480x270")
    W, H = 480, 270
    sc = scenegen.scene_3d(100_000, 4321)
    cam = scenegen.orbit_camera(0, 1, W, H)
    c = gs.make_camera(cam.viewmat, cam.fx, cam.fy, cam.cx, cam.cy, W, H, campos=cam.campos)
    pre = gs.preprocess(dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacities), dev(sc.sh), c)
    m2, rad, dep = host(pre["means2d"]), host(pre["radii"]), host(pre["depths"])
    bs = gs.bin_sort(pre["means2d"], pre["radii"], pre["depths"], W, H)
    ranges, ids = oracle.bin_splats(m2, rad, dep, W, H)
    N = bs.n_splats()
    assert N == len(ids) and np.array_equal(host(bs.sorted_ids)[:N].astype(np.uint32), ids)
    assert np.array_equal(host(bs.ranges).astype(np.uint32), ranges)
    opac = pre["log_opacities"]
    conics = host(pre["conics"]).astype(np.float64)
    rgb = host(pre["rgb"])
    r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, pre["means2d"], pre["conics"], opac,
                         pre["rgb"], "fp32")
    st = fp32_check(W, H, ranges, ids, m2, conics, sc.opacities, rgb, host(r.rgb), host(r.T))
    say(f"  fp32 max|err| {st['max_abs']:.2e}")
    ref = st["ref"]
    for prec in MFMA_PRECS:
        r = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, pre["means2d"], pre["conics"], opac,
                             pre["rgb"], prec)
        q = quality(host(r.rgb), ref["rgb"])
        say(f"  {prec}: PSNR {q['psnr']:.1f} dB within 2/255 {q['frac_2_255']:.5f}")
        check_mfma_quality(prec, q, host(r.rgb), W, H, ranges, ids, m2, conics, sc.opacities, rgb)


def test_tuned_launch_shapes_bit_identical():
    """Every one-view launch shape (splats per round 64/128/256, one- or
    two-row XCD chunks) renders bit-identical outputs, for the FP32 and the
    matrix-core kernels; the autotuner checks the same and installs the
    fastest."""
    from paper_2505_24796_amd import autotune
    W, H = 250, 190
    sc, d = scene2d_inputs(W, H, 3000, 7)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    bs = gs.bin_sort(d["means2d"], pre["radii"], d["depths"], W, H)
    for prec in ("fp32", "fp16_g2l_split", "bf16_g2l_split"):
        base = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"],
                                pre["log_opacities"], d["rgb"], prec)
        ref = (host(base.rgb), host(base.T), host(base.n_contrib))
        rz = gs.Rasterizer(W, H)
        res = autotune.tune_raster(rz, bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"],
                                   pre["log_opacities"], d["rgb"], prec, reps=2, warmup=1)
        say(f"tuned {prec}: {res['best']}")
        rz(bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"], pre["log_opacities"], d["rgb"], prec)
        got = (host(rz.rgb), host(rz.T), host(rz.n_contrib))
        assert all(np.array_equal(a, b) for a, b in zip(ref, got)), prec
    # timed in a frame's state: the bin/sort re-run ahead of every timed call
    # (same inputs, so the same lists) leaves the result unchanged
    calls = []

    def before():
        calls.append(1)
        bs(d["means2d"], pre["radii"], d["depths"])

    rz = gs.Rasterizer(W, H)
    res = autotune.tune_raster(rz, bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"],
                               pre["log_opacities"], d["rgb"], "fp16_g2l_split", reps=2, warmup=1,
                               before=before)
    assert len(calls) == len(res["table"]) * 3  # warm-up and timed calls of every shape
    rz(bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"], pre["log_opacities"], d["rgb"],
       "fp16_g2l_split")
    base = gs.rasterize_fwd(W, H, bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"],
                            pre["log_opacities"], d["rgb"], "fp16_g2l_split")
    assert np.array_equal(host(rz.rgb), host(base.rgb)) and np.array_equal(host(rz.T), host(base.T))


def test_forward_without_ncontrib_bit_identical():
    """gs_rasterize_fwd with out_ncontrib NULL runs kernel instances that do
    not track the last composited splat: colour and transmittance are bit
    for bit those of the full call, for every precision and launch shape,
    and the n_contrib buffer is left alone."""
    W, H = 250, 190
    sc, d = scene2d_inputs(W, H, 3000, 7)
    pre = gs.preprocess_2d(d["means2d"], d["cov2d"], d["opac"], W, H)
    bs = gs.bin_sort(d["means2d"], pre["radii"], d["depths"], W, H)
    for prec in gs.PRECISIONS:
        for tune in (None, gs.make_raster_tune(64, 1), gs.make_raster_tune(256, 2)):
            rz = gs.Rasterizer(W, H)
            rz(bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"], pre["log_opacities"], d["rgb"],
               prec, tune=tune)
            ref = (host(rz.rgb), host(rz.T))
            rz.n_contrib.fill_(-7)
            rz.rgb.fill_(float("nan"))
            rz.T.fill_(float("nan"))
            rz(bs.ranges, bs.sorted_ids, d["means2d"], pre["conics"], pre["log_opacities"], d["rgb"],
               prec, tune=tune, ncontrib=False)
            assert np.array_equal(host(rz.rgb), ref[0]), (prec, tune)
            assert np.array_equal(host(rz.T), ref[1]), (prec, tune)
            assert int(host(rz.n_contrib).max()) == -7 and int(host(rz.n_contrib).min()) == -7
        say(f"forward without n_contrib: {prec} bit-identical")
