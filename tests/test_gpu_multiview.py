"""Multi-view serving path: one multi-view preprocess, per-view bin/sort and
ONE persistent batched rasteriser launch, captured in a hipGraph.

* every view of the batched launch is bit-identical to the one-view kernel
  (same per-tile arithmetic), for every launch shape the autotuner tries;
* every view matches the FP64 oracle (exact lists, FP16/BF16 quality bar);
* graph replays reproduce the eager frame exactly;
* at the full multi-view size (2M Gaussians, 16 cameras of four resolutions)
  on sampled tiles per view."""
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
from paper_2505_24796_amd import autotune  # noqa: E402
from gpu_helpers import dev, host, quality  # noqa: E402

SMALL_RES = ((160, 120), (250, 190), (96, 80), (320, 176), (64, 48), (200, 200))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gs_cam(c):
    return gs.make_camera(c.viewmat, c.fx, c.fy, c.cx, c.cy, c.width, c.height, campos=c.campos)


def scene_tensors(sc):
    return dict(means3d=dev(sc.means), scales=dev(sc.scales), quats=dev(sc.quats), sh=dev(sc.sh),
                opacities=dev(sc.opacities))


def small_case(n_views=6, P=30000, seed=1015):
    sc = scenegen.scene_3d(P, seed)
    cams = [scenegen.orbit_camera(k, n_views, *SMALL_RES[k % len(SMALL_RES)])
            for k in range(n_views)]
    return sc, cams


def snapshot(mv):
    return [(host(r.rgb).copy(), host(r.T).copy(), host(r.n_contrib).copy()) for r in mv.images]


def assert_same(a, b, what):
    for v, (x, y) in enumerate(zip(a, b)):
        for k, (p, q) in enumerate(zip(x, y)):
            assert np.array_equal(p, q), f"{what}: view {v} output {k} differs"


@pytest.mark.parametrize("precise", [False, True])
def test_bin_sort_multiview_matches_per_view_and_oracle(precise):
    """One gs_bin_sort_multiview call builds, view after view, exactly the
    lists gs_bin_sort(_precise) builds for each view alone (ids, ranges,
    counts); the 3-sigma lists of two views equal the oracle's binning."""
    say(f"multi-view bin/sort, precise={precise}")
    sc, cams = small_case()
    gcams = [gs_cam(c) for c in cams]
    pre = gs.preprocess_multiview(dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacities),
                                  dev(sc.sh), gcams)
    opac = pre["log_opacities"]
    V, P = len(cams), sc.P
    kw = lambda v: dict(conics=pre["conics"][v], log_opacities=opac, precise=True) if precise else {}
    per = [gs.bin_sort(pre["means2d"][v], pre["radii"][v], pre["depths"][v], c.width, c.height,
                       **kw(v)) for v, c in enumerate(cams)]
    ns = [b.n_splats() for b in per]
    mb = gs.MultiViewBinSorter(P, sum(ns) + 100, [(c.width, c.height) for c in cams],
                               precise=precise)
    mb(pre["means2d"], pre["radii"], pre["depths"], pre["conics"], opac)
    assert mb.n_splats() == sum(ns) and mb.view_counts() == ns
    ids = host(mb.sorted_ids)
    start = 0
    for v in range(V):
        r1 = host(per[v].ranges).astype(np.int64)
        r2 = host(mb.ranges(v)).astype(np.int64)
        full = r1[:, 1] > r1[:, 0]
        assert np.array_equal(r1[full], r2[full] - start), f"view {v}: ranges differ"
        assert np.all(r2[~full, 0] == r2[~full, 1]), f"view {v}: extra tiles"
        assert np.array_equal(host(per[v].sorted_ids)[:ns[v]], ids[start:start + ns[v]]), v
        start += ns[v]
    if not precise:
        for v in (0, V - 1):
            W, H = cams[v].width, cams[v].height
            r_o, i_o = oracle.bin_splats(host(pre["means2d"][v]), host(pre["radii"][v]),
                                         host(pre["depths"][v]), W, H)
            r2 = host(mb.ranges(v)).astype(np.int64)
            base = sum(ns[:v])
            full = r_o[:, 1] > r_o[:, 0]
            assert np.array_equal(r_o[full].astype(np.int64), r2[full] - base), v
            assert np.array_equal(i_o, ids[base:base + ns[v]].astype(np.uint32)), v
    # overflow: nothing is built, the counts are still reported
    small = gs.MultiViewBinSorter(P, sum(ns) - 1, [(c.width, c.height) for c in cams],
                                  precise=precise)
    small(pre["means2d"], pre["radii"], pre["depths"], pre["conics"], opac)
    assert small.n_splats() == sum(ns) and small.view_counts() == ns
    rg = host(small.all_ranges)
    assert np.all(rg[:, 0] == rg[:, 1])


def test_bin_sort_multiview_empty_and_tiny_views():
    """Views that keep nothing (a camera turned away from the scene), a
    one-tile view and the most views one call takes: every view's lists are
    still exactly its one-view lists."""
    import dataclasses
    sc = scenegen.scene_3d(20000, 1016)
    base = [scenegen.orbit_camera(k, 8, *SMALL_RES[k % len(SMALL_RES)]) for k in range(8)]
    away = dataclasses.replace(base[1], viewmat=(np.diag([-1.0, 1.0, -1.0, 1.0]) @ base[1].viewmat)
                               .astype(np.float32))
    tiny = scenegen.orbit_camera(3, 8, 16, 16)
    cams = [base[0], away, tiny, base[2], away, base[5]]
    cams = cams + [base[k % 8] if k % 5 else away for k in range(gs.GS_MAX_BIN_VIEWS - len(cams))]
    assert len(cams) == gs.GS_MAX_BIN_VIEWS
    gcams = [gs_cam(c) for c in cams]
    pre = gs.preprocess_multiview(dev(sc.means), dev(sc.scales), dev(sc.quats), dev(sc.opacities),
                                  dev(sc.sh), gcams)
    ns = []
    per = []
    for v, c in enumerate(cams):
        b = gs.bin_sort(pre["means2d"][v], pre["radii"][v], pre["depths"][v], c.width, c.height)
        per.append(b)
        ns.append(b.n_splats())
    assert ns[1] == 0 and ns[4] == 0 and ns[0] > 0
    mb = gs.MultiViewBinSorter(sc.P, sum(ns) + 1, [(c.width, c.height) for c in cams])
    mb(pre["means2d"], pre["radii"], pre["depths"])
    assert mb.view_counts() == ns
    ids = host(mb.sorted_ids)
    start = 0
    for v in range(len(cams)):
        r1 = host(per[v].ranges).astype(np.int64)
        r2 = host(mb.ranges(v)).astype(np.int64)
        full = r1[:, 1] > r1[:, 0]
        assert np.array_equal(r1[full], r2[full] - start), v
        assert np.all(r2[~full, 0] == r2[~full, 1]), v
        assert np.array_equal(host(per[v].sorted_ids)[:ns[v]], ids[start:start + ns[v]]), v
        start += ns[v]


def test_bin_sort_multiview_no_gaussians():
    sizes = [(64, 48), (100, 60)]
    mb = gs.MultiViewBinSorter(0, 16, sizes)
    z2 = torch.zeros(2, 0, 2, dtype=torch.float32, device="cuda")
    mb(z2, torch.zeros(2, 0, dtype=torch.int32, device="cuda"),
       torch.zeros(2, 0, dtype=torch.float32, device="cuda"))
    assert mb.n_splats() == 0 and mb.view_counts() == [0, 0]
    assert int(host(mb.all_ranges).max()) == 0


def test_joint_and_per_view_binning_render_the_same():
    sc, cams = small_case()
    t = scene_tensors(sc)
    a = gs.MultiViewRenderer(t, [gs_cam(c) for c in cams], joint_bin=True)
    b = gs.MultiViewRenderer(t, [gs_cam(c) for c in cams], joint_bin=False)
    c4 = gs.MultiViewRenderer(t, [gs_cam(c) for c in cams], joint_bin=True, bin_groups=4)
    a.frame()
    b.frame()
    c4.frame()
    torch.cuda.synchronize()
    assert a.n_splats() == b.n_splats() == c4.n_splats()
    assert_same(snapshot(a), snapshot(b), "joint vs per-view binning")
    assert_same(snapshot(c4), snapshot(b), "four joint groups vs per-view binning")
    g = c4.capture()
    g.replay()
    torch.cuda.synchronize()
    assert_same(snapshot(c4), snapshot(b), "graph of four joint groups")


def test_preprocess_multiview_matches_single_and_oracle():
    sc, cams = small_case(n_views=5, P=20000)
    t = scene_tensors(sc)
    say("preprocess_multiview: 5 views, P=20000")
    mv = gs.preprocess_multiview(t["means3d"], t["scales"], t["quats"], t["opacities"], t["sh"],
                                 [gs_cam(c) for c in cams])
    for v, c in enumerate(cams):
        one = gs.preprocess(t["means3d"], t["scales"], t["quats"], t["opacities"], t["sh"],
                            gs_cam(c))
        # the two kernels share the projection code and round identically
        for k in ("radii", "tiles_touched", "means2d", "conics", "depths", "rgb"):
            assert np.array_equal(host(mv[k][v]), host(one[k])), (v, k)
        assert np.array_equal(host(mv["log_opacities"]), host(one["log_opacities"]))
        o = oracle.preprocess_3d(sc, c)
        rad = host(mv["radii"][v])
        same = rad == o["radii"]
        assert np.mean(same) > 0.999
        vis = same & (o["radii"] > 0)
        np.testing.assert_allclose(host(mv["means2d"][v])[vis], o["means2d"][vis], rtol=1e-5,
                                   atol=2e-3)
        np.testing.assert_allclose(host(mv["rgb"][v])[vis], o["rgb"][vis], atol=3e-5)


def test_many_views():
    """40 small views: the multi-camera preprocess runs in chunks of 16
    cameras, the plan holds 40 views; everything bit-identical to one call /
    one launch per view."""
    res = ((64, 48), (96, 80), (48, 64), (130, 70), (16, 16))
    sc = scenegen.scene_3d(8000, 1018)
    cams = [scenegen.orbit_camera(k, 40, *res[k % len(res)]) for k in range(40)]
    t = scene_tensors(sc)
    mvp = gs.preprocess_multiview(t["means3d"], t["scales"], t["quats"], t["opacities"], t["sh"],
                                  [gs_cam(c) for c in cams])
    for v in (0, 15, 16, 17, 39):
        one = gs.preprocess(t["means3d"], t["scales"], t["quats"], t["opacities"], t["sh"],
                            gs_cam(cams[v]))
        for k in ("radii", "means2d", "conics", "rgb", "depths"):
            assert np.array_equal(host(mvp[k][v]), host(one[k])), (v, k)
    mv = gs.MultiViewRenderer(t, [gs_cam(c) for c in cams])
    for tune in (gs.make_tune(64, 2, 1), gs.make_tune(128, 1, 0)):
        mv.frame(tune)
        torch.cuda.synchronize()
        batched = snapshot(mv)
        mv.raster_per_view()
        assert_same(batched, snapshot(mv), f"40 views, shape {tune.as_tuple()}")
    assert all(x > 0 for x in mv.latencies_ms())


@pytest.mark.parametrize("prec,joint", [("fp16_g2l_split", False), ("bf16_g2l_split", False),
                                        ("fp16_g2l_split", True)])
def test_batched_small_vs_single_and_oracle(prec, joint):
    sc, cams = small_case()
    say(f"batched {prec}: {len(cams)} views, P={sc.P}, joint binning {joint}")
    mv = gs.MultiViewRenderer(scene_tensors(sc), [gs_cam(c) for c in cams], precision=prec,
                              joint_bin=joint, bin_groups=2 if joint else 1)
    mv.frame()
    assert not any(mv.overflowed())
    batched = snapshot(mv)
    lat = mv.latencies_ms()
    assert all(x > 0 for x in lat), lat
    mv.raster_per_view()
    assert_same(batched, snapshot(mv), "batched vs one-view launch")
    for v, c in enumerate(cams):
        W, H = c.width, c.height
        m2 = host(mv.pre["means2d"][v])
        rad, dep = host(mv.pre["radii"][v]), host(mv.pre["depths"][v])
        r_o, i_o = oracle.bin_splats(m2, rad, dep, W, H)
        rg, ids = mv.view_lists(v)
        n = len(ids)
        assert n == len(i_o) == mv.n_splats()[v]
        assert np.array_equal(rg, r_o.astype(np.int64))
        assert np.array_equal(ids.astype(np.uint32), i_o)
        ref = oracle.render(W, H, r_o, i_o, m2, host(mv.pre["conics"][v]).astype(np.float64),
                            sc.opacities, host(mv.pre["rgb"][v]))
        q = quality(batched[v][0], ref["rgb"])
        say(f"  view {v} {W}x{H}: N={n}, PSNR {q['psnr']:.1f} dB, within 2/255 {q['frac_2_255']:.5f}")
        assert q["psnr"] >= 50.0 and q["frac_2_255"] >= 0.999


def test_autotune_shapes_bit_identical():
    sc, cams = small_case(n_views=4)
    mv = gs.MultiViewRenderer(scene_tensors(sc), [gs_cam(c) for c in cams])
    say("autotune over every launch shape (outputs compared bit for bit)")
    res = autotune.tune_batched(mv, space={"blocks_per_cu": (1, 3, 5)}, reps=2, warmup=1)
    assert len(res["table"]) == 3 * 3 * 2
    assert mv.tune.as_tuple() == (res["best"]["batch"], res["best"]["blocks_per_cu"],
                                  res["best"]["xcd_queues"])


def test_graph_replay_matches_eager():
    sc, cams = small_case(n_views=4, P=20000, seed=1016)
    mv = gs.MultiViewRenderer(scene_tensors(sc), [gs_cam(c) for c in cams])
    mv.frame()
    torch.cuda.synchronize()
    eager = snapshot(mv)
    g = mv.capture()
    for rep in range(3):
        for r in mv.images:  # eager work between replays
            r.rgb.fill_(-1.0)
            r.T.fill_(-1.0)
            r.n_contrib.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"graph replay {rep}")
        assert_same(eager, snapshot(mv), f"replay {rep}")
        assert all(x > 0 for x in mv.latencies_ms())


def test_pipelined_frame_and_graph():
    """Two-stream pipelined frame (per-view raster overlapping the next
    views' bin/sort): same images as the one-launch frame, eagerly and in a
    replayed graph."""
    sc, cams = small_case(n_views=5, P=20000, seed=1017)
    mv = gs.MultiViewRenderer(scene_tensors(sc), [gs_cam(c) for c in cams])
    mv.frame()
    torch.cuda.synchronize()
    ref = snapshot(mv)
    for r in mv.images:
        r.rgb.fill_(-1.0)
    mv.frame_pipelined()
    torch.cuda.synchronize()
    assert_same(ref, snapshot(mv), "pipelined eager")
    lat = mv.latencies_ms()
    assert all(x > 0 for x in lat), lat
    g = mv.capture(pipelined=True)
    for rep in range(3):
        for r in mv.images:
            r.rgb.fill_(-1.0)
            r.T.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"pipelined graph replay {rep}: latencies {[round(x, 3) for x in mv.latencies_ms()]}")
        assert_same(ref, snapshot(mv), f"pipelined replay {rep}")


def test_batched_rejects_bad_args():
    L = gs.lib()
    t = gs.make_tune(96, 5, 1)  # batch must be 64, 128 or 256
    ws = torch.zeros(256, dtype=torch.uint8, device="cuda")
    plan = torch.zeros(L.gs_batch_plan_bytes(1), dtype=torch.uint8, device="cuda")
    st = L.gs_rasterize_fwd_batched(1, gs._ptr(plan), 4, t, gs._ptr(ws), ws.numel(), None, None)
    assert st == 1
    st = L.gs_rasterize_fwd_batched(1, gs._ptr(plan), 0, gs.make_tune(), gs._ptr(ws), ws.numel(),
                                    None, None)
    assert st == 2  # FP32 is not served batched
    assert L.gs_batch_plan_bytes(0) == 0 and L.gs_batch_plan_bytes(65) == 0


def sample_tiles(ranges, gx, gy, n_random, n_heavy, seed):
    counts = ranges[:, 1].astype(np.int64) - ranges[:, 0].astype(np.int64)
    heavy = np.argsort(-counts, kind="stable")[:n_heavy]
    rnd = np.random.default_rng(seed).choice(gx * gy, n_random, replace=False)
    corner = np.array([gx * gy - 1])
    return np.unique(np.concatenate([heavy, rnd, corner])).astype(np.int32)


def test_multiview_fullsize_sampled():
    cfg = scenegen.CONFIGS["multiview_2M_16"]
    say(f"multiview_2M_16: generating P={cfg['P']}")
    sc = scenegen.make_scene(cfg)
    cams = scenegen.multiview_cameras(cfg)
    mv = gs.MultiViewRenderer(scene_tensors(sc), [gs_cam(c) for c in cams])
    g = mv.capture()
    g.replay()
    torch.cuda.synchronize()
    assert not any(mv.overflowed())
    batched = snapshot(mv)
    say(f"  splats per view: {mv.n_splats()}")
    mv.raster_per_view()
    assert_same(batched, snapshot(mv), "batched vs one-view launch")
    sel = np.random.default_rng(5).choice(sc.P, 20000, replace=False)
    sub = scenegen.Scene3D(means=sc.means[sel], scales=sc.scales[sel], quats=sc.quats[sel],
                           opacities=sc.opacities[sel], sh=sc.sh[sel])
    for v, c in enumerate(cams):
        W, H = c.width, c.height
        gx, gy = (W + 15) // 16, (H + 15) // 16
        m2 = host(mv.pre["means2d"][v])
        rad, dep = host(mv.pre["radii"][v]), host(mv.pre["depths"][v])
        o = oracle.preprocess_3d(sub, c)
        same = rad[sel] == o["radii"]
        assert np.mean(same) > 0.999
        vis = same & (o["radii"] > 0)
        np.testing.assert_allclose(m2[sel][vis], o["means2d"][vis], rtol=1e-5, atol=2e-3)
        ranges_g, ids_g = mv.view_lists(v)
        tiles = sample_tiles(ranges_g, gx, gy, n_random=5, n_heavy=2, seed=v)
        r_o, i_o = oracle.bin_tiles(m2, rad, dep, W, H, tiles)
        for j, t in enumerate(tiles):
            a = ids_g[ranges_g[t, 0]:ranges_g[t, 1]].astype(np.uint32)
            assert np.array_equal(a, i_o[r_o[j, 0]:r_o[j, 1]]), (v, t)
        full_r = np.zeros((gx * gy, 2), np.uint32)
        full_r[tiles] = r_o
        ref = oracle.render(W, H, full_r, i_o, m2, host(mv.pre["conics"][v]).astype(np.float64),
                            sc.opacities, host(mv.pre["rgb"][v]), tiles=tiles)
        mask = ~np.isnan(ref["T"])
        q = quality(batched[v][0], ref["rgb"], mask)
        say(f"  view {v} {W}x{H}: {len(tiles)} tiles, PSNR {q['psnr']:.1f} dB, "
            f"within 2/255 {q['frac_2_255']:.5f}")
        assert q["psnr"] >= 50.0 and q["frac_2_255"] >= 0.999
