"""gs_bin_sort_noalloc (the bin/sort entry point that allocates nothing and
works in the library's static per-device scratch array) against gs_bin_sort
with a caller-allocated workspace: identical lists, ranges and splat counts,
bit for bit, on two calls in a row (the second smaller, so stale contents of
the shared array from the first call must not leak into it), plus the
host-side rejection of sizes beyond the array."""
import sys

import numpy as np
import pytest

import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2505_24796_amd as gs  # noqa: E402


def _lists(sc, W, H, pre, capacity):
    ref = gs.BinSorter(sc.P, capacity, W, H)
    ref(pre["means2d"], pre["radii"], pre["depths"])
    gx, gy = gs.grid(W, H)
    ids = torch.full((capacity,), -7, dtype=torch.int32, device="cuda")
    ranges = torch.full((gx * gy, 2), -7, dtype=torch.int32, device="cuda")
    num = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    gs.bin_sort_noalloc(pre["means2d"], pre["radii"], pre["depths"], W, H, ids, ranges, num)
    torch.cuda.synchronize()
    return ref, ids, ranges, num


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_workspace_call(order):
    cases = [(150_000, 640, 480, 4321), (20_000, 200, 150, 77)]
    for P, W, H, seed in cases:
        print(f"noalloc bin/sort: P={P} {W}x{H} seed {seed}", flush=True)
        sc = scenegen.scene_3d(P, seed)
        cam = scenegen.orbit_camera(1, 8, W, H)
        gcam = gs.make_camera(cam.viewmat, cam.fx, cam.fy, cam.cx, cam.cy, W, H, campos=cam.campos)
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        pre = gs.preprocess(d(sc.means), d(sc.scales), d(sc.quats), d(sc.opacities), d(sc.sh), gcam)
        probe = gs.BinSorter(P, 0, W, H)
        probe(pre["means2d"], pre["radii"], pre["depths"])
        N = probe.n_splats()
        capacity = N + 1000
        need = gs.lib().gs_bin_sort_workspace_bytes(P, capacity, W, H)
        assert 0 < need <= gs.NOALLOC_SCRATCH_BYTES, need
        ref, ids, ranges, num = _lists(sc, W, H, pre, capacity)
        assert int(num.item()) == ref.n_splats() == N
        assert torch.equal(ids[:N], ref.sorted_ids[:N])
        assert torch.equal(ranges, ref.ranges)
        print(f"  N = {N}: lists and ranges identical", flush=True)
    # overflow behaves as gs_bin_sort's: every range empty, N still reported
    ref, ids, ranges, num = _lists(sc, W, H, pre, max(N // 2, 1))
    assert int(num.item()) == N and torch.equal(ranges, ref.ranges)
    assert int(ranges[:, 1].sub(ranges[:, 0]).abs().max().item()) == 0


def test_noalloc_rejects_sizes_beyond_scratch():
    P, W, H = 4_000_000, 1920, 1080
    cap = 1 << 28
    assert gs.lib().gs_bin_sort_workspace_bytes(P, cap, W, H) > gs.NOALLOC_SCRATCH_BYTES
    gx, gy = gs.grid(W, H)
    m2 = torch.zeros(P, 2, device="cuda")
    rad = torch.zeros(P, dtype=torch.int32, device="cuda")
    dep = torch.zeros(P, device="cuda")
    ranges = torch.zeros(gx * gy, 2, dtype=torch.int32, device="cuda")
    num = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = gs.lib().gs_bin_sort_noalloc(P, gs._ptr(m2), gs._ptr(rad), gs._ptr(dep), W, H, cap,
                                      gs._ptr(ranges), gs._ptr(ranges), gs._ptr(num), gs._stream())
    assert st == 4  # GS_ERR_CAPACITY, nothing enqueued
    print("oversize request rejected with GS_ERR_CAPACITY", flush=True)
    sys.stdout.flush()
