"""Host-side checks of the C ABI: the library builds, loads, exports every
symbol the header declares, and rejects invalid arguments before touching
the GPU (no compute call is made here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs.h")


@pytest.fixture(scope="module")
def gslib():
    import paper_2505_24796_amd as gs
    if not os.path.exists(gs.LIB_PATH):
        from paper_2505_24796_amd import build
        build.build()
    return gs.lib()


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("gs_preprocess", "gs_preprocess_2d", "gs_bin_sort", "gs_bin_sort_workspace_bytes",
              "gs_rasterize_fwd", "gs_rasterize_beta", "gs_status_string", "gs_version"):
        assert n in names


def test_library_exports_every_declared_symbol(gslib):
    import paper_2505_24796_amd as gs
    out = subprocess.run(["nm", "-D", "--defined-only", gs.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "gs.h"\nint main(void){gs_camera c; (void)c; return GS_OK;}\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-c", str(src), "-o", str(tmp_path / "t.o")], check=True)


def test_status_strings(gslib):
    assert gslib.gs_status_string(0) == b"GS_OK"
    assert gslib.gs_status_string(4) == b"GS_ERR_CAPACITY"
    assert gslib.gs_status_string(99) == b"GS_ERR_UNKNOWN"
    assert gslib.gs_version() == 202  # ln o across the boundary; out_ncontrib may be NULL; NOCULL ablation


def test_invalid_arguments_rejected_on_host(gslib):
    import paper_2505_24796_amd as gs
    v = ctypes.c_void_p
    cam = gs.make_camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1], 100, 100, 50, 50, 100, 100)
    # negative P
    assert gslib.gs_preprocess(-1, v(16), v(16), v(16), v(16), v(16), 3, ctypes.byref(cam), v(16),
                               v(16), v(16), v(16), v(16), v(16), v(16), v(0)) == 1
    # bad SH degree
    assert gslib.gs_preprocess(1, v(16), v(16), v(16), v(16), v(16), 4, ctypes.byref(cam), v(16),
                               v(16), v(16), v(16), v(16), v(16), v(16), v(0)) == 1
    # null output (means2d, then ln o)
    assert gslib.gs_preprocess(1, v(16), v(16), v(16), v(16), v(16), 3, ctypes.byref(cam), v(0),
                               v(16), v(16), v(16), v(16), v(16), v(16), v(0)) == 1
    assert gslib.gs_preprocess(1, v(16), v(16), v(16), v(16), v(16), 3, ctypes.byref(cam), v(16),
                               v(16), v(0), v(16), v(16), v(16), v(16), v(0)) == 1
    # null opacities
    assert gslib.gs_preprocess(1, v(16), v(16), v(16), v(0), v(16), 3, ctypes.byref(cam), v(16),
                               v(16), v(16), v(16), v(16), v(16), v(16), v(0)) == 1
    # misaligned quaternions (16 B required)
    assert gslib.gs_preprocess(1, v(16), v(16), v(20), v(16), v(16), 3, ctypes.byref(cam), v(16),
                               v(16), v(16), v(16), v(16), v(16), v(16), v(0)) == 1
    # oversized image; null opacities
    assert gslib.gs_preprocess_2d(1, v(16), v(16), v(16), 20000, 10, v(16), v(16), v(16), v(16),
                                  v(0)) == 1
    assert gslib.gs_preprocess_2d(1, v(16), v(16), v(0), 64, 64, v(16), v(16), v(16), v(16),
                                  v(0)) == 1
    assert gslib.gs_bin_sort_workspace_bytes(10, 100, 0, 10) == 0
    assert gslib.gs_bin_sort_workspace_bytes(10, 100, 64, 64) > 0
    # workspace too small -> capacity error
    assert gslib.gs_bin_sort(10, v(16), v(16), v(16), 64, 64, 100, v(256), 8, v(16), v(16), v(16),
                             v(0)) == 4
    # unknown precision
    bg = (ctypes.c_float * 3)(0, 0, 0)
    args = [64, 64, v(16), v(16), v(16), v(16), v(16), v(16), bg]
    assert gslib.gs_rasterize_fwd(*args, 9, v(16), v(16), v(16), v(0), v(0)) == 1
    assert gslib.gs_rasterize_fwd(*args, 7, v(16), v(16), v(16), v(0), v(0)) == 1
    # the EarlyCull-off ablation variant is forward-only
    assert gslib.gs_rasterize_bwd(*args, 6, *([v(16)] * 7), v(0)) == 1
    assert gslib.gs_rasterize_beta(64, 64, 0, v(16), v(16), v(16), v(16), v(16), 6, 32, v(16),
                                   v(0)) == 1
    # null output image
    assert gslib.gs_rasterize_fwd(*args, 0, v(0), v(16), v(16), v(0), v(0)) == 1
    # tuned launch: batch must be 64/128/256, chunk rows 1 or 2
    import paper_2505_24796_amd as gsm
    for bad in ((96, 2), (128, 3), (0, 1)):
        t = gsm.make_raster_tune(*bad)
        assert gslib.gs_rasterize_fwd_tuned(*args, 4, ctypes.byref(t), v(16), v(16), v(16), v(0),
                                            v(0)) == 1
    # beta dump: tile out of range, FP32 precision not allowed
    assert gslib.gs_rasterize_beta(64, 64, 16, v(16), v(16), v(16), v(16), v(16), 4, 32, v(16),
                                   v(0)) == 1
    assert gslib.gs_rasterize_beta(64, 64, 0, v(16), v(16), v(16), v(16), v(16), 0, 32, v(16),
                                   v(0)) == 1


def test_batched_and_precise_arguments_rejected_on_host(gslib):
    """The multi-view, batched and precise-binning entry points validate
    their arguments before any GPU call."""
    import paper_2505_24796_amd as gs
    v = ctypes.c_void_p
    cam = gs.make_camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1], 100, 100, 50, 50, 100, 100)
    cams = (gs.gs_camera * 2)(cam, cam)
    # multi-camera preprocess: no cameras, too many, a bad camera
    assert gslib.gs_preprocess_multiview(1, v(16), v(16), v(16), v(16), v(16), 3, 0, cams, v(16),
                                         v(16), v(16), v(16), v(16), v(16), v(16), v(0)) == 1
    assert gslib.gs_preprocess_multiview(1, v(16), v(16), v(16), v(16), v(16), 3, 65, cams, v(16),
                                         v(16), v(16), v(16), v(16), v(16), v(16), v(0)) == 1
    bad = (gs.gs_camera * 2)(cam, gs.make_camera([1] * 16, 100, 100, 50, 50, 0, 100))
    assert gslib.gs_preprocess_multiview(1, v(16), v(16), v(16), v(16), v(16), 3, 2, bad, v(16),
                                         v(16), v(16), v(16), v(16), v(16), v(16), v(0)) == 1
    # batched raster: plan and workspace sizes, view count, alignment, precision, shape
    assert gslib.gs_batch_plan_bytes(0) == 0 and gslib.gs_batch_plan_bytes(65) == 0
    assert gslib.gs_batch_plan_bytes(16) > 0 and gslib.gs_batch_workspace_bytes(16) >= 4 * (16 + 16)
    views = (gs.gs_view * 1)()
    views[0].width, views[0].height = 64, 64  # null buffers
    assert gslib.gs_batch_plan_write(1, views, v(256), 1 << 20) == 1
    assert gslib.gs_batch_plan_write(1, views, v(260), 1 << 20) == 1  # misaligned plan
    t = gs.make_tune(256, 5, 1)
    assert gslib.gs_rasterize_fwd_batched(0, v(256), 4, t, v(256), 1024, v(0), v(0)) == 1
    assert gslib.gs_rasterize_fwd_batched(1, v(256), 4, t, v(256), 4, v(0), v(0)) == 4
    assert gslib.gs_rasterize_fwd_batched(1, v(256), 1, t, v(256), 1024, v(0), v(0)) == 2
    assert gslib.gs_rasterize_fwd_batched(1, v(256), 6, t, v(256), 1024, v(0), v(0)) == 1
    assert gslib.gs_rasterize_fwd_batched(1, v(256), 4, gs.make_tune(96, 5, 1), v(256), 1024,
                                          v(0), v(0)) == 1
    assert gslib.gs_rasterize_fwd_batched(1, v(256), 4, gs.make_tune(64, 0, 1), v(256), 1024,
                                          v(0), v(0)) == 1
    assert gslib.gs_clock_stamp(v(0), v(0)) == 1
    # precise binning: conics / opacities required, capacity check
    assert gslib.gs_bin_sort_precise_workspace_bytes(10, 100, 64, 64) > \
        gslib.gs_bin_sort_workspace_bytes(10, 100, 64, 64)
    assert gslib.gs_bin_sort_precise(10, v(16), v(16), v(16), v(0), v(16), 64, 64, 100, v(256),
                                     1 << 20, v(16), v(16), v(16), v(0)) == 1
    assert gslib.gs_bin_sort_precise(10, v(16), v(16), v(16), v(16), v(16), 64, 64, 100, v(256),
                                     8, v(16), v(16), v(16), v(0)) == 4


def test_multiview_bin_sort_arguments_rejected_on_host(gslib):
    """gs_bin_sort_multiview checks views, sizes, pointers and workspace
    before any GPU call."""
    v = ctypes.c_void_p
    i32 = ctypes.c_int32
    W = (i32 * 3)(64, 100, 32)
    H = (i32 * 3)(48, 60, 32)
    q = gslib.gs_bin_sort_multiview_workspace_bytes
    assert q(3, 10, 100, W, H, 0) > 0
    assert q(3, 10, 100, W, H, 1) > q(3, 10, 100, W, H, 0)   # ellipse records
    assert q(0, 10, 100, W, H, 0) == 0 and q(65, 10, 100, W, H, 0) == 0
    assert q(3, 10, 100, None, H, 0) == 0
    assert q(3, -1, 100, W, H, 0) == 0 and q(3, 10, 0x80000000, W, H, 0) == 0
    Wbad = (i32 * 3)(64, 0, 32)
    assert q(3, 10, 100, Wbad, H, 0) == 0
    f = gslib.gs_bin_sort_multiview
    ok = (v(16), v(16), v(16), v(16), v(16))  # means2d radii depths conics opacities
    assert f(0, 10, W, H, *ok, 0, 100, v(256), 1 << 20, v(16), v(16), v(16), v(16), v(0)) == 1
    assert f(65, 10, W, H, *ok, 0, 100, v(256), 1 << 20, v(16), v(16), v(16), v(16), v(0)) == 1
    assert f(3, 10, None, H, *ok, 0, 100, v(256), 1 << 20, v(16), v(16), v(16), v(16), v(0)) == 1
    assert f(3, 10, Wbad, H, *ok, 0, 100, v(256), 1 << 20, v(16), v(16), v(16), v(16), v(0)) == 1
    # null means, misaligned workspace, misaligned per-view counts
    assert f(3, 10, W, H, v(0), v(16), v(16), v(16), v(16), 0, 100, v(256), 1 << 20, v(16), v(16),
             v(16), v(16), v(0)) == 1
    assert f(3, 10, W, H, *ok, 0, 100, v(260), 1 << 20, v(16), v(16), v(16), v(16), v(0)) == 1
    assert f(3, 10, W, H, *ok, 0, 100, v(256), 1 << 20, v(16), v(16), v(16), v(18), v(0)) == 1
    # precise needs conics and ln o
    assert f(3, 10, W, H, v(16), v(16), v(16), v(0), v(16), 1, 100, v(256), 1 << 20, v(16), v(16),
             v(16), v(16), v(0)) == 1
    # workspace too small
    assert f(3, 10, W, H, *ok, 0, 100, v(256), 8, v(16), v(16), v(16), v(16), v(0)) == 4


def test_zero_gaussians_is_noop(gslib):
    v = ctypes.c_void_p
    assert gslib.gs_preprocess_2d(0, v(0), v(0), v(0), 64, 64, v(0), v(0), v(0), v(0), v(0)) == 0


def test_oracle_independent_of_product():
    """The oracle and the product library share no code: no include, import
    or symbol crosses between them."""
    orc = open(os.path.join(ROOT, "oracle", "gs_oracle.c")).read()
    assert "gs.h" not in orc and "csrc" not in orc
    orc_py = open(os.path.join(ROOT, "oracle", "__init__.py")).read()
    assert "paper_2505_24796_amd" not in orc_py
    for f in os.listdir(os.path.join(ROOT, "paper_2505_24796_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2505_24796_amd", "csrc", f)).read()
    pkg = open(os.path.join(ROOT, "paper_2505_24796_amd", "__init__.py")).read()
    assert "import oracle" not in pkg and "from oracle" not in pkg
