"""FP64 CPU oracle (test infrastructure only).

A thin ctypes wrapper around ``gs_oracle.c``.  Only the test suite, the
package smoke check and the benchmark's CPU-baseline leg may import this
module; the product library never does, and this module never imports the
product package.  See ``gs_oracle.c`` for what each function computes and
which passage of the TC-GS paper it follows.

Every function here is pinned in ``tests/test_oracle_pins.py`` by closed
forms, invariants, brute force or library routines written independently of
``gs_oracle.c``; none is left "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_int64, c_uint32, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# exponent modes (see gs_oracle.c)
MODE_DEF = 0
MODE_F16_GLOBAL = 1
MODE_F16_G2L = 2
MODE_F16_SPLIT = 3
MODE_BF16_SPLIT = 4

TILE = 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                        "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_round_format.restype = c_double
        L.orc_round_format.argtypes = [c_double, c_int, c_int, c_double]
        L.orc_beta_emulated.restype = c_double
        L.orc_beta_emulated.argtypes = [c_int, c_void_p, c_void_p, c_double, c_void_p, c_void_p]
        L.orc_bin.restype = c_int64
        L.orc_num_threads.restype = c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def grid(W: int, H: int):
    return (W + TILE - 1) // TILE, (H + TILE - 1) // TILE


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (for timing)."""
    lib().orc_set_num_threads(c_int(int(n)))


def round_format(x: float, p: int, emin: int, maxval: float) -> float:
    return float(lib().orc_round_format(float(x), int(p), int(emin), float(maxval)))


def round_fp16(x: float) -> float:
    return round_format(x, 11, -14, 65504.0)


def round_bf16(x: float) -> float:
    return round_format(x, 8, -126, 255.0 * 2.0 ** 120)


def sh_basis(dirs: np.ndarray, deg: int = 3) -> np.ndarray:
    """Real SH basis (Condon-Shortley phase) at each direction; (n, (deg+1)^2)."""
    dirs = _f64(np.atleast_2d(dirs))
    out = np.zeros((dirs.shape[0], (deg + 1) ** 2), np.float64)
    row = np.zeros((deg + 1) ** 2, np.float64)
    for i in range(dirs.shape[0]):
        d = _f64(dirs[i])
        lib().orc_sh_basis(c_int(deg), _p(d), _p(row))
        out[i] = row
    return out


def preprocess_3d(scene, cam) -> dict:
    """FP64 projection of a 3D scene.  The paper prints no projection example,
    so the conventions are readings; their implementation is pinned by
    independent routes in the tests (Hamilton-product rotations, Rodrigues'
    formula for the SH basis, finite-difference Jacobians including the
    frustum-guard clamp)."""
    P = scene.P
    means, scales, quats = _f32(scene.means), _f32(scene.scales), _f32(scene.quats)
    sh = _f32(scene.sh.reshape(P, 48))
    camv = _f64(cam.as_array())
    out = dict(means2d=np.zeros((P, 2)), cov2d=np.zeros((P, 3)), conics=np.zeros((P, 3)),
               depths=np.zeros(P), radii=np.zeros(P, np.int32), rgb=np.zeros((P, 3)),
               tiles_touched=np.zeros(P, np.int32), rad_dist=np.zeros(P))
    lib().orc_preprocess_3d(c_int(P), _p(means), _p(scales), _p(quats), _p(sh), c_int(3), _p(camv),
                            _p(out["means2d"]), _p(out["cov2d"]), _p(out["conics"]),
                            _p(out["depths"]), _p(out["radii"]), _p(out["rgb"]),
                            _p(out["tiles_touched"]), _p(out["rad_dist"]))
    return out


def preprocess_2d(means2d, cov2d, W: int, H: int) -> dict:
    m, c = _f32(means2d), _f32(cov2d)
    P = m.shape[0]
    out = dict(conics=np.zeros((P, 3)), radii=np.zeros(P, np.int32),
               tiles_touched=np.zeros(P, np.int32), rad_dist=np.zeros(P))
    lib().orc_preprocess_2d(c_int(P), _p(m), _p(c), c_int(W), c_int(H), _p(out["conics"]),
                            _p(out["radii"]), _p(out["tiles_touched"]), _p(out["rad_dist"]))
    return out


def _precise_args(conics, opac):
    if conics is None:
        return None, None, c_void_p(0), c_void_p(0)
    c, o = _f64(conics), _f64(opac)
    return c, o, _p(c), _p(o)


def bin_splats(means2d, radii, depths, W: int, H: int, conics=None, opac=None):
    """Per-tile splat lists: returns (ranges (ntiles, 2) uint32, ids (N,) uint32).
    With ``conics`` and ``opac`` the precise Gaussian-tile test is applied
    inside the 3-sigma rectangle."""
    m, r, d = _f32(means2d), _i32(radii), _f32(depths)
    keep = _precise_args(conics, opac)
    P = m.shape[0]
    gx, gy = grid(W, H)
    ranges = np.zeros((gx * gy, 2), np.uint32)
    # first call counts (capacity 0), second fills
    N = int(lib().orc_bin(c_int(P), _p(m), _p(r), _p(d), c_int(W), c_int(H), _p(ranges),
                          c_void_p(0), c_int64(0), keep[2], keep[3]))
    if N < 0:
        raise MemoryError("oracle binning: allocation failed")
    ids = np.zeros(max(N, 1), np.uint32)
    N2 = int(lib().orc_bin(c_int(P), _p(m), _p(r), _p(d), c_int(W), c_int(H), _p(ranges),
                           _p(ids), c_int64(N), keep[2], keep[3]))
    assert N2 == N
    return ranges, ids[:N]


def bin_tiles(means2d, radii, depths, W: int, H: int, tiles, conics=None, opac=None):
    """Per-tile splat lists for the listed tiles only (same rule and order as
    bin_splats): returns (ranges (len(tiles), 2) uint32, ids uint32)."""
    m, r, d = _f32(means2d), _i32(radii), _f32(depths)
    keep = _precise_args(conics, opac)
    tl = _i32(tiles)
    P = m.shape[0]
    ranges = np.zeros((len(tl), 2), np.uint32)
    L = lib()
    L.orc_bin_tiles.restype = c_int64
    N = int(L.orc_bin_tiles(c_int(P), _p(m), _p(r), _p(d), c_int(W), c_int(H), c_int(len(tl)),
                            _p(tl), _p(ranges), c_void_p(0), c_int64(0), keep[2], keep[3]))
    if N < 0:
        raise MemoryError("oracle binning: allocation failed")
    ids = np.zeros(max(N, 1), np.uint32)
    L.orc_bin_tiles(c_int(P), _p(m), _p(r), _p(d), c_int(W), c_int(H), c_int(len(tl)), _p(tl),
                    _p(ranges), _p(ids), c_int64(N), keep[2], keep[3])
    return ranges, ids[:N]


def tile_slack(mx: float, my: float, conic, opac: float, tx: int, ty: int, W: int, H: int) -> float:
    """ln o - qmin/2 + ln 255 of the precise Gaussian-tile test (>= 0: kept)."""
    L = lib()
    L.orc_tile_slack.restype = ctypes.c_double
    S = _f64(conic)
    return float(L.orc_tile_slack(ctypes.c_double(mx), ctypes.c_double(my), _p(S),
                                  ctypes.c_double(opac), c_int(tx), c_int(ty), c_int(W), c_int(H)))


def render(W: int, H: int, ranges, ids, means2d, conics, opac, rgb, bg=(0.0, 0.0, 0.0),
           mode: int = MODE_DEF, delta_c: float = 0.0, delta_t: float = 0.0, tiles=None,
           delta_r: float = 0.0) -> dict:
    """Algorithm 1 per pixel in FP64.  With ``tiles`` only those tiles are
    rendered (other pixels are NaN / -1).  Colour is planar (3, H, W).
    A cull decision is flagged as near-threshold when |ln alpha + ln 255| <
    delta_c + delta_r * (sum of |terms| of q/2); a termination decision when
    |T(1 - alpha) - 1e-4| < delta_t * 1e-4.  ``sens`` (exact-definition mode)
    is, per pixel, the sum over composited fragments of alpha T times half
    the sum of |terms| of q: an evaluation whose exponent errs by at most
    rho times that term size moves the colour by at most 2 max|c| rho sens
    and T by at most rho sens (to first order)."""
    rg, idv = np.ascontiguousarray(ranges, np.uint32), np.ascontiguousarray(ids, np.uint32)
    if idv.size == 0:
        idv = np.zeros(1, np.uint32)
    m, c, o, col, b = _f64(means2d), _f64(conics), _f64(opac), _f64(rgb), _f64(bg)
    tl = _i32(tiles if tiles is not None else np.zeros(0))
    ntl = int(tl.size)
    out = dict(rgb=np.full((3, H, W), np.nan), T=np.full((H, W), np.nan),
               n_contrib=np.full((H, W), -1, np.int32), n_proc=np.full((H, W), -1, np.int32),
               f_blend=np.full((H, W), -1, np.int32), f_cull=np.full((H, W), -1, np.int32),
               term=np.full((H, W), -1, np.int32), n_amb=np.full((H, W), -1, np.int32),
               sens=np.full((H, W), np.nan))
    if tiles is not None and ntl == 0:
        return out
    lib().orc_render(c_int(W), c_int(H), _p(rg), _p(idv), _p(m), _p(c), _p(o), _p(col), _p(b),
                     c_int(mode), c_double(delta_c), c_double(delta_r), c_double(delta_t), c_int(ntl),
                     _p(tl) if ntl else c_void_p(0),
                     _p(out["rgb"]), _p(out["T"]), _p(out["n_contrib"]), _p(out["n_proc"]),
                     _p(out["f_blend"]), _p(out["f_cull"]), _p(out["term"]), _p(out["n_amb"]),
                     _p(out["sens"]))
    return out


def render_alternatives(W: int, H: int, ranges, ids, means2d, conics, opac, rgb, pix_xy,
                        bg=(0.0, 0.0, 0.0), mode: int = MODE_DEF, delta_c: float = 1e-5,
                        delta_t: float = 1e-3, delta_r: float = 0.0):
    """All results reachable by inverting up to the first four near-threshold
    decisions at each listed pixel: returns (rgb (n, 16, 3), T (n, 16))."""
    rg, idv = np.ascontiguousarray(ranges, np.uint32), np.ascontiguousarray(ids, np.uint32)
    if idv.size == 0:
        idv = np.zeros(1, np.uint32)
    m, c, o, col, b = _f64(means2d), _f64(conics), _f64(opac), _f64(rgb), _f64(bg)
    px = _i32(np.asarray(pix_xy).reshape(-1, 2))
    n = px.shape[0]
    alt_rgb = np.zeros((max(n, 1), 16, 3))
    alt_T = np.zeros((max(n, 1), 16))
    if n:
        lib().orc_render_alternatives(c_int(W), c_int(H), _p(rg), _p(idv), _p(m), _p(c), _p(o),
                                      _p(col), _p(b), c_int(mode), c_double(delta_c),
                                      c_double(delta_r), c_double(delta_t), c_int(n), _p(px),
                                      _p(alt_rgb), _p(alt_T))
    return alt_rgb[:n], alt_T[:n]


def beta_emulated(mode: int, mu, S, opac: float, p, tc) -> float:
    """Exponent (log2 units) that a reduced-precision matrix unit computes for
    one fragment, with exact accumulation."""
    mu, S, p, tc = _f64(mu), _f64(S), _f64(p), _f64(tc)
    return float(lib().orc_beta_emulated(c_int(mode), _p(mu), _p(S), c_double(opac), _p(p), _p(tc)))


def render_backward(W: int, H: int, ranges, ids, means2d, conics, opac, rgb, dL_dC,
                    bg=(0.0, 0.0, 0.0)) -> dict:
    """FP64 gradients of a loss with respect to means2d, conics, opacities and
    colours, given dL/dC per pixel (planar (3, H, W)), by reverse traversal of
    Algorithm 1 (definition mode)."""
    rg, idv = np.ascontiguousarray(ranges, np.uint32), np.ascontiguousarray(ids, np.uint32)
    if idv.size == 0:
        idv = np.zeros(1, np.uint32)
    m, c, o, col, b = _f64(means2d), _f64(conics), _f64(opac), _f64(rgb), _f64(bg)
    g = _f64(dL_dC)
    P = m.shape[0]
    out = dict(means2d=np.zeros((P, 2)), conics=np.zeros((P, 3)), opacities=np.zeros(P),
               rgb=np.zeros((P, 3)))
    lib().orc_render_backward(c_int(W), c_int(H), _p(rg), _p(idv), _p(m), _p(c), _p(o), _p(col),
                              _p(b), _p(g), _p(out["means2d"]), _p(out["conics"]),
                              _p(out["opacities"]), _p(out["rgb"]))
    return out
