"""Seeded synthetic inputs for the Gaussian rasteriser.

This module only draws random numbers and arranges them into input arrays
(scenes and cameras).  It contains none of the rendering method's arithmetic:
no projection, no conic inversion, no binning, no blending.  Both the FP64
oracle (``oracle/``) and the GPU library consume what it produces, which is
the only thing the two sides share.

Conventions
-----------
* Every draw uses ``numpy.random.Generator(PCG64(seed))`` in float64, in the
  order documented in each function, and is stored as float32 so that both
  sides see bit-identical inputs.
* World is Y-up.  Cameras use OpenCV axes (x right, y down, z forward); the
  view matrix is world->camera, row-major, 4x4.
* Pixel ``(x, y)`` has image-plane coordinate ``(x, y)``; the principal point
  is ``(W/2, H/2)`` and the 60 degree field of view is horizontal with
  ``fy = fx``.
* A 3D scene mimics a trained 3DGS model's parameter distributions: 64
  isotropic clusters in a 20 m box, log-normal scales, uniform rotations,
  ``opacity = sigmoid(N(0, 2))`` and degree-3 SH colour coefficients
  ``N(0, 0.3)`` (second parameter = standard deviation).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TILE = 16
SH_COEFFS = 16  # degree 3: (3 + 1)^2


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Camera:
    """Pinhole camera.  ``viewmat`` maps world to camera coordinates."""

    viewmat: np.ndarray  # (4, 4) float32, row-major
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near_z: float = 0.2
    frustum_guard: float = 1.3
    lowpass: float = 0.3
    campos: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))

    def as_array(self) -> np.ndarray:
        """Packed float64 record: viewmat(16), fx, fy, cx, cy, W, H, near,
        guard, lowpass, campos(3) -- 28 values."""
        return np.concatenate([
            self.viewmat.astype(np.float64).reshape(16),
            np.array([self.fx, self.fy, self.cx, self.cy, self.width, self.height,
                      self.near_z, self.frustum_guard, self.lowpass], np.float64),
            self.campos.astype(np.float64).reshape(3),
        ])


def orbit_camera(k: int, K: int, width: int, height: int, radius: float = 15.0,
                 fov_deg: float = 60.0) -> Camera:
    """Pose ``k`` of ``K`` on a horizontal orbit of the given radius, looking
    at the origin.  eye = radius*(sin t, 0, cos t), t = 2*pi*k/K."""
    t = 2.0 * np.pi * k / K
    eye = radius * np.array([np.sin(t), 0.0, np.cos(t)])
    f = -eye / np.linalg.norm(eye)
    r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    tvec = -R @ eye
    view = np.eye(4)
    view[:3, :3] = R
    view[:3, 3] = tvec
    fx = (width / 2.0) / np.tan(np.deg2rad(fov_deg) / 2.0)
    return Camera(viewmat=view.astype(np.float32), fx=float(np.float32(fx)),
                  fy=float(np.float32(fx)), cx=width / 2.0, cy=height / 2.0,
                  width=width, height=height, campos=eye.astype(np.float32))


@dataclass
class Scene3D:
    means: np.ndarray      # (P, 3) float32, metres
    scales: np.ndarray     # (P, 3) float32, metres (per-axis std)
    quats: np.ndarray      # (P, 4) float32, (w, x, y, z) unit quaternion
    opacities: np.ndarray  # (P,)   float32 in (0, 1)
    sh: np.ndarray         # (P, 16, 3) float32, degree-3 SH coefficients

    @property
    def P(self) -> int:
        return int(self.means.shape[0])


def scene_3d(P: int, seed: int, n_clusters: int = 64) -> Scene3D:
    """Clustered 3D scene.  Draw order: cluster centres U[-8,8]^3 (n_clusters x 3),
    cluster std U[0.5, 2] (n_clusters), offsets N(0, I3) (P x 3), log-scales
    N(-4, 1) (P x 3), quaternions N(0, I4) (P x 4), opacity logits N(0, 2) (P),
    SH coefficients N(0, 0.3) (P x 48).  Gaussian i belongs to cluster
    i mod n_clusters; its mean is clipped to [-10, 10]^3."""
    g = _rng(seed)
    centres = g.uniform(-8.0, 8.0, (n_clusters, 3))
    csig = g.uniform(0.5, 2.0, n_clusters)
    cl = np.arange(P) % n_clusters
    means = np.clip(centres[cl] + csig[cl, None] * g.standard_normal((P, 3)), -10.0, 10.0)
    scales = np.exp(g.normal(-4.0, 1.0, (P, 3)))
    q = g.standard_normal((P, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = 1.0 / (1.0 + np.exp(-g.normal(0.0, 2.0, P)))
    sh = g.normal(0.0, 0.3, (P, SH_COEFFS * 3)).reshape(P, SH_COEFFS, 3)
    return Scene3D(means=means.astype(np.float32), scales=scales.astype(np.float32),
                   quats=q.astype(np.float32), opacities=opac.astype(np.float32),
                   sh=sh.astype(np.float32))


def perturbed_scene(sc: Scene3D, seed: int, mean_std: float = 0.01, logit_std: float = 0.5,
                    sh_std: float = 0.05) -> Scene3D:
    """A perturbed copy of a 3D scene (the training step's target scene).
    Draw order: mean offsets N(0, mean_std) (P x 3), opacity-logit offsets
    N(0, logit_std) (P), SH offsets N(0, sh_std) (P x 48); scales and
    rotations are kept."""
    g = _rng(seed)
    P = sc.P
    means = sc.means.astype(np.float64) + g.normal(0.0, mean_std, (P, 3))
    o = np.clip(sc.opacities.astype(np.float64), 1e-7, 1.0 - 1e-7)
    logit = np.log(o) - np.log1p(-o) + g.normal(0.0, logit_std, P)
    opac = 1.0 / (1.0 + np.exp(-logit))
    sh = sc.sh.astype(np.float64) + g.normal(0.0, sh_std, (P, SH_COEFFS * 3)).reshape(P, SH_COEFFS, 3)
    return Scene3D(means=means.astype(np.float32), scales=sc.scales.copy(), quats=sc.quats.copy(),
                   opacities=opac.astype(np.float32), sh=sh.astype(np.float32))


@dataclass
class Scene2D:
    """Already-projected Gaussians (the rasteriser's own input format,
    except that the 2D covariance is given instead of its inverse)."""

    means2d: np.ndarray    # (P, 2) float32 pixel coordinates
    cov2d: np.ndarray      # (P, 3) float32 (a, b, c) = (S_xx, S_xy, S_yy)
    opacities: np.ndarray  # (P,) float32
    rgb: np.ndarray        # (P, 3) float32
    depths: np.ndarray     # (P,) float32
    width: int
    height: int

    @property
    def P(self) -> int:
        return int(self.means2d.shape[0])


def scene_2d(P: int, width: int, height: int, seed: int, s_min: float = 0.5,
             s_max: float = 8.0, o_min: float = 0.05, o_max: float = 0.99,
             grid: float | None = None) -> Scene2D:
    """Pre-projected 2D Gaussians.  Draw order: means U[0,W) x U[0,H) (P x 2),
    axis std exp(U[ln s_min, ln s_max]) (P x 2), rotation angle U[0, pi) (P),
    opacity U[o_min, o_max] (P), rgb U[0,1]^3 (P x 3), depth U[1, 100] (P).
    The covariance is R(theta) diag(s1^2, s2^2) R(theta)^T.  With ``grid`` the
    means are snapped to multiples of ``grid`` (used by translation tests)."""
    g = _rng(seed)
    mu = g.uniform(0.0, 1.0, (P, 2)) * np.array([width, height], np.float64)
    s = np.exp(g.uniform(np.log(s_min), np.log(s_max), (P, 2)))
    th = g.uniform(0.0, np.pi, P)
    o = g.uniform(o_min, o_max, P)
    rgb = g.uniform(0.0, 1.0, (P, 3))
    depth = g.uniform(1.0, 100.0, P)
    if grid is not None:
        mu = np.round(mu / grid) * grid
    c, sn = np.cos(th), np.sin(th)
    a = c * c * s[:, 0] ** 2 + sn * sn * s[:, 1] ** 2
    b = c * sn * (s[:, 0] ** 2 - s[:, 1] ** 2)
    cc = sn * sn * s[:, 0] ** 2 + c * c * s[:, 1] ** 2
    cov = np.stack([a, b, cc], axis=1)
    return Scene2D(means2d=mu.astype(np.float32), cov2d=cov.astype(np.float32),
                   opacities=o.astype(np.float32), rgb=rgb.astype(np.float32),
                   depths=depth.astype(np.float32), width=width, height=height)


def scene_2d_needles(P: int, width: int, height: int, seed: int, s_major=(4.0, 30.0),
                     ratio=(100.0, 300.0), theta_deg=(40.0, 50.0)) -> Scene2D:
    """Pre-projected needle-like Gaussians: major std exp(U[ln lo, ln hi]) px,
    minor std = major / exp(U[ln ratio_lo, ln ratio_hi]), rotation angle
    U[theta_lo, theta_hi] degrees, every second one turned by a further 90
    degrees.  Draw order: means (P x 2), major std (P), ratio (P), angle (P),
    opacity U[0.05, 0.99] (P), rgb (P x 3), depth U[1, 100] (P).  Near 45
    degrees the covariance entries a, c and b are of one size while
    ac - b^2 is (ratio)^-2 smaller: the FP32 determinant cancels."""
    g = _rng(seed)
    mu = g.uniform(0.0, 1.0, (P, 2)) * np.array([width, height], np.float64)
    s1 = np.exp(g.uniform(np.log(s_major[0]), np.log(s_major[1]), P))
    s2 = s1 / np.exp(g.uniform(np.log(ratio[0]), np.log(ratio[1]), P))
    th = np.deg2rad(g.uniform(theta_deg[0], theta_deg[1], P)) + 0.5 * np.pi * (np.arange(P) % 2)
    o = g.uniform(0.05, 0.99, P)
    rgb = g.uniform(0.0, 1.0, (P, 3))
    depth = g.uniform(1.0, 100.0, P)
    c, sn = np.cos(th), np.sin(th)
    a = c * c * s1 ** 2 + sn * sn * s2 ** 2
    b = c * sn * (s1 ** 2 - s2 ** 2)
    cc = sn * sn * s1 ** 2 + c * c * s2 ** 2
    return Scene2D(means2d=mu.astype(np.float32), cov2d=np.stack([a, b, cc], 1).astype(np.float32),
                   opacities=o.astype(np.float32), rgb=rgb.astype(np.float32),
                   depths=depth.astype(np.float32), width=width, height=height)


# Workloads.  "2d" configs are pre-projected; "3d" configs go through the
# projection stage.  Sizes follow the benchmark definitions.
CONFIGS = {
    "fp32_256_2k": dict(kind="2d", P=2000, width=256, height=256, seed=1001),
    "fwd_1080p_1M": dict(kind="3d", P=1_000_000, width=1920, height=1080, seed=1002,
                         pose=0, n_poses=1),
    "fwd_4k_6M": dict(kind="3d", P=6_000_000, width=3840, height=2160, seed=1003,
                      pose=0, n_poses=10),
    "train_1600x1064_1M": dict(kind="3d", P=1_000_000, width=1600, height=1064, seed=1004,
                               pose=0, n_poses=1, target_seed=2004),
    # one scene, 16 cameras on the orbit; camera k has resolution k mod 4
    "multiview_2M_16": dict(kind="3d", P=2_000_000, seed=1005, n_views=16,
                            resolutions=((640, 480), (1280, 720), (1920, 1080), (2560, 1440))),
}


def multiview_cameras(cfg: dict, n_views: int | None = None) -> list:
    """Cameras of a multi-view workload: pose k of n_views on the orbit, at
    resolution index k mod len(resolutions)."""
    n = cfg["n_views"] if n_views is None else n_views
    res = cfg["resolutions"]
    return [orbit_camera(k, n, *res[k % len(res)]) for k in range(n)]


def make_camera(cfg: dict, pose: int | None = None) -> Camera:
    k = cfg.get("pose", 0) if pose is None else pose
    return orbit_camera(k, cfg.get("n_poses", 1), cfg["width"], cfg["height"])


def make_scene(cfg: dict):
    if cfg["kind"] == "2d":
        return scene_2d(cfg["P"], cfg["width"], cfg["height"], cfg["seed"])
    return scene_3d(cfg["P"], cfg["seed"])
