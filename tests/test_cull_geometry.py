"""The geometry behind the matrix-core rasteriser's per-tile cull (Sec. 4.1:
a splat is dropped for a tile when its opacity-weighted Gaussian cannot
reach 1/255 anywhere in the tile's pixel box).

The kernel evaluates the minimum of the convex form q(d) = 1/2 d^T S d
(d = pixel - mean) over the box on two edges only: the vertical and the
horizontal edge on the mean's side.  These host tests check that claim in
FP64 against the minimum over all four edges and against a dense sampling of
the box, for random positive-definite S, means inside and outside the box,
and needle-thin splats.  No GPU is needed."""
import numpy as np
import pytest


def edge_min(S, m, x0, x1, y0, y1, xe=None, ye=None):
    """Minimum of q along the vertical edge x = xe or the horizontal edge
    y = ye of the box (one clamped 1D minimisation)."""
    a, b, c = S
    mx, my = m
    if xe is not None:
        dx = xe - mx
        dy = np.clip(-b / c * dx, y0 - my, y1 - my)
    else:
        dy = ye - my
        dx = np.clip(-b / a * dy, x0 - mx, x1 - mx)
    return 0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)


def box_min_four(S, m, x0, x1, y0, y1):
    mx, my = m
    if x0 <= mx <= x1 and y0 <= my <= y1:
        return 0.0
    return min(edge_min(S, m, x0, x1, y0, y1, xe=x0), edge_min(S, m, x0, x1, y0, y1, xe=x1),
               edge_min(S, m, x0, x1, y0, y1, ye=y0), edge_min(S, m, x0, x1, y0, y1, ye=y1))


def box_min_two(S, m, x0, x1, y0, y1):
    mx, my = m
    if x0 <= mx <= x1 and y0 <= my <= y1:
        return 0.0
    return min(edge_min(S, m, x0, x1, y0, y1, xe=x0 if mx < x0 else x1),
               edge_min(S, m, x0, x1, y0, y1, ye=y0 if my < y0 else y1))


def random_conic(rng, aniso_max):
    th = rng.uniform(0, np.pi)
    s1 = rng.uniform(0.3, 20.0)
    s2 = s1 / rng.uniform(1.0, aniso_max)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    cov = R @ np.diag([s1 * s1, s2 * s2]) @ R.T
    inv = np.linalg.inv(cov)
    return inv[0, 0], inv[0, 1], inv[1, 1]


@pytest.mark.parametrize("aniso_max", [4.0, 100.0, 1e4])
def test_two_facing_edges_hold_the_box_minimum(aniso_max):
    rng = np.random.default_rng(int(aniso_max))
    x0, y0 = 32.0, 48.0
    x1, y1 = x0 + 15.0, y0 + 15.0
    for _ in range(4000):
        S = random_conic(rng, aniso_max)
        m = (rng.uniform(x0 - 60, x1 + 60), rng.uniform(y0 - 60, y1 + 60))
        f4 = box_min_four(S, m, x0, x1, y0, y1)
        f2 = box_min_two(S, m, x0, x1, y0, y1)
        assert f2 == pytest.approx(f4, rel=1e-12, abs=1e-12), (S, m)


def test_box_minimum_matches_dense_sampling():
    """The analytic minimum is attained in the box: no sampled point is
    lower, and the finest sample comes within the grid spacing's reach."""
    rng = np.random.default_rng(7)
    x0, y0 = 0.0, 0.0
    x1, y1 = 15.0, 7.0  # also a half-height box
    g = np.linspace(0.0, 1.0, 241)
    X, Y = np.meshgrid(x0 + (x1 - x0) * g, y0 + (y1 - y0) * g)
    for _ in range(300):
        a, b, c = random_conic(rng, 50.0)
        m = (rng.uniform(-40, 55), rng.uniform(-40, 47))
        f2 = box_min_two((a, b, c), m, x0, x1, y0, y1)
        dx, dy = X - m[0], Y - m[1]
        q = 0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy)
        assert q.min() >= f2 - 1e-9 * max(1.0, f2)
        # the sampled minimum is close to the analytic one (grid step 1/16 px)
        step = (x1 - x0) / 240
        grad = np.hypot(a * dx + b * dy, b * dx + c * dy).max()
        assert q.min() <= f2 + grad * step * 1.5 + 1e-9


def test_mean_on_a_box_side_line():
    """A mean level with the box (inside the x-range, above it) leaves the
    vertical candidate on a side the mean does not violate: the horizontal
    edge still carries the minimum."""
    S = (0.5, 0.45, 0.5)  # strongly correlated
    x0, x1, y0, y1 = 0.0, 15.0, 0.0, 15.0
    for mx in np.linspace(-3.0, 18.0, 43):
        for my in (-9.0, -0.5, 15.5, 24.0):
            m = (mx, my)
            assert box_min_two(S, m, x0, x1, y0, y1) == pytest.approx(
                box_min_four(S, m, x0, x1, y0, y1), rel=1e-12, abs=1e-12)
