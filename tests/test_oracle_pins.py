"""Pins for the FP64 oracle against what the paper and mathematics fix.

None of these re-derive the oracle's own code: each checks a closed form, an
invariant, a library routine or a brute-force evaluation written differently
(citations are to the TC-GS paper, arXiv 2505.24796).
"""
import math

import numpy as np
import pytest

import scenegen

LN255 = math.log(255.0)


def one_tile_lists(n):
    """Ranges/ids for a single 16x16 tile holding Gaussians 0..n-1 in order."""
    return np.array([[0, n]], np.uint32), np.arange(n, dtype=np.uint32)


def conic_of(cov):
    a, b, c = cov
    return np.linalg.inv(np.array([[a, b], [b, c]]))


# ---------------------------------------------------------------- P1 -------
def test_single_gaussian_closed_form(orc):
    """Algorithm 1 with one Gaussian: C = c*alpha when alpha >= 1/255, with
    alpha = min(0.99, o exp(-q/2)); T_final = 1 - alpha (Sec. 3.1, Alg. 1)."""
    g = np.random.default_rng(7)
    for trial in range(200):
        o = g.uniform(0.004, 1.0)
        L = np.array([[g.uniform(0.3, 4), 0], [g.normal(0, 1), g.uniform(0.3, 4)]])
        Sinv = np.linalg.inv(L @ L.T)
        S = np.array([Sinv[0, 0], Sinv[0, 1], Sinv[1, 1]])
        mu = g.uniform(-4, 20, 2)
        col = g.uniform(0, 1, 3)
        ranges, ids = one_tile_lists(1)
        out = orc.render(16, 16, ranges, ids, mu[None], S[None], [o], col[None])
        for y in range(0, 16, 5):
            for x in range(0, 16, 3):
                d = mu - np.array([x, y], float)
                q = d @ Sinv @ d
                a = min(0.99, o * math.exp(-0.5 * q))
                if a < 1 / 255:
                    exp_c, exp_t = np.zeros(3), 1.0
                else:
                    exp_c, exp_t = col * a, 1 - a
                np.testing.assert_allclose(out["rgb"][:, y, x], exp_c, rtol=0, atol=1e-14)
                assert abs(out["T"][y, x] - exp_t) < 1e-14


def test_isotropic_and_axis_aligned(orc):
    """Special cases: isotropic q = |d|^2/s^2 and axis-aligned q = dx^2/a + dy^2/c."""
    ranges, ids = one_tile_lists(1)
    s2 = 9.0
    out = orc.render(16, 16, ranges, ids, [[7.0, 9.0]], [[1 / s2, 0, 1 / s2]], [0.8], [[1, 1, 1]])
    for (x, y) in [(7, 9), (0, 0), (15, 3)]:
        q = ((x - 7) ** 2 + (y - 9) ** 2) / s2
        a = 0.8 * math.exp(-q / 2)
        a = a if a >= 1 / 255 else 0.0
        assert abs(out["rgb"][0, y, x] - a) < 1e-15
    out = orc.render(16, 16, ranges, ids, [[3.5, 12.25]], [[1 / 4.0, 0, 1 / 25.0]], [0.5], [[1, 0, 0]])
    q = (10 - 3.5) ** 2 / 4 + (2 - 12.25) ** 2 / 25
    a = 0.5 * math.exp(-q / 2)
    assert abs(out["rgb"][0, 2, 10] - (a if a >= 1 / 255 else 0)) < 1e-15


def test_clamp_and_cull_boundaries(orc):
    """alpha is clamped at 0.99; alpha < 1/255 is culled (strict test)."""
    ranges, ids = one_tile_lists(1)
    out = orc.render(16, 16, ranges, ids, [[5.0, 5.0]], [[1.0, 0, 1.0]], [1.0], [[1, 1, 1]])
    assert abs(out["T"][5, 5] - 0.01) < 1e-15 and abs(out["rgb"][0, 5, 5] - 0.99) < 1e-15
    # opacity below 1/255 is culled everywhere
    out = orc.render(16, 16, ranges, ids, [[5.0, 5.0]], [[1.0, 0, 1.0]], [1 / 256], [[1, 1, 1]])
    assert np.all(out["T"] == 1.0) and np.all(out["rgb"] == 0.0)
    assert np.all(out["f_cull"] == 1) and np.all(out["f_blend"] == 0)


# ---------------------------------------------------------------- P2 -------
def test_two_gaussians_order(orc):
    """C = c1 a1 + c2 a2 (1 - a1); swapping depth order swaps the roles."""
    mu = np.array([[6.0, 6.0], [9.0, 7.0]])
    S = np.array([[0.2, 0.03, 0.1], [0.15, -0.02, 0.3]])
    o = np.array([0.7, 0.6])
    col = np.array([[1.0, 0.2, 0.1], [0.0, 0.5, 0.9]])
    for order in ([0, 1], [1, 0]):
        ranges = np.array([[0, 2]], np.uint32)
        ids = np.array(order, np.uint32)
        out = orc.render(16, 16, ranges, ids, mu, S, o, col)
        x, y = 7, 6
        al = []
        for g in order:
            d = mu[g] - [x, y]
            M = np.array([[S[g, 0], S[g, 1]], [S[g, 1], S[g, 2]]])
            al.append(min(0.99, o[g] * math.exp(-0.5 * d @ M @ d)))
        exp_c = col[order[0]] * al[0] + col[order[1]] * al[1] * (1 - al[0])
        np.testing.assert_allclose(out["rgb"][:, y, x], exp_c, atol=1e-14)
        assert abs(out["T"][y, x] - (1 - al[0]) * (1 - al[1])) < 1e-14


# ---------------------------------------------------------------- P3 -------
def test_termination_closed_form(orc):
    """Identical alpha = 0.8 fragments: T = 0.2^k; the sixth test gives
    0.2^6 = 6.4e-5 < 1e-4, so five are composited and the sixth stops
    the pixel without being composited (Alg. 1)."""
    n = 10
    ranges, ids = one_tile_lists(n)
    mu = np.tile([[4.0, 4.0]], (n, 1))
    S = np.tile([[1e-9, 0, 1e-9]], (n, 1))
    o = np.full(n, 0.8)
    col = np.tile([[1.0, 0.5, 0.25]], (n, 1))
    out = orc.render(16, 16, ranges, ids, mu, S, o, col)
    a = 0.8 * math.exp(-0.5 * 1e-9 * 0)  # centre pixel q = 0
    expC = sum(a * (1 - a) ** k for k in range(5))
    assert abs(out["rgb"][0, 4, 4] - expC) < 1e-12
    assert out["n_contrib"][4, 4] == 5 and out["term"][4, 4] == 1
    assert out["n_proc"][4, 4] == 6 and out["f_blend"][4, 4] == 5


def test_invariants_random_scene(orc):
    """With every colour 1, C = sum_i alpha_i T_i and C + T_final = 1 by the
    telescoping of T <- T - alpha T; T_final >= 1e-4; C <= max colour."""
    sc = scenegen.scene_2d(1500, 96, 80, seed=11, o_min=0.5)
    pre = orc.preprocess_2d(sc.means2d, sc.cov2d, 96, 80)
    ranges, ids = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, 96, 80)
    ones = np.ones((sc.P, 3))
    out = orc.render(96, 80, ranges, ids, sc.means2d, pre["conics"], sc.opacities, ones)
    np.testing.assert_allclose(out["rgb"][0] + out["T"], 1.0, atol=1e-12)
    assert out["T"].min() >= 1e-4
    assert (out["term"] == 1).any()  # the scene is dense enough to terminate somewhere
    out2 = orc.render(96, 80, ranges, ids, sc.means2d, pre["conics"], sc.opacities, sc.rgb)
    assert out2["rgb"].max() <= sc.rgb.max() + 1e-12 and out2["rgb"].min() >= 0
    # fragment accounting: processed = blended + culled + terminating
    assert np.all(out2["n_proc"] == out2["f_blend"] + out2["f_cull"] + out2["term"])


def test_sensitivity_single_gaussian_closed_form(orc):
    """One composited fragment: sens = alpha * (s11 dx^2 + 2 |s12 dx dy| +
    s22 dy^2) / 2 (with T = 1 in front of it); culled pixels carry 0."""
    ranges, ids = one_tile_lists(1)
    mu, S, o = np.array([6.3, 8.7]), np.array([0.31, -0.17, 0.22]), 0.7
    out = orc.render(16, 16, ranges, ids, mu[None], S[None], [o], [[0.2, 0.5, 0.9]])
    Sm = np.array([[S[0], S[1]], [S[1], S[2]]])
    for y in range(16):
        for x in range(16):
            d = mu - np.array([x, y], float)
            a = min(0.99, o * math.exp(-0.5 * d @ Sm @ d))
            terms = 0.5 * (abs(S[0]) * d[0] ** 2 + 2 * abs(S[1] * d[0] * d[1]) + abs(S[2]) * d[1] ** 2)
            want = a * terms if a >= 1 / 255 else 0.0
            assert abs(out["sens"][y, x] - want) <= 1e-14 * max(1.0, want)


def test_sensitivity_bounds_a_perturbed_exponent(orc):
    """The first-order bound the FP32 parity check uses: the conic
    (s11, s12, s22) -> (s11 (1 + r), s12 (1 - r), s22 (1 + r)) changes each
    exponent by at most r (sum of |terms| of q)/2, reaching it wherever the
    cross term opposes the squares (near a needle's axis, where q cancels).
    On pixels with no near-threshold decision the colour then moves by at
    most 2 max|c| r sens and T by at most r sens (plus second-order slack),
    and the bound is reached to within a small factor, so it is not vacuous,
    for well-conditioned splats and for near-degenerate needles alike."""
    W, H = 96, 80
    for sc in (scenegen.scene_2d(800, W, H, seed=12),
               scenegen.scene_2d_needles(300, W, H, seed=13)):
        pre = orc.preprocess_2d(sc.means2d, sc.cov2d, W, H)
        ranges, ids = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, H)
        r = 1e-7
        base = orc.render(W, H, ranges, ids, sc.means2d, pre["conics"], sc.opacities, sc.rgb,
                          delta_c=1e-5, delta_t=1e-3, delta_r=2 * r)
        con = pre["conics"] * np.array([1 + r, 1 - r, 1 + r])
        pert = orc.render(W, H, ranges, ids, sc.means2d, con, sc.opacities, sc.rgb)
        ok = base["n_amb"] == 0
        cm = float(np.abs(sc.rgb).max())
        dC = np.abs(pert["rgb"] - base["rgb"]).max(axis=0)[ok]
        dT = np.abs(pert["T"] - base["T"])[ok]
        sens = base["sens"][ok]
        assert np.all(dC <= 2 * cm * r * sens * (1 + 1e-3) + 1e-15)
        assert np.all(dT <= r * sens * (1 + 1e-3) + 1e-15)
        big = sens > np.percentile(sens, 90)
        assert np.max(dT[big] / (r * sens[big])) > 0.3


# ---------------------------------------------------------------- P4 / P7 --
def _exact_beta_log2(mu, S, o, p):
    d = np.asarray(mu, float) - np.asarray(p, float)
    M = np.array([[S[0], S[1]], [S[1], S[2]]])
    return (math.log(o) - 0.5 * d @ M @ d) / math.log(2)


def _uv(mu, S, o, p, org):
    """|u_i v_i| terms of the Frag2Mat dot product (log2-scaled), for the
    bound of the rounding-error proposition (Appendix A.3)."""
    dx, dy = mu[0] - org[0], mu[1] - org[1]
    px, py = p[0] - org[0], p[1] - org[1]
    v = np.array([math.log(o) - 0.5 * (S[0] * dx * dx + 2 * S[1] * dx * dy + S[2] * dy * dy),
                  S[0] * dx + S[1] * dy, S[1] * dx + S[2] * dy, -0.5 * S[0], -S[1], -0.5 * S[2]])
    u = np.array([1, px, py, px * px, px * py, py * py])
    return np.abs(u * v) / math.log(2)


def _u(p, org):
    px, py = p[0] - org[0], p[1] - org[1]
    return np.array([1, px, py, px * px, px * py, py * py])


@pytest.mark.parametrize("mode,unit", [(2, 2.0 ** -11), (3, 2.0 ** -22), (4, 2.0 ** -24)])
def test_emulated_beta_identity_and_bound(orc, mode, unit):
    """Frag2Mat (Sec. 4.2): u^T v equals ln o - 1/2 d^T S d; in local
    coordinates (Sec. 4.3) the only error is rounding v, bounded by
    unit * sum |u_i v_i| (Appendix A, with the exact-u and RNE refinements)."""
    g = np.random.default_rng(3)
    worst = 0.0
    for _ in range(3000):
        tc = np.array([16 * g.integers(0, 100) + 7.5, 16 * g.integers(0, 60) + 7.5])
        p = tc + g.integers(-7, 9, 2) - 0.5
        mu = tc + g.normal(0, 12, 2)
        L = np.array([[g.uniform(0.5, 30), 0], [g.normal(0, 3), g.uniform(0.5, 30)]])
        Si = np.linalg.inv(L @ L.T)
        S = np.array([Si[0, 0], Si[0, 1], Si[1, 1]])
        o = g.uniform(0.01, 1)
        b = orc.beta_emulated(mode, mu, S, o, p, tc)
        ex = _exact_beta_log2(mu, S, o, p)
        # relative part, plus half the FP16 subnormal spacing (2^-25) per
        # term for coefficients that fall below the FP16 normal range
        sub = 2.0 ** -25 * (np.abs(_u(p, tc)).sum() + 2) if mode in (2, 3) else 0.0
        bound = unit * _uv(mu, S, o, p, tc).sum() * (3 if mode == 2 else 1) + sub + 1e-12
        assert abs(b - ex) <= bound, (b, ex, bound)
        worst = max(worst, abs(b - ex) / bound)
    assert worst > 0.05  # the bound is reached to within a small factor: rounding is real


def test_global_fp16_collapses_local_recovers(orc):
    """Sec. 4.3 / Table 6: FP16 in global coordinates loses beta (quadratic
    terms of size w^2), local coordinates keep it at O(w + h) eps."""
    g = np.random.default_rng(5)
    err_g, err_l = [], []
    for _ in range(300):
        tc = np.array([16 * g.integers(5, 15) + 7.5, 16 * g.integers(5, 15) + 7.5])
        p = tc + g.integers(-7, 9, 2) - 0.5
        mu = p + g.normal(0, 3, 2)
        S = np.array([0.25, 0.02, 0.3])
        o = 0.9
        ex = _exact_beta_log2(mu, S, o, p)
        err_g.append(abs(orc.beta_emulated(1, mu, S, o, p, tc) - ex))
        err_l.append(abs(orc.beta_emulated(2, mu, S, o, p, tc) - ex))
    assert np.median(err_g) > 1.0       # whole units of beta lost
    assert np.max(err_l) < 0.05


def test_g2l_translation_invariance(orc):
    """G2L (Sec. 4.3): v depends on mu' - p(T) only, so shifting mu' and p by
    whole tiles leaves the emulated beta bit-identical; the global frame does not."""
    g = np.random.default_rng(9)
    diff_global = 0
    for _ in range(200):
        tc = np.array([16 * 3 + 7.5, 16 * 2 + 7.5])
        p = tc + g.integers(-7, 9, 2) - 0.5
        mu = np.round((tc + g.normal(0, 6, 2)) * 256) / 256
        S = np.array([0.3, -0.05, 0.2])
        sh = np.array([16.0 * 41, 16.0 * 17])
        for mode in (2, 3, 4):
            assert orc.beta_emulated(mode, mu, S, 0.7, p, tc) == \
                orc.beta_emulated(mode, mu + sh, S, 0.7, p + sh, tc + sh)
        diff_global += orc.beta_emulated(1, mu, S, 0.7, p, tc) != \
            orc.beta_emulated(1, mu + sh, S, 0.7, p + sh, tc + sh)
    assert diff_global > 100


# ---------------------------------------------------------------- rounding -
def test_round_fp16_matches_numpy(orc):
    g = np.random.default_rng(1)
    xs = np.concatenate([g.normal(0, 1, 2000), g.normal(0, 1e4, 500), g.uniform(-1e-6, 1e-6, 500),
                         [65504.0, 65519.0, 65520.0, -65520.0, 1e6, 2.0 ** -24, 2.0 ** -25,
                          3 * 2.0 ** -26, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11]])
    for x in xs:
        with np.errstate(over="ignore"):
            ref = float(np.float16(x))
        got = orc.round_fp16(float(x))
        assert (ref == got) or (math.isinf(ref) and math.isinf(got) and ref == got), (x, ref, got)


def test_round_bf16_matches_torch(orc):
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(2)
    xs = np.concatenate([g.normal(0, 1, 2000), g.normal(0, 1e20, 200), [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8]])
    xs = xs.astype(np.float32).astype(np.float64)  # torch converts from float32
    ref = torch.tensor(xs, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    for x, r in zip(xs, ref):
        assert orc.round_bf16(float(x)) == r


# ---------------------------------------------------------------- SH -------
def test_sh_orthonormal(orc):
    """The degree-3 real SH basis is orthonormal on the sphere (quadrature)."""
    nt, npf = 24, 48
    xg, wg = np.polynomial.legendre.leggauss(nt)  # in cos(theta)
    phi = (np.arange(npf) + 0.5) * 2 * np.pi / npf
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (np.repeat(wg, npf) * (2 * np.pi / npf))
    Y = orc.sh_basis(dirs, 3)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-10)
    assert abs(Y[0, 0] - 0.5 / math.sqrt(math.pi)) < 1e-15
    # degree 1 is proportional to (y, z, x) with the Condon-Shortley sign on m = +-1
    d = np.array([[0.3, -0.5, 0.8]])
    d = d / np.linalg.norm(d)
    Y1 = orc.sh_basis(d, 1)[0]
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y1[1:4], [-c1 * d[0, 1], c1 * d[0, 2], -c1 * d[0, 0]], atol=1e-15)


# ---------------------------------------------------------------- preprocess
def test_preprocess_2d_against_linalg(orc):
    """Conic = inverse covariance; r = ceil(3 sqrt(lambda_max)) when the
    eigenvalues are well separated; tiles_touched = brute-force count of
    tiles met by the pixel box [floor(mu) - r, floor(mu) + r]."""
    sc = scenegen.scene_2d(300, 100, 70, seed=4)
    out = orc.preprocess_2d(sc.means2d, sc.cov2d, 100, 70)
    for i in range(sc.P):
        C = np.array(sc.cov2d[i], float)
        M = np.array([[C[0], C[1]], [C[1], C[2]]])
        inv = np.linalg.inv(M)
        np.testing.assert_allclose(out["conics"][i], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-12)
        ev = np.linalg.eigvalsh(M)
        mid = 0.5 * (C[0] + C[2])
        if mid * mid - np.linalg.det(M) > 0.1:
            assert out["radii"][i] == math.ceil(3 * math.sqrt(ev[-1]))
        r = out["radii"][i]
        fx, fy = math.floor(sc.means2d[i, 0]), math.floor(sc.means2d[i, 1])
        cnt = 0
        for ty in range(5):
            for tx in range(7):
                if (fx + r >= 16 * tx and fx - r <= 16 * tx + 15 and fx - r <= 99 and
                        fy + r >= 16 * ty and fy - r <= 16 * ty + 15 and fy - r <= 69):
                    cnt += 1
        assert out["tiles_touched"][i] == cnt


def test_preprocess_3d_textbook(orc):
    """Projection checks: a Gaussian on the optical axis projects to the
    principal point with Sigma' = (f s / z)^2 I + 0.3 I; off axis, Sigma'
    equals the finite-difference Jacobian of the pinhole map pushed through
    the 3D covariance (Sec. 3.1: Sigma' = J W Sigma W^T J^T)."""
    cam = scenegen.orbit_camera(0, 1, 640, 480)
    P = 3
    means = np.array([[0, 0, 0], [1.5, -1.0, 2.0], [-2.0, 0.5, -3.0]], np.float32)
    scales = np.array([[0.1, 0.1, 0.1], [0.2, 0.05, 0.1], [0.02, 0.3, 0.08]], np.float32)
    q = np.array([[1, 0, 0, 0], [0.9, 0.1, -0.3, 0.2], [0.2, 0.7, 0.1, -0.4]], np.float32)
    sh = np.zeros((P, 16, 3), np.float32)
    sc = scenegen.Scene3D(means=means, scales=scales, quats=q, opacities=np.full(P, 0.5, np.float32), sh=sh)
    out = orc.preprocess_3d(sc, cam)
    f = cam.fx
    np.testing.assert_allclose(out["means2d"][0], [320, 240], atol=1e-9)
    np.testing.assert_allclose(out["cov2d"][0], [(f * 0.1 / 15) ** 2 + 0.3, 0, (f * 0.1 / 15) ** 2 + 0.3],
                               rtol=1e-6, atol=1e-9)
    assert abs(out["depths"][0] - 15.0) < 1e-6
    V = cam.viewmat.astype(np.float64)

    def proj(x):
        t = V[:3, :3] @ x + V[:3, 3]
        return np.array([f * t[0] / t[2] + cam.cx, f * t[1] / t[2] + cam.cy])

    for i in (1, 2):
        m = means[i].astype(np.float64)
        h = 1e-5
        Jfd = np.stack([(proj(m + h * e) - proj(m - h * e)) / (2 * h) for e in np.eye(3)], 1)
        w, x, y, z = (q[i] / np.linalg.norm(q[i])).astype(np.float64)
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        Sig = R @ np.diag(scales[i].astype(np.float64) ** 2) @ R.T
        C2 = Jfd @ Sig @ Jfd.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(out["cov2d"][i], [C2[0, 0], C2[0, 1], C2[1, 1]], rtol=1e-6)
        np.testing.assert_allclose(out["means2d"][i], proj(m), rtol=1e-12)
    # SH colour: with only the DC coefficient set, rgb = k00 Y00 + 0.5
    sh2 = sh.copy()
    sh2[:, 0, :] = [0.4, -0.2, -3.0]
    sc2 = scenegen.Scene3D(means=means, scales=scales, quats=q, opacities=sc.opacities, sh=sh2)
    out2 = orc.preprocess_3d(sc2, cam)
    y00 = 0.5 / math.sqrt(math.pi)
    np.testing.assert_allclose(out2["rgb"][0], [0.4 * y00 + 0.5, -0.2 * y00 + 0.5, 0.0], atol=1e-7)


def test_preprocess_3d_near_plane_and_rotation_invariance(orc):
    """Gaussians behind the near plane are dropped; a rotation about the
    Gaussian's own isotropic shape does not change its projection."""
    cam = scenegen.orbit_camera(0, 1, 320, 240)
    means = np.array([[0, 0, 14.9], [0, 0, 20.0], [0.3, 0.2, 1.0], [0.3, 0.2, 1.0]], np.float32)
    scales = np.array([[0.1] * 3, [0.1] * 3, [0.05] * 3, [0.05] * 3], np.float32)
    q = np.array([[1, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0], [0.5, 0.5, -0.5, 0.5]], np.float32)
    sc = scenegen.Scene3D(means=means, scales=scales, quats=q, opacities=np.full(4, .5, np.float32),
                          sh=np.zeros((4, 16, 3), np.float32))
    out = orc.preprocess_3d(sc, cam)
    assert out["radii"][0] == 0 and out["radii"][1] == 0   # depth 0.1 and -5
    np.testing.assert_allclose(out["cov2d"][2], out["cov2d"][3], rtol=1e-12)


# ---------------------------------------------------------------- R(q) -----
def _hamilton(p, q):
    """Hamilton product of quaternions (w, x, y, z)."""
    w1, x1, y1, z1 = p
    w2, x2, y2, z2 = q
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _rotate(q, v):
    """v rotated by the unit quaternion q as the product q (0, v) q*."""
    q = np.asarray(q, np.float64) / np.linalg.norm(q)
    qc = q * np.array([1.0, -1.0, -1.0, -1.0])
    return _hamilton(_hamilton(q, np.concatenate([[0.0], v])), qc)[1:]


def _cov2d_expected(cam, mean, Sigma, h=1e-5):
    """Sigma' = J Sigma J^T + 0.3 I with J the central finite-difference
    Jacobian of the pinhole map world -> pixel at the mean (Sec. 3.1)."""
    V = cam.viewmat.astype(np.float64)

    def proj(x):
        t = V[:3, :3] @ x + V[:3, 3]
        return np.array([cam.fx * t[0] / t[2] + cam.cx, cam.fy * t[1] / t[2] + cam.cy])

    J = np.stack([(proj(mean + h * e) - proj(mean - h * e)) / (2 * h) for e in np.eye(3)], 1)
    C2 = J @ Sigma @ J.T + 0.3 * np.eye(2)
    return np.array([C2[0, 0], C2[0, 1], C2[1, 1]])


def _scene(means, scales, quats, opac=None, sh=None):
    P = len(means)
    return scenegen.Scene3D(means=np.asarray(means, np.float32), scales=np.asarray(scales, np.float32),
                            quats=np.asarray(quats, np.float32),
                            opacities=np.full(P, 0.5, np.float32) if opac is None else np.asarray(opac, np.float32),
                            sh=np.zeros((P, 16, 3), np.float32) if sh is None else sh)


def test_rotation_from_hamilton_products(orc):
    """R(q) enters Sigma = R diag(s^2) R^T.  Here R is built column by column
    from the quaternion rotation v -> q v q* (Hamilton products, a route that
    shares nothing with a matrix formula), so a transposed or mis-signed R(q)
    changes the anisotropic 2D covariance and fails.  Non-unit quaternions
    are normalised first (the same result for q and 3.7 q)."""
    cam = scenegen.orbit_camera(0, 1, 640, 480)
    g = np.random.default_rng(31)
    P = 12
    means = np.column_stack([g.uniform(-2, 2, P), g.uniform(-1.5, 1.5, P), g.uniform(-3, 3, P)])
    scales = np.exp(g.uniform(np.log(0.02), np.log(0.3), (P, 3)))
    quats = g.standard_normal((P, 4))
    quats[1::2] *= 3.7  # not normalised on input
    sc = _scene(means, scales, quats)
    out = orc.preprocess_3d(sc, cam)
    assert (out["radii"] > 0).all()
    for i in range(P):
        q = sc.quats[i].astype(np.float64)
        R = np.stack([_rotate(q, e) for e in np.eye(3)], 1)
        # sanity of the independent route: orthonormal, det +1, composition
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R) - 1.0) < 1e-12
        Sigma = R @ np.diag(sc.scales[i].astype(np.float64) ** 2) @ R.T
        want = _cov2d_expected(cam, sc.means[i].astype(np.float64), Sigma)
        np.testing.assert_allclose(out["cov2d"][i], want, rtol=1e-6)
    q1, q2 = quats[0] / np.linalg.norm(quats[0]), quats[2] / np.linalg.norm(quats[2])
    R1 = np.stack([_rotate(q1, e) for e in np.eye(3)], 1)
    R2 = np.stack([_rotate(q2, e) for e in np.eye(3)], 1)
    R12 = np.stack([_rotate(_hamilton(q1, q2), e) for e in np.eye(3)], 1)
    np.testing.assert_allclose(R12, R1 @ R2, atol=1e-12)


@pytest.mark.parametrize("deg", [30.0, -50.0])
def test_rotation_about_world_axis_closed_form(orc, deg):
    """A needle-like Gaussian (std s along its own x axis, eps across) turned
    by +theta about the world z axis (q = (cos theta/2, 0, 0, sin theta/2))
    points along (cos theta, sin theta, 0).  Seen by the pose-0 orbit camera
    (camera x = world x, camera y = -world y) at the optical axis, depth 15:
    Sigma' = (f/15)^2 s^2 [[c^2, -c s_], [-c s_, s_^2]] + eps terms + 0.3 I.
    The sign of the off-diagonal pins the direction of rotation."""
    cam = scenegen.orbit_camera(0, 1, 640, 480)
    th = math.radians(deg)
    s, eps = 0.4, 0.01
    q = [math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)]
    out = orc.preprocess_3d(_scene([[0, 0, 0]], [[s, eps, eps]], [q]), cam)
    k = (cam.fx / 15.0) ** 2
    c, sn = math.cos(th), math.sin(th)
    # the eps axis in the image plane is (-sin, cos) in world -> (-sin, -cos) in camera
    want = [k * (s * s * c * c + eps * eps * sn * sn) + 0.3,
            k * (-s * s * c * sn + eps * eps * sn * c),
            k * (s * s * sn * sn + eps * eps * c * c) + 0.3]
    # inputs are stored as float32 (relative rounding ~6e-8)
    np.testing.assert_allclose(out["cov2d"][0], want, rtol=1e-6)
    assert np.sign(out["cov2d"][0][1]) == -np.sign(sn)


# ---------------------------------------------------------------- SH l=2,3 -
def _legendre_rodrigues(l, m, x):
    """Associated Legendre function with the Condon-Shortley phase from
    Rodrigues' formula: P_l(x) = 1/(2^l l!) d^l/dx^l (x^2 - 1)^l and
    P_l^m(x) = (-1)^m (1 - x^2)^(m/2) d^m/dx^m P_l(x) (exact polynomial
    derivatives, no recurrence)."""
    from numpy.polynomial import polynomial as Pn
    c = Pn.polypow([-1.0, 0.0, 1.0], l)
    c = Pn.polyder(c, l + m) / (2.0 ** l * math.factorial(l))
    return (-1.0) ** m * (1.0 - x * x) ** (m / 2.0) * Pn.polyval(x, c)


def test_sh_each_function_from_rodrigues(orc):
    """Every real SH function of degrees 0..3 (index l*l + l + m) equals
    sqrt(2) K_lm P_l^m(cos t) cos(m phi) for m > 0, sqrt(2) K_l|m|
    P_l^|m|(cos t) sin(|m| phi) for m < 0 and K_l0 P_l(cos t) for m = 0,
    K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), with P_l^m from Rodrigues'
    formula above.  Pins sign and order within each degree, which
    orthonormality alone leaves free."""
    g = np.random.default_rng(8)
    dirs = g.standard_normal((64, 3))
    dirs = np.vstack([dirs, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, -1, 0]]])
    Y = orc.sh_basis(dirs, 3)
    for i, d in enumerate(dirs):
        x, y, z = d / np.linalg.norm(d)
        phi = math.atan2(y, x)
        for l in range(4):
            for m in range(-l, l + 1):
                am = abs(m)
                K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
                P = _legendre_rodrigues(l, am, z)
                if m > 0:
                    want = math.sqrt(2) * K * P * math.cos(am * phi)
                elif m < 0:
                    want = math.sqrt(2) * K * P * math.sin(am * phi)
                else:
                    want = K * P
                assert abs(Y[i, l * l + l + m] - want) < 1e-13, (l, m, Y[i, l * l + l + m], want)


def test_sh_addition_theorem(orc):
    """For each degree l: sum_m Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a . b)
    (P_l from numpy's Legendre series), which holds for any orthonormal real
    basis of the degree and so pins each degree's span and normalisation."""
    from numpy.polynomial import legendre
    g = np.random.default_rng(9)
    a = g.standard_normal((40, 3))
    b = g.standard_normal((40, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya, Yb = orc.sh_basis(a, 3), orc.sh_basis(b, 3)
    for l in range(4):
        sl = slice(l * l, (l + 1) * (l + 1))
        lhs = np.sum(Ya[:, sl] * Yb[:, sl], axis=1)
        cos = np.sum(a * b, axis=1)
        rhs = (2 * l + 1) / (4 * math.pi) * legendre.legval(cos, [0] * l + [1])
        np.testing.assert_allclose(lhs, rhs, atol=1e-13)


# ---------------------------------------------------------------- guard ----
@pytest.mark.parametrize("side", ["+x", "-x", "+y", "+xy"])
def test_preprocess_3d_frustum_guard_clamp(orc, side):
    """Outside the guard band |t_x/t_z| > 1.3 tan(fov_x/2) (likewise y), the
    Jacobian J of the projection is taken at the camera-space point whose
    t_x/t_z (t_y/t_z) is clamped to the band edge, depth unchanged; the mean
    itself is projected unclamped.  Pinned with the finite-difference
    Jacobian of the pinhole map (t -> (f t_x/t_z + c_x, f t_y/t_z + c_y)) at
    that clamped point, and shown to differ from the unclamped Jacobian."""
    W, H = 320, 240
    cam = scenegen.orbit_camera(0, 1, W, H)
    V = cam.viewmat.astype(np.float64)
    limx, limy = 1.3 * (0.5 * W / cam.fx), 1.3 * (0.5 * H / cam.fy)
    tz = 5.0
    ratio = {"+x": (0.9, 0.1), "-x": (-1.1, 0.0), "+y": (0.2, 0.75), "+xy": (0.95, -0.7)}[side]
    tcam = np.array([ratio[0] * tz, ratio[1] * tz, tz])
    # camera -> world: x_w = R^T (t - t_wc)
    mean = V[:3, :3].T @ (tcam - V[:3, 3])
    scales = [0.9, 0.6, 1.2]
    q = np.array([0.8, 0.3, -0.4, 0.33])
    out = orc.preprocess_3d(_scene([mean], [scales], [q]), cam)
    assert out["radii"][0] > 0, "the test Gaussian must reach the image"
    R = np.stack([_rotate(q, e) for e in np.eye(3)], 1)
    Sigma = R @ np.diag(np.asarray(np.float32(scales), np.float64) ** 2) @ R.T
    m32 = np.asarray(np.float32(mean), np.float64)
    t = V[:3, :3] @ m32 + V[:3, 3]
    tc = np.array([np.clip(t[0] / t[2], -limx, limx) * t[2], np.clip(t[1] / t[2], -limy, limy) * t[2], t[2]])

    def pin(tt):
        return np.array([cam.fx * tt[0] / tt[2] + cam.cx, cam.fy * tt[1] / tt[2] + cam.cy])

    h = 1e-6
    Jc = np.stack([(pin(tc + h * e) - pin(tc - h * e)) / (2 * h) for e in np.eye(3)], 1)
    Ju = np.stack([(pin(t + h * e) - pin(t - h * e)) / (2 * h) for e in np.eye(3)], 1)

    def cov(J):
        C2 = J @ V[:3, :3] @ Sigma @ V[:3, :3].T @ J.T + 0.3 * np.eye(2)
        return np.array([C2[0, 0], C2[0, 1], C2[1, 1]])

    np.testing.assert_allclose(out["cov2d"][0], cov(Jc), rtol=1e-6)
    assert np.max(np.abs(cov(Ju) - cov(Jc)) / np.abs(cov(Jc)).max()) > 1e-2
    np.testing.assert_allclose(out["means2d"][0], pin(t), rtol=1e-12)


def test_preprocess_3d_invalid_inputs_dropped(orc):
    """Gaussians whose mean, scale or quaternion is not finite (or whose
    quaternion is zero) get radius 0 and no tiles; a finite neighbour is
    unaffected."""
    cam = scenegen.orbit_camera(0, 1, 320, 240)
    nan, inf = float("nan"), float("inf")
    means = [[0, 0, 0], [nan, 0, 0], [0, inf, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0]]
    scales = [[0.1] * 3, [0.1] * 3, [0.1] * 3, [nan, 0.1, 0.1], [0.1, inf, 0.1], [0.1] * 3, [0.1] * 3]
    quats = [[1, 0, 0, 0]] * 5 + [[0, 0, 0, 0], [nan, 0, 0, 1]]
    out = orc.preprocess_3d(_scene(means, scales, quats), cam)
    assert out["radii"][0] > 0 and out["tiles_touched"][0] > 0
    assert (out["radii"][1:] == 0).all() and (out["tiles_touched"][1:] == 0).all()


# ---------------------------------------------------------------- P5 / P6 --
def _brute_force(sc, conics, radii, W, H):
    """Per pixel: every Gaussian whose coverage box meets the pixel's tile, in
    (depth, index) order, then Algorithm 1.  Plain Python loops."""
    img = np.zeros((3, H, W))
    Tf = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            tx, ty = x // 16, y // 16
            cand = []
            for i in range(sc.P):
                r = int(radii[i])
                if r <= 0:
                    continue
                fx, fy = math.floor(sc.means2d[i, 0]), math.floor(sc.means2d[i, 1])
                x0, x1 = max(fx - r, 0), min(fx + r, W - 1)
                y0, y1 = max(fy - r, 0), min(fy + r, H - 1)
                if x0 > x1 or y0 > y1:
                    continue
                if x0 // 16 <= tx <= x1 // 16 and y0 // 16 <= ty <= y1 // 16:
                    cand.append((float(sc.depths[i]), i))
            cand.sort()
            T, C = 1.0, np.zeros(3)
            for _, i in cand:
                d = sc.means2d[i].astype(float) - [x, y]
                S = conics[i]
                q = S[0] * d[0] ** 2 + 2 * S[1] * d[0] * d[1] + S[2] * d[1] ** 2
                a = min(0.99, float(sc.opacities[i]) * math.exp(-0.5 * q))
                if a < 1 / 255:
                    continue
                if T - a * T < 1e-4:
                    break
                C += sc.rgb[i].astype(float) * a * T
                T = T - a * T
            img[:, y, x] = C
            Tf[y, x] = T
    return img, Tf


def test_tiled_matches_brute_force(orc):
    W, H = 32, 24
    for seed in (21, 22):
        sc = scenegen.scene_2d(20, W, H, seed=seed, s_min=0.8, s_max=5.0)
        pre = orc.preprocess_2d(sc.means2d, sc.cov2d, W, H)
        ranges, ids = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, H)
        out = orc.render(W, H, ranges, ids, sc.means2d, pre["conics"], sc.opacities, sc.rgb)
        img, Tf = _brute_force(sc, pre["conics"], pre["radii"], W, H)
        np.testing.assert_allclose(out["rgb"], img, atol=1e-12)
        np.testing.assert_allclose(out["T"], Tf, atol=1e-12)


def test_permutation_invariance(orc):
    """Shuffling the input order (distinct depths) leaves the image identical."""
    W, H = 64, 48
    sc = scenegen.scene_2d(150, W, H, seed=31)
    perm = np.random.default_rng(0).permutation(sc.P)
    outs = []
    for pr in (np.arange(sc.P), perm):
        m, cv, o, c, d = sc.means2d[pr], sc.cov2d[pr], sc.opacities[pr], sc.rgb[pr], sc.depths[pr]
        pre = orc.preprocess_2d(m, cv, W, H)
        ranges, ids = orc.bin_splats(m, pre["radii"], d, W, H)
        outs.append(orc.render(W, H, ranges, ids, m, pre["conics"], o, c)["rgb"])
    assert np.array_equal(outs[0], outs[1])


def test_binning_order_and_ties(orc):
    """Ties in depth are broken by Gaussian index; lists are sorted by depth."""
    W, H = 48, 32
    sc = scenegen.scene_2d(200, W, H, seed=41)
    d = sc.depths.copy()
    d[::3] = 5.0
    pre = orc.preprocess_2d(sc.means2d, sc.cov2d, W, H)
    ranges, ids = orc.bin_splats(sc.means2d, pre["radii"], d, W, H)
    assert ranges[-1, 1] == len(ids) or ranges[:, 1].max() == len(ids)
    for t in range(ranges.shape[0]):
        s, e = ranges[t]
        seg = ids[s:e]
        keys = list(zip(d[seg], seg))
        assert keys == sorted(keys)
    assert int(pre["tiles_touched"].sum()) == len(ids)


def test_alternatives_cover_nominal(orc):
    """The admissible set always contains the nominal result (mask 0)."""
    W, H = 64, 64
    sc = scenegen.scene_2d(300, W, H, seed=51)
    pre = orc.preprocess_2d(sc.means2d, sc.cov2d, W, H)
    ranges, ids = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, H)
    out = orc.render(W, H, ranges, ids, sc.means2d, pre["conics"], sc.opacities, sc.rgb,
                     delta_c=1e-2, delta_t=1e-1)
    ys, xs = np.nonzero(out["n_amb"] > 0)
    assert len(ys) > 0
    pix = np.stack([xs, ys], 1)[:50]
    alt, altT = orc.render_alternatives(W, H, ranges, ids, sc.means2d, pre["conics"], sc.opacities,
                                        sc.rgb, pix, delta_c=1e-2, delta_t=1e-1)
    for j, (x, y) in enumerate(pix):
        np.testing.assert_array_equal(alt[j, 0], out["rgb"][:, y, x])
        assert np.any(np.abs(alt[j] - alt[j, :1]).max(axis=1) > 0)  # a flip changes something


def test_emulated_render_quality(orc):
    """E6 analogue at 256x256: FP16 in global coordinates is far from the
    definition, local FP16 (K = 8 layout) is close, split variants closer."""
    W = H = 256
    sc = scenegen.scene_2d(2000, W, H, seed=1001)
    pre = orc.preprocess_2d(sc.means2d, sc.cov2d, W, H)
    ranges, ids = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, H)
    ref = orc.render(W, H, ranges, ids, sc.means2d, pre["conics"], sc.opacities, sc.rgb)["rgb"]

    def psnr(x):
        mse = np.mean((x - ref) ** 2)
        return 10 * np.log10(1.0 / mse) if mse > 0 else np.inf

    p = {m: psnr(orc.render(W, H, ranges, ids, sc.means2d, pre["conics"], sc.opacities, sc.rgb,
                            mode=m)["rgb"]) for m in (1, 2, 3, 4)}
    assert p[1] < 30
    assert p[2] > 50
    assert p[3] > p[2] and p[4] > p[2]


def test_bin_tiles_matches_full_binning(orc):
    """The tile-subset binning used for sampled checks of large frames gives
    exactly the full binning's lists for the listed tiles."""
    W, H = 250, 190
    sc = scenegen.scene_2d(3000, W, H, seed=7)
    pre = orc.preprocess_2d(sc.means2d, sc.cov2d, W, H)
    r_all, i_all = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, H)
    tl = np.array([5, 100, 17, 3, 191, 0])
    r_t, i_t = orc.bin_tiles(sc.means2d, pre["radii"], sc.depths, W, H, tl)
    for j, t in enumerate(tl):
        assert np.array_equal(i_all[r_all[t, 0]:r_all[t, 1]], i_t[r_t[j, 0]:r_t[j, 1]])


def _subsequence(a, b):
    """a is a subsequence of b (same relative order)."""
    it = iter(b.tolist())
    return all(x in it for x in a.tolist())


def test_precise_binning_brute_force(orc):
    """Precise Gaussian-tile intersection: every tile list is an ordered
    subsequence of the 3-sigma list, and it keeps every Gaussian whose raw
    opacity o exp(-q/2) reaches 1/255 at some pixel of the tile (brute force
    over the tile's pixels in FP64), so nothing that can contribute is lost."""
    W, H = 96, 80
    sc = scenegen.scene_2d(300, W, H, seed=61, o_min=0.01, o_max=0.99)
    pre = orc.preprocess_2d(sc.means2d, sc.cov2d, W, H)
    r3, i3 = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, H)
    rp, ip = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, H, conics=pre["conics"],
                            opac=sc.opacities)
    assert 0 < len(ip) < 0.8 * len(i3)
    gx = (W + 15) // 16
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    for t in range(r3.shape[0]):
        full, kept = i3[r3[t, 0]:r3[t, 1]], ip[rp[t, 0]:rp[t, 1]]
        assert _subsequence(kept, full)
        tx, ty = t % gx, t // gx
        px = xs[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16].ravel()
        py = ys[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16].ravel()
        for i in full:
            a, b, c = pre["conics"][i]
            dx, dy = px - sc.means2d[i, 0], py - sc.means2d[i, 1]
            q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
            reaches = np.any(sc.opacities[i] * np.exp(-0.5 * q) >= 1.0 / 255.0)
            if reaches:
                assert i in kept, (t, i)


def test_precise_binning_render_invariant(orc):
    """Dropping the tiles that fail the precise test changes no pixel of the
    FP64 render (the dropped fragments are culled everywhere)."""
    W, H = 256, 256
    sc = scenegen.scene_2d(2000, W, H, seed=1001)
    pre = orc.preprocess_2d(sc.means2d, sc.cov2d, W, H)
    r3, i3 = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, H)
    rp, ip = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, H, conics=pre["conics"],
                            opac=sc.opacities)
    assert len(ip) < len(i3)
    a = orc.render(W, H, r3, i3, sc.means2d, pre["conics"], sc.opacities, sc.rgb)
    b = orc.render(W, H, rp, ip, sc.means2d, pre["conics"], sc.opacities, sc.rgb)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["T"], b["T"])


@pytest.mark.parametrize("sigma,keeps_right", [(3.2, True), (3.1, False)])
def test_precise_binning_closed_form(orc, sigma, keeps_right):
    """Isotropic Gaussian at (8, 8), opacity 0.1: the raw opacity reaches
    1/255 out to radius R = sigma sqrt(2 ln 25.5) = 2.5456 sigma, so the tile
    to its right (x >= 16) is kept iff 8 + R >= 16 (sigma 3.2: R = 8.146;
    3.1: R = 7.891); the diagonal tile (box corner at distance 8 sqrt 2) is
    never kept; the 3-sigma rectangle (r = 10) covers all four tiles."""
    W = H = 48
    mu = np.array([[8.0, 8.0]], np.float32)
    cov = np.array([[sigma * sigma, 0.0, sigma * sigma]], np.float32)
    o = np.array([0.1], np.float32)
    pre = orc.preprocess_2d(mu, cov, W, H)
    assert pre["radii"][0] == 10
    d = np.array([1.0], np.float32)
    r3, _ = orc.bin_splats(mu, pre["radii"], d, W, H)
    rp, _ = orc.bin_splats(mu, pre["radii"], d, W, H, conics=pre["conics"], opac=o)
    n3 = r3[:, 1] - r3[:, 0]
    npr = rp[:, 1] - rp[:, 0]
    assert list(np.nonzero(n3)[0]) == [0, 1, 3, 4]
    expect = [0, 1, 3] if keeps_right else [0]
    assert list(np.nonzero(npr)[0]) == expect
    R = sigma * math.sqrt(2 * math.log(25.5))
    assert (8 + R >= 16) == keeps_right
    assert (orc.tile_slack(8.0, 8.0, pre["conics"][0], 0.1, 1, 0, W, H) >= 0) == keeps_right


def _fd_case(orc, seed=1014, P=200, W=64, bg=(0.2, 0.1, 0.3)):
    sc = scenegen.scene_2d(P, W, W, seed=seed, s_min=1.0, s_max=6.0)
    pre = orc.preprocess_2d(sc.means2d, sc.cov2d, W, W)
    ranges, ids = orc.bin_splats(sc.means2d, pre["radii"], sc.depths, W, W)
    params = dict(means2d=sc.means2d.astype(np.float64), conics=pre["conics"].copy(),
                  opacities=sc.opacities.astype(np.float64), rgb=sc.rgb.astype(np.float64))
    return sc, ranges, ids, params, bg


def test_gradient_matches_finite_differences(orc):
    """P11: the FP64 analytic gradient of L = sum w * C (random w) equals
    central finite differences of the FP64 forward, for parameters whose
    perturbation flips no cull/termination/clamp decision (detected by
    comparing the decision counts and the smoothness of the difference
    quotient at two step sizes)."""
    W = 64
    sc, ranges, ids, params, bg = _fd_case(orc)
    w = np.random.default_rng(3).normal(0, 1, (3, W, W))

    def loss(p):
        out = orc.render(W, W, ranges, ids, p["means2d"], p["conics"], p["opacities"], p["rgb"], bg=bg)
        return float(np.sum(w * out["rgb"])), out

    grads = orc.render_backward(W, W, ranges, ids, params["means2d"], params["conics"],
                                params["opacities"], params["rgb"], w, bg=bg)
    _, nominal = loss(params)
    rng = np.random.default_rng(4)
    used = np.unique(ids)
    checked = 0
    for name, shape in (("means2d", 2), ("conics", 3), ("opacities", 1), ("rgb", 3)):
        for _ in range(25):
            g = int(rng.choice(used))
            k = int(rng.integers(0, shape))
            idx = (g, k) if shape > 1 else (g,)
            val = params[name][idx]
            h = 1e-6 * max(1.0, abs(val))
            fd = []
            ok = True
            for hh in (h, 4 * h):
                vals = []
                for sgn in (1, -1):
                    p2 = {kk: v.copy() for kk, v in params.items()}
                    p2[name][idx] = val + sgn * hh
                    L, out = loss(p2)
                    for key in ("n_contrib", "f_blend", "f_cull", "term"):
                        if not np.array_equal(out[key], nominal[key]):
                            ok = False
                    vals.append(L)
                fd.append((vals[0] - vals[1]) / (2 * hh))
            an = grads[name][idx]
            if not ok or abs(fd[0] - fd[1]) > 1e-5 * max(1.0, abs(fd[0])):
                continue  # a decision or the 0.99 clamp is crossed: not differentiable here
            assert abs(an - fd[0]) <= 1e-5 * max(1.0, abs(fd[0])), (name, idx, an, fd)
            checked += 1
    assert checked >= 60
