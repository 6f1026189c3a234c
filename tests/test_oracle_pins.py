"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Sampling: de Casteljau (an independent curve algorithm), endpoint
interpolation, linear precision, continuity at composite joints, the paired
closed structure's boundary rows, straight-curve scales in closed form.
Blending: single- and two-Gaussian closed forms, partition of unity of the
compositing weights, zero opacity, transmittance bounds and monotonicity,
linearity in colours, integer translation equivariance, culled == brute
force, agreement with the untruncated blending sum of Sec. 3.4 within the
truncation bound.  Backward: central finite differences in float64 through
the oracle's own forward pass, plus closed-form derivatives.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2503_16424_amd import scenes
from tests.helpers import (closed_boundaries, composite_point, de_casteljau, gauss_set, rel_l2,
                           scene_from_curves, to_f64)

EXACT = dict(rho=2.0, sigma0_sq=0.0)


def _open(ctrl, K, width=1.5, color=(0.2, 0.5, 0.8), opacity=0.7, S=None):
    ctrl = np.asarray(ctrl, np.float64)
    S = S if S is not None else (len(ctrl) - 1) // 3
    return dict(kind=0, S=S, K=K, ctrl=ctrl, width=width, color=color, opacity=opacity)


def _closed(A, Bint, K, R, color=(0.9, 0.3, 0.1), opacity=0.6, tau=None):
    c = dict(kind=1, S=(len(A) - 1) // 3, K=K, R=R, ctrl=np.concatenate([A, Bint]),
             color=color, opacity=opacity)
    if tau is not None:
        c["tau"] = tau
    return c


# --------------------------------------------------------------------------
# Sampling (Sec. 3.3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("S,K", [(1, 2), (1, 16), (2, 9), (3, 24), (3, 7)])
def test_sample_points_match_de_casteljau(S, K):
    rng = np.random.default_rng(100 + S * 31 + K)
    P = rng.uniform(0, 500, (3 * S + 1, 2))
    sc = scene_from_curves(512, 512, [_open(P, K, S=S)])
    g = oracle.sample(sc, EXACT)
    assert g["mu"].shape == (K, 2)
    for k in range(K):
        X, _ = composite_point(P, S, k, K)
        np.testing.assert_allclose(g["mu"][k], X, rtol=0, atol=1e-11)
    # endpoint interpolation
    np.testing.assert_array_equal(g["mu"][0], P[0])
    np.testing.assert_allclose(g["mu"][-1], P[-1], rtol=0, atol=1e-12)


def test_linear_precision():
    """Collinear, equally spaced control points reproduce the straight segment."""
    S, K = 3, 13
    P0, P1 = np.array([3.0, 7.0]), np.array([40.0, 22.0])
    P = np.array([P0 + (j / (3 * S)) * (P1 - P0) for j in range(3 * S + 1)])
    sc = scene_from_curves(64, 64, [_open(P, K, S=S)])
    g = oracle.sample(sc, EXACT)
    for k in range(K):
        np.testing.assert_allclose(g["mu"][k], P0 + (k / (K - 1)) * (P1 - P0), atol=1e-12)


def test_continuity_at_joints():
    """Samples that land on a joint equal the shared control point."""
    S, K = 3, 7                                   # u = 1/3, 2/3 are columns 2, 4
    P = np.random.default_rng(5).uniform(0, 100, (10, 2))
    g = oracle.sample(scene_from_curves(128, 128, [_open(P, K, S=S)]), EXACT)
    np.testing.assert_allclose(g["mu"][2], P[3], atol=1e-12)
    np.testing.assert_allclose(g["mu"][4], P[6], atol=1e-12)


def test_per_segment_opacity_slots():
    S, K = 3, 7
    P = np.random.default_rng(6).uniform(0, 100, (10, 2))
    sc = scene_from_curves(128, 128, [_open(P, K, S=S, opacity=[0.1, 0.5, 0.9])])
    g = oracle.sample(sc, EXACT)
    want = [composite_point(P, S, k, K)[1] for k in range(K)]
    assert list(g["slot"]) == want == [0, 0, 1, 1, 2, 2, 2]
    np.testing.assert_array_equal(g["opac"], np.array([0.1, 0.5, 0.9])[want])


@pytest.mark.parametrize("R,K", [(0, 5), (3, 8), (20, 24)])
def test_closed_rows(R, K):
    """Rows 0 and R+1 are the two boundaries, all rows share the endpoints,
    and row r is the tau_r blend of the boundary samples (linearity)."""
    rng = np.random.default_rng(R * 7 + K)
    A = rng.uniform(0, 200, (4, 2))
    Bint = rng.uniform(0, 200, (2, 2))
    tau = scenes.cdf_tau(R).astype(np.float64)
    sc = scene_from_curves(256, 256, [_closed(A, Bint, K, R, tau=tau)])
    g = oracle.sample(sc, EXACT)
    Afull, Bfull = closed_boundaries(sc.ctrl, 1)
    mu = g["mu"].reshape(R + 2, K, 2)
    for k in range(K):
        XA = de_casteljau(Afull, k / (K - 1))
        XB = de_casteljau(Bfull, k / (K - 1))
        np.testing.assert_allclose(mu[0, k], XA, atol=1e-11)
        np.testing.assert_allclose(mu[R + 1, k], XB, atol=1e-11)
        for r in range(R + 2):
            np.testing.assert_allclose(mu[r, k], (1 - tau[r]) * XA + tau[r] * XB, atol=1e-11)
    np.testing.assert_allclose(mu[:, 0], np.broadcast_to(A[0], (R + 2, 2)), atol=1e-12)
    np.testing.assert_allclose(mu[:, -1], np.broadcast_to(A[3], (R + 2, 2)), atol=1e-12)
    assert np.all(g["row"].reshape(R + 2, K) == np.arange(R + 2)[:, None])


def test_cdf_tau_table():
    """Interior rows are denser near both boundaries; endpoints are 0 and 1."""
    t = scenes.cdf_tau(20).astype(np.float64)
    assert t[0] == 0.0 and t[-1] == 1.0 and np.all(np.diff(t) > 0)
    gaps = np.diff(t)
    assert gaps[0] < gaps[10] and gaps[-1] < gaps[10]
    np.testing.assert_allclose(t + t[::-1], 1.0, atol=1e-6)       # symmetric


def test_straight_stroke_scales():
    """Straight, evenly parametrised stroke: sigma_x = |P3-P0| / ((K-1) rho) at
    every sample, tangent along the stroke, sigma_y = width; horizontal
    stroke => Sigma^-1 = diag(1/sx^2, 1/sy^2)."""
    K, rho, w = 9, 2.0, 1.7
    P = np.array([[10.0, 20.0], [20.0, 20.0], [30.0, 20.0], [40.0, 20.0]])
    g = oracle.sample(scene_from_curves(64, 64, [_open(P, K, width=w)]), dict(rho=rho, sigma0_sq=0.0))
    sx = 30.0 / ((K - 1) * rho)
    np.testing.assert_allclose(g["sx2"], sx * sx, rtol=1e-13)
    np.testing.assert_allclose(g["sy2"], w * w, rtol=1e-13)
    np.testing.assert_allclose(g["tangent"], np.tile([1.0, 0.0], (K, 1)), atol=1e-15)
    np.testing.assert_allclose(g["conic"], np.tile([1 / sx**2, 0.0, 1 / w**2], (K, 1)), rtol=1e-13,
                               atol=1e-15)


def test_diagonal_stroke_covariance_axes():
    """45-degree stroke: the along-stroke direction is an eigenvector of Sigma
    with eigenvalue sigma_x^2 (+ dilation), the normal one with sigma_y^2."""
    K, rho, w, s0 = 6, 2.0, 0.8, 0.3
    P = np.array([[5.0, 5.0], [15.0, 15.0], [25.0, 25.0], [35.0, 35.0]])
    g = oracle.sample(scene_from_curves(64, 64, [_open(P, K, width=w)]), dict(rho=rho, sigma0_sq=s0))
    e = np.array([1.0, 1.0]) / math.sqrt(2)
    nrm = np.array([-1.0, 1.0]) / math.sqrt(2)
    sx2 = (30.0 * math.sqrt(2) / ((K - 1) * rho)) ** 2 + s0
    for q in g["conic"]:
        Sigma = np.linalg.inv(np.array([[q[0], q[1]], [q[1], q[2]]]))
        np.testing.assert_allclose(Sigma @ e, sx2 * e, rtol=1e-12)
        np.testing.assert_allclose(Sigma @ nrm, (w * w + s0) * nrm, rtol=1e-12)


def test_conic_inverts_rotated_scales():
    """Sigma = (R S)(R S)^T built here from de Casteljau neighbours and atan2
    (Eq. sigma, Eq. rotation, Eq. RSSR) times the oracle's conic is I."""
    rng = np.random.default_rng(9)
    rho, s0 = 2.0, 0.3
    curves = []
    for _ in range(3):
        A = rng.uniform(0, 100, (4, 2))
        curves.append(_closed(A, rng.uniform(0, 100, (2, 2)), 7, 2))
    curves.append(_open(rng.uniform(0, 100, (10, 2)), 11, width=2.5, S=3))
    sc = scene_from_curves(128, 128, curves)
    g = oracle.sample(sc, dict(rho=rho, sigma0_sq=s0))
    gi = 0
    for c_i, c in enumerate(curves):
        K = c["K"]
        if c["kind"] == 1:
            Afull, Bfull = closed_boundaries(c["ctrl"], 1)
            tau = scenes.cdf_tau(c["R"]).astype(np.float64)
            rowsP = [(1 - t) * Afull + t * Bfull for t in tau]
        else:
            rowsP = [c["ctrl"]]
        S = c["S"]
        X = np.array([[composite_point(Pr, S, k, K)[0] for k in range(K)] for Pr in rowsP])
        for r in range(len(rowsP)):
            for k in range(K):
                d = X[r, k + 1] - X[r, k] if k < K - 1 else X[r, K - 1] - X[r, K - 2]
                sx2 = d @ d / rho**2 + s0
                if c["kind"] == 1:
                    dy = X[r + 1, k] - X[r, k] if r < len(rowsP) - 1 else X[r, k] - X[r - 1, k]
                    sy2 = dy @ dy / rho**2 + s0
                else:
                    sy2 = c["width"] ** 2 + s0
                v = X[r, min(k + 1, K - 1)] - X[r, max(k - 1, 0)]
                th = math.atan2(v[1], v[0])
                Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
                Sm = np.diag([math.sqrt(sx2), math.sqrt(sy2)])
                Sigma = (Rm @ Sm) @ (Rm @ Sm).T
                q = g["conic"][gi]
                Q = np.array([[q[0], q[1]], [q[1], q[2]]])
                np.testing.assert_allclose(Q @ Sigma, np.eye(2), atol=1e-10)
                np.testing.assert_allclose(g["mu"][gi], X[r, k], atol=1e-10)
                gi += 1
    assert gi == g["mu"].shape[0]


def test_draw_order_follows_rank():
    sc = to_f64(scenes.small_mixed(3))
    g = oracle.sample(sc)
    order = np.argsort(sc.rank, kind="stable")
    seen = []
    for c in g["curve"]:
        if not seen or seen[-1] != c:
            seen.append(int(c))
    assert seen == list(order)


def test_translation_moves_means_only():
    sc = to_f64(scenes.small_mixed(4))
    g0 = oracle.sample(sc)
    sc2 = sc.copy()
    sc2.ctrl = sc.ctrl + np.array([17.0, -5.0])
    g1 = oracle.sample(sc2)
    np.testing.assert_allclose(g1["mu"], g0["mu"] + np.array([17.0, -5.0]), atol=1e-10)
    np.testing.assert_allclose(g1["conic"], g0["conic"], rtol=1e-8, atol=1e-12)


# --------------------------------------------------------------------------
# Forward blending (Sec. 3.4)
# --------------------------------------------------------------------------

BG = np.array([1.0, 1.0, 1.0])


def test_single_gaussian_centre_pixel():
    o, c = 0.63, np.array([0.1, 0.4, 0.7])
    g = gauss_set([[5.5, 6.5]], [[1.0, 0.2, 0.5]], [o], [c])
    r = oracle.render(g, 12, 12, BG)
    np.testing.assert_allclose(r["image"][:, 6, 5], o * c + (1 - o) * BG, atol=1e-15)
    assert abs(r["t_final"][6, 5] - (1 - o)) < 1e-15


def test_single_gaussian_profile():
    """Axis-aligned Gaussian: alpha follows exp(-(dx^2/sx^2 + dy^2/sy^2)/2),
    truncated at g_min and renormalised."""
    sx2, sy2, o, gm = 2.0, 0.7, 0.8, 1.0 / 255.0
    c = np.array([0.0, 0.5, 1.0])
    g = gauss_set([[10.5, 10.5]], [[1 / sx2, 0.0, 1 / sy2]], [o], [c])
    r = oracle.render(g, 21, 21, BG)
    for dx in range(-6, 7):
        for dy in range(-4, 5):
            G = math.exp(-0.5 * (dx * dx / sx2 + dy * dy / sy2))
            a = o * max(G - gm, 0.0) / (1 - gm)
            np.testing.assert_allclose(r["image"][:, 10 + dy, 10 + dx], a * c + (1 - a) * BG,
                                       atol=1e-14)


def test_two_gaussians_composite():
    o1, o2 = 0.5, 0.3
    c1, c2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])
    bg = np.array([0.2, 0.2, 0.2])
    g = gauss_set([[3.5, 3.5], [3.5, 3.5]], [[1, 0, 1], [2, 0.3, 1]], [o1, o2], [c1, c2])
    r = oracle.render(g, 8, 8, bg)
    want = c1 * o1 + c2 * o2 * (1 - o1) + bg * (1 - o1) * (1 - o2)
    np.testing.assert_allclose(r["image"][:, 3, 3], want, atol=1e-15)


def test_weights_sum_to_one():
    sc = to_f64(scenes.small_mixed(11))
    sc.color[:] = 1.0
    r = oracle.forward_backward(sc)
    np.testing.assert_allclose(r["image"], 1.0, atol=1e-12)


def test_zero_opacity_is_background_exactly():
    sc = to_f64(scenes.small_mixed(12))
    sc.opacity[:] = 0.0
    sc.bg = np.array([0.3, 0.6, 0.9])
    r = oracle.forward_backward(sc)
    assert np.all(r["image"] == sc.bg[:, None, None])
    assert np.all(r["t_final"] == 1.0)


def test_transmittance_bounds_and_monotone():
    sc = to_f64(scenes.small_mixed(13, n_closed=5, n_open=6))
    order = np.argsort(sc.rank)
    prev = np.ones((sc.height, sc.width))
    for m in range(1, sc.n_curves + 1):
        sub = sc.copy()
        sub.opacity = sub.opacity.copy()
        for i in order[m:]:                       # curves behind the first m: invisible
            sub.opacity[sub.opa_off[i]:sub.opa_off[i + 1]] = 0.0
        r = oracle.forward_backward(sub)
        T = r["t_final"]
        assert np.all(T >= 0.0) and np.all(T <= 1.0)
        assert np.all(T <= prev + 1e-15)
        prev = T


def test_termination_threshold():
    """Opaque stack: a pixel stops right after T falls below T_min."""
    n = 12
    g = gauss_set(np.tile([[2.5, 2.5]], (n, 1)), np.tile([[0.5, 0, 0.5]], (n, 1)), [0.8] * n,
                  np.tile([[0.3, 0.3, 0.3]], (n, 1)))
    r = oracle.render(g, 5, 5, BG, dict(t_min=1e-6))
    # alpha = 0.8 at the centre: T = 0.2^k, 0.2^8 = 2.56e-6, 0.2^9 = 5.12e-7
    assert r["n_contrib"][2, 2] == 9
    assert r["t_final"][2, 2] < 1e-6
    assert r["n_contrib"][2, 1] > 9                  # dimmer neighbour goes deeper


def test_image_affine_in_colours():
    sc = to_f64(scenes.small_mixed(14))
    rng = np.random.default_rng(1)
    ca, cb = rng.uniform(0, 1, sc.color.shape), rng.uniform(0, 1, sc.color.shape)
    lam = 0.3
    imgs = []
    for col in (ca, cb, lam * ca + (1 - lam) * cb):
        s2 = sc.copy()
        s2.color = col
        imgs.append(oracle.forward_backward(s2)["image"])
    np.testing.assert_allclose(imgs[2], lam * imgs[0] + (1 - lam) * imgs[1], atol=1e-13)


def test_integer_translation_equivariance():
    sc = to_f64(scenes.small_mixed(15, W=64, H=64, extent=(6.0, 14.0)))
    sc.ctrl = 20.0 + (sc.ctrl - 20.0) * 0.5       # keep everything well inside
    r0 = oracle.forward_backward(sc)["image"]
    s2 = sc.copy()
    s2.ctrl = sc.ctrl + np.array([7.0, 4.0])
    r1 = oracle.forward_backward(s2)["image"]
    np.testing.assert_allclose(r1[:, 4:, 7:], r0[:, :-4, :-7], atol=1e-12)


def test_culled_equals_brute_force():
    sc = to_f64(scenes.small_mixed(16))
    g = oracle.sample(sc)
    a = oracle.render(g, sc.width, sc.height, sc.bg)
    b = oracle.render(g, sc.width, sc.height, sc.bg, brute=True)
    assert np.array_equal(a["image"], b["image"])
    assert np.array_equal(a["n_contrib"], b["n_contrib"])


def _paper_blend(g, W, H, bg):
    """The blending sum of Sec. 3.4 with alpha = o exp(-1/2 d^T Sigma^-1 d),
    untruncated and unclamped, summed over every Gaussian."""
    img = np.zeros((3, H, W))
    ys, xs = np.mgrid[0:H, 0:W]
    qx, qy = xs + 0.5, ys + 0.5
    T = np.ones((H, W))
    for i in range(g["mu"].shape[0]):
        dx, dy = qx - g["mu"][i, 0], qy - g["mu"][i, 1]
        Q = g["conic"][i]
        a = g["opac"][i] * np.exp(-0.5 * (Q[0] * dx * dx + 2 * Q[1] * dx * dy + Q[2] * dy * dy))
        img += g["color"][i][:, None, None] * (a * T)[None]
        T = T * (1 - a)
    return img + bg[:, None, None] * T[None]


def test_untruncated_limit_matches_paper_blending():
    sc = to_f64(scenes.small_mixed(17, W=24, H=20, n_closed=2, n_open=2, K=6, R=2))
    g = oracle.sample(sc)
    want = _paper_blend(g, sc.width, sc.height, sc.bg)
    exact = oracle.render(g, sc.width, sc.height, sc.bg, dict(g_min=1e-15, alpha_max=1.0, t_min=0.0))
    np.testing.assert_allclose(exact["image"], want, atol=1e-12)
    # default truncation: |alpha~ - alpha| <= o g_min/(1-g_min) per Gaussian,
    # |dC/dalpha| <= 1, plus at most T_min from stopping early
    gm = oracle.DEFAULTS["g_min"]
    bound = g["opac"].sum() * gm / (1 - gm) + oracle.DEFAULTS["t_min"]
    trunc = oracle.render(g, sc.width, sc.height, sc.bg, dict(alpha_max=1.0))
    assert np.abs(trunc["image"] - want).max() <= bound


# --------------------------------------------------------------------------
# Backward
# --------------------------------------------------------------------------

NOSTOP = dict(t_min=0.0)


def _loss_gauss(g, W, H, bg, dimg, opts):
    return float((oracle.render(g, W, H, bg, opts)["image"] * dimg).sum())


def test_per_gaussian_gradients_finite_difference():
    rng = np.random.default_rng(21)
    n, W, H = 6, 14, 12
    mu = rng.uniform(2, 12, (n, 2))
    conic = []
    for _ in range(n):
        th, sx2, sy2 = rng.uniform(0, math.pi), rng.uniform(0.5, 6), rng.uniform(0.5, 6)
        c, s = math.cos(th), math.sin(th)
        conic.append([c * c / sx2 + s * s / sy2, c * s * (1 / sx2 - 1 / sy2), s * s / sx2 + c * c / sy2])
    g = gauss_set(mu, conic, rng.uniform(0.3, 0.9, n), rng.uniform(0, 1, (n, 3)))
    bg = np.array([0.9, 0.8, 0.7])
    dimg = rng.normal(size=(3, H, W))
    r = oracle.render(g, W, H, bg, NOSTOP, d_image=dimg)
    an = r["d_gauss"]
    num = np.zeros_like(an)
    for i in range(n):
        for j, (key, idx, h) in enumerate([("mu", 0, 1e-6), ("mu", 1, 1e-6), ("conic", 0, 1e-7),
                                          ("conic", 1, 1e-7), ("conic", 2, 1e-7), ("opac", None, 1e-7),
                                          ("color", 0, 1e-6), ("color", 1, 1e-6), ("color", 2, 1e-6)]):
            gp = {k: v.copy() for k, v in g.items()}
            gm = {k: v.copy() for k, v in g.items()}
            if idx is None:
                gp[key][i] += h
                gm[key][i] -= h
            else:
                gp[key][i, idx] += h
                gm[key][i, idx] -= h
            num[i, j] = (_loss_gauss(gp, W, H, bg, dimg, NOSTOP) -
                         _loss_gauss(gm, W, H, bg, dimg, NOSTOP)) / (2 * h)
    assert rel_l2(an, num) < 1e-6
    np.testing.assert_allclose(an, num, rtol=1e-4, atol=1e-7)


def _loss_scene(sc, dimg, opts):
    return float((oracle.forward_backward(sc, opts=opts)["image"] * dimg).sum())


@pytest.mark.parametrize("seed", [31, 32])
def test_curve_gradients_finite_difference(seed):
    sc = to_f64(scenes.small_mixed(seed, W=40, H=36, n_closed=2, n_open=3, K=7, R=3,
                                   extent=(8.0, 26.0)))
    sc.opacity = np.minimum(sc.opacity, 0.9)      # never clamped
    dimg = np.random.default_rng(seed).normal(size=(3, sc.height, sc.width))
    an = oracle.forward_backward(sc, dimg, NOSTOP)

    def fd(attr, idx, h):
        sp, sm = sc.copy(), sc.copy()
        getattr(sp, attr)[idx] += h
        getattr(sm, attr)[idx] -= h
        return (_loss_scene(sp, dimg, NOSTOP) - _loss_scene(sm, dimg, NOSTOP)) / (2 * h)

    num_ctrl = np.array([[fd("ctrl", (i, j), 1e-6) for j in range(2)] for i in range(sc.ctrl.shape[0])])
    num_w = np.array([fd("stroke_w", i, 1e-6) for i in range(sc.n_curves)])
    num_c = np.array([[fd("color", (i, j), 1e-6) for j in range(3)] for i in range(sc.n_curves)])
    num_o = np.array([fd("opacity", i, 1e-7) for i in range(sc.opacity.shape[0])])
    assert rel_l2(an["d_ctrl"], num_ctrl) < 1e-6
    assert rel_l2(an["d_width"], num_w) < 1e-6
    assert rel_l2(an["d_color"], num_c) < 1e-7
    assert rel_l2(an["d_opacity"], num_o) < 1e-6
    closed = sc.kind == 1
    assert np.all(an["d_width"][closed] == 0.0)


def test_colour_gradient_is_blend_weight():
    sc = to_f64(scenes.small_mixed(41))
    x, y = 20, 18
    for ch in range(3):
        dimg = np.zeros((3, sc.height, sc.width))
        dimg[ch, y, x] = 1.0
        r = oracle.forward_backward(sc, dimg)
        w = r["d_gauss"][:, 6 + ch]
        assert np.all(r["d_gauss"][:, 6 + (ch + 1) % 3] == 0.0)
        np.testing.assert_allclose(w.sum() + r["t_final"][y, x], 1.0, atol=1e-13)


def test_single_gaussian_opacity_gradient_closed_form():
    o, c, bg, gm = 0.4, np.array([0.2, 0.9, 0.5]), np.array([1.0, 0.5, 0.0]), 1.0 / 255.0
    g = gauss_set([[4.2, 3.9]], [[0.6, 0.1, 0.9]], [o], [c])
    dimg = np.zeros((3, 8, 8))
    dimg[:, 3, 5] = [1.0, -2.0, 0.5]
    r = oracle.render(g, 8, 8, bg, d_image=dimg)
    dx, dy = 5.5 - 4.2, 3.5 - 3.9
    G = math.exp(-0.5 * (0.6 * dx * dx + 0.2 * dx * dy + 0.9 * dy * dy))
    Gt = (G - gm) / (1 - gm)
    np.testing.assert_allclose(r["d_gauss"][0, 5], Gt * ((c - bg) @ dimg[:, 3, 5]), rtol=1e-13)


def test_zero_opacity_curve_still_gets_gradient():
    sc = to_f64(scenes.small_mixed(42))
    i = int(np.argmin(sc.rank))                      # the front curve
    sc.opacity[sc.opa_off[i]:sc.opa_off[i + 1]] = 0.0
    dimg = np.random.default_rng(2).normal(size=(3, sc.height, sc.width))
    r = oracle.forward_backward(sc, dimg)
    assert np.abs(r["d_opacity"][sc.opa_off[i]:sc.opa_off[i + 1]]).sum() > 0.0


def test_clamped_alpha_has_no_opacity_or_shape_gradient():
    g = gauss_set([[2.5, 2.5]], [[0.5, 0.0, 0.5]], [1.0], [[0.2, 0.2, 0.2]])
    dimg = np.zeros((3, 5, 5))
    dimg[:, 2, 2] = 1.0
    r = oracle.render(g, 5, 5, BG, d_image=dimg)
    assert np.all(r["d_gauss"][0, :6] == 0.0)       # alpha = alpha_max there
    np.testing.assert_allclose(r["d_gauss"][0, 6:], 0.99, atol=1e-15)


def test_sampled_pixels_match_full_render():
    sc = to_f64(scenes.small_mixed(43))
    r = oracle.forward_backward(sc)
    xs = np.array([0, 5, 17, 30, 47])
    ys = np.array([0, 9, 20, 33, 39])
    p = oracle.render_pixels(r["gauss"], sc.width, sc.height, sc.bg, xs, ys)
    np.testing.assert_array_equal(p["rgb"], r["image"][:, ys, xs].T)
    np.testing.assert_array_equal(p["n_contrib"], r["n_contrib"][ys, xs])


def test_rejects_bad_scenes():
    sc = to_f64(scenes.small_mixed(44))
    bad = sc.copy()
    bad.rank = np.zeros_like(sc.rank)               # not a permutation
    with pytest.raises(ValueError):
        oracle.sample(bad)
    bad = sc.copy()
    bad.k_samples = sc.k_samples.copy()
    bad.k_samples[0] = 1                             # K >= 2 is required
    with pytest.raises(ValueError):
        oracle.sample(bad)


# --- decision margins and tile depth (the parity report's diagnostics) -------

def test_margin_is_the_threshold_shift_that_flips_the_support_test():
    """One Gaussian, no clamp (alpha_max = 1 > every raw alpha) and no stop
    (t_min = 0): a pixel's only binding decision is the support test G > g_min.
    Moving g_min by 1.01x the reported margin towards G flips the pixel's
    contribution; by 0.99x it does not."""
    W, H = 40, 32
    g = gauss_set([20.3, 15.7], [0.05, 0.012, 0.11], [0.5], [0.2, 0.4, 0.6])
    base = dict(t_min=0.0, alpha_max=1.0)
    gm = oracle.DEFAULTS["g_min"]
    r = oracle.render(g, W, H, (1.0, 1.0, 1.0), opts=dict(base, g_min=gm))
    m, inside = r["margin"], r["n_contrib"] > 0
    sel = np.argwhere((m < 0.4) & (m > 1e-9))
    assert len(sel) > 40, "too few pixels near the support boundary"
    for s in (0.99, 1.01):
        for y, x in sel[:: max(1, len(sel) // 40)]:
            # G = gm (1 + m) inside, gm (1 - m) outside: shift g_min towards it
            gm2 = gm * (1.0 + s * m[y, x]) if inside[y, x] else gm * (1.0 - s * m[y, x])
            r2 = oracle.render(g, W, H, (1.0, 1.0, 1.0), opts=dict(base, g_min=gm2),
                               rows=(int(y), int(y) + 1))
            flipped = (r2["n_contrib"][y, x] > 0) != inside[y, x]
            assert flipped == (s > 1.0), (y, x, m[y, x], s)


def test_margin_is_zero_at_a_threshold_and_positive_elsewhere():
    """A pixel whose G equals g_min to rounding has margin ~0; the margin is
    never negative and infinite only where no Gaussian was evaluated."""
    gm = oracle.DEFAULTS["g_min"]
    # isotropic Gaussian, Q = I / s2, pixel (0, 0) at d = (0.5 - mx, 0.5 - my):
    # put it on the support boundary 1/2 |d|^2 / s2 = -ln gm
    s2 = 4.0
    r0 = math.sqrt(-2.0 * s2 * math.log(gm))
    mx, my = 0.5 + r0 / math.sqrt(2.0), 0.5 + r0 / math.sqrt(2.0)
    g = gauss_set([mx, my], [1.0 / s2, 0.0, 1.0 / s2], [0.5], [0.1, 0.1, 0.1])
    r = oracle.render(g, 32, 32, (1.0, 1.0, 1.0), opts=dict(t_min=0.0, alpha_max=1.0))
    assert r["margin"][0, 0] < 1e-12
    assert np.all(r["margin"][np.isfinite(r["margin"])] >= 0.0)
    assert np.all(r["margin"][1:, 1:] > 0.0)


def test_tile_depth_equals_brute_force_counts():
    """Without early stops every Gaussian with G > g_min at a pixel contributes
    there, so a tile's contributing-curve count is the number of curves with
    such a Gaussian at one of its pixels (brute force in numpy); the
    reaching-curve count lies between that and the curves whose Gaussians'
    support boxes (the exact ellipse's extent, padded by 2 px) meet the tile."""
    sc = to_f64(scenes.small_mixed(21, W=56, H=40, n_closed=4, n_open=6, K=8, R=3))
    g = oracle.sample(sc)
    W, H, tw, th = sc.width, sc.height, 16, 8
    opts = dict(t_min=0.0)
    d = oracle.tile_depth(g, sc.n_curves, W, H, (tw, th), opts=opts)
    gm = oracle.DEFAULTS["g_min"]
    ys, xs = np.mgrid[0:H, 0:W]
    px, py = xs.ravel() + 0.5, ys.ravel() + 0.5
    dx = px[None, :] - g["mu"][:, 0:1]
    dy = py[None, :] - g["mu"][:, 1:2]
    q = g["conic"]
    G = np.exp(-0.5 * (q[:, 0:1] * dx * dx + 2 * q[:, 1:2] * dx * dy + q[:, 2:3] * dy * dy))
    hit = G > gm                                       # [gauss, pixel]
    tile_of_px = (ys.ravel() // th) * (-(-W // tw)) + xs.ravel() // tw
    nt = (-(-W // tw)) * (-(-H // th))
    det = q[:, 0] * q[:, 2] - q[:, 1] ** 2
    hx = np.sqrt(-2 * math.log(gm) * q[:, 2] / det) + 2.0
    hy = np.sqrt(-2 * math.log(gm) * q[:, 0] / det) + 2.0
    for t in range(nt):
        cols = tile_of_px == t
        gs = np.nonzero(hit[:, cols].any(axis=1))[0]
        want = len(set(g["curve"][gs].tolist()))
        assert d["contrib"][t] == want, (t, d["contrib"][t], want)
        ty, tx = divmod(t, -(-W // tw))
        x0, x1, y0, y1 = tx * tw, min(W, tx * tw + tw), ty * th, min(H, ty * th + th)
        near = (g["mu"][:, 0] + hx > x0) & (g["mu"][:, 0] - hx < x1) & \
               (g["mu"][:, 1] + hy > y0) & (g["mu"][:, 1] - hy < y1)
        upper = len(set(g["curve"][near].tolist()))
        assert want <= d["support"][t] <= upper, (t, want, d["support"][t], upper)
    # with the paper's stop, no tile gains contributors
    d2 = oracle.tile_depth(g, sc.n_curves, W, H, (tw, th))
    assert np.all(d2["contrib"] <= d["contrib"])
