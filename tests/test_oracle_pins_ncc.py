"""Pins of the Eq. 10 oracle (batch geometric NCC loss) to facts that do not
come from the oracle itself: the homography against explicit ray-plane
intersection, bilinear sampling against affine images, NCC's invariances
and bounds, and the gradient against finite differences."""
import numpy as np

from oracle import ncc
from oracle.project import view_arrays
from synth import scenes


def _view(R, t, w=40, h=30, f=35.0):
    return scenes.View(width=w, height=h, fx=f, fy=f * 1.1, cx=w / 2 + 0.3, cy=h / 2 - 0.2,
                       R=np.asarray(R, np.float32), t=np.asarray(t, np.float32))


def _rot(ax, ang):
    ax = np.asarray(ax, float) / np.linalg.norm(ax)
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


def test_homography_matches_ray_plane_intersection():
    rng = np.random.default_rng(0)
    vr = view_arrays(_view(_rot([0.2, 1, 0.1], 0.3), [0.1, -0.2, 0.5]))
    vs = view_arrays(_view(_rot([1, 0.3, -0.2], -0.25), [-0.4, 0.1, 0.3]))
    n = np.array([0.1, -0.2, -1.0])
    d = 4.0                                   # plane n . X = -d in the reference frame
    H = ncc.homography(vr, vs, n, d)
    for _ in range(20):
        u, v = rng.uniform(0, 40), rng.uniform(0, 30)
        ray = np.array([(u - vr["cx"]) / vr["fx"], (v - vr["cy"]) / vr["fy"], 1.0])
        lam = -d / (n @ ray)
        X_r = lam * ray
        assert abs(n @ X_r + d) < 1e-9
        X_w = vr["R"].T @ (X_r - vr["t"])
        X_s = vs["R"] @ X_w + vs["t"]
        us = vs["fx"] * X_s[0] / X_s[2] + vs["cx"]
        ws = vs["fy"] * X_s[1] / X_s[2] + vs["cy"]
        q = H @ np.array([u, v, 1.0])
        np.testing.assert_allclose([q[0] / q[2], q[1] / q[2]], [us, ws], rtol=0, atol=1e-9)


def test_bilinear_reproduces_affine_images():
    W, H = 9, 7
    yy, xx = np.mgrid[0:H, 0:W]
    img = (0.3 * xx - 0.7 * yy + 2.0).ravel().astype(np.float64)
    rng = np.random.default_rng(1)
    sx, sy = rng.uniform(0, W - 1, 50), rng.uniform(0, H - 1, 50)
    np.testing.assert_allclose(ncc.bilinear(img, W, H, sx, sy), 0.3 * sx - 0.7 * sy + 2.0, atol=1e-12)
    # at integer positions it returns the pixel, including the last row and column
    np.testing.assert_allclose(ncc.bilinear(img, W, H, np.array([W - 1.0, 0.0]), np.array([H - 1.0, 0.0])),
                               [img[-1], img[0]], atol=1e-12)


def _pair_images(W, H, rng, ref_fn=None):
    """Two views' image dicts: source and reference rgb (3, npx), normal, D."""
    ims = []
    for _ in range(2):
        ims.append(dict(rgb=rng.uniform(0, 1, (3, W * H)), normal=np.tile([[0.0], [0.0], [-1.0]], (1, W * H)),
                        D=np.full(W * H, 5.0)))
    return ims


def test_identity_pair_has_zero_loss_and_ncc_one():
    rng = np.random.default_rng(2)
    v = _view(np.eye(3), [0, 0, 0])
    va = [view_arrays(v), view_arrays(v)]
    ims = _pair_images(40, 30, rng)
    ims[1]["rgb"] = ims[0]["rgb"].copy()
    centres = np.array([[[10, 10], [20, 15], [30, 20]]])
    loss, grads, info = ncc.ncc_loss(ims, va, centres)
    assert info["valid"].all()
    np.testing.assert_allclose(info["ncc"], 1.0, atol=1e-7)
    assert abs(loss) < 1e-7


def test_ncc_affine_invariance_and_sign():
    rng = np.random.default_rng(3)
    v = _view(np.eye(3), [0, 0, 0])
    va = [view_arrays(v), view_arrays(v)]
    ims = _pair_images(40, 30, rng)
    g = ims[0]["rgb"]
    for alpha, beta, expect in ((2.5, 0.1, 1.0), (-0.7, 0.9, -1.0)):
        ims[1]["rgb"] = alpha * g + beta
        _, _, info = ncc.ncc_loss(ims, va, np.array([[[12, 12], [25, 14]]]))
        np.testing.assert_allclose(info["ncc"], expect, atol=1e-6)


def test_invalid_patches_add_nothing():
    rng = np.random.default_rng(4)
    v = _view(np.eye(3), [0, 0, 0])
    va = [view_arrays(v), view_arrays(v)]
    ims = _pair_images(40, 30, rng)
    # touching the border, and a non-positive plane distance at the centre
    ims[1]["D"][15 * 40 + 20] = 0.0
    loss, grads, info = ncc.ncc_loss(ims, va, np.array([[[1, 10], [20, 15], [38, 28]]]))
    assert not info["valid"].any() and loss == 0.0 and not grads[1].any()


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    vs = _view(np.eye(3), [0, 0, 0], w=48, h=40)
    vr = _view(_rot([0, 1, 0], 0.05), [-0.1, 0.02, 0.0], w=48, h=40)
    va = [view_arrays(vs), view_arrays(vr)]
    ims = _pair_images(48, 40, rng)
    ims[1]["rgb"] = rng.uniform(0, 1, (3, 48 * 40))
    centres = np.array([[[20, 18], [24, 20], [15, 25]]])     # overlapping patches
    loss, grads, info = ncc.ncc_loss(ims, va, centres, weight=0.7)
    assert info["valid"].all()
    h = 1e-6
    for c, p in ((0, 18 * 48 + 20), (2, 20 * 48 + 23), (1, 25 * 48 + 15), (1, 19 * 48 + 21)):
        e = ims[1]["rgb"].copy()
        e[c, p] += h
        lp, _, _ = ncc.ncc_loss([ims[0], dict(ims[1], rgb=e)], va, centres, weight=0.7)
        e[c, p] -= 2 * h
        lm, _, _ = ncc.ncc_loss([ims[0], dict(ims[1], rgb=e)], va, centres, weight=0.7)
        np.testing.assert_allclose(grads[1][c, p], (lp - lm) / (2 * h), rtol=1e-5, atol=1e-9)
    assert not grads[0].any()          # stop-gradient on the source view
