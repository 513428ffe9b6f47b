"""Pins of the depth-prior oracle (Sec. 3.4, Step 2; row f4): the least-
squares scale / shift against a library solver and an exact recovery, and
the re-projection filter against homogeneous camera matrices, a plane seen
by two views and planted depth errors."""
import numpy as np
import pytest

from oracle import depth_prior as dp
from synth import scenes


def _pair(W=48, H=40):
    """Two nearby views with different sizes and intrinsics (fx != fy, an
    off-centre principal point), so that no parameter of one view can stand
    in for the other's."""
    v0 = scenes.look_at((0.3, -2.0, 3.0), (0.0, 0.0, 0.0), W, H)
    v1 = scenes.look_at((0.9, -1.7, 3.1), (0.05, 0.0, 0.0), W + 8, H - 4)
    v0.fy, v0.cx = v0.fx * 1.15, v0.cx + 1.7
    v1.fx, v1.cy = v1.fx * 0.9, v1.cy - 2.3
    return [v0, v1]


def _mats(view):
    R = np.asarray(view.R, np.float32).astype(np.float64).reshape(3, 3)
    t = np.asarray(view.t, np.float32).astype(np.float64)
    K = np.array([[np.float32(view.fx), 0, np.float32(view.cx)],
                  [0, np.float32(view.fy), np.float32(view.cy)], [0, 0, 1]], np.float64)
    E = np.eye(4)
    E[:3, :3], E[:3, 3] = R, t
    return K, E


def _plane_depth(view, n=np.array([0.0, 0.0, 1.0]), c=0.0):
    """z-depth of the plane n . X = c along every pixel ray (inf-free: the
    test views see the plane everywhere)."""
    K, E = _mats(view)
    W, H = int(view.width), int(view.height)
    J, I = np.divmod(np.arange(W * H), W)
    rays_c = np.linalg.solve(K, np.stack([I + 0.5, J + 0.5, np.ones(W * H)]))      # z = 1
    Rt = E[:3, :3].T
    cen = -Rt @ E[:3, 3]
    rays_w = Rt @ rays_c
    s = (c - n @ cen) / (n @ rays_w)
    return s                                                            # z-depth (ray z = 1)


def test_scale_shift_recovers_an_exact_affine_prior():
    v = _pair()[0]
    K, E = _mats(v)
    rng = np.random.default_rng(3)
    W, H = int(v.width), int(v.height)
    pix = rng.choice(W * H, 60, replace=False)
    z = rng.uniform(2.0, 6.0, pix.size)
    J, I = np.divmod(pix, W)
    pc = np.linalg.solve(K, np.stack([I + 0.5, J + 0.5, np.ones(pix.size)])) * z
    pw = np.linalg.solve(E[:3, :3], pc - E[:3, 3:4]).T      # exact inverse of the float32 R
    s0, t0 = 1.7, -0.35
    prior = rng.uniform(1.0, 3.0, W * H)
    prior[pix] = (z - t0) / s0
    st, aligned, n = dp.align_scale_shift([prior], pw, [v])
    assert n[0] == pix.size
    np.testing.assert_allclose(st[0], [s0, t0], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(aligned[0][pix], z, rtol=1e-9)


def test_scale_shift_matches_lstsq_on_noisy_pairs():
    """The pairs are found here with homogeneous matrices and solved with
    numpy's least squares."""
    v = _pair()[1]
    K, E = _mats(v)
    W, H = int(v.width), int(v.height)
    rng = np.random.default_rng(4)
    pw = np.stack([rng.uniform(-1.5, 1.5, 400), rng.uniform(-1.5, 1.5, 400), rng.uniform(-0.3, 0.3, 400)], 1)
    prior = rng.uniform(0.5, 4.0, W * H)
    prior[rng.random(W * H) < 0.1] = 0.0                      # pixels without a prior
    st, al, n = dp.align_scale_shift([prior], pw, [v])
    np.testing.assert_array_equal(al[0][prior == 0], 0.0)          # no prior stays no prior
    ph = E @ np.vstack([pw.T, np.ones(len(pw))])
    z = ph[2]
    q = K @ ph[:3]
    u, w = q[0] / q[2], q[1] / q[2]
    ok = (z > 0.2) & (u >= 0) & (u < W) & (w >= 0) & (w < H)
    d = prior[np.floor(w[ok]).astype(int) * W + np.floor(u[ok]).astype(int)]
    m = d > 0
    A = np.stack([d[m], np.ones(m.sum())], 1)
    ref = np.linalg.lstsq(A, z[ok][m], rcond=None)[0]
    assert n[0] == m.sum() > 50
    np.testing.assert_allclose(st[0], ref, rtol=1e-8)


def test_scale_shift_degenerate_cases_keep_identity():
    v = _pair()[0]
    W, H = int(v.width), int(v.height)
    st, al, n = dp.align_scale_shift([np.ones(W * H)], np.zeros((0, 3)), [v])
    np.testing.assert_array_equal(st[0], [1.0, 0.0])
    # every pair has the same prior value: a singular system
    st, _, n = dp.align_scale_shift([np.full(W * H, 2.0)], np.array([[0.0, 0, 0], [0.1, 0.1, 0]]), [v])
    assert n[0] == 2
    np.testing.assert_array_equal(st[0], [1.0, 0.0])


def test_reprojection_error_matches_homogeneous_cameras():
    """E for every reprojected pixel of a tilted plane, recomputed here with
    4x4 camera matrices and pixel lookups."""
    views = _pair()
    n = np.array([0.1, -0.05, 1.0])
    depth = [_plane_depth(v, n, 0.0) for v in views]
    out, frag, errs = dp.reprojection_filter(depth, views, [1, 0], tau=1.0)
    K0, E0 = _mats(views[0])
    K1, E1 = _mats(views[1])
    W, H = int(views[0].width), int(views[0].height)
    W1, H1 = int(views[1].width), int(views[1].height)
    checked = 0
    for p in range(0, W * H, 7):
        j, i = divmod(p, W)
        x0 = np.linalg.solve(K0, [i + 0.5, j + 0.5, 1.0]) * depth[0][p]
        xw = np.linalg.solve(E0, np.append(x0, 1.0))
        y1 = (E1 @ xw)[:3]
        q = K1 @ y1
        qx, qy = q[0] / q[2], q[1] / q[2]
        if not (0 <= qx < W1 and 0 <= qy < H1):
            assert out[0][p] == 0.0
            continue
        du = depth[1][int(np.floor(qy)) * W1 + int(np.floor(qx))]
        y = np.linalg.solve(K1, [qx, qy, 1.0]) * du
        back = (E0 @ np.linalg.solve(E1, np.append(y, 1.0)))[:3]
        pb = K0 @ back
        e = np.hypot(pb[0] / pb[2] - (i + 0.5), pb[1] / pb[2] - (j + 0.5))
        # the oracle inverts the stored rotation by its transpose; float32 R is
        # orthonormal to ~3e-8, worth ~1e-6 px here
        np.testing.assert_allclose(errs[0][p], e, rtol=0, atol=2e-5)
        if abs(e - 1.0) > 1e-4:
            assert (out[0][p] > 0) == (e < 1.0)
        checked += 1
    assert checked > 100


def test_filter_keeps_a_consistent_plane_and_removes_planted_errors():
    views = _pair()
    depth = [_plane_depth(v) for v in views]
    out, _, errs = dp.reprojection_filter(depth, views, [1, 0], tau=1.0)
    seen = np.isfinite(errs[0])
    assert seen.mean() > 0.5
    assert (out[0][seen] > 0).mean() > 0.95            # the plane is consistent across the views
    bad = np.random.default_rng(9).random(depth[0].size) < 0.1
    d2 = [np.where(bad, depth[0] * 1.3, depth[0]), depth[1]]
    out2, _, _ = dp.reprojection_filter(d2, views, [1, 0], tau=1.0)
    assert (out2[0][bad & seen] == 0).mean() > 0.95    # a 30 % depth error is not consistent
    np.testing.assert_array_equal(out2[0][~bad & (out[0] > 0)], depth[0][~bad & (out[0] > 0)])


def test_filter_without_a_nearby_view_keeps_every_prior():
    views = _pair()
    depth = [_plane_depth(v) for v in views]
    depth[0][::5] = 0.0
    out, _, _ = dp.reprojection_filter(depth, views, [-1, -1])
    np.testing.assert_array_equal(out[0], depth[0])


def _axis_pair(W=48, H=40):
    """View 0 at the world origin looking along +z; view 1 three units behind
    it on the same axis.  Pixel (24, 20) of either sits on the optical axis."""
    I3 = np.eye(3, dtype=np.float32)
    v0 = scenes.View(W, H, 40.0, 44.0, 24.5, 20.5, I3, np.zeros(3, np.float32), 0.2)
    v1 = scenes.View(W, H, 36.0, 38.0, 24.5, 20.5, I3, np.array([0, 0, 3], np.float32), 0.2)
    return [v0, v1]


def test_filter_on_the_optical_axis():
    """A point on the shared axis re-projects onto itself (E = 0) when view
    1's depth agrees; when view 1's depth lifts it behind view 0 it is
    removed although it projects back onto the same pixel."""
    views = _axis_pair()
    p = 20 * 48 + 24
    d0 = np.zeros(48 * 40)
    d0[p] = 2.0
    for du, kept in ((5.0, True), (1.0, False), (0.0, False)):
        d1 = np.zeros(48 * 40)
        d1[p] = du
        out, frag, errs = dp.reprojection_filter([d0, d1], views, [1, -1])
        assert not frag[0][p]
        assert (out[0][p] == 2.0) == kept
        if kept:
            assert errs[0][p] == 0.0
        np.testing.assert_array_equal(np.delete(out[0], p), 0.0)   # no depth, nothing kept
        assert np.isinf(np.delete(errs[0], p)).all()                # ... and nothing re-projected


def test_filter_on_the_optical_axis_from_behind():
    """The same pair seen from view 1 (three units behind view 0): a point
    behind view 0's near plane, or a missing depth in view 0, removes the
    pixel although the axis would re-project it onto itself."""
    views = _axis_pair()
    p = 20 * 48 + 24
    for d1p, d0p, kept in ((5.0, 2.0, True), (1.0, 2.0, False), (5.0, 0.0, False),
                           (5.0, np.inf, False), (5.0, np.nan, False)):
        d1 = np.zeros(48 * 40)
        d1[p] = d1p
        d0 = np.zeros(48 * 40)
        d0[p] = d0p
        out, frag, _ = dp.reprojection_filter([d0, d1], views, [-1, 0])
        assert not frag[1][p]
        assert (out[1][p] == d1p) == kept, (d1p, d0p)


def test_exact_pixel_edges_are_flagged_fragile():
    """On the shared optical axis with the principal point on the pixel
    grid, the axis pixel re-projects exactly onto a pixel corner of the
    nearby view: flagged fragile; the other pixels are not."""
    I3 = np.eye(3, dtype=np.float32)
    v0 = scenes.View(48, 40, 40.0, 44.0, 24.5, 20.5, I3, np.zeros(3, np.float32), 0.2)
    v1 = scenes.View(48, 40, 36.0, 38.0, 24.0, 20.0, I3, np.array([0, 0, 3], np.float32), 0.2)
    d0 = np.zeros(48 * 40)
    d0[20 * 48 + 24] = 2.0
    d0[5 * 48 + 7] = 2.0
    d1 = np.full(48 * 40, 5.0)
    _, frag, _ = dp.reprojection_filter([d0, d1], [v0, v1], [1, -1])
    assert frag[0][20 * 48 + 24]
    assert frag[0].sum() == 1
