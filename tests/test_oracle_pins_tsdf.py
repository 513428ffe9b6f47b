"""Pins of the TSDF fusion oracle (Sec. 4, mesh reconstruction; row f4):
closed forms for a fronto-parallel plane, the zero crossing at the surface,
the running average of two observations, the colour average, occlusion
beyond the truncation, batching independence, and a brute-force per-voxel
loop with homogeneous camera matrices."""
import numpy as np

from oracle import tsdf
from synth import scenes

I3 = np.eye(3, dtype=np.float32)


def _front_view(W=40, H=30, fx=20.0, fy=22.0, t=(0.0, 0.0, 0.0)):
    # camera at -t looking along +z; the principal point is 0.3 px off the
    # pixel grid, so that no grid voxel projects exactly onto a pixel edge
    return scenes.View(W, H, fx, fy, W / 2 + 0.3, H / 2 + 0.3, I3, np.asarray(t, np.float32), 0.2)


def _grid():
    # a block well inside the frustum of _front_view for z in [2, 4.8]:
    # half widths at z = 2 are 2 * 20 / 20 = 2 (x) and 2 * 15 / 22 = 1.36 (y)
    origin, voxel, dims = (-1.0, -0.8, 2.0), 0.1, (21, 17, 29)
    return origin, voxel, dims


def test_voxel_points_order():
    X = tsdf.voxel_points((1.0, 2.0, 3.0), 0.5, (3, 2, 2))
    np.testing.assert_array_equal(X[0], [1.0, 2.0, 3.0])
    np.testing.assert_array_equal(X[1], [1.5, 2.0, 3.0])          # i fastest
    np.testing.assert_array_equal(X[3], [1.0, 2.5, 3.0])          # then j
    np.testing.assert_array_equal(X[6], [1.0, 2.0, 3.5])          # then k


def test_fronto_parallel_plane_closed_form():
    origin, voxel, dims = _grid()
    v = _front_view()
    Z0, mu = 3.3, 0.35
    depth = [np.full(v.width * v.height, Z0)]
    T, Wt, C, frag = tsdf.integrate(origin, voxel, dims, mu, [v], depth)
    z = tsdf.voxel_points(origin, voxel, dims)[:, 2]
    upd = Z0 - z > -mu
    assert not frag.any()
    np.testing.assert_array_equal(Wt, np.where(upd, 1.0, 0.0))
    np.testing.assert_allclose(T, np.where(upd, np.minimum(1.0, (Z0 - z) / mu), 1.0), atol=1e-15)
    assert upd.sum() < upd.size                                      # some voxels are occluded


def test_zero_crossing_is_the_surface():
    origin, voxel, dims = _grid()
    v = _front_view()
    Z0, mu = 3.27, 0.4
    T, Wt, _, _ = tsdf.integrate(origin, voxel, dims, mu, [v], [np.full(v.width * v.height, Z0)])
    nx, ny, nz = dims
    Tc = T.reshape(nz, ny, nx)[:, 7, 9]
    zc = origin[2] + voxel * np.arange(nz)
    k = np.flatnonzero((Tc[:-1] > 0) & (Tc[1:] <= 0))[0]
    zero = zc[k] + voxel * Tc[k] / (Tc[k] - Tc[k + 1])
    np.testing.assert_allclose(zero, Z0, atol=1e-12)


def test_running_average_of_two_observations_and_colour():
    origin, voxel, dims = _grid()
    v = _front_view()
    n = v.width * v.height
    Z1, Z2, mu = 3.03, 3.22, 0.3
    c1, c2 = np.array([0.2, 0.4, 0.9]), np.array([0.6, 0.0, 0.1])
    rgb = [np.repeat(c1[:, None], n, 1), np.repeat(c2[:, None], n, 1)]
    T, Wt, C, _ = tsdf.integrate(origin, voxel, dims, mu, [v, v], [np.full(n, Z1), np.full(n, Z2)], rgb)
    z = tsdf.voxel_points(origin, voxel, dims)[:, 2]
    f1, f2 = np.minimum(1, (Z1 - z) / mu), np.minimum(1, (Z2 - z) / mu)
    both = (Z1 - z > -mu) & (Z2 - z > -mu)
    only2 = ~(Z1 - z > -mu) & (Z2 - z > -mu)
    assert both.any() and only2.any()
    np.testing.assert_allclose(T[both], (f1[both] + f2[both]) / 2, atol=1e-15)
    np.testing.assert_array_equal(Wt[both], 2.0)
    np.testing.assert_allclose(T[only2], f2[only2], atol=1e-15)
    np.testing.assert_array_equal(Wt[only2], 1.0)
    np.testing.assert_allclose(C[:, both], np.repeat(((c1 + c2) / 2)[:, None], both.sum(), 1), atol=1e-15)
    np.testing.assert_allclose(C[:, only2], np.repeat(c2[:, None], only2.sum(), 1), atol=1e-15)


def test_missing_depth_and_outside_voxels_are_untouched():
    origin, voxel, dims = (-4.0, -3.0, -0.9), 0.25, (33, 25, 21)      # behind, beside, inside the near plane
    v = _front_view()
    n = v.width * v.height
    D = np.full(n, 3.0)
    D[::3] = 0.0
    D[1::7] = np.nan
    D[2::11] = np.inf
    T, Wt, _, _ = tsdf.integrate(origin, voxel, dims, 0.3, [v], [D])
    X = tsdf.voxel_points(origin, voxel, dims)
    # projections written out on their own: pixel of each voxel in front
    zf = X[:, 2] > 0.2
    u = 20.0 * X[:, 0] / np.where(zf, X[:, 2], 1) + np.float32(20.3)
    w = 22.0 * X[:, 1] / np.where(zf, X[:, 2], 1) + np.float32(15.3)
    seen = zf & (u >= 0) & (u < 40) & (w >= 0) & (w < 30)
    assert (~seen).any() and seen.any()
    assert (Wt[~seen] == 0).all() and (T[~seen] == 1).all()
    pix = np.floor(w[seen]).astype(int) * 40 + np.floor(u[seen]).astype(int)
    bad = ~(np.isfinite(D[pix]) & (D[pix] > 0))
    assert bad.any()
    assert (Wt[seen][bad] == 0).all()


def test_batching_does_not_matter():
    origin, voxel, dims = _grid()
    views = [_front_view(), _front_view(t=(0.1, -0.05, 0.2)), _front_view(fx=18.0)]
    rng = np.random.default_rng(3)
    depth = [rng.uniform(2.5, 4.0, 1200) for _ in views]
    rgb = [rng.uniform(0, 1, (3, 1200)) for _ in views]
    full = tsdf.integrate(origin, voxel, dims, 0.25, views, depth, rgb)
    a = tsdf.integrate(origin, voxel, dims, 0.25, views[:1], depth[:1], rgb[:1])
    b = tsdf.integrate(origin, voxel, dims, 0.25, views[1:], depth[1:], rgb[1:], state=a[:3])
    for x, y in zip(full[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
    # each voxel is independent: a subset gives the same values
    idx = np.random.default_rng(4).choice(int(np.prod(dims)), 500, replace=False)
    sub = tsdf.integrate(origin, voxel, dims, 0.25, views, depth, rgb, voxels=idx)
    for x, y in zip(full[:2], sub[:2]):
        np.testing.assert_array_equal(x[idx], y)
    np.testing.assert_array_equal(full[2][:, idx], sub[2])


def test_brute_force_with_homogeneous_cameras():
    """Per-voxel loop with 3x4 projection matrices, a tilted camera and a
    random depth map."""
    v = scenes.look_at((0.4, -3.0, 1.5), (0.1, 0.2, 0.3), 24, 18, fov_deg=70.0)
    origin, voxel, dims, mu = (-0.6, -0.5, -0.2), 0.15, (9, 8, 7), 0.3
    rng = np.random.default_rng(8)
    D = rng.uniform(2.0, 4.0, 24 * 18)
    D[::9] = 0.0
    rgb = rng.uniform(0, 1, (3, 24 * 18))
    T, Wt, C, frag = tsdf.integrate(origin, voxel, dims, mu, [v], [D], [rgb])
    R = np.asarray(v.R, np.float32).astype(np.float64)
    t = np.asarray(v.t, np.float32).astype(np.float64)
    K = np.array([[np.float32(v.fx), 0, np.float32(v.cx)], [0, np.float32(v.fy), np.float32(v.cy)], [0, 0, 1]])
    P = K @ np.hstack([R, t[:, None]])
    n = 0
    for k in range(dims[2]):
        for j in range(dims[1]):
            for i in range(dims[0]):
                idx = i + dims[0] * (j + dims[1] * k)
                Xh = np.array([origin[0] + voxel * i, origin[1] + voxel * j, origin[2] + voxel * k, 1.0])
                q = P @ Xh
                z = q[2]
                if frag[idx]:
                    continue
                upd = False
                if z > np.float32(0.2):
                    u, w = q[0] / z, q[1] / z
                    if 0 <= u < 24 and 0 <= w < 18:
                        p = int(np.floor(w)) * 24 + int(np.floor(u))
                        if D[p] > 0 and D[p] - z > -mu:
                            upd = True
                            np.testing.assert_allclose(T[idx], min(1.0, (D[p] - z) / mu), atol=1e-9)
                            np.testing.assert_allclose(C[:, idx], rgb[:, p], atol=1e-12)
                            n += 1
                assert Wt[idx] == (1.0 if upd else 0.0), (i, j, k)
    assert n > 20


def test_exact_pixel_edges_are_flagged_fragile():
    """With the principal point on the pixel grid (cx = 20), voxel
    (i, j, k) at x = (i - 10) / 10, z = (20 + k) / 10 projects to
    u = 20 + 20 (i - 10) / (20 + k), exactly a pixel edge when 20 + k
    divides 20 (i - 10) (integer arithmetic); cy = 15.3 in float32 keeps w
    off the edges.  Exactly those voxels are flagged."""
    origin, voxel, dims = _grid()
    v = scenes.View(40, 30, 20.0, 22.0, 20.0, 15.3, I3, np.zeros(3, np.float32), 0.2)
    _, _, _, frag = tsdf.integrate(origin, voxel, dims, 0.35, [v], [np.full(1200, 3.3)])
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz)
    i, k = idx % nx, idx // (nx * ny)
    edge = (20 * (i - 10)) % (20 + k) == 0
    assert edge.sum() > nx * ny                     # the axis and more
    np.testing.assert_array_equal(frag, edge)
