"""Pins of the oracle's building blocks against library routines and exact
mathematics (CPU only)."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

from oracle import bf16, project, sh


# ---------------------------------------------------------------- bfloat16
def test_bf16_rounding_matches_torch_on_edge_cases():
    rng = np.random.default_rng(0)
    specials = np.array([0.0, -0.0, 1.0, -1.0, 1.00390625, 1.01171875, 1.0078125,
                         3.0e38, -3.0e38, 1e-40, -1e-40, 1.17549435e-38, 5e-45,
                         65504.0, 0.1, -0.3333333], np.float32)
    # every tie pattern in the low 16 bits around a few mantissas
    base = np.array([1.0, 1.5, -2.25, 1e-3, 7.0e20], np.float32).view(np.uint32)
    lows = np.array([0x0000, 0x7FFF, 0x8000, 0x8001, 0xFFFF, 0x4000, 0xC000], np.uint32)
    ties = ((base[:, None] & np.uint32(0xFFFF0000)) | lows[None]).ravel().view(np.float32)
    ties2 = ((base[:, None] & np.uint32(0xFFFE0000)) | np.uint32(0x10000) | lows[None]).ravel().view(np.float32)
    rand = rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 20000).astype(np.float32)
    x = np.concatenate([specials, ties, ties2, rand]).astype(np.float32)
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = bf16.round_to_bf16(x)
    same = (got == ref) | (np.isnan(got) & np.isnan(ref))
    assert same.all(), x[~same][:5]
    assert np.signbit(bf16.round_to_bf16(np.float32(-0.0)))


def test_bf16_from_bits():
    bits = np.array([0x3F80, 0xBF80, 0x0000, 0x4049], np.uint16)
    np.testing.assert_array_equal(bf16.from_bits(bits), [1.0, -1.0, 0.0, 3.140625])


# ---------------------------------------------------------------- SH basis
def _real_sh_scipy(l, m, theta, phi):
    """Real orthonormal SH without the Condon-Shortley phase, built from
    scipy's complex harmonics (which include it)."""
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    y = sph_harm_y(l, abs(m), theta, phi)
    cs = (-1.0) ** abs(m)
    if m > 0:
        return np.sqrt(2.0) * cs * y.real
    return np.sqrt(2.0) * cs * y.imag


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(1)
    v = rng.standard_normal((500, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    theta = np.arccos(np.clip(v[:, 2], -1, 1))
    phi = np.arctan2(v[:, 1], v[:, 0])
    Y = sh.basis(v, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            ref = _real_sh_scipy(l, m, theta, phi)
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-12,
                                       err_msg=f"l={l} m={m}")


def test_sh_orthonormal_by_quadrature():
    nt, nphi = 40, 80
    x, wx = np.polynomial.legendre.leggauss(nt)      # cos(theta)
    phi = np.arange(nphi) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wx[:, None] * np.full(nphi, 2 * np.pi / nphi)[None]).reshape(-1)
    Y = sh.basis(d, 3)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_gradient_by_finite_differences():
    rng = np.random.default_rng(2)
    v = rng.standard_normal((50, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    g = sh.basis_grad(v, 3)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        num = (sh.basis(v + e, 3) - sh.basis(v - e, 3)) / (2 * h)
        np.testing.assert_allclose(g[..., j], num, atol=1e-8)


# ---------------------------------------------------------------- geometry
def test_quat_to_rot_matches_scipy():
    rng = np.random.default_rng(3)
    q = rng.standard_normal((200, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    R = project.quat_to_rot(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()   # scipy: (x, y, z, w)
    np.testing.assert_allclose(R, ref, atol=1e-12)


def test_quat_to_rot_backward_by_finite_differences():
    rng = np.random.default_rng(4)
    q = rng.standard_normal((20, 4))
    dR = rng.standard_normal((20, 3, 3))
    g = project.quat_to_rot_backward(q, dR)
    h = 1e-6
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        num = np.sum((project.quat_to_rot(q + e) - project.quat_to_rot(q - e)) * dR, axis=(1, 2)) / (2 * h)
        np.testing.assert_allclose(g[:, j], num, atol=1e-7)


class _V:
    def __init__(self, W=64, H=48, f=55.0, R=None, t=(0.1, -0.2, 3.0)):
        self.width, self.height = W, H
        self.fx = self.fy = f
        self.cx, self.cy = W / 2, H / 2
        self.R = np.eye(3, dtype=np.float32) if R is None else np.asarray(R, np.float32)
        self.t = np.asarray(t, np.float32)
        self.z_near = 0.2
        self.bg = (0.0, 0.0, 0.0)


def test_camera_centre_and_point():
    rng = np.random.default_rng(5)
    R = Rotation.random(random_state=5).as_matrix().astype(np.float32)
    v = _V(R=R, t=(0.3, -1.0, 4.0))
    V = project.view_arrays(v)
    # the camera centre maps to the camera origin
    p = V["R"] @ V["c"] + V["t"]
    np.testing.assert_allclose(p, 0.0, atol=1e-6)   # R is float32, orthogonal to ~1e-7
    m = rng.standard_normal((10, 3))
    np.testing.assert_allclose(project.camera_point(V["R"], V["t"], m), m @ V["R"].T + V["t"], atol=1e-12)


def test_ewa_covariance_is_linearised_projection():
    """Sigma_2 - 0.3 I must equal Jn R Sigma R^T Jn^T where Jn is the
    numerical Jacobian of the pinhole map (no guard clamp active)."""
    rng = np.random.default_rng(6)
    R = Rotation.random(random_state=6).as_matrix().astype(np.float32)
    v = _V(R=R, t=(0.05, 0.1, 3.0))
    V = project.view_arrays(v)
    n = 20
    mu = (rng.uniform(-0.3, 0.3, (n, 3)) @ V["R"]).astype(np.float64)   # near the axis
    s = np.exp(rng.normal(-2.5, 0.3, (n, 3))).astype(np.float32)
    q = rng.standard_normal((n, 4))
    o = np.full(n, 0.5)
    P = project.project(mu, s, q, o, v, (16, 16), colour=np.zeros((n, 3)))

    def pix(x):
        pc = V["R"] @ x + V["t"]
        return np.array([V["fx"] * pc[0] / pc[2] + V["cx"], V["fy"] * pc[1] / pc[2] + V["cy"]])

    for i in range(n):
        h = 1e-6
        Jn = np.stack([(pix(mu[i] + h * e) - pix(mu[i] - h * e)) / (2 * h) for e in np.eye(3)], 1)
        qn = q[i] / np.linalg.norm(q[i])
        Rq = Rotation.from_quat(qn[[1, 2, 3, 0]]).as_matrix()
        Sig = Rq @ np.diag(s[i].astype(np.float64) ** 2) @ Rq.T
        ref = Jn @ Sig @ Jn.T + 0.3 * np.eye(2)
        got = np.array([[P["_A"][i], P["_B"][i]], [P["_B"][i], P["_C"][i]]])
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(P["conic"][i], [np.linalg.inv(ref)[0, 0], np.linalg.inv(ref)[0, 1],
                                                   np.linalg.inv(ref)[1, 1]], rtol=1e-6)
        lam = np.linalg.eigvalsh(ref).max()
        assert P["r"][i] == int(np.ceil(3 * np.sqrt(lam) - 1e-9))
        np.testing.assert_allclose([P["u"][i], P["w"][i]], pix(mu[i]), rtol=1e-12)


def test_pixel_box_is_the_square_test():
    """A pixel is inside a splat's box iff its centre is within r_x = min(r,
    e_x) of the 2-D mean in x and r_y = min(r, e_y) in y (and it lies in the
    image), with e_x = sqrt(2 ln(255 o) Sigma_2,xx) computed here from the
    inverted conic."""
    rng = np.random.default_rng(7)
    v = _V()
    n = 200
    mu = np.stack([rng.uniform(-1.5, 1.5, n), rng.uniform(-1.2, 1.2, n), rng.uniform(-1, 1, n)], 1)
    s = np.exp(rng.normal(-3, 0.6, (n, 3)))
    q = rng.standard_normal((n, 4))
    o = rng.uniform(0.002, 1.0, n)
    P = project.project(mu, s, q, o, v, (16, 16), colour=np.zeros((n, 3)))
    I, J = np.meshgrid(np.arange(v.width), np.arange(v.height))
    for i in range(n):
        if o[i] < 1.0 / 255.0:
            assert not P["valid"][i]
            continue
        S2 = np.linalg.inv(np.array([[P["conic"][i][0], P["conic"][i][1]],
                                     [P["conic"][i][1], P["conic"][i][2]]]))
        t = np.log(255.0 * o[i])
        rx = min(P["r"][i], np.sqrt(2 * t * S2[0, 0]))
        ry = min(P["r"][i], np.sqrt(2 * t * S2[1, 1]))
        inside = ((np.abs(I + 0.5 - P["u"][i]) <= rx) & (np.abs(J + 0.5 - P["w"][i]) <= ry))
        x0, x1, y0, y1 = P["box"][i]
        box = (I >= x0) & (I <= x1) & (J >= y0) & (J <= y1)
        if P["p"][i, 2] <= 0.2:
            assert not P["valid"][i]
            continue
        if P["frag_value"][i]:
            continue
        np.testing.assert_array_equal(box, inside)
        assert P["valid"][i] == inside.any()
        if P["valid"][i]:
            tx0, tx1, ty0, ty1 = P["tiles"][i]
            cols = np.nonzero(inside.any(0))[0]
            rows = np.nonzero(inside.any(1))[0]
            assert (tx0, tx1, ty0, ty1) == (cols.min() // 16, cols.max() // 16, rows.min() // 16, rows.max() // 16)


def test_depth_key_is_float32_bits_of_depth():
    rng = np.random.default_rng(8)
    v = _V(t=(0, 0, 5.0))
    mu = rng.uniform(-1, 1, (100, 3))
    P = project.project(mu, np.full((100, 3), 0.05), np.tile([1.0, 0, 0, 0], (100, 1)),
                        np.full(100, 0.5), v, (16, 16), colour=np.zeros((100, 3)))
    z = mu[:, 2] + 5.0
    np.testing.assert_array_equal(P["zbits"], z.astype(np.float32).view(np.uint32))
    # for positive floats the bit order is the numeric order
    o1 = np.argsort(P["zbits"], kind="stable")
    o2 = np.argsort(z.astype(np.float32), kind="stable")
    np.testing.assert_array_equal(o1, o2)


def test_normal_faces_camera_and_plane_distance():
    """Flat Gaussians: the normal is the rotated thin axis in camera frame,
    facing the camera; d is the distance from the camera centre to the
    Gaussian's plane, computed here in world coordinates."""
    rng = np.random.default_rng(9)
    R = Rotation.random(random_state=9).as_matrix().astype(np.float32)
    v = _V(R=R, t=(0.0, 0.0, 4.0))
    V = project.view_arrays(v)
    n = 50
    mu = rng.uniform(-0.5, 0.5, (n, 3))
    thin = rng.integers(0, 3, n)
    s = np.full((n, 3), 0.1)
    s[np.arange(n), thin] = 1e-4
    q = rng.standard_normal((n, 4))
    P = project.project(mu, s, q, np.full(n, 0.5), v, (16, 16), colour=np.zeros((n, 3)))
    for i in range(n):
        qn = q[i] / np.linalg.norm(q[i])
        axis_w = Rotation.from_quat(qn[[1, 2, 3, 0]]).as_matrix()[:, thin[i]]
        dist = abs(np.dot(axis_w, mu[i] - V["c"]))
        np.testing.assert_allclose(P["d"][i], dist, rtol=1e-6)   # float32 R: orthogonal to ~1e-7
        n_cam = V["R"] @ axis_w
        np.testing.assert_allclose(np.abs(P["normal"][i]), np.abs(n_cam), atol=1e-6)
        assert np.dot(P["normal"][i], P["p"][i]) <= 0


def test_opacity_box_keeps_every_drawable_pixel():
    """Brute force: inside the 3-sigma square, every pixel whose opacity
    o exp(power) reaches 1/255 lies in the (opacity-aware) box, and the box
    is never wider than the square."""
    rng = np.random.default_rng(8)
    v = _V()
    n = 300
    mu = np.stack([rng.uniform(-1.5, 1.5, n), rng.uniform(-1.2, 1.2, n), rng.uniform(-1, 1, n)], 1)
    s = np.exp(rng.normal(-3, 0.8, (n, 3)))
    q = rng.standard_normal((n, 4))
    o = rng.uniform(0.003, 1.0, n)
    P = project.project(mu, s, q, o, v, (16, 16), colour=np.zeros((n, 3)))
    I, J = np.meshgrid(np.arange(v.width), np.arange(v.height))
    tight = 0
    for i in np.nonzero(P["valid"])[0]:
        a, b, c = P["conic"][i]
        dx, dy = P["u"][i] - (I + 0.5), P["w"][i] - (J + 0.5)
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        drawn = (o[i] * np.exp(power) >= 1.0 / 255.0) & (power <= 0)
        square = (np.abs(dx) <= P["r"][i]) & (np.abs(dy) <= P["r"][i])
        x0, x1, y0, y1 = P["box"][i]
        box = (I >= x0) & (I <= x1) & (J >= y0) & (J <= y1)
        assert not (drawn & square & ~box).any(), i
        assert not (box & ~square).any(), i
        tight += int((square & ~box).sum())
    assert tight > 0      # the box is strictly smaller for some splats


def _rect_min_q(a, b, c, dx0, dx1, dy0, dy1):
    """min of Q = a dx^2 + 2 b dx dy + c dy^2 (positive definite) over the
    rectangle [dx0, dx1] x [dy0, dy1]: zero if it holds the origin, else the
    least of the four edge minima (each a clamped 1-D parabola)."""
    if dx0 <= 0.0 <= dx1 and dy0 <= 0.0 <= dy1:
        return 0.0
    best = np.inf
    for x in (dx0, dx1):
        y = min(max(-b * x / c, dy0), dy1)
        best = min(best, a * x * x + 2 * b * x * y + c * y * y)
    for y in (dy0, dy1):
        x = min(max(-b * y / a, dx0), dx1)
        best = min(best, a * x * x + 2 * b * x * y + c * y * y)
    return best


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_tile_mask_is_ellipse_rectangle_overlap(tile):
    """Ellipse-tile culling: for a box of 2 x 2 up to 64 tiles, bit r * nx + c is
    set iff the pixel-centre rectangle the tile shares with the box meets the
    drawable ellipse Q <= 2 ln(255 o) (checked through the conic by edge
    minimisation, a different route from the strip extents), and every tile
    holding a drawable pixel centre (brute force) keeps its bit; the culled
    count is the number of set bits."""
    tw, th = tile
    rng = np.random.default_rng(31)
    v = _V()
    n = 300
    mu = np.stack([rng.uniform(-1.5, 1.5, n), rng.uniform(-1.2, 1.2, n), rng.uniform(-1, 1, n)], 1)
    s = np.exp(rng.normal(-2.6, 0.8, (n, 3)))
    s[:, 0] *= np.exp(rng.uniform(0, 2.5, n))          # elongated splats
    q = rng.standard_normal((n, 4))
    o = rng.uniform(0.005, 1.0, n)
    P = project.project(mu, s, q, o, v, tile, colour=np.zeros((n, 3)))
    checked = culled = 0
    for i in np.nonzero(P["small"])[0]:
        a, b, c = P["conic"][i]
        t2 = 2.0 * np.log(255.0 * o[i])
        x_lo, x_hi, y_lo, y_hi = P["box"][i]
        tx0, tx1, ty0, ty1 = P["tiles"][i]
        nx = tx1 - tx0 + 1
        bits = int(P["tmask"][i])
        assert P["count"][i] == bin(bits).count("1")
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                bit = (bits >> ((ty - ty0) * nx + (tx - tx0))) & 1
                c0, c1 = max(tx * tw, x_lo), min(tx * tw + tw - 1, x_hi)
                r0, r1 = max(ty * th, y_lo), min(ty * th + th - 1, y_hi)
                xs = np.arange(c0, c1 + 1) + 0.5 - P["u"][i]
                ys = np.arange(r0, r1 + 1) + 0.5 - P["w"][i]
                X, Y = np.meshgrid(xs, ys)
                drawable = (a * X * X + 2 * b * X * Y + c * Y * Y <= t2).any()
                if drawable:
                    assert bit, (i, tx, ty)
                qmin = _rect_min_q(a, b, c, c0 + 0.5 - P["u"][i], c1 + 0.5 - P["u"][i],
                                   r0 + 0.5 - P["w"][i], r1 + 0.5 - P["w"][i])
                if not P["frag_value"][i]:
                    assert bit == (qmin <= t2), (i, tx, ty, qmin, t2)
                checked += 1
                culled += 1 - bit
    assert checked > 500
    assert culled > 0.05 * checked      # the ellipse leaves part of the box's tiles


def test_tanh_opacity_masks_non_positive():
    """Masked-opacity decoder variant: the same decoder outputs read as tanh
    instead of sigmoid, and every Gaussian with tanh(z) <= 0 is culled (not
    valid, no tiles) while the others project as they would with that
    opacity."""
    from oracle import anchors
    from synth import scenes
    wl = scenes.make_small_anchor(5, n_anchor=40, opacity_act=1)
    sc = wl.scene
    rows, _ = anchors.select(sc, wl.views)
    D = anchors.decode(sc, wl.views, rows)
    z = D["_z2"].reshape(rows.shape[0], -1, anchors.GAUSS_OUT)[..., 0].ravel()
    np.testing.assert_array_equal(D["opacity"], np.tanh(z))
    masked = z <= 0
    assert 0.2 < masked.mean() < 0.8
    v0 = rows[:, 0] == 0
    sel = np.repeat(v0, D["n"])
    P = project.project(D["mu"][sel], D["scales"][sel], D["quats"][sel], D["opacity"][sel],
                        wl.views[0], (16, 16), colour=D["rgb"][sel])
    assert not P["valid"][masked[sel]].any()
    assert (P["count"][masked[sel]] == 0).all()
    keep = ~masked[sel] & (D["opacity"][sel] >= 1.0 / 255.0)
    P2 = project.project(D["mu"][sel][keep], D["scales"][sel][keep], D["quats"][sel][keep],
                         D["opacity"][sel][keep], wl.views[0], (16, 16), colour=D["rgb"][sel][keep])
    np.testing.assert_array_equal(P2["box"], P["box"][keep])
