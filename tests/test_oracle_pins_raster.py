"""Pins of the oracle's binning, sort and compositing against closed forms,
brute force and invariants (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle import pipeline, project, raster
from synth import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class _Scene:
    def __init__(self, means, scales, quats, opacity, rgb):
        n = len(means)
        self.means = np.asarray(means, np.float32)
        self.scales = np.asarray(scales, np.float32)
        self.quats = np.asarray(quats, np.float32)
        self.opacity = np.asarray(opacity, np.float32)
        y00 = 0.5 / np.sqrt(np.pi)
        self.sh = ((np.asarray(rgb, np.float64) - 0.5) / y00).astype(np.float32).reshape(n, 1, 3)
        self.sh_degree = 0


def _view(W=48, H=40, f=50.0, t=(0.0, 0.0, 3.0), cx=None, cy=None):
    v = scenes.View(W, H, f, f, W / 2 if cx is None else cx, H / 2 if cy is None else cy,
                    np.eye(3, dtype=np.float32), np.asarray(t, np.float32))
    return v


def _sh_rgb(scene):
    """The colour that the SH-0 coefficients encode (clamped at 0), float64."""
    return np.maximum(scene.sh[:, 0, :].astype(np.float64) * (0.5 / np.sqrt(np.pi)) + 0.5, 0.0)


# ---------------------------------------------------------------- closed form
def test_single_flat_gaussian_closed_form():
    """A flat Gaussian (scales s, s, ~0, no rotation) on the optical axis at
    depth z projects to an isotropic 2-D Gaussian of variance (f s / z)^2 + 0.3
    centred on the principal point (derived by hand, Sec. 3.1 / Eq. 1)."""
    W, H, f, z = 64, 48, 60.0, 3.0
    s = 0.0625          # float32-exact inputs keep the closed form exact
    o = 0.75
    rgb = np.array([0.2, 0.5, 0.9])
    view = _view(W, H, f, t=(0, 0, z))
    sc = _Scene([[0, 0, 0]], [[s, s, 1e-6]], [[1, 0, 0, 0]], [o], [rgb])
    r = pipeline.render_explicit(sc, [view])
    img = r.images[0]
    var = (f * s / z) ** 2 + 0.3
    rad = np.ceil(3 * np.sqrt(var))
    I, J = np.meshgrid(np.arange(W), np.arange(H))
    dx, dy = I + 0.5 - W / 2, J + 0.5 - H / 2
    a = np.minimum(0.99, o * np.exp(-(dx ** 2 + dy ** 2) / (2 * var)))
    a = np.where((np.abs(dx) <= rad) & (np.abs(dy) <= rad) & (a >= 1 / 255), a, 0.0).ravel()
    rgb_img = _sh_rgb(sc)[0][:, None] * a[None]
    np.testing.assert_allclose(img["alpha"], a, atol=1e-14)
    np.testing.assert_allclose(img["rgb"], rgb_img, atol=1e-12)
    np.testing.assert_allclose(img["D"], z * a, atol=1e-12)
    np.testing.assert_allclose(img["normal"][2], -a, atol=1e-12)
    np.testing.assert_allclose(img["normal"][:2], 0.0, atol=1e-12)
    np.testing.assert_allclose(img["depth"], np.where(a > 0, z, 0.0), atol=1e-12)


def test_two_gaussian_blend_and_depth_order():
    """Two overlapping flat Gaussians: C = c1 a1 + c2 a2 (1 - a1) with the
    nearer one first, whatever their index order."""
    W, H, f = 32, 32, 40.0
    view = _view(W, H, f, t=(0, 0, 0))
    for near_first in (True, False):
        z = [2.0, 3.0] if near_first else [3.0, 2.0]
        sc = _Scene([[0, 0, z[0]], [0, 0, z[1]]], [[0.25, 0.25, 1e-6], [0.375, 0.375, 1e-6]],
                    [[1, 0, 0, 0]] * 2, [0.625, 0.6875], [[1, 0, 0], [0, 0, 1]])
        r = pipeline.render_explicit(sc, [view])
        img = r.images[0]
        c = _sh_rgb(sc)
        I, J = np.meshgrid(np.arange(W), np.arange(H))
        d2 = ((I + 0.5 - W / 2) ** 2 + (J + 0.5 - H / 2) ** 2).ravel()

        def alpha(i):
            var = (f * float(sc.scales[i, 0]) / z[i]) ** 2 + 0.3
            a = np.minimum(0.99, float(sc.opacity[i]) * np.exp(-d2 / (2 * var)))
            rad = np.ceil(3 * np.sqrt(var))
            inb = ((np.abs(I + 0.5 - W / 2) <= rad) & (np.abs(J + 0.5 - H / 2) <= rad)).ravel()
            return np.where(inb & (a >= 1 / 255), a, 0.0)

        a0, a1 = alpha(0), alpha(1)
        front, back = (0, 1) if z[0] < z[1] else (1, 0)
        af, ab = (a0, a1) if front == 0 else (a1, a0)
        expect = c[front][:, None] * af + c[back][:, None] * ab * (1 - af)
        np.testing.assert_allclose(img["rgb"], expect, atol=1e-12)
        np.testing.assert_allclose(img["alpha"], 1 - (1 - af) * (1 - ab), atol=1e-12)
        Dexp = z[front] * af + z[back] * ab * (1 - af)
        np.testing.assert_allclose(img["D"], Dexp, atol=1e-12)


def test_planar_unbiased_depth_is_exact():
    """Flat Gaussians lying in one plane n.X = -d (camera frame, any alpha,
    any count) give D^(p) = -d / (n . K^-1 p~) at every covered pixel
    (Eq. 7): the blending weights cancel."""
    rng = np.random.default_rng(11)
    W, H, f = 48, 40, 45.0
    view = _view(W, H, f, t=(0, 0, 0))
    nrm = np.array([0.2, -0.3, -1.0])
    nrm /= np.linalg.norm(nrm)
    dpl = 2.5                   # plane: n . X = -d  <=>  n . X + d = 0
    m = 30
    uv = rng.uniform(-0.6, 0.6, (m, 2))
    # points on the plane with camera-frame x, y = uv * z
    zs = -dpl / (nrm[0] * uv[:, 0] + nrm[1] * uv[:, 1] + nrm[2])
    pts = np.stack([uv[:, 0] * zs, uv[:, 1] * zs, zs], 1)
    # rotation taking local z to the plane normal
    zax = np.array([0.0, 0.0, 1.0])
    v = np.cross(zax, nrm)
    ang = np.arccos(np.dot(zax, nrm))
    axis = v / np.linalg.norm(v)
    q = np.concatenate([[np.cos(ang / 2)], axis * np.sin(ang / 2)])
    sc = _Scene(pts, np.tile([0.12, 0.08, 1e-7], (m, 1)), np.tile(q, (m, 1)),
                rng.uniform(0.3, 0.9, m), rng.uniform(0, 1, (m, 3)))
    r = pipeline.render_explicit(sc, [view])
    img = r.images[0]
    I, J = np.meshgrid(np.arange(W), np.arange(H))
    ray = np.stack([(I.ravel() + 0.5 - W / 2) / f, (J.ravel() + 0.5 - H / 2) / f, np.ones(W * H)], 1)
    n_face = -nrm if np.dot(nrm, pts[0]) > 0 else nrm
    d_face = -np.dot(n_face, pts[0])
    expect = -d_face / (ray @ n_face)
    cov = img["alpha"] > 1e-3
    assert cov.sum() > 200
    np.testing.assert_allclose(img["depth"][cov], expect[cov], rtol=1e-5)


# ---------------------------------------------------------------- brute force
def _brute_force(scene, view, rgb):
    """Per pixel: every valid splat whose box holds the pixel, sorted by
    (depth key, index), composited one by one in plain Python."""
    S = project.project(np.asarray(scene.means, np.float64), scene.scales, scene.quats,
                        scene.opacity, view, (16, 16), sh=scene.sh, sh_degree=scene.sh_degree)
    W, H = view.width, view.height
    out = np.zeros((3, H * W))
    acc = np.zeros(H * W)
    valid = np.nonzero(S["valid"])[0]
    order = sorted(valid, key=lambda i: (int(S["zbits"][i]), int(i)))
    for j in range(H):
        for i in range(W):
            T = 1.0
            C = np.zeros(3)
            for g in order:
                x0, x1, y0, y1 = S["box"][g]
                if not (x0 <= i <= x1 and y0 <= j <= y1):
                    continue
                a, b, c = S["conic"][g]
                # the compositor's 2-D mean is binary32
                dx = float(np.float32(S["u"][g])) - (i + 0.5)
                dy = float(np.float32(S["w"][g])) - (j + 0.5)
                pw = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
                if pw > 0:
                    continue
                al = min(0.99, S["opacity"][g] * np.exp(pw))
                if al < 1 / 255:
                    continue
                Tn = T * (1 - al)
                if Tn < 1e-4:
                    break
                C += S["rgb"][g] * al * T
                T = Tn
            out[:, j * W + i] = C
            acc[j * W + i] = 1 - T
    return out, acc


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8), (16, 8)])
def test_tiled_equals_brute_force(tile):
    wl = scenes.make_small_explicit(21, n=45, width=44, height=37, spread=0.6, log_scale=-2.2)
    view = wl.views[0]
    r = pipeline.render_explicit(wl.scene, [view], tile=tile)
    C, A = _brute_force(wl.scene, view, None)
    # same decisions and transmittances bit for bit; colour sums differ only
    # in summation order
    np.testing.assert_array_equal(r.images[0]["alpha"], A)
    np.testing.assert_allclose(r.images[0]["rgb"], C, rtol=0, atol=1e-14)
    assert (r.images[0]["alpha"] > 0).sum() > 300


def test_sort_matches_python_sorted():
    wl = scenes.make_small_explicit(22, n=60, width=70, height=50)
    r = pipeline.render_explicit(wl.scene, wl.views)
    S = r.splats[0]
    lay = r.layout
    entries = []
    for g in np.nonzero(S["valid"])[0]:
        tx0, tx1, ty0, ty1 = S["tiles"][g]
        nx = tx1 - tx0 + 1
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                bit = (ty - ty0) * nx + (tx - tx0)
                if S["small"][g] and not (int(S["tmask"][g]) >> bit) & 1:
                    continue      # a tile the drawable ellipse does not reach
                entries.append((ty * lay["TX"][0] + tx, int(S["zbits"][g]), int(g)))
    entries.sort()
    got = list(zip(r.sorted["gtile"].tolist(), r.sorted["zbits"].tolist(), r.sorted["gid"].tolist()))
    assert got == entries
    for t in range(lay["tile_off"][-1]):
        s0, s1 = r.sorted["ranges"][t]
        assert all(e[0] == t for e in got[s0:s1])
        assert sum(1 for e in got if e[0] == t) == s1 - s0


# ---------------------------------------------------------------- invariants
def test_compositing_invariants_c0():
    wl = scenes.make_c0()
    r = pipeline.render_explicit(wl.scene, wl.views)
    img = r.images[0]
    assert img["T"].min() >= 1e-4
    assert img["alpha"].max() <= 1 - 1e-4 + 1e-15
    assert (img["alpha"] >= 0).all()
    rgbmax = r.splats[0]["rgb"][r.splats[0]["valid"]].max()
    assert (img["rgb"] <= rgbmax * img["alpha"][None] + 1e-12).all()
    # transmittance is non-increasing along every pixel's list
    for gtile, (ent, I, J, pix, R) in list(img["tiles"].items())[:20]:
        if ent.size:
            Tp = np.cumprod(1 - R["a_inc"], axis=1)
            assert (np.diff(Tp, axis=1) <= 0).all()
    # only a handful of decisions sit within float32 reach of their bound
    assert img["tie"].mean() < 0.005


def test_transmittance_recovery_by_division():
    """The GPU's reverse walk recovers T_k = T_{k+1} / (1 - alpha_k); in
    float64 that equals the forward products to 1e-12."""
    wl = scenes.make_c0()
    r = pipeline.render_explicit(wl.scene, wl.views)
    worst = 0.0
    for gtile, (ent, I, J, pix, R) in r.images[0]["tiles"].items():
        if ent.size == 0:
            continue
        a = R["a_inc"]
        T = R["T"].copy()
        rec = np.zeros_like(a)
        for k in range(a.shape[1] - 1, -1, -1):
            T = T / (1 - a[:, k])
            rec[:, k] = T
        worst = max(worst, np.max(np.abs(rec - R["Tb"]) / R["Tb"]))
    assert worst < 1e-12


def test_tile_shape_invariance_c0():
    wl = scenes.make_c0()
    base = pipeline.render_explicit(wl.scene, wl.views, tile=(16, 16)).images[0]
    for tile in [(8, 8), (32, 16), (16, 8)]:
        other = pipeline.render_explicit(wl.scene, wl.views, tile=tile).images[0]
        np.testing.assert_array_equal(base["alpha"], other["alpha"])
        np.testing.assert_array_equal(base["last"] > 0, other["last"] > 0)
        for k in ("rgb", "D", "depth", "normal"):
            np.testing.assert_allclose(base[k], other[k], rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------- L1 seed
def test_l1_seed_hand_example():
    """Eq. 8 per-image mean over B = 2 images of 1 and 2 pixels, unit weights:
    worked out by hand in tests/golden/l1_seed.json."""
    with open(os.path.join(GOLDEN, "l1_seed.json")) as fh:
        g = json.load(fh)
    images = [dict(rgb=np.array(im["rgb"], float), depth=np.array(im["depth"], float),
                   normal=np.array(im["normal"], float)) for im in g["images"]]
    targets = dict(rgb=[np.array(t["rgb"], float) for t in g["targets"]],
                   depth=[np.array(t["depth"], float) for t in g["targets"]],
                   normal=[np.array(t["normal"], float) for t in g["targets"]])
    L, grads = raster.l1_seed(images, targets)
    assert abs(L - g["loss"]) < 1e-15
    for gr, ex in zip(grads, g["grads"]):
        np.testing.assert_array_equal(gr["rgb"], np.array(ex["rgb"]))
        np.testing.assert_array_equal(gr["depth"], np.array(ex["depth"]))
        np.testing.assert_array_equal(gr["normal"], np.array(ex["normal"]))


def _golden_l1(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        g = json.load(fh)
    images = [dict(rgb=np.array(im["rgb"], float), depth=np.array(im["depth"], float),
                   normal=np.array(im["normal"], float)) for im in g["images"]]
    targets = dict(rgb=[np.array(t["rgb"], float) for t in g["targets"]],
                   depth=[np.array(t["depth"], float) for t in g["targets"]],
                   normal=[np.array(t["normal"], float) for t in g["targets"]])
    return g, images, targets


def test_l1_seed_depth_mask_hand_example():
    """Sec. 3.4 Step 2: target depths that are not positive carry no prior;
    worked out by hand in tests/golden/l1_seed_masked.json."""
    g, images, targets = _golden_l1("l1_seed_masked.json")
    L, grads = raster.l1_seed(images, targets)
    assert abs(L - g["loss"]) < 1e-15
    for gr, ex in zip(grads, g["grads"]):
        for k in ("rgb", "depth", "normal"):
            np.testing.assert_array_equal(gr[k], np.array(ex[k]))


def test_l1_seed_nan_depth_is_masked():
    """A NaN target depth acts as a masked pixel: same loss and gradients as
    a zero target there, and the loss equals brute force over the kept
    pixels only."""
    rng = np.random.default_rng(3)
    npx = 37
    images = [dict(rgb=rng.random((3, npx)), depth=rng.uniform(1, 5, npx),
                   normal=rng.standard_normal((3, npx)))]
    td = rng.uniform(1, 5, npx)
    drop = rng.random(npx) < 0.4
    t0 = dict(rgb=[rng.random((3, npx))], depth=[np.where(drop, 0.0, td)],
              normal=[rng.standard_normal((3, npx))])
    tn = dict(rgb=t0["rgb"], depth=[np.where(drop, np.nan, td)], normal=t0["normal"])
    L0, g0 = raster.l1_seed(images, t0, (0.5, 2.0, 0.25))
    Ln, gn = raster.l1_seed(images, tn, (0.5, 2.0, 0.25))
    assert L0 == Ln
    for k in ("rgb", "depth", "normal"):
        np.testing.assert_array_equal(g0[0][k], gn[0][k])
    assert np.all(g0[0]["depth"][drop] == 0.0) and np.all(g0[0]["depth"][~drop] != 0.0)
    im = images[0]
    brute = 0.0
    for p in range(npx):
        brute += 0.5 * sum(abs(im["rgb"][c, p] - t0["rgb"][0][c, p]) for c in range(3))
        brute += 0.25 * sum(abs(im["normal"][c, p] - t0["normal"][0][c, p]) for c in range(3))
        if not drop[p]:
            brute += 2.0 * abs(im["depth"][p] - td[p])
    assert abs(L0 - brute / npx) < 1e-12


def test_sampled_tiles_equal_full_render():
    """Binning and compositing a subset of tiles gives exactly the entries
    and pixels of those tiles in the full render (the bounded-sample mode
    used at full workload sizes)."""
    wl = scenes.make_small_explicit(23, n=70, width=61, height=45)
    full = pipeline.render_explicit(wl.scene, wl.views)
    keep = [0, 3, 7, 11]
    part = pipeline.render_explicit(wl.scene, wl.views, keep_tiles=keep)
    for t in keep:
        a0, a1 = full.sorted["ranges"][t]
        b0, b1 = part.sorted["ranges"][t]
        np.testing.assert_array_equal(full.sorted["gid"][a0:a1], part.sorted["gid"][b0:b1])
        ent, I, J, pix, R = part.images[0]["tiles"][t]
        np.testing.assert_array_equal(part.images[0]["rgb"][:, pix], full.images[0]["rgb"][:, pix])
