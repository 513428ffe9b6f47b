"""Seeded synthetic scenes, cameras and loss targets for the five workloads.

This module only draws random inputs and places cameras; it holds none of
the rasterizer's arithmetic (no projection, decoding, binning or
compositing) and none of the depth prior's (no least squares, no
re-projection): for the depth-prior inputs it ray-casts a scene of boxes to
get the true depth that a monocular network would approximate, and turns
that into a pseudo depth with an unknown scale and shift.  Both the FP64 oracle's tests and the GPU path's tests and
benchmark consume the arrays it returns, so the two sides always see the
same bytes.

Workloads (sizes fixed by the benchmark definition; the paper publishes
none, its datasets are not available and are stood in for by these):

  C0  2,000 explicit Gaussians in the unit cube, one 128x128 pinhole view.
  C1  1,000,000 explicit Gaussians, SH degree 3, street scene, 1920x1080.
  C2  200,000 voxel anchors x 10 Gaussians over a 200x200x50 m city block,
      8 views of uneven resolution (960x540 .. 1920x1080).
  C3  600,000 anchors, 4 views at 3840x2160.
  C4  2,000,000 anchors over a 1x1 km aerial tile, 16 views at 1600x1200.

The voxel anchors are placed with the paper's LoD voxelisation (Sec. 3.2,
Eq. 2): a dense surface point cloud P is snapped to grids of size
delta/2^k for k = 0..K-1, and each level keeps a seeded subsample of its
unique grid points.

Seeds: scene = k, cameras = 10 + k, targets / loss weights = 100 + k
(numpy PCG64 via default_rng).  Arrays are float32; decoder weights are
returned as bfloat16 bit patterns (uint16, round-to-nearest-even of a
float32 draw) together with the float32 values they encode.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

N_OFFSETS = 10      # Gaussians per anchor (workload definition)
FEAT_DIM = 32       # anchor feature width (Sec. 3.2: F_v in R^32)
MLP_IN = FEAT_DIM + 4   # [feature, view direction (3), relative distance]
MLP_HIDDEN = 32
GAUSS_OUT = 11      # per Gaussian: opacity 1, rgb 3, scale 3, rotation 4
MLP_OUT = N_OFFSETS * GAUSS_OUT


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
@dataclass
class View:
    """Pinhole camera, OpenCV frame (x right, y down, z forward).

    R is the world->camera rotation (row-major 3x3), t the translation, so a
    world point X maps to R @ X + t.  Pixel (i, j) has its centre at
    (i + 0.5, j + 0.5).
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray          # (3, 3) float32
    t: np.ndarray          # (3,) float32
    z_near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def as_record(self) -> dict:
        return dict(width=int(self.width), height=int(self.height),
                    fx=float(np.float32(self.fx)), fy=float(np.float32(self.fy)),
                    cx=float(np.float32(self.cx)), cy=float(np.float32(self.cy)),
                    R=np.asarray(self.R, np.float32).reshape(9).tolist(),
                    t=np.asarray(self.t, np.float32).reshape(3).tolist(),
                    z_near=float(np.float32(self.z_near)),
                    bg=[float(np.float32(b)) for b in self.bg])


def focal_for_fov(width: int, fov_deg: float = 60.0) -> float:
    """Focal length in pixels for a horizontal field of view."""
    return width / (2.0 * np.tan(np.deg2rad(fov_deg) / 2.0))


def look_at(position, target, width, height, fov_deg=60.0, yaw_hint=0.0,
            z_near=0.2) -> View:
    """Camera at `position` looking at `target`, world up = +z.

    When the viewing direction is (anti)parallel to +z (nadir views) the
    right vector is taken from `yaw_hint` instead of the up vector.
    """
    c = np.asarray(position, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0])
    r = np.cross(f, up)
    if np.linalg.norm(r) < 1e-6:
        r = np.array([np.cos(yaw_hint), np.sin(yaw_hint), 0.0])
        r -= f * np.dot(r, f)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f]).astype(np.float32)
    t = (-R.astype(np.float64) @ c).astype(np.float32)
    fx = focal_for_fov(width, fov_deg)
    return View(width, height, fx, fx, width / 2.0, height / 2.0, R, t, z_near)


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------
def bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest, ties to even."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns -> float32 values."""
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32)


def random_quats(rng, n) -> np.ndarray:
    """Uniform rotations: normalised 4-D standard normals, (w, x, y, z)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def digest(arrays: dict) -> str:
    """SHA-256 over the arrays of a scene (names sorted), for reproducibility."""
    h = hashlib.sha256()
    for k in sorted(arrays):
        v = arrays[k]
        if isinstance(v, np.ndarray):
            h.update(k.encode())
            h.update(np.ascontiguousarray(v).tobytes())
    return h.hexdigest()


# --------------------------------------------------------------------------
# scene containers
# --------------------------------------------------------------------------
@dataclass
class ExplicitScene:
    means: np.ndarray       # (N, 3) f32
    scales: np.ndarray      # (N, 3) f32, > 0
    quats: np.ndarray       # (N, 4) f32, (w, x, y, z), not necessarily unit
    opacity: np.ndarray     # (N,) f32 in (0, 1)
    sh: np.ndarray          # (N, (deg+1)^2, 3) f32
    sh_degree: int

    @property
    def n(self):
        return self.means.shape[0]

    def arrays(self):
        return dict(means=self.means, scales=self.scales, quats=self.quats,
                    opacity=self.opacity, sh=self.sh)


@dataclass
class AnchorScene:
    x: np.ndarray           # (A, 3) f32 anchor positions
    l: np.ndarray           # (A, 3) f32 anchor scaling factors
    O: np.ndarray           # (A, n, 3) f32 learnable offsets
    F: np.ndarray           # (A, 32) f32 features
    level: np.ndarray       # (A,) u8 LoD level, 0 = coarsest
    W1_bits: np.ndarray     # (36, 32H) u16 bf16 bit patterns (input-major), H decoder heads
    b1: np.ndarray          # (32H,) f32
    W2_bits: np.ndarray     # (32, n G) u16 bf16 bit patterns, G = 11 or 14 outputs per Gaussian
    b2: np.ndarray          # (n G,) f32
    n_levels: int
    d_max: float
    opacity_act: int = 0    # 0: sigmoid; 1: tanh with non-positive opacities masked
    offset_mode: int = 0    # 0: offsets from the table O; 1: decoded (14 outputs per Gaussian)
    decoder_heads: int = 1  # 1: one shared MLP; 3: one MLP per attribute group

    @property
    def n(self):
        return self.x.shape[0]

    @property
    def W1(self):
        return bf16_value(self.W1_bits)

    @property
    def W2(self):
        return bf16_value(self.W2_bits)

    def arrays(self):
        return dict(x=self.x, l=self.l, O=self.O, F=self.F, level=self.level,
                    W1_bits=self.W1_bits, b1=self.b1, W2_bits=self.W2_bits,
                    b2=self.b2)


@dataclass
class Workload:
    name: str
    scene: object
    views: list
    targets: dict = field(default_factory=dict)   # per-view loss targets

    @property
    def pixels(self):
        return sum(v.width * v.height for v in self.views)


# --------------------------------------------------------------------------
# explicit Gaussians
# --------------------------------------------------------------------------
def _explicit_attrs(rng, n, sh_degree, rgb_dc=None):
    scales = np.exp(rng.normal(-4.0, 0.5, (n, 3))).astype(np.float32)
    quats = random_quats(rng, n)
    opacity = sigmoid(rng.standard_normal(n)).astype(np.float32)
    k = (sh_degree + 1) ** 2
    if rgb_dc is not None:
        sh = np.zeros((n, k, 3), np.float32)
        y00 = 0.5 / np.sqrt(np.pi)
        sh[:, 0, :] = ((rgb_dc - 0.5) / y00).astype(np.float32)
    else:
        sh = rng.normal(0.0, 0.2, (n, k, 3)).astype(np.float32)
    return scales, quats, opacity, sh


def make_c0(seed: int = 0) -> Workload:
    """C0: 2,000 Gaussians in the unit cube, one 128x128 view, SH degree 0."""
    rng = np.random.default_rng(seed)
    n = 2000
    means = rng.uniform(-0.5, 0.5, (n, 3)).astype(np.float32)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    scales, quats, opacity, sh = _explicit_attrs(rng, n, 0, rgb_dc=rgb)
    scene = ExplicitScene(means, scales, quats, opacity, sh, 0)
    W = H = 128
    fx = focal_for_fov(W)
    view = View(W, H, fx, fx, 64.0, 64.0, np.eye(3, dtype=np.float32),
                np.array([0.0, 0.0, 3.0], np.float32))
    wl = Workload("c0", scene, [view])
    wl.targets = make_targets(wl, seed=100 + 0, depth_range=(2.5, 3.5))
    return wl


def _box_surface_points(rng, n, boxes, ground, z_top_box=True):
    """Area-weighted points on a ground rectangle and the facades/roofs of
    axis-aligned boxes.  boxes: (m, 6) = (cx, cy, sx, sy, h, _)."""
    gx0, gx1, gy0, gy1 = ground
    areas = [(gx1 - gx0) * (gy1 - gy0)]
    kinds = [("ground", None)]
    for b in boxes:
        cx, cy, sx, sy, h = b[:5]
        areas += [sx * h, sx * h, sy * h, sy * h]
        kinds += [("fy0", b), ("fy1", b), ("fx0", b), ("fx1", b)]
        if z_top_box:
            areas.append(sx * sy)
            kinds.append(("roof", b))
    areas = np.asarray(areas)
    counts = rng.multinomial(n, areas / areas.sum())
    pts = []
    for (kind, b), c in zip(kinds, counts):
        if c == 0:
            continue
        u = rng.uniform(0, 1, c)
        v = rng.uniform(0, 1, c)
        if kind == "ground":
            p = np.stack([gx0 + u * (gx1 - gx0), gy0 + v * (gy1 - gy0), np.zeros(c)], 1)
        else:
            cx, cy, sx, sy, h = b[:5]
            x0, x1, y0, y1 = cx - sx / 2, cx + sx / 2, cy - sy / 2, cy + sy / 2
            if kind == "fy0":
                p = np.stack([x0 + u * sx, np.full(c, y0), v * h], 1)
            elif kind == "fy1":
                p = np.stack([x0 + u * sx, np.full(c, y1), v * h], 1)
            elif kind == "fx0":
                p = np.stack([np.full(c, x0), y0 + u * sy, v * h], 1)
            elif kind == "fx1":
                p = np.stack([np.full(c, x1), y0 + u * sy, v * h], 1)
            else:
                p = np.stack([x0 + u * sx, y0 + v * sy, np.full(c, h)], 1)
        pts.append(p)
    return np.concatenate(pts, 0)


def make_c1(seed: int = 1, n: int = 1_000_000) -> Workload:
    """C1: street scene, 1,000,000 Gaussians, SH degree 3, one 1920x1080 view."""
    rng = np.random.default_rng(seed)
    n_struct = int(round(0.7 * n))
    m = 30
    boxes = np.zeros((m, 6))
    boxes[:, 0:2] = rng.uniform(10, 90, (m, 2))
    boxes[:, 2:4] = rng.uniform(5, 15, (m, 2))
    boxes[:, 4] = rng.uniform(5, 30, m)
    struct = _box_surface_points(rng, n_struct, boxes, (0, 100, 0, 100))
    struct += rng.normal(0.0, 0.01, struct.shape)
    free = rng.uniform([0, 0, 0], [100, 100, 30], (n - n_struct, 3))
    means = np.concatenate([struct, free], 0).astype(np.float32)
    means = means[rng.permutation(n)]
    scales, quats, opacity, sh = _explicit_attrs(rng, n, 3)
    scene = ExplicitScene(means, scales, quats, opacity, sh, 3)
    view = look_at((50.0, -40.0, 35.0), (50.0, 50.0, 0.0), 1920, 1080)
    wl = Workload("c1", scene, [view])
    wl.targets = make_targets(wl, seed=100 + 1, depth_range=(20.0, 120.0))
    return wl


# --------------------------------------------------------------------------
# voxel anchors (Sec. 3.2, Eq. 2)
# --------------------------------------------------------------------------
def voxelise_levels(rng, points, delta, per_level):
    """Snap points to grids delta/2^k (Eq. 2) and subsample each level's
    unique grid points to per_level[k] anchors.  Returns (x, level)."""
    xs, levels = [], []
    for k, want in enumerate(per_level):
        size = delta / (2 ** k)
        g = np.round(points / size).astype(np.int64)
        g -= g.min(axis=0)
        span = g.max(axis=0) + 1
        code = (g[:, 0] * span[1] + g[:, 1]) * span[2] + g[:, 2]
        _, first = np.unique(code, return_index=True)
        if first.size < want:
            raise ValueError(f"level {k}: only {first.size} voxels, need {want}")
        pick = np.sort(rng.choice(first, want, replace=False))
        xs.append(np.round(points[pick] / size) * size)
        levels.append(np.full(want, k, np.uint8))
    return np.concatenate(xs, 0), np.concatenate(levels, 0)


def _anchor_attrs(rng, x, level, delta, d_max, n_levels=4):
    a = x.shape[0]
    size = (delta / (2.0 ** level.astype(np.float64)))[:, None]
    l = np.repeat(size, 3, axis=1).astype(np.float32)
    O = rng.normal(0.0, 0.5, (a, N_OFFSETS, 3)).astype(np.float32)
    F = rng.standard_normal((a, FEAT_DIM)).astype(np.float32)
    lim1 = 1.0 / np.sqrt(MLP_IN)
    lim2 = 1.0 / np.sqrt(MLP_HIDDEN)
    W1 = rng.uniform(-lim1, lim1, (MLP_IN, MLP_HIDDEN)).astype(np.float32)
    b1 = rng.uniform(-lim1, lim1, MLP_HIDDEN).astype(np.float32)
    W2 = rng.uniform(-lim2, lim2, (MLP_HIDDEN, MLP_OUT)).astype(np.float32)
    b2 = rng.uniform(-lim2, lim2, MLP_OUT).astype(np.float32)
    return AnchorScene(x.astype(np.float32), l, O, F, level.astype(np.uint8),
                       bf16_bits(W1), b1, bf16_bits(W2), b2, n_levels,
                       float(np.float32(d_max)))


def _split_counts(total, ratios=(1, 4, 16, 64)):
    r = np.asarray(ratios, np.float64)
    c = np.floor(total * r / r.sum()).astype(np.int64)
    c[-1] += total - c.sum()
    return c.tolist()


def make_city_block(seed, n_anchor, delta, n_boxes=40, n_points=None):
    """Anchors over a 200x200x50 m city block (C2, C3)."""
    rng = np.random.default_rng(seed)
    boxes = np.zeros((n_boxes, 6))
    boxes[:, 2:4] = rng.uniform(10, 30, (n_boxes, 2))
    boxes[:, 0:2] = rng.uniform(20, 180, (n_boxes, 2))
    boxes[:, 4] = rng.uniform(10, 50, n_boxes)
    per_level = _split_counts(n_anchor)
    if n_points is None:
        n_points = 12 * n_anchor
    pts = _box_surface_points(rng, n_points, boxes, (0, 200, 0, 200))
    x, level = voxelise_levels(rng, pts, delta, per_level)
    return _anchor_attrs(rng, x, level, delta, 400.0)


def make_aerial_tile(seed, n_anchor=2_000_000, delta=8.0, n_points=None):
    """Anchors over a 1x1 km aerial tile with log-normal building heights (C4)."""
    rng = np.random.default_rng(seed)
    cells = [(i, j) for i in range(20) for j in range(20)]
    boxes = []
    for (i, j) in cells:
        if rng.uniform() < 0.8:
            sx, sy = rng.uniform(15, 40, 2)
            h = float(np.exp(rng.normal(3.0, 0.5)))
            boxes.append((i * 50 + 25, j * 50 + 25, sx, sy, h, 0))
    boxes = np.asarray(boxes)
    per_level = _split_counts(n_anchor)
    if n_points is None:
        n_points = 10 * n_anchor
    pts = _box_surface_points(rng, n_points, boxes, (0, 1000, 0, 1000))
    x, level = voxelise_levels(rng, pts, delta, per_level)
    return _anchor_attrs(rng, x, level, delta, 2400.0)


def _ring_views(rng, n_views, centre, res_fn, radius, alt, look_box):
    views = []
    for i in range(n_views):
        ang = rng.uniform(0, 2 * np.pi)
        rad = rng.uniform(*radius)
        h = rng.uniform(*alt)
        pos = (centre[0] + rad * np.cos(ang), centre[1] + rad * np.sin(ang), h)
        tgt = (rng.uniform(*look_box), rng.uniform(*look_box), 0.0)
        W, H = res_fn(rng)
        views.append(look_at(pos, tgt, W, H))
    return views


def make_c2(seed: int = 2, n_anchor: int = 200_000, n_views: int = 8) -> Workload:
    """C2: 200k anchors (2M Gaussians), 8 views of uneven resolution."""
    scene = make_city_block(seed, n_anchor, 6.4)
    rng = np.random.default_rng(10 + seed)

    def res(r):
        s = r.uniform(0.5, 1.0)
        return 2 * int(round(960 * s)), 2 * int(round(540 * s))

    views = _ring_views(rng, n_views, (100.0, 100.0), res, (60, 250), (20, 150), (50, 150))
    wl = Workload("c2", scene, views)
    wl.targets = make_targets(wl, seed=100 + seed, depth_range=(30.0, 300.0))
    return wl


def make_c2_pairs(seed: int = 2, n_anchor: int = 200_000, n_pairs: int = 4) -> Workload:
    """The C2 scene seen by n_pairs pairs of nearby 1920x1080 cameras (views
    2i, 2i + 1 a few metres apart, aimed at the same point): the batch
    pairing of the geometric loss's training step."""
    scene = make_city_block(seed, n_anchor, 6.4)
    rng = np.random.default_rng(20 + seed)
    views = []
    for _ in range(n_pairs):
        ang = rng.uniform(0, 2 * np.pi)
        rad = rng.uniform(80, 160)
        h = rng.uniform(40, 120)
        pos = np.array([100.0 + rad * np.cos(ang), 100.0 + rad * np.sin(ang), h])
        tgt = (rng.uniform(70, 130), rng.uniform(70, 130), 0.0)
        step = rng.normal(0.0, 1.0, 3)
        step *= rng.uniform(2.0, 5.0) / np.linalg.norm(step)
        views.append(look_at(tuple(pos), tgt, 1920, 1080))
        views.append(look_at(tuple(pos + step), tgt, 1920, 1080))
    return Workload("c2_pairs", scene, views)


def make_c3(seed: int = 3, n_anchor: int = 600_000, n_views: int = 4) -> Workload:
    """C3: 600k anchors (6M Gaussians), 4 views at 3840x2160."""
    scene = make_city_block(seed, n_anchor, 4.0)
    rng = np.random.default_rng(10 + seed)
    views = _ring_views(rng, n_views, (100.0, 100.0), lambda r: (3840, 2160),
                        (60, 250), (20, 150), (50, 150))
    wl = Workload("c3", scene, views)
    wl.targets = make_targets(wl, seed=100 + seed, depth_range=(30.0, 300.0))
    return wl


def make_c4(seed: int = 4, n_anchor: int = 2_000_000, n_views: int = 16) -> Workload:
    """C4: 2M anchors (20M Gaussians) over 1x1 km, 16 nadir/oblique views."""
    scene = make_aerial_tile(seed, n_anchor)
    rng = np.random.default_rng(10 + seed)
    views = []
    centres = [125.0, 375.0, 625.0, 875.0]
    k = 0
    for gy in centres:
        for gx in centres:
            if k >= n_views:
                break
            alt = rng.uniform(150, 300)
            if k % 2 == 0:
                yaw = rng.uniform(0, 2 * np.pi)
                views.append(look_at((gx, gy, alt), (gx, gy, 0.0), 1600, 1200,
                                     yaw_hint=yaw))
            else:
                yaw = np.deg2rad(90.0 * rng.integers(0, 4) + rng.uniform(-10, 10))
                dx, dy = np.cos(yaw) * alt, np.sin(yaw) * alt   # 45 deg pitch
                views.append(look_at((gx, gy, alt), (gx + dx, gy + dy, 0.0), 1600, 1200))
            k += 1
    wl = Workload("c4", scene, views)
    wl.targets = make_targets(wl, seed=100 + seed, depth_range=(150.0, 450.0))
    return wl


def make_targets(wl: Workload, seed: int, depth_range=(1.0, 10.0)) -> dict:
    """Seeded L1 targets per view: rgb ~ U(0,1), unbiased depth ~ U(range),
    camera-facing unit normals (negative camera z)."""
    rng = np.random.default_rng(seed)
    rgb, depth, normal = [], [], []
    for v in wl.views:
        npx = v.width * v.height
        rgb.append(rng.uniform(0, 1, (3, npx)).astype(np.float32))
        depth.append(rng.uniform(*depth_range, npx).astype(np.float32))
        n = rng.standard_normal((3, npx))
        n[2] = -np.abs(n[2])
        n /= np.linalg.norm(n, axis=0, keepdims=True)
        normal.append(n.astype(np.float32))
    return dict(rgb=rgb, depth=depth, normal=normal)


def make(config: int, **kw) -> Workload:
    return [make_c0, make_c1, make_c2, make_c3, make_c4][config](**kw)


# --------------------------------------------------------------------------
# tiny scenes for tests
# --------------------------------------------------------------------------
def make_small_explicit(seed, n=40, width=48, height=40, sh_degree=0,
                        spread=0.5, log_scale=-2.5) -> Workload:
    """A small explicit scene whose Gaussians cover several tiles and a
    ragged image border; used by oracle and parity tests."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-spread, spread, (n, 3)).astype(np.float32)
    scales = np.exp(rng.normal(log_scale, 0.4, (n, 3))).astype(np.float32)
    quats = random_quats(rng, n)
    opacity = sigmoid(rng.standard_normal(n)).astype(np.float32)
    if sh_degree == 0:
        rgb = rng.uniform(0, 1, (n, 3))
        sh = ((rgb - 0.5) / (0.5 / np.sqrt(np.pi))).astype(np.float32)[:, None, :]
    else:
        sh = rng.normal(0, 0.3, (n, (sh_degree + 1) ** 2, 3)).astype(np.float32)
        sh[:, 0, :] += rng.uniform(-0.5, 0.5, (n, 3)).astype(np.float32)
    scene = ExplicitScene(means, scales, quats, opacity, sh, sh_degree)
    fx = focal_for_fov(width)
    view = View(width, height, fx, fx, width / 2.0, height / 2.0,
                np.eye(3, dtype=np.float32), np.array([0.0, 0.0, 2.5], np.float32))
    wl = Workload(f"small{seed}", scene, [view])
    wl.targets = make_targets(wl, seed=1000 + seed, depth_range=(2.0, 3.0))
    return wl


def head_layout(offset_mode, decoder_heads, n=N_OFFSETS):
    """(first attribute, width) per decoder head, and the decoder's output
    count per Gaussian: one shared head, or one head per attribute group
    (opacity 1, colour 3, scale and quaternion 7, decoded offsets 3)."""
    go = GAUSS_OUT + 3 if offset_mode else GAUSS_OUT
    if decoder_heads == 1:
        return [(0, go)], go
    groups = [(0, 1), (1, 3), (4, 7)] + ([(GAUSS_OUT, 3)] if offset_mode else [])
    return groups, go


def attribute_columns(offset_mode, decoder_heads, m, n=N_OFFSETS):
    """Decoder output columns of attribute m of Gaussians 0..n-1: head h
    owns the n * width columns from n * first, Gaussian k's attribute
    first + j at n * first + k * width + j."""
    for first, width in head_layout(offset_mode, decoder_heads, n)[0]:
        if first <= m < first + width:
            return n * first + np.arange(n) * width + (m - first)
    raise ValueError(m)


def decoder_variant(rng, scene, offset_mode=0, decoder_heads=1):
    """Fresh decoder weights for a variant: W1 36 x 32H, W2 32 x n*G with the
    head-grouped columns, uniform(+-1/sqrt(fan-in)) like the shared
    decoder; decoded offsets get biases of the table's spread and weights
    at half scale."""
    heads, go = head_layout(offset_mode, decoder_heads)
    n = scene.O.shape[1]
    hid = MLP_HIDDEN * len(heads)
    lim1, lim2 = 1.0 / np.sqrt(MLP_IN), 1.0 / np.sqrt(MLP_HIDDEN)
    W1 = rng.uniform(-lim1, lim1, (MLP_IN, hid)).astype(np.float32)
    b1 = rng.uniform(-lim1, lim1, hid).astype(np.float32)
    W2 = rng.uniform(-lim2, lim2, (MLP_HIDDEN, n * go)).astype(np.float32)
    b2 = rng.uniform(-lim2, lim2, n * go).astype(np.float32)
    if offset_mode:
        for c in range(3):
            cols = attribute_columns(offset_mode, decoder_heads, GAUSS_OUT + c, n)
            W2[:, cols] *= 0.5
            b2[cols] = rng.normal(0.0, 0.4, n).astype(np.float32)
    scene.W1_bits, scene.b1 = bf16_bits(W1), b1
    scene.W2_bits, scene.b2 = bf16_bits(W2), b2
    scene.offset_mode, scene.decoder_heads = int(offset_mode), int(decoder_heads)


def make_small_anchor(seed, n_anchor=60, n_views=2, sizes=((40, 32), (24, 36)),
                      d_max=12.0, opacity_act=0, offset_mode=0, decoder_heads=1) -> Workload:
    """A small anchor scene with two LoD levels and views of different
    sizes at different distances.  opacity_act = 1 selects the tanh opacity
    with non-positive opacities masked; the opacity biases are then spread
    around zero so that about half of the Gaussians are masked.
    offset_mode = 1 (decoded offsets) or decoder_heads = 3 (one MLP per
    attribute group) draw decoder weights of that shape."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, (n_anchor, 3)).astype(np.float32)
    x[:, 2] *= 0.3
    level = rng.integers(0, 3, n_anchor).astype(np.uint8)
    delta = 0.4
    scene = _anchor_attrs(rng, x, level, delta, d_max, n_levels=3)
    # keep the decoded Gaussians small relative to the views
    scene.O[:] = (scene.O * 0.8).astype(np.float32)
    if offset_mode or decoder_heads != 1:
        decoder_variant(np.random.default_rng(seed + 7000), scene, offset_mode, decoder_heads)
    if opacity_act:
        scene.opacity_act = int(opacity_act)
        n_off = scene.O.shape[1]
        cols = attribute_columns(scene.offset_mode, scene.decoder_heads, 0, n_off)
        scene.b2[cols] = rng.normal(0.0, 0.8, n_off).astype(np.float32)
    views = []
    for i in range(n_views):
        W, H = sizes[i % len(sizes)]
        dist = 2.5 + 2.0 * i
        ang = rng.uniform(0, 2 * np.pi)
        pos = (0.3 * np.cos(ang), 0.3 * np.sin(ang), dist)
        views.append(look_at(pos, (0.0, 0.0, 0.0), W, H, yaw_hint=ang))
    wl = Workload(f"small_anchor{seed}", scene, views)
    wl.targets = make_targets(wl, seed=2000 + seed, depth_range=(2.0, 6.0))
    return wl


def make_view_pairs(seed, n=3000, n_pairs=2, width=96, height=80) -> Workload:
    """Explicit Gaussians on a tilted, slightly rough plane seen by pairs of
    nearby cameras (views 2i, 2i+1), for the batch geometric loss: each
    pair's views overlap in most of their pixels."""
    rng = np.random.default_rng(seed)
    uv = rng.uniform(-1.0, 1.0, (n, 2))
    z = 0.25 * uv[:, 0] - 0.15 * uv[:, 1] + rng.normal(0.0, 0.02, n)
    means = np.stack([uv[:, 0], uv[:, 1], z], 1).astype(np.float32)
    scales = np.exp(rng.normal(-3.2, 0.3, (n, 3))).astype(np.float32)
    scales[:, 2] *= 0.2                       # flat splats, normals along the plane's
    quats = random_quats(rng, n) * 0.0
    quats[:, 0] = 1.0
    quats += rng.normal(0.0, 0.05, quats.shape).astype(np.float32)
    opacity = sigmoid(rng.normal(1.5, 0.5, n)).astype(np.float32)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    _, _, _, sh = _explicit_attrs(rng, n, 0, rgb_dc=rgb)
    scene = ExplicitScene(means, scales, quats.astype(np.float32), opacity, sh, 0)
    views = []
    for p in range(n_pairs):
        base = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), rng.uniform(2.6, 3.0)])
        for _ in range(2):
            pos = base + rng.normal(0.0, 0.06, 3)
            views.append(look_at(pos, rng.uniform(-0.1, 0.1, 3), width, height, fov_deg=50.0,
                                 yaw_hint=float(rng.uniform(0, 0.2))))
    wl = Workload("pairs", scene, views)
    wl.targets = make_targets(wl, seed=seed + 100, depth_range=(2.0, 3.5))
    return wl


def patch_centres(seed, views, n_patch, patch=7) -> np.ndarray:
    """Uniform integer patch centres, (n_views // 2, n_patch, 2) as (x, y), in
    each pair's second view, keeping the whole patch inside the image."""
    rng = np.random.default_rng(seed)
    h = patch // 2
    out = np.zeros((len(views) // 2, n_patch, 2), np.int32)
    for i in range(len(views) // 2):
        v = views[2 * i + 1]
        out[i, :, 0] = rng.integers(h, int(v.width) - h, n_patch)
        out[i, :, 1] = rng.integers(h, int(v.height) - h, n_patch)
    return out


# ---------------------------------------------------------------------------
# Depth-prior inputs (Sec. 3.4, Step 2): dense pseudo depths known only up to
# a per-view scale and shift, sparse points on the surfaces, nearby views.

@dataclass
class DepthPriorInputs:
    views: list
    prior: list             # per view (H*W,) f32 pseudo depth, 0 = no prior
    points: np.ndarray      # (N, 3) f32 sparse points (surface samples + outliers)
    nearby: list            # per view: index of its nearby view
    depth: list             # per view (H*W,) f64 true z-depth, 0 = nothing hit
    scale_shift: np.ndarray  # (B, 2) the (s, t) the prior was made with


def raycast_boxes(view, boxes):
    """True z-depth of every pixel of `view` on the ground plane z = 0 and
    the axis-aligned boxes (cx, cy, sx, sy, h) standing on it; 0 where the
    ray hits nothing.  Pixel rays are scaled to camera z = 1, so the ray
    parameter of a hit is its z-depth."""
    W, H = int(view.width), int(view.height)
    R = np.asarray(view.R, np.float64)
    t = np.asarray(view.t, np.float64)
    c = -R.T @ t
    J, I = np.divmod(np.arange(W * H), W)
    dc = np.stack([(I + 0.5 - view.cx) / view.fx, (J + 0.5 - view.cy) / view.fy, np.ones(W * H)])
    d = R.T @ dc                                                     # world ray directions
    with np.errstate(divide="ignore", invalid="ignore"):
        best = np.where(d[2] < 0, -c[2] / d[2], np.inf)
        inv = 1.0 / d
        for b in boxes:
            lo = np.array([b[0] - b[2] / 2, b[1] - b[3] / 2, 0.0])
            hi = np.array([b[0] + b[2] / 2, b[1] + b[3] / 2, b[4]])
            t1 = (lo[:, None] - c[:, None]) * inv
            t2 = (hi[:, None] - c[:, None]) * inv
            tn = np.nanmax(np.minimum(t1, t2), axis=0)
            tf = np.nanmin(np.maximum(t1, t2), axis=0)
            hit = (tf >= tn) & (tn > 0)
            best = np.where(hit & (tn < best), tn, best)
    return np.where(np.isfinite(best), best, 0.0)


def make_depth_prior(seed=5, n_pairs=4, width=1920, height=1080, n_points=1_000_000,
                     n_boxes=40, outliers=0.05, noise=0.01, blob_frac=0.05, sizes=None):
    """Pairs of nearby cameras (2-5 m apart, aimed at one point) over a
    200x200 m block of boxes.  Per view the pseudo depth is
    (z (1 + noise N(0,1)) - t) / s with s in [0.5, 2], t in [-5, 5]; square
    blobs covering about `blob_frac` of the pixels carry a 25 % depth error
    (the inconsistent regions the filter is for); sky has no prior.  The
    sparse points are true surface points of random pixels with 2 cm noise
    plus `outliers` of uniform points in the block.  `sizes` (one (W, H) per
    view) overrides width x height for uneven batches."""
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = [(width, height)] * (2 * n_pairs)
    boxes = np.zeros((n_boxes, 5))
    boxes[:, 0:2] = rng.uniform(20, 180, (n_boxes, 2))
    boxes[:, 2:4] = rng.uniform(10, 30, (n_boxes, 2))
    boxes[:, 4] = rng.uniform(10, 50, n_boxes)
    views, nearby = [], []
    for k in range(n_pairs):
        ang = rng.uniform(0, 2 * np.pi)
        rad = rng.uniform(80, 160)
        h = rng.uniform(40, 120)
        pos = np.array([100.0 + rad * np.cos(ang), 100.0 + rad * np.sin(ang), h])
        tgt = (rng.uniform(70, 130), rng.uniform(70, 130), 0.0)
        step = rng.normal(0.0, 1.0, 3)
        step *= rng.uniform(2.0, 5.0) / np.linalg.norm(step)
        views.append(look_at(tuple(pos), tgt, *sizes[2 * k]))
        views.append(look_at(tuple(pos + step), tgt, *sizes[2 * k + 1]))
        nearby += [2 * k + 1, 2 * k]
    depth, prior = [], []
    st = np.stack([rng.uniform(0.5, 2.0, len(views)), rng.uniform(-5.0, 5.0, len(views))], 1)
    for v, view in enumerate(views):
        z = raycast_boxes(view, boxes)
        depth.append(z)
        W, H = int(view.width), int(view.height)
        zn = z * (1.0 + noise * rng.standard_normal(z.size))
        err = np.zeros((H, W), bool)
        side = max(2, int(0.05 * min(W, H)))
        for _ in range(int(blob_frac * W * H / side ** 2)):
            i0, j0 = rng.integers(0, W - side + 1), rng.integers(0, H - side + 1)
            err[j0:j0 + side, i0:i0 + side] = True
        zn = np.where(err.ravel(), zn * 1.25, zn)
        p = (zn - st[v, 1]) / st[v, 0]
        prior.append(np.where(z > 0, p, 0.0).astype(np.float32))
    n_out = int(outliers * n_points)
    n_in = n_points - n_out
    pts = []
    vid = rng.integers(0, len(views), n_in)
    for v, view in enumerate(views):
        m = int((vid == v).sum())
        hitpix = np.flatnonzero(depth[v] > 0)
        pix = hitpix[rng.integers(0, hitpix.size, m)]
        W = int(view.width)
        J, I = np.divmod(pix, W)
        z = depth[v][pix]
        pc = np.stack([(I + 0.5 - view.cx) / view.fx * z, (J + 0.5 - view.cy) / view.fy * z, z])
        R = np.asarray(view.R, np.float64)
        pw = (R.T @ (pc - np.asarray(view.t, np.float64)[:, None])).T
        pts.append(pw + rng.normal(0.0, 0.02, pw.shape))
    pts.append(np.stack([rng.uniform(0, 200, n_out), rng.uniform(0, 200, n_out),
                         rng.uniform(0, 50, n_out)], 1))
    points = np.concatenate(pts).astype(np.float32)
    points = points[rng.permutation(len(points))]
    return DepthPriorInputs(views, prior, points, nearby, depth, st)
