"""Projective TSDF fusion of rendered depth and colour (Sec. 4, mesh
reconstruction: the rendered views are fused into a truncated signed
distance volume, following the 3DMatch fusion it cites) -- oracle, test
infrastructure only.

Readings of what the paper leaves to the cited method:

  * the volume is a regular grid of nx x ny x nz voxels of edge `voxel`;
    voxel (i, j, k) is the point origin + voxel * (i, j, k) (grid points,
    no half-voxel shift); its index is i + nx (j + ny k);
  * per view, in the given order: the voxel moves to camera space
    (p = R X + t); it is seen if p_z > z_near and its projection
    (u, w) = (fx p_x / p_z + cx, fy p_y / p_z + cy) lies in [0, W) x [0, H);
    the depth d is the rendered z-depth at pixel (floor u, floor w); a
    finite d > 0 is an observation.  With the signed distance
    diff = d - p_z along the optical axis and the truncation mu, a voxel with
    diff > -mu is updated (voxels further behind the surface are occluded
    and left alone):
        f = min(1, diff / mu),  W' = W + 1,
        T' = (T W + f) / W',    C' = (C W + c) / W'  (c the pixel's RGB);
  * the running average makes the result independent of how views are
    batched, only of their order;
  * float64 throughout; decisions (in front, inside, the pixel, diff > -mu)
    are fragile within FRAG (relative) of their bound.
"""
import numpy as np

from .project import view_arrays

FRAG = 1e-9


def voxel_points(origin, voxel, dims, index=None):
    """World positions of the grid points, index i + nx (j + ny k): (N, 3),
    of every voxel or of the given indices."""
    nx, ny, nz = dims
    idx = np.arange(nx * ny * nz) if index is None else np.asarray(index, np.int64)
    i, j, k = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    o = np.asarray(origin, np.float64)
    return np.stack([o[0] + voxel * i, o[1] + voxel * j, o[2] + voxel * k], 1)


def integrate(origin, voxel, dims, trunc, views, depth, rgb=None, state=None, voxels=None):
    """Fuse the views in order.  depth: list of (H*W,) z-depth maps; rgb:
    list of (3, H*W) planar images or None.  state: (T, W, C) to continue
    from (C (3, N)), default T = 1, W = 0, C = 0.  voxels: optional indices
    of the voxels to compute (each voxel is independent), N = their count.
    Returns (T, W, C, fragile) with fragile a bool per voxel."""
    X = voxel_points(origin, float(voxel), dims, voxels)
    N = X.shape[0]
    if state is None:
        T, Wt, C = np.ones(N), np.zeros(N), np.zeros((3, N))
    else:
        T, Wt, C = (np.array(a, np.float64) for a in state)
    mu = float(trunc)
    frag = np.zeros(N, bool)
    for v, view in enumerate(views):
        V = view_arrays(view)
        R, t = V["R"], V["t"]
        p = [((R[k, 0] * X[:, 0] + R[k, 1] * X[:, 1]) + R[k, 2] * X[:, 2]) + t[k] for k in range(3)]
        z = p[2]
        front = z > V["z_near"]
        zs = np.where(front, z, 1.0)
        u = (V["fx"] * p[0]) / zs + V["cx"]
        w = (V["fy"] * p[1]) / zs + V["cy"]
        inside = front & (u >= 0.0) & (u < V["W"]) & (w >= 0.0) & (w < V["H"])
        frag |= np.abs(z - V["z_near"]) < FRAG * (np.abs(z) + V["z_near"])
        frag |= front & ((np.abs(u - np.round(u)) < FRAG * (np.abs(u) + 1.0))
                         | (np.abs(w - np.round(w)) < FRAG * (np.abs(w) + 1.0)))
        pix = np.floor(np.where(inside, w, 0.0)).astype(np.int64) * V["W"] + \
            np.floor(np.where(inside, u, 0.0)).astype(np.int64)
        D = np.asarray(depth[v], np.float64)
        d = np.where(inside, D[pix], 0.0)
        obs = inside & (d > 0.0) & (d < np.inf)
        diff = d - z
        upd = obs & (diff > -mu)
        frag |= obs & (np.abs(diff + mu) < FRAG * (np.abs(diff) + mu))
        f = np.minimum(1.0, diff / mu)
        w1 = Wt + 1.0
        T = np.where(upd, (T * Wt + f) / w1, T)
        if rgb is not None:
            col = np.asarray(rgb[v], np.float64)
            for ch in range(3):
                C[ch] = np.where(upd, (C[ch] * Wt + col[ch][pix]) / w1, C[ch])
        Wt = np.where(upd, w1, Wt)
    return T, Wt, C, frag
