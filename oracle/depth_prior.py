"""Depth-prior recovery and filtering (Sec. 3.4, Step 2; row f4) -- oracle,
test infrastructure only.

The paper scales a monocular pseudo depth D_p to the scene with the least-
squares scale and shift against the sparse points P, then removes the
pixels whose re-projection error E between the target view and a nearby
view exceeds tau_d (tau_d = 1, Sec. 4), giving the filtered prior D~_f that
the depth L1 regularises against (its removed pixels are the zeros of the
depth mask).  Readings of what the paper leaves open:

  * depths are z-depths (camera-space z), like the rendered unbiased depth
    D^ of Eq. 7; a prior value <= 0 means "no prior" at that pixel;
  * scale / shift, per view: every point of P in front of the camera
    (z > z_near) whose projection falls inside the image gives a pair
    (d_i, z_i), d_i the prior at the pixel containing the projection (only
    if d_i > 0) and z_i the point's camera depth; (s, t) minimise
    sum (s d_i + t - z_i)^2 through the 2x2 normal equations; fewer than two
    pairs or a singular system leave (s, t) = (1, 0); the aligned prior is
    s D_p + t where D_p > 0 and 0 elsewhere;
  * re-projection error, for pixel p = (i + 1/2, j + 1/2) of view v with
    a finite depth d > 0 and its nearby view u: X = d K_v^-1 [p, 1] (camera v) is
    moved to camera u; if it is in front (z > z_near) and projects to q
    inside u's image, the depth d_u of u at the pixel containing q lifts q
    to Y = d_u K_u^-1 [q, 1] (camera u), which goes back to camera v and
    projects to p'; E = |p' - p|.  p is kept iff d_u > 0, Y is in front of
    v and E < tau_d; a removed pixel's filtered depth is 0;
  * float64 in a fixed operation order.  Decisions: the pixel containing a
    projection, the two in-front tests and E < tau_d; a pixel is flagged
    fragile when a projection is within FRAG (relative) of a pixel edge, a
    depth within FRAG of the near plane, or E^2 within FRAG of tau_d^2 --
    there another evaluation order of the same float64 arithmetic may
    decide the other way.
"""
import numpy as np

from .project import view_arrays

FRAG = 1e-9


def _cam(view):
    V = view_arrays(view)
    return (np.asarray(V["R"], np.float64), np.asarray(V["t"], np.float64), float(V["fx"]),
            float(V["fy"]), float(V["cx"]), float(V["cy"]), int(V["W"]), int(V["H"]),
            float(V["z_near"]))


def align_scale_shift(prior, points, views):
    """Per view (s, t) and the aligned prior.  prior: list of (H*W,) arrays
    (row-major), points: (N, 3) world positions.  Returns (st (B, 2),
    aligned list, n_pairs (B,))."""
    P = np.asarray(points, np.float64)
    st = np.zeros((len(views), 2))
    aligned, npairs = [], np.zeros(len(views), np.int64)
    for v, view in enumerate(views):
        R, t, fx, fy, cx, cy, W, H, zn = _cam(view)
        pc = [((R[k, 0] * P[:, 0] + R[k, 1] * P[:, 1]) + R[k, 2] * P[:, 2]) + t[k] for k in range(3)]
        z = pc[2]
        front = z > zn
        zs = np.where(front, z, 1.0)
        u = (fx * pc[0]) / zs + cx
        w = (fy * pc[1]) / zs + cy
        inside = front & (u >= 0.0) & (u < W) & (w >= 0.0) & (w < H)
        iu = np.floor(np.where(inside, u, 0.0)).astype(np.int64)
        iw = np.floor(np.where(inside, w, 0.0)).astype(np.int64)
        D = np.asarray(prior[v], np.float64)
        d = D[iw * W + iu]
        ok = inside & (d > 0.0)
        d, zz = d[ok], z[ok]
        n = float(ok.sum())
        npairs[v] = int(n)
        Sd, Sz, Sdd, Sdz = d.sum(), zz.sum(), (d * d).sum(), (d * zz).sum()
        det = n * Sdd - Sd * Sd
        if n >= 2 and det > 0.0:
            s = (n * Sdz - Sd * Sz) / det
            sh = (Sdd * Sz - Sd * Sdz) / det
        else:
            s, sh = 1.0, 0.0
        st[v] = (s, sh)
        aligned.append(np.where(D > 0.0, s * D + sh, 0.0))
    return st, aligned, npairs


def reprojection_filter(depth, views, nearby, tau=1.0):
    """Filtered depth per view and the fragile mask.  depth: list of (H*W,)
    z-depth maps; nearby[v]: index of the nearby view of view v (or -1: no
    filter, every pixel kept).  Returns (filtered list, fragile list,
    error list (inf where not reprojected))."""
    with np.errstate(invalid="ignore", over="ignore"):     # inf / NaN depths are no depth
        return _filter(depth, views, nearby, tau)


def _filter(depth, views, nearby, tau):
    out, frag, errs = [], [], []
    cams = [_cam(v) for v in views]
    for v in range(len(views)):
        R, t, fx, fy, cx, cy, W, H, zn = cams[v]
        D = np.asarray(depth[v], np.float64)
        if nearby[v] < 0:
            out.append(np.where(D > 0.0, D, 0.0))
            frag.append(np.zeros(D.size, bool))
            errs.append(np.zeros(D.size))
            continue
        Ru, tu, fxu, fyu, cxu, cyu, Wu, Hu, znu = cams[nearby[v]]
        Du = np.asarray(depth[nearby[v]], np.float64)
        J, I = np.divmod(np.arange(W * H), W)
        px, py = I + 0.5, J + 0.5
        d = D
        # camera v -> world: X_w = R^T (X_c - t)
        xc = [d * ((px - cx) / fx), d * ((py - cy) / fy), d]
        xw = [((R[0, k] * (xc[0] - t[0]) + R[1, k] * (xc[1] - t[1])) + R[2, k] * (xc[2] - t[2]))
              for k in range(3)]
        yc = [((Ru[k, 0] * xw[0] + Ru[k, 1] * xw[1]) + Ru[k, 2] * xw[2]) + tu[k] for k in range(3)]
        front = (d > 0.0) & (d < np.inf) & (yc[2] > znu)
        zs = np.where(front, yc[2], 1.0)
        qx = (fxu * yc[0]) / zs + cxu
        qy = (fyu * yc[1]) / zs + cyu
        inside = front & (qx >= 0.0) & (qx < Wu) & (qy >= 0.0) & (qy < Hu)
        near = (d > 0.0) & (np.abs(yc[2] - znu) < FRAG * (np.abs(yc[2]) + znu))
        fr = near | (front & ((np.abs(qx - np.round(qx)) < FRAG * (np.abs(qx) + 1.0))
                              | (np.abs(qy - np.round(qy)) < FRAG * (np.abs(qy) + 1.0))))
        iq = np.floor(np.where(inside, qx, 0.0)).astype(np.int64)
        jq = np.floor(np.where(inside, qy, 0.0)).astype(np.int64)
        du = np.where(inside, Du[jq * Wu + iq], 0.0)
        ok = inside & (du > 0.0) & (du < np.inf)
        # camera u -> world -> camera v
        yc2 = [du * ((qx - cxu) / fxu), du * ((qy - cyu) / fyu), du]
        yw = [((Ru[0, k] * (yc2[0] - tu[0]) + Ru[1, k] * (yc2[1] - tu[1])) + Ru[2, k] * (yc2[2] - tu[2]))
              for k in range(3)]
        zc = [((R[k, 0] * yw[0] + R[k, 1] * yw[1]) + R[k, 2] * yw[2]) + t[k] for k in range(3)]
        fr |= ok & (np.abs(zc[2] - zn) < FRAG * (np.abs(zc[2]) + zn))
        ok = ok & (zc[2] > zn)
        zz = np.where(ok, zc[2], 1.0)
        ex = ((fx * zc[0]) / zz + cx) - px
        ey = ((fy * zc[1]) / zz + cy) - py
        e2 = ex * ex + ey * ey
        t2 = tau * tau
        keep = ok & (e2 < t2)
        fr |= ok & (np.abs(e2 - t2) < FRAG * (t2 + e2))
        out.append(np.where(keep, d, 0.0))
        frag.append(fr)
        errs.append(np.where(ok, np.sqrt(e2), np.inf))
    return out, frag, errs
