"""EWA projection of 3-D Gaussians into one view, and its adjoint
(oracle, test infrastructure).

What is computed follows the 3DGS primitive of Sec. 3.1 (Eq. 1: alpha is
the opacity times the Gaussian evaluated with its projected covariance)
and the inputs the normal map and unbiased depth need (Sec. 3.3, Eqs. 6-7,
PGSR strategy).  Constants the paper leaves unstated are fixed here:

  * camera: p = R mu + t (OpenCV frame), culled unless p_z > z_near;
  * 2-D mean u = fx p_x / p_z + cx, w = fy p_y / p_z + cy;
  * Jacobian J of the perspective map with x/z, y/z clamped to 1.3 times
    the half field of view; Sigma_2 = J R Sigma R^T J^T + 0.3 I;
  * conic = Sigma_2^{-1}; radius r = ceil(3 sqrt(lambda_max(Sigma_2)));
  * pixel box: the pixels whose centre lies within r_x = min(r, e_x) of the
    2-D mean in x and r_y = min(r, e_y) in y, clipped to the image; culled
    if empty.  e_x = sqrt(2 ln(255 o) Sigma_2,xx) (e_y with Sigma_2,yy) is
    the reach along each axis of the ellipse where o exp(power) >= 1/255,
    so every pixel the compositor could draw inside the 3-sigma square is
    kept; a splat with o < 1/255 draws nothing;
  * depth key = IEEE binary32 bits of p_z rounded to nearest;
  * normal: the rotated axis of the smallest scale, in the camera frame,
    turned to face the camera; plane distance d = -n . p (>= 0);
  * colour: explicit Gaussians use max(0, SH(dir) k + 0.5) with dir the
    unit vector from the camera centre to mu; anchor Gaussians use the
    decoded colour.

Decision values (p, u, w, the box, the depth key) are computed in float64
with the fixed operation order written below, which the GPU path repeats
exactly; the continuous attributes are computed in float64 here.
"""
import numpy as np

from . import sh as shmod

DILATION = 0.3
GUARD = 1.3
FRAG = 1e-5          # relative margin below which a decision is fragile


def view_arrays(view):
    """float64 copies of a view's float32 parameters and its camera centre
    c = -R^T t (fixed order: ((R0j t0 + R1j t1) + R2j t2))."""
    R = np.asarray(view.R, np.float32).reshape(3, 3).astype(np.float64)
    t = np.asarray(view.t, np.float32).reshape(3).astype(np.float64)
    c = np.array([-((R[0, j] * t[0] + R[1, j] * t[1]) + R[2, j] * t[2]) for j in range(3)])
    f = lambda v: float(np.float32(v))   # noqa: E731
    return dict(R=R, t=t, c=c, W=int(view.width), H=int(view.height),
                fx=f(view.fx), fy=f(view.fy), cx=f(view.cx), cy=f(view.cy),
                z_near=f(view.z_near),
                bg=np.asarray(view.bg, np.float32).astype(np.float64))


def camera_point(R, t, m):
    """p_i = ((R_i0 m_0 + R_i1 m_1) + R_i2 m_2) + t_i, float64, no fused ops."""
    return np.stack([((R[i, 0] * m[:, 0] + R[i, 1] * m[:, 1]) + R[i, 2] * m[:, 2]) + t[i]
                     for i in range(3)], axis=1)


def quat_to_rot(qn):
    """Rotation matrix of a unit quaternion (w, x, y, z): (N, 3, 3)."""
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


def quat_to_rot_backward(qn, dR):
    """Adjoint of quat_to_rot: dR (N,3,3) -> d qn (N,4)."""
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    g = dR
    dw = 2 * (-z * g[:, 0, 1] + y * g[:, 0, 2] + z * g[:, 1, 0] - x * g[:, 1, 2]
              - y * g[:, 2, 0] + x * g[:, 2, 1])
    dx = 2 * (y * g[:, 0, 1] + z * g[:, 0, 2] + y * g[:, 1, 0] - 2 * x * g[:, 1, 1]
              - w * g[:, 1, 2] + z * g[:, 2, 0] + w * g[:, 2, 1] - 2 * x * g[:, 2, 2])
    dy = 2 * (-2 * y * g[:, 0, 0] + x * g[:, 0, 1] + w * g[:, 0, 2] + x * g[:, 1, 0]
              + z * g[:, 1, 2] - w * g[:, 2, 0] + z * g[:, 2, 1] - 2 * y * g[:, 2, 2])
    dz = 2 * (-2 * z * g[:, 0, 0] - w * g[:, 0, 1] + x * g[:, 0, 2] + w * g[:, 1, 0]
              - 2 * z * g[:, 1, 1] + y * g[:, 1, 2] + x * g[:, 2, 0] + y * g[:, 2, 1])
    return np.stack([dw, dx, dy, dz], 1)


MASK_TILES = 64     # boxes of 2 x 2 up to this many tiles carry a tile mask


def tile_mask(u, w, A, B, C, tau, x_lo, x_hi, y_lo, y_hi, tw, th, use, rel, du=0.0, dw=0.0):
    """Tiles of the pixel box that the drawable ellipse reaches (reading of
    the tile binning, Sec. 3.3; row f3's ellipse-tile culling): bit
    r * nx + c for tile row r and tile column c of the box, for the splats in
    `use` (boxes of at least two tile rows and columns and at most
    MASK_TILES tiles; a one-row or one-column box spans the ellipse's full
    extent along its other axis, so it keeps every tile).

    With d = p - (u, w) and the 2-D covariance [[A, B], [B, C]], a pixel
    centre p is drawable (alpha >= 1/255) iff d^T Sigma^-1 d <= 2 tau,
    tau = log(255 o).  At a fixed dy that ellipse spans
    dx in (B/C) dy -/+ sqrt((2 tau - dy^2 / C) det / C); over a strip of
    pixel-centre rows its left edge is convex in dy, with the minimum at
    the leftmost point dy = -B sqrt(2 tau / A) (the right edge mirrors it),
    so the strip's x-extent is the edge at that dy clamped into the strip.
    A tile of the row is kept iff the pixel-centre columns it shares with
    the box meet that extent.  The test is continuous, so a tile with a
    drawable pixel centre is never dropped.  Decisions are float64 in this
    operation order (the GPU evaluates the same expressions); a comparison
    closer than the float32 covariance can resolve (relative `rel`, times
    the conditioning of det), widened by the mean's error bound (du, dw
    pixels), marks the splat's tile set fragile.

    Returns (mask uint64, fragile bool, fragile-tile mask uint64) per splat:
    the third value has the bits of the tiles whose own test is that close."""
    n = u.size
    mask = np.zeros(n, np.uint64)
    frag = np.zeros(n, bool)
    fmask = np.zeros(n, np.uint64)
    idx = np.nonzero(use)[0]
    if idx.size == 0:
        return mask, frag, fmask
    u, w, A, B, C, tau = (np.asarray(a, np.float64)[idx] for a in (u, w, A, B, C, tau))
    rel = np.broadcast_to(np.asarray(rel, np.float64), (n,))[idx]
    du = np.broadcast_to(np.asarray(du, np.float64), (n,))[idx]
    dw = np.broadcast_to(np.asarray(dw, np.float64), (n,))[idx]
    xl_, xh_, yl_, yh_ = (np.asarray(a)[idx] for a in (x_lo, x_hi, y_lo, y_hi))
    tx0, tx1, ty0, ty1 = xl_ // tw, xh_ // tw, yl_ // th, yh_ // th
    nx, ny = tx1 - tx0 + 1, ty1 - ty0 + 1
    det = A * C - B * B
    t2 = 2.0 * tau
    ic = 1.0 / C
    ymax = np.sqrt(t2 * C)
    k = B * ic
    s = det * ic
    ye = B * np.sqrt(t2 / A)
    kappa = 1.0 + (A * C + B * B) / det
    m = np.zeros(idx.size, np.uint64)
    fm = np.zeros(idx.size, np.uint64)
    fr = np.zeros(idx.size, bool)
    one = np.uint64(1)
    for rr in range(int(ny.max())):
        live = rr < ny
        ty = ty0 + rr
        r0 = np.maximum(ty * th, yl_)
        r1 = np.minimum(ty * th + th - 1, yh_)
        lo = (r0 + 0.5) - w
        hi = (r1 + 0.5) - w
        dym = rel * kappa * (ymax + 1.0) + 1e-9 + dw
        rowfr = live & ((np.abs(lo - ymax) < dym) | (np.abs(hi + ymax) < dym))
        fr |= rowfr
        lo = np.maximum(lo, -ymax)
        hi = np.minimum(hi, ymax)
        row = live & (lo <= hi)
        dl = np.minimum(np.maximum(-ye, lo), hi)
        dr = np.minimum(np.maximum(ye, lo), hi)
        xl = u + (k * dl - np.sqrt(np.maximum(t2 - dl * dl * ic, 0.0) * s))
        xr = u + (k * dr + np.sqrt(np.maximum(t2 - dr * dr * ic, 0.0) * s))
        marg = rel * kappa * (np.abs(xl - u) + np.abs(xr - u) + np.sqrt(t2 * A) + 1.0) + 1e-9 + du
        for cc in range(int(nx.max())):
            on = row & (cc < nx)
            tx = tx0 + cc
            c0 = np.maximum(tx * tw, xl_)
            c1 = np.minimum(tx * tw + tw - 1, xh_)
            keep = on & ((c1 + 0.5) >= xl) & ((c0 + 0.5) <= xr)
            colfr = on & ((np.abs((c1 + 0.5) - xl) < marg) | (np.abs(xr - (c0 + 0.5)) < marg))
            fr |= colfr
            inbox = live & (cc < nx)
            bit = np.where(inbox, rr * nx + cc, 0).astype(np.uint64)
            m |= np.where(keep, np.left_shift(one, bit), np.uint64(0))
            fm |= np.where(colfr | (rowfr & inbox), np.left_shift(one, bit), np.uint64(0))
    mask[idx] = m
    frag[idx] = fr
    fmask[idx] = fm
    return mask, frag, fmask


def project(mu, scales, quats, opacity, view, tile, colour=None, sh=None, sh_degree=0,
            opacity_exact=True, mu_tol=None):
    """Project N Gaussians into one view.

    mu: (N,3) float64 centres (for explicit Gaussians the float32 inputs
    widened; for anchors x + O*l evaluated in float64).  scales (N,3),
    quats (N,4) raw (w,x,y,z), opacity (N,).  Colour is either given
    (N,3) or evaluated from sh (N,K,3).  tile = (tw, th).  opacity_exact:
    the GPU sees the same opacity (an input) rather than one it decoded
    itself in float32 (anchor Gaussians), which widens the fragile margin
    of the opacity-aware box.  mu_tol (N,3), optional: a bound on the
    error of the GPU's mean (decoded offsets); the decisions that depend on
    the mean widen their fragile margins by its image in pixels (du, dw)
    and the depth key may differ by ztol units in the last place.

    Returns a dict of per-Gaussian arrays; `valid` marks the splats that
    survive culling and touch at least one tile.
    """
    V = view_arrays(view)
    R, t, c = V["R"], V["t"], V["c"]
    W, H, fx, fy, cx, cy = V["W"], V["H"], V["fx"], V["fy"], V["cx"], V["cy"]
    tw, th = tile
    mu = np.asarray(mu, np.float64)
    n = mu.shape[0]
    s = np.asarray(scales, np.float64)
    q = np.asarray(quats, np.float64)
    o = np.asarray(opacity, np.float64)

    # ---- decision values, float64, fixed order --------------------------
    p = camera_point(R, t, mu)
    front = p[:, 2] > V["z_near"]
    pz = np.where(front, p[:, 2], 1.0)
    u = (fx * p[:, 0]) / pz + cx
    w = (fy * p[:, 1]) / pz + cy
    zbits = p[:, 2].astype(np.float32).view(np.uint32)
    if mu_tol is None:
        du = dw = np.zeros(n)
        ztol = np.zeros(n, np.int64)
    else:
        dp = np.asarray(mu_tol, np.float64) @ np.abs(R).T      # camera-frame error bound
        du = abs(fx) * (dp[:, 0] / pz + np.abs(p[:, 0]) * dp[:, 2] / (pz * pz))
        dw = abs(fy) * (dp[:, 1] / pz + np.abs(p[:, 1]) * dp[:, 2] / (pz * pz))
        ulp = np.spacing(np.abs(p[:, 2]).astype(np.float32)).astype(np.float64)
        ztol = np.where(front, np.ceil(dp[:, 2] / ulp) + 1, 0).astype(np.int64)

    # ---- EWA covariance --------------------------------------------------
    lim_x = (GUARD * W) / (2.0 * fx)
    lim_y = (GUARD * H) / (2.0 * fy)
    rx, ry = p[:, 0] / pz, p[:, 1] / pz
    clamp_x = (rx < -lim_x) | (rx > lim_x)
    clamp_y = (ry < -lim_y) | (ry > lim_y)
    txz = np.clip(rx, -lim_x, lim_x) * pz
    tyz = np.clip(ry, -lim_y, lim_y) * pz
    T0 = (fx / pz)[:, None] * R[0][None] - (fx * txz / pz ** 2)[:, None] * R[2][None]
    T1 = (fy / pz)[:, None] * R[1][None] - (fy * tyz / pz ** 2)[:, None] * R[2][None]
    qnorm = np.maximum(np.linalg.norm(q, axis=1), 1e-12)
    qn = q / qnorm[:, None]
    Rq = quat_to_rot(qn)
    M = Rq * s[:, None, :]
    V0 = np.einsum("nj,njk->nk", T0, M)
    V1 = np.einsum("nj,njk->nk", T1, M)
    A = np.sum(V0 * V0, 1) + DILATION
    B = np.sum(V0 * V1, 1)
    Cc = np.sum(V1 * V1, 1) + DILATION
    det = A * Cc - B * B
    ok = front & (det > 0)
    dets = np.where(ok, det, 1.0)
    conic = np.stack([Cc / dets, -B / dets, A / dets], 1)
    mid = 0.5 * (A + Cc)
    half = 0.5 * (A - Cc)
    lam = mid + np.sqrt(half * half + B * B)
    r3 = 3.0 * np.sqrt(lam)
    r3 = np.where(ok, r3, 0.0)
    r = np.ceil(np.minimum(r3, 1 << 20))
    frag_r = ok & (np.abs(r3 - np.round(r3)) < FRAG * np.maximum(r3, 1.0))

    # ---- opacity-aware reach per axis -------------------------------------
    tau = np.log(np.maximum(255.0 * o, 1e-300))
    ok = ok & (tau >= 0.0)
    frag_tau = np.abs(255.0 * o - 1.0) < FRAG
    tau0 = np.maximum(tau, 0.0)
    ex = np.sqrt(2.0 * tau0 * np.where(ok, A, 0.0))
    ey = np.sqrt(2.0 * tau0 * np.where(ok, Cc, 0.0))
    rxp = np.minimum(r, ex)
    ryp = np.minimum(r, ey)

    # ---- pixel box (exact given rx, ry) ----------------------------------
    x_lo = np.ceil(u - (rxp + 0.5))
    x_hi = np.floor(u + (rxp - 0.5))
    y_lo = np.ceil(w - (ryp + 0.5))
    y_hi = np.floor(w + (ryp - 0.5))
    # a reach from the float32 covariance and opacity may move a box edge
    # across a pixel centre: fragile when an edge is that close to one
    # (relative error of the reach ~ dA/2A + (do/o)/(2 tau))
    rel = FRAG + (0.0 if opacity_exact else FRAG / (2.0 * np.maximum(tau0, 1e-3)))
    marg_x = rel * rxp + 1e-9 + du
    marg_y = rel * ryp + 1e-9 + dw
    def _near_int(e, m):
        return np.abs(e - np.round(e)) < m
    frag_ext = ok & (((ex <= r) & (_near_int(u - (rxp + 0.5), marg_x) | _near_int(u + (rxp - 0.5), marg_x)))
                     | ((ey <= r) & (_near_int(w - (ryp + 0.5), marg_y) | _near_int(w + (ryp - 0.5), marg_y)))
                     | (np.abs(ex - r) < marg_x) | (np.abs(ey - r) < marg_y))
    # box edges (x_lo, x_hi, y_lo, y_hi) that may sit one pixel further or
    # shorter on the GPU: a radius ceiling that may round the other way
    # moves the edges it binds (r - 1 < e); a reach within rounding of the
    # radius moves both edges of its axis; a reach-bound edge within rounding
    # of a pixel centre moves that edge
    rc = frag_r & front & (det > 0)
    tx_, ty_ = np.abs(ex - r) < marg_x, np.abs(ey - r) < marg_y
    mx = (rc & (ex > r - 1.0 - marg_x)) | tx_
    my = (rc & (ey > r - 1.0 - marg_y)) | ty_
    frag_edge = (front & (det > 0) & (tau >= 0.0))[:, None] & np.stack([
        mx | ((ex <= r) & _near_int(u - (rxp + 0.5), marg_x)),
        mx | ((ex <= r) & _near_int(u + (rxp - 0.5), marg_x)),
        my | ((ey <= r) & _near_int(w - (ryp + 0.5), marg_y)),
        my | ((ey <= r) & _near_int(w + (ryp - 0.5), marg_y))], 1)
    frag_box = frag_edge.any(axis=1)
    frag_r = frag_r | frag_ext | (front & (det > 0) & frag_tau)
    x_lo = np.clip(np.where(ok, x_lo, W), 0, W).astype(np.int64)
    x_hi = np.clip(np.where(ok, x_hi, -1), -1, W - 1).astype(np.int64)
    y_lo = np.clip(np.where(ok, y_lo, H), 0, H).astype(np.int64)
    y_hi = np.clip(np.where(ok, y_hi, -1), -1, H - 1).astype(np.int64)
    valid = ok & (x_lo <= x_hi) & (y_lo <= y_hi)

    # ---- normal and plane distance (PGSR, Eqs. 6-7) ---------------------
    Rc = np.einsum("ij,njk->nik", R, Rq)
    jstar = np.argmin(s, axis=1)
    nvec = Rc[np.arange(n), :, jstar]
    ndp = np.sum(nvec * p, 1)
    sign = np.where(ndp > 0, -1.0, 1.0)
    nvec = nvec * sign[:, None]
    d = -np.sum(nvec * p, 1)
    ssort = np.sort(s, axis=1)
    frag_axis = (ssort[:, 1] - ssort[:, 0]) < FRAG * ssort[:, 0]
    frag_flip = np.abs(ndp) < FRAG * np.linalg.norm(p, axis=1)
    # the other outcome of a near-tie axis (the next-smallest scale's axis,
    # turned to the camera) or orientation (the opposite normal)
    j2 = np.argsort(s, axis=1, kind="stable")[:, 1]
    n2 = Rc[np.arange(n), :, j2]
    n2 = n2 * np.where(np.sum(n2 * p, 1) > 0, -1.0, 1.0)[:, None]
    n_alt = np.where(frag_axis[:, None], n2, -nvec)
    d_alt = -np.sum(n_alt * p, 1)

    # ---- colour ----------------------------------------------------------
    frag_colour = np.zeros(n, bool)
    dirs = None
    if colour is None:
        k = np.asarray(sh, np.float64)
        dv = mu - c[None]
        dn = np.linalg.norm(dv, axis=1)
        dirs = dv / dn[:, None]
        Y = shmod.basis(dirs, sh_degree)
        raw = np.einsum("nk,nkc->nc", Y, k) + 0.5
        rgb = np.maximum(raw, 0.0)
        frag_colour = np.any(np.abs(raw) < FRAG, 1)
    else:
        raw = np.asarray(colour, np.float64)
        rgb = raw

    # ---- tiles -------------------------------------------------------------
    TX = -(-W // tw)
    TY = -(-H // th)
    tx0, tx1 = x_lo // tw, x_hi // tw
    ty0, ty1 = y_lo // th, y_hi // th
    ntile = np.where(valid, (tx1 - tx0 + 1) * (ty1 - ty0 + 1), 0)
    small = valid & (ntile <= MASK_TILES) & (tx1 > tx0) & (ty1 > ty0)
    tmask, frag_cull, fmask = tile_mask(u, w, A, B, Cc, tau0, x_lo, x_hi, y_lo, y_hi, tw, th,
                                        small, rel, du, dw)
    count = np.where(small, np.bitwise_count(tmask).astype(np.int64), ntile)

    return dict(
        n=n, valid=valid, p=p, u=u, w=w, zbits=zbits, ztol=ztol, du=du, dw=dw,
        conic=conic, r=r.astype(np.int64),
        box=np.stack([x_lo, x_hi, y_lo, y_hi], 1), opacity=o, rgb=rgb, raw_rgb=raw,
        normal=nvec, d=d, sign=sign, jstar=jstar, normal_alt=n_alt, d_alt=d_alt,
        tiles=np.stack([tx0, tx1, ty0, ty1], 1), count=count, tmask=tmask, small=small,
        TX=TX, TY=TY,
        # near-tie decisions (float32 on the GPU, float64 here), per splat:
        # any of them (frag_value); box edges (frag_box); validity through
        # o vs 1/255 (frag_tau); tile-culling tests, per tile bit (fmask);
        # the normal's axis or orientation (frag_geom); and the ties that
        # only change the adjoint: the colour clamp and the Jacobian's guard
        # band (frag_grad)
        frag_value=(valid & (frag_r | frag_axis | frag_flip | frag_cull))
        | (front & (det > 0) & frag_tau),
        frag_ring=valid & frag_r, frag_geom=valid & (frag_axis | frag_flip),
        frag_box=frag_box, frag_edge=frag_edge, frag_tau=front & (det > 0) & frag_tau,
        fmask=fmask,
        frag_grad=valid & (frag_colour
                           | (np.abs(np.abs(rx) - lim_x) < FRAG * lim_x + du / abs(fx))
                           | (np.abs(np.abs(ry) - lim_y) < FRAG * lim_y + dw / abs(fy))),
        # intermediates for the adjoint
        _s=s, _q=q, _qn=qn, _qnorm=qnorm, _Rq=Rq, _M=M, _T0=T0, _T1=T1, _V0=V0, _V1=V1,
        _A=A, _B=B, _C=Cc, _det=dets, _pz=pz, _txz=txz, _tyz=tyz,
        _clamp_x=clamp_x, _clamp_y=clamp_y, _lim=(lim_x, lim_y), _dirs=dirs,
        _mu=mu, _view=V, _sh_degree=sh_degree,
        _sh=(None if sh is None else np.asarray(sh, np.float64)),
    )


def project_backward(P, g):
    """Adjoint of `project`.

    g: dict of per-splat gradients (N rows) with keys mean2d (N,2),
    conic (N,3), opacity (N,), rgb (N,3), d (N,), normal (N,3).
    Returns dict with mu (N,3), scales (N,3), quats (N,4) (raw quaternion),
    opacity (N,), and either sh (N,K,3) (explicit) or rgb (N,3) (given
    colour, before any clamp).
    """
    V = P["_view"]
    R = V["R"]
    fx, fy = V["fx"], V["fy"]
    n = P["n"]
    valid = P["valid"][:, None]
    z = lambda a: np.where(valid if a.ndim == 2 else P["valid"], a, 0.0)  # noqa: E731
    dmean = z(np.asarray(g["mean2d"], np.float64))
    dconic = z(np.asarray(g["conic"], np.float64))
    dop = z(np.asarray(g["opacity"], np.float64))
    drgb = z(np.asarray(g["rgb"], np.float64))
    dd = z(np.asarray(g["d"], np.float64))
    dnorm = z(np.asarray(g["normal"], np.float64))

    p, pz = P["p"], P["_pz"]
    dp = np.zeros((n, 3))
    # 2-D mean
    dp[:, 0] += dmean[:, 0] * fx / pz
    dp[:, 1] += dmean[:, 1] * fy / pz
    dp[:, 2] += -dmean[:, 0] * fx * p[:, 0] / pz ** 2 - dmean[:, 1] * fy * p[:, 1] / pz ** 2

    # conic -> Sigma_2 entries (A, B, C)
    A, B, Cc, det = P["_A"], P["_B"], P["_C"], P["_det"]
    dca, dcb, dcc = dconic[:, 0], dconic[:, 1], dconic[:, 2]
    dA = dcc / det
    dB = -dcb / det
    dC = dca / det
    ddet = -(dca * Cc + dcc * A) / det ** 2 + dcb * B / det ** 2
    dA += ddet * Cc
    dC += ddet * A
    dB += -2.0 * B * ddet
    V0, V1 = P["_V0"], P["_V1"]
    dV0 = 2 * dA[:, None] * V0 + dB[:, None] * V1
    dV1 = 2 * dC[:, None] * V1 + dB[:, None] * V0
    M, T0, T1 = P["_M"], P["_T0"], P["_T1"]
    dT0 = np.einsum("nk,njk->nj", dV0, M)
    dT1 = np.einsum("nk,njk->nj", dV1, M)
    dM = T0[:, :, None] * dV0[:, None, :] + T1[:, :, None] * dV1[:, None, :]

    # T rows -> p (through 1/z and the clamped x/z, y/z)
    txz, tyz = P["_txz"], P["_tyz"]
    a0 = np.sum(dT0 * R[0][None], 1)
    b0 = np.sum(dT0 * R[2][None], 1)
    a1 = np.sum(dT1 * R[1][None], 1)
    b1 = np.sum(dT1 * R[2][None], 1)
    dpz = -a0 * fx / pz ** 2 - a1 * fy / pz ** 2
    dpz += b0 * 2 * fx * txz / pz ** 3 + b1 * 2 * fy * tyz / pz ** 3
    dtx = -b0 * fx / pz ** 2
    dty = -b1 * fy / pz ** 2
    lim_x, lim_y = P["_lim"]
    rx, ry = p[:, 0] / pz, p[:, 1] / pz
    cxm, cym = P["_clamp_x"], P["_clamp_y"]
    dp[:, 0] += np.where(cxm, 0.0, dtx)
    dp[:, 1] += np.where(cym, 0.0, dty)
    dpz += np.where(cxm, dtx * np.clip(rx, -lim_x, lim_x), 0.0)
    dpz += np.where(cym, dty * np.clip(ry, -lim_y, lim_y), 0.0)
    dp[:, 2] += dpz

    # M = Rq diag(s)
    s, Rq = P["_s"], P["_Rq"]
    ds = np.sum(dM * Rq, 1)
    dRq = dM * s[:, None, :]

    # normal and plane distance: n = sign * R Rq[:, j*], d = -n.p
    nvec = P["normal"]
    dn_tot = dnorm - dd[:, None] * p
    dp += -dd[:, None] * nvec
    col = np.einsum("ji,nj->ni", R, dn_tot) * P["sign"][:, None]
    dRq[np.arange(n), :, P["jstar"]] += col

    # colour
    out = {}
    mu = P["_mu"]
    dmu = np.einsum("ji,nj->ni", R, dp)
    if P["_sh"] is not None:
        raw = P["raw_rgb"]
        geff = np.where(raw > 0, drgb, 0.0)
        dirs = P["_dirs"]
        Y = shmod.basis(dirs, P["_sh_degree"])
        out["sh"] = Y[:, :, None] * geff[:, None, :]
        dY = shmod.basis_grad(dirs, P["_sh_degree"])
        ddir = np.einsum("nc,nkc,nkj->nj", geff, P["_sh"], dY)
        dv = mu - V["c"][None]
        dn_ = np.linalg.norm(dv, axis=1)
        proj = ddir - dirs * np.sum(dirs * ddir, 1, keepdims=True)
        dmu += proj / dn_[:, None]
    else:
        out["rgb"] = drgb

    # quaternion: qn = q / |q|
    qn, qnorm = P["_qn"], P["_qnorm"]
    dqn = quat_to_rot_backward(qn, dRq)
    dq = (dqn - qn * np.sum(qn * dqn, 1, keepdims=True)) / qnorm[:, None]

    out.update(mu=dmu * valid, scales=ds * valid, quats=dq * valid, opacity=dop)
    if "sh" in out:
        out["sh"] = out["sh"] * valid[:, :, None]
    return out
