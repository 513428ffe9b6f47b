"""Tile binning, the (tile | depth) sort, front-to-back compositing of RGB,
depth and normal maps, the L1 seed and the reverse-order adjoint
(oracle, test infrastructure).

Follows Sec. 3.3: the batch images are cut into 16x16 patches (tiles),
Gaussians are ordered per tile (Eq. 5's reordering pi) and blended front to
back (Eqs. 1 and 5); the normal map (Eq. 6) and the blended distance map D
(Eq. 7, first line) use the same weights; the unbiased depth is
D / (N . K^-1 p~) (Eq. 7, second line).  Readings of what the paper leaves
open:

  * tile order: a splat is listed in every tile that its pixel box touches;
    per tile the list is sorted by the float32 depth key, ties by
    (view, Gaussian id) -- equivalent to a stable sort of 64-bit keys
    (global tile id << 32 | depth bits) over pairs emitted in splat order;
  * per pixel, walking the list: skip splats whose pixel box misses the
    pixel; power = -1/2 (a dx^2 + c dy^2) - b dx dy with dx = u - px,
    dy = w - py at the pixel centre, where (u, w) is the 2-D mean rounded
    to float32 (the paper fixes no precision; the compositor's input mean is
    read as binary32, as the depth key is, because at 1080p and above its
    rounding moves alpha by up to ~1e-4 relative); alpha = min(0.99, o exp(power)); skip
    alpha < 1/255; stop (without blending) when T (1 - alpha) < 1e-4;
  * the normal map stays in the camera frame and faces the camera, the
    plane distance is d = -n . p >= 0, and the unbiased depth is
    D / s with s = -N . (K^-1 p~), kept only where s > 1e-3 * alpha
    (else 0);
  * background colour bg is added with the final transmittance.
"""
import numpy as np

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
DHAT_GUARD = 1e-3
DHAT_COND = 20.0
FRAG_ALPHA = 1e-5
FRAG_T = 1e-4
FRAG_SIGN = 1e-5
# The compositor's 2-D mean is the float32 rounding of the float64 one.  The
# finite-difference pins switch this off: rounding makes the image a step
# function of the mean at the scale of those differences.
MEAN_F32 = True


# --------------------------------------------------------------------------
# batch layout
# --------------------------------------------------------------------------
def batch_layout(views, tile):
    """Per view: tiles across / down, global tile offset, pixel offset."""
    tw, th = tile
    TX = [-(-int(v.width) // tw) for v in views]
    TY = [-(-int(v.height) // th) for v in views]
    tile_off = np.concatenate([[0], np.cumsum([a * b for a, b in zip(TX, TY)])]).astype(np.int64)
    pix_off = np.concatenate([[0], np.cumsum([int(v.width) * int(v.height) for v in views])]).astype(np.int64)
    return dict(TX=TX, TY=TY, tile_off=tile_off, pix_off=pix_off, tile=tile)


# --------------------------------------------------------------------------
# a3-a5: binning and sort
# --------------------------------------------------------------------------
def _bin_sample(splats_per_view, layout, keep_tiles):
    """Entries of the global tiles in keep_tiles only (a bounded sample of a
    large workload): for each such tile, every valid splat whose tile
    rectangle contains it."""
    gt_all, zb_all, v_all, g_all = [], [], [], []
    for gtile in sorted(int(t) for t in keep_tiles):
        v = int(np.searchsorted(layout["tile_off"], gtile, side="right") - 1)
        local = gtile - int(layout["tile_off"][v])
        tx, ty = local % layout["TX"][v], local // layout["TX"][v]
        S = splats_per_view[v]
        t = S["tiles"]
        m = S["valid"] & (t[:, 0] <= tx) & (t[:, 1] >= tx) & (t[:, 2] <= ty) & (t[:, 3] >= ty)
        # boxes of at most 64 tiles: only the tiles the drawable ellipse reaches
        bit = np.where(m, (ty - t[:, 2]) * (t[:, 1] - t[:, 0] + 1) + (tx - t[:, 0]), 0)
        hit = (np.right_shift(S["tmask"], np.minimum(bit, 63).astype(np.uint64)) & np.uint64(1)) != 0
        m &= ~S["small"] | hit
        idx = np.nonzero(m)[0]
        gt_all.append(np.full(idx.size, gtile, np.int64))
        zb_all.append(S["zbits"][idx])
        v_all.append(np.full(idx.size, v, np.int64))
        g_all.append(idx.astype(np.int64))
    return gt_all, zb_all, v_all, g_all


def bin_and_sort(splats_per_view, layout, keep_tiles=None):
    """Emit one (global tile, depth bits, view, gid) entry per (splat, tile
    touched) and sort lexicographically.

    splats_per_view[v] is the dict from project.project for view v; the gid
    of a splat is its row index in that dict.  Returns dict with sorted
    arrays gtile (int64), zbits (uint32), view, gid, and ranges
    (n_tiles, 2) = [start, end) per global tile.  With keep_tiles, only the
    entries of those tiles are produced (other tiles have empty ranges).
    """
    if keep_tiles is not None:
        gt_all, zb_all, v_all, g_all = _bin_sample(splats_per_view, layout, keep_tiles)
        return _sort_entries(gt_all, zb_all, v_all, g_all, layout)
    gt_all, zb_all, v_all, g_all = [], [], [], []
    for v, S in enumerate(splats_per_view):
        idx = np.nonzero(S["valid"])[0]
        if idx.size == 0:
            continue
        tiles = S["tiles"][idx]
        tx0, tx1, ty0, ty1 = tiles.T
        nx = tx1 - tx0 + 1
        cnt = nx * (ty1 - ty0 + 1)
        rep = np.repeat(np.arange(idx.size), cnt)
        first = np.repeat(np.cumsum(cnt) - cnt, cnt)
        k = np.arange(rep.size) - first
        # boxes of at most 64 tiles: only the tiles the drawable ellipse reaches
        hit = (np.right_shift(S["tmask"][idx][rep], np.minimum(k, 63).astype(np.uint64))
               & np.uint64(1)) != 0
        sel = ~S["small"][idx][rep] | hit
        rep, k = rep[sel], k[sel]
        tx = tx0[rep] + k % nx[rep]
        ty = ty0[rep] + k // nx[rep]
        gt_all.append(layout["tile_off"][v] + ty * layout["TX"][v] + tx)
        zb_all.append(S["zbits"][idx][rep])
        v_all.append(np.full(rep.size, v, np.int64))
        g_all.append(idx[rep].astype(np.int64))
    return _sort_entries(gt_all, zb_all, v_all, g_all, layout)


def _sort_entries(gt_all, zb_all, v_all, g_all, layout):
    n_tiles = int(layout["tile_off"][-1])
    if not gt_all or sum(a.size for a in gt_all) == 0:
        e = np.zeros(0, np.int64)
        return dict(gtile=e, zbits=e.astype(np.uint32), view=e, gid=e,
                    ranges=np.zeros((n_tiles, 2), np.int64))
    gt = np.concatenate(gt_all)
    zb = np.concatenate(zb_all)
    vv = np.concatenate(v_all)
    gg = np.concatenate(g_all)
    order = np.lexsort((gg, vv, zb, gt))
    gt, zb, vv, gg = gt[order], zb[order], vv[order], gg[order]
    ranges = np.zeros((n_tiles, 2), np.int64)
    if gt.size:
        starts = np.searchsorted(gt, np.arange(n_tiles), side="left")
        ends = np.searchsorted(gt, np.arange(n_tiles), side="right")
        ranges[:, 0] = np.where(ends > starts, starts, 0)
        ranges[:, 1] = np.where(ends > starts, ends, 0)
    return dict(gtile=gt, zbits=zb, view=vv, gid=gg, ranges=ranges)


# --------------------------------------------------------------------------
# a6: forward compositing
# --------------------------------------------------------------------------
def _tile_pixels(view, layout, v, local_tile):
    tw, th = layout["tile"]
    TX = layout["TX"][v]
    tx, ty = local_tile % TX, local_tile // TX
    W, H = int(view.width), int(view.height)
    xs = np.arange(tx * tw, min((tx + 1) * tw, W))
    ys = np.arange(ty * th, min((ty + 1) * th, H))
    I, J = np.meshgrid(xs, ys)
    return I.ravel(), J.ravel()


def _tile_eval(S, ent, I, J):
    """alpha matrix (pixels x entries) and the per-entry decisions.  The
    compositor takes the 2-D mean as float32 (the binary32 rounding of the
    float64 projection, like the depth key); everything after is float64."""
    u, w = S["u"][ent], S["w"][ent]
    if MEAN_F32:
        u = u.astype(np.float32).astype(np.float64)
        w = w.astype(np.float32).astype(np.float64)
    a, b, c = S["conic"][ent].T
    box = S["box"][ent]
    px = I[:, None] + 0.5
    py = J[:, None] + 0.5
    dx = u[None] - px
    dy = w[None] - py
    inbox = ((I[:, None] >= box[None, :, 0]) & (I[:, None] <= box[None, :, 1])
             & (J[:, None] >= box[None, :, 2]) & (J[:, None] <= box[None, :, 3]))
    power = -0.5 * (a[None] * dx * dx + c[None] * dy * dy) - b[None] * dx * dy
    G = np.exp(np.minimum(power, 0.0))
    raw = S["opacity"][ent][None] * G
    alpha = np.minimum(ALPHA_MAX, raw)
    use = inbox & (power <= 0) & (alpha >= ALPHA_MIN)
    return dict(dx=dx, dy=dy, inbox=inbox, power=power, G=G, raw=raw, alpha=alpha, use=use)


def composite_tile(S, ent, I, J, view_arrays):
    """Front-to-back blend of one tile's sorted entries `ent` (indices into
    the splat dict S of that view) over pixels (I, J)."""
    E = _tile_eval(S, ent, I, J)
    use, alpha = E["use"], E["alpha"]
    npx, ne = use.shape
    a_use = np.where(use, alpha, 0.0)
    Tp_all = np.cumprod(1.0 - a_use, axis=1) if ne else np.ones((npx, 0))
    crossed = use & (Tp_all < T_MIN)
    has_stop = crossed.any(axis=1)
    stop = np.where(has_stop, np.argmax(crossed, axis=1), ne) if ne else np.zeros(npx, np.int64)
    kidx = np.arange(ne)[None]
    inc = use & (kidx < stop[:, None])
    a_inc = np.where(inc, alpha, 0.0)
    Tp = np.cumprod(1.0 - a_inc, axis=1) if ne else np.ones((npx, 0))
    Tb = np.concatenate([np.ones((npx, 1)), Tp[:, :-1]], axis=1) if ne else Tp
    wgt = a_inc * Tb
    T_final = Tp[:, -1] if ne else np.ones(npx)
    rgb = wgt @ S["rgb"][ent] if ne else np.zeros((npx, 3))
    D = wgt @ S["d"][ent] if ne else np.zeros(npx)
    N = wgt @ S["normal"][ent] if ne else np.zeros((npx, 3))
    # magnitude of the blend (sum of |terms|), the scale float32 error follows
    Nabs = wgt @ np.abs(S["normal"][ent]) if ne else np.zeros((npx, 3))
    last = (np.where(inc.any(axis=1), ne - np.argmax(inc[:, ::-1], axis=1), 0) if ne
            else np.zeros(npx, np.int64))
    walked = np.minimum(stop + 1, ne)

    # fragile decisions (float32 on the GPU vs float64 here)
    upto = kidx <= stop[:, None]
    frag = np.zeros(npx, bool)
    near_a = E["inbox"] & upto & (np.abs(E["raw"] * 255.0 - 1.0) < FRAG_ALPHA)
    frag |= near_a.any(axis=1)
    near_t = use & upto & (np.abs(Tp_all / T_MIN - 1.0) < FRAG_T)
    frag |= near_t.any(axis=1)
    frag_geom = np.zeros(npx, bool)
    if ne:
        # a fragile radius ceiling moves the box edge by one pixel: the ring
        # between the box shrunk and grown by one; a fragile normal axis or
        # orientation changes the splat's normal and plane distance
        box = S["box"][ent]
        grown = ((I[:, None] >= box[None, :, 0] - 1) & (I[:, None] <= box[None, :, 1] + 1)
                 & (J[:, None] >= box[None, :, 2] - 1) & (J[:, None] <= box[None, :, 3] + 1))
        shrunk = ((I[:, None] >= box[None, :, 0] + 1) & (I[:, None] <= box[None, :, 1] - 1)
                  & (J[:, None] >= box[None, :, 2] + 1) & (J[:, None] <= box[None, :, 3] - 1))
        frag |= (grown & ~shrunk & S["frag_ring"][ent][None] & upto).any(axis=1)
        frag_geom = (grown & S["frag_geom"][ent][None] & upto).any(axis=1)
    frag_grad = frag | (inc & (np.abs(E["raw"] / ALPHA_MAX - 1.0) < FRAG_ALPHA)).any(axis=1)
    if ne:
        frag_grad |= (inc & S["frag_grad"][ent][None]).any(axis=1)

    V = view_arrays
    rgb = rgb + T_final[:, None] * V["bg"][None]
    acc = 1.0 - T_final
    ray = np.stack([(I + 0.5 - V["cx"]) / V["fx"], (J + 0.5 - V["cy"]) / V["fy"], np.ones(npx)], 1)
    sdot = -np.sum(N * ray, 1)
    keep = sdot > DHAT_GUARD * acc
    dhat = np.where(keep, D / np.where(keep, sdot, 1.0), 0.0)
    frag |= (acc > 0) & (np.abs(sdot - DHAT_GUARD * acc)
                         < 10 * FRAG_ALPHA * np.maximum(np.abs(sdot), DHAT_GUARD * acc))
    # grazing incidence: s = -N . ray cancels terms DHAT_COND times its size;
    # float32 then loses more than four bits of s, and D^'s adjoint (1/s^2)
    # doubles that, so the pixel's gradients are not resolved to 1e-4
    sabs = np.sum(Nabs * np.abs(ray), 1)
    frag_grad = frag_grad | (keep & (sabs > DHAT_COND * np.abs(sdot)))
    return dict(rgb=rgb, D=D, N=N, Nabs=Nabs, alpha=acc, dhat=dhat, T=T_final, last=last,
                walked=walked, frag=frag, frag_geom=frag_geom,
                frag_grad=frag_grad | frag | frag_geom, inc=inc,
                keep=keep, sdot=sdot, ray=ray, E=E, Tb=Tb, wgt=wgt, a_inc=a_inc)


def render_images(splats_per_view, views, layout, sorted_, view_arrays, keep_tiles=None):
    """Composite every tile (or the global tile ids in keep_tiles) of every
    view.  Returns per-view planar images and per-tile state for the
    adjoint."""
    out = []
    for v, view in enumerate(views):
        W, H = int(view.width), int(view.height)
        img = dict(rgb=np.zeros((3, H * W)), depth=np.zeros(H * W), D=np.zeros(H * W),
                   normal=np.zeros((3, H * W)), normal_abs=np.zeros((3, H * W)),
                   alpha=np.zeros(H * W), T=np.ones(H * W),
                   last=np.zeros(H * W, np.int64), walked=np.zeros(H * W, np.int64),
                   frag=np.zeros(H * W, bool), frag_geom=np.zeros(H * W, bool),
                   frag_grad=np.zeros(H * W, bool),
                   covered=np.zeros(H * W, bool), tiles={})
        out.append(img)
    n_tiles_total = int(layout["tile_off"][-1])
    tiles = range(n_tiles_total) if keep_tiles is None else keep_tiles
    for gtile in tiles:
        v = int(np.searchsorted(layout["tile_off"], gtile, side="right") - 1)
        local = gtile - int(layout["tile_off"][v])
        I, J = _tile_pixels(views[v], layout, v, local)
        s0, s1 = sorted_["ranges"][gtile]
        ent = sorted_["gid"][s0:s1]
        R = composite_tile(splats_per_view[v], ent, I, J, view_arrays[v])
        pix = J * int(views[v].width) + I
        img = out[v]
        img["rgb"][:, pix] = R["rgb"].T
        img["depth"][pix] = R["dhat"]
        img["D"][pix] = R["D"]
        img["normal"][:, pix] = R["N"].T
        img["normal_abs"][:, pix] = R["Nabs"].T
        img["alpha"][pix] = R["alpha"]
        img["T"][pix] = R["T"]
        img["last"][pix] = R["last"]
        img["walked"][pix] = R["walked"]
        img["frag"][pix] = R["frag"]
        img["frag_geom"][pix] = R["frag_geom"]
        img["frag_grad"][pix] = R["frag_grad"]
        img["covered"][pix] = True
        img["tiles"][gtile] = (ent, I, J, pix, R)
    # a splat with a fragile radius ceiling may reach one pixel further or
    # shorter on the GPU: flag the ring between its box shrunk and grown by
    # one pixel; one with a fragile normal axis or orientation has another
    # normal and plane distance there: flag its grown box for the geometric
    # outputs (normal, D, unbiased depth); both for the gradients
    for v, view in enumerate(views):
        S = splats_per_view[v]
        W, H = int(view.width), int(view.height)
        img = out[v]
        for i in np.nonzero(S["frag_value"])[0]:
            bx0, bx1, by0, by1 = (int(t) for t in S["box"][i])
            x0, y0 = max(bx0 - 1, 0), max(by0 - 1, 0)
            x1, y1 = min(bx1 + 1, W - 1), min(by1 + 1, H - 1)
            if x0 > x1 or y0 > y1:
                continue
            xs, ys = np.arange(x0, x1 + 1), np.arange(y0, y1 + 1)
            blk = (ys[:, None] * W + xs[None]).ravel()
            img["frag_grad"][blk] = True
            if S["frag_geom"][i]:
                img["frag_geom"][blk] = True
            if S["frag_ring"][i]:
                inner = (((xs[None] >= bx0 + 1) & (xs[None] <= bx1 - 1))
                         & ((ys[:, None] >= by0 + 1) & (ys[:, None] <= by1 - 1))).ravel()
                img["frag"][blk[~inner]] = True
    return out


# --------------------------------------------------------------------------
# a7: L1 seed (Eq. 8, read per-image mean)
# --------------------------------------------------------------------------
def l1_seed(images, targets, weights=(1.0, 1.0, 1.0)):
    """L = (1/B) sum_b (1/(H_b W_b)) sum_px [w_rgb |C - C*|_1 + w_d |D^ - D^*|
    + w_n |N - N*|_1]; returns (L, per-view output gradients) with
    sign(0) = 0.  The plane-distance map D and alpha get zero gradient.

    Depth prior mask (Sec. 3.4, Step 2): the depth target is the filtered
    pseudo depth, which holds no value where the reprojection filter removed
    it.  A target depth that is not positive (the zero of a filtered pixel)
    or is NaN marks such a pixel: it adds no depth loss and no depth
    gradient, and the per-image scale still counts every pixel."""
    B = len(images)
    L = 0.0
    grads = []
    for b, img in enumerate(images):
        npx = img["depth"].size
        sc = 1.0 / (B * npx)
        er = img["rgb"] - np.asarray(targets["rgb"][b], np.float64)
        td = np.asarray(targets["depth"][b], np.float64)
        with np.errstate(invalid="ignore"):
            keep = td > 0.0                        # False for NaN
        ed = np.where(keep, img["depth"] - np.where(keep, td, 0.0), 0.0)
        en = img["normal"] - np.asarray(targets["normal"][b], np.float64)
        L += sc * (weights[0] * np.abs(er).sum() + weights[1] * np.abs(ed).sum()
                   + weights[2] * np.abs(en).sum())
        grads.append(dict(rgb=weights[0] * sc * np.sign(er), depth=weights[1] * sc * np.sign(ed),
                          normal=weights[2] * sc * np.sign(en), D=np.zeros(npx),
                          alpha=np.zeros(npx)))
        # sign(out - target) is a decision: a pixel whose output lies within
        # FRAG_SIGN of its target may take the other sign in float32
        if "frag_grad" in img:
            near = ((np.abs(er) < FRAG_SIGN).any(axis=0) | (keep & (np.abs(ed) < FRAG_SIGN))
                    | (np.abs(en) < FRAG_SIGN).any(axis=0))
            img["frag_grad"] = img["frag_grad"] | near
    return L, grads


# --------------------------------------------------------------------------
# a8: compositing adjoint
# --------------------------------------------------------------------------
def composite_backward(splats_per_view, views, images, grads, view_arrays):
    """Per-splat gradients (mean2d, conic, opacity, rgb, d, normal) for every
    view, from per-pixel output gradients.  Transmittances come from the
    forward products (no division)."""
    res = []
    for v, S in enumerate(splats_per_view):
        n = S["n"]
        res.append(dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), opacity=np.zeros(n),
                        rgb=np.zeros((n, 3)), d=np.zeros(n), normal=np.zeros((n, 3)),
                        frag=np.zeros(n, bool)))
    for v, img in enumerate(images):
        S = splats_per_view[v]
        Vv = view_arrays[v]
        g = grads[v]
        acc = res[v]
        for gtile, (ent, I, J, pix, R) in img["tiles"].items():
            if ent.size == 0:
                continue
            GC = g["rgb"][:, pix].T.copy()
            GD = g["D"][pix].copy()
            GN = g["normal"][:, pix].T.copy()
            GA = g["alpha"][pix].copy()
            Gh = g["depth"][pix]
            keep = R["keep"]
            sd = np.where(keep, R["sdot"], 1.0)
            GD += np.where(keep, Gh / sd, 0.0)
            GN += np.where(keep, Gh * R["D"] / sd ** 2, 0.0)[:, None] * R["ray"]
            dT = GC @ Vv["bg"] - GA
            E = R["E"]
            inc = R["inc"]
            a_inc, Tb, wgt = R["a_inc"], R["Tb"], R["wgt"]
            rgb, d, nrm = S["rgb"][ent], S["d"][ent], S["normal"][ent]
            val = GC @ rgb.T + GD[:, None] * d[None] + GN @ nrm.T
            wv = wgt * val
            suffix = np.cumsum(wv[:, ::-1], axis=1)[:, ::-1] - wv
            one_m = 1.0 - a_inc
            dalpha = Tb * val - suffix / one_m - (R["T"] * dT)[:, None] / one_m
            dalpha = np.where(inc, dalpha, 0.0)
            unclamped = inc & (E["raw"] < ALPHA_MAX)
            op = S["opacity"][ent][None]
            dop = np.where(unclamped, dalpha * E["G"], 0.0)
            dpower = np.where(unclamped, dalpha * op * E["G"], 0.0)
            a, b, c = S["conic"][ent].T
            dx, dy = E["dx"], E["dy"]
            du = dpower * (-(a[None] * dx + b[None] * dy))
            dw = dpower * (-(c[None] * dy + b[None] * dx))
            np.add.at(acc["mean2d"], ent, np.stack([du.sum(0), dw.sum(0)], 1))
            np.add.at(acc["conic"], ent, np.stack([(-0.5 * dx * dx * dpower).sum(0),
                                                   (-dx * dy * dpower).sum(0),
                                                   (-0.5 * dy * dy * dpower).sum(0)], 1))
            np.add.at(acc["opacity"], ent, dop.sum(0))
            np.add.at(acc["rgb"], ent, wgt.T @ GC)
            np.add.at(acc["d"], ent, wgt.T @ GD)
            np.add.at(acc["normal"], ent, wgt.T @ GN)
            fr = img["frag_grad"][pix]
            if fr.any():
                touched = (inc & fr[:, None]).any(axis=0)
                acc["frag"][ent[touched]] = True
    return res
