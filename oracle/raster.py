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
def _grown_tiles(S, layout, v):
    """Tile rectangle of each splat's pixel box grown by one pixel on every
    side (clipped to the image): the tiles a box edge one pixel further out
    could reach."""
    tw, th = layout["tile"]
    W, H = S["_view"]["W"], S["_view"]["H"]
    box = S["box"]
    gx0 = np.clip(box[:, 0] - 1, 0, W - 1) // tw
    gx1 = np.clip(box[:, 1] + 1, 0, W - 1) // tw
    gy0 = np.clip(box[:, 2] - 1, 0, H - 1) // th
    gy1 = np.clip(box[:, 3] + 1, 0, H - 1) // th
    return gx0, gx1, gy0, gy1


def _tile_entries(S, layout, v, tx, ty):
    """Entries of one tile (tx, ty) of view v.

    own: the splat's pixel box and, for a masked box, its drawable-ellipse
    tile mask contain the tile (the oracle's own binning);
    extra: not own, but one near-tie decision away from it -- a box edge
    (the tiles of the box grown by one pixel), the o vs 1/255 validity, or
    the tile-culling test of this very tile;
    cbit: this tile's culling test is itself a near tie.
    Returns (idx, own, cbit) over own | extra."""
    t = S["tiles"]
    inrect = (t[:, 0] <= tx) & (t[:, 1] >= tx) & (t[:, 2] <= ty) & (t[:, 3] >= ty)
    bit = np.where(inrect, (ty - t[:, 2]) * (t[:, 1] - t[:, 0] + 1) + (tx - t[:, 0]), 0)
    sh = np.minimum(bit, 63).astype(np.uint64)
    hit = (np.right_shift(S["tmask"], sh) & np.uint64(1)) != 0
    cbit = S["small"] & inrect & ((np.right_shift(S["fmask"], sh) & np.uint64(1)) != 0)
    own = S["valid"] & inrect & (~S["small"] | hit)
    gx0, gx1, gy0, gy1 = _grown_tiles(S, layout, v)
    near = (S["frag_box"] | S["frag_tau"]) & (gx0 <= tx) & (gx1 >= tx) & (gy0 <= ty) & (gy1 >= ty)
    cand = own | near | cbit
    idx = np.nonzero(cand)[0]
    return idx, own[idx], cbit[idx]


def _bin_tiles(splats_per_view, layout, tiles):
    """Entries (global tile, depth bits, view, gid, own, cbit) of the given
    global tiles, one tile at a time."""
    cols = [[] for _ in range(6)]
    for gtile in tiles:
        gtile = int(gtile)
        v = int(np.searchsorted(layout["tile_off"], gtile, side="right") - 1)
        local = gtile - int(layout["tile_off"][v])
        tx, ty = local % layout["TX"][v], local // layout["TX"][v]
        S = splats_per_view[v]
        idx, own, cbit = _tile_entries(S, layout, v, tx, ty)
        for c, a in zip(cols, (np.full(idx.size, gtile, np.int64), S["zbits"][idx],
                               np.full(idx.size, v, np.int64), idx.astype(np.int64), own, cbit)):
            c.append(a)
    return cols


def _bin_all(splats_per_view, layout):
    """Entries of every tile of every view, vectorised per view: the own
    pairs of the tile rectangle and mask, plus the one-tie-away pairs of
    the splats with a near-tie box edge or validity (grown rectangle) and of
    the near-tie culled tiles."""
    cols = [[] for _ in range(6)]
    for v, S in enumerate(splats_per_view):
        gx0, gx1, gy0, gy1 = _grown_tiles(S, layout, v)
        near = S["frag_box"] | S["frag_tau"]
        t = S["tiles"]
        # candidate rectangle: the box's tiles, or the grown box's tiles for
        # splats with a near-tie box edge or validity
        rx0 = np.where(near, np.minimum(gx0, t[:, 0]), t[:, 0])
        rx1 = np.where(near, np.maximum(gx1, t[:, 1]), t[:, 1])
        ry0 = np.where(near, np.minimum(gy0, t[:, 2]), t[:, 2])
        ry1 = np.where(near, np.maximum(gy1, t[:, 3]), t[:, 3])
        live = S["valid"] | near
        idx = np.nonzero(live & (rx1 >= rx0) & (ry1 >= ry0))[0]
        if idx.size == 0:
            continue
        nx = rx1[idx] - rx0[idx] + 1
        cnt = nx * (ry1[idx] - ry0[idx] + 1)
        rep = np.repeat(np.arange(idx.size), cnt)
        first = np.repeat(np.cumsum(cnt) - cnt, cnt)
        k = np.arange(rep.size) - first
        g = idx[rep]
        tx = rx0[g] + k % nx[rep]
        ty = ry0[g] + k // nx[rep]
        inrect = (t[g, 0] <= tx) & (t[g, 1] >= tx) & (t[g, 2] <= ty) & (t[g, 3] >= ty)
        bit = np.where(inrect, (ty - t[g, 2]) * (t[g, 1] - t[g, 0] + 1) + (tx - t[g, 0]), 0)
        sh = np.minimum(bit, 63).astype(np.uint64)
        hit = (np.right_shift(S["tmask"][g], sh) & np.uint64(1)) != 0
        cbit = S["small"][g] & inrect & ((np.right_shift(S["fmask"][g], sh) & np.uint64(1)) != 0)
        own = S["valid"][g] & inrect & (~S["small"][g] | hit)
        keep = own | near[g] | cbit
        g, tx, ty, own, cbit = g[keep], tx[keep], ty[keep], own[keep], cbit[keep]
        for c, a in zip(cols, (layout["tile_off"][v] + ty * layout["TX"][v] + tx, S["zbits"][g],
                               np.full(g.size, v, np.int64), g.astype(np.int64), own, cbit)):
            c.append(a)
    return cols


def bin_and_sort(splats_per_view, layout, keep_tiles=None):
    """Emit one (global tile, depth bits, view, gid) entry per (splat, tile
    touched) and sort lexicographically.

    splats_per_view[v] is the dict from project.project for view v; the gid
    of a splat is its row index in that dict.  Returns dict with sorted
    arrays gtile (int64), zbits (uint32), view, gid, and ranges
    (n_tiles, 2) = [start, end) per global tile.  With keep_tiles, only the
    entries of those tiles are produced (other tiles have empty ranges).

    The oracle's own pairs are the ones with own = True; the lists also
    hold, flagged own = False, the pairs one near-tie decision away (a box
    edge, the validity, a tile-culling test), which the GPU, deciding in
    float32, may equally take.  cbit marks an entry whose tile-culling test
    is itself a near tie; `certain` = own and no near tie on the pair;
    ztol is the depth key's tolerance in units in the last place (nonzero
    only for means that carry a decode error)."""
    if keep_tiles is not None:
        cols = _bin_tiles(splats_per_view, layout, sorted(int(t) for t in keep_tiles))
    else:
        cols = _bin_all(splats_per_view, layout)
    return _sort_entries(cols, splats_per_view, layout)


def _sort_entries(cols, splats_per_view, layout):
    n_tiles = int(layout["tile_off"][-1])
    if not cols[0] or sum(a.size for a in cols[0]) == 0:
        e = np.zeros(0, np.int64)
        b = np.zeros(0, bool)
        z = dict(gtile=e, zbits=e.astype(np.uint32), view=e, gid=e, own=b, cbit=b, certain=b,
                 ranges=np.zeros((n_tiles, 2), np.int64), ztol=e)
        z["own_sorted"] = dict(z)
        return z
    gt, zb, vv, gg, own, cbit = (np.concatenate(c) for c in cols)
    order = np.lexsort((gg, vv, zb, gt))
    gt, zb, vv, gg, own, cbit = (a[order] for a in (gt, zb, vv, gg, own, cbit))
    near = np.zeros(gt.size, bool)
    ztol = np.zeros(gt.size, np.int64)
    for v, S in enumerate(splats_per_view):
        m = vv == v
        near[m] = S["frag_box"][gg[m]] | S["frag_tau"][gg[m]]
        ztol[m] = S["ztol"][gg[m]]
    certain = own & ~cbit & ~near
    ranges = np.zeros((n_tiles, 2), np.int64)
    if gt.size:
        starts = np.searchsorted(gt, np.arange(n_tiles), side="left")
        ends = np.searchsorted(gt, np.arange(n_tiles), side="right")
        ranges[:, 0] = np.where(ends > starts, starts, 0)
        ranges[:, 1] = np.where(ends > starts, ends, 0)
    # the oracle's own binning alone (the pairs it takes itself)
    o = own
    ogt = gt[o]
    oranges = np.zeros((n_tiles, 2), np.int64)
    if ogt.size:
        starts = np.searchsorted(ogt, np.arange(n_tiles), side="left")
        ends = np.searchsorted(ogt, np.arange(n_tiles), side="right")
        oranges[:, 0] = np.where(ends > starts, starts, 0)
        oranges[:, 1] = np.where(ends > starts, ends, 0)
    return dict(gtile=gt, zbits=zb, view=vv, gid=gg, own=own, cbit=cbit, certain=certain,
                ranges=ranges, ztol=ztol,
                own_sorted=dict(gtile=ogt, zbits=zb[o], view=vv[o], gid=gg[o], ranges=oranges))


# --------------------------------------------------------------------------
# a6: forward compositing
# --------------------------------------------------------------------------
# Near ties in the compositing and what they allow (float32 on the GPU,
# float64 here): the alpha test within FRAG_ALPHA of 1/255; the transmittance
# stop within FRAG_T of 1e-4; the unbiased-depth guard within 10 FRAG_ALPHA;
# a box edge, validity or tile-culling test that is a near tie lets the GPU
# take or drop the splat at a pixel where its alpha passes (for validity and
# culling, only up to FRAG_CULL above 1/255: a tile or splat the GPU drops
# holds no pixel whose alpha clears the threshold by more than rounding and
# the float32 mean).  A pixel with at most MAX_TIES such pair decisions gets
# every combination, each walked with both outcomes of any transmittance or
# guard tie it meets; more is excluded and counted.
FRAG_CULL = 1e-3
MAX_TIES = 6
MAX_CANDIDATES = 256


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
    # how far the power (the log of the raw opacity) may move with the mean's
    # error bound (decoded offsets; zero otherwise)
    du, dw = S["du"][ent][None], S["dw"][ent][None]
    dpw = np.abs(a[None] * dx + b[None] * dy) * du + np.abs(b[None] * dx + c[None] * dy) * dw
    return dict(dx=dx, dy=dy, inbox=inbox, power=power, G=G, raw=raw, alpha=alpha, use=use,
                dpw=dpw)


def _pair_ties(S, ent, own, cbit, I, J, E):
    """(pixel, entry) decisions that are near ties: the GPU may take the
    entry where the oracle does not, or the reverse."""
    ne = ent.size
    if ne == 0:
        return np.zeros((I.size, 0), bool)
    fb = S["frag_box"][ent][None]
    ft = S["frag_tau"][ent][None]
    fe = S["frag_edge"][ent]
    box = S["box"][ent]
    Ic, Jc = I[:, None], J[:, None]
    x0, x1, y0, y1 = (box[None, :, i] for i in range(4))
    grown = (Ic >= x0 - 1) & (Ic <= x1 + 1) & (Jc >= y0 - 1) & (Jc <= y1 + 1)
    # the pixel column or row on either side of a near-tie box edge
    ring = grown & (((Ic == x0) | (Ic == x0 - 1)) & fe[None, :, 0]
                    | ((Ic == x1) | (Ic == x1 + 1)) & fe[None, :, 1]
                    | ((Jc == y0) | (Jc == y0 - 1)) & fe[None, :, 2]
                    | ((Jc == y1) | (Jc == y1 + 1)) & fe[None, :, 3])
    pw = E["power"] <= 0
    r255 = E["raw"] * 255.0
    band = FRAG_ALPHA + E["dpw"]
    passes = pw & (r255 >= 1.0 - band)
    near = pw & (np.abs(r255 - 1.0) < band)
    loose = passes & (r255 < 1.0 + FRAG_CULL)
    inb = E["inbox"] | (fb & grown)
    # an entry the oracle does not list itself (own False) is taken, if at
    # all, only at such a tie
    return inb & (near | (ring & passes) | ((fb | ft | cbit[None]) & loose))


def _t_err(alpha, dpw):
    """Relative error bound that the mean's error (dpw on the power) puts on
    each factor 1 - alpha of the transmittance (none where alpha is clamped)."""
    return np.where(alpha < ALPHA_MAX, alpha * dpw / np.maximum(1.0 - alpha, 1e-12), 0.0)


def _walk(use, alpha, vals, dpw=None):
    """Front-to-back walk of one pixel over the entries with use: every
    outcome of the transmittance-stop near ties it meets (widened by the
    transmittance's share of the mean's error bound, dpw).  Returns a list
    of (weighted sums of vals, final T, per-entry weights)."""
    idx = np.nonzero(use)[0]
    te = np.zeros(use.size) if dpw is None else _t_err(alpha, dpw)
    out = []
    stack = [(0, 1.0, np.zeros(vals.shape[1]), np.zeros(use.size), 0.0)]
    while stack and len(out) < MAX_CANDIDATES:
        pos, T, acc, wts, err = stack.pop()
        for m in range(pos, idx.size):
            k = idx[m]
            Tn = T * (1.0 - alpha[k])
            w = alpha[k] * T
            err = err + te[k]
            if abs(Tn / T_MIN - 1.0) < FRAG_T + err:
                w2 = wts.copy()
                w2[k] = w
                stack.append((m + 1, Tn, acc + w * vals[k], w2, err))
                break
            if Tn < T_MIN:
                break
            acc = acc + w * vals[k]
            wts = wts.copy()
            wts[k] = w
            T = Tn
        out.append((acc, T, wts))
    return out


def _pixel_candidates(use0, amb, alpha, vals, nabs, bg, ray, alts=(), dpw=None, swaps=()):
    """Every output (rgb 3, D, N 3, alpha, unbiased depth, |N| blend 3) one
    pixel may take under its near ties, or None when there are more than
    MAX_TIES ties.  alts: (entry, its other (d, normal) outcome) for the
    entries whose normal is a near tie; swaps: entry pairs (i, j) whose
    depth keys may sort either way (walked in both orders)."""
    aidx = np.nonzero(amb)[0]
    na, nl = aidx.size, len(alts)
    if na + nl + len(swaps) > MAX_TIES:
        return None
    cands = []
    ne = use0.size
    for m in range(1 << (na + nl + len(swaps))):
        use = use0.copy()
        for b, k in enumerate(aidx):
            if (m >> b) & 1:
                use[k] = ~use[k]
        vv, nb = vals, nabs
        for b, (k, alt) in enumerate(alts):
            if (m >> (na + b)) & 1:
                vv = vv.copy()
                nb = nb.copy()
                vv[k, 3:7] = alt
                nb[k] = np.abs(alt[1:4])
        perm = np.arange(ne)
        for b, (i, j) in enumerate(swaps):
            if (m >> (na + nl + b)) & 1:
                pi, pj = int(np.nonzero(perm == i)[0][0]), int(np.nonzero(perm == j)[0][0])
                perm[pi], perm[pj] = perm[pj], perm[pi]
        dp = None if dpw is None else dpw[perm]
        for acc, T, wts in _walk(use[perm], alpha[perm], vv[perm], dp):
            rgb = acc[0:3] + T * bg
            D = acc[3]
            N = acc[4:7]
            a = 1.0 - T
            sd = -float(N @ ray)
            nab = wts @ nb[perm]
            dh = [D / sd if sd > DHAT_GUARD * a else 0.0]
            if a > 0 and abs(sd - DHAT_GUARD * a) < 10 * FRAG_ALPHA * max(abs(sd), DHAT_GUARD * a):
                dh = [D / sd if sd != 0 else 0.0, 0.0]
            cond = max(1.0, float(nab @ np.abs(ray)) / abs(sd)) if sd != 0 else 1.0
            for d in dh:
                cands.append(np.concatenate([rgb, [D], N, [a, d], nab, [abs(d) * cond]]))
        if len(cands) >= MAX_CANDIDATES:
            break
    return np.array(cands)


def composite_tile(S, ent, I, J, view_arrays, own=None, cbit=None):
    """Front-to-back blend of one tile's sorted entries `ent` (indices into
    the splat dict S of that view) over pixels (I, J).  own marks the
    entries the oracle lists itself (default: all); the others, and cbit,
    come from bin_and_sort's near-tie entries."""
    ne = ent.size
    own = np.ones(ne, bool) if own is None else np.asarray(own, bool)
    cbit = np.zeros(ne, bool) if cbit is None else np.asarray(cbit, bool)
    E = _tile_eval(S, ent, I, J)
    E["use"] = E["use"] & own[None]
    use, alpha = E["use"], E["alpha"]
    npx = use.shape[0]
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
    # list entries walked (the work measure): the oracle's own entries up to
    # and including the one that stops the pixel, or all of them
    own_before = np.concatenate([[0], np.cumsum(own)])
    walked = own_before[np.minimum(stop + 1, ne)]

    V = view_arrays
    rgb = rgb + T_final[:, None] * V["bg"][None]
    acc = 1.0 - T_final
    ray = np.stack([(I + 0.5 - V["cx"]) / V["fx"], (J + 0.5 - V["cy"]) / V["fy"], np.ones(npx)], 1)
    sdot = -np.sum(N * ray, 1)
    keep = sdot > DHAT_GUARD * acc
    dhat = np.where(keep, D / np.where(keep, sdot, 1.0), 0.0)

    # near ties: pair decisions, transmittance stop, depth guard
    upto = kidx <= stop[:, None]
    amb = _pair_ties(S, ent, own, cbit, I, J, E)
    terr = np.cumsum(np.where(use, _t_err(alpha, E["dpw"]), 0.0), axis=1) if ne else Tp_all
    near_t = use & upto & (np.abs(Tp_all / T_MIN - 1.0) < FRAG_T + terr)
    dtie = (acc > 0) & (np.abs(sdot - DHAT_GUARD * acc)
                        < 10 * FRAG_ALPHA * np.maximum(np.abs(sdot), DHAT_GUARD * acc))
    tie = dtie.copy()
    geo = np.zeros((npx, ne), bool)
    if ne:
        # a splat whose normal is a near tie, used (or one tie away) here
        geo = (inc | amb) & S["frag_geom"][ent][None]
        tie |= amb.any(axis=1) | near_t.any(axis=1) | geo.any(axis=1)
    cands, excl = {}, np.zeros(npx, bool)
    # entries whose depth keys lie within their tolerance of each other
    # (decoded offsets) may be sorted either way: a pixel that blends both
    # takes either order
    swaps = {}
    if ne > 1 and S["ztol"][ent].any():
        zb = S["zbits"][ent].astype(np.int64)
        zt = S["ztol"][ent]
        ztmax = int(zt.max())
        blended = inc | amb
        for i in range(ne - 1):
            j = i + 1
            while j < ne and zb[j] - zb[i] <= zt[i] + ztmax:
                if zb[j] - zb[i] <= zt[i] + zt[j]:
                    for p in np.nonzero(blended[:, i] & blended[:, j])[0]:
                        swaps.setdefault(int(p), []).append((i, j))
                        tie[p] = True
                j += 1
    if tie.any():
        vals = np.concatenate([S["rgb"][ent], S["d"][ent][:, None], S["normal"][ent]], 1)
        nabs = np.abs(S["normal"][ent])
        alt = np.concatenate([S["d_alt"][ent][:, None], S["normal_alt"][ent]], 1) if ne else None
        for p in np.nonzero(tie)[0]:
            alts = [(int(k), alt[k]) for k in np.nonzero(geo[p])[0]] if ne else []
            c = _pixel_candidates(use[p], amb[p] if ne else np.zeros(0, bool), alpha[p],
                                  vals, nabs, V["bg"], ray[p], alts, E["dpw"][p] if ne else None,
                                  swaps.get(int(p), ()))
            if c is None:
                excl[p] = True
            else:
                cands[int(p)] = c
    # decisions that change only the adjoint, or the geometric outputs:
    # the 0.99 clamp, a splat's own near ties (colour clamp, guard band,
    # decoder ReLU; its normal's axis or orientation), and grazing incidence
    # (s = -N . ray cancels terms DHAT_COND times its size: float32 loses more
    # than four bits of s, and the adjoint's 1/s^2 doubles that)
    touch = inc | amb if ne else inc
    geom = geo.any(axis=1)
    gonly = np.zeros(npx, bool)
    if ne:
        gonly = ((inc & (np.abs(E["raw"] / ALPHA_MAX - 1.0) < FRAG_ALPHA)).any(axis=1)
                 | (touch & S["frag_grad"][ent][None]).any(axis=1))
    sabs = np.sum(Nabs * np.abs(ray), 1)
    grazing = keep & (sabs > DHAT_COND * np.abs(sdot))
    # scale of the float32 error of D / s: s is a sum of terms of size sabs
    dmag = np.abs(dhat) * np.maximum(1.0, sabs / np.where(sdot != 0, np.abs(sdot), 1.0))
    tie_grad = tie | excl | geom | gonly | grazing
    return dict(rgb=rgb, D=D, N=N, Nabs=Nabs, alpha=acc, dhat=dhat, dmag=dmag, T=T_final,
                last=last,
                walked=walked, tie=tie, excl=excl, frag_geom=geom, frag_grad=tie_grad,
                cands=cands, n_pair_ties=int(amb.sum()) if ne else 0, n_order_ties=len(swaps),
                inc=inc, keep=keep, sdot=sdot, ray=ray, E=E, Tb=Tb, wgt=wgt, a_inc=a_inc)


def render_images(splats_per_view, views, layout, sorted_, view_arrays, keep_tiles=None):
    """Composite every tile (or the global tile ids in keep_tiles) of every
    view.  Returns per-view planar images and per-tile state for the
    adjoint.  Per pixel: `tie` (a near-tie decision; `cands` holds every
    output it may take), `excl` (more ties than are enumerated), `frag_geom`
    (a contributing splat's normal is a near tie) and `frag_grad` (any of
    these, or a tie that changes only the adjoint)."""
    out = []
    for v, view in enumerate(views):
        W, H = int(view.width), int(view.height)
        img = dict(rgb=np.zeros((3, H * W)), depth=np.zeros(H * W), depth_mag=np.zeros(H * W),
                   D=np.zeros(H * W),
                   normal=np.zeros((3, H * W)), normal_abs=np.zeros((3, H * W)),
                   alpha=np.zeros(H * W), T=np.ones(H * W),
                   last=np.zeros(H * W, np.int64), walked=np.zeros(H * W, np.int64),
                   tie=np.zeros(H * W, bool), excl=np.zeros(H * W, bool),
                   frag_geom=np.zeros(H * W, bool), frag_grad=np.zeros(H * W, bool),
                   covered=np.zeros(H * W, bool), cands={}, n_pair_ties=0, n_order_ties=0,
                   tiles={})
        out.append(img)
    n_tiles_total = int(layout["tile_off"][-1])
    tiles = range(n_tiles_total) if keep_tiles is None else keep_tiles
    for gtile in tiles:
        v = int(np.searchsorted(layout["tile_off"], gtile, side="right") - 1)
        local = gtile - int(layout["tile_off"][v])
        I, J = _tile_pixels(views[v], layout, v, local)
        s0, s1 = sorted_["ranges"][gtile]
        ent = sorted_["gid"][s0:s1]
        R = composite_tile(splats_per_view[v], ent, I, J, view_arrays[v],
                           own=sorted_["own"][s0:s1], cbit=sorted_["cbit"][s0:s1])
        pix = J * int(views[v].width) + I
        img = out[v]
        img["rgb"][:, pix] = R["rgb"].T
        img["depth"][pix] = R["dhat"]
        img["depth_mag"][pix] = R["dmag"]
        img["D"][pix] = R["D"]
        img["normal"][:, pix] = R["N"].T
        img["normal_abs"][:, pix] = R["Nabs"].T
        img["alpha"][pix] = R["alpha"]
        img["T"][pix] = R["T"]
        img["last"][pix] = R["last"]
        img["walked"][pix] = R["walked"]
        img["tie"][pix] = R["tie"]
        img["excl"][pix] = R["excl"]
        img["frag_geom"][pix] = R["frag_geom"]
        img["frag_grad"][pix] = R["frag_grad"]
        img["covered"][pix] = True
        img["n_pair_ties"] += R["n_pair_ties"]
        img["n_order_ties"] += R["n_order_ties"]
        for p, c in R["cands"].items():
            img["cands"][int(pix[p])] = c
        img["tiles"][gtile] = (ent, I, J, pix, R)
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
def composite_backward(splats_per_view, views, images, grads, view_arrays, magnitude=False):
    """Per-splat gradients (mean2d, conic, opacity, rgb, d, normal) for every
    view, from per-pixel output gradients.  Transmittances come from the
    forward products (no division).

    magnitude=True (the tests' conditioning model) returns instead, per
    element, the same sums taken over the absolute values of every term
    that enters them, cancelling differences included (the alpha adjoint
    T val - suffix / (1 - alpha) counts |T val| + |suffix| / (1 - alpha)):
    the scale of the rounding error a float32 evaluation of the element may
    make."""
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
            ab = np.abs if magnitude else (lambda x: x)
            GC = ab(g["rgb"][:, pix].T.copy())
            GD = ab(g["D"][pix].copy())
            GN = ab(g["normal"][:, pix].T.copy())
            GA = ab(g["alpha"][pix].copy())
            Gh = ab(g["depth"][pix])
            keep = R["keep"]
            sd = ab(np.where(keep, R["sdot"], 1.0))
            GD += np.where(keep, Gh / sd, 0.0)
            GN += np.where(keep, Gh * ab(R["D"]) / sd ** 2, 0.0)[:, None] * ab(R["ray"])
            dT = (GC @ Vv["bg"] + GA) if magnitude else (GC @ Vv["bg"] - GA)
            E = R["E"]
            inc = R["inc"]
            a_inc, Tb, wgt = R["a_inc"], R["Tb"], R["wgt"]
            rgb, d, nrm = ab(S["rgb"][ent]), ab(S["d"][ent]), ab(S["normal"][ent])
            val = GC @ rgb.T + GD[:, None] * d[None] + GN @ nrm.T
            wv = wgt * val
            suffix = np.cumsum(wv[:, ::-1], axis=1)[:, ::-1] - wv
            one_m = 1.0 - a_inc
            if magnitude:
                dalpha = Tb * val + suffix / one_m + (R["T"] * dT)[:, None] / one_m
            else:
                dalpha = Tb * val - suffix / one_m - (R["T"] * dT)[:, None] / one_m
            dalpha = np.where(inc, dalpha, 0.0)
            unclamped = inc & (E["raw"] < ALPHA_MAX)
            op = S["opacity"][ent][None]
            dop = np.where(unclamped, dalpha * E["G"], 0.0)
            dpower = np.where(unclamped, dalpha * op * E["G"], 0.0)
            a, b, c = ab(S["conic"][ent].T)
            dx, dy = ab(E["dx"]), ab(E["dy"])
            if magnitude:
                du = dpower * (a[None] * dx + b[None] * dy)
                dw = dpower * (c[None] * dy + b[None] * dx)
            else:
                du = dpower * (-(a[None] * dx + b[None] * dy))
                dw = dpower * (-(c[None] * dy + b[None] * dx))
            np.add.at(acc["mean2d"], ent, np.stack([du.sum(0), dw.sum(0)], 1))
            sg_ = 1.0 if magnitude else -1.0
            np.add.at(acc["conic"], ent, np.stack([(sg_ * 0.5 * dx * dx * dpower).sum(0),
                                                   (sg_ * dx * dy * dpower).sum(0),
                                                   (sg_ * 0.5 * dy * dy * dpower).sum(0)], 1))
            np.add.at(acc["opacity"], ent, dop.sum(0))
            np.add.at(acc["rgb"], ent, wgt.T @ GC)
            np.add.at(acc["d"], ent, wgt.T @ GD)
            np.add.at(acc["normal"], ent, wgt.T @ GN)
            fr = img["frag_grad"][pix]
            if fr.any():
                touched = (inc & fr[:, None]).any(axis=0)
                acc["frag"][ent[touched]] = True
    return res
