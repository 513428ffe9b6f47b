"""Batch-level geometric loss of Sec. 3.4, Eq. 10 (oracle, test
infrastructure): normalised cross-correlation between a 7x7 patch of one
view of a pair and the same surface patch seen from the other view, the
latter found through the plane-induced homography of the rendered normal
and plane distance, under a stop-gradient.

Readings of what the paper leaves open:

  * pairs are views (2i, 2i+1) of the batch (0-based); the patch centres
    p lie in the second view (the reference, which receives the gradient)
    and the warped patch is sampled from the first view (the source, under
    stop-gradient); an odd last view has no partner;
  * the caller supplies P integer patch centres per pair (the random draw of
    the paper is an input); a patch is valid when all its pixels are inside
    the reference image, the rendered plane distance at its centre is
    positive, every warped pixel centre lies in front of the source camera
    and inside the source image's sampling range [0, W-1] x [0, H-1] (in
    pixel-index coordinates); invalid patches add zero;
  * the plane is the reference view's rendered plane at the patch centre:
    normal n = N(p) and distance d = D(p) in the reference camera frame, so
    that n . X = -d on the plane (d = -n . X >= 0); n is used unnormalised,
    only the ratio n / d enters, which the blend weights do not change when
    all contributors share one plane;
  * with X_s = R_rel X_r + t_rel (R_rel = R_s R_r^T, t_rel = t_s - R_rel
    t_r), the homography from reference to source pixels is
    H = K_s (R_rel - t_rel n^T / d) K_r^-1 on homogeneous pixel centres
    (x + 0.5, y + 0.5, 1);
  * intensities are the mean of the three RGB channels; the source is
    sampled bilinearly at (u - 0.5, v - 0.5) in pixel-index coordinates;
  * NCC(a, b) = sum(A B) / sqrt(sum(A^2) sum(B^2) + eps), A = a - mean(a),
    B = b - mean(b), eps = 1e-8;
  * L = (1 / n_pairs) sum_pairs (1 / P) sum_valid patches (1 - NCC), scaled by
    a weight w.
"""
import numpy as np

NCC_EPS = 1e-8
FRAG_EDGE = 1e-4


def _K(va):
    return np.array([[va["fx"], 0.0, va["cx"]], [0.0, va["fy"], va["cy"]], [0.0, 0.0, 1.0]])


def homography(va_r, va_s, n, d):
    """Plane-induced homography reference -> source (3x3, float64)."""
    R_rel = va_s["R"] @ va_r["R"].T
    t_rel = va_s["t"] - R_rel @ va_r["t"]
    M = R_rel - np.outer(t_rel, n) / d
    return _K(va_s) @ M @ np.linalg.inv(_K(va_r))


def gray(img_rgb):
    """Mean of the RGB channels; img_rgb is (3, npx)."""
    return (img_rgb[0] + img_rgb[1] + img_rgb[2]) / 3.0


def bilinear(img, W, H, sx, sy):
    """Bilinear sample of a (H*W,) image at pixel-index coordinates."""
    x0 = np.floor(sx).astype(np.int64)
    y0 = np.floor(sy).astype(np.int64)
    x0 = np.clip(x0, 0, W - 2)
    y0 = np.clip(y0, 0, H - 2)
    fx = sx - x0
    fy = sy - y0
    g = img.reshape(H, W)
    return ((1 - fy) * ((1 - fx) * g[y0, x0] + fx * g[y0, x0 + 1])
            + fy * ((1 - fx) * g[y0 + 1, x0] + fx * g[y0 + 1, x0 + 1]))


def ncc_loss(images, view_arrays, centres, patch=7, weight=1.0):
    """Eq. 10 over the batch.

    images: per-view dicts with rgb (3, npx), normal (3, npx), D (npx);
    view_arrays: per-view dicts from project.view_arrays;
    centres: int array (n_pairs, P, 2) of (x, y) in each pair's reference view.
    Returns (loss, grads, info): grads is a list of per-view (3, npx) arrays
    of dL/drgb (zero for source views); info holds per-patch validity, NCC
    and a fragile flag (a validity decision within FRAG_EDGE of its bound).
    """
    B = len(images)
    n_pairs = B // 2
    centres = np.asarray(centres, np.int64).reshape(n_pairs, -1, 2)
    P = centres.shape[1]
    h = patch // 2
    oy, ox = np.mgrid[-h:h + 1, -h:h + 1]
    ox, oy = ox.ravel(), oy.ravel()
    grads = [np.zeros_like(np.asarray(im["rgb"], np.float64)) for im in images]
    # per pixel, the sum of |terms| of its gradient (the scale of float32 error
    # in a sum that nearly cancels when NCC is close to 1)
    gmag = [np.zeros_like(g) for g in grads]
    valid = np.zeros((n_pairs, P), bool)
    fragile = np.zeros((n_pairs, P), bool)
    nccs = np.zeros((n_pairs, P))
    loss = 0.0
    for i in range(n_pairs):
        s, r = 2 * i, 2 * i + 1
        vr, vs = view_arrays[r], view_arrays[s]
        Wr, Hr, Ws, Hs = vr["W"], vr["H"], vs["W"], vs["H"]
        a_img = gray(np.asarray(images[r]["rgb"], np.float64))
        b_img = gray(np.asarray(images[s]["rgb"], np.float64))
        for k in range(P):
            cx, cy = int(centres[i, k, 0]), int(centres[i, k, 1])
            px, py = cx + ox, cy + oy
            if px.min() < 0 or py.min() < 0 or px.max() >= Wr or py.max() >= Hr:
                continue
            pc = cy * Wr + cx
            n = np.asarray(images[r]["normal"], np.float64)[:, pc]
            d = float(images[r]["D"][pc])
            if not d > 0.0:
                continue
            Hm = homography(vr, vs, n, d)
            q = Hm @ np.stack([px + 0.5, py + 0.5, np.ones(px.size)])
            if not np.all(q[2] > 0):
                continue
            sx = q[0] / q[2] - 0.5
            sy = q[1] / q[2] - 0.5
            lo = min(sx.min(), sy.min())
            hi_x, hi_y = sx.max() - (Ws - 1), sy.max() - (Hs - 1)
            edge = min(abs(sx.min()), abs(sy.min()), abs(hi_x), abs(hi_y))
            if lo < 0 or hi_x > 0 or hi_y > 0:
                fragile[i, k] = edge < FRAG_EDGE
                continue
            fragile[i, k] = edge < FRAG_EDGE
            a = a_img[py * Wr + px]
            b = bilinear(b_img, Ws, Hs, sx, sy)
            A = a - a.mean()
            Bc = b - b.mean()
            sab, saa, sbb = np.sum(A * Bc), np.sum(A * A), np.sum(Bc * Bc)
            den = np.sqrt(saa * sbb + NCC_EPS)
            ncc = sab / den
            valid[i, k] = True
            nccs[i, k] = ncc
            scale = weight / (n_pairs * P)
            loss += scale * (1.0 - ncc)
            # d ncc / d a_j = B_j / den - sab sbb A_j / den^3 (sum B = 0)
            dn = Bc / den - sab * sbb * A / den ** 3
            ga = -scale * dn / 3.0
            gm = scale * (np.abs(Bc / den) + np.abs(sab * sbb * A / den ** 3)) / 3.0
            for c in range(3):
                np.add.at(grads[r][c], py * Wr + px, ga)
                np.add.at(gmag[r][c], py * Wr + px, gm)
    return loss, grads, dict(valid=valid, ncc=nccs, fragile=fragile, gmag=gmag)
