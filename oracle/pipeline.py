"""The whole rasterizer chain, explicit Gaussians or voxel anchors, forward
and adjoint (oracle, test infrastructure).

Chain (Sec. 3.2-3.3): [anchor selection -> decode (Eq. 4)] -> projection ->
tile binning and (tile | depth) sort -> front-to-back compositing of RGB,
D, N and alpha (Eqs. 5-7) -> unbiased depth; then the adjoint in reverse.
"""
import numpy as np

from . import anchors as anc
from . import project as prj
from . import raster as ras


class Result:
    """Forward state kept for the adjoint."""


def render_explicit(scene, views, tile=(16, 16), keep_tiles=None):
    """Render every view of an explicit-Gaussian scene.  Splat gid = the
    Gaussian's index."""
    layout = ras.batch_layout(views, tile)
    means = np.asarray(scene.means, np.float64)
    splats, varr = [], []
    for view in views:
        S = prj.project(means, scene.scales, scene.quats, scene.opacity, view, tile,
                        sh=scene.sh, sh_degree=scene.sh_degree)
        splats.append(S)
        varr.append(prj.view_arrays(view))
    srt = ras.bin_and_sort(splats, layout, keep_tiles)
    imgs = ras.render_images(splats, views, layout, srt, varr, keep_tiles)
    r = Result()
    r.kind, r.layout, r.splats, r.sorted, r.images, r.varr, r.views = (
        "explicit", layout, splats, srt, imgs, varr, views)
    return r


def render_anchor(scene, views, tile=(16, 16), emulate_bf16=True, keep_tiles=None):
    """Render every view of an anchor scene.  Splat gid within a view =
    row_in_view * n + k (rows in anchor order), so gid order equals
    (anchor, k) order."""
    layout = ras.batch_layout(views, tile)
    rows, offs = anc.select(scene, views)
    D = anc.decode(scene, views, rows, emulate_bf16)
    n = D["n"]
    splats, varr = [], []
    for v, view in enumerate(views):
        sl = slice(offs[v] * n, offs[v + 1] * n)
        S = prj.project(D["mu"][sl], D["scales"][sl], D["quats"][sl], D["opacity"][sl],
                        view, tile, colour=D["rgb"][sl], opacity_exact=False,
                        mu_tol=None if D["mu_tol"] is None else D["mu_tol"][sl])
        rfr = np.repeat(D["frag_relu"][offs[v]:offs[v + 1]], n)
        S["frag_grad"] = S["frag_grad"] | (S["valid"] & rfr)
        splats.append(S)
        varr.append(prj.view_arrays(view))
    srt = ras.bin_and_sort(splats, layout, keep_tiles)
    imgs = ras.render_images(splats, views, layout, srt, varr, keep_tiles)
    r = Result()
    r.kind, r.layout, r.splats, r.sorted, r.images, r.varr, r.views = (
        "anchor", layout, splats, srt, imgs, varr, views)
    r.rows, r.row_off, r.decoded = rows, offs, D
    return r


def output_grads_l1(r, targets, weights=(1.0, 1.0, 1.0)):
    return ras.l1_seed(r.images, targets, weights)


def output_grads_linear(r, rng):
    """A smooth linear loss L = sum w * out with w ~ N(0,1) on every output
    (rgb, unbiased depth, plane distance, normal, alpha); used for gradient
    checks so that finite differences never meet an L1 kink."""
    gs = []
    L = 0.0
    for img in r.images:
        npx = img["depth"].size
        g = dict(rgb=rng.standard_normal((3, npx)), depth=rng.standard_normal(npx),
                 D=rng.standard_normal(npx), normal=rng.standard_normal((3, npx)),
                 alpha=rng.standard_normal(npx))
        L += (np.sum(g["rgb"] * img["rgb"]) + np.sum(g["depth"] * img["depth"])
              + np.sum(g["D"] * img["D"]) + np.sum(g["normal"] * img["normal"])
              + np.sum(g["alpha"] * img["alpha"]))
        gs.append(g)
    return L, gs


def linear_loss(r, gs):
    L = 0.0
    for img, g in zip(r.images, gs):
        L += (np.sum(g["rgb"] * img["rgb"]) + np.sum(g["depth"] * img["depth"])
              + np.sum(g["D"] * img["D"]) + np.sum(g["normal"] * img["normal"])
              + np.sum(g["alpha"] * img["alpha"]))
    return L


def backward(r, out_grads, scene, sg_hook=None):
    """Adjoint of the whole chain.  Returns (scene gradients, per-view splat
    gradients).  Explicit: means, scales, quats, opacity, sh (summed over
    views).  Anchor: x, l, O, F, W1, b1, W2, b2.  sg_hook (tests'
    conditioning probes) may replace the per-view splat gradients before the
    projection adjoint."""
    sg = ras.composite_backward(r.splats, r.views, r.images, out_grads, r.varr)
    if sg_hook is not None:
        sg = sg_hook(sg)
    if r.kind == "explicit":
        acc = None
        for v, S in enumerate(r.splats):
            pg = prj.project_backward(S, sg[v])
            if acc is None:
                acc = {k: pg[k].copy() for k in ("mu", "scales", "quats", "opacity", "sh")}
            else:
                for k in acc:
                    acc[k] += pg[k]
        grads = dict(means=acc["mu"], scales=acc["scales"], quats=acc["quats"],
                     opacity=acc["opacity"], sh=acc["sh"])
        # Gaussians that draw on a pixel with a near-tie decision
        frag = np.zeros(scene.means.shape[0], bool)
        for v, S in enumerate(r.splats):
            frag |= sg[v]["frag"]
        grads["frag"] = frag
        return grads, sg
    n = r.decoded["n"]
    parts = {k: [] for k in ("mu", "scales", "quats", "opacity", "rgb")}
    frag_rows = []
    for v, S in enumerate(r.splats):
        pg = prj.project_backward(S, sg[v])
        for k in parts:
            parts[k].append(pg[k])
        frag_rows.append(sg[v]["frag"].reshape(-1, n).any(axis=1))
    g = {k: np.concatenate(v, 0) for k, v in parts.items()}
    grads = anc.decode_backward(scene, r.decoded, g)
    frag_rows = np.concatenate(frag_rows) if frag_rows else np.zeros(0, bool)
    fa = np.zeros(scene.x.shape[0], bool)
    np.logical_or.at(fa, r.rows[:, 1], frag_rows)
    grads["frag"] = fa
    return grads, sg
