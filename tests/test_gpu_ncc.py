"""GPU parity of the batch geometric loss (Sec. 3.4, Eq. 10) against the
FP64 oracle, through the C ABI: the loss kernel on identical input images,
then the whole chain forward -> loss -> backward raster -> projection
adjoint."""
import copy

import numpy as np
import pytest
import torch

from oracle import ncc, pipeline
from synth import scenes
from tests.parity import (SENS_EPS, _perturbed, check_close, check_grad, compare_images,
                          oracle_images_packed, rounding_sensitivity)

pytestmark = pytest.mark.gpu


def _oracle_ncc(r, centres, weight):
    return ncc.ncc_loss(r.images, r.varr, centres, weight=weight)


def _to_planar(grads):
    """Per-view (3, npx) arrays -> the packed planar layout of the ABI."""
    return np.concatenate([np.asarray(g, np.float64).ravel() for g in grads])


def _fragile_pixels(r, centres, info):
    """Packed-rgb mask of the pixels of patches with a fragile validity decision."""
    masks = [np.zeros((3, im["depth"].size), bool) for im in r.images]
    h = 3
    for i, k in zip(*np.nonzero(info["fragile"])):
        v = r.views[2 * i + 1]
        cx, cy = centres[i, k]
        for dy in range(-h, h + 1):
            for dx in range(-h, h + 1):
                x, y = cx + dx, cy + dy
                if 0 <= x < v.width and 0 <= y < v.height:
                    masks[2 * i + 1][:, y * v.width + x] = True
    return np.concatenate([m.ravel() for m in masks])


def test_ncc_kernel_on_oracle_images():
    print("case: NCC loss kernel, 2 pairs x 64 patches, oracle images as input", flush=True)
    from paper_2503_23044_amd import render
    wl = scenes.make_view_pairs(11)
    centres = scenes.patch_centres(12, wl.views, 64)
    r = pipeline.render_explicit(wl.scene, wl.views)
    rd = render.Renderer(0, (16, 16))
    sc = render.scene_from(wl.scene)
    rd.forward(wl.views, sc)                       # fills the workspace view table
    imgs = {k: torch.as_tensor(oracle_images_packed(r, ok, c).astype(np.float32), device="cuda")
            for k, ok, c in (("rgb", "rgb", 3), ("normal", "normal", 3), ("plane_d", "D", 1))}
    # the oracle sees exactly the float32 images the kernel reads
    r32 = copy.copy(r)
    r32.images = []
    for im in r.images:
        d = dict(im)
        for k in ("rgb", "normal", "D"):
            d[k] = np.asarray(im[k], np.float32).astype(np.float64)
        r32.images.append(d)
    weight = 0.8
    loss_ref, g_ref, info = _oracle_ncc(r32, centres, weight)
    assert info["valid"].sum() > 64
    g, loss = rd.ncc_loss(wl.views, imgs, torch.as_tensor(centres), weight)
    torch.cuda.synchronize()
    n_frag = int(info["fragile"].sum())
    scale = weight / (len(wl.views) // 2 * centres.shape[1])
    assert abs(loss.item() - loss_ref) <= 1e-5 * weight + 2 * scale * n_frag, (loss.item(), loss_ref)
    # the two terms of d NCC / d a nearly cancel when NCC is close to 1: the
    # float32 error follows the sum of |terms| (as for the normal map)
    check_close("d_rgb (NCC)", g.cpu().numpy(), _to_planar(g_ref), _fragile_pixels(r32, centres, info),
                mag=_to_planar(info["gmag"]))
    # accumulation: a second call adds the same amounts
    g2, loss2 = rd.ncc_loss(wl.views, imgs, torch.as_tensor(centres), weight, grad_rgb=g.clone(), loss=loss.clone())
    torch.cuda.synchronize()
    np.testing.assert_allclose(g2.cpu().numpy(), 2 * g.cpu().numpy(), rtol=1e-6, atol=1e-12)
    assert abs(loss2.item() - 2 * loss.item()) <= 1e-6 * abs(loss.item()) + 1e-12


def _chain_grads(scene, views, centres, weight, r=None):
    r = r or pipeline.render_explicit(scene, views)
    _, g_rgb, info = _oracle_ncc(r, centres, weight)
    og = []
    for img, gr in zip(r.images, g_rgb):
        n = img["depth"].size
        og.append(dict(rgb=gr, depth=np.zeros(n), D=np.zeros(n), normal=np.zeros((3, n)), alpha=np.zeros(n)))
    g, _ = pipeline.backward(r, og, scene)
    return g, r, og, info


def _tied_patches(r, centres, patch=7):
    """Patches that read a pixel with a near-tie decision: in their
    reference window (view 2i+1) or in the bilinear footprint of their
    warped window in the source view (2i).  The GPU seeds the NCC gradient
    from its own images, which may resolve those ties the other way."""
    h = patch // 2
    n_pairs = len(r.images) // 2
    centres = np.asarray(centres).reshape(n_pairs, -1, 2)
    tied = np.zeros(centres.shape[:2], bool)
    oy, ox = np.mgrid[-h:h + 1, -h:h + 1]
    for i in range(n_pairs):
        s_, t_ = 2 * i, 2 * i + 1
        vr, vs = r.varr[t_], r.varr[s_]
        ref_tie, src_tie = r.images[t_]["frag_grad"], r.images[s_]["frag_grad"]
        for k, (cx, cy) in enumerate(centres[i]):
            px, py = (cx + ox).ravel(), (cy + oy).ravel()
            ok = (px >= 0) & (py >= 0) & (px < vr["W"]) & (py < vr["H"])
            if ref_tie[(py * vr["W"] + px)[ok]].any():
                tied[i, k] = True
                continue
            if not ok.all():
                continue
            pc = cy * vr["W"] + cx
            n = r.images[t_]["normal"][:, pc]
            d = float(r.images[t_]["D"][pc])
            if not d > 0:
                continue
            q = ncc.homography(vr, vs, n, d) @ np.stack([px + 0.5, py + 0.5, np.ones(px.size)])
            if not np.all(q[2] > 0):
                continue
            sx, sy = q[0] / q[2] - 0.5, q[1] / q[2] - 0.5
            x0 = np.clip(np.floor(sx).astype(np.int64), 0, vs["W"] - 2)
            y0 = np.clip(np.floor(sy).astype(np.int64), 0, vs["H"] - 2)
            foot = np.concatenate([y * vs["W"] + x for y in (y0, y0 + 1) for x in (x0, x0 + 1)])
            tied[i, k] = bool(src_tie[foot].any())
    return tied


def test_ncc_through_backward_matches_oracle():
    print("case: forward -> NCC -> backward, 2 pairs x 48 patches", flush=True)
    from paper_2503_23044_amd import render
    wl = scenes.make_view_pairs(21)
    centres = scenes.patch_centres(22, wl.views, 48)
    weight = 1.0
    r = pipeline.render_explicit(wl.scene, wl.views)
    # patches that read a near-tie pixel (the GPU may resolve the tie the
    # other way) or whose validity is itself a near tie are moved outside
    # the image, where both sides drop them: every other patch is compared
    # exactly, with no share of the gradient set aside
    _, _, info0 = _oracle_ncc(r, centres, weight)
    tied = _tied_patches(r, centres) | info0["fragile"].reshape(-1, centres.shape[1])
    print(f"  patches reading a near-tie pixel: {int(tied.sum())}/{tied.size}", flush=True)
    assert tied.mean() < 0.2
    c_eff = np.asarray(centres).reshape(tied.shape[0], -1, 2).copy()
    c_eff[tied] = -100
    c_eff = c_eff.reshape(np.asarray(centres).shape)
    ref, r, og, info = _chain_grads(wl.scene, wl.views, c_eff, weight, r=r)
    rd = render.Renderer(0, (16, 16))
    sc = render.scene_from(wl.scene)
    out = rd.forward(wl.views, sc)
    compare_images(out, r)
    g_rgb, loss = rd.ncc_loss(wl.views, out, torch.as_tensor(c_eff), weight)
    zero = torch.zeros_like(out["depth"])
    gout = dict(rgb=g_rgb, depth=zero, plane_d=zero, normal=torch.zeros_like(out["normal"]), alpha=zero)
    gr = rd.backward(wl.views, sc, out, gout)
    torch.cuda.synchronize()
    loss_ref, _, _ = _oracle_ncc(r, c_eff, weight)
    assert abs(loss.item() - loss_ref) <= 1e-4 * abs(loss_ref) + 1e-6, (loss.item(), loss_ref)
    # conditioning of the whole chain: the oracle's gradient under float32-size input perturbation
    sens = None
    for seed in (4321, 8765):
        rng = np.random.default_rng(seed)
        sc2 = copy.copy(wl.scene)
        for k in ("means", "scales", "quats", "opacity", "sh"):
            setattr(sc2, k, _perturbed(getattr(wl.scene, k), rng))
        g1, _, _, _ = _chain_grads(sc2, wl.views, c_eff, weight)
        d = {k: np.abs(ref[k] - g1[k]) for k in ("means", "scales", "quats", "opacity", "sh")}
        sens = d if sens is None else {k: np.maximum(sens[k], d[k]) for k in d}
    assert SENS_EPS > 0
    keys = ("means", "scales", "quats", "opacity", "sh")
    sr = rounding_sensitivity(r, og, wl.scene, keys, g0=ref)
    for k in keys:
        check_grad("d_" + k, gr[k].cpu().numpy(), ref[k], None, dict(sens=sens[k], round=sr[k]))


def test_ncc_fused_in_chain_matches_oracle():
    """The fused chain with the Eq. 10 term: forward, then the L1 seeds and
    the NCC gradient folded into one backward prologue; against the oracle's
    L1 + NCC output gradients through its backward pass."""
    print("case: fused chain forward -> L1 + NCC -> backward, 2 pairs x 48 patches", flush=True)
    from paper_2503_23044_amd import render
    from tests.parity import targets_at_ties, zero_ties
    wl = scenes.make_view_pairs(23)
    centres = scenes.patch_centres(24, wl.views, 48)
    weight, w3 = 0.5, (1.0, 0.5, 0.25)
    r = pipeline.render_explicit(wl.scene, wl.views)
    _, _, info0 = _oracle_ncc(r, centres, weight)
    tied = _tied_patches(r, centres) | info0["fragile"].reshape(-1, centres.shape[1])
    print(f"  patches reading a near-tie pixel: {int(tied.sum())}/{tied.size}", flush=True)
    assert tied.mean() < 0.2
    c_eff = np.asarray(centres).reshape(tied.shape[0], -1, 2).copy()
    c_eff[tied] = -100
    rd = render.Renderer(0, (16, 16))
    sc = render.scene_from(wl.scene)
    out0 = rd.forward(wl.views, sc)
    torch.cuda.synchronize()
    compare_images(out0, r)
    targets = targets_at_ties(out0, r, wl.targets)
    cat = lambda xs: torch.as_tensor(np.concatenate([np.asarray(x).ravel() for x in xs]), device="cuda")  # noqa: E731
    tgt = dict(rgb=cat(targets["rgb"]), depth=cat(targets["depth"]), normal=cat(targets["normal"]))
    loss = torch.zeros(1, device="cuda")
    out, gr = rd.fwd_bwd_l1(wl.views, sc, tgt, w3, loss=loss, ncc=(torch.as_tensor(c_eff), weight))
    torch.cuda.synchronize()
    for k in out:
        assert torch.equal(out[k], out0[k]), k
    c_flat = c_eff.reshape(np.asarray(centres).shape)

    def fused_ref(scene, r=None):
        r = r or pipeline.render_explicit(scene, wl.views)
        L, og = pipeline.output_grads_l1(r, targets, w3)
        og = zero_ties(r, og)
        Ln, g_rgb, _ = _oracle_ncc(r, c_flat, weight)
        for o, g in zip(og, g_rgb):
            o["rgb"] = o["rgb"] + g
        g, _ = pipeline.backward(r, og, scene)
        return g, L + Ln, og

    ref, L_ref, og = fused_ref(wl.scene, r)
    assert abs(loss.item() - L_ref) <= 1e-4 * abs(L_ref), (loss.item(), L_ref)
    keys = ("means", "scales", "quats", "opacity", "sh")
    sens = None
    for seed in (4321, 8765):
        rng = np.random.default_rng(seed)
        sc2 = copy.copy(wl.scene)
        for k in keys:
            setattr(sc2, k, _perturbed(getattr(wl.scene, k), rng))
        g1, _, _ = fused_ref(sc2)
        d = {k: np.abs(ref[k] - g1[k]) for k in keys}
        sens = d if sens is None else {k: np.maximum(sens[k], d[k]) for k in d}
    sr = rounding_sensitivity(r, og, wl.scene, keys, g0=ref)
    for k in keys:
        check_grad("d_" + k, gr[k].cpu().numpy(), ref[k], None, dict(sens=sens[k], round=sr[k]))
