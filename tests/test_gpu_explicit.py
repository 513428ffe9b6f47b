"""GPU parity of the explicit-Gaussian path (a2-a9) against the FP64 oracle,
through the C ABI.  Images and gradients within 1e-4 relative (floored),
sorted pairs bit-exact."""
import copy

import numpy as np
import pytest
import torch

from oracle import pipeline
from synth import scenes
from tests.parity import (check_grad, compare_images, compare_sort_explicit,
                          explicit_sensitivity)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2503_23044_amd import render
    return render


def _run_forward(R, wl, tile=(16, 16)):
    rd = R.Renderer(0, tile)
    sc = R.scene_from(wl.scene)
    out = rd.forward(wl.views, sc)
    torch.cuda.synchronize()
    return rd, sc, out


def _explicit_grads_check(gr, ref, frag, sh_degree, delta, report=None):
    ex = frag
    K = (sh_degree + 1) ** 2
    for k, c in (("means", 3), ("scales", 3), ("quats", 4), ("opacity", 1), ("sh", 3 * K)):
        check_grad("d_" + k, gr[k].cpu().numpy(), ref[k], np.repeat(ex, c), delta[k], report=report)


def test_c0_forward_and_sort(R):
    print("case: C0 forward", flush=True)
    wl = scenes.make_c0()
    rd, sc, out = _run_forward(R, wl)
    r = pipeline.render_explicit(wl.scene, wl.views)
    compare_images(out, r)
    dbg = rd.debug()
    assert dbg["info"]["n_pairs"] == r.sorted["gtile"].size
    compare_sort_explicit(dbg, r, wl.scene.n)
    walked = sum(int(img["walked"].sum()) for img in r.images)
    assert dbg["info"]["entries_fwd"] == walked


@pytest.mark.parametrize("masked", [False, True])
def test_c0_fused_l1_backward(R, masked):
    print(f"case: C0 fused L1 masked={masked}", flush=True)
    wl = scenes.make_c0()
    if masked:
        # depth-prior mask: pixels the filter removed carry a non-positive or
        # NaN target depth and add no depth term
        rng = np.random.default_rng(41)
        dep = []
        for t in wl.targets["depth"]:
            t = np.array(t, np.float32)
            u = rng.random(t.size)
            t[u < 0.30] = 0.0
            t[(u >= 0.30) & (u < 0.35)] = np.nan
            t[(u >= 0.35) & (u < 0.40)] = -1.0
            dep.append(t)
        wl.targets["depth"] = dep
    rd = R.Renderer(0, (16, 16))
    sc = R.scene_from(wl.scene)
    P = wl.pixels
    tgt = dict(rgb=torch.as_tensor(np.concatenate([t.ravel() for t in wl.targets["rgb"]]), device="cuda"),
               depth=torch.as_tensor(np.concatenate(wl.targets["depth"]), device="cuda"),
               normal=torch.as_tensor(np.concatenate([t.ravel() for t in wl.targets["normal"]]), device="cuda"))
    loss = torch.zeros(1, device="cuda")
    out, gr = rd.fwd_bwd_l1(wl.views, sc, tgt, (1.0, 1.0, 1.0), loss=loss)
    torch.cuda.synchronize()
    r = pipeline.render_explicit(wl.scene, wl.views)
    compare_images(out, r)
    L, og = pipeline.output_grads_l1(r, wl.targets)
    ref, _ = pipeline.backward(r, og, wl.scene)
    assert abs(loss.item() - L) <= 1e-4 * abs(L)
    delta = explicit_sensitivity(wl.scene, wl.views, og)
    _explicit_grads_check(gr, ref, ref["frag"], 0, delta)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8)])
def test_small_explicit_sh3_tiles_backward(R, tile):
    print(f"case: small SH3 tile {tile}", flush=True)
    wl = scenes.make_small_explicit(5, n=60, width=45, height=37, sh_degree=3, spread=0.5,
                                    log_scale=-2.3)
    v = wl.views[0]
    v.R = np.array([[0.98, -0.17, 0.1], [0.17, 0.985, 0.0], [-0.1, 0.02, 0.995]], np.float32)
    v.R = (np.linalg.qr(v.R.astype(np.float64))[0] * np.sign(np.diag(np.linalg.qr(v.R.astype(np.float64))[1]))).astype(np.float32)
    rd, sc, out = _run_forward(R, wl, tile)
    r = pipeline.render_explicit(wl.scene, wl.views, tile=tile)
    compare_images(out, r)
    compare_sort_explicit(rd.debug(), r, wl.scene.n)
    rng = np.random.default_rng(77)
    L, og = pipeline.output_grads_linear(r, rng)
    ref, _ = pipeline.backward(r, og, wl.scene)
    delta = explicit_sensitivity(wl.scene, wl.views, og, tile=tile)
    gout = {}
    for key, okey, c in (("rgb", "rgb", 3), ("depth", "depth", 1), ("plane_d", "D", 1),
                         ("normal", "normal", 3), ("alpha", "alpha", 1)):
        gout[key] = torch.as_tensor(np.concatenate([g[okey].ravel() for g in og]).astype(np.float32),
                                    device="cuda")
    gr = rd.backward(wl.views, sc, out, gout)
    torch.cuda.synchronize()
    _explicit_grads_check(gr, ref, ref["frag"], 3, delta)


def test_two_views_ragged_background(R):
    print("case: two views ragged", flush=True)
    wl = scenes.make_small_explicit(9, n=80, width=50, height=29, sh_degree=1, spread=0.6)
    v2 = copy.deepcopy(wl.views[0])
    v2.width, v2.height, v2.cx, v2.cy = 23, 41, 11.5, 20.5
    v2.t = np.array([0.1, -0.05, 2.2], np.float32)
    v2.bg = (0.25, 0.5, 0.75)
    views = [wl.views[0], v2]
    wl.views = views
    rd, sc, out = _run_forward(R, wl)
    r = pipeline.render_explicit(wl.scene, views)
    compare_images(out, r)
    compare_sort_explicit(rd.debug(), r, wl.scene.n)
    rng = np.random.default_rng(78)
    L, og = pipeline.output_grads_linear(r, rng)
    ref, _ = pipeline.backward(r, og, wl.scene)
    delta = explicit_sensitivity(wl.scene, views, og)
    gout = {}
    for key, okey, c in (("rgb", "rgb", 3), ("depth", "depth", 1), ("plane_d", "D", 1),
                         ("normal", "normal", 3), ("alpha", "alpha", 1)):
        gout[key] = torch.as_tensor(np.concatenate([g[okey].ravel() for g in og]).astype(np.float32),
                                    device="cuda")
    gr = rd.backward(views, sc, out, gout)
    torch.cuda.synchronize()
    _explicit_grads_check(gr, ref, ref["frag"], 1, delta)


def test_degenerate_scenes(R):
    print("case: degenerate", flush=True)
    wl = scenes.make_small_explicit(3, n=20)
    # everything behind the camera: nothing is drawn, alpha = 0, depth = 0
    wl.scene.means[:, 2] = -10.0
    rd, sc, out = _run_forward(R, wl)
    assert float(out["alpha"].abs().max()) == 0.0
    assert float(out["depth"].abs().max()) == 0.0
    assert rd.info()["n_pairs"] == 0
    # an empty scene
    wl0 = scenes.make_small_explicit(3, n=1)
    for k in ("means", "scales", "quats", "opacity", "sh"):
        setattr(wl0.scene, k, getattr(wl0.scene, k)[:0])
    rd0, sc0, out0 = _run_forward(R, wl0)
    assert float(out0["alpha"].abs().max()) == 0.0
    gout = {k: torch.ones_like(v) for k, v in out0.items()}
    gr = rd0.backward(wl0.views, sc0, out0, gout)
    torch.cuda.synchronize()
    assert gr["means"].numel() == 0
