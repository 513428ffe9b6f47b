"""GPU parity of the explicit-Gaussian path (a2-a9) against the FP64 oracle,
through the C ABI.  Images and gradients within 1e-4 relative (floored),
sorted pairs bit-exact with nothing dropped; near ties resolved by the
oracle's enumeration of their outcomes."""
import copy

import numpy as np
import pytest
import torch

from oracle import pipeline
from synth import scenes
from tests.parity import (check_grad, check_sort_properties, compare_images,
                          compare_sort_explicit, explicit_sensitivity, linear_grads, packed_grads,
                          targets_at_ties, tie_fraction, zero_ties)

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


def _explicit_grads_check(gr, ref, sh_degree, delta, report=None):
    for k in ("means", "scales", "quats", "opacity", "sh"):
        check_grad("d_" + k, gr[k].cpu().numpy(), ref[k], None, delta[k], report=report)


def test_c0_forward_and_sort(R):
    print("case: C0 forward", flush=True)
    wl = scenes.make_c0()
    rd, sc, out = _run_forward(R, wl)
    r = pipeline.render_explicit(wl.scene, wl.views)
    compare_images(out, r)
    dbg = rd.debug()
    n, took, left = compare_sort_explicit(dbg, r, wl.scene.n)
    rec, _ = rd.debug_splats()
    N = wl.scene.n
    assert check_sort_properties(dbg, rec, wl.views, rd.tile, lambda s: s // N) == n
    # work counters (off by default): entries walked forward equal the
    # oracle's count over its own lists, up to the pixels of near ties and
    # the near-tie pairs the GPU took (each adds at most one entry to each of
    # its tile's pixels)
    assert dbg["info"]["entries_fwd"] == 0 and dbg["info"]["evals_fwd"] == 0
    rd.count_work(True)
    out2 = rd.forward(wl.views, sc)
    torch.cuda.synchronize()
    for k in out:
        assert torch.equal(out[k], out2[k]), k
    info = rd.info()
    walked = sum(int(img["walked"].sum()) for img in r.images)
    ties = sum(int(img["tie"].sum()) for img in r.images)
    slack = ties * 8 + took * rd.tile[0] * rd.tile[1]
    assert abs(info["entries_fwd"] - walked) <= slack, (info["entries_fwd"], walked, slack)
    assert 0 < info["evals_fwd"] <= info["entries_fwd"]


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
    rd, sc, out0 = _run_forward(R, wl)
    r = pipeline.render_explicit(wl.scene, wl.views)
    compare_images(out0, r)
    # targets equal to the GPU's own outputs at the near-tie pixels: both
    # seeds vanish there
    targets = targets_at_ties(out0, r, wl.targets)
    tgt = dict(rgb=torch.as_tensor(np.concatenate([t.ravel() for t in targets["rgb"]]), device="cuda"),
               depth=torch.as_tensor(np.concatenate(targets["depth"]), device="cuda"),
               normal=torch.as_tensor(np.concatenate([t.ravel() for t in targets["normal"]]), device="cuda"))
    loss = torch.zeros(1, device="cuda")
    out, gr = rd.fwd_bwd_l1(wl.views, sc, tgt, (1.0, 1.0, 1.0), loss=loss)
    torch.cuda.synchronize()
    for k in out:
        assert torch.equal(out[k], out0[k]), k
    L, og = pipeline.output_grads_l1(r, targets)
    og = zero_ties(r, og)
    ref, _ = pipeline.backward(r, og, wl.scene)
    assert abs(loss.item() - L) <= 1e-4 * abs(L)
    delta = explicit_sensitivity(wl.scene, wl.views, og, r0=r)
    _explicit_grads_check(gr, ref, 0, delta)


def _linear_case(R, wl, tile, seed, sh_degree, views=None):
    views = views or wl.views
    rd, sc, out = _run_forward(R, wl, tile)
    r = pipeline.render_explicit(wl.scene, views, tile=tile)
    compare_images(out, r)
    compare_sort_explicit(rd.debug(), r, wl.scene.n)
    og = linear_grads(r, np.random.default_rng(seed))
    print(f"  output gradients zeroed on {tie_fraction(r):.2e} of the pixels (near ties)", flush=True)
    ref, _ = pipeline.backward(r, og, wl.scene)
    delta = explicit_sensitivity(wl.scene, views, og, tile=tile, r0=r)
    gr = rd.backward(views, sc, out, packed_grads(og))
    torch.cuda.synchronize()
    _explicit_grads_check(gr, ref, sh_degree, delta)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8)])
def test_small_explicit_sh3_tiles_backward(R, tile):
    print(f"case: small SH3 tile {tile}", flush=True)
    wl = scenes.make_small_explicit(5, n=60, width=45, height=37, sh_degree=3, spread=0.5,
                                    log_scale=-2.3)
    v = wl.views[0]
    v.R = np.array([[0.98, -0.17, 0.1], [0.17, 0.985, 0.0], [-0.1, 0.02, 0.995]], np.float32)
    v.R = (np.linalg.qr(v.R.astype(np.float64))[0] * np.sign(np.diag(np.linalg.qr(v.R.astype(np.float64))[1]))).astype(np.float32)
    _linear_case(R, wl, tile, 77, 3)


def test_c0_linear_backward(R):
    print("case: C0 linear-loss backward", flush=True)
    _linear_case(R, scenes.make_c0(), (16, 16), 79, 0)


def test_two_views_ragged_background(R):
    print("case: two views ragged", flush=True)
    wl = scenes.make_small_explicit(9, n=80, width=50, height=29, sh_degree=1, spread=0.6)
    v2 = copy.deepcopy(wl.views[0])
    v2.width, v2.height, v2.cx, v2.cy = 23, 41, 11.5, 20.5
    v2.t = np.array([0.1, -0.05, 2.2], np.float32)
    v2.bg = (0.25, 0.5, 0.75)
    wl.views = [wl.views[0], v2]
    _linear_case(R, wl, (16, 16), 78, 1)


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
