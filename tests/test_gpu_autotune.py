"""Tile-shape autotuner and tile-shape invariance.  Images do not depend on
the tile shape (the pixel-box test and the per-pixel (depth, slot) order are
shape independent), so the forward images of every compiled shape must be
bit-identical; the autotuner must time every shape and pick one of them."""
import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu


def _targets(wl):
    cat = lambda xs: torch.as_tensor(np.concatenate([x.ravel() for x in xs]), device="cuda")  # noqa: E731
    return dict(rgb=cat(wl.targets["rgb"]), depth=cat(wl.targets["depth"]), normal=cat(wl.targets["normal"]))


def test_forward_identical_across_tile_shapes():
    print("case: tile-shape invariance, two-view anchor scene", flush=True)
    from paper_2503_23044_amd import binding as B
    from paper_2503_23044_amd import render
    wl = scenes.make_small_anchor(5, n_anchor=120, n_views=2, sizes=((77, 45), (40, 64)))
    sc = render.scene_from(wl.scene)
    ref = None
    for shape in B.TILE_SHAPES:
        rd = render.Renderer(0, shape)
        out = rd.forward(wl.views, sc)
        torch.cuda.synchronize()
        if ref is None:
            ref = {k: v.clone() for k, v in out.items()}
            continue
        for k in ref:
            assert torch.equal(out[k], ref[k]), (shape, k)


def test_autotune_picks_a_timed_shape(tmp_path):
    print("case: autotune C0", flush=True)
    from paper_2503_23044_amd import binding as B
    from paper_2503_23044_amd import render
    wl = scenes.make_c0()
    sc = render.scene_from(wl.scene)
    tgt = _targets(wl)
    cache = str(tmp_path / "tiles.json")
    rd = render.Renderer(0, (16, 16))
    best, ms = rd.autotune(wl.views, sc, tgt, reps=2, cache=cache)
    assert best in B.TILE_SHAPES and rd.tile == best
    assert set(ms) == set(B.TILE_SHAPES)
    assert all(v > 0 for v in ms.values()), ms
    assert ms[best] == min(ms.values())
    # the renderer keeps working with the chosen shape, and the cache answers next time
    loss = torch.zeros(1, device="cuda")
    rd.fwd_bwd_l1(wl.views, sc, tgt, loss=loss)
    torch.cuda.synchronize()
    assert np.isfinite(loss.item()) and loss.item() > 0
    rd2 = render.Renderer(0, (16, 16))
    best2, ms2 = rd2.autotune(wl.views, sc, tgt, cache=cache)
    assert best2 == best and ms2 == {}
