"""The radix sorts' digit width is a speed knob only (binning, Sec. 3.3):
the pairs' order is that of the 64-bit (tile | depth) keys with slot ties
whatever the digit split, so every width gives the same sorted pairs, tile
ranges and images, bit for bit.  Run on the C2 workload (16-bit tile ids:
two 8-bit passes at widths 9 and 8, three at 7; the 32-bit depth keys take
four passes at 9 and 8, five at 7) and on a 17-bit-tile anchor scene."""
import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu


def _run(R, wl, bits, tile=(16, 16)):
    rd = R.Renderer(0, tile)
    rd.set_sort_digit_bits(bits)
    sc = R.scene_from(wl.scene)
    out = rd.forward(wl.views, sc)
    torch.cuda.synchronize()
    dbg = rd.debug()
    return rd, {k: v.clone() for k, v in out.items()}, dbg


@pytest.mark.parametrize("case", ["c2", "tiles17"])
def test_digit_widths_sort_identically(case):
    print(f"case: sort digit widths, {case}", flush=True)
    from paper_2503_23044_amd import render as R
    if case == "c2":
        wl = scenes.make_c2()
        tile = (16, 16)
    else:
        # 8x8 tiles over two 1600x1200 views: 60,000 tiles, 16 bits; with a
        # third view 90,000 tiles, 17 bits (9 + 8 at width 9, 6 + 6 + 5 at 7)
        wl = scenes.make_c4(n_anchor=200_000, n_views=3)
        tile = (8, 8)
    ref = None
    for bits in (9, 8, 7):
        rd, out, dbg = _run(R, wl, bits, tile)
        info = dbg["info"]
        assert info["overflow"] == 0
        if ref is None:
            ref = (out, dbg)
            assert info["n_pairs"] > 0
            continue
        out0, dbg0 = ref
        for k in ("tile", "zbits", "slot", "ranges"):
            assert np.array_equal(dbg[k], dbg0[k]), (bits, k)
        for k in out0:
            assert torch.equal(out[k], out0[k]), (bits, k)


def test_digit_setting_and_tuner():
    print("case: digit setting and tuner", flush=True)
    from paper_2503_23044_amd import binding as B
    from paper_2503_23044_amd import render as R
    wl = scenes.make_small_anchor(41, n_anchor=80, n_views=3, sizes=((40, 32), (24, 36), (33, 17)))
    rd = R.Renderer(0, (16, 16))
    assert B.cgx_get_sort_digit_bits(rd.ctx) == 9
    sc = R.scene_from(wl.scene)
    cat = lambda xs: torch.as_tensor(np.concatenate([x.ravel() for x in xs]), device="cuda")  # noqa: E731
    tgt = dict(rgb=cat(wl.targets["rgb"]), depth=cat(wl.targets["depth"]), normal=cat(wl.targets["normal"]))
    shape, ms = rd.autotune(wl.views, sc, tgt, reps=2)
    assert rd.digit_bits in B.DIGIT_CHOICES
    assert B.cgx_get_sort_digit_bits(rd.ctx) == rd.digit_bits
    assert set(rd.digit_ms) == set(B.DIGIT_CHOICES) and all(v > 0 for v in rd.digit_ms.values())
    assert shape in B.TILE_SHAPES and ms[shape] > 0
