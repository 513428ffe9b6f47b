"""The Python boundary above the C ABI and the batching invariant.

* torch.autograd through RenderExplicit and RenderAnchor (the tanh masked
  opacity variant included) gives the oracle's gradients;
* each autograd forward call keeps its own state: two forward calls, then
  their backward calls in reverse order, each give their own gradients;
* batching (Sec. 3.3, views rendered together): the batched forward of the
  8-view C2 workload equals its eight single-view forward calls bit for
  bit, and the batched gradients equal the sum of the single-view ones to
  the atomics' rounding noise.
"""
import numpy as np
import pytest
import torch

from oracle import pipeline
from synth import scenes
from tests.parity import (anchor_sensitivity, check_grad, compare_images, explicit_sensitivity,
                          linear_grads, packed_grads)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2503_23044_amd import render
    return render


def _linear_loss(outs, og):
    g = packed_grads(og)
    names = ("rgb", "depth", "plane_d", "normal", "alpha")
    return sum((o.double() * g[k].double()).sum() for o, k in zip(outs, names))


def _explicit_leaves(sc):
    return [sc[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacity", "sh")]


def test_autograd_explicit(R):
    print("case: autograd through RenderExplicit, small SH1 scene", flush=True)
    wl = scenes.make_small_explicit(9, n=80, width=50, height=29, sh_degree=1, spread=0.6)
    rd = R.Renderer(0, (16, 16))
    sc = R.scene_from(wl.scene)
    leaves = _explicit_leaves(sc)
    outs = R.RenderExplicit.apply(rd, wl.views, wl.scene.sh_degree, *leaves)
    r = pipeline.render_explicit(wl.scene, wl.views)
    compare_images(dict(zip(("rgb", "depth", "plane_d", "normal", "alpha"), outs)), r)
    og = linear_grads(r, np.random.default_rng(3))
    grads = torch.autograd.grad(_linear_loss(outs, og), leaves)
    ref, _ = pipeline.backward(r, og, wl.scene)
    delta = explicit_sensitivity(wl.scene, wl.views, og, r0=r)
    for k, g in zip(("means", "scales", "quats", "opacity", "sh"), grads):
        check_grad("d_" + k, g.cpu().numpy(), ref[k], None, delta[k])


def _anchor_meta(sc):
    return dict(level=sc["level"], W1=sc["W1"], W2=sc["W2"], n_levels=sc["n_levels"],
                d_max=sc["d_max"], opacity_act=sc["opacity_act"], offset_mode=sc["offset_mode"],
                decoder_heads=sc["decoder_heads"])


def _anchor_leaves(sc):
    leaves = [sc[k].clone().requires_grad_(True) for k in ("x", "l", "O", "F", "b1", "b2")]
    W1f = torch.zeros(sc["W1"].shape, dtype=torch.float32, device="cuda", requires_grad=True)
    W2f = torch.zeros(sc["W2"].shape, dtype=torch.float32, device="cuda", requires_grad=True)
    return leaves + [W1f, W2f]


@pytest.mark.parametrize("act,offsets,heads", [(0, 0, 1), (1, 0, 1), (1, 1, 3)])
def test_autograd_anchor(R, act, offsets, heads):
    print(f"case: autograd through RenderAnchor, opacity_act={act} offset_mode={offsets} "
          f"decoder_heads={heads}", flush=True)
    wl = scenes.make_small_anchor(17 if act else 12, n_anchor=70, n_views=3,
                                  sizes=((40, 32), (24, 36), (33, 17)), opacity_act=act,
                                  offset_mode=offsets, decoder_heads=heads)
    rd = R.Renderer(0, (16, 16))
    sc = R.scene_from(wl.scene)
    assert (sc["opacity_act"], sc["offset_mode"], sc["decoder_heads"]) == (act, offsets, heads)
    leaves = _anchor_leaves(sc)
    outs = R.RenderAnchor.apply(rd, wl.views, _anchor_meta(sc), *leaves)
    r = pipeline.render_anchor(wl.scene, wl.views)
    compare_images(dict(zip(("rgb", "depth", "plane_d", "normal", "alpha"), outs)), r)
    og = linear_grads(r, np.random.default_rng(4))
    grads = torch.autograd.grad(_linear_loss(outs, og), leaves)
    ref, _ = pipeline.backward(r, og, wl.scene)
    delta = anchor_sensitivity(wl.scene, wl.views, og, r0=r)
    for k, g in zip(("x", "l", "O", "F", "b1", "b2", "W1", "W2"), grads):
        check_grad("d_" + k, g.cpu().numpy(), ref[k], None, delta[k])


def test_autograd_state_is_per_call(R):
    """Two forward calls on one renderer (different scenes, different
    capacities), then the backward calls in reverse order: each equals the
    gradient of a fresh single call."""
    print("case: two autograd forward calls before their backward calls", flush=True)
    wa = scenes.make_small_explicit(9, n=80, width=50, height=29, sh_degree=1, spread=0.6)
    wb = scenes.make_small_explicit(5, n=300, width=45, height=37, sh_degree=1, spread=0.5)
    wb.views = [wb.views[0]]
    rd = R.Renderer(0, (16, 16))
    sa, sb = R.scene_from(wa.scene), R.scene_from(wb.scene)
    la, lb = _explicit_leaves(sa), _explicit_leaves(sb)
    oa = R.RenderExplicit.apply(rd, wa.views, 1, *la)
    ob = R.RenderExplicit.apply(rd, wb.views, 1, *lb)
    ra = pipeline.render_explicit(wa.scene, wa.views)
    rb = pipeline.render_explicit(wb.scene, wb.views)
    ga_og, gb_og = linear_grads(ra, np.random.default_rng(5)), linear_grads(rb, np.random.default_rng(6))
    gb = torch.autograd.grad(_linear_loss(ob, gb_og), lb)
    ga = torch.autograd.grad(_linear_loss(oa, ga_og), la)
    for leaves, outs_og, wl, got in ((la, ga_og, wa, ga), (lb, gb_og, wb, gb)):
        fresh = R.Renderer(0, (16, 16))
        l2 = [t.detach().clone().requires_grad_(True) for t in leaves]
        o2 = R.RenderExplicit.apply(fresh, wl.views, 1, *l2)
        want = torch.autograd.grad(_linear_loss(o2, outs_og), l2)
        for a, b in zip(got, want):
            d = float((a.double() - b.double()).norm() / max(float(b.double().norm()), 1e-30))
            assert d < 1e-5, d


def test_batched_equals_per_view_c2(R):
    """The 8-view C2 batch rendered in one call and view by view: images bit
    for bit, gradients to the atomics' rounding noise."""
    print("case: C2 batched vs 8 single-view calls", flush=True)
    wl = scenes.make_c2()
    sc = R.scene_from(wl.scene)
    rd = R.Renderer(0, (16, 16))
    out = rd.forward(wl.views, sc)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    P = [int(v.width) * int(v.height) for v in wl.views]
    off = np.concatenate([[0], np.cumsum(P)])
    gout = {k: torch.as_tensor(rng.standard_normal(c * off[-1]).astype(np.float32), device="cuda")
            for k, c in (("rgb", 3), ("depth", 1), ("plane_d", 1), ("normal", 3), ("alpha", 1))}
    g_b = rd.backward(wl.views, sc, out, gout)
    torch.cuda.synchronize()
    g_sum = None
    for v, view in enumerate(wl.views):
        r1 = R.Renderer(0, (16, 16))
        o1 = r1.forward([view], sc)
        for k, c in (("rgb", 3), ("depth", 1), ("plane_d", 1), ("normal", 3), ("alpha", 1)):
            part = out[k][c * off[v]: c * off[v + 1]]
            assert torch.equal(o1[k], part), (v, k)
        g1out = {k: gout[k][c * off[v]: c * off[v + 1]].contiguous()
                 for k, c in (("rgb", 3), ("depth", 1), ("plane_d", 1), ("normal", 3), ("alpha", 1))}
        g1 = r1.backward([view], sc, o1, g1out)
        torch.cuda.synchronize()
        g_sum = {k: t.double() for k, t in g1.items()} if g_sum is None else \
            {k: g_sum[k] + g1[k].double() for k in g1}
    for k in g_b:
        a, b = g_b[k].double(), g_sum[k]
        d = float((a - b).norm() / max(float(b.norm()), 1e-30))
        print(f"  d_{k}: batched vs sum of single-view, norm rel diff {d:.2e}", flush=True)
        assert d < 1e-5, (k, d)
