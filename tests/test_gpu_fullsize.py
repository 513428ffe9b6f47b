"""GPU parity at the full benchmark shapes, on a seeded sample of tiles.

The whole workload is rendered on the GPU in the benchmark's launch
configuration; the oracle selects, decodes and projects everything but bins,
sorts and composites only the sampled tiles.  The backward pass is driven
by a linear loss that is non-zero only on the sampled tiles' pixels (and
zero at the pixels with a near-tie decision), so every gradient the GPU
returns comes from pixels the oracle also computes, and every gradient
element is compared.
"""
import numpy as np
import pytest
import torch

from oracle import pipeline
from synth import scenes
from tests.parity import (anchor_sensitivity, check_grad, check_sort_properties, compare_images,
                          compare_sorted, explicit_sensitivity, linear_grads, packed_grads,
                          tie_fraction)

pytestmark = pytest.mark.gpu


def _sample_tiles(layout, n, seed):
    rng = np.random.default_rng(seed)
    total = int(layout["tile_off"][-1])
    return np.sort(rng.choice(total, min(n, total), replace=False))


def _anchor_slot_map(rows, r, n_off=10):
    def s2vg(slots):
        row, k = slots // n_off, slots % n_off
        v = rows[row, 0]
        return v, (row - r.row_off[v]) * n_off + k
    return s2vg


def _check_anchor_grads(gr, ref, delta):
    for k in ("x", "l", "O", "F", "W1", "b1", "W2", "b2"):
        check_grad("d_" + k, gr[k].cpu().numpy(), ref[k], None, delta[k])


def test_c2_full_size_sampled_tiles():
    print("case: C2 full size, 24 sampled tiles", flush=True)
    from paper_2503_23044_amd import render
    wl = scenes.make_c2()
    rd = render.Renderer(0, (16, 16))
    sc = render.scene_from(wl.scene)
    out = rd.forward(wl.views, sc)
    torch.cuda.synchronize()
    dbg = rd.debug()
    rows_gpu = dbg["rows"].astype(np.int64)
    rec, _ = rd.debug_splats()
    assert check_sort_properties(dbg, rec, wl.views, (16, 16), lambda s: rows_gpu[s // 10, 0]) > 10**6
    layout = pipeline.ras.batch_layout(wl.views, (16, 16))
    keep = _sample_tiles(layout, 24, seed=2024)
    r = pipeline.render_anchor(wl.scene, wl.views, keep_tiles=keep)
    np.testing.assert_array_equal(dbg["rows"].astype(np.int64), r.rows)
    n, took, left = compare_sorted(dbg, r, _anchor_slot_map(r.rows, r), tiles=keep)
    print(f"  sorted pairs of the sampled tiles: {n} bit-exact (near-tie taken {took}, left {left})")
    assert n > 1000
    compare_images(out, r, covered_only=True)
    og = linear_grads(r, np.random.default_rng(7), covered_only=True)
    print(f"  output gradients zeroed on {tie_fraction(r):.2e} of the pixels (near ties)", flush=True)
    ref, _ = pipeline.backward(r, og, wl.scene)
    gr = rd.backward(wl.views, sc, out, packed_grads(og))
    torch.cuda.synchronize()
    d2 = anchor_sensitivity(wl.scene, wl.views, og, keep_tiles=keep, r0=r)
    _check_anchor_grads(gr, ref, d2)


def test_c1_full_size_sampled_tiles():
    print("case: C1 full size (1M Gaussians, SH3, 1080p), 20 sampled tiles", flush=True)
    from paper_2503_23044_amd import render
    wl = scenes.make_c1()
    rd = render.Renderer(0, (16, 16))
    sc = render.scene_from(wl.scene)
    out = rd.forward(wl.views, sc)
    torch.cuda.synchronize()
    dbg = rd.debug()
    layout = pipeline.ras.batch_layout(wl.views, (16, 16))
    keep = _sample_tiles(layout, 20, seed=2025)
    r = pipeline.render_explicit(wl.scene, wl.views, keep_tiles=keep)
    N = wl.scene.n
    n, took, left = compare_sorted(dbg, r, lambda s: (s // N, s % N), tiles=keep)
    print(f"  sorted pairs of the sampled tiles: {n} bit-exact (near-tie taken {took}, left {left})")
    assert n > 1000
    compare_images(out, r, covered_only=True)
    og = linear_grads(r, np.random.default_rng(8), covered_only=True)
    print(f"  output gradients zeroed on {tie_fraction(r):.2e} of the pixels (near ties)", flush=True)
    ref, _ = pipeline.backward(r, og, wl.scene)
    gr = rd.backward(wl.views, sc, out, packed_grads(og))
    torch.cuda.synchronize()
    delta = explicit_sensitivity(wl.scene, wl.views, og, keep_tiles=keep, r0=r)
    for k in ("means", "scales", "quats", "opacity", "sh"):
        check_grad("d_" + k, gr[k].cpu().numpy(), ref[k], None, delta[k])


def _grads_view0(r, n_total, rng):
    """Linear output gradients on view 0's sampled tiles (zero at near ties),
    zero on the other views, packed for the whole batch."""
    og = linear_grads(r, rng, covered_only=True)
    g = og[0]
    n0 = g["depth"].size
    pad = n_total - n0
    # the packed layout is view-major: view 0's planes, then the other views'
    z3 = lambda a: np.concatenate([np.asarray(a).ravel(), np.zeros(3 * pad)])  # noqa: E731
    z1 = lambda a: np.concatenate([a, np.zeros(pad)])  # noqa: E731
    dev = dict(rgb=z3(g["rgb"]), depth=z1(g["depth"]), plane_d=z1(g["D"]), normal=z3(g["normal"]),
               alpha=z1(g["alpha"]))
    dev = {k: torch.as_tensor(v.ravel().astype(np.float32), device="cuda") for k, v in dev.items()}
    return og, dev


def _anchor_view0_case(wl, rd, sc, out, n_tiles, seed, tile=(16, 16)):
    """Sort, images and gradients of view 0 on sampled tiles against the
    single-view oracle (views are independent: view 0's rows, pairs and
    pixels are its own; anchor gradients get only view 0's share because
    the output gradients vanish elsewhere)."""
    v0 = wl.views[0]
    dbg = rd.debug()
    rows_all = dbg["rows"].astype(np.int64)
    rec, _ = rd.debug_splats()
    check_sort_properties(dbg, rec, wl.views, tile, lambda s: rows_all[s // 10, 0])
    layout = pipeline.ras.batch_layout([v0], tile)
    keep = _sample_tiles(layout, n_tiles, seed=seed)
    r = pipeline.render_anchor(wl.scene, [v0], tile=tile, keep_tiles=keep)
    rows_gpu = dbg["rows"].astype(np.int64)
    rows0 = rows_gpu[rows_gpu[:, 0] == 0]
    np.testing.assert_array_equal(rows0, r.rows)

    def s2vg(slots):
        row, k = slots // 10, slots % 10
        v = rows_gpu[row, 0]
        assert np.all(v == 0)
        return v, (row - 0) * 10 + k       # view 0's rows come first

    n, took, left = compare_sorted(dbg, r, s2vg, tiles=keep)
    print(f"  sorted pairs of the sampled tiles: {n} bit-exact (near-tie taken {took}, left {left})")
    assert n > 500
    W, H = v0.width, v0.height
    view0 = {k: out[k][:c * W * H] for k, c in (("rgb", 3), ("depth", 1), ("plane_d", 1), ("normal", 3),
                                              ("alpha", 1))}
    compare_images(view0, r, covered_only=True)
    og, gdev = _grads_view0(r, int(out["depth"].numel()), np.random.default_rng(seed + 1))
    print(f"  output gradients zeroed on {tie_fraction(r):.2e} of the pixels (near ties)", flush=True)
    ref, _ = pipeline.backward(r, og, wl.scene)
    gr = rd.backward(wl.views, sc, out, gdev)
    torch.cuda.synchronize()
    sens = anchor_sensitivity(wl.scene, [v0], og, tile=tile, keep_tiles=keep, r0=r)
    _check_anchor_grads(gr, ref, sens)
    return dbg


def test_c3_full_size_sampled_tiles():
    print("case: C3 full size (600k anchors, 4 views 3840x2160), 16 sampled tiles of view 0", flush=True)
    from paper_2503_23044_amd import render
    wl = scenes.make_c3()
    rd = render.Renderer(0, (16, 16))
    sc = render.scene_from(wl.scene)
    out = rd.forward(wl.views, sc)
    torch.cuda.synchronize()
    info = rd.info()
    print(f"  rows {info['n_rows']} pairs {info['n_pairs']}", flush=True)
    _anchor_view0_case(wl, rd, sc, out, 16, seed=2030)


def test_c4_graph_autotuned_sampled_tiles():
    print("case: C4 full size (2M anchors, 16 views 1600x1200), autotuned tile, graph replay", flush=True)
    from paper_2503_23044_amd import binding as B
    from paper_2503_23044_amd import render
    wl = scenes.make_c4()
    sc = render.scene_from(wl.scene)
    cat = lambda xs: torch.as_tensor(np.concatenate([x.ravel() for x in xs]), device="cuda")  # noqa: E731
    tgt = dict(rgb=cat(wl.targets["rgb"]), depth=cat(wl.targets["depth"]), normal=cat(wl.targets["normal"]))
    rd = render.Renderer(0, (16, 16))
    tile, ms = rd.autotune(wl.views, sc, tgt, reps=1)
    print(f"  autotuned tile {tile}: {ms}", flush=True)
    loss = torch.zeros(1, device="cuda")
    out, gr = rd.fwd_bwd_l1(wl.views, sc, tgt, loss=loss)      # eager, fits the capacities
    out, gr = rd.fwd_bwd_l1(wl.views, sc, tgt, out=out, grads=gr, loss=loss)
    torch.cuda.synchronize()
    ref_out = {k: v.clone() for k, v in out.items()}
    ref_gr = {k: v.clone() for k, v in gr.items()}
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g = B.cgx_graph_capture_fwd_bwd_l1(rd.ctx, wl.views, sc, rd.cap, rd.ws, tgt, (1.0, 1.0, 1.0),
                                           out, gr, loss, side)
    side.synchronize()
    try:
        for v in list(out.values()) + list(gr.values()):
            v.fill_(float("nan"))
        torch.cuda.synchronize()
        B.cgx_graph_launch(g, side)
        side.synchronize()
        assert B.cgx_read_info(rd.ctx, rd.ws)["overflow"] == 0
        for k in ref_out:
            assert torch.equal(out[k], ref_out[k]), k
        for k in ref_gr:
            a, b = gr[k].double(), ref_gr[k].double()
            assert float((a - b).norm() / max(float(b.norm()), 1e-30)) < 1e-5, k
    finally:
        B.cgx_graph_destroy(g)
    # the replayed images against the oracle, view 0, in the tuned tile shape
    dbg = _anchor_view0_case(wl, rd, sc, out, 16, seed=2040, tile=tuple(tile))
    # With this many slots a depth-sort entry keeps 7 bits for the splat's
    # tile count above its slot; larger counts hold the escape and are read
    # from the slot. Both kinds occur here, and every splat's pair count was
    # checked above.
    n_slots = int(rd.cap["max_rows"]) * 10
    bits = max(1, (n_slots - 1).bit_length())
    esc = (1 << (32 - bits)) - 1
    counts = np.asarray(dbg["counts"]).astype(np.int64)
    print(f"  slot bits {bits}: {int((counts >= esc).sum())} splats at the count escape {esc}",
          flush=True)
    assert 32 - bits >= 4
    assert (counts >= esc).any() and ((counts > 0) & (counts < esc)).any()
