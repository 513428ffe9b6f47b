"""The fused chain captured in a hipGraph: every replay, with eager work and
synchronisations between replays, must reproduce the eager result (images
bit-identical; gradients equal up to the order of float atomics)."""
import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["anchor", "explicit_ncc"])
def test_graph_replays_match_eager(case):
    """anchor: a small anchor scene; explicit_ncc: two view pairs with the
    Eq. 10 term in the chain (its gradient plane is cleared by a kernel of
    the graph on every replay)."""
    print(f"case: graph replay, {case}", flush=True)
    from paper_2503_23044_amd import binding as B
    from paper_2503_23044_amd import render
    nt = None
    if case == "anchor":
        wl = scenes.make_small_anchor(31, n_anchor=80, n_views=3, sizes=((40, 32), (24, 36), (33, 17)))
    else:
        wl = scenes.make_view_pairs(25)
        c = torch.as_tensor(scenes.patch_centres(26, wl.views, 48), dtype=torch.int32, device="cuda")
        nt = dict(centres=c, n_patch=int(c.shape[1]), weight=0.5)
    rd = render.Renderer(0, (16, 16))
    sc = render.scene_from(wl.scene)
    cat = lambda xs: torch.as_tensor(np.concatenate([x.ravel() for x in xs]), device="cuda")  # noqa: E731
    tgt = dict(rgb=cat(wl.targets["rgb"]), depth=cat(wl.targets["depth"]), normal=cat(wl.targets["normal"]))
    loss = torch.zeros(1, device="cuda")
    out, gr = rd.fwd_bwd_l1(wl.views, sc, tgt, (1.0, 1.0, 1.0), loss=loss,
                            ncc=None if nt is None else (nt["centres"], nt["weight"]))
    torch.cuda.synchronize()
    ref_out = {k: v.clone() for k, v in out.items()}
    ref_gr = {k: v.clone() for k, v in gr.items()}
    ref_loss = loss.item()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g = B.cgx_graph_capture_fwd_bwd_l1(rd.ctx, wl.views, sc, rd.cap, rd.ws, tgt, (1.0, 1.0, 1.0),
                                           out, gr, loss, side, ncc=nt)
    side.synchronize()
    try:
        for rep in range(3):
            for v in list(out.values()) + list(gr.values()):
                v.fill_(float("nan"))
            loss.fill_(-1.0)
            junk = torch.randn(1000, device="cuda").sum()      # eager work between replays
            torch.cuda.synchronize()
            B.cgx_graph_launch(g, side)
            side.synchronize()
            for k in ref_out:
                assert torch.equal(out[k], ref_out[k]), (rep, k)
            for k in ref_gr:
                a, b = gr[k].double(), ref_gr[k].double()
                err = float((a - b).norm() / max(float(b.norm()), 1e-30))
                assert err < 1e-5, (rep, k, err)
            assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss), (rep, loss.item(), ref_loss)
            info = B.cgx_read_info(rd.ctx, rd.ws)
            assert info["overflow"] == 0
            del junk
    finally:
        B.cgx_graph_destroy(g)
