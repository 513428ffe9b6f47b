"""The allocation-free depth-prior alignment (cgx_depth_prior_align_noalloc)
against the workspace entry point (cgx_depth_prior_align) it varies, through
the C ABI: both run the same kernels in the same order, so the per-view
scale / shift and the aligned prior must be bit-identical.  Two calls in a
row, the second on a smaller input (fewer views and points), check that the
fixed partial-sum array carries nothing over from the first call.  Views
beyond the array's bound are rejected before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from synth import scenes

pytestmark = pytest.mark.gpu


def _inputs(X, n_views, n_points):
    views = X.views[:n_views]
    prior = torch.from_numpy(np.concatenate(X.prior[:n_views]).astype(np.float32)).cuda()
    pts = torch.from_numpy(np.ascontiguousarray(X.points[:n_points], np.float32)).cuda()
    return views, prior, pts


def _with_workspace(B, ctx, views, prior, pts):
    ws = torch.empty(B.cgx_depth_align_workspace_size(len(views)), dtype=torch.uint8, device="cuda")
    st = torch.empty(len(views), 2, dtype=torch.float64, device="cuda")
    al = torch.empty_like(prior)
    B.cgx_depth_prior_align(ctx, views, prior, pts, ws, st, al)
    return st, al


def _no_alloc(B, ctx, views, prior, pts):
    st = torch.full((len(views), 2), float("nan"), dtype=torch.float64, device="cuda")
    al = torch.full_like(prior, float("nan"))
    B.cgx_depth_prior_align_noalloc(ctx, views, prior, pts, st, al)
    return st, al


def test_no_alloc_alignment_matches_workspace_call():
    print("case: allocation-free depth-prior alignment, 8 then 3 views", flush=True)
    from paper_2503_23044_amd import binding as B
    from paper_2503_23044_amd import render
    rd = render.Renderer(0)
    X = scenes.make_depth_prior(n_pairs=4, width=640, height=360, n_points=200_000)
    for n_views, n_points in ((8, 200_000), (3, 50_000)):
        views, prior, pts = _inputs(X, n_views, n_points)
        st_ref, al_ref = _with_workspace(B, rd.ctx, views, prior, pts)
        st, al = _no_alloc(B, rd.ctx, views, prior, pts)
        torch.cuda.synchronize()
        assert torch.equal(st, st_ref), (n_views, st.cpu().numpy(), st_ref.cpu().numpy())
        assert torch.equal(al, al_ref), n_views
        s = st.cpu().numpy()
        assert np.all(np.isfinite(s)) and np.all(s[:, 0] != 1.0), s    # aligned from the points
        print(f"  {n_views} views, {n_points} points: scale/shift and aligned prior bit-identical",
              flush=True)


def test_no_alloc_alignment_rejects_too_many_views():
    print("case: allocation-free alignment, view bound", flush=True)
    from paper_2503_23044_amd import binding as B
    from paper_2503_23044_amd import render
    rd = render.Renderer(0)
    X = scenes.make_depth_prior(n_pairs=1, width=64, height=48, n_points=100)
    views = list(X.views) * 17          # 34 views > the 32 the array holds
    prior = torch.zeros(sum(int(v.width) * int(v.height) for v in views), device="cuda")
    st = torch.zeros(len(views), 2, dtype=torch.float64, device="cuda")
    lib = B.load_library()
    rc = lib.cgx_depth_prior_align_noalloc(rd.ctx, B.make_views(views), len(views),
                                           ctypes.c_void_p(prior.data_ptr()), None, 0,
                                           ctypes.c_void_p(st.data_ptr()), None, None)
    assert rc != 0
