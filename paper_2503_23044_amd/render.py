"""Object wrapper over the C ABI: device tensors in, images and gradients
out, with workspace sizing and capacity growth, and a torch.autograd.Function.

All work runs in libcgx.so on torch's current stream; this module only
allocates tensors and marshals pointers.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import binding as B

IMAGE_CHANNELS = {"rgb": 3, "depth": 1, "plane_d": 1, "normal": 3, "alpha": 1}


def explicit_scene(means, scales, quats, opacity, sh, sh_degree, device="cuda"):
    """Device tensors of an explicit-Gaussian scene (float32, contiguous)."""
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)  # noqa: E731
    return dict(kind=B.CGX_SCENE_EXPLICIT, means=f(means), scales=f(scales), quats=f(quats),
                opacity=f(opacity), sh=f(sh), sh_degree=int(sh_degree))


def anchor_scene(x, l, O, F, level, W1_bits, b1, W2_bits, b2, n_levels, d_max, device="cuda",
                 opacity_act=B.OPACITY_SIGMOID, offset_mode=B.OFFSETS_TABLE,
                 decoder_heads=B.DECODER_SHARED):
    """Device tensors of a voxel-anchor scene; decoder weights as bfloat16
    bit patterns (held in int16 tensors).  opacity_act: B.OPACITY_SIGMOID or
    B.OPACITY_TANH_MASK (tanh, non-positive opacities masked); offset_mode:
    B.OFFSETS_TABLE (O) or B.OFFSETS_DECODED (14 decoder outputs per
    Gaussian); decoder_heads: B.DECODER_SHARED (W1 36 x 32) or
    B.DECODER_PER_ATTRIBUTE (W1 36 x 96, or 36 x 128 with decoded offsets)."""
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=device)  # noqa: E731
    bits = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.uint16).view(np.int16), device=device)  # noqa: E731
    return dict(kind=B.CGX_SCENE_ANCHOR, x=f(x), l=f(l), O=f(O), F=f(F),
                level=torch.as_tensor(np.ascontiguousarray(level, np.uint8), device=device),
                W1=bits(W1_bits), b1=f(b1), W2=bits(W2_bits), b2=f(b2),
                n_levels=int(n_levels), d_max=float(d_max), opacity_act=int(opacity_act),
                offset_mode=int(offset_mode), decoder_heads=int(decoder_heads))


def scene_from(obj, device="cuda"):
    """Build the device scene from a generator scene object."""
    if hasattr(obj, "means"):
        return explicit_scene(obj.means, obj.scales, obj.quats, obj.opacity, obj.sh, obj.sh_degree, device)
    return anchor_scene(obj.x, obj.l, obj.O, obj.F, obj.level, obj.W1_bits, obj.b1, obj.W2_bits,
                        obj.b2, obj.n_levels, obj.d_max, device,
                        getattr(obj, "opacity_act", B.OPACITY_SIGMOID),
                        getattr(obj, "offset_mode", B.OFFSETS_TABLE),
                        getattr(obj, "decoder_heads", B.DECODER_SHARED))


def pixel_offsets(views):
    sizes = [int(v.width) * int(v.height) if not isinstance(v, dict) else int(v["width"]) * int(v["height"])
             for v in views]
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def split_image(flat, views, channels):
    """Per-view [C, H, W] views of a packed planar image."""
    off = pixel_offsets(views)
    out = []
    for i, v in enumerate(views):
        W = int(v.width) if not isinstance(v, dict) else int(v["width"])
        H = int(v.height) if not isinstance(v, dict) else int(v["height"])
        out.append(flat[channels * off[i]: channels * off[i + 1]].view(channels, H, W))
    return out


def grad_buffers(scene, device="cuda"):
    if scene["kind"] == B.CGX_SCENE_EXPLICIT:
        return {k: torch.zeros_like(scene[k]) for k in ("means", "scales", "quats", "opacity", "sh")}
    g = {k: torch.zeros_like(scene[k]) for k in ("x", "l", "O", "F", "b1", "b2")}
    g["W1"] = torch.zeros(scene["W1"].shape, dtype=torch.float32, device=device)
    g["W2"] = torch.zeros(scene["W2"].shape, dtype=torch.float32, device=device)
    return g


def workload_key(views, scene):
    """Signature of a workload for the tile-shape cache: scene kind and
    size, SH degree, and the view resolutions."""
    if scene["kind"] == B.CGX_SCENE_EXPLICIT:
        head = f"explicit:n={scene['means'].shape[0]}:sh={scene['sh_degree']}"
    else:
        head = f"anchor:n={scene['x'].shape[0]}"
    dim = lambda v, k: int(v[k] if isinstance(v, dict) else getattr(v, k))  # noqa: E731
    res = ",".join(f"{dim(v, 'width')}x{dim(v, 'height')}" for v in views)
    return f"{head}:views={res}"


class Renderer:
    """One rasterizer context (device, tile shape) with its workspace."""

    def __init__(self, device: int = 0, tile=(16, 16)):
        self.device = device
        self.tile = tuple(tile)
        self.ctx = B.cgx_create(device, tile[0], tile[1])
        self.digit_bits = B.cgx_get_sort_digit_bits(self.ctx)
        self.digit_ms = {}
        self.ws = None
        self.depth_ws = None
        self.tsdf_ws = None
        self.cap = {}

    def __del__(self):
        try:
            if getattr(self, "ctx", None) is not None:
                B.cgx_destroy(self.ctx)
        except Exception:
            pass

    # ------------------------------------------------------------------
    # first-call capacities: a run that needs more overflows, reports what it
    # needed, and is repeated with grown capacities
    FIRST_ROWS = 1 << 22
    FIRST_PAIRS = 1 << 26

    def ensure_workspace(self, views, scene, cap=None):
        if cap is None and getattr(self, "_next_cap", None) is not None:
            cap, self._next_cap = self._next_cap, None
        cap = dict(cap or self.cap)
        if not cap:
            if scene["kind"] == B.CGX_SCENE_ANCHOR:
                rows = min(int(scene["x"].shape[0]) * len(views), self.FIRST_ROWS)
                splats = rows * int(scene["O"].shape[1])
                cap = dict(max_rows=rows)
            else:
                splats = int(scene["means"].shape[0]) * len(views)
            cap["max_pairs"] = min(max(8 * splats, 1024), self.FIRST_PAIRS)
        n = B.cgx_workspace_size(self.ctx, views, scene, cap)
        n = (n + 255) // 256 * 256
        if self.ws is None or self.ws.numel() < n or self.ws.numel() > 2 * n:
            self.ws = None
            self.ws = torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")
        self.cap = cap
        return self.ws

    def alloc_images(self, views):
        P = int(pixel_offsets(views)[-1])
        dev = f"cuda:{self.device}"
        return {k: torch.empty(c * P, dtype=torch.float32, device=dev) for k, c in IMAGE_CHANNELS.items()}

    def _grow(self, info):
        cap = dict(self.cap)
        if info["overflow"] & 4:
            cap["max_pairs"] = int(info["need_pairs"] * 1.25) + 1024
        if info["overflow"] & 1:
            cap["max_rows"] = int(info["need_rows"] * 1.25) + 64
        self.cap = cap

    def _fit(self, info, scene):
        """After a run within capacity: capacities more than 4x what it
        needed are brought down to 1.25x for the NEXT forward call (the
        kernels' grids and the workspace are sized by them; the state of the
        run just made stays valid for its backward).  A later run that needs
        more overflows and grows them again."""
        cap = dict(self.cap)
        want_pairs = int(info["n_pairs"] * 1.25) + 1024
        if cap.get("max_pairs", 0) == 0 or cap["max_pairs"] > 4 * want_pairs:
            cap["max_pairs"] = want_pairs
        if scene["kind"] == B.CGX_SCENE_ANCHOR:
            want_rows = int(info["n_rows"] * 1.25) + 64
            if cap.get("max_rows", 0) == 0 or cap["max_rows"] > 4 * want_rows:
                cap["max_rows"] = want_rows
        self._next_cap = cap if cap != self.cap else None

    def forward(self, views, scene, out=None, check=True):
        """Render; returns the packed images.  With check, reads the status
        (synchronises) and re-runs with larger capacities on overflow."""
        for _ in range(4):
            ws = self.ensure_workspace(views, scene)
            out = out if out is not None else self.alloc_images(views)
            B.cgx_render_forward(self.ctx, views, scene, self.cap, ws, out)
            if not check:
                return out
            info = B.cgx_read_info(self.ctx, ws, raise_on_capacity=False)
            if not info["overflow"]:
                self.last_info = info
                self._fit(info, scene)
                return out
            self._grow(info)
        raise B.CgxError(B.CGX_ERR_CAPACITY, "capacity still exceeded after growing")

    def backward(self, views, scene, out, grad_out, grads=None, state=None):
        """Gradients of the forward call whose state is `state` (from
        take_state), or of this renderer's last forward call."""
        grads = grads if grads is not None else grad_buffers(scene, f"cuda:{self.device}")
        if state is None:
            B.cgx_render_backward(self.ctx, views, scene, self.cap, self.ws, out, grad_out, grads)
            return grads
        if state["ctx"] is not self.ctx or state["tile"] != self.tile:
            raise RuntimeError("the renderer's tile shape changed between this forward call and its "
                               "backward call")
        B.cgx_render_backward(self.ctx, views, scene, state["cap"], state["ws"], out, grad_out, grads)
        return grads

    def take_state(self):
        """Detach the forward state of the last forward call (its workspace,
        capacities and tile shape) from the renderer: the next forward call
        gets a workspace of its own, so the detached state stays valid for a
        later backward call."""
        state = dict(ws=self.ws, cap=dict(self.cap), tile=self.tile, ctx=self.ctx)
        self.ws = None
        return state

    def fwd_bwd_l1(self, views, scene, target, weights=(1.0, 1.0, 1.0), out=None, grads=None,
                   loss=None, check=True, ncc=None):
        """Fused forward, L1 loss (Eq. 8) and backward; ncc=(centres, weight)
        adds the geometric loss of Eq. 10 with patch centres given as an
        int32 device tensor (n_views // 2, n_patch, 2)."""
        nt = None
        if ncc is not None:
            c = ncc[0].to(device=f"cuda:{self.device}", dtype=torch.int32).contiguous()
            nt = dict(centres=c, n_patch=int(c.shape[1]), weight=float(ncc[1]))
        for _ in range(4):
            ws = self.ensure_workspace(views, scene)
            out = out if out is not None else self.alloc_images(views)
            grads = grads if grads is not None else grad_buffers(scene, f"cuda:{self.device}")
            B.cgx_render_fwd_bwd_l1(self.ctx, views, scene, self.cap, ws, target, weights, out,
                                    grads, loss, ncc=nt)
            if not check:
                return out, grads
            info = B.cgx_read_info(self.ctx, ws, raise_on_capacity=False)
            if not info["overflow"]:
                self.last_info = info
                self._fit(info, scene)
                return out, grads
            self._grow(info)
        raise B.CgxError(B.CGX_ERR_CAPACITY, "capacity still exceeded after growing")

    def set_tile(self, tile):
        tile = tuple(int(t) for t in tile)
        if tile != self.tile:
            ctx = B.cgx_create(self.device, tile[0], tile[1])
            B.cgx_set_sort_digit_bits(ctx, self.digit_bits)
            B.cgx_destroy(self.ctx)
            self.ctx, self.tile = ctx, tile

    def set_sort_digit_bits(self, bits):
        B.cgx_set_sort_digit_bits(self.ctx, int(bits))
        self.digit_bits = int(bits)

    def autotune(self, views, scene, target, weights=(1.0, 1.0, 1.0), reps=3, cache=None):
        """Switch to the fastest tile shape for this workload, timed by
        cgx_tune_tile_shape on the fused chain, then to the fastest sort
        digit width at that shape (cgx_tune_sort_digits; its timings are kept
        in self.digit_ms).  `cache` is an optional JSON file keyed by the
        workload signature, holding [tw, th, digit bits].  Returns
        (shape, {shape: ms}), with an empty dict when the choice came from
        the cache."""
        key = workload_key(views, scene)
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                entry = table[key]
                if len(entry) > 2:
                    self.set_sort_digit_bits(entry[2])
                self.set_tile(entry[:2])
                return self.tile, {}
        out, grads = self.fwd_bwd_l1(views, scene, target, weights)   # capacities for this shape
        loss = torch.zeros(1, device=f"cuda:{self.device}")
        for _ in range(4):
            need = 0
            for shape in B.TILE_SHAPES:
                c = B.cgx_create(self.device, shape[0], shape[1])
                try:
                    need = max(need, B.cgx_workspace_size(c, views, scene, self.cap))
                finally:
                    B.cgx_destroy(c)
            need = (need + 255) // 256 * 256
            if self.ws is None or self.ws.numel() < need:
                self.ws = None
                self.ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
            best, ms = B.cgx_tune_tile_shape(self.ctx, views, scene, self.cap, self.ws, target,
                                             weights, out, grads, loss, reps)
            if all(v != -2.0 for v in ms.values()):
                break
            # a smaller tile shape exceeded the pair capacity: double it and time again
            cap = dict(self.cap)
            cap["max_pairs"] = 2 * max(int(cap.get("max_pairs", 0)), int(self.last_info["n_pairs"]), 1024)
            self.cap = cap
        self.set_tile(best)
        bits, self.digit_ms = B.cgx_tune_sort_digits(self.ctx, views, scene, self.cap, self.ws,
                                                     target, weights, out, grads, loss, reps)
        self.set_sort_digit_bits(bits)
        if cache:
            table[key] = list(best) + [bits]
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return self.tile, ms

    def ncc_loss(self, views, out, centres, weight=1.0, grad_rgb=None, loss=None):
        """Batch geometric loss (Eq. 10) of the last forward's images `out`;
        centres is an int32 device tensor (n_views // 2, n_patch, 2) of patch
        centres in each pair's second view.  Returns (grad_rgb, loss): the
        gradient is added to grad_rgb (zeros when not given)."""
        dev = f"cuda:{self.device}"
        if grad_rgb is None:
            grad_rgb = torch.zeros_like(out["rgb"])
        if loss is None:
            loss = torch.zeros(1, device=dev)
        c = centres.to(device=dev, dtype=torch.int32).contiguous()
        n_patch = int(c.shape[1]) if c.dim() == 3 else int(c.numel() // 2 // max(len(views) // 2, 1))
        B.cgx_ncc_loss(self.ctx, views, self.ws, out, c, n_patch, weight, grad_rgb, loss)
        return grad_rgb, loss

    def depth_prior(self, views, prior, points, nearby, tau=1.0, aligned=None, filtered=None,
                    keep_aligned=True):
        """Depth prior of Sec. 3.4 (Step 2): per-view scale / shift of the
        packed float32 pseudo-depth `prior` against the sparse float32 (N, 3)
        `points`, then the multi-view filter with nearby[v] (or -1) at
        tau_d = `tau` pixels.  Returns (filtered, aligned, scale_shift (B, 2)
        float64); with keep_aligned=False the aligned image is not written
        (None is returned for it) and the filter aligns on the fly."""
        dev = f"cuda:{self.device}"
        nbytes = B.cgx_depth_align_workspace_size(len(views))
        if self.depth_ws is None or self.depth_ws.numel() * 8 < nbytes:
            self.depth_ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dev)
        st = torch.empty(len(views), 2, dtype=torch.float64, device=dev)
        if filtered is None:
            filtered = torch.empty_like(prior)
        if not keep_aligned:
            B.cgx_depth_prior_align(self.ctx, views, prior, points, self.depth_ws, st, None)
            B.cgx_depth_prior_filter(self.ctx, views, prior, nearby, tau, filtered, scale_shift=st)
            return filtered, None, st
        if aligned is None:
            aligned = torch.empty_like(prior)
        B.cgx_depth_prior_align(self.ctx, views, prior, points, self.depth_ws, st, aligned)
        B.cgx_depth_prior_filter(self.ctx, views, aligned, nearby, tau, filtered)
        return filtered, aligned, st

    def tsdf_volume(self, origin, voxel, dims, trunc, color=True):
        """An empty TSDF volume (Sec. 4 mesh reconstruction): a dict of the
        grid and its device arrays tsdf = 1, weight = 0, color = 0 (3, N)."""
        dev = f"cuda:{self.device}"
        n = int(dims[0]) * int(dims[1]) * int(dims[2])
        vol = dict(origin=tuple(float(x) for x in origin), voxel=float(voxel), trunc=float(trunc),
                   dims=tuple(int(x) for x in dims),
                   tsdf=torch.empty(n, dtype=torch.float32, device=dev),
                   weight=torch.empty(n, dtype=torch.float32, device=dev),
                   color=torch.empty(3, n, dtype=torch.float32, device=dev) if color else None)
        B.cgx_tsdf_init(self.ctx, vol)
        return vol

    def tsdf_integrate(self, views, depth, vol, rgb=None, texels=True):
        """Fuse the views' rendered z-depth (packed float32, e.g. out["depth"]
        of forward) and optional planar rgb into vol, in order; with colour
        and texels=True depth and colour are first interleaved into a
        workspace of 16 bytes per pixel (identical results, fewer gathers)."""
        ws = None
        if texels and rgb is not None and vol.get("color") is not None:
            nbytes = B.cgx_tsdf_workspace_size(views)
            if self.tsdf_ws is None or self.tsdf_ws.numel() * 16 < nbytes:
                self.tsdf_ws = torch.empty((nbytes + 15) // 16, 4, dtype=torch.float32,
                                           device=f"cuda:{self.device}")
            ws = self.tsdf_ws
        B.cgx_tsdf_integrate(self.ctx, views, depth, rgb, vol, ws)
        return vol

    def info(self):
        return B.cgx_read_info(self.ctx, self.ws)

    def count_work(self, on=True):
        """Count the raster work (list entries walked, opacity evaluations)
        in the following launches; slower, for measurement only."""
        B.cgx_count_enable(self.ctx, on)

    def debug(self):
        return B.cgx_debug_copy(self.ctx, self.ws)

    def debug_splats(self):
        """(splat records, gradient records) of the last chain, per slot."""
        return B.cgx_debug_splats(self.ctx, self.ws)


_EXPLICIT_KEYS = ("means", "scales", "quats", "opacity", "sh")


class RenderExplicit(torch.autograd.Function):
    """Differentiable render of explicit Gaussians: returns the packed
    (rgb, depth, plane_d, normal, alpha) images; the backward pass runs the
    library's reverse-order rasterizer and projection adjoint on the
    forward state of this very call (kept per call, so several forward calls
    may precede their backward calls)."""

    @staticmethod
    def forward(ctx, renderer, views, sh_degree, means, scales, quats, opacity, sh):
        scene = dict(kind=B.CGX_SCENE_EXPLICIT, means=means.detach().contiguous(),
                     scales=scales.detach().contiguous(), quats=quats.detach().contiguous(),
                     opacity=opacity.detach().contiguous(), sh=sh.detach().contiguous(),
                     sh_degree=sh_degree)
        out = renderer.forward(views, scene)
        ctx.renderer, ctx.views, ctx.scene, ctx.out = renderer, views, scene, out
        ctx.state = renderer.take_state()
        return out["rgb"], out["depth"], out["plane_d"], out["normal"], out["alpha"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_plane, g_normal, g_alpha):
        c = lambda t: None if t is None else t.contiguous()   # noqa: E731
        gout = dict(rgb=c(g_rgb), depth=c(g_depth), plane_d=c(g_plane), normal=c(g_normal),
                    alpha=c(g_alpha))
        grads = ctx.renderer.backward(ctx.views, ctx.scene, ctx.out, gout, state=ctx.state)
        ctx.state = None
        return (None, None, None) + tuple(grads[k] for k in _EXPLICIT_KEYS)


_ANCHOR_KEYS = ("x", "l", "O", "F", "b1", "b2")


class RenderAnchor(torch.autograd.Function):
    """Differentiable render of voxel anchors.  meta holds the non-trainable
    parts: level (uint8), the decoder weights W1, W2 as bfloat16 bit tensors,
    n_levels, d_max, opacity_act, offset_mode and decoder_heads; the
    gradients of W1 and W2 are returned
    through the float tensors passed as W1f / W2f (their values are not
    read: the weights are the bfloat16 bits).  The forward state is kept per
    call, as for RenderExplicit."""

    @staticmethod
    def forward(ctx, renderer, views, meta, x, l, O, F, b1, b2, W1f, W2f):
        d = lambda t: t.detach().contiguous()   # noqa: E731
        scene = dict(kind=B.CGX_SCENE_ANCHOR, x=d(x), l=d(l), O=d(O), F=d(F), level=meta["level"],
                     W1=meta["W1"], W2=meta["W2"], b1=d(b1), b2=d(b2), n_levels=meta["n_levels"],
                     d_max=meta["d_max"], opacity_act=int(meta.get("opacity_act", B.OPACITY_SIGMOID)),
                     offset_mode=int(meta.get("offset_mode", B.OFFSETS_TABLE)),
                     decoder_heads=int(meta.get("decoder_heads", B.DECODER_SHARED)))
        out = renderer.forward(views, scene)
        ctx.renderer, ctx.views, ctx.scene, ctx.out = renderer, views, scene, out
        ctx.state = renderer.take_state()
        return out["rgb"], out["depth"], out["plane_d"], out["normal"], out["alpha"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_plane, g_normal, g_alpha):
        c = lambda t: None if t is None else t.contiguous()   # noqa: E731
        gout = dict(rgb=c(g_rgb), depth=c(g_depth), plane_d=c(g_plane), normal=c(g_normal),
                    alpha=c(g_alpha))
        grads = ctx.renderer.backward(ctx.views, ctx.scene, ctx.out, gout, state=ctx.state)
        ctx.state = None
        return (None, None, None) + tuple(grads[k] for k in _ANCHOR_KEYS) + (grads["W1"], grads["W2"])
