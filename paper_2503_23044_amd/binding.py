"""ctypes binding of libcgx (include/cgx.h) with the same names, plus a
small object wrapper and a torch.autograd.Function.

Argument marshalling only: every step of the rasterizer runs in the HIP
kernels of libcgx.so.  PyTorch provides device memory and the stream.
Importing this module never falls back to anything else: if the library
is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgx.so")

CGX_ABI_VERSION = 8
OPACITY_SIGMOID, OPACITY_TANH_MASK = 0, 1
OFFSETS_TABLE, OFFSETS_DECODED = 0, 1
DECODER_SHARED, DECODER_PER_ATTRIBUTE = 1, 3
CGX_OK = 0
CGX_ERR_INVALID_ARG = 1
CGX_ERR_UNSUPPORTED = 2
CGX_ERR_CAPACITY = 3
CGX_ERR_HIP = 4
CGX_ERR_WORKSPACE = 5
CGX_SCENE_EXPLICIT = 0
CGX_SCENE_ANCHOR = 1
STATUS_NAMES = {0: "CGX_OK", 1: "CGX_ERR_INVALID_ARG", 2: "CGX_ERR_UNSUPPORTED",
                3: "CGX_ERR_CAPACITY", 4: "CGX_ERR_HIP", 5: "CGX_ERR_WORKSPACE"}


class cgx_view(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("z_near", C.c_float), ("bg", C.c_float * 3)]


class cgx_explicit_scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("means", C.c_void_p),
                ("scales", C.c_void_p), ("quats", C.c_void_p), ("opacity", C.c_void_p),
                ("sh", C.c_void_p)]


class cgx_anchor_scene(C.Structure):
    _fields_ = [("n_anchor", C.c_int64), ("n_offsets", C.c_int32), ("n_levels", C.c_int32),
                ("d_max", C.c_float), ("opacity_act", C.c_int32), ("offset_mode", C.c_int32),
                ("decoder_heads", C.c_int32), ("x", C.c_void_p),
                ("l", C.c_void_p), ("O", C.c_void_p),
                ("F", C.c_void_p), ("level", C.c_void_p), ("W1", C.c_void_p), ("b1", C.c_void_p),
                ("W2", C.c_void_p), ("b2", C.c_void_p)]


class cgx_ncc_term(C.Structure):
    _fields_ = [("centres", C.c_void_p), ("n_patch", C.c_int32), ("weight", C.c_float)]


class cgx_scene(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ex", cgx_explicit_scene), ("an", cgx_anchor_scene)]


class cgx_images(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("plane_d", C.c_void_p),
                ("normal", C.c_void_p), ("alpha", C.c_void_p)]


class cgx_grads(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("means", "scales", "quats", "opacity", "sh", "x", "l", "O",
                                          "F", "W1", "b1", "W2", "b2")]


class cgx_tsdf_volume(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("voxel", C.c_float), ("trunc", C.c_float),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("tsdf", C.c_void_p), ("weight", C.c_void_p), ("color", C.c_void_p)]


class cgx_capacity(C.Structure):
    _fields_ = [("max_rows", C.c_int64), ("max_splats", C.c_int64), ("max_pairs", C.c_int64)]


class cgx_run_info(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("n_splats", C.c_int64), ("n_pairs", C.c_int64),
                ("overflow", C.c_int32), ("reserved", C.c_int32), ("need_rows", C.c_int64),
                ("need_splats", C.c_int64), ("need_pairs", C.c_int64), ("loss", C.c_double),
                ("entries_fwd", C.c_uint64), ("entries_bwd", C.c_uint64), ("n_tiles", C.c_int64),
                ("n_pixels", C.c_int64), ("evals_fwd", C.c_uint64), ("evals_bwd", C.c_uint64),
                ("sort_passes", C.c_int32), ("n_visible", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcgx.so and declare every entry point.  Raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libcgx.so not built at {path}; run __graft_entry__.build()")
    lib = C.CDLL(path)
    lib.cgx_abi_version.restype = C.c_int32
    if lib.cgx_abi_version() != CGX_ABI_VERSION:
        raise RuntimeError(f"{path} has ABI version {lib.cgx_abi_version()}, the binding expects "
                           f"{CGX_ABI_VERSION}; rebuild with __graft_entry__.build()")
    P = C.c_void_p
    sig = {
        "cgx_abi_version": (C.c_int32, []),
        "cgx_create": (C.c_int32, [C.POINTER(P), C.c_int32, C.c_int32, C.c_int32]),
        "cgx_destroy": (C.c_int32, [P]),
        "cgx_last_error": (C.c_char_p, [P]),
        "cgx_workspace_size": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32, C.POINTER(cgx_scene),
                                           C.POINTER(cgx_capacity), C.POINTER(C.c_size_t)]),
        "cgx_render_forward": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32, C.POINTER(cgx_scene),
                                           C.POINTER(cgx_capacity), P, C.c_size_t,
                                           C.POINTER(cgx_images), P]),
        "cgx_render_backward": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32, C.POINTER(cgx_scene),
                                            C.POINTER(cgx_capacity), P, C.c_size_t,
                                            C.POINTER(cgx_images), C.POINTER(cgx_images),
                                            C.POINTER(cgx_grads), P]),
        "cgx_render_fwd_bwd_l1": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32,
                                              C.POINTER(cgx_scene), C.POINTER(cgx_capacity), P,
                                              C.c_size_t, C.POINTER(cgx_images),
                                              C.POINTER(C.c_float), C.POINTER(cgx_ncc_term),
                                              C.POINTER(cgx_images), C.POINTER(cgx_grads), P, P]),
        "cgx_read_info": (C.c_int32, [P, P, P, C.POINTER(cgx_run_info)]),
        "cgx_debug_copy": (C.c_int32, [P, P, P, P, P, P, P, P, P]),
        "cgx_graph_capture_fwd_bwd_l1": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32,
                                                     C.POINTER(cgx_scene), C.POINTER(cgx_capacity),
                                                     P, C.c_size_t, C.POINTER(cgx_images),
                                                     C.POINTER(C.c_float), C.POINTER(cgx_ncc_term),
                                                     C.POINTER(cgx_images), C.POINTER(cgx_grads),
                                                     P, P, C.POINTER(P)]),
        "cgx_graph_launch": (C.c_int32, [P, P]),
        "cgx_graph_destroy": (C.c_int32, [P]),
        "cgx_ncc_loss": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32, P, C.POINTER(cgx_images), P,
                                     C.c_int32, C.c_float, P, P, P]),
        "cgx_depth_align_workspace_size": (C.c_size_t, [C.c_int32]),
        "cgx_depth_prior_align": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32, P, P, C.c_int32, P,
                                              C.c_size_t, P, P, P]),
        "cgx_depth_prior_align_noalloc": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32, P, P,
                                                      C.c_int32, P, P, P]),
        "cgx_depth_prior_filter": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32, P, P,
                                               C.POINTER(C.c_int32), C.c_float, P, P]),
        "cgx_tsdf_init": (C.c_int32, [P, C.POINTER(cgx_tsdf_volume), P]),
        "cgx_tsdf_integrate": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32, P, P,
                                           C.POINTER(cgx_tsdf_volume), P, C.c_size_t, P]),
        "cgx_tsdf_workspace_size": (C.c_size_t, [C.POINTER(cgx_view), C.c_int32]),
        "cgx_tune_tile_shape": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32,
                                            C.POINTER(cgx_scene), C.POINTER(cgx_capacity), P,
                                            C.c_size_t, C.POINTER(cgx_images),
                                            C.POINTER(C.c_float), C.POINTER(cgx_images),
                                            C.POINTER(cgx_grads), P, C.c_int32, P,
                                            C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                            C.POINTER(C.c_float)]),
        "cgx_tune_sort_digits": (C.c_int32, [P, C.POINTER(cgx_view), C.c_int32,
                                             C.POINTER(cgx_scene), C.POINTER(cgx_capacity), P,
                                             C.c_size_t, C.POINTER(cgx_images),
                                             C.POINTER(C.c_float), C.POINTER(cgx_images),
                                             C.POINTER(cgx_grads), P, C.c_int32, P,
                                             C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
        "cgx_set_sort_digit_bits": (C.c_int32, [P, C.c_int32]),
        "cgx_get_sort_digit_bits": (C.c_int32, [P, C.POINTER(C.c_int32)]),
        "cgx_timing_enable": (C.c_int32, [P, C.c_int32]),
        "cgx_count_enable": (C.c_int32, [P, C.c_int32]),
        "cgx_debug_splats": (C.c_int32, [P, P, P, P, P]),
        "cgx_timing_read": (C.c_int32, [P, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class CgxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


# --------------------------------------------------------------------------
# thin wrappers, same names as the C ABI
# --------------------------------------------------------------------------
def cgx_abi_version():
    return load_library().cgx_abi_version()


def cgx_create(device=0, tile_w=16, tile_h=16):
    lib = load_library()
    h = C.c_void_p()
    rc = lib.cgx_create(C.byref(h), device, tile_w, tile_h)
    if rc != CGX_OK:
        raise CgxError(rc, "cgx_create")
    return h


def cgx_destroy(ctx):
    return load_library().cgx_destroy(ctx)


def cgx_last_error(ctx):
    m = load_library().cgx_last_error(ctx)
    return m.decode() if m else ""


def _check(ctx, rc, what):
    if rc != CGX_OK:
        raise CgxError(rc, f"{what}: {cgx_last_error(ctx)}")


def make_views(views) -> "C.Array":
    """Pack view objects (attributes width, height, fx, fy, cx, cy, R, t,
    z_near, bg) or dicts into a host cgx_view array."""
    arr = (cgx_view * len(views))()
    for i, v in enumerate(views):
        g = (lambda k: v[k]) if isinstance(v, dict) else (lambda k: getattr(v, k))
        arr[i].width = int(g("width"))
        arr[i].height = int(g("height"))
        arr[i].fx, arr[i].fy = float(g("fx")), float(g("fy"))
        arr[i].cx, arr[i].cy = float(g("cx")), float(g("cy"))
        R = np.asarray(g("R"), np.float32).reshape(9)
        t = np.asarray(g("t"), np.float32).reshape(3)
        for k in range(9):
            arr[i].R[k] = float(R[k])
        for k in range(3):
            arr[i].t[k] = float(t[k])
        arr[i].z_near = float(g("z_near"))
        bg = np.asarray(g("bg"), np.float32).reshape(3)
        for k in range(3):
            arr[i].bg[k] = float(bg[k])
    return arr


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def make_scene(scene: dict) -> cgx_scene:
    """scene: dict of device tensors.  Explicit: kind=0, means, scales, quats,
    opacity, sh, sh_degree.  Anchor: kind=1, x, l, O, F, level (uint8), W1,
    W2 (int16 tensors holding bfloat16 bits), b1, b2, n_levels, d_max and
    optionally opacity_act, offset_mode, decoder_heads."""
    s = cgx_scene()
    s.kind = int(scene["kind"])
    if s.kind == CGX_SCENE_EXPLICIT:
        s.ex.n = int(scene["means"].shape[0])
        s.ex.sh_degree = int(scene["sh_degree"])
        for k in ("means", "scales", "quats", "opacity", "sh"):
            setattr(s.ex, k, _ptr(scene[k]))
    else:
        s.an.n_anchor = int(scene["x"].shape[0])
        s.an.n_offsets = int(scene["O"].shape[1])
        s.an.n_levels = int(scene["n_levels"])
        s.an.d_max = float(scene["d_max"])
        s.an.opacity_act = int(scene.get("opacity_act", OPACITY_SIGMOID))
        s.an.offset_mode = int(scene.get("offset_mode", OFFSETS_TABLE))
        s.an.decoder_heads = int(scene.get("decoder_heads", DECODER_SHARED))
        for k in ("x", "l", "O", "F", "level", "W1", "b1", "W2", "b2"):
            setattr(s.an, k, _ptr(scene[k]))
    return s


def make_images(d) -> cgx_images:
    im = cgx_images()
    if d is not None:
        for k in ("rgb", "depth", "plane_d", "normal", "alpha"):
            setattr(im, k, _ptr(d.get(k)))
    return im


def make_grads(d) -> cgx_grads:
    g = cgx_grads()
    for k in ("means", "scales", "quats", "opacity", "sh", "x", "l", "O", "F", "W1", "b1", "W2", "b2"):
        setattr(g, k, _ptr(d.get(k)))
    return g


def make_capacity(cap) -> cgx_capacity:
    c = cgx_capacity()
    if cap:
        c.max_rows = int(cap.get("max_rows", 0))
        c.max_splats = int(cap.get("max_splats", 0))
        c.max_pairs = int(cap.get("max_pairs", 0))
    return c


def cgx_workspace_size(ctx, views, scene, cap=None):
    lib = load_library()
    va = make_views(views)
    sc = make_scene(scene) if isinstance(scene, dict) else scene
    n = C.c_size_t()
    rc = lib.cgx_workspace_size(ctx, va, len(views), C.byref(sc), C.byref(make_capacity(cap)),
                                C.byref(n))
    _check(ctx, rc, "cgx_workspace_size")
    return n.value


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def cgx_render_forward(ctx, views, scene, cap, ws, out):
    lib = load_library()
    va = make_views(views)
    sc = make_scene(scene)
    im = make_images(out)
    rc = lib.cgx_render_forward(ctx, va, len(views), C.byref(sc), C.byref(make_capacity(cap)),
                                C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(im), _stream())
    _check(ctx, rc, "cgx_render_forward")


def cgx_render_backward(ctx, views, scene, cap, ws, out, grad_out, grads):
    lib = load_library()
    va = make_views(views)
    sc = make_scene(scene)
    rc = lib.cgx_render_backward(ctx, va, len(views), C.byref(sc), C.byref(make_capacity(cap)),
                                 C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(make_images(out)),
                                 C.byref(make_images(grad_out)), C.byref(make_grads(grads)),
                                 _stream())
    _check(ctx, rc, "cgx_render_backward")


def make_ncc(ncc):
    """ncc: None, or dict(centres=int32 device tensor of (x, y) pairs,
    pair-major, n_patch=patches per view pair, weight=float)."""
    if ncc is None:
        return None
    t = cgx_ncc_term()
    t.centres = _ptr(ncc["centres"])
    t.n_patch = int(ncc["n_patch"])
    t.weight = float(ncc["weight"])
    return t


def _byref_or_null(x):
    return C.byref(x) if x is not None else None


def cgx_render_fwd_bwd_l1(ctx, views, scene, cap, ws, target, weights, out, grads, loss_dev=None,
                          ncc=None):
    lib = load_library()
    va = make_views(views)
    sc = make_scene(scene)
    w = (C.c_float * 3)(*[float(x) for x in weights])
    nt = make_ncc(ncc)
    rc = lib.cgx_render_fwd_bwd_l1(ctx, va, len(views), C.byref(sc), C.byref(make_capacity(cap)),
                                   C.c_void_p(ws.data_ptr()), ws.numel(),
                                   C.byref(make_images(target)), w, _byref_or_null(nt),
                                   C.byref(make_images(out)), C.byref(make_grads(grads)),
                                   _ptr(loss_dev), _stream())
    _check(ctx, rc, "cgx_render_fwd_bwd_l1")


def cgx_ncc_loss(ctx, views, ws, images, centres, n_patch, weight, grad_rgb, loss_dev=None):
    """Eq. 10 loss on the forward images held in `images` (rgb, normal,
    plane_d); ADDS dloss/drgb into grad_rgb and the loss into loss_dev."""
    lib = load_library()
    va = make_views(views)
    rc = lib.cgx_ncc_loss(ctx, va, len(views), C.c_void_p(ws.data_ptr()), C.byref(make_images(images)),
                          _ptr(centres), int(n_patch), float(weight), _ptr(grad_rgb), _ptr(loss_dev),
                          _stream())
    _check(ctx, rc, "cgx_ncc_loss")


def cgx_depth_align_workspace_size(n_views):
    return int(load_library().cgx_depth_align_workspace_size(int(n_views)))


def cgx_depth_prior_align(ctx, views, prior, points, ws, scale_shift, aligned):
    """Per-view least-squares (s, t) of the packed float32 prior against the
    float32 (N, 3) points; writes scale_shift (float64, 2 per view) and
    aligned (float32, packed; may be prior itself)."""
    lib = load_library()
    va = make_views(views)
    n = int(points.numel() // 3) if points is not None else 0
    rc = lib.cgx_depth_prior_align(ctx, va, len(views), _ptr(prior), _ptr(points) if n else None, n,
                                   C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                   _ptr(scale_shift), _ptr(aligned), _stream())
    _check(ctx, rc, "cgx_depth_prior_align")


def cgx_depth_prior_align_noalloc(ctx, views, prior, points, scale_shift, aligned):
    """cgx_depth_prior_align with the library's fixed partial-sum array (no
    workspace; for callers that cannot allocate)."""
    lib = load_library()
    va = make_views(views)
    n = int(points.numel() // 3) if points is not None else 0
    rc = lib.cgx_depth_prior_align_noalloc(ctx, va, len(views), _ptr(prior),
                                           _ptr(points) if n else None, n, _ptr(scale_shift),
                                           _ptr(aligned), _stream())
    _check(ctx, rc, "cgx_depth_prior_align_noalloc")


def cgx_depth_prior_filter(ctx, views, depth, nearby, tau, filtered, scale_shift=None):
    """Multi-view consistency filter of the packed float32 depth maps;
    nearby is a host sequence (one view index or -1 per view).  With
    scale_shift (float64 (B, 2) device), depth is the raw prior, aligned on
    the fly."""
    lib = load_library()
    va = make_views(views)
    nb = (C.c_int32 * len(views))(*[int(x) for x in nearby])
    rc = lib.cgx_depth_prior_filter(ctx, va, len(views), _ptr(depth), _ptr(scale_shift), nb, float(tau),
                                    _ptr(filtered), _stream())
    _check(ctx, rc, "cgx_depth_prior_filter")


def make_volume(vol: dict) -> cgx_tsdf_volume:
    """vol: origin (3 floats), voxel, trunc, dims (nx, ny, nz), device
    float32 tensors tsdf (N), weight (N) and color (3, N) or None."""
    v = cgx_tsdf_volume()
    for k in range(3):
        v.origin[k] = float(vol["origin"][k])
    v.voxel = float(vol["voxel"])
    v.trunc = float(vol["trunc"])
    v.nx, v.ny, v.nz = (int(x) for x in vol["dims"])
    v.tsdf = vol["tsdf"].data_ptr()
    v.weight = vol["weight"].data_ptr()
    v.color = vol["color"].data_ptr() if vol.get("color") is not None else None
    return v


def cgx_tsdf_init(ctx, vol):
    lib = load_library()
    rc = lib.cgx_tsdf_init(ctx, C.byref(make_volume(vol)), _stream())
    _check(ctx, rc, "cgx_tsdf_init")


def cgx_tsdf_workspace_size(views):
    return int(load_library().cgx_tsdf_workspace_size(make_views(views), len(views)))


def cgx_tsdf_integrate(ctx, views, depth, rgb, vol, ws=None):
    """Fuse the views' packed z-depth (and planar rgb, or None) into vol;
    ws (device, cgx_tsdf_workspace_size bytes) enables the texel path."""
    lib = load_library()
    va = make_views(views)
    nbytes = ws.numel() * ws.element_size() if ws is not None else 0
    rc = lib.cgx_tsdf_integrate(ctx, va, len(views), _ptr(depth), _ptr(rgb), C.byref(make_volume(vol)),
                                _ptr(ws), nbytes, _stream())
    _check(ctx, rc, "cgx_tsdf_integrate")


TILE_SHAPES = [(16, 16), (8, 8), (16, 8), (32, 8), (32, 16)]


def cgx_tune_tile_shape(ctx, views, scene, cap, ws, target, weights, out, grads, loss_dev=None,
                        reps=3):
    """Time the fused chain per tile shape; returns ((tw, th), {shape: ms})
    with -1 for shapes whose workspace does not fit, -2 for capacity overflow."""
    lib = load_library()
    va = make_views(views)
    sc = make_scene(scene)
    w = (C.c_float * 3)(*[float(x) for x in weights])
    tw, th = C.c_int32(0), C.c_int32(0)
    ms = (C.c_float * len(TILE_SHAPES))()
    rc = lib.cgx_tune_tile_shape(ctx, va, len(views), C.byref(sc), C.byref(make_capacity(cap)),
                                 C.c_void_p(ws.data_ptr()), ws.numel(),
                                 C.byref(make_images(target)), w, C.byref(make_images(out)),
                                 C.byref(make_grads(grads)), _ptr(loss_dev), int(reps), _stream(),
                                 C.byref(tw), C.byref(th), ms)
    _check(ctx, rc, "cgx_tune_tile_shape")
    return (tw.value, th.value), {s: ms[i] for i, s in enumerate(TILE_SHAPES)}


DIGIT_CHOICES = [9, 8, 7]


def cgx_tune_sort_digits(ctx, views, scene, cap, ws, target, weights, out, grads, loss_dev=None,
                         reps=3):
    """Time the fused chain per sort digit width at the context's tile
    shape; returns (bits, {bits: ms})."""
    lib = load_library()
    va = make_views(views)
    sc = make_scene(scene)
    w = (C.c_float * 3)(*[float(x) for x in weights])
    bits = C.c_int32(0)
    ms = (C.c_float * len(DIGIT_CHOICES))()
    rc = lib.cgx_tune_sort_digits(ctx, va, len(views), C.byref(sc), C.byref(make_capacity(cap)),
                                  C.c_void_p(ws.data_ptr()), ws.numel(),
                                  C.byref(make_images(target)), w, C.byref(make_images(out)),
                                  C.byref(make_grads(grads)), _ptr(loss_dev), int(reps), _stream(),
                                  C.byref(bits), ms)
    _check(ctx, rc, "cgx_tune_sort_digits")
    return bits.value, {b: ms[i] for i, b in enumerate(DIGIT_CHOICES)}


def cgx_set_sort_digit_bits(ctx, bits):
    _check(ctx, load_library().cgx_set_sort_digit_bits(ctx, int(bits)), "cgx_set_sort_digit_bits")


def cgx_get_sort_digit_bits(ctx):
    b = C.c_int32(0)
    _check(ctx, load_library().cgx_get_sort_digit_bits(ctx, C.byref(b)), "cgx_get_sort_digit_bits")
    return b.value


def cgx_read_info(ctx, ws, raise_on_capacity=True):
    lib = load_library()
    info = cgx_run_info()
    rc = lib.cgx_read_info(ctx, C.c_void_p(ws.data_ptr()), _stream(), C.byref(info))
    if rc not in (CGX_OK, CGX_ERR_CAPACITY) or (rc == CGX_ERR_CAPACITY and raise_on_capacity):
        _check(ctx, rc, "cgx_read_info")
    return {f: getattr(info, f) for f, _ in cgx_run_info._fields_}


def cgx_debug_copy(ctx, ws):
    lib = load_library()
    info = cgx_read_info(ctx, ws)
    P, T = info["n_pairs"], info["n_tiles"]
    R, S = info["n_rows"], info["n_splats"]
    tiles = np.zeros(P, np.uint32)
    zb = np.zeros(P, np.uint32)
    slots = np.zeros(P, np.uint32)
    ranges = np.zeros((T, 2), np.uint32)
    rows = np.zeros((R, 2), np.int32)
    counts = np.zeros(S, np.uint32)
    p = lambda a: a.ctypes.data_as(C.c_void_p)   # noqa: E731
    rc = lib.cgx_debug_copy(ctx, C.c_void_p(ws.data_ptr()), _stream(), p(tiles), p(zb), p(slots),
                            p(ranges), p(rows), p(counts))
    _check(ctx, rc, "cgx_debug_copy")
    return dict(tile=tiles, zbits=zb, slot=slots, ranges=ranges, rows=rows, counts=counts, info=info)


SPLAT_RECORD = np.dtype([("u", "<f4"), ("w", "<f4"), ("pa", "<f4"), ("pb", "<f4"), ("pc", "<f4"),
                         ("lno", "<f4"), ("rgb", "<f4", 3), ("d", "<f4"), ("normal", "<f4", 3),
                         ("bx", "<u4"), ("by", "<u4"), ("inv_o", "<f4")])


def cgx_debug_splats(ctx, ws):
    """Per-slot splat records (structured array) and 16-float gradient
    records of the last chain."""
    lib = load_library()
    info = cgx_read_info(ctx, ws)
    S = info["n_splats"]
    rec = np.zeros(S, SPLAT_RECORD)
    grads = np.zeros((S, 16), np.float32)
    p = lambda a: a.ctypes.data_as(C.c_void_p)   # noqa: E731
    _check(ctx, lib.cgx_debug_splats(ctx, C.c_void_p(ws.data_ptr()), _stream(), p(rec), p(grads)),
           "cgx_debug_splats")
    return rec, grads


PHASES = ["select", "project", "scan", "duplicate", "sort", "ranges", "raster_fwd", "raster_bwd",
          "project_bwd", "wgrad"]


def cgx_timing_enable(ctx, n_records):
    _check(ctx, load_library().cgx_timing_enable(ctx, int(n_records)), "cgx_timing_enable")


def cgx_count_enable(ctx, on):
    """Switch the raster work counters (entries_fwd, evals_fwd, evals_bwd)."""
    _check(ctx, load_library().cgx_count_enable(ctx, 1 if on else 0), "cgx_count_enable")


def cgx_timing_read(ctx):
    n = len(PHASES)
    ms = (C.c_double * n)()
    cnt = (C.c_int32 * n)()
    _check(ctx, load_library().cgx_timing_read(ctx, ms, cnt, n), "cgx_timing_read")
    return {PHASES[i]: (ms[i], cnt[i]) for i in range(n)}


def cgx_graph_capture_fwd_bwd_l1(ctx, views, scene, cap, ws, target, weights, out, grads,
                                 loss_dev, stream, ncc=None):
    """Capture the fused chain on `stream` (a torch.cuda.Stream, not the
    default stream) into a graph handle."""
    lib = load_library()
    va = make_views(views)
    sc = make_scene(scene)
    w = (C.c_float * 3)(*[float(x) for x in weights])
    nt = make_ncc(ncc)
    g = C.c_void_p()
    rc = lib.cgx_graph_capture_fwd_bwd_l1(ctx, va, len(views), C.byref(sc),
                                          C.byref(make_capacity(cap)), C.c_void_p(ws.data_ptr()),
                                          ws.numel(), C.byref(make_images(target)), w,
                                          _byref_or_null(nt), C.byref(make_images(out)),
                                          C.byref(make_grads(grads)), _ptr(loss_dev),
                                          C.c_void_p(stream.cuda_stream), C.byref(g))
    _check(ctx, rc, "cgx_graph_capture_fwd_bwd_l1")
    return g


def cgx_graph_launch(graph, stream):
    rc = load_library().cgx_graph_launch(graph, C.c_void_p(stream.cuda_stream))
    if rc != CGX_OK:
        raise CgxError(rc, "cgx_graph_launch")


def cgx_graph_destroy(graph):
    return load_library().cgx_graph_destroy(graph)
