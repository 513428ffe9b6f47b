"""The C ABI without a GPU: every function that include/cgx.h declares is
exported by libcgx.so, and the host-side parts of the library (argument
validation and workspace sizing) behave as the header states.  Nothing here
launches a kernel."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgx.h")


def _header():
    with open(HEADER) as f:
        return f.read()


def _declared():
    text = re.sub(r"/\*.*?\*/", "", _header(), flags=re.S)
    return sorted(set(re.findall(r"\b(cgx_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def B():
    from paper_2503_23044_amd import binding, build_lib
    if not os.path.exists(binding.LIB_PATH):
        build_lib.build()
    binding.load_library()
    return binding


def test_every_declared_symbol_is_exported(B):
    names = _declared()
    assert len(names) >= 15, names
    lib = C.CDLL(B.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version_matches_header(B):
    m = re.search(r"#define\s+CGX_ABI_VERSION\s+(\d+)", _header())
    assert B.cgx_abi_version() == int(m.group(1)) == B.CGX_ABI_VERSION


def _view(w=64, h=48):
    return dict(width=w, height=h, fx=50.0, fy=50.0, cx=w / 2, cy=h / 2, R=np.eye(3), t=np.zeros(3),
                z_near=0.2, bg=np.zeros(3))


def _explicit(n=100, deg=0):
    f = lambda *s: torch.zeros(*s, dtype=torch.float32)  # noqa: E731  (host tensors: never read)
    K = (deg + 1) ** 2
    return dict(kind=0, means=f(n, 3), scales=f(n, 3), quats=f(n, 4), opacity=f(n), sh=f(n, K, 3),
                sh_degree=deg)


def _anchor(a=50):
    f = lambda *s: torch.zeros(*s, dtype=torch.float32)  # noqa: E731
    return dict(kind=1, x=f(a, 3), l=f(a, 3), O=f(a, 10, 3), F=f(a, 32),
                level=torch.zeros(a, dtype=torch.uint8), W1=torch.zeros(36, 32, dtype=torch.int16),
                b1=f(32), W2=torch.zeros(32, 110, dtype=torch.int16), b2=f(110), n_levels=4, d_max=100.0)


def _status(B, fn, *args):
    try:
        fn(*args)
    except B.CgxError as e:
        return str(e).split(":")[0]
    return "CGX_OK"


def test_create_rejects_unsupported_tiles(B):
    for tw, th in ((16, 16), (8, 8), (16, 8), (32, 8), (32, 16)):
        B.cgx_destroy(B.cgx_create(0, tw, th))
    for tw, th in ((4, 4), (16, 32), (0, 16)):
        assert _status(B, B.cgx_create, 0, tw, th) == "CGX_ERR_UNSUPPORTED"


def test_workspace_size_validation(B):
    ctx = B.cgx_create(0, 16, 16)
    try:
        ok = B.cgx_workspace_size(ctx, [_view()], _explicit())
        assert ok > 0
        bad_v = _view()
        bad_v["fx"] = 0.0
        assert _status(B, B.cgx_workspace_size, ctx, [bad_v], _explicit()) == "CGX_ERR_INVALID_ARG"
        bad_v = _view()
        bad_v["z_near"] = 0.0
        assert _status(B, B.cgx_workspace_size, ctx, [bad_v], _explicit()) == "CGX_ERR_INVALID_ARG"
        assert _status(B, B.cgx_workspace_size, ctx, [_view(0, 10)], _explicit()) == "CGX_ERR_INVALID_ARG"
        assert _status(B, B.cgx_workspace_size, ctx, [_view()], _explicit(deg=4)) == "CGX_ERR_UNSUPPORTED"
        sc = _anchor()
        sc["O"] = torch.zeros(50, 8, 3)
        assert _status(B, B.cgx_workspace_size, ctx, [_view()], sc) == "CGX_ERR_UNSUPPORTED"
        sc = _anchor()
        sc["d_max"] = 0.0
        assert _status(B, B.cgx_workspace_size, ctx, [_view()], sc) == "CGX_ERR_INVALID_ARG"
        assert _status(B, B.cgx_workspace_size, ctx, [_view()] * 33, _explicit()) == "CGX_ERR_INVALID_ARG"
        sc = _anchor()
        sc["opacity_act"] = 2
        assert _status(B, B.cgx_workspace_size, ctx, [_view()], sc) == "CGX_ERR_INVALID_ARG"
        sc["opacity_act"] = B.OPACITY_TANH_MASK
        assert B.cgx_workspace_size(ctx, [_view()], sc) > 0
        base = B.cgx_workspace_size(ctx, [_view()], _anchor())
        assert base > 0
        for key, bad in (("offset_mode", 2), ("offset_mode", -1), ("decoder_heads", 2),
                         ("decoder_heads", 4), ("decoder_heads", 0)):
            sc = _anchor()
            sc[key] = bad
            assert _status(B, B.cgx_workspace_size, ctx, [_view()], sc) == "CGX_ERR_INVALID_ARG", (key, bad)
        # wider decoders keep more per row: the workspace grows with them
        sizes = []
        for mode, heads in ((B.OFFSETS_TABLE, B.DECODER_SHARED), (B.OFFSETS_DECODED, B.DECODER_SHARED),
                            (B.OFFSETS_TABLE, B.DECODER_PER_ATTRIBUTE),
                            (B.OFFSETS_DECODED, B.DECODER_PER_ATTRIBUTE)):
            sc = _anchor()
            sc["offset_mode"], sc["decoder_heads"] = mode, heads
            sizes.append(B.cgx_workspace_size(ctx, [_view()], sc))
        assert sizes[0] == base and sizes[0] < sizes[1] < sizes[3] and sizes[0] < sizes[2] < sizes[3]
    finally:
        B.cgx_destroy(ctx)


def test_workspace_size_bounds(B):
    """The workspace holds at least the 64-byte splat record, the per-pixel
    forward state (8 B) and the double-buffered pair arrays (16 B) that the
    chain needs, and grows with every one of them."""
    ctx = B.cgx_create(0, 16, 16)
    try:
        v = [_view(64, 48), _view(33, 17)]
        px = 64 * 48 + 33 * 17
        n = 1000
        for cap_pairs in (10_000, 20_000):
            ws = B.cgx_workspace_size(ctx, v, _explicit(n), dict(max_pairs=cap_pairs))
            assert ws >= 64 * n * 2 + 8 * px + 16 * cap_pairs
        a = B.cgx_workspace_size(ctx, v, _explicit(n), dict(max_pairs=10_000))
        b = B.cgx_workspace_size(ctx, v, _explicit(n), dict(max_pairs=20_000))
        c = B.cgx_workspace_size(ctx, v, _explicit(2 * n), dict(max_pairs=10_000))
        d = B.cgx_workspace_size(ctx, v + [_view(640, 480)], _explicit(n), dict(max_pairs=10_000))
        slack = 4 * 256   # regions are 256-byte aligned
        assert b - a >= 16 * 10_000 - slack and c > a and d - a >= 8 * 640 * 480 - slack
    finally:
        B.cgx_destroy(ctx)


def test_entry_points_reject_bad_arguments_before_any_launch(B):
    lib = B.load_library()
    ctx = B.cgx_create(0, 16, 16)
    try:
        va = B.make_views([_view()])
        sc = B.make_scene(_explicit())
        cap = B.make_capacity(None)
        img = B.cgx_images()
        rc = lib.cgx_render_forward(ctx, va, 1, C.byref(sc), C.byref(cap), None, 0, C.byref(img), None)
        assert rc == B.CGX_ERR_INVALID_ARG and b"workspace" in lib.cgx_last_error(ctx)
        rc = lib.cgx_render_forward(ctx, va, 1, C.byref(sc), C.byref(cap), C.c_void_p(256), 16,
                                    C.byref(img), None)
        assert rc == B.CGX_ERR_WORKSPACE
        rc = lib.cgx_render_forward(None, va, 1, C.byref(sc), C.byref(cap), None, 0, C.byref(img), None)
        assert rc == B.CGX_ERR_INVALID_ARG
        tw, th = C.c_int32(0), C.c_int32(0)
        g = B.cgx_grads()
        rc = lib.cgx_tune_tile_shape(ctx, va, 1, C.byref(sc), C.byref(cap), None, 0, C.byref(img), None,
                                     C.byref(img), C.byref(g), None, 0, None, C.byref(tw), C.byref(th),
                                     None)
        assert rc == B.CGX_ERR_INVALID_ARG and b"reps" in lib.cgx_last_error(ctx)
        rc = lib.cgx_tune_tile_shape(None, va, 1, C.byref(sc), C.byref(cap), None, 0, C.byref(img), None,
                                     C.byref(img), C.byref(g), None, 3, None, C.byref(tw), C.byref(th),
                                     None)
        assert rc == B.CGX_ERR_INVALID_ARG
        bits = C.c_int32(0)
        rc = lib.cgx_tune_sort_digits(ctx, va, 1, C.byref(sc), C.byref(cap), None, 0, C.byref(img),
                                      None, C.byref(img), C.byref(g), None, 0, None, C.byref(bits),
                                      None)
        assert rc == B.CGX_ERR_INVALID_ARG and b"reps" in lib.cgx_last_error(ctx)
        rc = lib.cgx_tune_sort_digits(ctx, va, 1, C.byref(sc), C.byref(cap), None, 0, C.byref(img),
                                      None, C.byref(img), C.byref(g), None, 3, None, None, None)
        assert rc == B.CGX_ERR_INVALID_ARG
        # sort digit width: 6..9, default 9, per context
        assert lib.cgx_get_sort_digit_bits(ctx, C.byref(bits)) == B.CGX_OK and bits.value == 9
        for bad in (5, 10, 0, -1):
            assert lib.cgx_set_sort_digit_bits(ctx, bad) == B.CGX_ERR_INVALID_ARG
            assert b"digit" in lib.cgx_last_error(ctx)
        assert lib.cgx_set_sort_digit_bits(ctx, 7) == B.CGX_OK
        assert lib.cgx_get_sort_digit_bits(ctx, C.byref(bits)) == B.CGX_OK and bits.value == 7
        assert lib.cgx_set_sort_digit_bits(None, 8) == B.CGX_ERR_INVALID_ARG
        assert lib.cgx_timing_enable(ctx, -1) == B.CGX_ERR_INVALID_ARG
        assert lib.cgx_graph_launch(None, None) == B.CGX_ERR_INVALID_ARG
        assert lib.cgx_graph_destroy(None) == B.CGX_OK
    finally:
        B.cgx_destroy(ctx)
    assert lib.cgx_last_error(None) == b"no context"


def test_depth_prior_entry_points_reject_bad_arguments(B):
    lib = B.load_library()
    ctx = B.cgx_create(0, 16, 16)
    try:
        va = B.make_views([_view(), _view(32, 16)])
        need = lib.cgx_depth_align_workspace_size(2)
        assert need == B.cgx_depth_align_workspace_size(2) > 0
        assert lib.cgx_depth_align_workspace_size(0) == 0
        fake = C.c_void_p(4096)                      # never dereferenced: every call below fails first
        rc = lib.cgx_depth_prior_align(ctx, va, 2, fake, fake, 10, fake, need - 8, fake, fake, None)
        assert rc == B.CGX_ERR_WORKSPACE
        rc = lib.cgx_depth_prior_align(ctx, va, 2, None, fake, 10, fake, need, fake, fake, None)
        assert rc == B.CGX_ERR_INVALID_ARG
        rc = lib.cgx_depth_prior_align(ctx, va, 2, fake, None, 10, fake, need, fake, fake, None)
        assert rc == B.CGX_ERR_INVALID_ARG and b"points" in lib.cgx_last_error(ctx)
        rc = lib.cgx_depth_prior_align(ctx, va, 2, fake, fake, -1, fake, need, fake, fake, None)
        assert rc == B.CGX_ERR_INVALID_ARG
        rc = lib.cgx_depth_prior_align(ctx, va, 2, fake, fake, 10, C.c_void_p(4100), need, fake, fake, None)
        assert rc == B.CGX_ERR_INVALID_ARG and b"aligned" in lib.cgx_last_error(ctx)
        nb = lambda *x: (C.c_int32 * 2)(*x)  # noqa: E731
        other = C.c_void_p(8192)
        for bad in ((0, -1), (2, 0), (-2, 0)):
            rc = lib.cgx_depth_prior_filter(ctx, va, 2, fake, None, nb(*bad), 1.0, other, None)
            assert rc == B.CGX_ERR_INVALID_ARG and b"nearby" in lib.cgx_last_error(ctx)
        rc = lib.cgx_depth_prior_filter(ctx, va, 2, fake, None, nb(1, 0), 1.0, fake, None)
        assert rc == B.CGX_ERR_INVALID_ARG and b"alias" in lib.cgx_last_error(ctx)
        for tau in (0.0, -1.0, float("nan"), float("inf")):
            rc = lib.cgx_depth_prior_filter(ctx, va, 2, fake, None, nb(1, 0), tau, other, None)
            assert rc == B.CGX_ERR_INVALID_ARG
        rc = lib.cgx_depth_prior_filter(ctx, va, 2, fake, None, None, 1.0, other, None)
        assert rc == B.CGX_ERR_INVALID_ARG
        rc = lib.cgx_depth_prior_filter(ctx, va, 2, fake, C.c_void_p(4100), nb(1, 0), 1.0, other, None)
        assert rc == B.CGX_ERR_INVALID_ARG and b"scale_shift" in lib.cgx_last_error(ctx)
        assert rc == B.CGX_ERR_INVALID_ARG
        rc = lib.cgx_depth_prior_filter(None, va, 2, fake, None, nb(1, 0), 1.0, other, None)
        assert rc == B.CGX_ERR_INVALID_ARG
    finally:
        B.cgx_destroy(ctx)


def test_tsdf_entry_points_reject_bad_arguments(B):
    lib = B.load_library()
    ctx = B.cgx_create(0, 16, 16)
    try:
        va = B.make_views([_view()])
        fake = C.c_void_p(4096)                      # never dereferenced: every call below fails first

        def vol(**kw):
            v = B.cgx_tsdf_volume()
            d = dict(voxel=0.1, trunc=0.3, nx=4, ny=5, nz=6, tsdf=4096, weight=8192, color=None)
            d.update(kw)
            for k, x in d.items():
                setattr(v, k, x)
            return v

        assert lib.cgx_tsdf_init(ctx, None, None) == B.CGX_ERR_INVALID_ARG
        for bad in (dict(tsdf=None), dict(weight=None), dict(nx=0), dict(nz=-1), dict(voxel=0.0),
                    dict(trunc=-1.0), dict(trunc=float("inf")), dict(nx=2048, ny=2048, nz=512)):
            v = vol(**bad)
            assert lib.cgx_tsdf_init(ctx, C.byref(v), None) == B.CGX_ERR_INVALID_ARG, bad
            assert lib.cgx_tsdf_integrate(ctx, va, 1, fake, None, C.byref(v), None, 0, None) == B.CGX_ERR_INVALID_ARG
        v = vol()
        v.origin[1] = float("nan")
        assert lib.cgx_tsdf_integrate(ctx, va, 1, fake, None, C.byref(v), None, 0, None) == B.CGX_ERR_INVALID_ARG
        assert b"origin" in lib.cgx_last_error(ctx)
        v = vol()
        assert lib.cgx_tsdf_integrate(ctx, va, 1, None, None, C.byref(v), None, 0, None) == B.CGX_ERR_INVALID_ARG
        assert b"depth" in lib.cgx_last_error(ctx)
        assert lib.cgx_tsdf_integrate(ctx, va, 0, fake, None, C.byref(v), None, 0, None) == B.CGX_ERR_INVALID_ARG
        assert lib.cgx_tsdf_workspace_size(va, 1) == 16 * 64 * 48
        assert lib.cgx_tsdf_workspace_size(None, 1) == 0
    finally:
        B.cgx_destroy(ctx)
