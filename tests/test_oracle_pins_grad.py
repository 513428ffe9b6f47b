"""The oracle's analytic adjoint against central finite differences of its
own forward, in float64, on tiny scenes where no discrete decision moves
under the perturbation (CPU only)."""
import copy

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import pipeline
from oracle import raster as ras
from synth import scenes


@pytest.fixture(autouse=True)
def _exact_means(monkeypatch):
    """Finite differences need the exact (float64) 2-D mean in the
    compositor; its float32 rounding is a step function at this scale."""
    monkeypatch.setattr(ras, "MEAN_F32", False)


def _signature(r):
    """Everything discrete about a render: sorted pairs and, per tile, the
    included-entry mask of every pixel."""
    parts = [r.sorted["gtile"], r.sorted["gid"]]
    for img in r.images:
        for gt in sorted(img["tiles"]):
            parts.append(img["tiles"][gt][4]["inc"].ravel().astype(np.int64))
            parts.append(img["tiles"][gt][4]["keep"].astype(np.int64))
    return np.concatenate([np.asarray(p, np.int64).ravel() for p in parts])


def _fd(scene, render, gs, attr, idx, base_sig, h_rel=1e-6):
    arr = getattr(scene, attr)
    orig = float(arr[idx])
    h = h_rel * max(1.0, abs(orig))
    vals = []
    for sgn in (1, -1):
        arr[idx] = orig + sgn * h
        r = render(scene)
        if not np.array_equal(_signature(r), base_sig):
            arr[idx] = orig
            return None
        vals.append(pipeline.linear_loss(r, gs))
    arr[idx] = orig
    return (vals[0] - vals[1]) / (2 * h)


def _check(scene, render, backward_keys, n_per_attr, seed):
    rng = np.random.default_rng(seed)
    r = render(scene)
    L, gs = pipeline.output_grads_linear(r, rng)
    grads, _ = pipeline.backward(r, gs, scene)
    base_sig = _signature(r)
    checked = 0
    for attr, gkey in backward_keys:
        arr = getattr(scene, attr)
        g = grads[gkey]
        scale = np.max(np.abs(g)) + 1e-12
        flat = np.argsort(-np.abs(g).ravel())
        picks = list(flat[:n_per_attr // 2]) + list(rng.choice(flat, n_per_attr - n_per_attr // 2, replace=False))
        for f in picks:
            idx = np.unravel_index(f, arr.shape)
            num = _fd(scene, render, gs, attr, idx, base_sig)
            if num is None:
                continue
            ana = g[idx]
            assert abs(num - ana) <= 1e-6 * abs(ana) + 2e-7 * scale, (attr, idx, num, ana)
            checked += 1
    return checked


def _explicit_scene(seed, sh_degree):
    wl = scenes.make_small_explicit(seed, n=14, width=30, height=26, sh_degree=sh_degree,
                                    spread=0.45, log_scale=-2.0)
    sc = wl.scene
    for k in ("means", "scales", "quats", "opacity", "sh"):
        setattr(sc, k, np.asarray(getattr(sc, k), np.float64).copy())
    R = Rotation.from_euler("xyz", [0.2, -0.3, 0.1]).as_matrix().astype(np.float32)
    v = wl.views[0]
    v.R = R
    v.t = np.array([0.05, -0.02, 2.5], np.float32)
    return sc, wl.views


@pytest.mark.parametrize("sh_degree", [0, 3])
def test_explicit_gradients_by_finite_differences(sh_degree):
    sc, views = _explicit_scene(31 + sh_degree, sh_degree)
    render = lambda s: pipeline.render_explicit(s, views)   # noqa: E731
    keys = [("means", "means"), ("scales", "scales"), ("quats", "quats"),
            ("opacity", "opacity"), ("sh", "sh")]
    n = _check(sc, render, keys, 10, seed=7)
    assert n >= 35


def test_explicit_gradients_two_views_background():
    sc, views = _explicit_scene(35, 1)
    v2 = copy.deepcopy(views[0])
    v2.width, v2.height = 22, 34
    v2.cx, v2.cy = 11.0, 17.0
    v2.bg = (0.25, 0.5, 0.125)
    v2.t = np.array([-0.1, 0.05, 2.2], np.float32)
    views = [views[0], v2]
    render = lambda s: pipeline.render_explicit(s, views)   # noqa: E731
    keys = [("means", "means"), ("scales", "scales"), ("quats", "quats"), ("opacity", "opacity")]
    assert _check(sc, render, keys, 8, seed=8) >= 25


@pytest.mark.parametrize("act", [0, 1])
def test_anchor_gradients_by_finite_differences(act):
    """Decoder adjoint by central differences; act = 1 reads the opacity as
    tanh with non-positive opacities masked (about half of them here)."""
    wl = scenes.make_small_anchor(41, n_anchor=16, opacity_act=act)
    sc = wl.scene
    for k in ("x", "l", "O", "F", "b1", "b2"):
        setattr(sc, k, np.asarray(getattr(sc, k), np.float64).copy())
    sc.W1_exact = sc.W1.astype(np.float64).copy()
    sc.W2_exact = sc.W2.astype(np.float64).copy()
    render = lambda s: pipeline.render_anchor(s, wl.views, emulate_bf16=False)   # noqa: E731
    r = render(sc)
    assert r.rows.shape[0] >= 8
    keys = [("x", "x"), ("l", "l"), ("O", "O"), ("F", "F"), ("b1", "b1"), ("b2", "b2"),
            ("W1_exact", "W1"), ("W2_exact", "W2")]
    assert _check(sc, render, keys, 8, seed=9) >= 45
