"""Pins of the per-attribute decoder heads of the oracle (row f3; Sec. 3.2,
Eq. 4, "a set of shared Gaussian Decoders"): heads with equal hidden
layers are the shared decoder with its output columns regrouped; a head
whose hidden layer is switched off outputs its biases and leaves the other
heads alone; the adjoint matches central differences in every head's
weights."""
import copy

import numpy as np
import pytest

from oracle import anchors
from synth import scenes

N = 10


def _rows(wl):
    rows, _ = anchors.select(wl.scene, wl.views)
    assert rows.shape[0] > 4
    return rows


def _regrouped(sc, offset_mode):
    """A per-attribute-heads twin of a shared decoder: every head's hidden
    layer is the shared one, and head (first, width) takes the shared
    decoder's columns k * G + first + j, k = 0..n-1, j < width, as its
    columns n * first + k * width + j."""
    go = 14 if offset_mode else 11
    groups = [(0, 1), (1, 3), (4, 7)] + ([(11, 3)] if offset_mode else [])
    W1 = anchors.bfmod.from_bits(sc.W1_bits)
    W2 = anchors.bfmod.from_bits(sc.W2_bits)
    b2 = np.asarray(sc.b2, np.float64)
    W2h = np.zeros_like(W2)
    b2h = np.zeros_like(b2)
    for first, width in groups:
        for k in range(N):
            for j in range(width):
                W2h[:, N * first + k * width + j] = W2[:, k * go + first + j]
                b2h[N * first + k * width + j] = b2[k * go + first + j]
    d = copy.copy(sc)
    d.W1_exact = np.tile(W1, (1, len(groups)))
    d.b1 = np.tile(np.asarray(sc.b1, np.float64), len(groups))
    d.W2_exact = W2h
    d.b2 = b2h
    d.decoder_heads = anchors.DECODER_PER_ATTRIBUTE
    return d


@pytest.mark.parametrize("offset_mode", [0, 1])
def test_equal_hidden_layers_are_the_shared_decoder(offset_mode):
    wl = scenes.make_small_anchor(31, offset_mode=offset_mode)
    sc = wl.scene
    rows = _rows(wl)
    A = anchors.decode(sc, wl.views, rows)
    B = anchors.decode(_regrouped(sc, offset_mode), wl.views, rows)
    assert len(B["_heads"]) == 3 + offset_mode
    for k in ("mu", "scales", "quats", "opacity", "rgb"):
        np.testing.assert_allclose(B[k], A[k], rtol=1e-12, atol=1e-14)


def test_switched_off_head_outputs_its_biases():
    """Zeroing head h's hidden block of W1 and b1 leaves z1 = 0 there, so
    that head's outputs are its biases exactly, while the other heads'
    outputs do not change."""
    wl = scenes.make_small_anchor(32, decoder_heads=3, offset_mode=1)
    sc = wl.scene
    rows = _rows(wl)
    base = anchors.decode(sc, wl.views, rows)
    l = np.asarray(sc.l, np.float64)[rows[:, 1]]
    x = np.asarray(sc.x, np.float64)[rows[:, 1]]
    R = rows.shape[0]
    b2 = np.asarray(sc.b2, np.float64)
    W1 = anchors.bfmod.from_bits(sc.W1_bits)
    expect = {  # attribute read from the biases of its head, per Gaussian
        0: lambda: dict(opacity=np.tile(anchors.sigmoid(b2[0:N]), R)),
        1: lambda: dict(rgb=np.tile(anchors.sigmoid(b2[N:4 * N].reshape(N, 3)), (R, 1))),
        2: lambda: dict(scales=(l[:, None, :] * anchors.sigmoid(b2[4 * N:11 * N].reshape(N, 7)[None, :, :3])).reshape(-1, 3),
                        quats=np.tile(b2[4 * N:11 * N].reshape(N, 7)[:, 3:], (R, 1))),
        3: lambda: dict(mu=(x[:, None, :] + b2[11 * N:14 * N].reshape(N, 3)[None] * l[:, None, :]).reshape(-1, 3)),
    }
    owner = dict(opacity=0, rgb=1, scales=2, quats=2, mu=3)
    for h in range(4):
        d = copy.copy(sc)
        Wz = W1.copy()
        Wz[:, 32 * h:32 * (h + 1)] = 0.0
        bz = np.asarray(sc.b1, np.float64).copy()
        bz[32 * h:32 * (h + 1)] = 0.0
        d.W1_exact, d.b1 = Wz, bz
        D = anchors.decode(d, wl.views, rows)
        for key, want in expect[h]().items():
            np.testing.assert_allclose(D[key], want, rtol=1e-14, atol=1e-15, err_msg=f"head {h} {key}")
        for key, o in owner.items():
            if o != h:
                np.testing.assert_array_equal(D[key], base[key], err_msg=f"head {h} moved {key}")


@pytest.mark.parametrize("offset_mode", [0, 1])
def test_head_adjoint_matches_finite_differences(offset_mode):
    wl = scenes.make_small_anchor(33, decoder_heads=3, offset_mode=offset_mode)
    sc = copy.copy(wl.scene)
    sc.W1_exact = anchors.bfmod.from_bits(sc.W1_bits)
    sc.W2_exact = anchors.bfmod.from_bits(sc.W2_bits)
    rows = _rows(wl)
    rng = np.random.default_rng(7)
    D = anchors.decode(sc, wl.views, rows, emulate_bf16=False)
    R = D["mu"].shape[0]
    w = {k: rng.normal(0, 1, (R, c)) for k, c in (("mu", 3), ("scales", 3), ("quats", 4), ("rgb", 3))}
    w["opacity"] = rng.normal(0, 1, R)

    def loss(scene):
        E = anchors.decode(scene, wl.views, rows, emulate_bf16=False)
        return sum(float(np.sum(w[k] * E[k])) for k in w)

    g = anchors.decode_backward(sc, D, w)
    h = 1e-6

    def fd(name, idx):
        e = copy.copy(sc)
        arr = np.array(getattr(sc, name), np.float64)
        arr[idx] += h
        setattr(e, name, arr)
        lp = loss(e)
        arr[idx] -= 2 * h
        lm = loss(e)
        return (lp - lm) / (2 * h)

    n_heads = 3 + offset_mode
    go = 14 if offset_mode else 11
    for hh in range(n_heads):
        for (i, j) in ((3, 32 * hh + 5), (34, 32 * hh + 30), (35, 32 * hh)):
            np.testing.assert_allclose(g["W1"][i, j], fd("W1_exact", (i, j)), rtol=2e-5, atol=1e-6)
        np.testing.assert_allclose(g["b1"][32 * hh + 7], fd("b1", 32 * hh + 7), rtol=2e-5, atol=1e-6)
    for c in (0, 9, N + 4, 4 * N + 13, 11 * N - 1, go * N - 1):
        for i in (0, 17):
            np.testing.assert_allclose(g["W2"][i, c], fd("W2_exact", (i, c)), rtol=2e-5, atol=1e-6)
        np.testing.assert_allclose(g["b2"][c], fd("b2", c), rtol=2e-5, atol=1e-6)
    a = int(rows[0, 1])
    for name in ("x", "l", "F"):
        for j in (0, 2):
            np.testing.assert_allclose(g[name][a, j], fd(name, (a, j)), rtol=2e-5, atol=1e-6)
    if offset_mode:
        np.testing.assert_array_equal(g["O"], 0.0)
    assert g["W1"].shape == (36, 32 * n_heads) and g["W2"].shape == (32, go * N)
