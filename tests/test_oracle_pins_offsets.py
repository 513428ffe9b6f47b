"""Pins of the decoder-emitted offsets variant of the oracle decoder (row
f3; Sec. 3.2, Eq. 4): an exact reduction to the learned-offset decoder,
and finite differences of the adjoint."""
import copy

import numpy as np

from oracle import anchors
from synth import scenes


def _base(seed=21):
    wl = scenes.make_small_anchor(seed)
    sc = wl.scene
    rows, _ = anchors.select(sc, wl.views)
    assert rows.shape[0] > 4
    return wl, sc, rows


def _decoded_twin(sc, rng, shared_O=True):
    """The same scene with offset_mode = 1 and a 32 x 14n decoder whose
    first 11 outputs per Gaussian are the original ones."""
    n = sc.O.shape[1]
    W2 = anchors.bfmod.from_bits(sc.W2_bits).reshape(32, n, 11)
    b2 = np.asarray(sc.b2, np.float64).reshape(n, 11)
    W2d = np.zeros((32, n, 14))
    b2d = np.zeros((n, 14))
    W2d[..., :11], b2d[:, :11] = W2, b2
    d = copy.copy(sc)
    if shared_O:
        O = rng.normal(0, 0.5, (n, 3))
        b2d[:, 11:14] = O
        d.O = np.broadcast_to(O, sc.O.shape).astype(np.float64)
    else:
        W2d[..., 11:14] = rng.normal(0, 0.2, (32, n, 3))
        b2d[:, 11:14] = rng.normal(0, 0.5, (n, 3))
    d.W2_exact = W2d.reshape(32, n * 14)
    d.b2 = b2d.reshape(-1)
    d.offset_mode = anchors.OFFSETS_DECODED
    return d


def test_decoded_offsets_reduce_to_learned_offsets():
    """Offset columns with zero weights and biases equal to a shared O give
    exactly the learned-offset decoder with that O in every anchor."""
    wl, sc, rows = _base()
    rng = np.random.default_rng(5)
    d = _decoded_twin(sc, rng)
    learned = copy.copy(sc)
    learned.O = d.O
    A = anchors.decode(learned, wl.views, rows)
    B = anchors.decode(d, wl.views, rows)
    # the offset columns add exactly zero to O, so the means match bit for
    # bit; the other outputs come from a wider matrix product whose BLAS
    # blocking may sum in another order
    np.testing.assert_array_equal(A["mu"], B["mu"])
    for k in ("scales", "quats", "opacity", "rgb"):
        np.testing.assert_allclose(A[k], B[k], rtol=1e-13, atol=1e-15)
    assert B["_z2"].shape[1] == 14 * sc.O.shape[1]


def test_decoded_offsets_adjoint_matches_finite_differences():
    """A random linear functional of the decoded Gaussians; its gradient with
    respect to W2 (offset columns included), b2, l and x by central
    differences against decode_backward."""
    wl, sc, rows = _base(22)
    rng = np.random.default_rng(6)
    d = _decoded_twin(sc, rng, shared_O=False)
    D = anchors.decode(d, wl.views, rows, emulate_bf16=False)
    R = D["mu"].shape[0]
    w = {k: rng.normal(0, 1, (R, c)) for k, c in (("mu", 3), ("scales", 3), ("quats", 4), ("rgb", 3))}
    w["opacity"] = rng.normal(0, 1, R)

    def loss(scene):
        E = anchors.decode(scene, wl.views, rows, emulate_bf16=False)
        return sum(float(np.sum(w[k] * E[k])) for k in w)

    g = anchors.decode_backward(d, D, w)
    n = sc.O.shape[1]
    h = 1e-6
    # offset columns and other columns of W2, biases of both kinds
    for (i, c) in ((3, 11), (7, 12), (30, 14 * 2 + 13), (5, 0), (9, 14 + 4)):
        e = copy.copy(d)
        e.W2_exact = d.W2_exact.copy()
        e.W2_exact[i, c] += h
        lp = loss(e)
        e.W2_exact[i, c] -= 2 * h
        lm = loss(e)
        np.testing.assert_allclose(g["W2"][i, c], (lp - lm) / (2 * h), rtol=2e-5, atol=1e-6)
    for c in (11, 14 * 3 + 12, 2):
        e = copy.copy(d)
        e.b2 = d.b2.copy()
        e.b2[c] += h
        lp = loss(e)
        e.b2[c] -= 2 * h
        lm = loss(e)
        np.testing.assert_allclose(g["b2"][c], (lp - lm) / (2 * h), rtol=2e-5, atol=1e-6)
    a = int(rows[0, 1])
    for arr, key in (("l", "l"), ("x", "x")):
        for j in range(3):
            e = copy.copy(d)
            setattr(e, arr, np.array(getattr(d, arr), np.float64).copy())
            getattr(e, arr)[a, j] += h
            lp = loss(e)
            getattr(e, arr)[a, j] -= 2 * h
            lm = loss(e)
            np.testing.assert_allclose(g[key][a, j], (lp - lm) / (2 * h), rtol=2e-5, atol=1e-6)
    np.testing.assert_array_equal(g["O"], 0.0)        # the table's offsets are unused
    assert n == d.O.shape[1]


def test_decoded_offset_error_bound_holds_in_float32():
    """The oracle's margin for a decoded offset's float32 error (mu_tol / l)
    covers float32 evaluations of the decoder in two summation orders
    (BLAS and strictly sequential) at least four times over, and is not
    vacuous (within 2^8 of the largest error)."""
    wl = scenes.make_small_anchor(61, n_anchor=70, n_views=3, sizes=((40, 32), (24, 36), (33, 17)),
                                  offset_mode=1)
    sc = wl.scene
    rows, _ = anchors.select(sc, wl.views)
    D = anchors.decode(sc, wl.views, rows)
    n = sc.O.shape[1]
    l = np.asarray(sc.l, np.float64)[rows[:, 1]]
    bound = (D["mu_tol"].reshape(-1, n, 3) / l[:, None, :])
    O64 = D["_O"]
    f32 = np.float32
    z0, W1, b1 = D["_z0"].astype(f32), D["_W1"].astype(f32), np.asarray(sc.b1, f32)
    W2, b2 = D["_W2"].astype(f32), np.asarray(sc.b2, f32)
    cols = (np.arange(n)[:, None] * 14 + 11 + np.arange(3)[None]).ravel()
    z1 = np.maximum(z0 @ W1 + b1, f32(0))
    O_blas = (z1 @ W2[:, cols] + b2[cols]).reshape(-1, n, 3)
    # strictly sequential float32 accumulation (first 40 rows)
    m = 40
    z1s = np.zeros((m, 32), f32)
    for j in range(32):
        acc = np.full(m, b1[j], f32)
        for i in range(36):
            acc = f32(acc + z0[:m, i] * W1[i, j])
        z1s[:, j] = np.maximum(acc, f32(0))
    O_seq = np.zeros((m, cols.size), f32)
    for q, c in enumerate(cols):
        acc = np.full(m, b2[c], f32)
        for j in range(32):
            acc = f32(acc + z1s[:, j] * W2[j, c])
        O_seq[:, q] = acc
    O_seq = O_seq.reshape(m, n, 3)
    worst = 0.0
    for O32, sl in ((O_blas, slice(None)), (O_seq, slice(0, m))):
        ratio = np.abs(O32.astype(np.float64) - O64[sl]) / bound[sl]
        worst = max(worst, float(ratio.max()))
    assert 2.0 ** -8 < worst <= 0.25, worst
