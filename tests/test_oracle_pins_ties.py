"""Pins of the oracle's near-tie certification (the decisions it lets the
GPU take either way).

The GPU takes the pixel boxes' centres, the depth keys and the compositor's
2-D mean from float64 arithmetic it shares with the oracle (so those agree
exactly); what float32 changes are the covariance, conic, opacity, colour
and normal, by a few rounding errors.  So the oracle run again with the
scales, rotations, opacities and colours (explicit Gaussians) or the decoder
weights and biases (anchors) perturbed by four float32 ulps must (i) change
no decision the oracle certified as clear: every pixel without a tie keeps
its value to 1e-4, and every pixel with ties lands on one of the outcomes
the oracle enumerated for it; (ii) keep every pair the oracle is certain of
and take no pair it does not list, in the same (depth bits, view, id)
order.  A tie bound set too tight (a planted mistake) makes this fail."""
import copy

import numpy as np
import pytest

from oracle import pipeline
from oracle import project as prj
from oracle import raster as ras
from synth import scenes
from tests import parity

PERT = 2.0 ** -22          # four float32 ulps, relative


def _perturb(scene, keys, rng):
    sc = copy.copy(scene)
    for k in keys:
        a = np.asarray(getattr(scene, k))
        if a.dtype.kind == "f":
            setattr(sc, k, a.astype(np.float64) * (1.0 + PERT * rng.standard_normal(a.shape)))
    return sc


def _packed(r):
    out = {}
    for key, okey, c, _ in parity.CHANNELS:
        out[key] = np.concatenate([img[okey].reshape(c, -1).ravel() if c > 1 else img[okey].ravel()
                                   for img in r.images])
    return out


def _as_dbg(r1):
    """A perturbed oracle run's own binning, in the library's debug layout
    (slot = view * 2^20 + id)."""
    o = r1.sorted["own_sorted"]
    return dict(tile=o["gtile"], zbits=o["zbits"].astype(np.int64), slot=o["view"] * (1 << 20) + o["gid"],
                ranges=o["ranges"])


def _check(r0, r1):
    # decisions are the subject here: the norm-wise image bound is taken at
    # the element-wise 1e-4 (the perturbations are several ulps, not one)
    old = parity.NORM_RTOL
    parity.NORM_RTOL = parity.RTOL
    try:
        parity.compare_images(_packed(r1), r0)
    finally:
        parity.NORM_RTOL = old
    n, took, left = parity.compare_sorted(_as_dbg(r1), r0, lambda s: (s >> 20, s & ((1 << 20) - 1)))
    assert n == r1.sorted["own_sorted"]["gtile"].size
    return took + left


EXPLICIT = ("scales", "quats", "opacity", "sh")


def _anchor_perturbed(scene, rng, pert=PERT):
    sc = copy.copy(scene)
    for k in ("b1", "b2"):
        a = np.asarray(getattr(scene, k), np.float64)
        setattr(sc, k, a * (1.0 + pert * rng.standard_normal(a.shape)))
    sc.W1_exact = np.asarray(scene.W1, np.float64) * (1 + pert * rng.standard_normal(scene.W1.shape))
    sc.W2_exact = np.asarray(scene.W2, np.float64) * (1 + pert * rng.standard_normal(scene.W2.shape))
    return sc


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_perturbed_c0_stays_within_ties(seed):
    wl = scenes.make_c0()
    r0 = pipeline.render_explicit(wl.scene, wl.views)
    r1 = pipeline.render_explicit(_perturb(wl.scene, EXPLICIT, np.random.default_rng(seed)), wl.views)
    _check(r0, r1)


@pytest.mark.parametrize("seed,tile", [(11, (16, 16)), (13, (32, 8))])
def test_perturbed_anchor_stays_within_ties(seed, tile):
    wl = scenes.make_small_anchor(seed, n_anchor=70, n_views=3, sizes=((40, 32), (24, 36), (33, 17)))
    r0 = pipeline.render_anchor(wl.scene, wl.views, tile=tile)
    r1 = pipeline.render_anchor(_anchor_perturbed(wl.scene, np.random.default_rng(seed)), wl.views,
                                tile=tile)
    _check(r0, r1)


def _own_row(img, p):
    return np.concatenate([img["rgb"][:, p], [img["D"][p]], img["normal"][:, p],
                           [img["alpha"][p], img["depth"][p]]])


def test_candidates_are_the_other_outcomes():
    """At 64 ulps the perturbed runs do resolve some ties the other way; each
    such pixel then equals one of the oracle's other enumerated outcomes (to
    a tolerance that covers 64 ulps of conditioning), so the candidates are
    the outcomes a float32 evaluation reaches."""
    wl = scenes.make_small_anchor(11, n_anchor=70, n_views=3, sizes=((40, 32), (24, 36), (33, 17)))
    r0 = pipeline.render_anchor(wl.scene, wl.views)
    other = 0
    for seed in range(8):
        r1 = pipeline.render_anchor(_anchor_perturbed(wl.scene, np.random.default_rng(100 + seed),
                                                      2.0 ** -18), wl.views)
        for a, b in zip(r0.images, r1.images):
            for p, C in a["cands"].items():
                got = _own_row(b, p)
                dist = np.abs(C[:, :9] - got[None]).max(1) / (np.abs(got).max() + 1e-3)
                k = int(np.argmin(dist))
                assert dist[k] < 1e-3, (p, dist[k])
                k0 = int(np.argmin(np.abs(C[:, :9] - _own_row(a, p)[None]).max(1)))
                if k != k0 and np.abs(C[k, :9] - C[k0, :9]).max() > 1e-6:
                    other += 1
    assert other > 0


def test_too_tight_bound_is_caught(monkeypatch):
    """Planted mistake: with the tie bounds near zero the oracle enumerates
    no outcomes, and an output that resolves its near ties the other way (a
    correct float32 result) fails the comparison."""
    wl = scenes.make_small_anchor(11, n_anchor=70, n_views=3, sizes=((40, 32), (24, 36), (33, 17)))
    r0 = pipeline.render_anchor(wl.scene, wl.views)
    out = _packed(r0)
    img = r0.images[0]
    HW = img["depth"].size
    flipped = 0
    for p, C in img["cands"].items():
        own = _own_row(img, p)
        k = int(np.argmax(np.abs(C[:, :9] - own[None]).max(1)))
        if np.abs(C[k, :9] - own).max() < 1e-3:
            continue
        for key, okey, c, cols in parity.CHANNELS:
            for ch in range(c):
                out[key][ch * HW + p] = C[k, cols][ch]
        flipped += 1
    assert flipped > 0
    parity.compare_images(out, r0)
    monkeypatch.setattr(ras, "FRAG_ALPHA", 1e-12)
    monkeypatch.setattr(ras, "FRAG_T", 1e-12)
    monkeypatch.setattr(prj, "FRAG", 1e-12)
    r_tight = pipeline.render_anchor(wl.scene, wl.views)
    with pytest.raises(AssertionError):
        parity.compare_images(out, r_tight)


def test_unflagged_decisions_have_margin():
    """Every pixel without a tie has each alpha decision of its walked list at
    least FRAG_ALPHA from 1/255 and each transmittance step at least FRAG_T
    from 1e-4 (in relative terms)."""
    wl = scenes.make_c0()
    r = pipeline.render_explicit(wl.scene, wl.views)
    img = r.images[0]
    checked = 0
    for gtile, (ent, I, J, pix, R) in img["tiles"].items():
        if ent.size == 0:
            continue
        E = R["E"]
        clear = ~R["tie"]
        pw = E["power"] <= 0
        inb = E["inbox"] & pw
        m = np.abs(E["raw"] * 255.0 - 1.0)
        assert np.all(m[clear][inb[clear]] >= ras.FRAG_ALPHA)
        a_use = np.where(E["use"], E["alpha"], 0.0)
        Tp = np.cumprod(1.0 - a_use, axis=1)
        mt = np.abs(Tp / ras.T_MIN - 1.0)
        assert np.all(mt[clear][E["use"][clear]] >= ras.FRAG_T)
        checked += int(clear.sum())
    assert checked > 4000
