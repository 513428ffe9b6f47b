"""The tie-aware comparison of the GPU parity tests, exercised on the CPU
with the oracle's own outputs standing in for the GPU's: they must pass,
so must an output that resolves a near tie the other way, and planted
mistakes (a wrong pixel, a missing or foreign pair, a reordered list, a
wrong depth key) must fail."""
import numpy as np
import pytest

from oracle import pipeline
from synth import scenes
from tests import parity


def _packed(r):
    """The oracle's images packed like the library's planar outputs."""
    out = {}
    for key, okey, c, _ in parity.CHANNELS:
        out[key] = np.concatenate([img[okey].reshape(c, -1).ravel() if c > 1 else img[okey].ravel()
                                   for img in r.images])
    return out


def _dbg(r):
    """The oracle's own sorted pairs in the library's debug layout (explicit
    slots view * N + id)."""
    o = r.sorted["own_sorted"]
    return o


@pytest.fixture(scope="module")
def c0():
    wl = scenes.make_c0()
    return wl, pipeline.render_explicit(wl.scene, wl.views)


@pytest.fixture(scope="module")
def anchor11():
    wl = scenes.make_small_anchor(11, n_anchor=70, n_views=3, sizes=((40, 32), (24, 36), (33, 17)))
    return wl, pipeline.render_anchor(wl.scene, wl.views)


@pytest.fixture(scope="module")
def decoded80():
    """Decoded offsets: depth keys that the decode's error may sort either
    way (order ties) on about 60 pixels."""
    wl = scenes.make_small_anchor(80, n_anchor=40, offset_mode=1)
    return wl, pipeline.render_anchor(wl.scene, wl.views)


def test_oracle_outputs_pass(c0, anchor11, decoded80):
    for wl, r in (c0, anchor11, decoded80):
        res = parity.compare_images(_packed(r), r)
        assert res["excluded"] == 0


def _other_outcomes(r):
    """The oracle's images with every near-tie pixel set to the candidate
    farthest from the oracle's own output; returns (packed, pixels moved)."""
    out = _packed(r)
    moved = 0
    offs = 0
    for img in r.images:
        HW = img["depth"].size
        for p, C in img["cands"].items():
            if C.shape[0] < 2:
                continue
            own = np.concatenate([img["rgb"][:, p], [img["D"][p]], img["normal"][:, p],
                                  [img["alpha"][p], img["depth"][p]]])
            d = np.abs(C[:, :9] - own[None]).sum(1)
            k = int(np.argmax(d))
            moved += int(d[k] > 1e-6)
            for key, okey, c, cols in parity.CHANNELS:
                for ch in range(c):
                    out[key][c * offs + ch * HW + p] = C[k, cols][ch]
        offs += HW
    return out, moved


def test_other_tie_outcome_passes(anchor11, decoded80):
    for wl, r in (anchor11, decoded80):
        out, moved = _other_outcomes(r)
        assert moved > 0, "the scene has near-tie pixels with two outcomes"
        parity.compare_images(out, r)
    # the order ties of the decoded scene change the pixels they touch
    wl, r = decoded80
    assert r.images[0]["n_order_ties"] > 20


def test_wrong_pixel_fails(c0):
    wl, r = c0
    out = _packed(r)
    img = r.images[0]
    p = int(np.nonzero(~img["tie"] & (img["alpha"] > 0.5))[0][0])
    out["rgb"][p] *= 1.001
    with pytest.raises(AssertionError):
        parity.compare_images(out, r)


def test_wrong_tie_pixel_fails(anchor11):
    wl, r = anchor11
    out = _packed(r)
    img = r.images[0]
    p = next(iter(img["cands"]))
    out["alpha"][p] = img["alpha"][p] + 0.01
    with pytest.raises(AssertionError):
        parity.compare_images(out, r)


def _dbg_explicit(r, N, drop=None, swap=None, zflip=None):
    o = r.sorted
    sel = o["own"].copy()
    gt, zb, vv, gg = o["gtile"][sel], o["zbits"][sel].astype(np.int64), o["view"][sel], o["gid"][sel]
    if drop is not None:
        keep = np.ones(gt.size, bool)
        keep[drop] = False
        gt, zb, vv, gg = gt[keep], zb[keep], vv[keep], gg[keep]
    if swap is not None:
        i = swap
        for a in (zb, vv, gg):
            a[[i, i + 1]] = a[[i + 1, i]]
    if zflip is not None:
        zb = zb.copy()
        zb[zflip] ^= 1
    n_tiles = o["ranges"].shape[0]
    st = np.searchsorted(gt, np.arange(n_tiles), side="left")
    en = np.searchsorted(gt, np.arange(n_tiles), side="right")
    ranges = np.stack([np.where(en > st, st, 0), np.where(en > st, en, 0)], 1)
    return dict(tile=gt, zbits=zb, slot=vv * N + gg, ranges=ranges)


def test_sort_check(c0):
    wl, r = c0
    N = wl.scene.n
    parity.compare_sort_explicit(_dbg_explicit(r, N), r, N)
    o = r.sorted
    own = np.nonzero(o["own"])[0]
    cert_pos = int(np.nonzero(o["certain"][own])[0][10])
    with pytest.raises(AssertionError):
        parity.compare_sort_explicit(_dbg_explicit(r, N, drop=cert_pos), r, N)
    # two neighbours of one tile with different depth keys, swapped
    gt = o["gtile"][own]
    zb = o["zbits"][own]
    i = int(np.nonzero((gt[:-1] == gt[1:]) & (zb[:-1] != zb[1:]))[0][0])
    with pytest.raises(AssertionError):
        parity.compare_sort_explicit(_dbg_explicit(r, N, swap=i), r, N)
    with pytest.raises(AssertionError):
        parity.compare_sort_explicit(_dbg_explicit(r, N, zflip=i), r, N)


def test_sort_check_accepts_near_tie_pairs(anchor11):
    """A pair one near tie away from the oracle's own binning (a box edge or
    a culling test) may be taken or left."""
    wl, r = anchor11
    o = r.sorted
    extra = ~o["own"]
    uncertain_own = o["own"] & ~o["certain"]
    assert extra.any() or uncertain_own.any()


def test_zero_ties_and_coverage(anchor11, c0):
    for wl, r in (c0, anchor11):
        rng = np.random.default_rng(5)
        og = parity.linear_grads(r, rng)
        for img, g in zip(r.images, og):
            assert np.all(g["rgb"][:, img["frag_grad"]] == 0)
            assert np.all(g["alpha"][~img["frag_grad"]] != 0)
        assert parity.tie_fraction(r) < 0.02


def test_check_grad_slack_budget():
    """The conditioning slack may carry only a small share of the elements:
    elements beyond the plain 1e-4 bound are counted against the budget even
    when their slack covers them."""
    ref = np.linspace(-1, 1, 1000)
    parity.check_grad("ok", ref * (1 + 1e-6), ref, None, np.zeros(1000))
    # huge slack everywhere is harmless while the elements meet the plain bound
    parity.check_grad("slack unused", ref * (1 + 1e-6), ref, None, np.full(1000, 1.0))
    # a few elements (within the budget) may use it
    got = ref.copy()
    got[250:255] *= 1 + 1e-3
    parity.check_grad("few", got, ref, None, np.full(1000, 1e-3 / parity.SENS_K))
    # more than the budget may not, however large their slack
    got[:50] *= 1 + 1e-3
    with pytest.raises(AssertionError):
        parity.check_grad("many", got, ref, None, np.full(1000, 1.0))
    # without slack, one element off fails
    with pytest.raises(AssertionError):
        parity.check_grad("off", ref * (1 + 1e-3), ref, None, np.zeros(1000))


def _prop_inputs(r, N):
    """The oracle's own binning of C0 in the layout the sort-stage property
    check reads from the library (pairs, ranges, per-slot counts, records
    with the pixel box)."""
    o = r.sorted["own_sorted"]
    n_views = len(r.splats)
    counts = np.zeros(n_views * N, np.int64)
    rec = np.zeros(n_views * N, [("bx", "<u4"), ("by", "<u4")])
    for v, S in enumerate(r.splats):
        counts[v * N:(v + 1) * N] = np.where(S["valid"], S["count"], 0)
        b = S["box"]
        rec["bx"][v * N:(v + 1) * N] = (np.clip(b[:, 0], 0, None) | (np.clip(b[:, 1], 0, None) << 16))
        rec["by"][v * N:(v + 1) * N] = (np.clip(b[:, 2], 0, None) | (np.clip(b[:, 3], 0, None) << 16))
    dbg = dict(tile=o["gtile"].copy(), zbits=o["zbits"].astype(np.int64), slot=o["view"] * N + o["gid"],
               ranges=o["ranges"].copy(), counts=counts)
    return dbg, rec


def test_sort_property_check(c0):
    wl, r = c0
    N = wl.scene.n
    view = lambda s: s // N   # noqa: E731
    dbg, rec = _prop_inputs(r, N)
    assert parity.check_sort_properties(dbg, rec, wl.views, (16, 16), view) > 1000
    # planted mistakes: two pairs of a tile swapped, a pair dropped, a depth
    # key changed, a pair moved outside its splat's rectangle
    gt, zb = dbg["tile"], dbg["zbits"]
    i = int(np.nonzero((gt[:-1] == gt[1:]) & (zb[:-1] != zb[1:]))[0][0])
    bad = {k: v.copy() for k, v in dbg.items()}
    for k in ("zbits", "slot"):
        bad[k][[i, i + 1]] = bad[k][[i + 1, i]]
    with pytest.raises(AssertionError):
        parity.check_sort_properties(bad, rec, wl.views, (16, 16), view)
    bad = {k: v.copy() for k, v in dbg.items()}
    bad["counts"][bad["slot"][i]] += 1
    with pytest.raises(AssertionError):
        parity.check_sort_properties(bad, rec, wl.views, (16, 16), view)
    bad = {k: v.copy() for k, v in dbg.items()}
    s = bad["slot"][i]
    j = int(np.nonzero(bad["slot"] == s)[0][-1])
    if j != i:
        bad["zbits"][j] += 1
    else:
        bad["zbits"][i] += 1
        bad["counts"][s] += 1      # (a lone pair: fail on the count instead)
    with pytest.raises(AssertionError):
        parity.check_sort_properties(bad, rec, wl.views, (16, 16), view)
    bad_rec = rec.copy()
    bad_rec["bx"][dbg["slot"][i]] = 0          # box shrunk to column 0
    with pytest.raises(AssertionError):
        parity.check_sort_properties(dbg, bad_rec, wl.views, (16, 16), view)


def test_magnitude_mode_bounds_the_signed_sums(c0, anchor11):
    """composite_backward(magnitude=True) takes the same sums over |terms|:
    every element is at least the absolute value of the signed one, and
    strictly more where terms cancel."""
    from oracle import raster as ras
    for wl, r in (c0, anchor11):
        og = parity.linear_grads(r, np.random.default_rng(9))
        S = ras.composite_backward(r.splats, r.views, r.images, og, r.varr)
        M = ras.composite_backward(r.splats, r.views, r.images, og, r.varr, magnitude=True)
        for s_v, m_v in zip(S, M):
            for k in ("mean2d", "conic", "opacity", "rgb", "d", "normal"):
                a, b = np.abs(np.asarray(s_v[k])), np.asarray(m_v[k])
                assert np.all(b >= a * (1 - 1e-12) - 1e-300), k
                assert np.all(b >= 0), k
        # some element does cancel: the magnitude strictly exceeds it
        assert any(np.any(np.asarray(m_v["mean2d"]) > np.abs(np.asarray(s_v["mean2d"])) * 1.01)
                   for s_v, m_v in zip(S, M))
