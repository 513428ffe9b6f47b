"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare with the FP64 oracle on the same seeded inputs.

Near ties.  A decision fed by float32 on the GPU and float64 in the oracle
(a box edge, the alpha threshold, the transmittance stop, the depth guard, a
splat's normal axis) is a near tie when the oracle's margin is below the
stated bound; then both outcomes are correct.  The oracle certifies every
such tie and enumerates the outputs a pixel may take under them
(`cands`); the GPU's pixel must equal one of those outputs.  Pixels with
more ties than the oracle enumerates are excluded and counted, within a
budget of 1e-4 of the compared pixels.  For gradients, the output gradients
of the pixels with a tie (`frag_grad`) are zero on both sides (the linear
losses of the gradient tests), so every gradient element is compared; the
fused L1 tests, whose seed the GPU computes itself, give those pixels'
share of each element as slack instead.
"""
import os
import re

import numpy as np

RTOL = 1e-4          # images and gradients, relative (fp32 GPU vs fp64 oracle)
# Relative floor: the tolerance never falls below RTOL * FLOOR * max|ref| of
# the tensor.  Signed channels (normal x/y, gradients) are sums whose float32
# error scales with the sum of |terms|, not with the net value, so elements
# that cancel to a small fraction of the tensor's range get this slack.
FLOOR = 1e-3
NORM_RTOL = 1e-5     # norm-wise relative error over the compared elements
EXCL_BUDGET = 1e-4   # pixels excluded (more ties than enumerated), per compared pixel


def check_close(name, got, ref, exclude=None, rtol=RTOL, floor=FLOOR, report=None, mag=None,
                quiet=False):
    """Element-wise |got - ref| <= rtol * max(m, floor * max|ref|) on every
    element not excluded, where m is |ref| or, for a blended signed quantity,
    the blend of |terms| (mag)."""
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    ex = np.zeros(ref.shape, bool) if exclude is None else np.asarray(exclude, bool).ravel()
    keep = ~ex
    scale = np.max(np.abs(ref[keep])) if keep.any() else 0.0
    m = np.abs(ref) if mag is None else np.maximum(np.abs(ref), np.asarray(mag, np.float64).ravel())
    tol = rtol * np.maximum(m, floor * scale)
    err = np.abs(got - ref)
    bad = (err > tol) & keep
    assert np.all(np.isfinite(got[keep])), f"{name}: non-finite values"
    rel = np.max(err[keep] / np.maximum(m[keep], floor * scale + 1e-300)) if keep.any() else 0.0
    # the norm-wise error is taken over the elements whose float32 error scale
    # is their own size (a blend of |terms| more than 10x the net value, as at
    # grazing incidence, is held to the element-wise bound only)
    wc = keep & (m <= 10.0 * np.maximum(np.abs(ref), floor * scale))
    nrm = np.linalg.norm(ref[wc])
    nrel = float(np.linalg.norm((got - ref)[wc]) / nrm) if nrm > 0 else float(np.linalg.norm(got[wc]))
    if report is not None:
        report[name] = dict(max_rel=float(rel), norm_rel=nrel, excluded=int(ex.sum()), n=int(ref.size))
    if not quiet:
        print(f"  {name}: max floored rel err {rel:.2e}, norm rel err {nrel:.2e}, "
              f"set aside {int(ex.sum())}/{ref.size}", flush=True)
    if bad.any():
        i = np.argmax(np.where(bad, err / np.maximum(tol, 1e-300), 0))
        raise AssertionError(f"{name}: {int(bad.sum())}/{keep.sum()} elements out of tolerance; "
                             f"worst idx {i}: got {got[i]!r} ref {ref[i]!r} tol {tol[i]:.3g}")
    assert nrel <= NORM_RTOL, f"{name}: norm-wise relative error {nrel:.3g} > {NORM_RTOL}"
    return rel


# Image channels: (key in the library's output, key in the oracle image,
# channels, columns of an oracle candidate row).  A candidate row holds
# rgb 3, plane distance D, normal 3, alpha, unbiased depth, |normal| blend 3,
# and the unbiased depth's error scale (|D^| times the cancellation of its
# denominator s = -N . ray, the sum of |terms| over |s|).
CHANNELS = (("rgb", "rgb", 3, slice(0, 3)), ("plane_d", "D", 1, slice(3, 4)),
            ("normal", "normal", 3, slice(4, 7)), ("alpha", "alpha", 1, slice(7, 8)),
            ("depth", "depth", 1, slice(8, 9)))
NABS = slice(9, 12)
DMAG = slice(12, 13)


def _np(a):
    return a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)


def _gather(out, r, covered_only):
    """Per channel: GPU and oracle values (pixels x channels) over the
    compared pixels of every view, with the tie / exclusion masks and the
    global pixel ids (view, pixel)."""
    pix_off = r.layout["pix_off"]
    res = {}
    ids = []
    for v, img in enumerate(r.images):
        HW = img["depth"].size
        pix = np.nonzero(img["covered"])[0] if covered_only else np.arange(HW)
        ids.append(np.stack([np.full(pix.size, v), pix], 1))
    ids = np.concatenate(ids)
    for key, okey, c, _ in CHANNELS:
        g = _np(out[key]).astype(np.float64)
        gv, rv = [], []
        for v, img in enumerate(r.images):
            HW = img["depth"].size
            pix = ids[ids[:, 0] == v, 1]
            base = c * int(pix_off[v])
            gv.append(np.stack([g[base + ch * HW + pix] for ch in range(c)], 1))
            a = img[okey].reshape(c, HW) if c > 1 else img[okey].reshape(1, HW)
            rv.append(a[:, pix].T)
        res[key] = (np.concatenate(gv), np.concatenate(rv))
    nab = np.concatenate([img["normal_abs"].reshape(3, -1)[:, ids[ids[:, 0] == v, 1]].T
                          for v, img in enumerate(r.images)])
    dmag = np.concatenate([img["depth_mag"][ids[ids[:, 0] == v, 1]][:, None]
                           for v, img in enumerate(r.images)])
    tie = np.concatenate([img["tie"][ids[ids[:, 0] == v, 1]] for v, img in enumerate(r.images)])
    excl = np.concatenate([img["excl"][ids[ids[:, 0] == v, 1]] for v, img in enumerate(r.images)])
    return res, nab, dmag, tie, excl, ids


def compare_images(out, r, report=None, covered_only=False):
    """out: dict of packed GPU images (torch or numpy) for the views of the
    oracle result r.  Pixels without a near tie are compared element-wise
    with the oracle's own outputs; a pixel with ties must match one of the
    oracle's candidate outputs in every channel; pixels with more ties than
    enumerated are excluded, within EXCL_BUDGET.  Returns the counts."""
    res, nab, dmag, tie, excl, ids = _gather(out, r, covered_only)
    npx = ids.shape[0]
    aside = tie | excl
    scales = {}
    for key, okey, c, _ in CHANNELS:
        got, ref = res[key]
        mag = nab if key == "normal" else (dmag if key == "depth" else None)
        check_close(key, got, ref, np.repeat(aside[:, None], c, 1), report=report, mag=mag)
        keep = ~aside
        scales[key] = np.max(np.abs(ref[keep])) if keep.any() else 0.0
    # tie pixels: one of the oracle's candidates, all channels at once
    worst = 0.0
    for i in np.nonzero(tie & ~excl)[0]:
        v, p = ids[i]
        C = r.images[v]["cands"][int(p)]
        ok = np.ones(C.shape[0], bool)
        ratio = np.zeros(C.shape[0])
        for key, okey, c, cols in CHANNELS:
            g = res[key][0][i]
            ref = C[:, cols]
            m = np.abs(ref)
            if key == "normal":
                m = np.maximum(m, C[:, NABS])
            if key == "depth":
                m = np.maximum(m, C[:, DMAG])
            tol = RTOL * np.maximum(m, FLOOR * scales[key]) + 1e-300
            q = np.max(np.abs(g[None] - ref) / tol, axis=1)
            ratio = np.maximum(ratio, q)
        best = float(ratio.min())
        assert best <= 1.0, (f"pixel {p} of view {v}: no oracle outcome of its {C.shape[0]} "
                             f"candidates matches (best error {best:.3g} x tolerance); "
                             f"got rgb {res['rgb'][0][i]} alpha {res['alpha'][0][i]}")
        worst = max(worst, best)
        assert ok.any()
    n_tie, n_ex = int((tie & ~excl).sum()), int(excl.sum())
    print(f"  near-tie pixels matched to an oracle outcome: {n_tie}/{npx} (worst {worst:.2f} x tol); "
          f"excluded {n_ex}", flush=True)
    assert n_ex <= EXCL_BUDGET * npx, f"excluded pixels {n_ex} > {EXCL_BUDGET} of {npx}"
    if report is not None:
        report["pixels"] = dict(n=npx, ties=n_tie, excluded=n_ex)
    return dict(n=npx, ties=n_tie, excluded=n_ex)


def compare_sorted(dbg, r, slot_to_view_gid, tiles=None):
    """Sorted pairs, nothing dropped.  For every tile (or the given global
    tiles) the GPU's list must hold every pair the oracle is certain of, only
    pairs the oracle lists (its own, or one near tie away), with depth keys
    bit-identical to the oracle's (within the oracle's key tolerance where
    the mean carries a decode error), in (depth bits, view, id) order, with
    the ranges of the GPU's sorted tile ids.  Returns (pairs checked, near-tie
    pairs the GPU took, near-tie pairs it left)."""
    gt = dbg["tile"].astype(np.int64)
    gz = dbg["zbits"].astype(np.int64)
    slots = dbg["slot"].astype(np.int64)
    gr = dbg["ranges"].astype(np.int64)
    o = r.sorted
    n_tiles = o["ranges"].shape[0]
    if tiles is None:
        tiles = np.arange(n_tiles)
        assert np.all(np.diff(gt) >= 0), "GPU tile ids not sorted"
        starts = np.searchsorted(gt, np.arange(n_tiles), side="left")
        ends = np.searchsorted(gt, np.arange(n_tiles), side="right")
        want = np.stack([np.where(ends > starts, starts, 0), np.where(ends > starts, ends, 0)], 1)
        # an empty tile's range may be any [s, s)
        norm = np.where((gr[:, 1] > gr[:, 0])[:, None], gr, 0)
        np.testing.assert_array_equal(norm, want, err_msg="tile ranges")
    n_checked = n_took = n_left = 0
    for t in tiles:
        t = int(t)
        g0, g1 = gr[t]
        g1 = max(g1, g0)
        o0, o1 = o["ranges"][t]
        assert np.all(gt[g0:g1] == t), f"tile {t}: foreign pairs in its range"
        v, gid = slot_to_view_gid(slots[g0:g1])
        got = np.stack([gz[g0:g1], v, gid], 1)
        # the GPU list is in (depth bits, view, id) order
        order = np.lexsort((got[:, 2], got[:, 1], got[:, 0]))
        np.testing.assert_array_equal(order, np.arange(got.shape[0]), err_msg=f"tile {t}: order")
        ref = np.stack([o["zbits"][o0:o1].astype(np.int64), o["view"][o0:o1], o["gid"][o0:o1]], 1)
        own, cert = o["own"][o0:o1], o["certain"][o0:o1]
        rk = {(int(a), int(b)): i for i, (a, b) in enumerate(ref[:, 1:])}
        idx = np.array([rk.get((int(a), int(b)), -1) for a, b in got[:, 1:]], np.int64)
        assert np.all(idx >= 0), (f"tile {t}: GPU pairs the oracle does not list: "
                                  f"{got[idx < 0][:5].tolist()}")
        # bit-identical, or within the key's tolerance where the mean carries
        # a decode error (decoded offsets)
        ztol = o["ztol"][o0:o1][idx]
        bad = np.abs(got[:, 0] - ref[idx, 0]) > ztol
        assert not bad.any(), (f"tile {t}: depth keys {got[bad, 0][:5].tolist()} vs "
                               f"{ref[idx, 0][bad][:5].tolist()} (tolerance {ztol[bad][:5].tolist()})")
        taken = np.zeros(ref.shape[0], bool)
        taken[idx] = True
        assert np.all(taken[cert]), (f"tile {t}: GPU lacks certain pairs "
                                     f"{ref[cert & ~taken][:5].tolist()}")
        n_checked += got.shape[0]
        n_took += int((taken & ~cert).sum())
        n_left += int((~taken & own & ~cert).sum())
    return n_checked, n_took, n_left


def check_sort_properties(dbg, rec, views, tile, slot_view):
    """The sort stage over every tile, from properties that hold at any
    size (no oracle, nothing set aside): the pairs are in strictly
    increasing (tile, depth bits, slot) order, the tile ranges delimit the
    tile ids, each visible splat has exactly its tile count of pairs, all
    with one depth key, each in the tile rectangle of its pixel box, and
    only splats whose box spans at least 2 x 2 and at most 64 tiles (those
    that carry a tile mask) have fewer pairs than their rectangle holds.
    rec: the splat records of cgx_debug_splats; slot_view(slots) -> views.
    Returns the number of pairs checked."""
    tw, th = tile
    gt = dbg["tile"].astype(np.int64)
    zb = dbg["zbits"].astype(np.int64)
    sl = dbg["slot"].astype(np.int64)
    counts = dbg["counts"].astype(np.int64)
    P = gt.size
    if P > 1:
        dt, dz, ds = np.diff(gt), np.diff(zb), np.diff(sl)
        inc = (dt > 0) | ((dt == 0) & ((dz > 0) | ((dz == 0) & (ds > 0))))
        bad = np.nonzero(~inc)[0]
        assert bad.size == 0, f"pairs out of (tile, depth, slot) order at {bad[:5].tolist()}"
    TX = np.array([-(-int(v.width) // tw) for v in views], np.int64)
    TY = np.array([-(-int(v.height) // th) for v in views], np.int64)
    tile_off = np.concatenate([[0], np.cumsum(TX * TY)])
    n_tiles = int(tile_off[-1])
    gr = dbg["ranges"].astype(np.int64)
    assert gr.shape[0] == n_tiles
    starts = np.searchsorted(gt, np.arange(n_tiles), side="left")
    ends = np.searchsorted(gt, np.arange(n_tiles), side="right")
    want = np.stack([np.where(ends > starts, starts, 0), np.where(ends > starts, ends, 0)], 1)
    norm = np.where((gr[:, 1] > gr[:, 0])[:, None], gr, 0)
    np.testing.assert_array_equal(norm, want, err_msg="tile ranges")
    assert P == 0 or (gt[0] >= 0 and gt[-1] < n_tiles)
    # per splat: the pair count and one depth key
    np.testing.assert_array_equal(np.bincount(sl, minlength=counts.size)[:counts.size], counts,
                                  err_msg="pairs per splat vs its tile count")
    assert P == 0 or sl.max() < counts.size
    order = np.argsort(sl, kind="stable")
    s_sorted, z_sorted = sl[order], zb[order]
    same = s_sorted[1:] == s_sorted[:-1]
    assert np.all(z_sorted[1:][same] == z_sorted[:-1][same]), "a splat's pairs carry two depth keys"
    # each pair in the tile rectangle of its splat's pixel box
    v = np.asarray(slot_view(sl), np.int64)
    bx, by = rec["bx"][sl].astype(np.int64), rec["by"][sl].astype(np.int64)
    x0, x1, y0, y1 = bx & 0xFFFF, bx >> 16, by & 0xFFFF, by >> 16
    local = gt - tile_off[v]
    tx, ty = local % TX[v], local // TX[v]
    inside = (local >= 0) & (local < TX[v] * TY[v]) & (tx >= x0 // tw) & (tx <= x1 // tw) \
        & (ty >= y0 // th) & (ty <= y1 // th)
    bad = np.nonzero(~inside)[0]
    assert bad.size == 0, f"pairs outside their splat's tile rectangle at {bad[:5].tolist()}"
    # fewer pairs than the rectangle only where a tile mask is carried
    vis = np.nonzero(counts > 0)[0]
    bxv, byv = rec["bx"][vis].astype(np.int64), rec["by"][vis].astype(np.int64)
    nx = (bxv >> 16) // tw - (bxv & 0xFFFF) // tw + 1
    ny = (byv >> 16) // th - (byv & 0xFFFF) // th + 1
    masked = (nx > 1) & (ny > 1) & (nx * ny <= 64)
    assert np.all(counts[vis] <= nx * ny), "more pairs than the rectangle"
    full = ~masked
    assert np.all(counts[vis][full] == (nx * ny)[full]), "unmasked splat without its full rectangle"
    print(f"  sort stage, every tile: {P} pairs of {vis.size} splats in order, ranges, "
          f"counts and rectangles consistent ({int(masked.sum())} splats with a tile mask)",
          flush=True)
    return P


def compare_sort_explicit(dbg, r, N):
    """Explicit scenes: slot = view * N + Gaussian.  Returns (pairs checked,
    near-tie pairs the GPU took, near-tie pairs it left)."""
    n, took, left = compare_sorted(dbg, r, lambda s: (s // N, s % N))
    assert n == int(dbg["tile"].size), (n, dbg["tile"].size)
    print(f"  sorted pairs: {n} bit-exact (near-tie pairs taken {took}, left {left})", flush=True)
    return n, took, left


def compare_sort_anchor(dbg, r, n_off):
    """Anchor path: rows bit-exact; each slot (row * n + k) maps to its
    view-local id (row - first row of the view) * n + k."""
    rows = dbg["rows"].astype(np.int64)
    np.testing.assert_array_equal(rows, r.rows)

    def s2vg(slot):
        row, k = slot // n_off, slot % n_off
        view = rows[row, 0]
        return view, (row - r.row_off[view]) * n_off + k

    n, took, left = compare_sorted(dbg, r, s2vg)
    assert n == int(dbg["tile"].size), (n, dbg["tile"].size)
    print(f"  sorted pairs: {n} bit-exact (near-tie pairs taken {took}, left {left})", flush=True)
    return n


# ---------------------------------------------------------------------------
# gradients: 1e-4 relative where the element is well conditioned
# ---------------------------------------------------------------------------
SENS_EPS = 2.0 ** -24      # relative input perturbation of float32 rounding size
SENS_K = 16.0              # float32 rounding events the GPU chain may accumulate per input one
ROUND_K = 4.0              # multiple of the per-splat rounding-scale probe (rounding_sensitivity)
GRAD_NORM_RTOL = 1e-4
# At most this share of a gradient tensor's gradient-bearing elements (and
# at least SLACK_MIN elements of a small tensor) may lie beyond the plain
# 1e-4 bound, inside their conditioning slack.  Measured on MI355X over the
# whole GPU suite: at most 0.9 % of a tensor's elements needed it (sums
# whose terms cancel, e.g. the first-layer decoder weights), at most 1 of
# the 32 first-layer biases.
SLACK_SHARE = 0.02
SLACK_MIN = 2


def check_grad(name, got, ref, exclude, delta, rtol=RTOL, floor=FLOOR, report=None):
    """Every element: |got - ref| <= rtol * max(|ref|, floor * max|ref|) + slack,
    where delta is a dict {"sens": d, "round": e, "frag": f}: d is how far
    the FP64 oracle's own gradient moves when every float input is perturbed
    at float32 rounding size (the element's conditioning), e its response to
    rounding-size errors of the per-splat gradient sums (rounding_sensitivity)
    and f the share of the element that comes from pixels with a near tie
    (zero when their output gradients are zero); slack = SENS_K d + ROUND_K e
    + 2 f.  The slack may carry
    at most SLACK_SHARE of the gradient-bearing elements (those beyond the
    plain relative bound), and the norm-wise relative error over all of them
    must stay <= GRAD_NORM_RTOL."""
    if isinstance(delta, dict):
        frag = np.asarray(delta.get("frag", 0.0), np.float64)
        delta = (SENS_K * np.asarray(delta["sens"], np.float64) + 2.0 * frag
                 + ROUND_K * np.asarray(delta.get("round", 0.0), np.float64))
    else:
        delta = SENS_K * np.asarray(delta, np.float64)
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    d = np.broadcast_to(np.asarray(delta, np.float64).ravel(), ref.shape)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    ex = np.zeros(ref.shape, bool) if exclude is None else np.asarray(exclude, bool).ravel()
    keep = ~ex
    scale = np.max(np.abs(ref[keep])) if keep.any() else 0.0
    plain = rtol * np.maximum(np.abs(ref), floor * scale)
    tol = plain + d
    err = np.abs(got - ref)
    bad = (err > tol) & keep
    assert np.all(np.isfinite(got[keep])), f"{name}: non-finite values"
    rel = np.max(err[keep] / np.maximum(np.abs(ref[keep]), floor * scale + 1e-300)) if keep.any() else 0.0
    bearing = keep & ((ref != 0) | (got != 0))
    nrm = np.linalg.norm(ref[bearing])
    nrel = (float(np.linalg.norm((got - ref)[bearing]) / nrm) if nrm > 0
            else float(np.linalg.norm(got[bearing])))
    beyond = bearing & (err > plain)
    n_b, n_bear = int(beyond.sum()), int(bearing.sum())
    print(f"  {name}: max floored rel err {rel:.2e}, norm rel err {nrel:.2e}, gradient-bearing "
          f"{n_bear}/{ref.size}, beyond the plain bound {n_b} (within their conditioning slack)",
          flush=True)
    if report is not None:
        report[name] = dict(max_rel=float(rel), norm_rel=nrel, excluded=int(ex.sum()),
                            beyond=n_b, bearing=n_bear, n=int(ref.size))
    dump = os.environ.get("CGX_PARITY_DUMP")
    if dump:
        # diagnostic mode: keep the compared arrays
        test = os.environ.get("PYTEST_CURRENT_TEST", "run").split(" ")[0]
        tag = re.sub(r"[^A-Za-z0-9_.-]+", "_", test)
        os.makedirs(dump, exist_ok=True)
        np.savez_compressed(os.path.join(dump, f"{tag}__{name}.npz"), got=got, ref=ref, d=d,
                            keep=keep)
    if bad.any():
        i = np.argmax(np.where(bad, err / np.maximum(tol, 1e-300), 0))
        raise AssertionError(f"{name}: {int(bad.sum())}/{keep.sum()} elements out of tolerance; "
                             f"worst idx {i}: got {got[i]!r} ref {ref[i]!r} tol {tol[i]:.3g} "
                             f"delta {d[i]:.3g}")
    assert n_b <= max(SLACK_MIN, SLACK_SHARE * n_bear), (
        f"{name}: {n_b}/{n_bear} gradient-bearing elements need the conditioning slack")
    assert nrel <= GRAD_NORM_RTOL, f"{name}: norm-wise relative error {nrel:.3g}"
    return rel


def targets_at_ties(out, r, targets):
    """L1 targets whose near-tie pixels hold the GPU's own outputs: the
    pixels of frag_grad, and those where a target lies within the L1 sign's
    near-tie bound of the oracle's output.  The GPU's fused L1 seed is then
    exactly zero there (sign(0) = 0), as the linear-loss tests zero those
    pixels' output gradients; the pixels join frag_grad, so zero_ties zeroes
    the oracle's seed at the same pixels."""
    from oracle.raster import FRAG_SIGN
    pix_off = r.layout["pix_off"]
    new = {k: [np.array(t, np.float32, copy=True) for t in targets[k]] for k in targets}
    for v, img in enumerate(r.images):
        HW = img["depth"].size
        near = np.zeros(HW, bool)
        with np.errstate(invalid="ignore"):
            near |= (np.abs(img["rgb"] - np.asarray(targets["rgb"][v], np.float64).reshape(3, HW))
                     < FRAG_SIGN).any(axis=0)
            near |= (np.abs(img["normal"] - np.asarray(targets["normal"][v], np.float64).reshape(3, HW))
                     < FRAG_SIGN).any(axis=0)
            near |= np.abs(img["depth"] - np.asarray(targets["depth"][v], np.float64).ravel()) < FRAG_SIGN
        img["frag_grad"] = img["frag_grad"] | near
        m = img["frag_grad"]
        for key, c in (("rgb", 3), ("depth", 1), ("normal", 3)):
            if key not in new:
                continue
            g = _np(out[key]).astype(np.float32).ravel()
            base = c * int(pix_off[v])
            vals = g[base:base + c * HW].reshape(c, HW)
            t = new[key][v]
            shape = t.shape
            t = t.reshape(c, HW)
            t[:, m] = vals[:, m]
            new[key][v] = t.reshape(shape)
    return new


def zero_ties(r, og):
    """Output gradients with the pixels of near-tie decisions zeroed: the
    linear loss of a gradient test then has no term whose gradient depends on
    a tie's outcome."""
    out = []
    for img, g in zip(r.images, og):
        m = img["frag_grad"]
        h = {}
        for k, a in g.items():
            a = np.array(a, np.float64, copy=True)
            if a.ndim == 2:
                a[:, m] = 0.0
            else:
                a[m] = 0.0
            h[k] = a
        out.append(h)
    return out


def tie_fraction(r):
    """Share of the composited pixels whose output gradients a tie zeroes."""
    n = sum(int(img["covered"].sum()) for img in r.images)
    t = sum(int((img["frag_grad"] & img["covered"]).sum()) for img in r.images)
    return t / max(n, 1)


# kept for the older name used by the full-size tests
_without_fragile = zero_ties


def linear_grads(r, rng, covered_only=False):
    """Linear-loss output gradients w ~ N(0, 1) on every output, zero at the
    pixels with a near tie (and, with covered_only, outside the composited
    tiles)."""
    out = []
    for img in r.images:
        npx = img["depth"].size
        m = img["covered"] if covered_only else np.ones(npx, bool)
        g = dict(rgb=rng.standard_normal((3, npx)) * m, depth=rng.standard_normal(npx) * m,
                 D=rng.standard_normal(npx) * m, normal=rng.standard_normal((3, npx)) * m,
                 alpha=rng.standard_normal(npx) * m)
        out.append(g)
    return zero_ties(r, out)


def packed_grads(og, device="cuda"):
    """Per-view oracle output gradients packed like the library's images."""
    import torch
    d = {}
    for key, okey in (("rgb", "rgb"), ("depth", "depth"), ("plane_d", "D"), ("normal", "normal"),
                      ("alpha", "alpha")):
        d[key] = torch.as_tensor(np.concatenate([g[okey].ravel() for g in og]).astype(np.float32),
                                 device=device)
    return d


def _perturbed(a, rng):
    a = np.asarray(a)
    if a.dtype.kind != "f":
        return a
    return (a.astype(np.float64) * (1.0 + SENS_EPS * rng.standard_normal(a.shape)))


EXPLICIT_KEYS = ("means", "scales", "quats", "opacity", "sh")
ANCHOR_KEYS = ("x", "l", "O", "F", "W1", "b1", "W2", "b2")


def rounding_sensitivity(r, og, scene, keys, seeds=(4321, 8765), g0=None):
    """Response of the oracle's scene gradient to rounding-size errors in the
    per-splat gradients: each per-splat element moves by SENS_EPS times its
    rounding scale (the sum of |terms| it is formed from, cancelling
    differences included; oracle.raster.composite_backward(magnitude=True))
    with a random sign, and the projection / decoder adjoint carries that
    to the scene gradient.  Models the float32 error of the sums the GPU's
    backward raster forms, which input perturbations do not reach when a
    pixel's alpha adjoint cancels large terms."""
    from oracle import pipeline
    from oracle import raster as ras
    M = ras.composite_backward(r.splats, r.views, r.images, og, r.varr, magnitude=True)
    if g0 is None:
        g0, _ = pipeline.backward(r, og, scene)
    sens = None
    for seed in seeds:
        rng = np.random.default_rng(seed + 17)

        def hook(sg):
            out = []
            for d, m in zip(sg, M):
                e = dict(d)
                for k, a in d.items():
                    if k in m and k != "frag":
                        e[k] = a + SENS_EPS * np.asarray(m[k]) * rng.standard_normal(np.shape(a))
                out.append(e)
            return out

        g1, _ = pipeline.backward(r, og, scene, sg_hook=hook)
        d = {k: np.abs(g0[k] - g1[k]) for k in keys}
        sens = d if sens is None else {k: np.maximum(sens[k], d[k]) for k in d}
    return sens


def explicit_sensitivity(scene, views, og, tile=(16, 16), seeds=(4321, 8765), keep_tiles=None,
                         r0=None):
    """Per gradient element: the larger response of the oracle's gradient to
    two independent float32-size perturbations of every float input (one
    draw can miss an element's worst direction), and the share of the
    element from pixels with a near tie."""
    import copy

    from oracle import pipeline
    r0 = r0 or pipeline.render_explicit(scene, views, tile=tile, keep_tiles=keep_tiles)
    g0, _ = pipeline.backward(r0, og, scene)
    sens = None
    for seed in seeds:
        rng = np.random.default_rng(seed)
        sc = copy.copy(scene)
        for k in EXPLICIT_KEYS:
            setattr(sc, k, _perturbed(getattr(scene, k), rng))
        r1 = pipeline.render_explicit(sc, views, tile=tile, keep_tiles=keep_tiles)
        g1, _ = pipeline.backward(r1, og, sc)
        d = {k: np.abs(g0[k] - g1[k]) for k in EXPLICIT_KEYS}
        sens = d if sens is None else {k: np.maximum(sens[k], d[k]) for k in d}
    sr = rounding_sensitivity(r0, og, scene, EXPLICIT_KEYS, seeds, g0=g0)
    g2, _ = pipeline.backward(r0, zero_ties(r0, og), scene)
    return {k: dict(sens=sens[k], round=sr[k], frag=np.abs(g0[k] - g2[k])) for k in EXPLICIT_KEYS}


def anchor_sensitivity(scene, views, og, tile=(16, 16), seeds=(4321, 8765), keep_tiles=None,
                       r0=None):
    """Same for anchor scenes (features, offsets, positions, scalings,
    biases and the decoder weights' values)."""
    import copy

    from oracle import pipeline
    r0 = r0 or pipeline.render_anchor(scene, views, tile=tile, keep_tiles=keep_tiles)
    g0, _ = pipeline.backward(r0, og, scene)
    sens = None
    for seed in seeds:
        rng = np.random.default_rng(seed)
        sc = copy.copy(scene)
        for k in ("x", "l", "O", "b1", "b2"):
            setattr(sc, k, _perturbed(getattr(scene, k), rng))
        sc.W1_exact = _perturbed(scene.W1, rng)
        sc.W2_exact = _perturbed(scene.W2, rng)
        r1 = pipeline.render_anchor(sc, views, tile=tile, keep_tiles=keep_tiles)
        g1, _ = pipeline.backward(r1, og, sc)
        d = {k: np.abs(g0[k] - g1[k]) for k in ANCHOR_KEYS}
        sens = d if sens is None else {k: np.maximum(sens[k], d[k]) for k in d}
    sr = rounding_sensitivity(r0, og, scene, ANCHOR_KEYS, seeds, g0=g0)
    g2, _ = pipeline.backward(r0, zero_ties(r0, og), scene)
    return {k: dict(sens=sens[k], round=sr[k], frag=np.abs(g0[k] - g2[k])) for k in ANCHOR_KEYS}


def oracle_images_packed(r, key, channels):
    """Oracle per-view images packed like the library's planar layout."""
    parts = []
    for img in r.images:
        a = img[key]
        parts.append(a.reshape(channels, -1).ravel() if channels > 1 else a.ravel())
    return np.concatenate(parts)
