"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare with the FP64 oracle on the same seeded inputs."""
import numpy as np

RTOL = 1e-4          # images and gradients, relative (fp32 GPU vs fp64 oracle)
# Relative floor: the tolerance never falls below RTOL * FLOOR * max|ref| of
# the tensor.  Signed channels (normal x/y, gradients) are sums whose float32
# error scales with the sum of |terms|, not with the net value, so elements
# that cancel to a small fraction of the tensor's range get this slack.
FLOOR = 1e-2
NORM_RTOL = 1e-5     # norm-wise relative error over the compared elements


def check_close(name, got, ref, exclude=None, rtol=RTOL, floor=FLOOR, report=None, mag=None):
    """Element-wise |got - ref| <= rtol * max(m, floor * max|ref|) on every
    element not excluded (excluded = touched by a fragile decision), where m
    is |ref| or, for a blended signed quantity, the blend of |terms| (mag)."""
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
    nrm = np.linalg.norm(ref[keep])
    nrel = float(np.linalg.norm((got - ref)[keep]) / nrm) if nrm > 0 else float(np.linalg.norm(got[keep]))
    if report is not None:
        report[name] = dict(max_rel=float(rel), norm_rel=nrel, excluded=int(ex.sum()), n=int(ref.size))
    print(f"  {name}: max floored rel err {rel:.2e}, norm rel err {nrel:.2e}, "
          f"excluded {int(ex.sum())}/{ref.size}", flush=True)
    if bad.any():
        i = np.argmax(np.where(bad, err / np.maximum(tol, 1e-300), 0))
        raise AssertionError(f"{name}: {int(bad.sum())}/{keep.sum()} elements out of tolerance; "
                             f"worst idx {i}: got {got[i]!r} ref {ref[i]!r} tol {tol[i]:.3g}")
    assert nrel <= NORM_RTOL, f"{name}: norm-wise relative error {nrel:.3g} > {NORM_RTOL}"
    return rel


def oracle_images_packed(r, key, channels):
    """Oracle per-view images packed like the library's planar layout."""
    parts = []
    for img in r.images:
        a = img[key]
        parts.append(a.reshape(channels, -1).ravel() if channels > 1 else a.ravel())
    return np.concatenate(parts)


def oracle_mask_packed(r, key, channels):
    parts = []
    for img in r.images:
        m = img[key]
        parts.append(np.tile(m, channels) if channels > 1 else m)
    return np.concatenate(parts)


def compare_images(out, r, report=None):
    """out: dict of packed GPU images (torch or numpy); r: oracle result."""
    chans = dict(rgb=("rgb", 3), depth=("depth", 1), plane_d=("D", 1), normal=("normal", 3),
                 alpha=("alpha", 1))
    for k, (ok, c) in chans.items():
        g = out[k].detach().cpu().numpy() if hasattr(out[k], "detach") else out[k]
        mag = oracle_images_packed(r, "normal_abs", 3) if k == "normal" else None
        check_close(k, g, oracle_images_packed(r, ok, c), image_fragile(r, k, c),
                    report=report, mag=mag)


GEOMETRIC = ("normal", "plane_d", "depth")


def image_fragile(r, key, channels):
    """Packed mask of pixels with a fragile decision for output `key`: the
    geometric outputs also exclude pixels whose splat normal is fragile."""
    m = oracle_mask_packed(r, "frag", channels)
    if key in GEOMETRIC:
        m = m | oracle_mask_packed(r, "frag_geom", channels)
    return m


def compare_sort_explicit(dbg, r, N):
    """Sorted pairs: bit-exact against the oracle's (tile, depth bits, view,
    id) order, after dropping the pairs of splats with a fragile tile set."""
    slot = dbg["slot"].astype(np.int64)
    g_view, g_id = slot // N, slot % N
    frag = np.zeros((len(r.splats), N), bool)
    for v, S in enumerate(r.splats):
        frag[v] = S["frag_value"]
    keep_g = ~frag[g_view, g_id]
    o = r.sorted
    keep_o = ~frag[o["view"], o["gid"]]
    got = np.stack([dbg["tile"].astype(np.int64)[keep_g], dbg["zbits"].astype(np.int64)[keep_g],
                    g_view[keep_g], g_id[keep_g]], 1)
    ref = np.stack([o["gtile"][keep_o], o["zbits"].astype(np.int64)[keep_o], o["view"][keep_o],
                    o["gid"][keep_o]], 1)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    np.testing.assert_array_equal(got, ref)
    if not frag.any():
        np.testing.assert_array_equal(dbg["ranges"].astype(np.int64), o["ranges"])
    return int((~keep_g).sum())


def compare_sort_anchor(dbg, r, n_off):
    """Anchor path: rows bit-exact; sorted pairs bit-exact after mapping each
    slot (row * n + k) to its view-local id (row - first row of the view) * n + k
    and dropping the pairs of splats with a fragile tile set."""
    rows = dbg["rows"].astype(np.int64)
    np.testing.assert_array_equal(rows, r.rows)
    slot = dbg["slot"].astype(np.int64)
    row, k = slot // n_off, slot % n_off
    view = rows[row, 0]
    gid = (row - r.row_off[view]) * n_off + k
    frag = [S["frag_value"] for S in r.splats]
    keep_g = np.array([not frag[v][g] for v, g in zip(view, gid)], bool)
    o = r.sorted
    keep_o = np.array([not frag[v][g] for v, g in zip(o["view"], o["gid"])], bool)
    got = np.stack([dbg["tile"].astype(np.int64)[keep_g], dbg["zbits"].astype(np.int64)[keep_g],
                    view[keep_g], gid[keep_g]], 1)
    ref = np.stack([o["gtile"][keep_o], o["zbits"].astype(np.int64)[keep_o], o["view"][keep_o],
                    o["gid"][keep_o]], 1)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    np.testing.assert_array_equal(got, ref)
    return int((~keep_g).sum())


# ---------------------------------------------------------------------------
# gradients: 1e-4 relative where the element is well conditioned
# ---------------------------------------------------------------------------
SENS_EPS = 2.0 ** -24      # relative input perturbation of float32 rounding size
SENS_K = 16.0              # float32 rounding events the GPU chain may accumulate per input one
GRAD_NORM_RTOL = 1e-4


def check_grad(name, got, ref, exclude, delta, rtol=RTOL, floor=FLOOR, report=None):
    """|got - ref| <= rtol * max(|ref|, floor * max|ref|) + slack, where delta
    is a dict {"sens": d, "frag": f}: d is how far the FP64 oracle's own
    gradient moves when every float input is perturbed at float32 rounding
    size (the element's conditioning) and f is the share of the element that
    comes from pixels with a fragile decision; slack = SENS_K d + 2 f.  The
    norm-wise relative error must also stay <= GRAD_NORM_RTOL."""
    if isinstance(delta, dict):
        delta = SENS_K * np.asarray(delta["sens"], np.float64) + 2.0 * np.asarray(delta["frag"], np.float64)
    else:
        delta = SENS_K * np.asarray(delta, np.float64)
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    d = np.asarray(delta, np.float64).ravel()
    assert got.shape == ref.shape == d.shape, (name, got.shape, ref.shape, d.shape)
    ex = np.zeros(ref.shape, bool) if exclude is None else np.asarray(exclude, bool).ravel()
    keep = ~ex
    scale = np.max(np.abs(ref[keep])) if keep.any() else 0.0
    tol = rtol * np.maximum(np.abs(ref), floor * scale) + d
    err = np.abs(got - ref)
    bad = (err > tol) & keep
    assert np.all(np.isfinite(got[keep])), f"{name}: non-finite values"
    rel = np.max(err[keep] / np.maximum(np.abs(ref[keep]), floor * scale + 1e-300)) if keep.any() else 0.0
    # norm-wise error over the elements whose conditioning allows 1e-4
    wc = keep & (d <= rtol * np.maximum(np.abs(ref), floor * scale))
    nrm = np.linalg.norm(ref[wc])
    nrel = float(np.linalg.norm((got - ref)[wc]) / nrm) if nrm > 0 else float(np.linalg.norm(got[wc]))
    cond = int((keep & ~wc).sum())
    print(f"  {name}: max floored rel err {rel:.2e}, norm rel err {nrel:.2e}, excluded "
          f"{int(ex.sum())}/{ref.size}, ill-conditioned {cond}", flush=True)
    if bad.any():
        i = np.argmax(np.where(bad, err / np.maximum(tol, 1e-300), 0))
        raise AssertionError(f"{name}: {int(bad.sum())}/{keep.sum()} elements out of tolerance; "
                             f"worst idx {i}: got {got[i]!r} ref {ref[i]!r} tol {tol[i]:.3g} "
                             f"delta {d[i]:.3g}")
    assert nrel <= GRAD_NORM_RTOL, f"{name}: norm-wise relative error {nrel:.3g}"
    return rel


def _without_fragile(r, og):
    """Output gradients with the pixels of fragile decisions zeroed."""
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


def _perturbed(a, rng):
    a = np.asarray(a)
    if a.dtype.kind != "f":
        return a
    return (a.astype(np.float64) * (1.0 + SENS_EPS * rng.standard_normal(a.shape)))


def explicit_sensitivity(scene, views, og, tile=(16, 16), seed=4321):
    """|g(inputs) - g(inputs perturbed at float32 rounding size)| of the
    oracle, per gradient element (explicit scenes)."""
    import copy

    from oracle import pipeline
    rng = np.random.default_rng(seed)
    r0 = pipeline.render_explicit(scene, views, tile=tile)
    g0, _ = pipeline.backward(r0, og, scene)
    sc = copy.copy(scene)
    for k in ("means", "scales", "quats", "opacity", "sh"):
        setattr(sc, k, _perturbed(getattr(scene, k), rng))
    r1 = pipeline.render_explicit(sc, views, tile=tile)
    g1, _ = pipeline.backward(r1, og, sc)
    g2, _ = pipeline.backward(r0, _without_fragile(r0, og), scene)
    return {k: dict(sens=np.abs(g0[k] - g1[k]), frag=np.abs(g0[k] - g2[k]))
            for k in ("means", "scales", "quats", "opacity", "sh")}


def anchor_sensitivity(scene, views, og, tile=(16, 16), seed=4321):
    """Same for anchor scenes (features, offsets, positions, scalings,
    biases and the decoder weights' values)."""
    import copy

    from oracle import pipeline
    rng = np.random.default_rng(seed)
    r0 = pipeline.render_anchor(scene, views, tile=tile)
    g0, _ = pipeline.backward(r0, og, scene)
    sc = copy.copy(scene)
    for k in ("x", "l", "O", "b1", "b2"):
        setattr(sc, k, _perturbed(getattr(scene, k), rng))
    sc.W1_exact = _perturbed(scene.W1, rng)
    sc.W2_exact = _perturbed(scene.W2, rng)
    r1 = pipeline.render_anchor(sc, views, tile=tile)
    g1, _ = pipeline.backward(r1, og, sc)
    g2, _ = pipeline.backward(r0, _without_fragile(r0, og), scene)
    return {k: dict(sens=np.abs(g0[k] - g1[k]), frag=np.abs(g0[k] - g2[k]))
            for k in ("x", "l", "O", "F", "W1", "b1", "W2", "b2")}
