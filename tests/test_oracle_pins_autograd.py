"""An independent pin of the oracle's analytic adjoint: a brute-force
renderer written here in torch.float64 on the CPU and differentiated by
torch.autograd.

It shares no code with the oracle.  Every pixel takes every splat whose
pixel box holds it, in (float32 depth, id) order, with the compositing
rules of Eqs. 1 and 5 (alpha = min(0.99, o exp(power)), skip alpha < 1/255,
stop before T falls below 1e-4), the normal and plane distance of Eq. 6 and
the unbiased depth of Eq. 7; anchors are decoded by the MLP of Eq. 4 first.
There are no tiles, no sorted pair lists and no reverse walk: the gradient
is autograd's.  On tiny scenes whose discrete decisions are clear of their
bounds (no near tie), the oracle's gradient must equal autograd's to 1e-8.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import pipeline
from oracle import raster as ras
from synth import scenes

f64 = torch.float64


@pytest.fixture(autouse=True)
def _exact_means(monkeypatch):
    """Both sides composite with the exact 2-D mean here."""
    monkeypatch.setattr(ras, "MEAN_F32", False)


def _view(v):
    R = torch.tensor(np.asarray(v.R, np.float32).reshape(3, 3).astype(np.float64), dtype=f64)
    t = torch.tensor(np.asarray(v.t, np.float32).astype(np.float64), dtype=f64)
    g = lambda a: float(np.float32(a))   # noqa: E731
    return dict(R=R, t=t, W=int(v.width), H=int(v.height), fx=g(v.fx), fy=g(v.fy), cx=g(v.cx),
                cy=g(v.cy), zn=g(v.z_near), bg=torch.tensor(np.asarray(v.bg, np.float32), dtype=f64))


def _rotation(q):
    qn = q / q.norm(dim=1, keepdim=True).clamp_min(1e-12)
    w, x, y, z = qn.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)


def _sh(dirs, k, degree):
    """Real orthonormal SH of degree <= 1 (no Condon-Shortley phase, index
    l^2 + l + m): Y00 = 1 / (2 sqrt(pi)), (Y1-1, Y10, Y11) = sqrt(3 / (4 pi))
    (y, z, x)."""
    terms = [torch.full_like(dirs[:, 0], 0.5 / math.sqrt(math.pi))]
    if degree >= 1:
        c = math.sqrt(3.0 / (4.0 * math.pi))
        terms += [c * dirs[:, 1], c * dirs[:, 2], c * dirs[:, 0]]
    Y = torch.stack(terms, 1)
    return torch.einsum("nk,nkc->nc", Y, k[:, :Y.shape[1]])


def render_view(mu, s, q, o, colour, V):
    """Brute-force RGB, D, N, alpha and unbiased depth of one view."""
    R, t = V["R"], V["t"]
    p = mu @ R.T + t
    pz = p[:, 2]
    front = (pz > V["zn"]).detach()
    pzs = torch.where(front, pz, torch.ones_like(pz))
    u = V["fx"] * p[:, 0] / pzs + V["cx"]
    w = V["fy"] * p[:, 1] / pzs + V["cy"]
    lx, ly = 1.3 * V["W"] / (2 * V["fx"]), 1.3 * V["H"] / (2 * V["fy"])
    tx = torch.clamp(p[:, 0] / pzs, -lx, lx) * pzs
    ty = torch.clamp(p[:, 1] / pzs, -ly, ly) * pzs
    J0 = (V["fx"] / pzs)[:, None] * R[0][None] - (V["fx"] * tx / pzs ** 2)[:, None] * R[2][None]
    J1 = (V["fy"] / pzs)[:, None] * R[1][None] - (V["fy"] * ty / pzs ** 2)[:, None] * R[2][None]
    Rq = _rotation(q)
    M = Rq * s[:, None, :]
    a0 = torch.einsum("nj,njk->nk", J0, M)
    a1 = torch.einsum("nj,njk->nk", J1, M)
    A = (a0 * a0).sum(1) + 0.3
    B = (a0 * a1).sum(1)
    C = (a1 * a1).sum(1) + 0.3
    det = A * C - B * B
    with torch.no_grad():
        lam = 0.5 * (A + C) + torch.sqrt((0.5 * (A - C)) ** 2 + B * B)
        r = torch.ceil(3 * torch.sqrt(lam))
        tau = torch.log(255.0 * o)
        ok = front & (det > 0) & (tau >= 0)
        tau0 = tau.clamp_min(0)
        rx = torch.minimum(r, torch.sqrt(2 * tau0 * A))
        ry = torch.minimum(r, torch.sqrt(2 * tau0 * C))
        x0 = torch.ceil(u - (rx + 0.5)).clamp(0, V["W"])
        x1 = torch.floor(u + (rx - 0.5)).clamp(-1, V["W"] - 1)
        y0 = torch.ceil(w - (ry + 0.5)).clamp(0, V["H"])
        y1 = torch.floor(w + (ry - 0.5)).clamp(-1, V["H"] - 1)
        valid = ok & (x0 <= x1) & (y0 <= y1)
        zkey = pz.detach().to(torch.float32)
    # normal: rotated axis of the smallest scale, in the camera frame, facing
    # the camera; plane distance d = -n . p
    j = torch.argmin(s.detach(), 1)
    n = torch.einsum("ij,njk->nik", R, Rq)[torch.arange(mu.shape[0]), :, j]
    flip = ((n * p).sum(1) > 0).detach()
    n = torch.where(flip[:, None], -n, n)
    d = -(n * p).sum(1)
    # every splat in (float32 depth, id) order
    order = sorted(range(mu.shape[0]), key=lambda i: (float(zkey[i]), i))
    order = torch.tensor(order, dtype=torch.long)
    I, Jp = torch.meshgrid(torch.arange(V["W"], dtype=f64), torch.arange(V["H"], dtype=f64),
                           indexing="xy")
    I, Jp = I.reshape(-1), Jp.reshape(-1)
    ca, cb, cc = (C / det)[order], (-B / det)[order], (A / det)[order]
    dx = u[order][None] - (I[:, None] + 0.5)
    dy = w[order][None] - (Jp[:, None] + 0.5)
    power = -0.5 * (ca[None] * dx * dx + cc[None] * dy * dy) - cb[None] * dx * dy
    raw = o[order][None] * torch.exp(power)
    alpha = torch.clamp(raw, max=0.99)
    with torch.no_grad():
        box = ((I[:, None] >= x0[order][None]) & (I[:, None] <= x1[order][None])
               & (Jp[:, None] >= y0[order][None]) & (Jp[:, None] <= y1[order][None]))
        use = box & valid[order][None] & (power <= 0) & (alpha >= 1.0 / 255.0)
        a_use = torch.where(use, alpha, torch.zeros_like(alpha))
        Tn = torch.cumprod(1 - a_use, 1)
        crossed = use & (Tn < 1e-4)
        first = torch.where(crossed.any(1), crossed.float().argmax(1), torch.full_like(I, alpha.shape[1]).long())
        inc = use & (torch.arange(alpha.shape[1])[None] < first[:, None])
    a_inc = torch.where(inc, alpha, torch.zeros_like(alpha))
    Tafter = torch.cumprod(1 - a_inc, 1)
    Tbefore = torch.cat([torch.ones_like(Tafter[:, :1]), Tafter[:, :-1]], 1)
    wgt = a_inc * Tbefore
    T = Tafter[:, -1]
    rgb = wgt @ colour[order] + T[:, None] * V["bg"][None]
    D = wgt @ d[order]
    N = wgt @ n[order]
    acc = 1 - T
    ray = torch.stack([(I + 0.5 - V["cx"]) / V["fx"], (Jp + 0.5 - V["cy"]) / V["fy"],
                       torch.ones_like(I)], 1)
    sd = -(N * ray).sum(1)
    keep = (sd > 1e-3 * acc).detach()
    dhat = torch.where(keep, D / torch.where(keep, sd, torch.ones_like(sd)), torch.zeros_like(sd))
    return dict(rgb=rgb.T, D=D, normal=N.T, alpha=acc, depth=dhat)


def _loss(imgs, og):
    L = 0.0
    for img, g in zip(imgs, og):
        for k, ok in (("rgb", "rgb"), ("depth", "depth"), ("D", "D"), ("normal", "normal"),
                      ("alpha", "alpha")):
            L = L + (img[k] * torch.tensor(g[ok], dtype=f64)).sum()
    return L


def _explicit_scene(seed, sh_degree):
    wl = scenes.make_small_explicit(seed, n=14, width=30, height=26, sh_degree=sh_degree,
                                    spread=0.45, log_scale=-2.0)
    sc = wl.scene
    for k in ("means", "scales", "quats", "opacity", "sh"):
        setattr(sc, k, np.asarray(getattr(sc, k), np.float64).copy())
    v = wl.views[0]
    v.R = Rotation.from_euler("xyz", [0.2, -0.3, 0.1]).as_matrix().astype(np.float32)
    v.t = np.array([0.05, -0.02, 2.5], np.float32)
    return sc, wl.views


def _close(name, got, want):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    scale = np.max(np.abs(want)) + 1e-300
    err = np.max(np.abs(got - want)) / scale
    assert err <= 1e-8, (name, err)
    return err


def _no_ties(r):
    for img in r.images:
        assert not img["tie"].any() and not img["frag_grad"].any()


@pytest.mark.parametrize("seed,sh_degree", [(31, 0), (32, 1), (33, 1)])
def test_explicit_adjoint_equals_autograd(seed, sh_degree):
    sc, views = _explicit_scene(seed, sh_degree)
    r = pipeline.render_explicit(sc, views)
    _no_ties(r)
    L, og = pipeline.output_grads_linear(r, np.random.default_rng(seed))
    ref, _ = pipeline.backward(r, og, sc)
    leaves = [torch.tensor(np.asarray(getattr(sc, k), np.float64), requires_grad=True)
              for k in ("means", "scales", "quats", "opacity", "sh")]
    mu, s, q, o, k = leaves
    imgs = []
    for view in views:
        V = _view(view)
        dirs = mu - (-(V["R"].T @ V["t"]))[None]
        dirs = dirs / dirs.norm(dim=1, keepdim=True)
        colour = torch.clamp_min(_sh(dirs, k, sh_degree) + 0.5, 0.0)
        imgs.append(render_view(mu, s, q, o, colour, V))
    # the two forward passes agree
    for a, b in zip(imgs, r.images):
        for key in ("rgb", "D", "normal", "alpha", "depth"):
            _close(key, a[key].detach().numpy(), b[key])
    grads = torch.autograd.grad(_loss(imgs, og), leaves)
    n_nonzero = 0
    for name, g in zip(("means", "scales", "quats", "opacity", "sh"), grads):
        _close("d_" + name, ref[name], g.numpy())
        n_nonzero += int((np.abs(ref[name]) > 0).sum())
    assert n_nonzero > 100


def _select(scene, views):
    """Active (view, anchor) rows: level 0, or distance^2 * 4^level <= d_max^2
    (the level of detail by observation distance), and the anchor centre in
    front of the camera within 1.3 times the half field of view."""
    x = torch.tensor(np.asarray(scene.x, np.float64), dtype=f64)
    level = torch.tensor(np.asarray(scene.level).astype(np.int64))
    dmax = float(np.float32(scene.d_max))
    rows = []
    for v, view in enumerate(views):
        V = _view(view)
        c = -(V["R"].T @ V["t"])
        d2 = ((c[None] - x) ** 2).sum(1)
        lod = (level == 0) | (d2 * (4.0 ** level.to(f64)) <= dmax * dmax)
        p = x @ V["R"].T + V["t"]
        gx, gy = 1.3 * V["W"] / (2 * V["fx"]), 1.3 * V["H"] / (2 * V["fy"])
        inside = (p[:, 2] > V["zn"]) & (p[:, 0].abs() <= gx * p[:, 2]) & (p[:, 1].abs() <= gy * p[:, 2])
        a = torch.nonzero(lod & inside)[:, 0].numpy()
        rows.append(np.stack([np.full(a.size, v), a], 1))
    return np.concatenate(rows).astype(np.int64)


def _decode(scene, views, rows, x, l, O, F, W1, b1, W2, b2, act, offsets=0, heads=1):
    """Eq. 4 per active (view, anchor) row: z0 = [bf16(F), direction to the
    camera, distance / d_max] -> 32 (ReLU) -> 11 per Gaussian (opacity, rgb,
    scale, quaternion); mu = x + O * l.  offsets = 1: 3 more outputs per
    Gaussian are its offset O.  heads = 3: one such MLP per attribute group
    (opacity, colour, scale + quaternion, offsets), each with 32 hidden
    units of W1 and a block of n * width columns of W2."""
    a = torch.tensor(rows[:, 1], dtype=torch.long)
    cams = torch.stack([-(_view(v)["R"].T @ _view(v)["t"]) for v in views])
    delta = cams[torch.tensor(rows[:, 0], dtype=torch.long)] - x[a]
    dist = delta.norm(dim=1)
    dmax = float(np.float32(scene.d_max))
    # F rounded to bfloat16, the rounding passed straight through
    Fa = F[a]
    Fb = Fa + (Fa.detach().to(torch.float32).to(torch.bfloat16).to(f64) - Fa.detach())
    z0 = torch.cat([Fb, delta / dist[:, None], (dist / dmax)[:, None]], 1)
    n = O.shape[1]
    go = 14 if offsets else 11
    if heads == 1:
        g = (torch.relu(z0 @ W1 + b1) @ W2 + b2).reshape(-1, n, go)
    else:
        widths = [1, 3, 7] + ([3] if offsets else [])
        parts, c0 = [], 0
        for h, w in enumerate(widths):
            z1 = torch.relu(z0 @ W1[:, 32 * h:32 * h + 32] + b1[32 * h:32 * h + 32])
            y = z1 @ W2[:, c0:c0 + n * w] + b2[c0:c0 + n * w]
            parts.append(y.reshape(-1, n, w))
            c0 += n * w
        g = torch.cat(parts, 2)
    op = torch.tanh(g[..., 0]) if act == 1 else torch.sigmoid(g[..., 0])
    rgb = torch.sigmoid(g[..., 1:4])
    s = l[a][:, None, :] * torch.sigmoid(g[..., 4:7])
    off = g[..., 11:14] if offsets else O[a]
    mu = x[a][:, None, :] + off * l[a][:, None, :]
    return mu, s, g[..., 7:11], op, rgb


@pytest.mark.parametrize("seed,act,offsets,heads", [(46, 0, 0, 1), (50, 0, 0, 1), (41, 1, 0, 1),
                                                   (54, 1, 0, 1), (53, 0, 1, 1), (55, 0, 0, 3),
                                                   (58, 1, 1, 3)])
def test_anchor_adjoint_equals_autograd(seed, act, offsets, heads):
    wl = scenes.make_small_anchor(seed, n_anchor=16, opacity_act=act, offset_mode=offsets,
                                  decoder_heads=heads)
    sc = wl.scene
    r = pipeline.render_anchor(sc, wl.views)
    if offsets:
        # a decoded mean carries the decoder's float32 error on the GPU, which
        # widens every near-tie band; none of them matters between two
        # float64 evaluations, but the pixels flagged are left out of the
        # loss all the same
        assert sum(int(i["frag_grad"].sum()) for i in r.images) <= 0.01 * sum(
            i["alpha"].size for i in r.images)
    else:
        _no_ties(r)
    assert r.rows.shape[0] >= 8
    L, og = pipeline.output_grads_linear(r, np.random.default_rng(5))
    for img, g in zip(r.images, og):
        for k in g:
            g[k][..., img["frag_grad"]] = 0.0
    ref, _ = pipeline.backward(r, og, sc)
    names = ("x", "l", "O", "F", "W1", "b1", "W2", "b2")
    arrs = [sc.x, sc.l, sc.O, sc.F, sc.W1, sc.b1, sc.W2, sc.b2]
    leaves = [torch.tensor(np.asarray(a, np.float64), requires_grad=True) for a in arrs]
    x, l, O, F, W1, b1, W2, b2 = leaves
    all_rows = _select(sc, wl.views)
    np.testing.assert_array_equal(all_rows, r.rows)
    imgs = []
    for v, view in enumerate(wl.views):
        rows = all_rows[all_rows[:, 0] == v]
        mu, s, q, o, rgb = _decode(sc, wl.views, rows, x, l, O, F, W1, b1, W2, b2, act,
                                   offsets, heads)
        imgs.append(render_view(mu.reshape(-1, 3), s.reshape(-1, 3), q.reshape(-1, 4),
                                o.reshape(-1), rgb.reshape(-1, 3), _view(view)))
    for a, b in zip(imgs, r.images):
        for key in ("rgb", "D", "normal", "alpha", "depth"):
            _close(key, a[key].detach().numpy(), b[key])
    # with decoded offsets the table O is unused: its gradient is zero
    grads = torch.autograd.grad(_loss(imgs, og), leaves, allow_unused=bool(offsets))
    for name, g, leaf in zip(names, grads, leaves):
        g = torch.zeros_like(leaf) if g is None else g
        _close("d_" + name, ref[name], g.numpy())
