"""Voxel-anchor selection, decoding into Gaussians, and the decode adjoint
(oracle, test infrastructure).

Sec. 3.2 gives each voxel anchor a feature F in R^32, a scaling factor l
in R^3, a position x and n learnable offsets O in R^{n x 3}; a shared
decoder F_de maps (F, relative viewing distance, direction to the camera)
to n Gaussians' opacity, colour and covariance, and the means are
mu_k = x + O_k * l (Eq. 4).  Sec. 3.1 selects the level of detail by
observation distance; Sec. 3.3 searches the voxels that intersect the
view.  Readings of what the paper leaves open:

  * LoD: anchor a is active in view v when level[a] <= clamp(
    floor(log2(d_max / |x_a - c_v|)), 0, K-1), evaluated exactly as
    level == 0 or |x_a - c_v|^2 * 4^level <= d_max^2 (float64, fixed
    order); and its centre passes the frustum test p_z > z_near,
    |p_x| <= g_x p_z, |p_y| <= g_y p_z with g = 1.3 W / (2 f);
  * rows are the active (view, anchor) pairs in (view, anchor) order;
  * decoder: one MLP 36 -> 32 (ReLU) -> 110, input z0 = [bf16(F),
    d~ = (c_v - x_a)/|c_v - x_a|, Delta = |c_v - x_a| / d_max], output per
    Gaussian k the 11 values z2[11k : 11k+11] = (opacity, rgb, scale,
    quaternion) with o = sigmoid, rgb = sigmoid, s = l * sigmoid and the
    raw quaternion normalised at projection;
  * opacity variant (row f3): o = tanh(z) with the Gaussians of o <= 0
    masked out (the stream compaction of the masked-opacity decoders); a
    masked Gaussian, like any with o < 1/255, draws nothing and gets no
    tiles, so the mask needs no separate decision;
  * mu_k = x + O_k * l elementwise, in float64;
  * offset variant (row f3, decoder-emitted offsets): with offset_mode = 1
    the decoder has 14 outputs per Gaussian, the 11 above followed by the
    offset O_k itself (no activation), z2[14k+11 : 14k+14]; then
    mu_k = x + O_k * l with that O_k, and the anchor table's offsets are
    not used (their gradient is zero);
  * head variant (row f3, "a set of shared Gaussian Decoders"): with
    decoder_heads = 3 each attribute group has an MLP of its own, 36 -> 32
    (ReLU) -> n * width: opacity (width 1), colour (3), covariance (scale
    and quaternion, 7), and with decoded offsets a fourth, the offsets (3).
    Their weights sit side by side: W1 is 36 x 32H with head h reading
    hidden columns 32h .. 32h+31, b1 has 32H entries, and W2 (32 x n*G)
    and b2 keep the per-Gaussian output count G of the shared decoder but
    group their columns by head: head h owns the n * width_h columns that
    start at n * first_h, and Gaussian k's attribute first_h + j is its
    column n * first_h + k * width_h + j.  With one head this is the
    shared decoder's layout (column k * G + j);
  * the feature F is rounded to bfloat16 (weights are given in bfloat16);
    every other decoder value is carried exactly (float64 here);
  * decoded offsets move the mean by the decoder's own float32 error, which
    the GPU cannot avoid.  Each decoder output is a float32 sum of at most
    97 terms (hidden units times split terms, and the bias); its error is
    taken as at most DEC_ERR = 2^-20 (16 unit roundoffs) of the sum of the
    terms' magnitudes, plus the hidden layer's own error of that size
    carried through |W2|.  That is a margin, like the other near-tie
    margins, not a worst-case bound (recursive summation allows 97 unit
    roundoffs): float32 evaluations in BLAS and sequential order stay below
    one unit roundoff of it.  decode() returns it on the mean, l times the
    offset's, as mu_tol; the decisions and depth keys that depend on the
    mean treat it as rounding (near ties, key tolerance).
"""
import numpy as np

from . import bf16 as bfmod
from .project import view_arrays

GAUSS_OUT = 11
FRAG = 1e-5
OPACITY_SIGMOID = 0
OPACITY_TANH_MASK = 1
OFFSETS_LEARNED = 0
OFFSETS_DECODED = 1
DECODER_SHARED = 1
DECODER_PER_ATTRIBUTE = 3
HIDDEN = 32
DEC_ERR = 2.0 ** -20


def _per_gauss(scene):
    """Decoder outputs per Gaussian: 11, or 14 with decoder-emitted offsets."""
    return GAUSS_OUT + 3 if int(getattr(scene, "offset_mode", OFFSETS_LEARNED)) == OFFSETS_DECODED \
        else GAUSS_OUT


def head_groups(scene):
    """(first attribute, width) of the per-Gaussian outputs of each decoder
    head: one shared head of all G outputs, or one head per attribute group
    (opacity, colour, covariance, and the offsets when they are decoded)."""
    go = _per_gauss(scene)
    heads = int(getattr(scene, "decoder_heads", DECODER_SHARED))
    if heads == DECODER_SHARED:
        return [(0, go)]
    if heads != DECODER_PER_ATTRIBUTE:
        raise ValueError(f"decoder_heads {heads} is neither 1 nor 3")
    groups = [(0, 1), (1, 3), (4, 7)]
    if go > GAUSS_OUT:
        groups.append((GAUSS_OUT, 3))
    return groups


def select(scene, views):
    """a0: active (view, anchor) rows in (view, anchor) order.

    Returns (rows (R,2) int64, per-view row offsets (B+1,))."""
    x = np.asarray(scene.x, np.float64)
    level = np.asarray(scene.level).astype(np.int64)
    dmax = float(np.float32(scene.d_max))
    dmax2 = dmax * dmax
    rows, offs = [], [0]
    for v, view in enumerate(views):
        V = view_arrays(view)
        c, R, t = V["c"], V["R"], V["t"]
        d0, d1, d2 = c[0] - x[:, 0], c[1] - x[:, 1], c[2] - x[:, 2]
        dist2 = (d0 * d0 + d1 * d1) + d2 * d2
        lod_ok = (level == 0) | (dist2 * (4.0 ** level) <= dmax2)
        p = [((R[i, 0] * x[:, 0] + R[i, 1] * x[:, 1]) + R[i, 2] * x[:, 2]) + t[i] for i in range(3)]
        gx = (1.3 * V["W"]) / (2.0 * V["fx"])
        gy = (1.3 * V["H"]) / (2.0 * V["fy"])
        inside = (p[2] > V["z_near"]) & (np.abs(p[0]) <= gx * p[2]) & (np.abs(p[1]) <= gy * p[2])
        act = np.nonzero(lod_ok & inside)[0]
        rows.append(np.stack([np.full(act.size, v), act], 1))
        offs.append(offs[-1] + act.size)
    rows = np.concatenate(rows, 0) if rows else np.zeros((0, 2), np.int64)
    return rows.astype(np.int64), np.asarray(offs, np.int64)


def decoder_input(scene, views, rows, emulate_bf16=True):
    """z0 per row: [F (bf16-rounded unless emulate_bf16 is False), d~, Delta]."""
    a = rows[:, 1]
    if emulate_bf16:
        F = bfmod.round_to_bf16(np.asarray(scene.F, np.float32)[a])
    else:
        F = np.asarray(scene.F, np.float64)[a]
    x = np.asarray(scene.x, np.float64)[a]
    cams = np.stack([view_arrays(v)["c"] for v in views])
    delta = cams[rows[:, 0]] - x
    dist = np.linalg.norm(delta, axis=1)
    dirn = delta / dist[:, None]
    dmax = float(np.float32(scene.d_max))
    z0 = np.concatenate([F, dirn, (dist / dmax)[:, None]], 1)
    return z0, dict(delta=delta, dist=dist, dirn=dirn, dmax=dmax)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def decode(scene, views, rows, emulate_bf16=True):
    """a1: decode every row into n Gaussians.

    Returns dict with per-Gaussian arrays (R*n rows, row-major (row, k)):
    mu (float64), scales, quats (raw), opacity, rgb; and the MLP
    intermediates for the adjoint."""
    n = scene.O.shape[1]
    z0, geo = decoder_input(scene, views, rows, emulate_bf16)
    # decoder weights: the bfloat16 values (a float64 override is honoured so
    # that finite differences can perturb them)
    W1 = getattr(scene, "W1_exact", None)
    W1 = bfmod.from_bits(scene.W1_bits) if W1 is None else np.asarray(W1, np.float64)
    W2 = getattr(scene, "W2_exact", None)
    W2 = bfmod.from_bits(scene.W2_bits) if W2 is None else np.asarray(W2, np.float64)
    b1 = np.asarray(scene.b1, np.float64)
    b2 = np.asarray(scene.b2, np.float64)
    r = rows.shape[0]
    go = _per_gauss(scene)
    heads = head_groups(scene)
    # each head is an MLP of its own: hidden block h of W1 / b1, then its
    # column block of W2 / b2; g collects the per-Gaussian outputs
    g = np.empty((r, n, go))
    pre1, z1, z2 = [], [], []
    for h, (first, width) in enumerate(heads):
        hid = slice(HIDDEN * h, HIDDEN * (h + 1))
        cols = slice(n * first, n * (first + width))
        p = z0 @ W1[:, hid] + b1[hid]
        z = np.maximum(p, 0.0)
        y = z @ W2[:, cols] + b2[cols]
        g[..., first:first + width] = y.reshape(r, n, width)
        pre1.append(p)
        z1.append(z)
        z2.append(y)
    pre1, z1, z2 = (np.concatenate(t, 1) for t in (pre1, z1, z2))
    a = rows[:, 1]
    x = np.asarray(scene.x, np.float64)[a]
    l = np.asarray(scene.l, np.float64)[a]
    O = g[..., 11:14] if go > GAUSS_OUT else np.asarray(scene.O, np.float64)[a]
    mu = x[:, None, :] + O * l[:, None, :]
    act = int(getattr(scene, "opacity_act", OPACITY_SIGMOID))
    op = np.tanh(g[..., 0]) if act == OPACITY_TANH_MASK else sigmoid(g[..., 0])
    rgb = sigmoid(g[..., 1:4])
    ssig = sigmoid(g[..., 4:7])
    scales = l[:, None, :] * ssig
    quats = g[..., 7:11]
    frag_relu = np.any(np.abs(pre1) < FRAG * (np.abs(z0) @ np.abs(W1) + np.abs(b1)), axis=1)
    mu_tol = None
    if go > GAUSS_OUT:
        e1 = DEC_ERR * (np.abs(z0) @ np.abs(W1) + np.abs(b1))       # hidden-layer error bound
        eO = np.zeros((r, n, 3))
        for h, (first, width) in enumerate(heads):
            hid = slice(HIDDEN * h, HIDDEN * (h + 1))
            for c in range(3):
                m = GAUSS_OUT + c
                if not first <= m < first + width:
                    continue
                cols = n * first + np.arange(n) * width + (m - first)
                aW = np.abs(W2[:, cols])
                eO[..., c] = (DEC_ERR * (np.abs(z1[:, hid]) @ aW + np.abs(b2[cols]))
                              + e1[:, hid] @ aW)
        mu_tol = (eO * l[:, None, :]).reshape(-1, 3)
    return dict(
        n=n, rows=rows, mu=mu.reshape(-1, 3), scales=scales.reshape(-1, 3),
        quats=quats.reshape(-1, 4), opacity=op.reshape(-1), rgb=rgb.reshape(-1, 3),
        frag_relu=frag_relu, mu_tol=mu_tol,
        _z0=z0, _pre1=pre1, _z1=z1, _z2=z2, _W1=W1, _W2=W2, _geo=geo, _l=l, _O=O,
        _ssig=ssig, _op=op, _rgb=rgb, _act=act, _go=go, _heads=heads)


def decode_backward(scene, D, g):
    """a10: adjoint of `decode`.

    g: per-Gaussian gradients (R*n rows): mu (3), scales (3), quats (4),
    opacity, rgb (3).  Returns gradients of the anchor table (x, l, O, F,
    summed over every row of the anchor) and of the decoder (W1, b1, W2,
    b2).  The bfloat16 rounding of F is passed straight through."""
    rows = D["rows"]
    r, n = rows.shape[0], D["n"]
    gm = np.asarray(g["mu"], np.float64).reshape(r, n, 3)
    gs = np.asarray(g["scales"], np.float64).reshape(r, n, 3)
    gq = np.asarray(g["quats"], np.float64).reshape(r, n, 4)
    go = np.asarray(g["opacity"], np.float64).reshape(r, n)
    gc = np.asarray(g["rgb"], np.float64).reshape(r, n, 3)
    op, rgb, ssig, l, O = D["_op"], D["_rgb"], D["_ssig"], D["_l"], D["_O"]
    go_ = D.get("_go", GAUSS_OUT)
    dz2 = np.zeros((r, n, go_))
    dz2[..., 0] = go * ((1 - op * op) if D["_act"] == OPACITY_TANH_MASK else op * (1 - op))
    dz2[..., 1:4] = gc * rgb * (1 - rgb)
    dz2[..., 4:7] = gs * l[:, None, :] * ssig * (1 - ssig)
    dz2[..., 7:11] = gq
    dl = np.sum(gs * ssig, axis=1) + np.sum(gm * O, axis=1)
    dO = gm * l[:, None, :]
    if go_ > GAUSS_OUT:                 # decoder-emitted offsets: dmu/dO_k = l
        dz2[..., 11:14] = dO
        dO = np.zeros_like(dO)
    dx = np.sum(gm, axis=1)
    W1, W2 = D["_W1"], D["_W2"]
    z0, z1, pre1 = D["_z0"], D["_z1"], D["_pre1"]
    dW1, db1 = np.zeros_like(W1), np.zeros(W1.shape[1])
    dW2, db2 = np.zeros_like(W2), np.zeros(W2.shape[1])
    dz0 = np.zeros_like(z0)
    for h, (first, width) in enumerate(D.get("_heads", [(0, go_)])):
        hid = slice(HIDDEN * h, HIDDEN * (h + 1))
        cols = slice(n * first, n * (first + width))
        dy = dz2[..., first:first + width].reshape(r, n * width)
        dW2[:, cols] = z1[:, hid].T @ dy
        db2[cols] = dy.sum(0)
        dz1 = (dy @ W2[:, cols].T) * (pre1[:, hid] > 0)
        dW1[:, hid] = z0.T @ dz1
        db1[hid] = dz1.sum(0)
        dz0 += dz1 @ W1[:, hid].T
    geo = D["_geo"]
    dF = dz0[:, :32]
    ddir, ddel = dz0[:, 32:35], dz0[:, 35]
    dirn, dist = geo["dirn"], geo["dist"]
    # d~ = delta/|delta|, Delta = |delta|/d_max, delta = c - x
    ddelta = (ddir - dirn * np.sum(dirn * ddir, 1, keepdims=True)) / dist[:, None]
    ddelta += (ddel / geo["dmax"])[:, None] * dirn
    dx += -ddelta
    A = scene.x.shape[0]
    a = rows[:, 1]
    out = dict(x=np.zeros((A, 3)), l=np.zeros((A, 3)), O=np.zeros((A, n, 3)),
               F=np.zeros((A, 32)), W1=dW1, b1=db1, W2=dW2, b2=db2)
    np.add.at(out["x"], a, dx)
    np.add.at(out["l"], a, dl)
    np.add.at(out["O"], a, dO)
    np.add.at(out["F"], a, dF)
    return out
