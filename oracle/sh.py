"""Real spherical-harmonic basis, degree <= 3 (oracle, test infrastructure).

The paper's colour comes from the anchor decoder; spherical harmonics are
used only for the explicit-Gaussian workloads.  Convention: real,
orthonormal on the unit sphere, no Condon-Shortley phase, coefficient index
l*l + l + m for m = -l..l, evaluated at a unit direction (x, y, z).

    Y_l^m = sqrt(2) K_l^|m| P_l^|m|(cos t) sin(|m| p)   m < 0
    Y_l^0 = K_l^0 P_l^0(cos t)
    Y_l^m = sqrt(2) K_l^m  P_l^m(cos t)  cos(m p)        m > 0
    K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)

written out below as polynomials in x, y, z.  Colour per channel is
max(0, sum_i Y_i(dir) k_i + 0.5).
"""
import numpy as np

PI = np.pi


def _consts():
    s = np.sqrt
    return dict(
        c00=0.5 / s(PI),
        c1=s(3.0 / (4.0 * PI)),
        c2a=0.5 * s(15.0 / PI),        # xy, yz, xz
        c20=0.25 * s(5.0 / PI),        # 3z^2 - 1
        c22=0.25 * s(15.0 / PI),       # x^2 - y^2
        c33=0.25 * s(35.0 / (2.0 * PI)),   # y(3x^2-y^2), x(x^2-3y^2)
        c32=0.5 * s(105.0 / PI),       # xyz
        c31=0.25 * s(21.0 / (2.0 * PI)),   # y(5z^2-1), x(5z^2-1)
        c30=0.25 * s(7.0 / PI),        # z(5z^2-3)
        c32b=0.25 * s(105.0 / PI),     # z(x^2-y^2)
    )


C = _consts()


def basis(dirs, degree):
    """dirs: (..., 3) unit vectors -> (..., (degree+1)^2) basis values."""
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    out = [np.full_like(x, C["c00"])]
    if degree >= 1:
        out += [C["c1"] * y, C["c1"] * z, C["c1"] * x]
    if degree >= 2:
        out += [C["c2a"] * x * y, C["c2a"] * y * z, C["c20"] * (3 * z * z - 1),
                C["c2a"] * x * z, C["c22"] * (x * x - y * y)]
    if degree >= 3:
        out += [C["c33"] * y * (3 * x * x - y * y), C["c32"] * x * y * z,
                C["c31"] * y * (5 * z * z - 1), C["c30"] * z * (5 * z * z - 3),
                C["c31"] * x * (5 * z * z - 1), C["c32b"] * z * (x * x - y * y),
                C["c33"] * x * (x * x - 3 * y * y)]
    return np.stack(out, axis=-1)


def basis_grad(dirs, degree):
    """Partial derivatives of the polynomials above with respect to x, y, z:
    (..., (degree+1)^2, 3).  Only the tangential part matters once chained
    through the normalisation of the direction."""
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    zero = np.zeros_like(x)
    g = [(zero, zero, zero)]
    if degree >= 1:
        c = C["c1"]
        g += [(zero, c + zero, zero), (zero, zero, c + zero), (c + zero, zero, zero)]
    if degree >= 2:
        a, b, e = C["c2a"], C["c20"], C["c22"]
        g += [(a * y, a * x, zero), (zero, a * z, a * y), (zero, zero, 6 * b * z),
              (a * z, zero, a * x), (2 * e * x, -2 * e * y, zero)]
    if degree >= 3:
        c33, c32, c31, c30, c32b = C["c33"], C["c32"], C["c31"], C["c30"], C["c32b"]
        g += [(c33 * 6 * x * y, c33 * (3 * x * x - 3 * y * y), zero),
              (c32 * y * z, c32 * x * z, c32 * x * y),
              (zero, c31 * (5 * z * z - 1), c31 * 10 * y * z),
              (zero, zero, c30 * (15 * z * z - 3)),
              (c31 * (5 * z * z - 1), zero, c31 * 10 * x * z),
              (c32b * 2 * x * z, -c32b * 2 * y * z, c32b * (x * x - y * y)),
              (c33 * (3 * x * x - 3 * y * y), -c33 * 6 * x * y, zero)]
    return np.stack([np.stack(t, axis=-1) for t in g], axis=-2)
