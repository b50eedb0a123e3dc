"""Spherical-harmonic colour (Sec. 3.1: the colour of a 2D Gaussian is computed
from a set of SH coefficients and the viewing direction).

The paper does not fix a basis.  Reading: real SH of degree <= 3 in the sign
convention of 3DGS, i.e. basis function (l, m), m = -l..l, is (-1)^m times the
real harmonic built without the Condon-Shortley phase; coefficient index
b = l*l + l + m.  Colour = max(0, sum_b f_b Y_b(dir) + 0.5) per channel.

Two independent constructions are given and pinned against each other and
against orthonormality on the sphere (`tests/test_oracle_sh.py`):
  * `basis_scipy`: from scipy.special.sph_harm_y (complex, CS phase included);
  * `basis_poly`:  the textbook Cartesian polynomials with their normalisation
                   written as closed forms; usable with numpy or torch (the
                   FP64 autograd reference uses it).
"""

from __future__ import annotations

import math

import numpy as np


def n_basis(degree: int) -> int:
    return (degree + 1) ** 2


def basis_scipy(dirs, degree: int) -> np.ndarray:
    """(n, 3) unit directions -> (n, (L+1)^2) FP64 basis values."""
    from scipy.special import sph_harm_y

    d = np.asarray(dirs, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    out = np.zeros((d.shape[0], n_basis(degree)))
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)       # CS phase included
            if m == 0:
                real = Y.real
            elif m > 0:
                real = math.sqrt(2.0) * (-1) ** m * Y.real   # CS phase removed
            else:
                real = math.sqrt(2.0) * (-1) ** abs(m) * Y.imag
            out[:, l * l + l + m] = (-1) ** abs(m) * real  # 3DGS sign convention
    return out


def basis_poly(dirs, degree: int, xp=np):
    """Cartesian real-SH polynomials (unit `dirs`), 3DGS sign convention.
    Works on numpy arrays or torch tensors (xp = numpy or torch)."""
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    pi = math.pi
    cols = [xp.ones_like(x) * (0.5 / math.sqrt(pi))]
    if degree >= 1:
        k1 = math.sqrt(3.0 / (4.0 * pi))
        cols += [-k1 * y, k1 * z, -k1 * x]
    if degree >= 2:
        k2a = 0.5 * math.sqrt(15.0 / pi)
        k2b = 0.25 * math.sqrt(5.0 / pi)
        k2c = 0.25 * math.sqrt(15.0 / pi)
        xx, yy, zz = x * x, y * y, z * z
        cols += [k2a * x * y, -k2a * y * z, k2b * (2 * zz - xx - yy),
                 -k2a * x * z, k2c * (xx - yy)]
    if degree >= 3:
        k3a = 0.25 * math.sqrt(35.0 / (2 * pi))
        k3b = 0.5 * math.sqrt(105.0 / pi)
        k3c = 0.25 * math.sqrt(21.0 / (2 * pi))
        k3d = 0.25 * math.sqrt(7.0 / pi)
        k3e = 0.25 * math.sqrt(105.0 / pi)
        cols += [-k3a * y * (3 * xx - yy), k3b * x * y * z, -k3c * y * (4 * zz - xx - yy),
                 k3d * z * (2 * zz - 3 * xx - 3 * yy), -k3c * x * (4 * zz - xx - yy),
                 k3e * z * (xx - yy), -k3a * x * (xx - 3 * yy)]
    return xp.stack(cols, -1)


def colour(coeffs, dirs, degree: int, xp=np):
    """Per-Gaussian RGB from (n, B, 3) coefficients and (n, 3) unit directions:
    max(0, sum_b f_b Y_b + 0.5)."""
    Y = basis_poly(dirs, degree, xp)                 # (n, B)
    raw = (Y[..., :, None] * coeffs).sum(-2) + 0.5   # (n, 3)
    if xp is np:
        return np.maximum(raw, 0.0), raw
    return xp.clamp(raw, min=0.0), raw
