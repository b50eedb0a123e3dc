"""Pins of the real-SH colour basis (Sec. 3.1 SH colour; 3DGS sign convention)."""

import math

import numpy as np

from oracle import sh


def _sphere_quadrature(n_theta=40, n_phi=80):
    """Gauss-Legendre in cos(theta) x uniform phi: exact for polynomials of
    degree < 2 n_theta on the sphere."""
    x, w = np.polynomial.legendre.leggauss(n_theta)
    phi = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct * ct)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(n_phi, 2 * math.pi / n_phi)[None, :]).ravel()
    return dirs, wts


def test_basis_orthonormal():
    dirs, wts = _sphere_quadrature()
    Y = sh.basis_poly(dirs, 3)
    G = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-10)


def test_poly_equals_scipy_construction():
    rng = np.random.default_rng(11)
    d = rng.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    np.testing.assert_allclose(sh.basis_poly(d, 3), sh.basis_scipy(d, 3), atol=1e-12)


def test_degree_zero_colour():
    f0 = np.array([[[0.7, -2.0, 0.0]]])
    d = np.array([[0.0, 0.6, 0.8]])
    rgb, raw = sh.colour(f0, d, 0)
    np.testing.assert_allclose(raw[0], 0.5 + f0[0, 0] / (2 * math.sqrt(math.pi)), atol=1e-15)
    assert rgb[0, 1] == 0.0 and raw[0, 1] < 0          # clamp at zero


def test_degree_one_sign_convention():
    """Basis 1..3 are -k y, k z, -k x with k = sqrt(3 / 4 pi)."""
    k = math.sqrt(3 / (4 * math.pi))
    Y = sh.basis_poly(np.eye(3), 1)
    np.testing.assert_allclose(Y[:, 1:], [[0, 0, -k], [-k, 0, 0], [0, k, 0]], atol=1e-15)
