"""Pins of the oracle's spherical-harmonic basis (colour from SH, Sec. 3.4 /
prior 3DGS appearance): orthonormality by quadrature, agreement with scipy's
complex harmonics, and the gradient against central differences."""
import numpy as np
import pytest
from scipy.special import sph_harm_y

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _dirs(theta, phi):
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], -1)


def test_orthonormal_by_quadrature(oracle):
    xg, wg = np.polynomial.legendre.leggauss(64)          # cos(theta) nodes
    nphi = 128
    phi = 2 * np.pi * (np.arange(nphi) + 0.5) / nphi
    G = np.zeros((16, 16))
    for ct, w in zip(xg, wg):
        th = np.arccos(ct)
        for ph in phi:
            Y, _ = oracle.sh_basis(3, _dirs(th, ph))
            G += w * (2 * np.pi / nphi) * np.outer(Y, Y)
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_matches_scipy_real_combinations(oracle):
    rng = np.random.default_rng(7)
    for _ in range(50):
        th, ph = np.arccos(rng.uniform(-1, 1)), rng.uniform(0, 2 * np.pi)
        Y, _ = oracle.sh_basis(3, _dirs(th, ph))
        for l in range(4):
            for m in range(-l, l + 1):
                c = sph_harm_y(l, abs(m), th, ph)     # includes the (-1)^m phase
                ref = c.real if m == 0 else (np.sqrt(2) * (c.real if m > 0 else c.imag))
                assert abs(Y[l * l + l + m] - ref) < 1e-13, (l, m)


def test_gradient_matches_central_differences(oracle):
    rng = np.random.default_rng(8)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        _, dY = oracle.sh_basis(3, d)
        h = 1e-6
        for a in range(3):
            e = np.zeros(3); e[a] = h
            Yp, _ = oracle.sh_basis(3, d + e)
            Ym, _ = oracle.sh_basis(3, d - e)
            assert np.allclose((Yp - Ym) / (2 * h), dY[:, a], atol=1e-8)
