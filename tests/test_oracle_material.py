"""Pins of the oracle's constitutive helpers (CPU only): Lame constants of the
C1 matrix, the hand-evaluated 2D energy split of Sec. 2.4 (eq. energy), and
psi+ + psi- = psi in 2D and 3D."""
import numpy as np

from oracle import material as mat


def test_lame_c1_matrix():
    lam, mu = mat.lame(30e9, 0.2)
    assert abs(lam - 30e9 * 0.2 / (1.2 * 0.6)) < 1e-3
    assert abs(mu - 1.25e10) < 1e-3


def test_psi_plus_2d_by_hand():
    lam, mu = 2.0, 3.0
    for a, b, s in [(1e-3, 2e-3, 5e-4), (-3e-3, 1e-3, -2e-4), (-1e-3, -2e-3, 0.0)]:
        eps = np.array([[a, s], [s, b]])
        tr = a + b
        dev = np.array([[a - tr / 2, s], [s, b - tr / 2]])
        expect = 0.5 * (lam + mu) * max(tr, 0.0) ** 2 + mu * np.sum(dev * dev)
        assert abs(mat.psi_plus(eps, lam, mu) - expect) < 1e-18
        # dev : dev by hand for this 2x2 case
        assert abs(np.sum(dev * dev) - ((a - b) ** 2 / 2 + 2 * s * s)) < 1e-18


def test_split_sums_to_energy():
    rng = np.random.default_rng(1)
    for dim in (2, 3):
        t = rng.standard_normal((dim, dim, 5))
        eps = 0.5 * (t + np.swapaxes(t, 0, 1))
        lam, mu = 1.3, 0.7
        psi = 0.5 * lam * np.trace(eps) ** 2 + mu * np.einsum("ij...,ij...->...", eps, eps)
        split = mat.psi_plus(eps, lam, mu) + mat.psi_minus(eps, lam, mu)
        assert np.allclose(split, psi, rtol=1e-14)
        assert np.allclose(mat.energy_density(eps, lam, mu), psi, rtol=1e-14)
