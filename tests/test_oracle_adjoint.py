"""Pins of the oracle's adjoint gradient (CPU only): central finite differences
of the objective itself, the envelope closed form for the energy, and the
Hill-Mandel closed form dC11/dE_x = eps:sigma / (N eps11^2 E_x)."""
import numpy as np
import pytest

from oracle import adjoint, material as mat

H = 5e-6


def _field(seed, n=8):
    rng = np.random.default_rng(seed)
    E = np.where(rng.random((n, n)) < 0.35, 3e8, 30e9) * (1 + 0.1 * rng.random((n, n)))
    d = 0.3 * rng.random((n, n))
    return E, d


@pytest.mark.parametrize("objective", ["W", "C11"])
def test_adjoint_matches_central_differences(objective):
    E, d = _field(1)
    em = (1e-3, 0.0, 0.0)
    J, g, _ = adjoint.gradient_E(E, 0.2, em, H, objective, d=d, kappa=1e-6)
    rng = np.random.default_rng(2)
    for _ in range(4):
        iy, ix = rng.integers(0, 8, 2)
        step = 1e-4 * E[iy, ix]
        Ep, Em = E.copy(), E.copy()
        Ep[iy, ix] += step
        Em[iy, ix] -= step
        Jp = adjoint.gradient_E(Ep, 0.2, em, H, objective, d=d, kappa=1e-6)[0]
        Jm = adjoint.gradient_E(Em, 0.2, em, H, objective, d=d, kappa=1e-6)[0]
        fd = (Jp - Jm) / (2 * step)
        assert abs(fd - g[iy, ix]) < 1e-6 * abs(g).max(), (objective, fd, g[iy, ix])


def test_closed_forms():
    E, d = _field(3)
    e11 = 1e-3
    N = E.size
    Jw, gw, fw = adjoint.gradient_E(E, 0.2, (e11, 0.0, 0.0), H, "W", d=d, kappa=1e-6)
    Jc, gc, _ = adjoint.gradient_E(E, 0.2, (e11, 0.0, 0.0), H, "C11", d=d, kappa=1e-6)
    lam, mu = mat.lame(E, 0.2)
    gdeg = mat.degradation(d, 1e-6)
    eps = mat.from_voigt(fw["strain"], 2)
    sig = mat.stress(eps, gdeg * lam, gdeg * mu)
    dens = np.sum(eps * sig, axis=(0, 1))
    assert np.allclose(gw, 0.5 * H ** 2 * dens / E, rtol=1e-9, atol=0)
    assert np.allclose(gc, dens / (N * e11 ** 2 * E), rtol=1e-8, atol=1e-12 * np.abs(gc).max())
    # Hill-Mandel links the two objectives
    assert abs(Jc - 2 * Jw / (N * H ** 2 * e11 ** 2)) < 1e-10 * Jc
