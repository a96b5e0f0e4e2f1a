"""Pins of the oracle's static diffusion homogenisation (Sec. 2.1) and the
concentration reconstruction (eqs. micro-gradient to concentration-correct),
CPU only.

* the projected CG reaches the sparse direct solution of the real-space
  stencil problem (no FFT);
* laminates: grid-aligned layers give the exact harmonic (across the layers)
  and arithmetic (along them) means, zero cross terms;
* <grad c> = grad c_mac; Hill-Mandel <grad c . j> = <grad c> . <j>;
* D_eff is symmetric and lies between the harmonic and arithmetic means;
* a homogeneous medium has no fluctuation;
* reconstruction: phi recovered from a gradient built with the sparse
  forward-difference matrix (no FFT); the reconstructed c has finite
  differences h grad c between voxels of one phase, solid mean 0 and pore
  mean c_mac / eta.
"""
import numpy as np
import pytest

from oracle import direct, homogenisation as hm

H = 5e-6


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _Dfield(grid, seed, contrast=1e3):
    rng = np.random.default_rng(seed)
    phase = (rng.random(grid) < 0.6).astype(np.uint8)  # 0 pore
    return phase, np.where(phase == 0, 1e-9, 1e-9 / contrast)


@pytest.mark.parametrize("grid", [(8, 8), (6, 10), (4, 4, 6)])
def test_matches_direct_solve(grid):
    phase, Df = _Dfield(grid, 3)
    g = (0.7, -0.4, 0.2)[:len(grid)]
    r = hm.diffusion_homogenise(Df, g, H, tol=1e-14, maxit=5000)
    q = direct.diffusion_static_direct(Df, g, H)
    assert r["status"] == 0
    assert rel(r["grad_c"], q["grad_c"]) < 1e-11
    phi = hm.fluctuation_from_gradient(r["grad_c"], H)
    assert np.max(np.abs(phi - q["phi"])) < 1e-11 * np.max(np.abs(q["phi"]))


@pytest.mark.parametrize("axis", [0, 1])
def test_laminate_exact(axis):
    n = 12
    vals = np.array([1e-9, 3e-12, 5e-10, 1e-9, 2e-11, 7e-10, 1e-9, 1e-9, 4e-12, 8e-10, 6e-10, 1e-11])
    Df = np.broadcast_to(vals[None, :], (n, n)).copy() if axis == 0 else np.broadcast_to(vals[:, None], (n, n)).copy()
    Deff, _ = hm.effective_diffusivity(Df, H, tol=1e-15)
    harm, arith = 1.0 / np.mean(1.0 / vals), np.mean(vals)
    across, along = (0, 1) if axis == 0 else (1, 0)
    assert abs(Deff[across, across] - harm) < 1e-12 * harm
    assert abs(Deff[along, along] - arith) < 1e-12 * arith
    assert abs(Deff[0, 1]) < 1e-12 * arith and abs(Deff[1, 0]) < 1e-12 * arith


def test_mean_gradient_and_hill_mandel():
    phase, Df = _Dfield((16, 12), 5, contrast=1e4)
    g = (0.3, 1.1)
    r = hm.diffusion_homogenise(Df, g, H, tol=1e-14, maxit=20000)
    gc, j = r["grad_c"], r["flux"]
    assert np.allclose([gc[0].mean(), gc[1].mean()], g, rtol=1e-13, atol=1e-15)
    lhs = np.mean(np.sum(gc * j, axis=0))
    rhs = float(np.dot([gc[0].mean(), gc[1].mean()], r["mean_flux"]))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_effective_diffusivity_symmetric_and_bounded():
    phase, Df = _Dfield((12, 12), 7)
    Deff, iters = hm.effective_diffusivity(Df, H, tol=1e-14)
    assert abs(Deff[0, 1] - Deff[1, 0]) < 1e-9 * abs(Deff[0, 0])
    w = np.linalg.eigvalsh(0.5 * (Deff + Deff.T))
    assert w.min() >= (1.0 / np.mean(1.0 / Df)) * (1 - 1e-12)
    assert w.max() <= np.mean(Df) * (1 + 1e-12)
    assert min(iters) > 0


def test_homogeneous_no_iteration():
    Df = np.full((8, 12), 2e-9)
    r = hm.diffusion_homogenise(Df, (0.5, -2.0), H, tol=1e-12)
    # the right-hand side is zero up to the rounding of the transforms
    assert r["iters"] <= 1
    assert np.max(np.abs(r["grad_c"][0] - 0.5)) < 1e-14 and np.max(np.abs(r["grad_c"][1] + 2.0)) < 1e-14
    assert np.allclose(r["mean_flux"], [-1e-9, 4e-9], rtol=1e-15)


def test_reconstruction_round_trip_and_phase_means():
    grid = (10, 12)
    rng = np.random.default_rng(11)
    phi0 = rng.standard_normal(grid)
    g = (0.8, -0.3)
    B = [direct.fwd_diff_matrix(grid, a, H) for a in range(2)]
    grad = np.array([g[a] + (B[a] @ phi0.ravel()).reshape(grid) for a in range(2)])
    phi = hm.fluctuation_from_gradient(grad, H)
    assert np.max(np.abs(phi - (phi0 - phi0.mean()))) < 1e-12 * np.max(np.abs(phi0))
    phase = (rng.random(grid) < 0.5).astype(np.uint8)
    c_mac = 0.37
    r = hm.concentration(phase, grad, g, c_mac, H)
    c = r["c"]
    pore = phase == 0
    eta = pore.mean()
    assert abs(c[~pore].mean()) < 1e-12 and abs(c[pore].mean() - c_mac / eta) < 1e-12
    assert abs(c.mean() - c_mac) < 1e-12
    # within one phase and away from the periodic seam: c(x + e_a) - c(x) = h grad_a c(x)
    for a, (dy, dx) in enumerate(((0, 1), (1, 0))):
        y, x = np.meshgrid(np.arange(grid[0] - dy), np.arange(grid[1] - dx), indexing="ij")
        same = phase[y, x] == phase[y + dy, x + dx]
        diff = (c[y + dy, x + dx] - c[y, x])[same]
        assert np.allclose(diff, H * grad[a][y, x][same], rtol=0, atol=1e-12 * np.max(np.abs(c)))
