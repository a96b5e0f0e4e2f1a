"""Pins of the oracle's displacement-form preconditioned CG (CPU only).

* unit Green operator: after k iterations the strain equals the strain of k
  iterations of the paper's projected CG in strain form (oracle.mech), the
  equivalence the GPU mechanics solver is built on;
* reference-medium Green operator: a homogeneous medium equal to the
  reference is solved in one iteration; a two-phase medium at contrast 1e4
  converges to the sparse direct solution; the reference symbol is the
  Fourier symbol of the stiffness stencil of a homogeneous medium.
"""
import numpy as np
import pytest

from oracle import direct, material as mat, mech, precond, spectral as sp, fft

H = 5e-6
E_TAB = (3e6, 30e9)
NU_TAB = (0.2, 0.2)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _case(grid, seed):
    rng = np.random.default_rng(seed)
    phase = (rng.random(grid) < 0.6).astype(np.uint8)
    e = 1e-3 * rng.random(grid) * (phase == 0)
    d = 0.3 * rng.random(grid)
    return phase, e, d


@pytest.mark.parametrize("k", [1, 5, 30])
def test_unit_green_equals_projected_cg_iterates(k):
    phase, e, d = _case((8, 12), 1)
    em = (1e-3, -2e-4, 3e-4)
    a = mech.mech_solve(phase, E_TAB, NU_TAB, em, H, d=d, kappa=1e-6, e=e, fixed_iters=k)
    b = precond.mech_pcg(phase, E_TAB, NU_TAB, em, H, d=d, kappa=1e-6, e=e, fixed_iters=k)
    assert rel(b["strain"], a["strain"]) < 1e-12


def test_reference_symbol_is_the_homogeneous_stencil():
    grid = (6, 10)
    lam0, mu0 = 3.0, 2.0
    E = mu0 * (3 * lam0 + 2 * mu0) / (lam0 + mu0)
    nu = lam0 / (2 * (lam0 + mu0))
    u = np.random.default_rng(2).standard_normal((2,) + grid)
    q = direct.mech_stiffness_apply(np.zeros(grid, np.uint8), (E,), (nu,), u, H)
    D = sp.grad_symbols(grid, H)
    K0 = precond.reference_stiffness_symbol(D, lam0, mu0)
    u_hat = fft.fftn(u, (-2, -1))
    q_hat = np.einsum("ij...,j...->i...", K0, u_hat)
    assert rel(fft.ifftn(q_hat, (-2, -1)).real, q) < 1e-13


def test_reference_green_homogeneous_one_iteration():
    grid = (8, 8)
    E, nu = 30e9, 0.2
    lam0, mu0 = mat.lame(E, nu)
    rng = np.random.default_rng(4)
    e = 1e-3 * rng.random(grid)
    r = precond.mech_pcg(np.zeros(grid, np.uint8), (E,), (nu,), (0.0, 0.0, 0.0), H, e=e,
                         reference=(float(lam0), float(mu0)), tol=1e-13)
    q = direct.mech_direct(np.zeros(grid, np.uint8), (E,), (nu,), (0.0, 0.0, 0.0), H, e=e)
    assert r["iters"] <= 1
    assert rel(r["strain"], q["strain"]) < 1e-12


@pytest.mark.parametrize("reference", [None, "matrix"])
def test_converges_to_direct_at_high_contrast(reference):
    phase, e, d = _case((10, 8), 3)
    em = (1e-3, 0.0, 2e-4)
    ref = None if reference is None else tuple(float(v) for v in mat.lame(30e9, 0.2))
    r = precond.mech_pcg(phase, E_TAB, NU_TAB, em, H, e=e, reference=ref, tol=1e-14, maxit=20000)
    q = direct.mech_direct(phase, E_TAB, NU_TAB, em, H, e=e)
    assert r["status"] == 0
    assert rel(r["strain"], q["strain"]) < 1e-10
