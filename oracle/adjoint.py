"""Gradient of a mechanical objective with respect to the per-voxel Young's
modulus by the adjoint method (test infrastructure).

Forward problem (Sec. 2.3): eps = eps_mac + x, with x the compatible
fluctuation solving G[C:x] = -G[C:eps_mac] (no eigenstrain here; the
stiffness of a voxel is C_x = g(d_x) E_x C_hat(nu), so dC_x/dE_x = C_x/E_x).

For J(eps, E) with gradient field g = dJ/deps (a symmetric tensor per voxel),
differentiating the equilibrium condition gives

    dJ/dE_x = dJ/dE_x|_eps - lam_x : C_x : eps_x / E_x,

where lam is compatible and solves the adjoint problem G[C:lam] = G[g]:
the same symmetric operator as the forward solve, so the adjoint is a second
projected CG solve with the right-hand side G[g].

Objectives:
* W = h^dim/2 sum_x eps : C : eps (total elastic energy): g = h^dim C:eps,
  and G[C:eps] = 0 at equilibrium, so lam = 0 (envelope theorem);
* C11_eff = <sigma_11> / eps_11 = sum_x (C:eps)_11 / (N eps_11):
  g = C:e11 / (N eps_11) with e11 the unit 11 strain.
"""
import numpy as np

from . import cg as _cg
from . import fft as _fft
from . import material as _mat
from . import mech as _mech
from . import spectral as _sp


def _proj(t, D):
    dim = D.shape[0]
    axes = tuple(range(-dim, 0))
    return _fft.ifftn(_sp.project_full(_fft.fftn(t, axes), D), axes).real


def gradient_E(E_field, nu, eps_mac, h, objective, d=None, kappa=0.0, tol=1e-13, maxit=50000):
    """Returns (J, dJ/dE [grid], forward solution dict)."""
    E_field = np.asarray(E_field, dtype=np.float64)
    grid = E_field.shape
    dim = E_field.ndim
    N = E_field.size
    phase = np.zeros(grid, dtype=np.uint8)
    fw = _mech.mech_solve(phase, None, None, eps_mac, h, d=d, kappa=kappa, E_field=E_field, nu=nu, tol=tol,
                          maxit=maxit)
    lam_, mu_ = _mat.lame(E_field, nu)
    gdeg = np.ones(grid) if d is None else _mat.degradation(np.asarray(d), kappa)
    glam, gmu = gdeg * lam_, gdeg * mu_
    eps = _mat.from_voigt(fw["strain"], dim)
    sig = _mat.stress(eps, glam, gmu)
    D = _sp.grad_symbols(grid, h)
    if objective == "W":
        J = 0.5 * h ** dim * float(np.sum(eps * sig))
        g = h ** dim * sig
        explicit = 0.5 * h ** dim * np.sum(eps * sig, axis=(0, 1)) / E_field
    elif objective == "C11":
        e11 = eps_mac[0]
        J = float(np.sum(sig[0, 0])) / (N * e11)
        unit = np.zeros((dim, dim) + grid)
        unit[0, 0] = 1.0
        g = _mat.stress(unit, glam, gmu) / (N * e11)
        explicit = sig[0, 0] / (N * e11 * E_field)
    else:
        raise ValueError(objective)
    A = lambda v: _proj(_mat.stress(_mat.sym(v), glam, gmu), D)
    rhs = _proj(g, D)
    lam_eps, iters, rel, status = _cg.cg(A, rhs, tol=tol, maxit=maxit)
    lam_eps = _mat.sym(lam_eps)
    grad = explicit - np.sum(lam_eps * sig, axis=(0, 1)) / E_field
    return J, grad, fw
