"""Projected-CG mechanical equilibrium with eigenstrain (test infrastructure).

Follows Sec. 2.3 (eq. solid and eq. solid-final) and App. A:

    find the periodic fluctuation x = grad u (range of the projection) with
    G[ g C : (eps_mac + sym(x) - e I) ] = 0,

solved as the linear system  G[g C : sym(x)] = -G[g C : (eps_mac - e I)]  by
CG.  The problem is linear, so the Newton loop of Alg. 1 converges after its
first linear solve.  g = (1 - d)^2 + kappa (Sec. 2.4), C is isotropic per phase
(Sec. 2.3) or built from a per-voxel Young's modulus with a uniform Poisson
ratio.  The eigenstrain is isotropic, eps* = e(x) I (eq. eigen-simplify).

Two unknown storages:
* "full": the non-symmetric displacement gradient (dim x dim), projected row
  by row with the fourth-order projection of App. A;
* "sym": the symmetric strain, projected with the symmetric projection.
Both reach the same discrete solution.  Inner products are Frobenius sums
over the stored tensor, so shear counts twice in either storage.

Outputs (post-processing): total strain eps = eps_mac + sym(x), stress
sigma = g C : (eps - e I), the mean stress over all voxels, and the elastic
energy W = h^dim / 2 * sum_x (eps - e I) : sigma.
"""
import numpy as np

from . import cg as _cg
from . import fft as _fft
from . import material as _mat
from . import spectral as _sp


def voxel_lame(phase, E_tab, nu_tab, E_field=None, nu=None):
    if E_field is not None:
        return _mat.lame(np.asarray(E_field, dtype=np.float64), nu)
    lam_tab, mu_tab = _mat.lame(np.asarray(E_tab), np.asarray(nu_tab))
    return lam_tab[phase], mu_tab[phase]


def _axes(dim):
    return tuple(range(-dim, 0))


def mech_operator(p, glam, gmu, D, storage="full"):
    dim = D.shape[0]
    eps = _mat.sym(p) if storage == "full" else p
    sig = _mat.stress(eps, glam, gmu)
    sig_hat = _fft.fftn(sig, _axes(dim))
    if storage == "full":
        out_hat = _sp.project_full(sig_hat, D)
    else:
        out_hat = _sp.project_sym(sig_hat, D)
    return _fft.ifftn(out_hat, _axes(dim)).real


def macro_tensor(eps_mac_voigt, dim, grid):
    t = np.zeros((dim, dim) + tuple(grid))
    for c, (i, j) in enumerate(_mat.voigt_pairs(dim)):
        t[i, j] = eps_mac_voigt[c]
        t[j, i] = eps_mac_voigt[c]
    return t


def eigen_tensor(e, dim, grid):
    t = np.zeros((dim, dim) + tuple(grid))
    if e is not None:
        for i in range(dim):
            t[i, i] = e
    return t


def mech_solve(phase, E_tab, nu_tab, eps_mac, h, d=None, kappa=0.0, e=None,
               tol=1e-10, maxit=20000, storage="full", E_field=None, nu=None,
               fixed_iters=None, return_x=False, op="forward"):
    phase = np.asarray(phase)
    grid = phase.shape
    dim = phase.ndim
    lam, mu = voxel_lame(phase, E_tab, nu_tab, E_field, nu)
    g = np.ones(grid) if d is None else _mat.degradation(np.asarray(d), kappa)
    glam, gmu = g * lam, g * mu
    D = _sp.grad_symbols(grid, h, op)
    E0 = macro_tensor(eps_mac, dim, grid) - eigen_tensor(e, dim, grid)
    b = -mech_operator(E0, glam, gmu, D, storage)
    A = lambda p: mech_operator(p, glam, gmu, D, storage)
    x, iters, rel, status = _cg.cg(A, b, tol=tol, maxit=maxit,
                                   fixed_iters=fixed_iters)
    eps = macro_tensor(eps_mac, dim, grid) + _mat.sym(x)
    el = eps - eigen_tensor(e, dim, grid)
    sig = _mat.stress(el, glam, gmu)
    out = dict(
        strain=_mat.to_voigt(eps),
        stress=_mat.to_voigt(sig),
        mean_stress=np.array([np.mean(s) for s in _mat.to_voigt(sig)]),
        energy=0.5 * h ** dim * float(np.sum(el * sig)),
        iters=iters, rel_res=rel, status=status, bnorm=np.sqrt(np.sum(b * b)),
    )
    if return_x:
        out["x"] = x
        out["b"] = b
    return out


def mech_residual(strain_voigt, phase, E_tab, nu_tab, h, d=None, kappa=0.0,
                  e=None, E_field=None, nu=None):
    """||G[g C:(eps - e I)]|| / ||G[g C:(<eps> - e I)]|| for a given total strain.

    A size-independent property check: the projected stress vanishes at the
    solution, relative to the right-hand side of the linear system.
    """
    phase = np.asarray(phase)
    grid = phase.shape
    dim = phase.ndim
    lam, mu = voxel_lame(phase, E_tab, nu_tab, E_field, nu)
    g = np.ones(grid) if d is None else _mat.degradation(np.asarray(d), kappa)
    D = _sp.grad_symbols(grid, h)
    eps = _mat.from_voigt(np.asarray(strain_voigt), dim)
    el = eps - eigen_tensor(e, dim, grid)
    res = mech_operator(el, g * lam, g * mu, D, "full")
    mac = np.array([np.mean(c) for c in np.asarray(strain_voigt)])
    E0 = macro_tensor(mac, dim, grid) - eigen_tensor(e, dim, grid)
    b = mech_operator(E0, g * lam, g * mu, D, "full")
    return float(np.sqrt(np.sum(res * res)) / max(np.sqrt(np.sum(b * b)), 1e-300))
