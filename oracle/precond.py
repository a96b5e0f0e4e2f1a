"""Displacement-form preconditioned CG for the mechanics, with the Green
operator of a unit or an isotropic reference medium (test infrastructure).

The compatible strain fluctuations of Sec. 2.3 with the forward-difference
gradient of Sec. 2.6 are exactly the discrete symmetric gradients of periodic
displacements, and the projection of App. A factors through the
displacement.  The equilibrium problem of eq. solid-final is then

    K u = f,   K = L^T g C L,   f = -L^T g C (eps_mac - e I),

with L u = sym(grad u) (the sparse stencil matrices of ``oracle.direct``, no
transform).  CG on K preconditioned with M is:

* M = (grad^H grad)^-1 per component ("unit" medium): iterate by iterate the
  projected CG of the paper on the strain (same alpha, beta, residual norms);
* M = K0^-1 with K0 the stiffness of a homogeneous isotropic reference medium
  (lam0, mu0): in Fourier space a dim x dim Hermitian matrix per mode,
  K0(k) = mu0 |D|^2 I + lam0 conj(D) D^T + mu0 D D^H, inverted mode by mode
  (zero at k = 0).  For a medium close to the reference this is close to the
  inverse of K; the paper names the property contrast as what limits the
  efficiency of its solver (Sec. 5).

M is applied with the transforms of ``oracle.fft``; the mean (k = 0) of the
displacement is irrelevant and stays zero.
"""
import numpy as np

from . import cg as _cg
from . import direct as _direct
from . import fft as _fft
from . import material as _mat
from . import mech as _mech
from . import spectral as _sp


def _axes(dim):
    return tuple(range(-dim, 0))


def reference_stiffness_symbol(D, lam0, mu0):
    """K0(k) as an array (dim, dim, *grid): mu0 |D|^2 I + lam0 conj(D) D^T + mu0 D D^H."""
    dim = D.shape[0]
    n2 = _sp.norm2(D)
    K0 = np.zeros((dim, dim) + D.shape[1:], dtype=np.complex128)
    for i in range(dim):
        for j in range(dim):
            K0[i, j] = lam0 * np.conj(D[i]) * D[j] + mu0 * D[i] * np.conj(D[j])
        K0[i, i] = K0[i, i] + mu0 * n2
    return K0


def apply_green(r, D, lam0=None, mu0=None):
    """z = M r for a displacement-like field r (dim, *grid): the unit Green
    operator (lam0 None) or the reference-medium one."""
    dim = D.shape[0]
    r_hat = _fft.fftn(r, _axes(dim))
    n2 = _sp.norm2(D)
    nz = n2 > 0
    z_hat = np.zeros_like(r_hat)
    if lam0 is None:
        z_hat[:, nz] = r_hat[:, nz] / n2[nz]
    else:
        K0 = reference_stiffness_symbol(D, lam0, mu0)
        A = np.moveaxis(K0[:, :, nz], -1, 0)          # (m, dim, dim)
        rhs = np.moveaxis(r_hat[:, nz], -1, 0)[..., None]
        z_hat[:, nz] = np.moveaxis(np.linalg.solve(A, rhs)[..., 0], 0, -1)
    return _fft.ifftn(z_hat, _axes(dim)).real


def mech_pcg(phase, E_tab, nu_tab, eps_mac, h, d=None, kappa=0.0, e=None, E_field=None, nu=None,
             reference=None, tol=1e-10, maxit=20000, fixed_iters=None):
    """Displacement-form PCG.  reference: None for the unit Green operator or
    (lam0, mu0) of the isotropic reference medium.  Returns the total strain
    (Voigt), the displacement, iterations, residual and status."""
    phase = np.asarray(phase)
    grid = phase.shape
    dim = phase.ndim
    lam, mu = _mech.voxel_lame(phase, E_tab, nu_tab, E_field, nu)
    g = np.ones(grid) if d is None else _mat.degradation(np.asarray(d), kappa)
    C = _direct._stiffness_matrix(g * lam, g * mu)
    L = _direct._symgrad_matrix(grid, h)
    E0 = _mech.macro_tensor(eps_mac, dim, grid) - _mech.eigen_tensor(e, dim, grid)
    f = -(L.T @ (C @ E0.reshape(-1))).reshape((dim,) + grid)
    A = lambda u: (L.T @ (C @ (L @ u.reshape(-1)))).reshape((dim,) + grid)
    D = _sp.grad_symbols(grid, h)
    lam0, mu0 = (None, None) if reference is None else reference
    M = lambda r: apply_green(r, D, lam0, mu0)
    u, iters, rel, status = _cg.pcg(A, M, f, tol=tol, maxit=maxit, fixed_iters=fixed_iters)
    eps = _mech.macro_tensor(eps_mac, dim, grid) + (L @ u.reshape(-1)).reshape((dim, dim) + grid)
    return dict(strain=_mat.to_voigt(eps), u=u, iters=iters, rel_res=rel, status=status)
