"""Static diffusion homogenisation and concentration reconstruction (test infrastructure).

Sec. 2.1 solves the static diffusion problem on the representative volume in
gradient-primary form.  With the flux j = -D(x) grad c and D(x) defined point
by point through the phase indicator, eq. diffusion asks for div j = 0 with
<grad c> = grad c_mac.  Eq. diffusion-weak-form and eq. diffusion-final turn
this into: find the compatible fluctuation x of the concentration gradient
(x in the range of the vector projection G of App. A, built from the
forward-difference symbol of Sec. 2.6) such that

    G[ D (grad c_mac + x) ] = 0,   i.e.   G[D x] = -G[D grad c_mac],

a symmetric linear system on compatible fields that CG solves (the diffusion
block of Alg. 1; the problem is linear, so its Newton loop ends after the
first linear solve).  Then grad c = grad c_mac + x (eq. micro-gradient).

Concentration reconstruction, eqs. micro-gradient to concentration-correct:
the periodic fluctuation phi has grad phi = x, so in Fourier space
phi_hat = (iXi)^-1 . (grad c)_hat with the inverse gradient of eq. g-42 (the
constant grad c_mac only has the k = 0 mode, where the inverse gradient is
zero; this is the Fourier form of eq. phi-fft and of the "periodic
fluctuations" line of Alg. 1).  Then c(x) = grad c_mac . x + phi(x) + beta with
one constant per phase (eq. psi-two-values): beta_pore makes the pore mean
c_mac / eta, beta_solid makes the solid mean zero.

Effective diffusivity: <j> = -D_eff grad c_mac, so column a of D_eff is
-<j> for grad c_mac = e_a (the quantity of the sensitivity study of App. B).

Readings (the paper does not fix them):
* the position x of voxel (i_x, i_y, ...) is (i_x h, i_y h, ...): the origin
  at voxel 0, one grid spacing per index;
* phase 0 is pore (omega = 0), every other phase is solid (omega = 1).
"""
import numpy as np

from . import cg as _cg
from . import fft as _fft
from . import spectral as _sp


def _axes(dim):
    return tuple(range(-dim, 0))


def macro_gradient_field(grad_cmac, grid):
    dim = len(grid)
    g = np.zeros((dim,) + tuple(grid))
    for a in range(dim):
        g[a] = grad_cmac[a]
    return g


def projected_flux_operator(x, Dfield, D):
    """x -> G[D x] for a vector field x (components first), eq. diffusion-final."""
    dim = D.shape[0]
    j_hat = _fft.fftn(Dfield[None] * x, _axes(dim))
    return _fft.ifftn(_sp.project_vector(j_hat, D), _axes(dim)).real


def diffusion_homogenise(Dfield, grad_cmac, h, tol=1e-10, maxit=20000, fixed_iters=None, op="forward"):
    """Projected CG for the compatible gradient fluctuation (Sec. 2.1).

    Returns grad_c (dim, *grid), the flux j = -D grad c, its mean, the CG
    iteration count, the final relative residual and the status."""
    Dfield = np.asarray(Dfield, dtype=np.float64)
    grid = Dfield.shape
    D = _sp.grad_symbols(grid, h, op)
    g0 = macro_gradient_field(grad_cmac, grid)
    A = lambda v: projected_flux_operator(v, Dfield, D)
    b = -A(g0)
    x, iters, rel, status = _cg.cg(A, b, tol=tol, maxit=maxit, fixed_iters=fixed_iters)
    grad_c = g0 + x
    flux = -Dfield[None] * grad_c
    return dict(grad_c=grad_c, flux=flux, mean_flux=np.array([np.mean(f) for f in flux]),
                iters=iters, rel_res=rel, status=status)


def fluctuation_from_gradient(grad_c, h, op="forward"):
    """phi with grad phi = the fluctuation of grad_c (eq. phi-fft through the
    inverse gradient of eq. g-42); mean zero."""
    grad_c = np.asarray(grad_c, dtype=np.float64)
    dim = grad_c.shape[0]
    D = _sp.grad_symbols(grad_c.shape[1:], h, op)
    g_hat = _fft.fftn(grad_c, _axes(dim))
    phi_hat = np.sum(_sp.inverse_gradient(D) * g_hat, axis=0)
    return _fft.ifftn(phi_hat, _axes(dim)).real


def position_dot(grad_cmac, grid, h):
    """grad c_mac . x with x = voxel index times h (origin at voxel 0)."""
    dim = len(grid)
    out = np.zeros(grid)
    for a in range(dim):
        axis = dim - 1 - a
        shape = [1] * dim
        shape[axis] = grid[axis]
        out = out + grad_cmac[a] * h * np.arange(grid[axis]).reshape(shape)
    return out


def concentration(phase, grad_c, grad_cmac, c_mac, h, op="forward"):
    """c(x) = grad c_mac . x + phi(x) + beta_phase (eqs. concentration,
    psi-two-values, concentration-correct).  Returns c, phi, beta_pore,
    beta_solid."""
    phase = np.asarray(phase)
    grid = phase.shape
    pore = phase == 0
    solid = ~pore
    eta = float(np.mean(pore))
    phi = fluctuation_from_gradient(grad_c, h, op)
    lin = position_dot(grad_cmac, grid, h)
    beta_pore = (c_mac / eta - float(np.mean(lin[pore])) - float(np.mean(phi[pore]))) if pore.any() else 0.0
    beta_solid = (-float(np.mean(lin[solid])) - float(np.mean(phi[solid]))) if solid.any() else 0.0
    c = lin + phi + np.where(pore, beta_pore, beta_solid)
    return dict(c=c, phi=phi, beta_pore=beta_pore, beta_solid=beta_solid)


def effective_diffusivity(Dfield, h, tol=1e-12, maxit=20000, op="forward"):
    """D_eff with <j> = -D_eff grad c_mac, one homogenisation per axis."""
    Dfield = np.asarray(Dfield, dtype=np.float64)
    dim = Dfield.ndim
    Deff = np.zeros((dim, dim))
    iters = []
    for a in range(dim):
        e = np.zeros(dim)
        e[a] = 1.0
        r = diffusion_homogenise(Dfield, e, h, tol=tol, maxit=maxit, op=op)
        Deff[:, a] = -r["mean_flux"]
        iters.append(r["iters"])
    return Deff, iters
