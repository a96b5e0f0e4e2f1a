"""Transient heterogeneous diffusion-reaction step (test infrastructure).

Flux j = -D(x) grad c with D mixed per phase (Sec. 2.1); the gradient is the
forward difference of Sec. 2.6, so the divergence is its adjoint,
-div = D^H.  One backward-Euler step of dc/dt = div(D grad c) - k_r(x) c reads

    A c = (1/dt + k_r(x)) c + sum_a F^-1[ conj(D_a) F[ D(x) F^-1[ D_a F[c] ] ] ]
        = c^n / dt,

with k_r = k in pores and 0 in the solid (first-order precipitation sink).
Voxels in the Dirichlet band keep c = c_dir: the CG unknowns are the free
voxels, the operator is M A M with M the free-voxel mask, the right-hand side
is b_F = M (c^n/dt - A c_B) with c_B = c_dir on the band, and CG starts from
M c^n.  With no band, M = I.
"""
import numpy as np

from . import cg as _cg
from . import fft as _fft
from . import spectral as _sp


def diffusion_operator(c, Dfield, react, dt, D):
    dim = c.ndim
    axes = tuple(range(-dim, 0))
    c_hat = _fft.fftn(c, axes)
    div = np.zeros(c.shape)
    for a in range(dim):
        grad_a = _fft.ifftn(D[a] * c_hat, axes).real
        j_hat = _fft.fftn(Dfield * grad_a, axes)
        div += _fft.ifftn(np.conj(D[a]) * j_hat, axes).real
    return (1.0 / dt + react) * c + div


def diffusion_step(c_n, Dfield, react, dt, h, band=None, c_dir=1.0,
                   tol=1e-10, maxit=20000, fixed_iters=None, op="forward"):
    c_n = np.asarray(c_n, dtype=np.float64)
    D = _sp.grad_symbols(c_n.shape, h, op)
    if band is None:
        M = np.ones(c_n.shape)
        cB = np.zeros(c_n.shape)
    else:
        band = np.asarray(band, dtype=bool)
        M = (~band).astype(np.float64)
        cB = np.where(band, c_dir, 0.0)
    A = lambda v: M * diffusion_operator(M * v, Dfield, react, dt, D)
    b = M * (c_n / dt - diffusion_operator(cB, Dfield, react, dt, D))
    x, iters, rel, status = _cg.cg(A, b, x0=M * c_n, tol=tol, maxit=maxit,
                                   fixed_iters=fixed_iters)
    return dict(c=M * x + cB, iters=iters, rel_res=rel, status=status)
