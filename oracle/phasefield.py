"""AT2 hybrid phase-field damage solve (test infrastructure).

Sec. 2.4, eq. crack and eq. crack-fft:

    -(Gc l0 / 2) lap(d) + (Gc / (2 l0)) d + H d = H,

with the Laplacian applied in Fourier space.  With the forward-difference
gradient D of Sec. 2.6 the Laplacian symbol is taken as -D^H D = -|D|^2 (the
reading that keeps the operator symmetric positive definite),
so the operator is

    A d = (Gc / (2 l0) + H) d + (Gc l0 / 2) F^-1[ |D|^2 F[d] ],

solved by CG from the previous damage field (the paper names GMRES; on an SPD
operator CG reaches the same solution).  H is the history field
H = max over time of psi+ (Sec. 2.4).
"""
import numpy as np

from . import cg as _cg
from . import fft as _fft
from . import spectral as _sp


def pf_operator(d, H, Gc, l0, n2):
    dim = d.ndim
    axes = tuple(range(-dim, 0))
    lap = _fft.ifftn(n2 * _fft.fftn(d, axes), axes).real
    return (Gc / (2.0 * l0) + H) * d + 0.5 * Gc * l0 * lap


def phasefield_solve(H, Gc, l0, h, d0=None, tol=1e-10, maxit=20000,
                     fixed_iters=None, op="forward"):
    H = np.asarray(H, dtype=np.float64)
    n2 = _sp.norm2(_sp.grad_symbols(H.shape, h, op))
    A = lambda v: pf_operator(v, H, Gc, l0, n2)
    x, iters, rel, status = _cg.cg(A, H.copy(), x0=d0, tol=tol, maxit=maxit,
                                   fixed_iters=fixed_iters)
    return dict(d=x, iters=iters, rel_res=rel, status=status)
