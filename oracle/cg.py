"""Textbook conjugate gradients (test infrastructure).

The paper solves each discretised linear problem with "a linear iterative
solver" (Sec. 2.1 after eq. diffusion-final; Sec. 2.3; Alg. 1).  The operators
used here are symmetric positive (semi-)definite on the space the iterates
live in, so this is plain Hestenes-Stiefel CG with the stopping rule
||r_k|| <= tol ||b||, checked before every iteration.

Status codes: 0 converged, 1 iteration limit reached, -3 breakdown
(p.Ap <= 0 or a non-finite scalar).
"""
import numpy as np


def frob(a, b):
    return float(np.sum(a * b))


def cg(apply_A, b, x0=None, tol=1e-10, maxit=10000, fixed_iters=None,
       inner=frob):
    bnorm = np.sqrt(inner(b, b))
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0, 0
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = np.array(x0, dtype=np.float64, copy=True)
        r = b - apply_A(x)
    p = r.copy()
    rr = inner(r, r)
    k = 0
    limit = maxit if fixed_iters is None else fixed_iters
    status = 0
    while True:
        if fixed_iters is None and np.sqrt(rr) <= tol * bnorm:
            status = 0
            break
        if k >= limit:
            status = 1 if fixed_iters is None else 0
            break
        q = apply_A(p)
        pq = inner(p, q)
        if not (np.isfinite(pq) and pq > 0.0):
            status = -3
            break
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = inner(r, r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        k += 1
    return x, k, float(np.sqrt(rr) / bnorm), status


def pcg(apply_A, apply_M, b, tol=1e-10, maxit=10000, fixed_iters=None, inner=frob):
    """Textbook preconditioned CG from x = 0.  The stopping rule measures the
    preconditioned residual, r.M r <= tol^2 r0.M r0, checked before every
    iteration (for the projected systems of the paper with the unit Green
    operator as M this is the norm of the projected residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_M(r)
    rz = inner(r, z)
    rz0 = rz
    if rz0 == 0.0:
        return x, 0, 0.0, 0
    p = z.copy()
    k = 0
    limit = maxit if fixed_iters is None else fixed_iters
    status = 0
    while True:
        if fixed_iters is None and rz <= tol * tol * rz0:
            status = 0
            break
        if k >= limit:
            status = 1 if fixed_iters is None else 0
            break
        q = apply_A(p)
        pq = inner(p, q)
        if not (np.isfinite(pq) and pq > 0.0):
            status = -3
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        z = apply_M(r)
        rz_new = inner(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        k += 1
    return x, k, float(np.sqrt(max(rz, 0.0) / rz0)), status
