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
