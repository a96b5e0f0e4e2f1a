"""Gradient symbols and compatibility projections (test infrastructure).

Grid convention: a scalar field on an n_y x n_x grid is an array of shape
(n_y, n_x) (3D: (n_z, n_y, n_x)); spatial direction alpha = 0 is x, the LAST
array axis.  Tensor fields carry their tensor indices first: a second-order
field has shape (dim, dim) + grid, index [i, j] meaning component x_i x_j.

* Forward-difference gradient symbol, Sec. 2.6: D_a(k) = (exp(i theta_a) - 1)/h
  with theta_a = 2 pi k_a / n_a, which is the transform of the stencil
  (f(x + h e_a) - f(x)) / h under the forward DFT sign of ``oracle.fft``.
  The other operators of Sec. 2.6 (the Gibbs-ringing comparison):
  "central": i sin(theta)/h, the transform of (f(x + h) - f(x - h)) / (2 h)
  (the printed form "(i sin(xi Delta) - 1)/Delta" is read as this);
  "central8": the eighth-order central difference,
  sum_{m=1..4} a_m (f(x + m h) - f(x - m h)) / h with
  a = (4/5, -1/5, 4/105, -1/280), symbol (2 i / h) sum a_m sin(m theta);
  "fourier": i xi = i 2 pi k / (n h) with the signed wavenumber k in
  (-n/2, n/2), zero at the Nyquist wavenumber of even n.
* Inverse gradient, App. A eq. g-42: (iXi)^{-1} = conj(D) / (D . conj(D)),
  zero where D . conj(D) = 0.
* Vector projection, App. A: A_i = g_ij f_j with g_ij = D_i (iXi)^{-1}_j.
* Fourth-order projection on full displacement gradients, App. A:
  A_ij = delta_im g_jl eps_ml, i.e. each row of the gradient is projected
  with the vector projection.
* Symmetric-strain projection: the orthogonal projection (Frobenius inner
  product) of a symmetric tensor onto {sym(u (x) D)}, obtained from the normal
  equations; used for 6-component storage in 3D.
"""
import numpy as np


CENTRAL8 = (4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0)
OPERATORS = ("forward", "central", "central8", "fourier")


def diff_symbol_1d(n, h, op="forward"):
    """Gradient symbol on n points of spacing h for the operators of Sec. 2.6."""
    k = np.arange(n)
    theta = 2.0 * np.pi * k / n
    if op == "forward":
        return (np.exp(1j * theta) - 1.0) / h
    # sin(m theta) is exactly zero where 2 m k is a multiple of n (k = 0 and
    # the Nyquist wavenumber): set so, rather than the rounding of sin(pi)
    sinm = lambda m: np.where((2 * m * k) % n == 0, 0.0, np.sin(m * theta))
    if op == "central":
        return 1j * sinm(1) / h
    if op == "central8":
        return 2j * sum(a * sinm(m + 1) for m, a in enumerate(CENTRAL8)) / h
    if op == "fourier":
        ks = np.where(k < (n + 1) // 2, k, k - n).astype(np.float64)
        if n % 2 == 0:
            ks[n // 2] = 0.0
        return 1j * 2.0 * np.pi * ks / (n * h)
    raise ValueError(op)


def grad_symbols(grid_shape, h, op="forward"):
    """D_alpha over the whole grid, shape (dim,) + grid; alpha = 0 is x."""
    dim = len(grid_shape)
    out = []
    for alpha in range(dim):
        axis = dim - 1 - alpha
        shape = [1] * dim
        shape[axis] = grid_shape[axis]
        d1 = diff_symbol_1d(grid_shape[axis], h, op).reshape(shape)
        out.append(np.broadcast_to(d1, grid_shape))
    return np.array(out)


def norm2(D):
    return np.sum(np.abs(D) ** 2, axis=0)


def inverse_gradient(D):
    """App. A eq. g-42: conj(D)/|D|^2, zero where |D|^2 = 0."""
    n2 = norm2(D)
    safe = np.where(n2 > 0, n2, 1.0)
    return np.where(n2 > 0, np.conj(D) / safe, 0.0)


def project_vector(f_hat, D):
    """Vector projection: out_i = D_i sum_j (iXi)^{-1}_j f_j."""
    inv = inverse_gradient(D)
    s = np.sum(inv * f_hat, axis=0)
    return D * s


def project_full(t_hat, D):
    """Fourth-order projection on a full (dim x dim) gradient field.

    out_ij = D_j * sum_l (iXi)^{-1}_l t_il: row i is projected as a vector.
    """
    dim = D.shape[0]
    out = np.empty_like(t_hat, dtype=np.complex128)
    for i in range(dim):
        out[i] = project_vector(t_hat[i], D)
    return out


def project_sym(t_hat, D):
    """Orthogonal projection of a symmetric tensor field onto sym(u (x) D).

    The normal equations  t conj(D) = sym(u (x) D) conj(D)  read
    (|D|^2/2) u + (D/2) (D^H u) = t conj(D); contracting with D^H gives
    D^H u = D^H t_c / |D|^2 with t_c = t conj(D), hence
    u = (2/|D|^2) [t_c - D (D^H t_c) / (2 |D|^2)], and the output is
    sym(u (x) D).  Zero where |D|^2 = 0.
    """
    dim = D.shape[0]
    n2 = norm2(D)
    safe = np.where(n2 > 0, n2, 1.0)
    tc = np.einsum("ij...,j...->i...", t_hat, np.conj(D))
    dhtc = np.sum(np.conj(D) * tc, axis=0)
    u = (2.0 / safe) * (tc - D * dhtc / (2.0 * safe))
    u = np.where(n2 > 0, u, 0.0)
    out = np.empty((dim, dim) + D.shape[1:], dtype=np.complex128)
    for i in range(dim):
        for j in range(dim):
            out[i, j] = 0.5 * (u[i] * D[j] + u[j] * D[i])
    return out
