"""Pins of the oracle's DFT, gradient symbols and projections (CPU only).

FFT: brute-force double sums on tiny inputs, round trip, Parseval, and the
library ``numpy.fft`` as an independent check.  Symbols: the inverse transform
of D_a f_hat equals the periodic forward-difference stencil of Sec. 2.6.
Projections (App. A): idempotent, self-adjoint, identity on gradients, zero on
constants, real output for real input.
"""
import numpy as np
import pytest

from oracle import fft, spectral as sp

SIZES = [1, 2, 3, 4, 5, 6, 8, 9, 12, 16, 24, 32, 48, 64, 96]


def brute_dft(x, sign):
    n = len(x)
    out = []
    for k in range(n):
        s = 0j
        for j in range(n):
            s += x[j] * complex(np.cos(2 * np.pi * k * j / n), sign * np.sin(2 * np.pi * k * j / n))
        out.append(s)
    return np.array(out)


@pytest.mark.parametrize("n", SIZES)
def test_fft_matches_brute_force(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert np.allclose(fft.fft(x), brute_dft(x, -1), rtol=0, atol=1e-12 * max(1, n))
    assert np.allclose(fft.ifft(x) * n, brute_dft(x, +1), rtol=0, atol=1e-12 * max(1, n))


@pytest.mark.parametrize("n", [8, 12, 64, 384, 1024])
def test_fft_round_trip_parseval_and_library(n):
    rng = np.random.default_rng(7 + n)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    X = fft.fft(x, axis=-1)
    assert np.max(np.abs(fft.ifft(X, axis=-1) - x)) < 1e-13
    assert np.allclose(np.sum(np.abs(X) ** 2, axis=-1) / n, np.sum(np.abs(x) ** 2, axis=-1), rtol=1e-13)
    assert np.max(np.abs(X - np.fft.fft(x, axis=-1))) < 1e-12 * np.sqrt(n) * np.max(np.abs(X))


def test_fft_axis_handling():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((6, 8, 12))
    assert np.allclose(fft.fftn(x, (0, 1, 2)), np.fft.fftn(x), atol=1e-12)
    assert np.allclose(fft.fft(x, axis=1), np.fft.fft(x, axis=1), atol=1e-12)


def _stencil(f, alpha, h):
    axis = f.ndim - 1 - alpha
    return (np.roll(f, -1, axis=axis) - f) / h


@pytest.mark.parametrize("grid", [(8, 8), (6, 10), (4, 6, 8)])
def test_forward_difference_symbol_is_stencil(grid):
    rng = np.random.default_rng(11)
    f = rng.standard_normal(grid)
    h = 0.37
    D = sp.grad_symbols(grid, h)
    axes = tuple(range(len(grid)))
    fh = fft.fftn(f, axes)
    for a in range(len(grid)):
        g = fft.ifftn(D[a] * fh, axes)
        assert np.max(np.abs(g.imag)) < 1e-12
        assert np.allclose(g.real, _stencil(f, a, h), atol=1e-12)


def _rand_tensor(grid, dim, rng, symmetric=False):
    t = rng.standard_normal((dim, dim) + grid)
    if symmetric:
        t = 0.5 * (t + np.swapaxes(t, 0, 1))
    return t


def _apply(proj, t, D):
    dim = D.shape[0]
    axes = tuple(range(-dim, 0))
    return fft.ifftn(proj(fft.fftn(t, axes), D), axes)


@pytest.mark.parametrize("grid", [(8, 8), (6, 8), (4, 6, 8)])
@pytest.mark.parametrize("kind", ["full", "sym"])
def test_projection_properties(grid, kind):
    rng = np.random.default_rng(5)
    dim = len(grid)
    h = 0.5
    D = sp.grad_symbols(grid, h)
    proj = sp.project_full if kind == "full" else sp.project_sym
    a = _rand_tensor(grid, dim, rng, symmetric=(kind == "sym"))
    b = _rand_tensor(grid, dim, rng, symmetric=(kind == "sym"))
    Ga = _apply(proj, a, D)
    # real output for real input
    assert np.max(np.abs(Ga.imag)) < 1e-12
    Ga = Ga.real
    # idempotent
    assert np.max(np.abs(_apply(proj, Ga, D).real - Ga)) < 1e-12 * np.max(np.abs(Ga))
    # self-adjoint in the Frobenius inner product
    Gb = _apply(proj, b, D).real
    assert abs(np.sum(Ga * b) - np.sum(a * Gb)) < 1e-12 * np.sum(np.abs(a * b))
    # constants are annihilated
    c = np.zeros_like(a)
    c[0, 0] += 1.7
    c[1, 1] -= 0.4
    assert np.max(np.abs(_apply(proj, c, D))) < 1e-12
    # gradients of periodic fields are left unchanged
    u = rng.standard_normal((dim,) + grid)
    gu = np.array([[_stencil(u[i], j, h) for j in range(dim)] for i in range(dim)])
    if kind == "sym":
        gu = 0.5 * (gu + np.swapaxes(gu, 0, 1))
    assert np.max(np.abs(_apply(proj, gu, D).real - gu)) < 1e-11 * np.max(np.abs(gu))


def test_vector_projection_and_inverse_gradient():
    rng = np.random.default_rng(9)
    grid = (8, 12)
    h = 0.25
    D = sp.grad_symbols(grid, h)
    axes = (1, 2)
    f = rng.standard_normal((2,) + grid)
    Gf = fft.ifftn(sp.project_vector(fft.fftn(f, axes), D), axes)
    assert np.max(np.abs(Gf.imag)) < 1e-12
    # the projected field is the gradient of phi = (iXi)^-1 . f  (eq. g-42)
    phi_hat = np.sum(sp.inverse_gradient(D) * fft.fftn(f, axes), axis=0)
    phi = fft.ifftn(phi_hat, (0, 1)).real
    for a in range(2):
        assert np.allclose(Gf.real[a], _stencil(phi, a, h), atol=1e-12)
    # least squares: the residual is orthogonal to every gradient
    u = rng.standard_normal(grid)
    gu = np.array([_stencil(u, a, h) for a in range(2)])
    assert abs(np.sum((f - Gf.real) * gu)) < 1e-10


# --------------------------------------------------------------------------
# Gradient operators of Sec. 2.6 (the Gibbs-ringing comparison)

@pytest.mark.parametrize("op", ["central", "central8"])
def test_difference_symbols_are_their_stencils(op):
    from oracle import direct
    grid, h = (10, 14), 0.3
    f = np.random.default_rng(4).standard_normal(grid)
    D = sp.grad_symbols(grid, h, op)
    for a in range(2):
        via_fft = fft.ifftn(D[a] * fft.fftn(f, (0, 1)), (0, 1)).real
        stencil = (direct.diff_matrix(grid, a, h, op) @ f.ravel()).reshape(grid)
        assert np.max(np.abs(via_fft - stencil)) < 1e-12 * np.max(np.abs(stencil))


@pytest.mark.parametrize("n", [9, 16])
def test_fourier_symbol_exact_on_trig_polynomials(n):
    from oracle import direct
    h = 0.1
    L = n * h
    x = h * np.arange(n)
    f = np.sin(2 * np.pi * 2 * x / L) + 0.5 * np.cos(2 * np.pi * 3 * x / L)
    df = (2 * np.pi / L) * (2 * np.cos(2 * np.pi * 2 * x / L) - 1.5 * np.sin(2 * np.pi * 3 * x / L))
    D = sp.diff_symbol_1d(n, h, "fourier")
    got = fft.ifftn(D * fft.fftn(f, (0,)), (0,)).real
    assert np.max(np.abs(got - df)) < 1e-12 * np.max(np.abs(df))
    # the closed-form differentiation matrix agrees (independent of the transform)
    M = direct.diff_matrix((1, n), 0, h, "fourier").toarray()
    assert np.max(np.abs(M @ f - df)) < 1e-11 * np.max(np.abs(df))


def test_central8_is_eighth_order():
    errs = []
    for n in (16, 32):
        h = 1.0 / n
        x = h * np.arange(n)
        f = np.sin(2 * np.pi * x)
        df = 2 * np.pi * np.cos(2 * np.pi * x)
        D = sp.diff_symbol_1d(n, h, "central8")
        errs.append(np.max(np.abs(fft.ifftn(D * fft.fftn(f, (0,)), (0,)).real - df)))
    assert errs[0] / errs[1] > 240  # 2^8 = 256


@pytest.mark.parametrize("op", ["central", "central8", "fourier"])
def test_operator_variants_reach_their_direct_solutions(op):
    """Mechanics (symmetric storage) and the diffusion homogenisation with each
    operator against least-squares solves of the real-space systems built
    from the difference matrices (odd grid: the central operators have no
    spurious Nyquist null modes there)."""
    from oracle import direct, homogenisation as hm, mech
    grid = (9, 15)
    rng = np.random.default_rng(5)
    phase = (rng.random(grid) < 0.6).astype(np.uint8)
    e = 1e-3 * (phase == 0)
    em = (1e-3, -2e-4, 3e-4)
    r = mech.mech_solve(phase, (3e7, 30e9), (0.2, 0.2), em, 5e-6, e=e, tol=1e-14, maxit=20000, storage="sym", op=op)
    q = direct.mech_direct_op(phase, (3e7, 30e9), (0.2, 0.2), em, 5e-6, op, e=e)
    assert np.linalg.norm(r["strain"] - q["strain"]) < 1e-10 * np.linalg.norm(q["strain"])
    Df = np.where(phase == 0, 1e-9, 1e-11)
    g = hm.diffusion_homogenise(Df, (0.6, -0.3), 5e-6, tol=1e-14, maxit=20000, op=op)["grad_c"]
    gd = direct.diffusion_static_direct_op(Df, (0.6, -0.3), 5e-6, op)
    assert np.linalg.norm(g - gd) < 1e-10 * np.linalg.norm(gd)
