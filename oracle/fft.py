"""Naive recursive mixed-radix discrete Fourier transform (test infrastructure).

The paper evaluates every convolution with the projection operator in Fourier
space (Sec. 2.1, eq. diffusion-final; Sec. 2.3, eq. solid-final).  This module
is the plain definition of that transform:

    forward   f_hat(k) = sum_x f(x) exp(-2 pi i k x / n)
    inverse   f(x)     = (1/n) sum_k f_hat(k) exp(+2 pi i k x / n)

computed by Cooley-Tukey decimation in time that splits off the smallest prime
factor of n and falls back to the O(n^2) sum when n is prime.  No blocking, no
real-to-complex packing and no twiddle tables: every twiddle is evaluated from
its definition.  Vectorised over all axes but the transformed one.
"""
import numpy as np


def _smallest_prime_factor(n):
    f = 2
    while f * f <= n:
        if n % f == 0:
            return f
        f += 1
    return n


def dft_direct(a, sign=-1):
    """O(n^2) DFT along the last axis, straight from the definition."""
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[-1]
    k = np.arange(n)
    w = np.exp(sign * 2j * np.pi * np.outer(k, k) / n)
    return a @ w.T


def _fft_last(a, sign):
    n = a.shape[-1]
    if n == 1:
        return np.array(a, dtype=np.complex128, copy=True)
    p = _smallest_prime_factor(n)
    if p == n:
        return dft_direct(a, sign)
    m = n // p
    # X[k] = sum_r exp(sign 2 pi i r k / n) * DFT_m(a[r::p])[k mod m]
    subs = [_fft_last(a[..., r::p], sign) for r in range(p)]
    k = np.arange(n)
    out = np.zeros(a.shape[:-1] + (n,), dtype=np.complex128)
    for r in range(p):
        out += np.exp(sign * 2j * np.pi * r * k / n) * subs[r][..., k % m]
    return out


def fft(a, axis=-1):
    a = np.moveaxis(np.asarray(a, dtype=np.complex128), axis, -1)
    return np.moveaxis(_fft_last(a, -1), -1, axis)


def ifft(a, axis=-1):
    a = np.moveaxis(np.asarray(a, dtype=np.complex128), axis, -1)
    n = a.shape[-1]
    return np.moveaxis(_fft_last(a, +1) / n, -1, axis)


def fftn(a, axes):
    out = np.asarray(a, dtype=np.complex128)
    for ax in axes:
        out = fft(out, ax)
    return out


def ifftn(a, axes):
    out = np.asarray(a, dtype=np.complex128)
    for ax in axes:
        out = ifft(out, ax)
    return out
