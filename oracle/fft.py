"""Discrete Fourier transforms for the oracle (plain, slow, FP64).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.

Conventions (paper, "Numerical results": box of side 2*pi, Fourier spectral
discretisation with periodic boundaries; the spectral sub-steps of the
time-evolution section):

* grid ``x_j = 2*pi*j/N``, integer wavenumbers in "fftfreq" order
  ``0, 1, ..., N/2-1, -N/2, ..., -1`` (for even N the index N/2 is the
  Nyquist mode and carries k = -N/2);
* forward transform ``c_k = N^-d * sum_x f(x) exp(-i k.x)`` (normalised);
* inverse transform ``f(x) = sum_k c_k exp(+i k.x)``.

Two independent 1-D engines are provided (and, for measuring the FP64 floor
between correct implementations only, ``library_engine``):

* ``dft_axis``   -- the definition itself: a dense N x N matrix
  ``W[j, k] = exp(-2*pi*i*((j*k) mod N)/N)`` applied along one axis, O(N^2);
* ``fft_axis``   -- a straightforward recursive mixed-radix (2, 3, general
  prime) Cooley-Tukey FFT, vectorised over the other axes.

``fft3``/``ifft3`` pick the dense DFT for N <= 64 and the FFT above, or the
engine named by ``engine=``.  ``engine`` may also be a callable
``engine(a, axis, sign)`` that returns the unnormalised 1-D transform along
``axis``; it exists so that a driver can split the independent pencils of one
transform over several processes (each process still calling ``transform_axis``
with the default rule), which leaves every value unchanged.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "kvec", "dft_axis", "fft_axis", "transform_axis", "fft3", "ifft3",
    "fftn_unnorm", "ifftn_unnorm", "smallest_factor",
]

NAIVE_MAX = 64


def kvec(n: int) -> np.ndarray:
    """Integer wavenumbers of an n-point periodic grid on [0, 2*pi), fftfreq order."""
    j = np.arange(n, dtype=np.int64)
    return np.where(j < (n + 1) // 2, j, j - n) if n % 2 else np.where(j < n // 2, j, j - n)


def _unit_roots(n: int, sign: int) -> np.ndarray:
    """exp(sign * 2*pi*i*m/n) for m = 0..n-1 (FP64, m already reduced mod n)."""
    m = np.arange(n, dtype=np.float64)
    return np.exp(sign * 2j * np.pi * m / n)


def dft_axis(a: np.ndarray, axis: int, sign: int = -1) -> np.ndarray:
    """Unnormalised DFT along ``axis`` by the dense definition.

    out[k] = sum_j a[j] * exp(sign*2*pi*i*j*k/N); the exponent index j*k is
    reduced mod N exactly in integers before the FP64 exponential.
    """
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[axis]
    j = np.arange(n, dtype=np.int64)
    w = _unit_roots(n, sign)[(j[:, None] * j[None, :]) % n]      # W[j, k]
    moved = np.moveaxis(a, axis, -1)
    out = moved @ w                                               # sum over j
    return np.moveaxis(out, -1, axis)


def smallest_factor(n: int) -> int:
    for p in (2, 3, 5, 7):
        if n % p == 0:
            return p
    p = 11
    while p * p <= n:
        if n % p == 0:
            return p
        p += 2
    return n


def _fft_last(a: np.ndarray, sign: int) -> np.ndarray:
    """Recursive decimation-in-time FFT along the last axis (unnormalised).

    N = p*m with p the smallest prime factor: the p interleaved subsequences
    a[r::p] are transformed (length m), then combined with
    X[k + m*q] = sum_r exp(sign*2*pi*i*r*(k+m*q)/N) * F_r[k].
    """
    n = a.shape[-1]
    if n == 1:
        return a.copy()
    p = smallest_factor(n)
    if p == n:                                   # prime length: dense definition
        return dft_axis(a, -1, sign)
    m = n // p
    subs = [_fft_last(a[..., r::p], sign) for r in range(p)]   # each (..., m)
    roots = _unit_roots(n, sign)
    k = np.arange(m, dtype=np.int64)
    out = np.empty(a.shape, dtype=np.complex128)
    for q in range(p):
        kk = k + m * q
        acc = np.zeros(a.shape[:-1] + (m,), dtype=np.complex128)
        for r in range(p):
            acc += roots[(r * kk) % n] * subs[r]
        out[..., m * q:m * (q + 1)] = acc
    return out


def fft_axis(a: np.ndarray, axis: int, sign: int = -1) -> np.ndarray:
    """Unnormalised mixed-radix FFT along ``axis`` (same result as ``dft_axis``)."""
    a = np.asarray(a, dtype=np.complex128)
    moved = np.ascontiguousarray(np.moveaxis(a, axis, -1))
    return np.moveaxis(_fft_last(moved, sign), -1, axis)


def library_engine(workers: int = 1):
    """A third, independent 1-D engine: scipy's FFT (pocketfft) as a library
    primitive, unnormalised in both directions like the two above.  Used only to
    measure how far two correct FP64 implementations of the same split step drift
    apart over a long run (their twiddles and operation orders round
    differently), which is the floor against which a GPU run is judged."""
    import scipy.fft as sf

    def engine(a, axis, sign):
        a = np.asarray(a, dtype=np.complex128)
        if sign < 0:
            return sf.fft(a, axis=axis, norm="backward", workers=workers)
        return sf.ifft(a, axis=axis, norm="forward", workers=workers)
    return engine


def transform_axis(a: np.ndarray, axis: int, sign: int, engine: str | None = None) -> np.ndarray:
    if callable(engine):
        return engine(a, axis, sign)
    n = np.shape(a)[axis]
    if engine is None:
        engine = "dft" if n <= NAIVE_MAX else "fft"
    if engine == "dft":
        return dft_axis(a, axis, sign)
    if engine == "fft":
        return fft_axis(a, axis, sign)
    raise ValueError(f"unknown engine {engine!r}")


def fftn_unnorm(a: np.ndarray, sign: int = -1, engine: str | None = None,
                axes=None) -> np.ndarray:
    """Unnormalised multi-dimensional transform: one 1-D transform per axis."""
    out = np.asarray(a, dtype=np.complex128)
    axes = range(out.ndim) if axes is None else axes
    for ax in axes:
        out = transform_axis(out, ax, sign, engine)
    return out


def ifftn_unnorm(a: np.ndarray, engine: str | None = None, axes=None) -> np.ndarray:
    return fftn_unnorm(a, +1, engine, axes)


def fft3(psi: np.ndarray, engine: str | None = None) -> np.ndarray:
    """Normalised forward transform c_k = N^-3 sum_x psi(x) exp(-i k.x)."""
    return fftn_unnorm(psi, -1, engine) / float(np.prod(np.shape(psi)))


def ifft3(c: np.ndarray, engine: str | None = None) -> np.ndarray:
    """Inverse transform psi(x) = sum_k c_k exp(+i k.x)."""
    return fftn_unnorm(c, +1, engine)
