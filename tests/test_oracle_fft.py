"""Pins of the oracle's transforms: definition vs FFT, closed forms, Parseval.

numpy.fft appears here only as an outside third opinion."""
import numpy as np
import pytest

from oracle import fft as F

SIZES = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96]


@pytest.mark.parametrize("n", SIZES)
def test_dft_equals_fft_and_numpy(n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((5, n)) + 1j * rng.standard_normal((5, n))
    d = F.dft_axis(a, 1)
    f = F.fft_axis(a, 1)
    ref = np.fft.fft(a, axis=1)
    scale = np.abs(ref).max()
    assert np.abs(d - ref).max() <= 1e-13 * scale * max(1, n)
    assert np.abs(f - ref).max() <= 1e-13 * scale * max(1, np.log2(max(n, 2)))
    di = F.dft_axis(a, 1, +1)
    assert np.abs(di - np.fft.ifft(a, axis=1) * n).max() <= 1e-13 * scale * max(1, n)


@pytest.mark.parametrize("n", [8, 12, 16])
def test_plane_wave_to_single_coefficient(n):
    x = 2 * np.pi * np.arange(n) / n
    k = F.kvec(n)
    for kz, ky, kx in [(1, 0, 0), (0, -2, 1), (n // 2 - 1, 1, -(n // 2)), (0, 0, -(n // 2))]:
        psi = np.exp(1j * (kz * x[:, None, None] + ky * x[None, :, None] + kx * x[None, None, :]))
        for engine in ("dft", "fft"):
            c = F.fft3(psi, engine)
            iz, iy, ix = (np.where(k == kz)[0][0], np.where(k == ky)[0][0], np.where(k == kx)[0][0])
            assert abs(c[iz, iy, ix] - 1.0) < 1e-13
            c[iz, iy, ix] = 0
            assert np.abs(c).max() < 1e-13


def test_kvec_fftfreq_order():
    assert list(F.kvec(8)) == [0, 1, 2, 3, -4, -3, -2, -1]
    assert list(F.kvec(6)) == [0, 1, 2, -3, -2, -1]
    assert list(F.kvec(3)) == [0, 1, -1]
    assert list(F.kvec(1)) == [0]


@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 8, 16), (6, 4, 3)])
def test_roundtrip_and_parseval(shape):
    rng = np.random.default_rng(7)
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    for engine in ("dft", "fft"):
        c = F.fft3(psi, engine)
        back = F.ifft3(c, engine)
        assert np.abs(back - psi).max() < 1e-13
        # Parseval with the normalised forward transform: mean|psi|^2 = sum|c|^2
        assert abs(np.mean(np.abs(psi) ** 2) - np.sum(np.abs(c) ** 2)) < 1e-13


def test_engines_agree_3d():
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((24, 16, 12)) + 1j * rng.standard_normal((24, 16, 12))
    assert np.abs(F.fft3(psi, "dft") - F.fft3(psi, "fft")).max() < 1e-15 * 24 * 16 * 12 + 1e-14


@pytest.mark.parametrize("n", [2, 3, 12, 48, 64, 96])
def test_library_engine_equals_the_definition(n):
    """The library-FFT engine (used only to measure the FP64 floor between two
    implementations) is the unnormalised transform of the definition in both
    directions, along every axis."""
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, 3, 5)) + 1j * rng.standard_normal((n, 3, 5))
    eng = F.library_engine(2)
    for axis in range(3):
        b = np.moveaxis(a, 0, axis)
        for sign in (-1, 1):
            want = F.dft_axis(b, axis, sign)
            got = F.transform_axis(b, axis, sign, eng)
            assert np.abs(got - want).max() < 1e-13 * max(1.0, np.abs(want).max())
