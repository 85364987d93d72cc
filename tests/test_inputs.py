"""Pins of the seeded input generators (initial conditions of the paper)."""
import math

import numpy as np

import gp_inputs as I


def test_srp_mode_counts_and_band_limit():
    assert I.srp_mode_count(4) == 256
    assert I.srp_mode_count(6) == 924
    th = I.srp_fourier_theta(32, 4, 0)
    assert abs(math.sqrt(np.mean(th ** 2)) - 1.0) < 1e-14
    c = np.fft.fftn(th)
    k = np.fft.fftfreq(32, 1 / 32)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    assert np.abs(c[k2 > 16]).max() < 1e-9 * np.abs(c).max()
    assert abs(c[0, 0, 0]) < 1e-9
    # deterministic in the seed, different across seeds
    assert np.array_equal(th, I.srp_fourier_theta(32, 4, 0))
    assert not np.allclose(th, I.srp_fourier_theta(32, 4, 1))


def test_tg_ansatz_zero_lines():
    """psi_e vanishes where (lambda, mu) hits one of the four shifted origins,
    e.g. z = 0, cos x = 1/2, y = pi/2  ->  (lambda, mu) = (1/sqrt2, 0)."""
    n = 12
    psi = I.tg_psi(n, 0.1, 2)
    assert abs(psi[0, n // 4, n // 6]) < 1e-14
    assert np.abs(psi).max() <= 1.0 + 1e-12
    # away from the zero lines the modulus approaches 1 for a thin core
    thin = I.tg_psi(n, 1e-3, 1)
    assert abs(abs(thin[1, 1, 1]) - 1.0) < 1e-6


def test_pade_profile():
    assert abs(I.PADE_A1 - 0.3282168768) < 1e-10
    assert abs(I.PADE_A2 - 0.0382148615) < 1e-10
    assert abs(I.PADE_B1 - 0.3664317383) < 1e-10
    assert I.pade_f(0.0, 1.0) == 0.0
    assert abs(I.pade_f(1e4, 1.0) - 1.0) < 1e-6
    r = np.linspace(1e-3, 20, 200)
    assert np.all(np.diff(I.pade_f(r, 1.0)) > 0)


def test_rvr_structure():
    n, xi = 32, 0.15
    psi = I.rvr_psi(n, xi, 3, seed=1)
    assert psi.shape == (n, n, n)
    assert np.all(np.isfinite(psi))
    assert np.abs(psi).max() <= 1.0 + 1e-12
    assert np.abs(psi).min() < 0.3          # vortex cores present
    d = I.rvr_draws(3, 1)
    assert all(0.3 <= p["R"] <= 0.8 and p["d"] == 2 * p["R"] and 0 <= p["perm"] < 6 for p in d)


def test_workload_parameters():
    w2 = I.WORKLOADS["tg256"]
    assert abs(w2["alpha"] * w2["beta"] - 2.0) < 1e-12
    assert abs(w2["alpha"] - 0.0694200) < 1e-6 and abs(w2["beta"] - 28.81012) < 1e-4
    assert w2["ic"][1]["exponent"] == 2
    w3 = I.WORKLOADS["rvr1024"]
    assert abs(w3["alpha"] - 0.0260325) < 1e-6 and abs(w3["beta"] - 76.82699) < 1e-4
    assert len(I.WORKLOADS["ens48"]["runs"]) == 48


def test_srp_spline_matches_the_periodic_cubic_spline_of_scipy():
    """The paper's spline SRP (SRP section) is the periodic uniform cubic spline
    through the control values, axis by axis: scipy's CubicSpline with periodic end
    conditions gives the same values on 1-D lines and, applied along each axis in
    turn, on the whole grid; the control values are reproduced exactly."""
    from scipy.interpolate import CubicSpline
    import gp_inputs as I
    n, nr, K = 32, 4, 8 * np.pi
    ns = n // nr
    th = I.srp_spline_theta(n, K, nr, seed=3)
    c = np.random.default_rng(3).uniform(-K, K, (nr, nr, nr))
    assert np.abs(th[::ns, ::ns, ::ns] - c).max() < 1e-12
    assert np.abs(th).max() <= 2 * K
    knots = np.arange(nr + 1) * ns
    fine = np.arange(n)
    ref = c
    for axis in (2, 1, 0):
        ext = np.concatenate([ref, np.take(ref, [0], axis=axis)], axis=axis)
        ref = CubicSpline(knots, ext, axis=axis, bc_type="periodic")(fine)
    assert np.abs(th - ref).max() < 1e-10 * K
    # a single line is C2 and periodic: second differences change smoothly across the wrap
    line = th[0, 0, :]
    d2 = np.roll(line, -1) - 2 * line + np.roll(line, 1)
    assert np.abs(np.diff(np.concatenate([d2, d2[:1]]))).max() < 0.5 * np.abs(d2).max()


def test_srp_spline_rejects_bad_sizes_and_is_seeded():
    import gp_inputs as I
    import pytest as _pt
    with _pt.raises(ValueError):
        I.srp_spline_theta(30, 1.0, 4, 0)
    a = I.srp_spline_theta(16, 1.0, 4, 5)
    assert np.array_equal(a, I.srp_spline_theta(16, 1.0, 4, 5))
    assert not np.array_equal(a, I.srp_spline_theta(16, 1.0, 4, 6))


def test_rvr_blocks_equal_the_whole_field():
    """Sub-blocks of the ring-pair field (used to sample the paper-size generator)
    are the corresponding parts of the whole field, bit for bit."""
    a = I.rvr_psi(16, 0.2, 3, 1)
    b = I.rvr_psi(16, 0.2, 3, 1, zslab=(3, 7), yslab=(2, 9), xslab=(5, 16))
    assert np.array_equal(a[3:7, 2:9, 5:16], b)
    c = np.concatenate([I.rvr_psi(16, 0.2, 3, 1, zslab=(0, 5)), I.rvr_psi(16, 0.2, 3, 1, zslab=(5, 16))])
    assert np.array_equal(a, c)
