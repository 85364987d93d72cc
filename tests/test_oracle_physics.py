"""Pins of the oracle's split step and diagnostics against closed forms,
invariants, an independent 1-D solver and the paper's printed parameters."""
import math
import os

import numpy as np
import pytest

from oracle import gp
from oracle.fft import fft3, ifft3, kvec
import gp_inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid3(n):
    x = 2 * np.pi * np.arange(n) / n
    return x[:, None, None], x[None, :, None], x[None, None, :]   # z, y, x


def plane_wave(n, kz, ky, kx, A):
    z, y, x = _grid3(n)
    return A * np.exp(1j * (kz * z + ky * y + kx * x)) * np.ones((n, n, n))


# ------------------------------------------------------------------ step
@pytest.mark.parametrize("k0", [(1, -2, 3), (0, 0, -8), (5, 7, -8)])
def test_plane_wave_exact_phase(k0):
    """|psi| = A const: the split step is exact and psi picks up
    exp(-i (alpha |k0|^2 + beta (A^2 - 1)) t)."""
    n, alpha, beta, dt, A, steps = 16, 0.7, 1.3, 0.01, 1.2, 40
    psi0 = plane_wave(n, *k0, A)
    psi = gp.evolve(psi0, alpha, beta, dt, steps)
    k2 = sum(k * k for k in k0)
    expect = psi0 * np.exp(-1j * (alpha * k2 + beta * (A * A - 1)) * steps * dt)
    assert np.abs(psi - expect).max() < 1e-12


def test_constant_field_phase():
    n, beta, dt, A = 8, 2.5, 0.03, 0.8
    psi = gp.evolve(np.full((n, n, n), A, dtype=complex), 0.9, beta, dt, 25)
    assert np.abs(psi - A * np.exp(-1j * beta * (A * A - 1) * 25 * dt)).max() < 1e-13


def test_mass_conserved_to_roundoff():
    psi0 = I.random_field((12, 8, 16), seed=1)
    m0 = gp.mass(psi0)
    psi = gp.evolve(psi0, 0.4, 3.0, 0.01, 60)
    assert abs(gp.mass(psi) - m0) / m0 < 1e-13


def test_time_reversibility():
    psi0 = np.exp(1j * I.srp_fourier_theta(16, 3, 11))
    fwd = gp.evolve(psi0, 1.0, 1.0, 0.01, 40)
    back = gp.evolve(fwd, 1.0, 1.0, 0.01, -40)
    assert np.linalg.norm(back - psi0) / np.linalg.norm(psi0) < 1e-12


def test_conjugation_symmetry():
    psi0 = I.random_field(8, seed=4)
    a = np.conj(gp.evolve(np.conj(psi0), 0.5, 2.0, 0.02, 5))
    b = gp.evolve(psi0, 0.5, 2.0, -0.02, 5)
    assert np.abs(a - b).max() < 1e-13


def test_energy_drift_second_order():
    """Halving dt at fixed final time divides the max energy drift by ~4
    (second-order splitting)."""
    psi0 = np.exp(1j * I.srp_fourier_theta(16, 2, 5))
    alpha, beta, T = 0.5, 1.0, 2.0
    E0 = gp.energy(psi0, alpha, beta)
    drifts = []
    for dt in (0.04, 0.02):
        d = [0.0]
        gp.evolve(psi0, alpha, beta, dt, int(round(T / dt)),
                  callback=lambda s, p: d.append(abs(gp.energy(p, alpha, beta) - E0) / E0), every=1)
        drifts.append(max(d))
    assert 3.5 < drifts[0] / drifts[1] < 4.5


def test_bogoliubov_dispersion():
    """psi0 = sqrt(1 + eps cos x): the density mode oscillates as cos(w t) with
    w^2 = alpha^2 k^4 + 2 alpha beta k^2 (Bogoliubov relation, paper units)."""
    n, alpha, beta, eps, dt = 16, 0.5, 2.0, 1e-4, 2e-3
    z, y, x = _grid3(n)
    psi = np.sqrt(1 + eps * np.cos(x)) * np.ones((n, n, n))
    w = math.sqrt(alpha ** 2 + 2 * alpha * beta)
    steps = 100
    for block in range(1, 6):
        psi = gp.evolve(psi, alpha, beta, dt, steps)
        t = block * steps * dt
        rho = np.abs(psi) ** 2
        amp = np.mean(rho * np.exp(-1j * x)).real          # coefficient of e^{ix}
        assert abs(amp / (eps / 2) - math.cos(w * t)) < 2e-3


def test_reduces_to_1d_nls():
    """A field independent of y and z evolves as the 1-D split step (written
    here with numpy.fft as an outside implementation)."""
    n, alpha, beta, dt = 32, 0.3, 4.0, 0.005
    rng = np.random.default_rng(2)
    f = (1 + 0.2 * rng.standard_normal(n)) * np.exp(1j * rng.random(n))
    psi = np.broadcast_to(f[None, None, :], (4, 6, n)).astype(complex)
    k = np.fft.fftfreq(n, 1.0 / n)
    g = f.copy()
    for _ in range(30):
        g = np.fft.ifft(np.exp(-1j * alpha * k * k * dt / 2) * np.fft.fft(g))
        g = g * np.exp(-1j * beta * (np.abs(g) ** 2 - 1) * dt)
        g = np.fft.ifft(np.exp(-1j * alpha * k * k * dt / 2) * np.fft.fft(g))
    psi = gp.evolve(psi, alpha, beta, dt, 30)
    assert np.abs(psi - g[None, None, :]).max() < 1e-12


def test_directional_substeps_compose_to_3d():
    psi = I.random_field((8, 12, 16), seed=9)
    a = gp.linear_substep(psi, 0.8, 0.07)
    b = psi
    for ax in (2, 1, 0):
        b = gp.linear_substep_axis(b, 0.8, 0.07, ax)
    assert np.abs(a - b).max() < 1e-13


def test_engines_agree_over_steps():
    psi0 = I.random_field(16, seed=5)
    a = gp.evolve(psi0, 0.6, 2.0, 0.01, 5, engine="dft")
    b = gp.evolve(psi0, 0.6, 2.0, 0.01, 5, engine="fft")
    assert np.abs(a - b).max() < 1e-13


# ------------------------------------------------------------------ diagnostics
def test_plane_wave_diagnostics():
    n, alpha, beta, A = 16, 0.35, 2.0, 1.1
    k0 = (1, -2, 3)                                   # (kz, ky, kx)
    psi = plane_wave(n, *k0, A)
    w, _ = gp.momentum_w(psi, alpha)
    for j in range(3):
        assert np.abs(w[j] - 2 * alpha * A * k0[j]).max() < 1e-12
    d = gp.diagnostics(psi, alpha, beta)
    k2 = sum(k * k for k in k0)
    ekin = 2 * alpha ** 2 * A ** 2 * k2
    eint = alpha * beta * (A * A - 1) ** 2
    assert abs(d["e_kin"] - ekin) < 1e-12
    assert abs(d["e_kin_i"] - ekin) < 1e-12          # k = 0 mode is incompressible
    assert abs(d["e_kin_c"]) < 1e-24
    assert abs(d["e_q"]) < 1e-24
    assert abs(d["e_int"] - eint) < 1e-13
    assert abs(d["energy"] - (ekin + eint)) < 1e-12
    assert abs(d["mass"] - A * A) < 1e-13
    # the whole spectrum of E_kin^i sits in shell 0 (uniform w)
    assert abs(d["spec"][0][0] - ekin) < 1e-12 and np.abs(d["spec"][0][1:]).max() < 1e-24


def test_quantum_energy_closed_form():
    """sqrt(rho) = 1 + eps cos(2x) with a constant phase: E_q = 2 alpha^2 <|grad sqrt rho|^2>
    = 2 alpha^2 * 4 eps^2 / 2, all in shell 2."""
    n, alpha, beta, eps = 16, 0.4, 1.5, 0.1
    z, y, x = _grid3(n)
    a = (1 + eps * np.cos(2 * x)) * np.ones((n, n, n))
    d = gp.diagnostics(a.astype(complex), alpha, beta)
    assert abs(d["e_q"] - 2 * alpha ** 2 * 4 * eps ** 2 / 2) < 1e-13
    assert abs(d["spec"][2][2] - d["e_q"]) < 1e-13
    assert abs(d["e_kin"]) < 1e-24


def test_quantum_energy_ignores_nyquist_reading():
    """Reading of the paper: first derivatives drop the Nyquist mode, so an
    amplitude modulation (-1)^j carries no quantum energy."""
    n = 8
    j = np.arange(n)
    a = (1 + 0.1 * (-1.0) ** j)[None, None, :] * np.ones((n, n, n))
    d = gp.diagnostics(a.astype(complex), 0.5, 1.0)
    assert abs(d["e_q"]) < 1e-24


def test_kinetic_plus_quantum_is_the_gradient_energy():
    """Pointwise, |w|^2 + |q|^2 = 4 alpha^2 |grad psi|^2 (w and q are the imaginary and
    real parts of 2 alpha conj(psi) grad psi / |psi|), so by Parseval
    e_kin + e_q = 2 alpha^2 sum_k |k~|^2 |c_k|^2 with the first-derivative k~, for any
    field without exact zeros -- vortex cores included.  E differs from this sum only
    through the Nyquist entries of |k|^2."""
    alpha, beta = 0.3, 2.0
    for psi in (I.random_field((12, 16, 8), seed=22), I.tg_psi(16, math.sqrt(alpha / beta), 2)):
        d = gp.diagnostics(psi, alpha, beta)
        c = fft3(psi)
        shape = psi.shape
        fz = gp.first_derivative_k(shape[0])[:, None, None]
        fy = gp.first_derivative_k(shape[1])[None, :, None]
        fx = gp.first_derivative_k(shape[2])[None, None, :]
        grad_e = 2 * alpha ** 2 * float(np.sum((fx * fx + fy * fy + fz * fz) * np.abs(c) ** 2))
        assert abs(d["e_kin"] + d["e_q"] - grad_e) < 1e-12 * grad_e
        assert d["e_q"] > 1e-3 * d["e_kin"]
    # a field with no Nyquist content: E = e_kin + e_q + e_int exactly
    n = 16
    z, y, x = _grid3(n)
    psi = (1 + 0.2 * np.cos(x - 2 * z)) * np.exp(1j * (np.sin(y) + 0.5 * np.cos(x + z))) * np.ones((n, n, n))
    c = fft3(psi)
    c[n // 2] = 0; c[:, n // 2] = 0; c[:, :, n // 2] = 0
    psi = ifft3(c)
    d = gp.diagnostics(psi, alpha, beta)
    assert abs(d["e_kin"] + d["e_q"] + d["e_int"] - d["energy"]) < 1e-12 * d["energy"]


def test_quantum_field_is_grad_amplitude():
    """q = 2 alpha grad |psi| for a smooth field with a band-limited phase and amplitude
    (checked against the analytic gradient, up to the spectral truncation of psi)."""
    n, alpha = 32, 0.25
    z, y, x = _grid3(n)
    amp = 1.0 + 0.3 * np.sin(y) * np.cos(z)
    psi = amp * np.exp(1j * 0.2 * np.cos(x))
    q = gp.quantum_q(psi, alpha)
    exact = [-0.3 * 2 * alpha * np.sin(y) * np.sin(z), 0.3 * 2 * alpha * np.cos(y) * np.cos(z) + 0 * x, 0 * x + 0 * y * z]
    for j in range(3):
        assert np.abs(q[j] - exact[j]).max() < 1e-10


def test_helmholtz_pure_fields():
    n = 12
    z, y, x = _grid3(n)
    one = np.ones((n, n, n))
    # divergence-free: (w_x, w_y, w_z) = (sin y, sin z, sin x)
    wdf = [np.sin(x) * one, np.sin(z) * one, np.sin(y) * one]         # [w_z, w_y, w_x]
    # curl-free: gradient of -(cos x + cos y + cos z)
    wcf = [np.sin(z) * one, np.sin(y) * one, np.sin(x) * one]
    for w, pure in ((wdf, "i"), (wcf, "c")):
        from oracle.fft import fft3
        wi, wc = gp.helmholtz([fft3(c) for c in w], (n, n, n))
        ei = 0.5 * sum(np.sum(np.abs(c) ** 2) for c in wi)
        ec = 0.5 * sum(np.sum(np.abs(c) ** 2) for c in wc)
        tot = 0.5 * sum(np.mean(c ** 2) for c in w)
        if pure == "i":
            assert abs(ei - tot) < 1e-14 and ec < 1e-28
        else:
            assert abs(ec - tot) < 1e-14 and ei < 1e-28


def test_srp_initial_state_diagnostics():
    """psi = exp(i theta): rho = 1, so E_int = E_q = 0; w is a gradient so
    E_kin^i is only spectral truncation; the spectra sum to the physical-space
    energies (Parseval)."""
    theta = I.srp_fourier_theta(32, 4, 0)
    psi = np.exp(1j * theta)
    d = gp.diagnostics(psi, 1.0, 1.0)
    # rho = 1 exactly; q = 2 alpha Re(conj(psi) grad psi) vanishes up to the spectral
    # truncation of exp(i theta) (gone at 64^3)
    assert d["e_int"] < 1e-28 and abs(d["e_q"]) < 1e-4 * d["e_kin"]
    d64 = gp.diagnostics(np.exp(1j * I.srp_fourier_theta(64, 4, 0)), 1.0, 1.0)
    assert abs(d64["e_q"]) < 1e-12 * d64["e_kin"]
    assert d["e_kin_i"] < 1e-3 * d["e_kin"]
    assert abs(d["e_kin_i"] + d["e_kin_c"] - d["e_kin"]) < 1e-13 * d["e_kin"]
    assert abs(d["energy"] - d["e_kin"]) < 1e-2 * d["e_kin"]


def test_spectra_sum_rules_random():
    psi = I.random_field((12, 16, 8), seed=21)
    d = gp.diagnostics(psi, 0.3, 2.0)
    assert abs(d["spec"][3].sum() - d["e_int"]) < 1e-13 * max(1.0, d["e_int"])
    assert abs(d["spec"][0].sum() + d["spec"][1].sum() - d["e_kin"]) < 1e-12 * d["e_kin"]
    assert d["spec"].shape == (4, gp.nshell((12, 16, 8)))


def test_w_bounded_by_gradient():
    psi = I.random_field(12, seed=8)
    alpha = 0.7
    w, dpsi = gp.momentum_w(psi, alpha)
    wn = np.sqrt(sum(c ** 2 for c in w))
    gn = np.sqrt(sum(np.abs(c) ** 2 for c in dpsi))
    assert np.all(wn <= 2 * alpha * gn * (1 + 1e-12) + 1e-300)


def test_shell_index_brute_force():
    k2 = np.arange(0, 200000)
    s = gp.shell_index(k2)
    assert np.array_equal(s, np.rint(np.sqrt(k2.astype(np.float64))).astype(np.int64))
    assert [gp.nshell((n, n, n)) for n in (32, 64, 96, 128, 256, 1024)] == [29, 56, 84, 112, 223, 888]


def test_structure_function_matches_autocorrelation():
    """S2(m) = 2 (C(0) - C(m)) with C the autocorrelation along each axis."""
    psi = I.random_field(8, seed=3)
    s = gp.structure_function_density(psi, 2)
    rho = np.abs(psi) ** 2
    n = 8
    ref = np.zeros(n // 2)
    for ax in range(3):
        f = np.fft.fft(rho, axis=ax)
        c = np.real(np.fft.ifft(np.abs(f) ** 2, axis=ax))
        c = np.mean(np.moveaxis(c, ax, 0), axis=(1, 2)) / n     # sum over the axis -> mean
        ref += 2 * (c[0] - c[1:n // 2 + 1])
    assert np.abs(s - ref / 3).max() < 1e-12


def test_velocity_structure_function_closed_form():
    """psi = exp(i a cos x) (|psi| = 1): v = -2 alpha a sin(x) e_x, so
    S_x(m) = (2 alpha a)^2 (1 - cos(2 pi m / N)) and S_y = S_z = 0; <v_x^2> = 2 (alpha a)^2,
    and the mean of S_x over all lags (S(N - m) = S(m)) is 2 <v_x^2>, the large-lag
    value of eq. strfunc-verif for a decorrelating field.  The
    spectral derivative of exp(i a cos x) is exact to round-off (its modes decay
    like J_k(a))."""
    n, alpha, a = 32, 0.3, 0.5
    z, y, x = _grid3(n)
    psi = np.exp(1j * a * np.cos(x)) * np.ones((n, n, n))
    s, mv2 = gp.structure_function_velocity(psi, alpha)
    r = 2 * np.pi * np.arange(1, n // 2 + 1) / n
    assert np.abs(s[0] - (2 * alpha * a) ** 2 * (1 - np.cos(r))).max() < 1e-13
    assert np.abs(s[1:]).max() < 1e-26
    assert abs(mv2[0] - 2 * (alpha * a) ** 2) < 1e-14
    assert abs((2 * s[0][:-1].sum() + s[0][-1]) / n - 2 * mv2[0]) < 1e-13
    # y-dependence moves to the second row
    psi_y = np.exp(1j * a * np.cos(y)) * np.ones((n, n, n))
    s_y, _ = gp.structure_function_velocity(psi_y, alpha)
    assert np.abs(s_y[1] - s[0]).max() < 1e-13 and np.abs(s_y[0]).max() < 1e-26


def test_velocity_structure_function_matches_autocorrelation():
    """On a random field (and a vortex-carrying one) the lag sums equal
    2 (C(0) - C(m)) from the FFT autocorrelation of v_j along axis j."""
    alpha = 0.25
    for psi in (I.random_field(8, seed=4), I.tg_psi(16, 0.1, 1)):
        n = psi.shape[0]
        s, mv2 = gp.structure_function_velocity(psi, alpha)
        vz, vy, vx = gp.velocity(psi, alpha)
        for j, (v, ax) in enumerate(((vx, 2), (vy, 1), (vz, 0))):
            f = np.fft.fft(v, axis=ax)
            c = np.real(np.fft.ifft(np.abs(f) ** 2, axis=ax))
            c = np.mean(np.moveaxis(c, ax, 0), axis=(1, 2)) / n
            assert np.abs(s[j] - 2 * (c[0] - c[1:n // 2 + 1])).max() < 1e-11 * max(1.0, c[0])
            assert abs(mv2[j] - c[0]) < 1e-12 * max(1.0, c[0])


def test_velocity_is_momentum_over_amplitude():
    """v = w / sqrt(rho) (eq. scaling-rhov), 0 where psi = 0; for a plane wave
    A exp(i k.x), v = 2 alpha k."""
    n, alpha = 16, 0.35
    psi = plane_wave(n, 1, -2, 3, 1.7)
    v = gp.velocity(psi, alpha)
    for j, k in enumerate((1, -2, 3)):
        assert np.abs(v[j] - 2 * alpha * k).max() < 1e-12
    psi = I.random_field(8, seed=9)
    psi[0, 0, 0] = 0
    v = gp.velocity(psi, alpha)
    w, _ = gp.momentum_w(psi, alpha)
    amp = np.abs(psi)
    for j in range(3):
        assert v[j][0, 0, 0] == 0.0
        m = amp > 0
        assert np.abs(v[j][m] * amp[m] - w[j][m]).max() < 1e-12


def test_mach_numbers():
    """Plane wave A exp(i k.x): |w| = 2 alpha |k| A everywhere, so M_max = M_rms =
    2 alpha |k| A / c with c = sqrt(2 alpha beta); on any field M_rms = sqrt(2 E_kin)/c
    (eq. Mach-Number) and M_max >= M_rms.  The paper's Mach table is consistent with
    c = 2 at alpha beta = 2: its M_rms of ABC_c equals sqrt(2 (E_kin^i + E_kin^c))/2 of
    the printed ABC_cIT energies."""
    n, alpha, beta, A = 16, 0.3, 2.0, 1.2
    k = (1, -2, 3)
    mmax, mrms = gp.mach_numbers(plane_wave(n, *k, A), alpha, beta)
    want = 2 * alpha * math.sqrt(sum(x * x for x in k)) * A / math.sqrt(2 * alpha * beta)
    assert abs(mmax - want) < 1e-12 and abs(mrms - want) < 1e-12
    psi = I.random_field(12, seed=5)
    mmax, mrms = gp.mach_numbers(psi, alpha, beta)
    d = gp.diagnostics(psi, alpha, beta)
    assert abs(mrms - math.sqrt(2 * d["e_kin"]) / math.sqrt(2 * alpha * beta)) < 1e-12 and mmax > mrms
    e_kin_c = 0.9884992 + 0.0006486                 # ABC_cIT, E_kin^i + E_kin^c
    assert abs(math.sqrt(2 * e_kin_c) / 2.0 - 0.703259) < 2e-6


# ------------------------------------------------------------------ parameters
def _golden_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_params.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


def test_table1_parameters():
    rows = _golden_table1()
    assert len(rows) == 4
    for n, alpha, beta, kxi, dxxi, xi, nv in rows:
        p = gp.table1_params(int(n))
        assert abs(p["alpha"] - alpha) < 5e-6
        assert abs(p["beta"] - beta) < 1e-9
        assert abs(p["kmax_xi"] - kxi) < 5e-3
        assert abs(p["dx_over_xi"] - dxxi) < 5e-4
        assert abs(p["xi"] - xi) < 5e-7
        assert int(p["Nv1d"]) == int(nv)
        assert abs(p["c"] - 2.0) < 1e-12


def test_gamma_d_quarter():
    assert [gp.gamma_d_quarter(gp.table1_params(n)["alpha"]) for n in (128, 256, 512, 1024)] == [3, 6, 12, 25]


def test_chaotic_regime_parity_floor():
    """The oracle run twice on the 32^3 smoothed-random-phase workload (alpha = beta
    = 1, dt = 1e-3, 200 steps), once with the dense DFT and once with the
    mixed-radix FFT: the two transforms differ only in rounding order, so their
    distance is the floor any complex128 parity claim stands on.  It must stay
    well under the 1e-12 relative tolerance of the GPU parity tests."""
    w = I.WORKLOADS["srp32"]
    psi0 = np.exp(1j * I.srp_fourier_theta(32, 4, 0))
    floors = []
    a = b = psi0
    for _ in range(w["steps"] // 40):
        a = gp.evolve(a, w["alpha"], w["beta"], w["dt"], 40, engine="dft")
        b = gp.evolve(b, w["alpha"], w["beta"], w["dt"], 40, engine="fft")
        floors.append(np.linalg.norm(a - b) / np.linalg.norm(b))
    print("rel-L2 DFT vs FFT every 40 steps:", " ".join(f"{f:.1e}" for f in floors))
    assert max(floors) < 1e-12 / 4
