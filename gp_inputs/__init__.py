"""Seeded synthetic inputs for the Gross-Pitaevskii split step.

This module holds only input construction (initial fields, random directions,
workload descriptions).  It contains none of the method's arithmetic (no split
step, no diagnostics) and imports neither the oracle nor the HIP library, so
both sides can take their inputs from it.

Initial conditions follow the paper's "Initial data preparation" section:

* ``srp_fourier_theta`` -- smoothed random phase.  The paper interpolates random
  control values with periodic cubic splines; the workloads here ask instead
  for Gaussian random Fourier modes with |k| <= K, so theta is band-limited.
  Recipe: numpy PCG64(seed); for every integer k with 0 < |k|^2 <= K^2 in
  lexicographic (kz, ky, kx) order draw a, b ~ N(0, 1) and set
  theta_hat_k = a + i b (folded mod N); Hermitian-symmetrise, zero the mean
  mode, transform to real space and scale to rms(theta) = 1.  psi = exp(i theta).
* ``srp_spline_theta`` -- the paper's own smoothed random phase: theta uniform in
  [-K, K] at N_r^3 control points (spacing N_s = N / N_r grid points), drawn with
  numpy PCG64(seed) as one (N_r, N_r, N_r) array in [z][y][x] order, then a
  periodic uniform cubic spline along x, y and z in turn (second derivatives from
  the cyclic tridiagonal system N_s^2 (M_{i-1} + 4 M_i + M_{i+1}) =
  6 (c_{i-1} - 2 c_i + c_{i+1}) over neighbouring control points; values between
  them from the A, B, C, D weights of the SRP section).
* ``tg_psi`` -- Taylor-Green ansatz: Clebsch potentials (eq. clebsch3d),
  psi_e (eq. psie, tanh argument read as r / (sqrt(2) xi)), the product of
  four shifted copies (eq. psi4) raised to [1/(2 pi alpha)] (eq. psitot3d),
  evaluated directly on [0, 2 pi)^3; no imaginary-time relaxation.
* ``abc_velocity`` / ``abc_psi`` -- the sum of two Arnold-Beltrami-Childress
  flows (eq. ABC with k = 1 and k = 2; the paper's large-scale spectrum has
  exactly these two modes) and the phase-only ansatz psi_ABC^(1) psi_ABC^(2)
  (eq. ABCphi0, eq. ABCphi): per flow and coefficient a phase that is linear in
  the two other coordinates with integer slopes [A sin(kx)/(2 alpha)],
  [A cos(kx)/(2 alpha)] (nearest integer, numpy rint), so psi is periodic.
* ``rvr_psi`` -- random vortex-ring pairs: Pade profile (eq. Pade and its
  coefficients), ring phase atan2(z~, r - R), pair psi_VR(z - d/2) conj
  psi_VR(z + d/2), six mirror-conjugate images (eq. psiRP), random translation
  by direct evaluation at (x - X) mod 2 pi, random axis permutation
  (eq. psiRVR), product over pairs.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "grid", "srp_fourier_theta", "srp_mode_count", "srp_spline_theta", "tg_psi", "tg_velocity", "abc_velocity", "abc_psi",
    "ABC_COEFFS", "pade_f",
    "PADE_A1", "PADE_A2", "PADE_B1", "rvr_psi", "rvr_draws", "random_field",
    "random_real", "alpha_beta_from_xi", "alpha_beta_table1", "WORKLOADS",
]

TWO_PI = 2.0 * math.pi


def grid(n: int) -> np.ndarray:
    """Grid coordinates x_j = 2 pi j / n."""
    return TWO_PI * np.arange(n, dtype=np.float64) / n


# ------------------------------------------------------------------ SRP
def _modes(K: int):
    r = range(-K, K + 1)
    return [(kz, ky, kx) for kz in r for ky in r for kx in r
            if 0 < kz * kz + ky * ky + kx * kx <= K * K]


def srp_mode_count(K: int) -> int:
    return len(_modes(K))


def srp_fourier_theta(shape, K: int, seed: int, rms: float = 1.0) -> np.ndarray:
    """Band-limited Gaussian random phase theta (FP64, C-order [z][y][x])."""
    if isinstance(shape, int):
        shape = (shape, shape, shape)
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    modes = _modes(K)
    ab = rng.standard_normal((len(modes), 2))
    hat = np.zeros(shape, dtype=np.complex128)
    for (kz, ky, kx), (a, b) in zip(modes, ab):
        hat[kz % nz, ky % ny, kx % nx] += a + 1j * b
    mirror = np.conj(hat[(-np.arange(nz)) % nz][:, (-np.arange(ny)) % ny][:, :, (-np.arange(nx)) % nx])
    hat = 0.5 * (hat + mirror)
    hat[0, 0, 0] = 0.0
    theta = np.real(np.fft.ifftn(hat))
    s = math.sqrt(float(np.mean(theta * theta)))
    if s == 0.0:
        return theta
    return theta * (rms / s)


# ------------------------------------------------------------------ TG
def tg_velocity(n: int):
    """Taylor-Green velocity field v_TG (eq. tg3d) on an n^3 grid, as the
    components [v_z, v_y, v_x] (FP64, each shaped [z][y][x])."""
    x = grid(n)
    sx, cx = np.sin(x), np.cos(x)
    vx = sx[None, None, :] * cx[None, :, None] * cx[:, None, None]
    vy = -cx[None, None, :] * sx[None, :, None] * cx[:, None, None]
    vz = np.zeros((n, n, n))
    return [vz, np.ascontiguousarray(np.broadcast_to(vy, (n, n, n))),
            np.ascontiguousarray(np.broadcast_to(vx, (n, n, n)))]


def _spline_axis(c, ns: int, axis: int):
    """Periodic uniform cubic spline along `axis` of control values c (spacing ns grid
    points): returns the values at all ns * len grid points of that axis."""
    c = np.moveaxis(np.asarray(c, dtype=np.float64), axis, 0)
    nr = c.shape[0]
    # cyclic tridiagonal system for the second derivatives M at the control points
    a = np.zeros((nr, nr))
    for i in range(nr):
        a[i, i] += 4.0
        a[i, (i - 1) % nr] += 1.0
        a[i, (i + 1) % nr] += 1.0
    rhs = 6.0 * (np.roll(c, 1, axis=0) - 2.0 * c + np.roll(c, -1, axis=0)) / (ns * ns)
    m = np.tensordot(np.linalg.inv(a), rhs, axes=(1, 0))
    out = np.empty((nr * ns,) + c.shape[1:])
    for s in range(ns):
        A = (ns - s) / ns
        B = s / ns
        C = (A ** 3 - A) * ns * ns / 6.0
        D = (B ** 3 - B) * ns * ns / 6.0
        out[s::ns] = A * c + B * np.roll(c, -1, axis=0) + C * m + D * np.roll(m, -1, axis=0)
    return np.moveaxis(out, 0, axis)


def srp_spline_theta(n: int, K: float, nr: int, seed: int) -> np.ndarray:
    """The SRP phase of the paper (SRP section): uniform random values in [-K, K] at
    nr^3 control points, periodic cubic spline interpolation along each axis; n must
    be a multiple of nr.  Returns theta [z][y][x] (FP64)."""
    if n % nr:
        raise ValueError("n must be a multiple of nr")
    ns = n // nr
    c = np.random.default_rng(seed).uniform(-K, K, (nr, nr, nr))
    for axis in (2, 1, 0):                      # x, then y, then z
        c = _spline_axis(c, ns, axis)
    return c


ABC_COEFFS = (0.9 / math.sqrt(3.0), 1.0 / math.sqrt(3.0), 1.1 / math.sqrt(3.0))   # (A, B, C)


def abc_velocity(n: int, coeffs=ABC_COEFFS, ks=(1, 2)):
    """v_ABC = sum over k in ks of the ABC flow of wavenumber k (eq. ABC), as the
    components [v_z, v_y, v_x] (FP64, each shaped [z][y][x])."""
    A, B, C = coeffs
    x = grid(n)
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    vx = sum(B * np.cos(k * Y) + C * np.sin(k * Z) for k in ks)
    vy = sum(C * np.cos(k * Z) + A * np.sin(k * X) for k in ks)
    vz = sum(A * np.cos(k * X) + B * np.sin(k * Y) for k in ks)
    full = (n, n, n)
    return [np.ascontiguousarray(np.broadcast_to(c, full)) for c in (vz, vy, vx)]


def abc_psi(n: int, alpha: float, coeffs=ABC_COEFFS, ks=(1, 2)) -> np.ndarray:
    """Phase-only ABC ansatz prod_k psi_{A,k}^{x,y,z} psi_{B,k}^{y,z,x} psi_{C,k}^{z,x,y}
    (eq. ABCphi0, eq. ABCphi): psi_{A,k}^{x,y,z} = exp(i [A sin(kx)/(2 alpha)] y
    + i [A cos(kx)/(2 alpha)] z), the others by cyclic permutation of (x, y, z)."""
    A, B, C = coeffs
    x = grid(n)
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    h = 1.0 / (2.0 * alpha)
    theta = np.zeros((n, n, n))
    for k in ks:
        theta = theta + np.rint(A * h * np.sin(k * X)) * Y + np.rint(A * h * np.cos(k * X)) * Z
        theta = theta + np.rint(B * h * np.sin(k * Y)) * Z + np.rint(B * h * np.cos(k * Y)) * X
        theta = theta + np.rint(C * h * np.sin(k * Z)) * X + np.rint(C * h * np.cos(k * Z)) * Y
    return np.exp(1j * theta)


def tg_psi(n: int, xi: float, exponent: int) -> np.ndarray:
    """Taylor-Green ansatz psi_4^exponent on an n^3 grid (complex128)."""
    x = grid(n)
    cz = np.cos(x)[:, None, None]
    cy = np.cos(x)[None, :, None]
    cx = np.cos(x)[None, None, :]
    root = np.sqrt(2.0 * np.abs(cz))
    lam = cx * root
    mu = cy * root * np.sign(cz)
    lam, mu = np.broadcast_arrays(lam, mu)

    def psi_e(l, m):
        r = np.sqrt(l * l + m * m)
        safe = np.where(r > 0.0, r, 1.0)
        return np.where(r > 0.0, (l + 1j * m) * np.tanh(r / (math.sqrt(2.0) * xi)) / safe, 0.0)

    s = 1.0 / math.sqrt(2.0)
    psi4 = psi_e(lam - s, mu) * psi_e(lam, mu - s) * psi_e(lam + s, mu) * psi_e(lam, mu + s)
    return psi4 ** exponent


# ------------------------------------------------------------------ RVR
PADE_A1 = (73.0 + 3.0 * math.sqrt(201.0)) / 352.0
PADE_A2 = (6.0 + math.sqrt(201.0)) / 528.0
PADE_B1 = (21.0 + math.sqrt(201.0)) / 96.0


def pade_f(r, xi):
    """Pade vortex-core profile f(r) (eq. Pade)."""
    e2 = (np.asarray(r, dtype=np.float64) / xi) ** 2
    e4 = e2 * e2
    return np.sqrt((PADE_A1 * e2 + PADE_A2 * e4) / (1.0 + PADE_B1 * e2 + PADE_A2 * e4))


def _ring(x, y, z, R, xi):
    xt, yt, zt = x - math.pi, y - math.pi, z - math.pi
    rc = np.sqrt(xt * xt + yt * yt)
    dr = rc - R
    return pade_f(np.sqrt(dr * dr + zt * zt), xi) * np.exp(1j * np.arctan2(zt, dr))


def _pair(x, y, z, R, d, xi):
    return _ring(x, y, z - 0.5 * d, R, xi) * np.conj(_ring(x, y, z + 0.5 * d, R, xi))


def _pair_periodic(x, y, z, R, d, xi):
    L = TWO_PI
    out = _pair(x, y, z, R, d, xi)
    for args in ((2 * L - x, y, z), (-x, y, z), (x, 2 * L - y, z), (x, -y, z),
                 (x, y, 2 * L - z), (x, y, -z)):
        out = out * np.conj(_pair(*args, R, d, xi))
    return out


PERMUTATIONS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def rvr_draws(n_pairs: int, seed: int, rmin: float = 0.3, rmax: float = 0.8):
    """Per pair, in draw order: R, d = 2R, X, Y, Z, permutation index."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_pairs):
        R = float(rng.uniform(rmin, rmax))
        X, Y, Z = (float(v) for v in rng.uniform(0.0, TWO_PI, 3))
        perm = int(rng.integers(0, 6))
        out.append({"R": R, "d": 2.0 * R, "X": X, "Y": Y, "Z": Z, "perm": perm})
    return out


def rvr_psi(n: int, xi: float, n_pairs: int, seed: int, rmin=0.3, rmax=0.8,
            zslab=None, yslab=None, xslab=None) -> np.ndarray:
    """Product of n_pairs random vortex-ring pairs on an n^3 grid (complex128).
    ``zslab = (lo, hi)`` (likewise ``yslab``, ``xslab``) evaluates only the points
    with lo <= z < hi; every point is computed on its own, so blocks put together
    equal the whole field."""
    g = grid(n)
    zl, zh = (0, n) if zslab is None else zslab
    yl, yh = (0, n) if yslab is None else yslab
    xl, xh = (0, n) if xslab is None else xslab
    coords = (g[None, None, xl:xh], g[None, yl:yh, None], g[zl:zh, None, None])   # x, y, z
    psi = np.ones((zh - zl, yh - yl, xh - xl), dtype=np.complex128)
    for p in rvr_draws(n_pairs, seed, rmin, rmax):
        a = [coords[i] for i in PERMUTATIONS[p["perm"]]]
        sx = np.mod(a[0] - p["X"], TWO_PI)
        sy = np.mod(a[1] - p["Y"], TWO_PI)
        sz = np.mod(a[2] - p["Z"], TWO_PI)
        sx, sy, sz = np.broadcast_arrays(sx, sy, sz)
        psi *= _pair_periodic(sx, sy, sz, p["R"], p["d"], xi)
    return psi


# ------------------------------------------------------------------ generic
def random_field(shape, seed: int, amp_noise: float = 0.3) -> np.ndarray:
    """Complex test field (1 + amp_noise*g1) exp(i 2 pi u) with seeded white noise."""
    if isinstance(shape, int):
        shape = (shape, shape, shape)
    rng = np.random.default_rng(seed)
    amp = 1.0 + amp_noise * rng.standard_normal(shape)
    ph = TWO_PI * rng.random(shape)
    return amp * np.exp(1j * ph)


def random_real(shape, seed: int) -> np.ndarray:
    if isinstance(shape, int):
        shape = (shape, shape, shape)
    return np.random.default_rng(seed).standard_normal(shape)


# ------------------------------------------------------------------ workloads
def alpha_beta_from_xi(xi: float, mach: float = 0.5):
    """alpha, beta with xi = sqrt(alpha/beta) and alpha beta = 1/(2 M^2)."""
    ab = 1.0 / (2.0 * mach * mach)
    alpha = math.sqrt(ab) * xi
    return alpha, ab / alpha


def alpha_beta_table1(n: int):
    """alpha = 6.4/N, beta = N/3.2 (parameter table of the results section)."""
    return 6.4 / n, n / 3.2


_XI2 = 2.0 * (TWO_PI / 256)
_XI3 = 3.0 * (TWO_PI / 1024)
_XI3S = 3.0 * (TWO_PI / 256)
_A2, _B2 = alpha_beta_from_xi(_XI2)
_A3, _B3 = alpha_beta_from_xi(_XI3)
_A3S, _B3S = alpha_beta_from_xi(_XI3S)

WORKLOADS = {
    "srp32": dict(n=32, prec=("c128",), alpha=1.0, beta=1.0, dt=1e-3, steps=200,
                  ic=("srp", dict(K=4, seed=0)), diag_every=20),
    "tg256": dict(n=256, prec=("c128", "c64"), alpha=_A2, beta=_B2, dt=5e-4, steps=1000,
                  ic=("tg", dict(xi=_XI2, exponent=int(math.floor(1.0 / (TWO_PI * _A2))))),
                  diag_every=100),
    "rvr1024": dict(n=1024, prec=("c64",), alpha=_A3, beta=_B3, dt=2.5e-4, steps=500,
                    ic=("rvr", dict(xi=_XI3, n_pairs=40, seed=1)), diag_every=50),
    # the 1024^3 random-vortex-ring construction at 256^3: the same 40 pairs (seed 1),
    # core width three grid spacings, alpha beta = 2, the same dt and final time
    "rvr256": dict(n=256, prec=("c128", "c64"), alpha=_A3S, beta=_B3S, dt=2.5e-4, steps=500,
                   ic=("rvr", dict(xi=_XI3S, n_pairs=40, seed=1)), diag_every=50),
    "adj128": dict(n=128, prec=("c128",), alpha=0.05, beta=40.0, dt=1e-3, steps=400,
                   ic=("srp", dict(K=6, seed=2)), ckpt=20, smin=4, smax=12,
                   fd_h=1e-6, fd_dirs=16, fd_seed0=1000),
    # Taylor-Green preparation by the imaginary-time (ARGLE) procedure, run TG_aIT
    # of the paper's TG parameter table: 128^3, alpha = 0.05, beta = 40,
    # dtau = 1.25e-2, tau_f = 60, ansatz psi_4^[gamma_d/4] with [gamma_d/4] = 3,
    # xi = sqrt(alpha/beta)
    "tg128_argle": dict(n=128, prec=("c128",), alpha=0.05, beta=40.0, dtau=1.25e-2, steps=4800,
                        ic=("tg", dict(xi=math.sqrt(0.05 / 40.0), exponent=3)), velocity="tg"),
    # ABC preparation, run ABC_aIT of the paper's ABC parameter table: 128^3,
    # alpha = 0.05, beta = 40 (parameter-table rule), dtau = 4e-3, tau_f = 30
    "abc128_argle": dict(n=128, prec=("c128",), alpha=0.05, beta=40.0, dtau=4e-3, steps=7500,
                         ic=("abc", {}), velocity="abc"),
    # paper-size ensembles of the SRP and RVR benchmarks at 128^3 (runs SRP_a and
    # RVR_a of their parameter tables; alpha, beta from the parameter-table rule);
    # ten seeds each, as the paper's ensemble averages
    "srp128_paper": dict(n=128, prec=("c128",), alpha=0.05, beta=40.0, dt=1.0 / 1024, t_final=8.0,
                         K=8 * math.pi, nr=4, seeds=tuple(range(10))),
    "rvr128_paper": dict(n=128, prec=("c128",), alpha=0.05, beta=40.0, dt=1.0 / 1024, t_final=8.0,
                         n_pairs=200, R=math.pi / 2, seeds=tuple(range(10))),
    "ens48": dict(runs=[dict(n=64, alpha=0.1, beta=20.0, seed=100 + i) for i in range(32)]
                  + [dict(n=96, alpha=6.4 / 96, beta=30.0, seed=132 + i) for i in range(16)],
                  prec=("c64",), dt=1e-3, steps=300, K=4, diag_every=50),
}
