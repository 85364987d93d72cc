"""Gross-Pitaevskii split step and spectral diagnostics -- the oracle.

TEST INFRASTRUCTURE ONLY (plain, slow, FP64, obviously correct).  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may use it; the product never does.

Everything is written from the paper (arXiv:2003.03590) in its own scaling
(section "Scaling and dimensionless equations", tildes dropped):

    i psi_t = ( -alpha lap + beta (|psi|^2 - 1) ) psi          (eq. gpe-num)

on the periodic box [0, 2*pi)^3.  Readings of points the paper leaves open:

* the "-1" of eq. gpe-num is kept in the nonlinear sub-step (the splitting
  section writes the operator without it; the two differ only by the global
  phase exp(i beta t));
* no dealiasing; the propagator uses k^2 = N^2/4 at the Nyquist index, first
  derivatives use k = 0 there; the Helmholtz projection uses k = -N/2;
* k = 0 counts as incompressible;
* spectra: integer shells s(k) = round(|k|), computed in integers, normalised
  so that the shell sum is the energy (Parseval, per unit volume);
* E_q and its spectrum come from q = 2 alpha grad sqrt(rho) evaluated pointwise
  as 2 alpha Re(conj(psi) grad psi)/|psi| (the companion of w), not from the
  transform of |psi|: |psi| has a cusp at every vortex core and is far from
  band-limited, while psi is.  With this reading the quantum energies of the
  prepared Taylor-Green state agree with the paper's table of energies at the
  end of the preparation.
"""
from __future__ import annotations

import math

import numpy as np

from .fft import fft3, ifft3, fftn_unnorm, ifftn_unnorm, kvec

__all__ = [
    "grids_k", "ksq", "linear_substep", "nonlinear_substep", "strang_step",
    "evolve", "mass", "energy", "gradient", "momentum_w", "quantum_q", "helmholtz",
    "shell_index", "nshell", "diagnostics", "structure_function_density",
    "velocity", "structure_function_velocity", "mach_numbers",
    "table1_params", "gamma_d_quarter",
]


# ---------------------------------------------------------------- wavenumbers
def grids_k(shape):
    """Broadcastable integer wavenumber arrays (kz, ky, kx) for a C-order
    [z][y][x] array of the given shape."""
    nz, ny, nx = shape
    kz = kvec(nz)[:, None, None]
    ky = kvec(ny)[None, :, None]
    kx = kvec(nx)[None, None, :]
    return kz, ky, kx


def first_derivative_k(n: int) -> np.ndarray:
    """k used by a first derivative: fftfreq with the Nyquist entry zeroed."""
    k = kvec(n).astype(np.float64)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def ksq(shape) -> np.ndarray:
    """|k|^2 = kx^2 + ky^2 + kz^2 (integers; Nyquist contributes N^2/4)."""
    kz, ky, kx = grids_k(shape)
    return kx * kx + ky * ky + kz * kz


# ---------------------------------------------------------------- time step
def linear_substep(psi, alpha, tau, engine=None):
    """Exact linear sub-step S(tau, L) = F^-1 exp(-i alpha |k|^2 tau) F
    (spectral sub-step of the time-evolution section; the product of the three
    1-D sub-steps S(tau, L_x) S(tau, L_y) S(tau, L_z) equals this 3-D form
    because the three operators commute)."""
    c = fft3(psi, engine)
    c *= np.exp(-1j * alpha * ksq(psi.shape) * tau)
    return ifft3(c, engine)


def linear_substep_axis(psi, alpha, tau, axis, engine=None):
    """One directional sub-step S(tau, L_j) = F_j^-1 exp(-i alpha k_j^2 tau) F_j.
    ``axis`` is the array axis (0 = z, 1 = y, 2 = x)."""
    from .fft import transform_axis
    n = psi.shape[axis]
    k = kvec(n).astype(np.float64)
    shape = [1, 1, 1]
    shape[axis] = n
    mult = np.exp(-1j * alpha * (k * k) * tau).reshape(shape) / n
    c = transform_axis(psi, axis, -1, engine) * mult
    return transform_axis(c, axis, +1, engine)


def nonlinear_substep(psi, beta, tau):
    """Exact nonlinear sub-step S(tau, N): |psi| is invariant under
    psi_t = -i beta (|psi|^2 - 1) psi, so psi <- exp(-i beta (|psi|^2-1) tau) psi."""
    rho = psi.real * psi.real + psi.imag * psi.imag
    return psi * np.exp(-1j * beta * (rho - 1.0) * tau)


def strang_step(psi, alpha, beta, dt, engine=None):
    """One second-order Strang step (eq. adi_looptime, literal 3-D form):
    half linear step, full nonlinear rotation, half linear step."""
    psi = linear_substep(psi, alpha, 0.5 * dt, engine)
    psi = nonlinear_substep(psi, beta, dt)
    return linear_substep(psi, alpha, 0.5 * dt, engine)


def evolve(psi, alpha, beta, dt, nsteps, engine=None, callback=None, every=0):
    """n literal repetitions of ``strang_step`` (negative nsteps: steps of -dt).
    ``callback(step, psi)`` is called at step 0 and every ``every`` steps."""
    psi = np.array(psi, dtype=np.complex128)
    h = dt if nsteps >= 0 else -dt
    if callback is not None:
        callback(0, psi)
    for n in range(1, abs(int(nsteps)) + 1):
        psi = strang_step(psi, alpha, beta, h, engine)
        if callback is not None and every and n % every == 0:
            callback(n, psi)
    return psi


# ---------------------------------------------------------------- diagnostics
def mass(psi) -> float:
    """Scaled number of particles N = (1/L^3) int |psi|^2 (eq. scaling-N)."""
    return float(np.mean(np.abs(psi) ** 2))


def energy(psi, alpha, beta, engine=None) -> float:
    """Scaled total energy per unit volume (eq. scaling-energy):
    E = 2 alpha^2 sum_k |k|^2 |c_k|^2 + alpha beta <(|psi|^2 - 1)^2>.
    The gradient term uses the propagator's |k|^2, so the linear sub-step
    conserves it exactly."""
    c = fft3(psi, engine)
    kin = 2.0 * alpha * alpha * float(np.sum(ksq(psi.shape) * np.abs(c) ** 2))
    rho = np.abs(psi) ** 2
    return kin + alpha * beta * float(np.mean((rho - 1.0) ** 2))


def gradient(f, engine=None):
    """Spectral first derivatives (d/dz, d/dy, d/dx) = F^-1 (i k_j F f), the
    Nyquist component of k_j set to zero."""
    c = fft3(f, engine)
    out = []
    for ax, n in enumerate(f.shape):
        shape = [1, 1, 1]
        shape[ax] = n
        kj = first_derivative_k(n).reshape(shape)
        out.append(ifft3(1j * kj * c, engine))
    return out


def momentum_w(psi, alpha, engine=None):
    """w = sqrt(rho) v = 2 alpha Im(conj(psi) grad psi) / |psi|
    (eq. scaling-rhov divided by sqrt(rho)); w = 0 where |psi| = 0 exactly.
    Returns [w_z, w_y, w_x] (real arrays) and the derivatives used."""
    d = gradient(psi, engine)
    amp = np.abs(psi)
    safe = np.where(amp > 0.0, amp, 1.0)
    w = [np.where(amp > 0.0, 2.0 * alpha * np.imag(np.conj(psi) * dj) / safe, 0.0) for dj in d]
    return w, d


def quantum_q(psi, alpha, engine=None):
    """q = 2 alpha grad sqrt(rho) = 2 alpha Re(conj(psi) grad psi) / |psi|, the
    field whose energy 1/2 <|q|^2> is the quantum term 2 alpha^2 <|grad sqrt rho|^2>
    of eq. scaling-energy-mod-rho, taken pointwise from the spectral derivatives
    of psi as w is; q = 0 where |psi| = 0 exactly.  Returns [q_z, q_y, q_x]."""
    d = gradient(psi, engine)
    amp = np.abs(psi)
    safe = np.where(amp > 0.0, amp, 1.0)
    return [np.where(amp > 0.0, 2.0 * alpha * np.real(np.conj(psi) * dj) / safe, 0.0) for dj in d]


def helmholtz(w_hat, shape):
    """Split a normalised vector spectrum w_hat = [wz, wy, wx] (each shape N^3)
    into compressible (parallel to k) and incompressible parts
    (eq. def-ekin-decomp): w^c = k (k . w)/|k|^2 for k != 0, w^c(0) = 0."""
    kz, ky, kx = grids_k(shape)
    kz = np.broadcast_to(kz, shape).astype(np.float64)
    ky = np.broadcast_to(ky, shape).astype(np.float64)
    kx = np.broadcast_to(kx, shape).astype(np.float64)
    k2 = kx * kx + ky * ky + kz * kz
    kdotw = kz * w_hat[0] + ky * w_hat[1] + kx * w_hat[2]
    coef = np.where(k2 > 0, kdotw / np.where(k2 > 0, k2, 1.0), 0.0)
    wc = [kz * coef, ky * coef, kx * coef]
    wi = [w_hat[j] - wc[j] for j in range(3)]
    return wi, wc


def shell_index(k2) -> np.ndarray:
    """Integer shell s = round(|k|): the unique s with (2s-1)^2 <= 4|k|^2 < (2s+1)^2,
    computed as (isqrt(4|k|^2) + 1) // 2 in integers (no floating-point ties)."""
    q = 4 * np.asarray(k2, dtype=np.int64)
    r = np.floor(np.sqrt(q.astype(np.float64))).astype(np.int64)
    # exact integer square root correction
    r = np.where(r * r > q, r - 1, r)
    r = np.where((r + 1) * (r + 1) <= q, r + 1, r)
    return (r + 1) // 2


def nshell(shape) -> int:
    kmax2 = sum((n // 2) ** 2 for n in shape)
    return int(shell_index(np.array([kmax2]))[0]) + 1


def diagnostics(psi, alpha, beta, engine=None):
    """Mass, energy, its hydrodynamic decomposition and shell spectra
    (eq. scaling-energy-mod-rho, eq. def-ekin-decomp, spectra section).

    Returns a dict with scalars mass, energy, e_kin, e_kin_i, e_kin_c, e_q,
    e_int and spectra 'spec' of shape (4, nshell): rows E_kin^i(s), E_kin^c(s),
    E_q(s), E_int(s), each summing to its energy.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    shape = psi.shape
    npts = float(np.prod(shape))
    rho = np.abs(psi) ** 2
    w, _ = momentum_w(psi, alpha, engine)
    e_kin = 0.5 * float(np.mean(w[0] ** 2 + w[1] ** 2 + w[2] ** 2))
    e_int = alpha * beta * float(np.mean((rho - 1.0) ** 2))

    w_hat = [fft3(wj, engine) for wj in w]
    wi, wc = helmholtz(w_hat, shape)
    dens_i = 0.5 * sum(np.abs(x) ** 2 for x in wi)
    dens_c = 0.5 * sum(np.abs(x) ** 2 for x in wc)

    q = quantum_q(psi, alpha, engine)
    dens_q = 0.5 * sum(np.abs(fft3(qj, engine)) ** 2 for qj in q)
    kz, ky, kx = grids_k(shape)

    b_hat = fft3(rho - 1.0, engine)
    dens_int = alpha * beta * np.abs(b_hat) ** 2

    k2 = kx * kx + ky * ky + kz * kz
    s = np.broadcast_to(shell_index(k2), shape).ravel()
    ns = nshell(shape)
    spec = np.zeros((4, ns))
    for row, dens in enumerate((dens_i, dens_c, dens_q, dens_int)):
        spec[row] = np.bincount(s, weights=np.broadcast_to(dens, shape).ravel(), minlength=ns)

    return {
        "mass": float(np.mean(rho)),
        "energy": energy(psi, alpha, beta, engine),
        "e_kin": e_kin,
        "e_kin_i": float(spec[0].sum()),
        "e_kin_c": float(spec[1].sum()),
        "e_q": float(spec[2].sum()),
        "e_int": e_int,
        "spec": spec,
        "npts": npts,
    }


def structure_function_density(psi, p: int = 2):
    """Second-order (or order p) structure function of rho = |psi|^2 along the
    three axes, from the definition (strfunc-def with v -> rho, spatial mean):
    S(m) = (1/3) sum_axes <(rho(x + m dx e) - rho(x))^p>, m = 1..N/2.
    Returns an array of shape (N/2,) for a cubic grid."""
    rho = np.abs(np.asarray(psi)) ** 2
    n = rho.shape[0]
    out = np.zeros(n // 2)
    for m in range(1, n // 2 + 1):
        acc = 0.0
        for ax in range(3):
            acc += float(np.mean((np.roll(rho, -m, axis=ax) - rho) ** p))
        out[m - 1] = acc / 3.0
    return out


def velocity(psi, alpha, engine=None):
    """Superfluid velocity v = 2 alpha Im(conj(psi) grad psi) / |psi|^2 (eq. scaling-rhov
    divided by rho), 0 where |psi| = 0 exactly.  Returns [v_z, v_y, v_x]."""
    d = gradient(psi, engine)
    rho = np.abs(psi) ** 2
    safe = np.where(rho > 0.0, rho, 1.0)
    return [np.where(rho > 0.0, 2.0 * alpha * np.imag(np.conj(psi) * dj) / safe, 0.0) for dj in d]


def structure_function_velocity(psi, alpha, p: int = 2, engine=None):
    """Longitudinal velocity structure functions of eq. strfunc-def, one per axis,
    by direct lag sums: S_j(m) = < (v_j(x + m dx e_j) - v_j(x))^p >, m = 1..N_j/2
    (spatial mean over the periodic box).  Returns an array [3][N/2] in the order
    (x, y, z) for a cubic grid, and <v_j^2> per axis (the large-lag limit of S_j is
    2 <v_j^2> when v_j decorrelates, eq. strfunc-verif)."""
    vz, vy, vx = velocity(psi, alpha, engine)
    n = psi.shape[0]
    out = np.zeros((3, n // 2))
    comps = ((vx, 2), (vy, 1), (vz, 0))           # (component, array axis along it)
    for j, (v, ax) in enumerate(comps):
        for m in range(1, n // 2 + 1):
            out[j, m - 1] = float(np.mean((np.roll(v, -m, axis=ax) - v) ** p))
    mean_v2 = np.array([float(np.mean(v * v)) for v, _ in comps])
    return out, mean_v2


def mach_numbers(psi, alpha, beta, engine=None):
    """Maximum and rms Mach numbers of eq. Mach-Number: M_max = max |sqrt(rho) v| / c,
    M_rms = sqrt(2 E_kin) / c, with sqrt(rho) v = w and c = sqrt(2 alpha beta) (the sound
    speed in the paper's scaling, from xi^2 c^2 = 2 alpha^2 and xi^2 = alpha / beta)."""
    w, _ = momentum_w(psi, alpha, engine)
    w2 = w[0] ** 2 + w[1] ** 2 + w[2] ** 2
    c = math.sqrt(2.0 * alpha * beta)
    return float(np.sqrt(w2.max())) / c, math.sqrt(float(np.mean(w2))) / c


# ---------------------------------------------------------------- parameters
def table1_params(n: int):
    """Parameter rule of the numerical-results section (Table of parameters):
    L = 2 pi, M_ref = 0.5 (alpha beta = 2), k_max xi fixed, alpha = 6.4/N,
    beta = N/3.2.  Returns alpha, beta, xi, k_max xi, dx/xi, N_v^1d."""
    alpha = 6.4 / n
    beta = n / 3.2
    xi = math.sqrt(alpha / beta)                         # eq. scaling-ab
    dx = 2.0 * math.pi / n
    kmax_xi = (n / 2.0) * xi                             # k_max = pi/dx = N/2
    chi = dx / xi                                        # eq. scaling-chi
    nv1d = (2.0 * math.pi / 2.0) * math.sqrt(beta / alpha)   # eq. scaling-Nv1d
    return {"alpha": alpha, "beta": beta, "xi": xi, "kmax_xi": kmax_xi,
            "dx_over_xi": chi, "Nv1d": nv1d, "c": math.sqrt(2 * alpha * beta)}


def gamma_d_quarter(alpha: float) -> int:
    """[gamma_d / 4] = [1/(2 pi alpha)] (integer part), gamma_d = 2/(pi alpha)."""
    return int(math.floor(1.0 / (2.0 * math.pi * alpha)))
