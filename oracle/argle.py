"""Imaginary-time (ARGLE) preparation of a driven stationary state -- the oracle.

TEST INFRASTRUCTURE ONLY (plain, slow, FP64, obviously correct).  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may use it; the product never does.

Section "Numerical method to compute stationary solutions" of the paper: the
advective real Ginzburg-Landau equation (eq. gradient-flow)

    phi_tau = ( alpha lap - i v.grad - |v|^2/(4 alpha) + beta - beta |phi|^2 ) phi

with a prescribed divergence-free velocity v = v_ext, advanced by the
semi-implicit backward Euler scheme (eq. semi-backward-Euler): half of the
Laplacian at the new level, everything else at the old one,

    (phi^{n+1} - phi^n)/dtau = (alpha/2) lap phi^{n+1}
        + ( (alpha/2) lap - i v.grad - |v|^2/(4 alpha) + beta - beta |phi^n|^2 ) phi^n,

solved with Fourier transforms, where the implicit operator is diagonal.  The
energy it decreases is E_v (eq. energy-num-ext-vel), per unit volume

    E_v = 2 alpha < alpha |grad phi - i v phi / (2 alpha)|^2 + (beta/2) (|phi|^2 - 1)^2 >.

Readings (the same as for the real-time oracle): the Laplacian uses |k|^2 with
the Nyquist entry N^2/4; first derivatives (v.grad, E_v) use k with the Nyquist
entry set to zero; the field written with a tilde at the old level in
eq. semi-backward-Euler is phi^n itself.  Convergence tests of the paper:
eq. crit1 (sup norm of the update over dtau) and eq. crit2 (relative energy
change over dtau).

Velocity fields are inputs (components [v_z, v_y, v_x], each shaped like phi).
"""
from __future__ import annotations

import numpy as np

from .fft import fft3, ifft3
from .gp import gradient, ksq

__all__ = ["explicit_part", "argle_step", "argle", "energy_v", "crit_sup", "crit_energy", "argle_run"]


def explicit_part(phi, v, alpha, beta, engine=None):
    """(-i v.grad - |v|^2/(4 alpha) + beta - beta |phi|^2) phi: the part of the
    right-hand side of eq. semi-backward-Euler other than the Laplacian."""
    dz, dy, dx = gradient(phi, engine)
    vz, vy, vx = v
    adv = vx * dx + vy * dy + vz * dz
    v2 = vx * vx + vy * vy + vz * vz
    return -1j * adv + (beta - v2 / (4.0 * alpha) - beta * np.abs(phi) ** 2) * phi


def argle_step(phi, v, alpha, beta, dtau, engine=None):
    """One step of eq. semi-backward-Euler: in Fourier space
    (1 + dtau alpha |k|^2 / 2) c^{n+1} = (1 - dtau alpha |k|^2 / 2) c^n + dtau n^,
    with n = explicit_part(phi^n)."""
    k2 = ksq(phi.shape).astype(np.float64)
    c = fft3(phi, engine)
    cn = fft3(explicit_part(phi, v, alpha, beta, engine), engine)
    a = 0.5 * dtau * alpha
    return ifft3(((1.0 - a * k2) * c + dtau * cn) / (1.0 + a * k2), engine)


def argle(phi, v, alpha, beta, dtau, nsteps, engine=None, callback=None, every=0):
    """nsteps pseudo-time steps; callback(step, phi) every `every` steps."""
    phi = np.asarray(phi, dtype=np.complex128)
    for s in range(nsteps):
        phi = argle_step(phi, v, alpha, beta, dtau, engine)
        if callback is not None and every and (s + 1) % every == 0:
            callback(s + 1, phi)
    return phi


def energy_v(phi, v, alpha, beta, engine=None) -> float:
    """E_v of eq. energy-num-ext-vel, per unit volume of the periodic box."""
    d = gradient(phi, engine)
    g = sum(np.abs(dj - 1j * vj * phi / (2.0 * alpha)) ** 2 for dj, vj in zip(d, v))
    rho = np.abs(phi) ** 2
    return float(2.0 * alpha * np.mean(alpha * g + 0.5 * beta * (rho - 1.0) ** 2))


def crit_sup(phi_new, phi_old, dtau) -> float:
    """Left side of eq. crit1: ||phi^{n+1} - phi^n||_inf / dtau."""
    return float(np.max(np.abs(phi_new - phi_old)) / dtau)


def crit_energy(e_new, e_old, dtau) -> float:
    """Left side of eq. crit2: |E_v^{n+1} - E_v^n| / (dtau E_v^n)."""
    return abs(e_new - e_old) / (dtau * e_old)


def argle_run(phi, v, alpha, beta, dtau, max_steps, check_every, eps, engine=None):
    """The ARGLE procedure with its stopping rule (section on stationary solutions):
    step until eq. crit1 holds or max_steps steps are done.  The criteria are
    evaluated on every check_every-th step and on the last one (a check costs one
    extra E_v evaluation and a saved copy of phi^n); the run stops at the first
    check whose crit_sup <= eps.  Returns (phi, steps, crit_sup, crit_energy, e_v,
    converged) with the values of the last check; crit_energy is eq. crit2, the
    fallback measure when crit1 is not reached.  With max_steps = 0 nothing is
    checked: crit_sup = crit_energy = nan, e_v = E_v(phi)."""
    phi = np.asarray(phi, dtype=np.complex128)
    steps, cs, ce = 0, float("nan"), float("nan")
    while steps < max_steps:
        check = (steps + 1) % check_every == 0 or steps + 1 == max_steps
        if check:
            old, e_old = phi, energy_v(phi, v, alpha, beta, engine)
        phi = argle_step(phi, v, alpha, beta, dtau, engine)
        steps += 1
        if check:
            cs = crit_sup(phi, old, dtau)
            ce = crit_energy(energy_v(phi, v, alpha, beta, engine), e_old, dtau)
            if cs <= eps:
                return phi, steps, cs, ce, energy_v(phi, v, alpha, beta, engine), True
    return phi, steps, cs, ce, energy_v(phi, v, alpha, beta, engine), False
