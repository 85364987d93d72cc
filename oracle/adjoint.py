"""Adjoint of the Strang split step and the spectral loss -- the oracle.

TEST INFRASTRUCTURE ONLY (plain numpy FP64).

Real inner product on complex fields: <a, b> = Re sum_x conj(a) b.  A
gradient field ``lam`` of a real functional J(psi) is defined by
dJ = <lam, dpsi>.

Forward step (time-evolution section, eq. adi_looptime):
    psi_{n+1} = L(h) N(L(h) psi_n),   h = dt/2,
    L(h) = F^-1 exp(-i alpha |k|^2 h) F,   N(phi) = u phi,
    u = exp(-i beta (|phi|^2 - 1) dt).
Adjoints:
    L(h)^dagger = L(-h)                         (L is unitary),
    N'(phi)^dagger lam = conj(u) lam + 2 beta dt Im(conj(lam) u phi) phi,
so one backward step is lam_n = L(-h) N'(phi_n)^dagger L(-h) lam_{n+1} with
phi_n = L(h) psi_n.

Loss (final-time spectral energy): J = 1/2 sum_{k: smin <= s(k) <= smax} |w^i_k|^2
with w = 2 alpha Im(conj(psi) grad psi)/|psi| and w^i its incompressible part.
Its gradient, derived by the chain rule with the spectral derivative D_j
(antisymmetric because its Nyquist entry is zero):
    G_j = N^-3 * inverse-unnormalised(mask * w^i)_j       (real fields)
    h_j = 2 alpha G_j / |psi|
    lam = sum_j [ -i h_j D_j psi  - i D_j(h_j psi)  - G_j w_j psi / |psi|^2 ]
(terms with 1/|psi| are zero where |psi| = 0 exactly).
Phase gradient for psi_0 = exp(i theta): dJ/dtheta = Im(lam_0 conj(psi_0)).
"""
from __future__ import annotations

import numpy as np

from .fft import fft3, ifft3
from .gp import (linear_substep, nonlinear_substep, gradient, momentum_w,
                 helmholtz, shell_index, grids_k, first_derivative_k)

__all__ = ["inner", "nonlinear_adjoint", "nonlinear_tangent", "step_adjoint",
           "forward_states", "loss_ekin_i_shells", "loss_gradient",
           "phase_gradient", "gradient_theta"]


def inner(a, b) -> float:
    """Real inner product Re sum conj(a) b."""
    return float(np.real(np.vdot(a, b)))


def nonlinear_tangent(phi, dphi, beta, dt):
    """Linearisation of N at phi applied to dphi:
    N'(phi) dphi = u dphi - 2 i beta dt Re(conj(phi) dphi) u phi."""
    rho = np.abs(phi) ** 2
    u = np.exp(-1j * beta * (rho - 1.0) * dt)
    return u * dphi - 2j * beta * dt * np.real(np.conj(phi) * dphi) * u * phi


def nonlinear_adjoint(phi, lam, beta, dt):
    """N'(phi)^dagger lam = conj(u) lam + 2 beta dt Im(conj(lam) u phi) phi."""
    rho = np.abs(phi) ** 2
    u = np.exp(-1j * beta * (rho - 1.0) * dt)
    psi_p = u * phi
    return np.conj(u) * lam + 2.0 * beta * dt * np.imag(np.conj(lam) * psi_p) * phi


def step_adjoint(psi_n, lam_next, alpha, beta, dt, engine=None):
    """One backward step lam_n = L(-h) N'(phi_n)^dagger L(-h) lam_{n+1}."""
    h = 0.5 * dt
    phi = linear_substep(psi_n, alpha, h, engine)
    lam = linear_substep(lam_next, alpha, -h, engine)
    lam = nonlinear_adjoint(phi, lam, beta, dt)
    return linear_substep(lam, alpha, -h, engine)


def forward_states(psi0, alpha, beta, dt, nsteps, engine=None):
    """All states psi_0 .. psi_n of the literal Strang evolution."""
    from .gp import strang_step
    states = [np.array(psi0, dtype=np.complex128)]
    for _ in range(nsteps):
        states.append(strang_step(states[-1], alpha, beta, dt, engine))
    return states


def _shell_mask(shape, smin, smax):
    kz, ky, kx = grids_k(shape)
    s = shell_index(kx * kx + ky * ky + kz * kz)
    return np.broadcast_to((s >= smin) & (s <= smax), shape)


def loss_ekin_i_shells(psi, alpha, smin, smax, engine=None) -> float:
    """J = 1/2 sum over shells smin..smax of |w^i_k|^2 (normalised spectra)."""
    w, _ = momentum_w(psi, alpha, engine)
    w_hat = [fft3(wj, engine) for wj in w]
    wi, _ = helmholtz(w_hat, psi.shape)
    m = _shell_mask(psi.shape, smin, smax)
    return 0.5 * float(sum(np.sum(np.abs(x[m]) ** 2) for x in wi))


def loss_gradient(psi, alpha, smin, smax, engine=None):
    """(J, lam) with dJ = <lam, dpsi> (formula in the module docstring)."""
    psi = np.asarray(psi, dtype=np.complex128)
    shape = psi.shape
    npts = float(np.prod(shape))
    w, d = momentum_w(psi, alpha, engine)
    w_hat = [fft3(wj, engine) for wj in w]
    wi, _ = helmholtz(w_hat, shape)
    m = _shell_mask(shape, smin, smax)
    J = 0.5 * float(sum(np.sum(np.abs(x[m]) ** 2) for x in wi))
    # G_j = N^-3 * unnormalised inverse transform of the masked w^i
    G = [np.real(ifft3(np.where(m, x, 0.0), engine)) / npts for x in wi]
    amp = np.abs(psi)
    nz = amp > 0.0
    safe = np.where(nz, amp, 1.0)
    lam = np.zeros(shape, dtype=np.complex128)
    for j in range(3):
        hj = np.where(nz, 2.0 * alpha * G[j] / safe, 0.0)
        # spectral derivative of h_j psi along axis j
        c = fft3(hj * psi, engine)
        sh = [1, 1, 1]
        sh[j] = shape[j]
        kj = first_derivative_k(shape[j]).reshape(sh)
        d_hpsi = ifft3(1j * kj * c, engine)
        lam += -1j * hj * d[j] - 1j * d_hpsi
        lam -= np.where(nz, G[j] * w[j] * psi / (safe * safe), 0.0)
    return J, lam


def phase_gradient(psi0, lam0):
    """dJ/dtheta for psi0 = exp(i theta): Im(lam0 conj(psi0))."""
    return np.imag(lam0 * np.conj(psi0))


def gradient_theta(theta, alpha, beta, dt, nsteps, smin, smax, engine=None):
    """Full reverse-mode gradient of J(psi_M(theta)) by storing every state."""
    psi0 = np.exp(1j * np.asarray(theta, dtype=np.float64))
    states = forward_states(psi0, alpha, beta, dt, nsteps, engine)
    J, lam = loss_gradient(states[-1], alpha, smin, smax, engine)
    for n in range(nsteps - 1, -1, -1):
        lam = step_adjoint(states[n], lam, alpha, beta, dt, engine)
    return J, phase_gradient(psi0, lam), lam
