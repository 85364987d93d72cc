"""Helicity and regularized helicity of the superfluid -- the oracle.

TEST INFRASTRUCTURE ONLY (plain, slow, FP64, obviously correct).  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may use it; the product never does.

Section "Helicity" of the paper: H = <v . omega> (eq. helicity, per unit volume)
with omega = curl v, and the regularized helicity H_reg = <v_reg . omega>
(eq. Hreg) with, in the paper's scaling (hbar/m -> 2 alpha),

    W       = (2 alpha / i) grad psi* x grad psi = 4 alpha grad(Re psi) x grad(Im psi)
    v_par   = 2 alpha W . J / (|W| |grad psi|^2),
              J_i = Im( sum_j (d_i d_j psi) (d_j psi)* )
    v_reg   = v_par W / |W|      (0 where |W| = 0 or grad psi = 0).

Readings: v_par divides by |grad psi|^2, which vanishes at the critical points
of psi (not at vortex cores, where |grad psi|^2 ~ 1/(2 xi^2)); there v_reg is
set to 0 where |grad psi|^2 <= 1e-12 <|grad psi|^2> (a symmetric field such as
the Taylor-Green state has such points exactly on the grid, and the quantum
vorticity vanishes there).  The floor is not a free parameter: the values of
|grad psi|^2 it removes are rounding-level zeros (below 1e-24 of the mean), and
H_reg is unchanged to 1e-12 as the floor moves from 1e-20 to 1e-10
(tests/test_oracle_helicity.py).  All derivatives are spectral with the first-derivative wavenumbers
(Nyquist entry 0), second derivatives are two first derivatives (-k_i k_j);
v = 2 alpha Im(psi* grad psi)/|psi|^2 (0 where psi = 0); omega = curl v taken
spectrally from that v.  Spectra: integer shells round(|k|), H(k) = sum over the
shell of Re(conj(v_k) . omega_k) with per-unit-volume normalised transforms, so
each spectrum sums to its helicity (Parseval).
"""
from __future__ import annotations

import numpy as np

from .fft import fft3, ifft3
from .gp import first_derivative_k, gradient, grids_k, nshell, shell_index, velocity

__all__ = ["derivative", "curl", "pseudo_vorticity", "v_parallel", "helicity", "G2_FLOOR"]

G2_FLOOR = 1e-12     # v_reg = 0 where |grad psi|^2 <= G2_FLOOR <|grad psi|^2>


def derivative(f, axis: int, engine=None):
    """Spectral first derivative of a complex or real field along array axis
    (0 = z, 1 = y, 2 = x) with the Nyquist entry zeroed."""
    n = f.shape[axis]
    shape = [1, 1, 1]
    shape[axis] = n
    k = first_derivative_k(n).reshape(shape)
    out = ifft3(1j * k * fft3(f, engine), engine)
    return out.real if np.isrealobj(f) else out


def curl(v, engine=None):
    """omega = curl v for v = [v_z, v_y, v_x]; returns [omega_z, omega_y, omega_x]."""
    vz, vy, vx = v
    d = lambda f, ax: derivative(f, ax, engine)
    wx = d(vz, 1) - d(vy, 0)          # d_y v_z - d_z v_y
    wy = d(vx, 0) - d(vz, 2)          # d_z v_x - d_x v_z
    wz = d(vy, 2) - d(vx, 1)          # d_x v_y - d_y v_x
    return [wz, wy, wx]


def pseudo_vorticity(psi, alpha, engine=None):
    """W = 4 alpha grad(Re psi) x grad(Im psi), as [W_z, W_y, W_x]."""
    dz, dy, dx = gradient(psi, engine)
    ax, ay, az = dx.real, dy.real, dz.real
    bx, by, bz = dx.imag, dy.imag, dz.imag
    wx = ay * bz - az * by
    wy = az * bx - ax * bz
    wz = ax * by - ay * bx
    return [4 * alpha * wz, 4 * alpha * wy, 4 * alpha * wx]


def v_parallel(psi, alpha, engine=None):
    """v_par and the unit vector W/|W| ([z, y, x]); both 0 where |W| = 0 or
    |grad psi|^2 <= G2_FLOOR <|grad psi|^2>."""
    d = gradient(psi, engine)                      # [d_z, d_y, d_x] psi
    hess = [[derivative(d[j], i, engine) for j in range(3)] for i in range(3)]   # hess[i][j] = d_i d_j psi
    J = [np.imag(sum(hess[i][j] * np.conj(d[j]) for j in range(3))) for i in range(3)]
    W = pseudo_vorticity(psi, alpha, engine)
    wn = np.sqrt(W[0] ** 2 + W[1] ** 2 + W[2] ** 2)
    g2 = sum(np.abs(dj) ** 2 for dj in d)
    ok = (wn > 0.0) & (g2 > G2_FLOOR * float(np.mean(g2)))
    wn_s = np.where(ok, wn, 1.0)
    g2_s = np.where(ok, g2, 1.0)
    vpar = np.where(ok, 2.0 * alpha * (W[0] * J[0] + W[1] * J[1] + W[2] * J[2]) / (wn_s * g2_s), 0.0)
    unit = [np.where(ok, Wi / wn_s, 0.0) for Wi in W]
    return vpar, unit


def helicity(psi, alpha, engine=None):
    """H, H_reg (per unit volume) and their shell spectra [2][nshell]."""
    psi = np.asarray(psi, dtype=np.complex128)
    shape = psi.shape
    v = velocity(psi, alpha, engine)
    om = curl(v, engine)
    vpar, unit = v_parallel(psi, alpha, engine)
    vreg = [vpar * u for u in unit]
    H = float(np.mean(sum(v[j] * om[j] for j in range(3))))
    Hreg = float(np.mean(sum(vreg[j] * om[j] for j in range(3))))
    oh = [fft3(o, engine) for o in om]
    dens_h = sum(np.real(np.conj(fft3(v[j], engine)) * oh[j]) for j in range(3))
    dens_r = sum(np.real(np.conj(fft3(vreg[j], engine)) * oh[j]) for j in range(3))
    kz, ky, kx = grids_k(shape)
    s = np.broadcast_to(shell_index(kx * kx + ky * ky + kz * kz), shape).ravel()
    ns = nshell(shape)
    spec = np.zeros((2, ns))
    spec[0] = np.bincount(s, weights=dens_h.ravel(), minlength=ns)
    spec[1] = np.bincount(s, weights=dens_r.ravel(), minlength=ns)
    return {"H": H, "H_reg": Hreg, "spec": spec}
