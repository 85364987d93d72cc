"""Pins of the oracle's adjoint: dot-product identities per sub-operator,
brute-force finite differences of the whole gradient, invariances."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import gp
import gp_inputs as I


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_nonlinear_tangent_is_derivative():
    """N'(phi) dphi from the linearisation equals central differences of N."""
    phi = I.random_field(6, seed=1)
    dphi = _rand((6, 6, 6), 2)
    beta, dt, h = 3.0, 0.05, 1e-6
    fd = (gp.nonlinear_substep(phi + h * dphi, beta, dt) - gp.nonlinear_substep(phi - h * dphi, beta, dt)) / (2 * h)
    assert np.abs(fd - A.nonlinear_tangent(phi, dphi, beta, dt)).max() < 1e-8


def test_dot_product_nonlinear():
    phi, lam, d = I.random_field(6, seed=3), _rand((6, 6, 6), 4), _rand((6, 6, 6), 5)
    beta, dt = 2.0, 0.1
    lhs = A.inner(lam, A.nonlinear_tangent(phi, d, beta, dt))
    rhs = A.inner(A.nonlinear_adjoint(phi, lam, beta, dt), d)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_dot_product_linear():
    lam, d = _rand((8, 6, 4), 6), _rand((8, 6, 4), 7)
    lhs = A.inner(lam, gp.linear_substep(d, 0.6, 0.3))
    rhs = A.inner(gp.linear_substep(lam, 0.6, -0.3), d)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_step_adjoint_dot_product():
    """<lam, S'(psi) d> = <S'(psi)^dagger lam, d>, S' from central differences."""
    psi = I.random_field(6, seed=8)
    lam, d = _rand((6, 6, 6), 9), _rand((6, 6, 6), 10)
    alpha, beta, dt, h = 0.4, 2.0, 0.05, 1e-6
    Sd = (gp.strang_step(psi + h * d, alpha, beta, dt) - gp.strang_step(psi - h * d, alpha, beta, dt)) / (2 * h)
    lhs = A.inner(lam, Sd)
    rhs = A.inner(A.step_adjoint(psi, lam, alpha, beta, dt), d)
    assert abs(lhs - rhs) < 1e-8 * abs(lhs)


def test_loss_gradient_fd_random_directions():
    psi = I.random_field(8, seed=11, amp_noise=0.2)
    alpha, smin, smax = 0.3, 1, 3
    J, lam = A.loss_gradient(psi, alpha, smin, smax)
    assert abs(J - A.loss_ekin_i_shells(psi, alpha, smin, smax)) < 1e-14 * J
    for s in range(4):
        d = _rand((8, 8, 8), 100 + s)
        h = 1e-6
        fd = (A.loss_ekin_i_shells(psi + h * d, alpha, smin, smax)
              - A.loss_ekin_i_shells(psi - h * d, alpha, smin, smax)) / (2 * h)
        assert abs(fd - A.inner(lam, d)) < 1e-7 * abs(fd)


def test_full_gradient_brute_force_every_component():
    """dJ/dtheta at every one of the 8^3 grid points against central differences."""
    n, alpha, beta, dt, steps, smin, smax = 8, 0.3, 2.0, 0.01, 6, 1, 3
    theta = I.srp_fourier_theta(n, 2, 31)
    J, g, _ = A.gradient_theta(theta, alpha, beta, dt, steps, smin, smax)
    h = 1e-6
    fd = np.zeros_like(theta)
    flat = theta.ravel()
    for i in range(flat.size):
        tp = flat.copy(); tp[i] += h
        tm = flat.copy(); tm[i] -= h
        Jp = A.loss_ekin_i_shells(gp.evolve(np.exp(1j * tp.reshape(theta.shape)), alpha, beta, dt, steps), alpha, smin, smax)
        Jm = A.loss_ekin_i_shells(gp.evolve(np.exp(1j * tm.reshape(theta.shape)), alpha, beta, dt, steps), alpha, smin, smax)
        fd.ravel()[i] = (Jp - Jm) / (2 * h)
    scale = np.abs(fd).max()
    assert np.abs(fd - g).max() < 1e-7 * scale


def test_global_phase_invariance():
    """J is invariant under psi -> exp(ic) psi, so sum_x dJ/dtheta = 0."""
    theta = I.srp_fourier_theta(8, 2, 5)
    _, g, _ = A.gradient_theta(theta, 0.3, 2.0, 0.01, 10, 1, 3)
    assert abs(g.sum()) < 1e-12 * np.abs(g).sum()


def test_grid_shift_equivariance():
    """Shifting theta by whole grid cells shifts the gradient the same way."""
    theta = I.srp_fourier_theta(8, 2, 6)
    _, g, _ = A.gradient_theta(theta, 0.3, 2.0, 0.01, 5, 1, 3)
    _, gs, _ = A.gradient_theta(np.roll(theta, (1, 2, 3), axis=(0, 1, 2)), 0.3, 2.0, 0.01, 5, 1, 3)
    assert np.abs(np.roll(g, (1, 2, 3), axis=(0, 1, 2)) - gs).max() < 1e-12 * np.abs(g).max()


def test_adjoint_reversibility_of_forward():
    """Forward then backward (time-reversed) steps return the start state."""
    psi0 = I.random_field(8, seed=13)
    st = A.forward_states(psi0, 0.5, 2.0, 0.02, 20)
    back = gp.evolve(st[-1], 0.5, 2.0, 0.02, -20)
    assert np.linalg.norm(back - psi0) / np.linalg.norm(psi0) < 1e-13
