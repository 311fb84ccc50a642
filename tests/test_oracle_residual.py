"""Pins for the residual of scheme (2.20) and its Jacobian (Sections 2 and 3.1)."""
import math

import numpy as np
import pytest

from acch_inputs import perturbed_pair
from oracle import jacobian, newton, scalar, scheme
from oracle.params import Problem

LENGTHS = (1.0, 1.3, 0.8)


def prob_for(shape, bc, **kw):
    return Problem(bc=bc, lengths=LENGTHS[:len(shape)], **kw)


@pytest.mark.parametrize("shape", [(7,), (5, 6), (4, 5, 6)])
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("mob", ["midpoint", "average", "explicit"])
def test_vectorised_matches_loop_residual(shape, bc, mob):
    prob = prob_for(shape, bc, mobility=mob, alpha=4.0, beta=2.0, gamma=0.005, rho=0.001)
    u1, v1, u0, v0 = perturbed_pair(shape, 11, amp=0.04)
    dt = 0.05
    Fu, Fv = scheme.residual(u1, v1, u0, v0, dt, prob)
    Gu, Gv = scalar.residual_loops(u1, v1, u0, v0, dt, prob)
    assert np.max(np.abs(Fu - Gu)) <= 1e-12 * np.max(np.abs(Fu))
    assert np.max(np.abs(Fv - Gv)) <= 1e-12 * np.max(np.abs(Fv))


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_constant_state_is_a_root(bc):
    shape = (6, 7)
    prob = prob_for(shape, bc)
    u = np.full(shape, 0.43)
    v = np.full(shape, 0.08)
    Fu, Fv = scheme.residual(u, v, u, v, 0.1, prob)
    # mu is constant so the flux vanishes; v != 0 makes nu != 0, so F_v = c nu / rho
    assert np.max(np.abs(Fu)) < 1e-14
    mu, nu = scheme.discrete_variational_derivative(u, v, u, v, prob)
    assert np.allclose(Fv, scheme.mobility(u, v) * nu / prob.rho, rtol=1e-14, atol=0)
    v0 = np.zeros(shape)
    Fu, Fv = scheme.residual(u, v0, u, v0, 0.1, prob)
    assert np.max(np.abs(Fu)) < 1e-14 and np.max(np.abs(Fv)) == 0.0


@pytest.mark.parametrize("shape", [(5, 6), (4, 5, 6)])
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_flux_form_conserves_mass(shape, bc):
    """sum_k F_u,k = sum_k (u1 - u0)/dt for any state: the flux terms telescope."""
    prob = prob_for(shape, bc)
    u1, v1, u0, v0 = perturbed_pair(shape, 3)
    dt = 0.02
    Fu, _ = scheme.residual(u1, v1, u0, v0, dt, prob)
    want = np.sum(u1 - u0) / dt
    assert abs(np.sum(Fu) - want) < 1e-12 * np.sum(np.abs(Fu))


def test_zero_order_parameter_stays_zero():
    """v = 0 at both levels gives p = q, hence nu = 0 and F_v = 0 exactly."""
    shape = (8, 8)
    prob = prob_for(shape, "periodic")
    u1, _, u0, _ = perturbed_pair(shape, 4)
    z = np.zeros(shape)
    _, Fv = scheme.residual(u1, z, u0, z, 0.01, prob)
    assert np.all(Fv == 0.0)


def test_neumann_equals_periodic_on_mirrored_data():
    """A cell-centred mirror image reproduces the ghost rule: Neumann on N cells equals
    periodic on 2N cells with the data reflected (in every direction)."""
    ny, nx = 5, 6
    probN = Problem(bc="neumann", lengths=(1.0, 1.3))
    probP = Problem(bc="periodic", lengths=(2.0, 2.6))
    u1, v1, u0, v0 = perturbed_pair((ny, nx), 8)
    mirror = lambda f: np.block([[f, f[:, ::-1]], [f[::-1, :], f[::-1, ::-1]]])
    Fn = scheme.residual(u1, v1, u0, v0, 0.03, probN)
    Fp = scheme.residual(mirror(u1), mirror(v1), mirror(u0), mirror(v0), 0.03, probP)
    for a, b in zip(Fn, Fp):
        assert np.max(np.abs(b[:ny, :nx] - a)) < 1e-12 * np.max(np.abs(a))
    assert abs(4 * scheme.energy(u1, v1, probN) - scheme.energy(mirror(u1), mirror(v1), probP)) \
        < 1e-12 * abs(scheme.energy(u1, v1, probN))


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_dimension_reductions(bc):
    """y-independent 2D data reduce to 1D; z-independent 3D data reduce to 2D."""
    u1, v1, u0, v0 = perturbed_pair((7,), 6)
    p1 = Problem(bc=bc, lengths=(1.0,))
    p2 = Problem(bc=bc, lengths=(1.0, 0.7))
    F1 = scheme.residual(u1, v1, u0, v0, 0.01, p1)
    tile = lambda f: np.tile(f, (4, 1))
    F2 = scheme.residual(tile(u1), tile(v1), tile(u0), tile(v0), 0.01, p2)
    for a, b in zip(F1, F2):
        assert np.max(np.abs(b - a[None, :])) < 1e-12 * np.max(np.abs(a))
    a1, b1, a0, b0 = perturbed_pair((5, 6), 12)
    p3 = Problem(bc=bc, lengths=(1.0, 0.7, 0.9))
    p2b = Problem(bc=bc, lengths=(1.0, 0.7))
    F2 = scheme.residual(a1, b1, a0, b0, 0.01, p2b)
    t3 = lambda f: np.tile(f, (3, 1, 1))
    F3 = scheme.residual(t3(a1), t3(b1), t3(a0), t3(b0), 0.01, p3)
    for a, b in zip(F2, F3):
        assert np.max(np.abs(b - a[None])) < 1e-12 * np.max(np.abs(a))


@pytest.mark.parametrize("field", ["u", "v"])
def test_linearised_single_mode_growth(field):
    """About (ubar, 0) a Fourier mode of amplitude eps is multiplied by
    g = (1 - dt a/2)/(1 + dt a/2) per step, with
    a_u = c lambda_h (-alpha + 2 theta/(u(1-u)) + gamma lambda_h) and
    a_v = (c/rho)(-beta + 2 theta/(u(1-u)) + gamma lambda_h), c = u(1-u)/4 —
    the Crank–Nicolson symbol of the linearised discrete operator."""
    n, ub, eps, m = 32, 0.45, 1e-7, 3
    prob = Problem(bc="periodic", lengths=(1.0, 1.0), alpha=1.2, beta=1.2, theta=0.1, gamma=1e-3)
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    mode = np.tile(np.cos(2 * math.pi * m * x), (n, 1))
    u0 = np.full((n, n), ub)
    v0 = np.zeros((n, n))
    if field == "u":
        u0 = u0 + eps * mode
    else:
        v0 = v0 + eps * mode
    dt = 2e-3
    res = newton.solve_step(u0, v0, dt, prob, newton.NewtonOptions(rtol=1e-14, atol=1e-15, max_it=20))
    X = res.X
    u1 = X[:n * n].reshape(n, n)
    v1 = X[n * n:].reshape(n, n)
    f1 = (u1 - ub) if field == "u" else v1
    amp = np.sum(f1 * mode) / np.sum(mode * mode) / eps
    lam = 4 / h ** 2 * math.sin(2 * math.pi * m * h / 2) ** 2
    cbar = ub * (1 - ub) / 4
    core = 2 * prob.theta / (ub * (1 - ub)) + prob.gamma * lam
    a = cbar * lam * (-prob.alpha + core) if field == "u" else cbar / prob.rho * (-prob.beta + core)
    g = (1 - dt * a / 2) / (1 + dt * a / 2)
    assert abs(amp - g) < 1e-6


@pytest.mark.parametrize("shape", [(6, 5), (4, 4, 5)])
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("mob", ["midpoint", "average"])
def test_jacobian_matches_complex_step(shape, bc, mob):
    """The analytic Jacobian equals the complex-step derivative Im F(X + i t e_k)/t
    (exact to rounding for the analytic residual)."""
    prob = prob_for(shape, bc, mobility=mob)
    u1, v1, u0, v0 = perturbed_pair(shape, 21, amp=0.05)
    dt = 0.05
    n = u1.size
    X = np.concatenate([u1.ravel(), v1.ravel()]).astype(complex)
    U0 = np.concatenate([u0.ravel(), v0.ravel()]).astype(complex)
    J = jacobian.jacobian(u1, v1, u0, v0, dt, prob).toarray()
    Jcs = np.zeros_like(J)
    t = 1e-30
    for k in range(2 * n):
        Xc = X.copy()
        Xc[k] += 1j * t
        Jcs[:, k] = scheme.residual_vec(Xc, U0, dt, prob, shape).imag / t
    assert np.max(np.abs(J - Jcs)) <= 1e-14 * np.max(np.abs(J))


def test_jacobian_matches_central_differences():
    shape = (5, 6)
    prob = prob_for(shape, "neumann")
    u1, v1, u0, v0 = perturbed_pair(shape, 2)
    J = jacobian.jacobian(u1, v1, u0, v0, 0.01, prob).toarray()
    Jfd = jacobian.jacobian_fd(u1, v1, u0, v0, 0.01, prob)
    assert np.max(np.abs(J - Jfd)) <= 1e-6 * np.max(np.abs(J))


def test_jacobian_structure_2d():
    """Row patterns: F_u couples u on the radius-2 diamond and v on the radius-1 star;
    F_v couples v on the star and u at the cell (24 entries per cell in 2D)."""
    shape = (8, 9)
    prob = prob_for(shape, "periodic")
    u1, v1, u0, v0 = perturbed_pair(shape, 2)
    J = jacobian.jacobian(u1, v1, u0, v0, 0.01, prob)
    n = u1.size
    nnz = (np.abs(J.toarray()) > 0).sum(axis=1)
    assert np.all(nnz[:n] == 13 + 5)
    assert np.all(nnz[n:] == 5 + 1)
