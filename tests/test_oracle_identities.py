"""Pins for the discrete operators and energy of Section 2: summation by parts
(eq. summation), semi-positivity (eq. neq:02), the DVD identity (eq. DVD) for each
part of the energy, and closed forms of the energy on simple states."""
import math

import numpy as np
import pytest

from acch_inputs import perturbed_pair
from oracle import scheme
from oracle.params import Problem

SHAPES = [(7,), (6, 9), (5, 4, 6)]
LENGTHS = (1.0, 1.3, 0.8)


def prob_for(shape, bc, **kw):
    return Problem(bc=bc, lengths=LENGTHS[:len(shape)], **kw)


def inner(a, b, prob, shape):
    return float(np.sum(a * b) * scheme.cell_volume(shape, prob))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_summation_by_parts(shape, bc):
    """-sum phi [D c D psi] = 1/2 sum (c_{+} D+phi D+psi + c_{-} D-phi D-psi) per axis."""
    prob = prob_for(shape, bc)
    h = prob.spacing(shape)
    rng = np.random.default_rng(1)
    phi, psi = rng.standard_normal(shape), rng.standard_normal(shape)
    c = rng.uniform(0.1, 1.0, size=shape)
    lhs = -np.sum(phi * scheme.div_c_grad(c, psi, h, bc))
    rhs = 0.0
    for a in range(len(shape)):
        cf = scheme.face_avg(c, a, bc)
        dphi = scheme.face_diff(phi, a, bc) / h[a]
        dpsi = scheme.face_diff(psi, a, bc) / h[a]
        terms = cf * dphi * dpsi
        lo = [slice(None)] * len(shape)
        hi = [slice(None)] * len(shape)
        lo[a] = slice(0, -1)
        hi[a] = slice(1, None)
        rhs += 0.5 * np.sum(terms[tuple(hi)] + terms[tuple(lo)])
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_operator_semi_positive_and_symmetric(shape, bc):
    prob = prob_for(shape, bc)
    h = prob.spacing(shape)
    rng = np.random.default_rng(2)
    phi, psi = rng.standard_normal(shape), rng.standard_normal(shape)
    c = rng.uniform(0.0, 1.0, size=shape)
    A = lambda f: -scheme.div_c_grad(c, f, h, bc)
    assert np.sum(phi * A(phi)) >= 0
    assert abs(np.sum(phi * A(psi)) - np.sum(psi * A(phi))) < 1e-11 * np.sum(np.abs(phi * A(psi)))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_dvd_identity_polynomial_parts(shape, bc):
    """E1 and E3 parts: E(U1) - E(U0) = <G_i . (U1 - U0)> exactly (eq. DVD)."""
    prob = prob_for(shape, bc, alpha=4.0, beta=2.0, gamma=0.005, theta=0.1)
    h = prob.spacing(shape)
    u1, v1, u0, v0 = perturbed_pair(shape, 5, amp=0.05)
    vol = scheme.cell_volume(shape, prob)
    e1 = lambda u, v: np.sum(0.5 * prob.alpha * u * (1 - u) - 0.5 * prob.beta * v * v) * vol
    G1u = -0.5 * prob.alpha * (u1 + u0 - 1)
    G1v = -0.5 * prob.beta * (v1 + v0)
    lhs = e1(u1, v1) - e1(u0, v0)
    rhs = inner(G1u, u1 - u0, prob, shape) + inner(G1v, v1 - v0, prob, shape)
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1e-300) + 1e-17
    e3 = lambda u, v: 0.5 * prob.gamma * np.sum(scheme.gradient_energy_density(u, h, bc)
                                                + scheme.gradient_energy_density(v, h, bc)) * vol
    G3u = -0.5 * prob.gamma * (scheme.laplacian(u1, h, bc) + scheme.laplacian(u0, h, bc))
    G3v = -0.5 * prob.gamma * (scheme.laplacian(v1, h, bc) + scheme.laplacian(v0, h, bc))
    lhs = e3(u1, v1) - e3(u0, v0)
    rhs = inner(G3u, u1 - u0, prob, shape) + inner(G3v, v1 - v0, prob, shape)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_dvd_identity_full_energy(shape, bc):
    """E~(U1) - E~(U0) = <G~ . (U1 - U0)> with the exact divided difference G2 of eq. D2,
    and the series G2^S reproduces it within its truncation error."""
    prob = prob_for(shape, bc, alpha=4.0, beta=2.0, gamma=0.005, theta=0.1)
    h = prob.spacing(shape)
    u1, v1, u0, v0 = perturbed_pair(shape, 9, amp=0.05)
    phi = scheme.g2_exact(u1 + v1, u0 + v0)
    psi = scheme.g2_exact(u1 - v1, u0 - v0)
    Gu = (-0.5 * prob.alpha * (u1 + u0 - 1) + prob.theta * (phi + psi)
          - 0.5 * prob.gamma * (scheme.laplacian(u1, h, bc) + scheme.laplacian(u0, h, bc)))
    Gv = (-0.5 * prob.beta * (v1 + v0) + prob.theta * (phi - psi)
          - 0.5 * prob.gamma * (scheme.laplacian(v1, h, bc) + scheme.laplacian(v0, h, bc)))
    dE = scheme.energy(u1, v1, prob) - scheme.energy(u0, v0, prob)
    rhs = inner(Gu, u1 - u0, prob, shape) + inner(Gv, v1 - v0, prob, shape)
    assert abs(dE - rhs) <= 1e-11 * abs(dE)
    mu, nu = scheme.discrete_variational_derivative(u1, v1, u0, v0, prob)
    rhs_s = inner(mu, u1 - u0, prob, shape) + inner(nu, v1 - v0, prob, shape)
    assert abs(dE - rhs_s) <= 1e-11 * abs(dE)


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_energy_of_constant_state(bc):
    """A constant state carries only bulk energy: E = |Omega| e(u, v)."""
    shape = (6, 8)
    prob = prob_for(shape, bc, alpha=4.0, beta=2.0, theta=0.1)
    u, v = 0.41, -0.07
    U = np.full(shape, u)
    V = np.full(shape, v)
    area = LENGTHS[0] * LENGTHS[1]
    Phi = lambda z: z * math.log(z) + (1 - z) * math.log(1 - z)
    e = 0.5 * 4.0 * u * (1 - u) - 0.5 * 2.0 * v * v + 0.1 * (Phi(u + v) + Phi(u - v))
    assert abs(scheme.energy(U, V, prob) - area * e) < 1e-14 * abs(area * e) + 1e-16


def test_gradient_energy_of_fourier_mode():
    """u = A cos(k x) on a periodic 1D grid: sum of (D^±u)^2 equals N A^2 (1 - cos kh)/h^2."""
    n, L, A, m = 24, 1.0, 0.1, 3
    h = L / n
    x = (np.arange(n) + 0.5) * h
    k = 2 * math.pi * m / L
    u = A * np.cos(k * x)
    got = np.sum(scheme.gradient_energy_density(u, (h,), "periodic"))
    want = n * A * A * (1 - math.cos(k * h)) / (h * h)
    assert abs(got - want) < 1e-12 * want


def test_laplacian_symbol():
    """The 5-point Laplacian acting on a periodic mode multiplies it by -lambda_h."""
    ny, nx = 12, 16
    prob = Problem(bc="periodic", lengths=(1.0, 1.5))
    hy, hx = prob.spacing((ny, nx))
    X, Y = np.meshgrid((np.arange(nx) + 0.5) * hx, (np.arange(ny) + 0.5) * hy)
    kx, ky = 2 * math.pi * 2 / 1.0, 2 * math.pi * 1 / 1.5
    f = np.cos(kx * X) * np.cos(ky * Y)
    lam = 4 / hx ** 2 * math.sin(kx * hx / 2) ** 2 + 4 / hy ** 2 * math.sin(ky * hy / 2) ** 2
    assert np.max(np.abs(scheme.laplacian(f, (hy, hx), "periodic") + lam * f)) < 1e-10 * lam
