"""Pins for the oracle's discrete adjoint: each building block against complex-step
derivatives, and the whole gradient against central differences of the forward run."""
import numpy as np
import pytest

from acch_inputs import perturbed_pair, random_ic
from oracle import adjoint, scheme
from oracle.newton import NewtonOptions
from oracle.params import Problem


def _complex_step(fun, x, t=1e-30):
    return fun(x + 1j * t).imag / t


def _energy(u, v, prob):
    """E~ without the float() of scheme.energy, so that a complex step survives."""
    return np.sum(scheme.energy_density(u, v, prob)) * scheme.cell_volume(u.shape, prob)


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("mob", ["midpoint", "average", "explicit"])
def test_previous_state_jacobian_matches_complex_step(bc, mob):
    shape = (5, 6)
    prob = Problem(bc=bc, lengths=(1.0, 1.2), mobility=mob)
    u1, v1, u0, v0 = perturbed_pair(shape, 3, amp=0.04)
    dt = 0.02
    n = u1.size
    X1 = np.concatenate([u1.ravel(), v1.ravel()]).astype(complex)
    X0 = np.concatenate([u0.ravel(), v0.ravel()]).astype(complex)
    B = adjoint.previous_state_jacobian(u1, v1, u0, v0, dt, prob).toarray()
    Bcs = np.zeros_like(B)
    for k in range(2 * n):
        e = np.zeros(2 * n, dtype=complex)
        e[k] = 1.0
        Bcs[:, k] = _complex_step(lambda z: scheme.residual_vec(X1, X0 + z * e, dt, prob, shape), 0.0)
    assert np.max(np.abs(B - Bcs)) <= 1e-14 * np.max(np.abs(B))


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_parameter_derivatives_match_complex_step(bc):
    shape = (6, 5)
    u1, v1, u0, v0 = perturbed_pair(shape, 4, amp=0.04)
    base = Problem(bc=bc, lengths=(1.0, 0.9))
    dt = 0.03
    pd = adjoint.parameter_derivatives(u1, v1, u0, v0, dt, base)
    X1 = np.concatenate([u1.ravel(), v1.ravel()])
    X0 = np.concatenate([u0.ravel(), v0.ravel()])
    for name in adjoint.PARAMS:
        val = getattr(base, name)
        got = _complex_step(lambda z: scheme.residual_vec(X1.astype(complex), X0.astype(complex), dt,
                                                          base.with_(**{name: val + z}), shape), 0.0)
        assert np.max(np.abs(pd[name] - got)) <= 1e-13 * np.max(np.abs(got))


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_energy_gradient_matches_complex_step(bc):
    shape = (6, 7)
    u, v = random_ic(shape, 5)
    prob = Problem(bc=bc, lengths=(1.0, 1.1))
    gu, gv, gp = adjoint.energy_gradient(u, v, prob)
    for k in [(0, 0), (2, 3), (5, 6)]:
        e = np.zeros(shape)
        e[k] = 1.0
        assert abs(gu[k] - _complex_step(lambda z: _energy(u + z * e, v, prob), 0.0)) < 1e-13
        assert abs(gv[k] - _complex_step(lambda z: _energy(u, v + z * e, prob), 0.0)) < 1e-13
    for name in adjoint.PARAMS:
        val = getattr(prob, name)
        cs = _complex_step(lambda z: _energy(u, v, prob.with_(**{name: val + z})), 0.0)
        assert abs(gp[name] - cs) <= 1e-13 * max(1.0, abs(cs)), name


@pytest.mark.slow
@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_adjoint_gradient_matches_central_differences(bc):
    """dE~(U^N)/d(u0, v0, alpha, beta, theta, gamma) with the dt sequence frozen, against
    central differences of the forward run with tight Newton tolerances (relative error
    <= 1e-6)."""
    shape = (8, 8)
    prob = Problem(bc=bc, alpha=1.2, beta=1.2, theta=0.1, gamma=2e-3)
    u0, v0 = random_ic(shape, 7)
    dts = [2e-3, 3e-3, 3e-3]
    opts = NewtonOptions(rtol=1e-12, atol=1e-11)
    E, gu, gv, gp = adjoint.gradient(u0, v0, dts, prob, opts)

    def energy_of(u, v, p):
        st = adjoint.forward(u, v, dts, p, opts)
        return scheme.energy(*st[-1], p)

    h = 1e-6
    for name in adjoint.PARAMS:
        g = gp[name]
        val = getattr(prob, name)
        fd = (energy_of(u0, v0, prob.with_(**{name: val + h * val}))
              - energy_of(u0, v0, prob.with_(**{name: val - h * val}))) / (2 * h * val)
        assert abs(g - fd) <= 1e-6 * abs(fd), (name, g, fd)
    rng = np.random.default_rng(0)
    d = rng.uniform(-1, 1, shape)
    eps = 1e-5
    fd = (energy_of(u0, v0 + eps * d, prob) - energy_of(u0, v0 - eps * d, prob)) / (2 * eps)
    assert abs(np.sum(gv * d) - fd) <= 1e-6 * abs(fd)
    fd = (energy_of(u0 + eps * d, v0, prob) - energy_of(u0 - eps * d, v0, prob)) / (2 * eps)
    assert abs(np.sum(gu * d) - fd) <= 1e-6 * abs(fd)
