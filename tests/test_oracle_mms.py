"""Manufactured-solution order test of the oracle's scheme (2.20).

A smooth admissible periodic pair (u*, v*) is chosen; the forcing that makes it an
exact solution of the continuous system (1) is derived symbolically from the
continuous equations with the exact logarithmic Phi (not from the discrete
scheme), evaluated at cell centres at the half step t_{n+1/2}, and the oracle
solves F(U^{n+1}; U^n, dt) = f at every step.  The scheme is claimed second order
in space and time (Section 4.1): the error against (u*, v*) must fall by about 4
each time h or dt halves.  A discretisation of a different equation (a wrong
coefficient, sign or term anywhere in F) converges to something else, so its error
stalls instead.
"""
import math

import numpy as np
import pytest

from oracle import newton
from oracle.params import Problem

sy = pytest.importorskip("sympy")


def _manufactured(prob):
    x, y, t = sy.symbols("x y t", real=True)
    u = sy.Rational(1, 2) + sy.Rational(3, 10) * sy.sin(2 * sy.pi * x) * sy.sin(2 * sy.pi * y) * sy.cos(6 * t)
    v = sy.Rational(1, 10) * sy.cos(2 * sy.pi * x) * sy.sin(2 * sy.pi * y) * sy.cos(5 * t)
    a, b, th, g, rho = [sy.nsimplify(q) for q in (prob.alpha, prob.beta, prob.theta, prob.gamma, prob.rho)]
    dPhi = lambda z: sy.log(z) - sy.log(1 - z)
    lap = lambda f: sy.diff(f, x, 2) + sy.diff(f, y, 2)
    # variational derivatives of the free energy (Section 1) and the mobility c(u, v)
    mu = -a * (u - sy.Rational(1, 2)) + th * dPhi(u + v) + th * dPhi(u - v) - g * lap(u)
    nu = -b * v + th * dPhi(u + v) - th * dPhi(u - v) - g * lap(v)
    c = u * (1 - u) * (sy.Rational(1, 4) - v ** 2)
    # system (1): u_t = div(c grad mu), v_t = -(c / rho) nu, plus the forcing
    fu = sy.diff(u, t) - (sy.diff(c * sy.diff(mu, x), x) + sy.diff(c * sy.diff(mu, y), y))
    fv = sy.diff(v, t) + c * nu / rho
    lam = lambda e: sy.lambdify((x, y, t), e, "numpy")
    return lam(u), lam(v), lam(fu), lam(fv)


def _error(prob, fns, n, dt, T):
    uf, vf, fuf, fvf = fns
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc, indexing="xy")     # arrays [j][i], x fastest
    u = uf(X, Y, 0.0)
    v = vf(X, Y, 0.0)
    t = 0.0
    opts = newton.NewtonOptions(rtol=1e-9, atol=1e-12)
    for _ in range(int(round(T / dt))):
        th = t + 0.5 * dt
        f = np.concatenate([np.broadcast_to(fuf(X, Y, th), u.shape).ravel(),
                            np.broadcast_to(fvf(X, Y, th), u.shape).ravel()])
        res = newton.solve_step(u, v, dt, prob, opts, forcing=f)
        assert res.converged, res.reason
        u = res.X[:u.size].reshape(u.shape)
        v = res.X[u.size:].reshape(u.shape)
        t += dt
    return math.sqrt(np.mean((u - uf(X, Y, t)) ** 2 + (v - vf(X, Y, t)) ** 2))


@pytest.fixture(scope="module")
def mms_paper():
    """The parameters of the convergence study of Section 4.1 (rho = 1e-3 makes the
    v equation's reaction term large, so every term of F_v matters)."""
    prob = Problem(bc="periodic", alpha=4.0, beta=2.0, gamma=0.005, theta=0.1, rho=0.001)
    return prob, _manufactured(prob)


@pytest.fixture(scope="module")
def mms_bench():
    """The benchmark parameters (alpha = beta = 1.2, theta = 0.1, gamma = 1e-3, rho = 1):
    mild enough for steps of T/4 over T = 0.5, so the temporal error dominates."""
    prob = Problem(bc="periodic")
    return prob, _manufactured(prob)


@pytest.mark.slow
def test_mms_second_order_in_space(mms_paper):
    """dt = T/16 (temporal error ~1e-6) and h = 1/16, 1/32, 1/64: order 2 in h."""
    prob, fns = mms_paper
    T = 0.05
    e = [_error(prob, fns, n, T / 16, T) for n in (16, 32, 64)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(1.85 < o < 2.15 for o in orders), (e, orders)
    assert e[-1] < 5e-4


@pytest.mark.slow
def test_mms_second_order_in_time(mms_bench):
    """h = 1/32 (spatial error ~1e-4) and dt = T/4, T/8, T/16 over T = 0.5: order 2
    in dt while the temporal error dominates."""
    prob, fns = mms_bench
    T = 0.5
    e = [_error(prob, fns, 32, T / k, T) for k in (4, 8, 16)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert 1.9 < orders[0] < 2.1 and 1.75 < orders[1] < 2.1, (e, orders)
