"""Discrete adjoint of the time-step map of scheme (2.20) — FP64, sparse direct solves.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Step n maps U^n to U^{n+1} through F_n(U^{n+1}; U^n, dt_n, p) = 0 (Section 3.1).  For a
loss L = E~(U^N) (the discrete energy of eq. freeenergy at the last state) the chain rule
with the dt sequence held fixed gives, with A_n = dF_n/dU^{n+1} and B_n = dF_n/dU^n,

  g_N = dE~/dU^N,
  A_n^T lambda_n = g_{n+1},   g_n = -B_n^T lambda_n,   dL/dp += -lambda_n . dF_n/dp,

for n = N-1, ..., 0, plus the explicit dE~/dp at U^N.  g_0 = dL/dU^0.

Parameters p: alpha, beta, theta, gamma.  Pins (tests/test_oracle_adjoint.py): B_n, dF/dp
and dE~/d(U, p) against complex-step derivatives; the whole gradient against central
differences of the forward run.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .params import Problem
from . import scheme, jacobian
from .newton import NewtonOptions, solve_step


def g2_series_d0(x1, x0, S: int):
    """d/dx0 of g2_series: with z = (x1+x0)/2, s = (x1-x0)/2,
    1/2[f_x(z,s) - f_s(z,s) + f_x(1-z,s) + f_s(1-z,s)]."""
    zeta = 0.5 * (x1 + x0)
    sig = 0.5 * (x1 - x0)

    def fx_fs(x):
        r = sig / x
        ax = np.ones_like(r)
        asg = np.zeros_like(r)
        for m in range(1, S + 1):
            ax = ax + r ** (2 * m) / (2 * m + 1)
            asg = asg + r ** (2 * m - 1) / (2 * m + 1)
        return ax / x, -asg / x

    fx1, fs1 = fx_fs(zeta)
    fx2, fs2 = fx_fs(1.0 - zeta)
    return 0.5 * (fx1 - fs1 + fx2 + fs2)


def previous_state_jacobian(u1, v1, u0, v0, dt, prob: Problem):
    """B = dF/d(u0, v0) as a CSR matrix in the stacked order [u; v] (same operator
    composition as oracle.jacobian, differentiated in the level-n state)."""
    shape = u1.shape
    n = int(np.prod(shape))
    ops, L = jacobian.operators(shape, prob)
    mu, nu = scheme.discrete_variational_derivative(u1, v1, u0, v0, prob)
    if prob.mobility == "midpoint":
        ub = 0.5 * (u1 + u0)
        vb = 0.5 * (v1 + v0)
        c = ub * (1 - ub) * (0.25 - vb * vb)
        cu = 0.5 * (1 - 2 * ub) * (0.25 - vb * vb)
        cv = -ub * (1 - ub) * vb
    elif prob.mobility == "average":
        c = 0.5 * (scheme.mobility(u1, v1) + scheme.mobility(u0, v0))
        cu = 0.5 * (1 - 2 * u0) * (0.25 - v0 * v0)
        cv = -u0 * (1 - u0) * v0
    else:
        c = scheme.mobility(u0, v0)
        cu = (1 - 2 * u0) * (0.25 - v0 * v0)
        cv = -2 * u0 * (1 - u0) * v0
    dphi = g2_series_d0(u1 + v1, u0 + v0, prob.S)
    dpsi = g2_series_d0(u1 - v1, u0 - v0, prob.S)
    mu_u = -0.5 * prob.alpha + prob.theta * (dphi + dpsi)
    mu_v = prob.theta * (dphi - dpsi)
    nu_u = prob.theta * (dphi - dpsi)
    nu_v = -0.5 * prob.beta + prob.theta * (dphi + dpsi)
    f = lambda a: a.ravel()
    dg = sp.diags
    I = sp.identity(n, format="csr")
    Buu = -I / dt
    Buv = sp.csr_matrix((n, n))
    for G, A, D, ha in ops:
        gmu = G @ f(mu)
        ct = A @ f(c)
        Buu = Buu - D @ (dg(gmu) @ A @ dg(f(cu)) + dg(ct) @ G @ (dg(f(mu_u)) - 0.5 * prob.gamma * L)) / (ha * ha)
        Buv = Buv - D @ (dg(gmu) @ A @ dg(f(cv)) + dg(ct) @ G @ dg(f(mu_v))) / (ha * ha)
    Bvv = -I / dt + (dg(f(nu * cv)) + dg(f(c)) @ (dg(f(nu_v)) - 0.5 * prob.gamma * L)) / prob.rho
    Bvu = dg(f(nu * cu + c * nu_u)) / prob.rho
    return sp.bmat([[Buu, Buv], [Bvu, Bvv]], format="csr")


PARAMS = ("alpha", "beta", "theta", "gamma")


def parameter_derivatives(u1, v1, u0, v0, dt, prob: Problem):
    """dF/dp for p in alpha, beta, theta, gamma as stacked vectors.  F_u depends on a
    parameter only through mu (inside the flux), F_v only through nu (eq. dvds-2):
      d mu/d alpha = -(u1 + u0 - 1)/2,  d nu/d beta = -(v1 + v0)/2,
      d mu/d theta = phi + psi,         d nu/d theta = phi - psi,
      d mu/d gamma = -(Lap u1 + Lap u0)/2, d nu/d gamma = -(Lap v1 + Lap v0)/2."""
    h = prob.spacing(u1.shape)
    c = scheme.operator_mobility(u1, v1, u0, v0, prob)
    phi = scheme.g2_series(u1 + v1, u0 + v0, prob.S)
    psi = scheme.g2_series(u1 - v1, u0 - v0, prob.S)
    lap = lambda a: scheme.laplacian(a, h, prob.bc)
    zero = np.zeros_like(u1)
    out = {}
    for name, dmu, dnu in [("alpha", -0.5 * (u1 + u0 - 1.0), zero),
                           ("beta", zero, -0.5 * (v1 + v0)),
                           ("theta", phi + psi, phi - psi),
                           ("gamma", -0.5 * (lap(u1) + lap(u0)), -0.5 * (lap(v1) + lap(v0)))]:
        Fu = -scheme.div_c_grad(c, dmu, h, prob.bc)
        Fv = c * dnu / prob.rho
        out[name] = np.concatenate([Fu.ravel(), Fv.ravel()])
    return out


def energy_gradient(u, v, prob: Problem):
    """dE~/du, dE~/dv (fields) and dE~/dp of eqs. relations/freeenergy: the cell volume
    times alpha/2 (1-2u) + theta(Phi'(u+v) + Phi'(u-v)) - gamma Lap u, and
    -beta v + theta(Phi'(u+v) - Phi'(u-v)) - gamma Lap v; each parameter's own terms
    divided by it for dE~/dp."""
    h = prob.spacing(u.shape)
    vol = scheme.cell_volume(u.shape, prob)
    dPhi = lambda z: np.log(z) - np.log(1.0 - z)
    lap = lambda a: scheme.laplacian(a, h, prob.bc)
    gu = vol * (0.5 * prob.alpha * (1 - 2 * u) + prob.theta * (dPhi(u + v) + dPhi(u - v)) - prob.gamma * lap(u))
    gv = vol * (-prob.beta * v + prob.theta * (dPhi(u + v) - dPhi(u - v)) - prob.gamma * lap(v))
    gp = {"alpha": vol * 0.5 * float(np.sum(u * (1.0 - u))),
          "beta": -vol * 0.5 * float(np.sum(v * v)),
          "theta": vol * float(np.sum(scheme.Phi(u + v) + scheme.Phi(u - v))),
          "gamma": vol * 0.5 * float(np.sum(scheme.gradient_energy_density(u, h, prob.bc)
                                            + scheme.gradient_energy_density(v, h, prob.bc)))}
    return gu, gv, gp


def forward(u0, v0, dts, prob: Problem, opts: NewtonOptions):
    """States U^0..U^N of the run with the given dt sequence."""
    states = [(u0.copy(), v0.copy())]
    n = u0.size
    for dt in dts:
        u, v = states[-1]
        res = solve_step(u, v, dt, prob, opts)
        if not res.converged:
            raise RuntimeError(f"oracle forward step failed: {res.reason}")
        states.append((res.X[:n].reshape(u.shape).copy(), res.X[n:].reshape(u.shape).copy()))
    return states


def adjoint_step(u1, v1, u0, v0, dt, prob: Problem, g1):
    """One step back: solve A^T lambda = g1, return (g0, lambda, {p: -lambda . dF/dp})."""
    A = jacobian.jacobian(u1, v1, u0, v0, dt, prob)
    lam = spla.spsolve(A.T.tocsc(), g1)
    pd = parameter_derivatives(u1, v1, u0, v0, dt, prob)
    dp = {k: -float(lam @ pd[k]) for k in PARAMS}
    B = previous_state_jacobian(u1, v1, u0, v0, dt, prob)
    return -(B.T @ lam), lam, dp


def gradient(u0, v0, dts, prob: Problem, opts: NewtonOptions = None, states=None):
    """E~(U^N) and its gradient with respect to u0, v0 and the parameters (dict), the
    dt sequence held fixed.  `states` may hold U^0..U^N of an earlier forward run."""
    opts = opts or NewtonOptions(rtol=1e-12, atol=1e-11)
    if states is None:
        states = forward(u0, v0, dts, prob, opts)
    uN, vN = states[-1]
    E = scheme.energy(uN, vN, prob)
    gu, gv, gp = energy_gradient(uN, vN, prob)
    g = np.concatenate([gu.ravel(), gv.ravel()])
    for k in range(len(dts) - 1, -1, -1):
        (ua, va), (ub, vb) = states[k], states[k + 1]
        g, _, dp = adjoint_step(ub, vb, ua, va, dts[k], prob, g)
        for name in PARAMS:
            gp[name] += dp[name]
    n = u0.size
    return E, g[:n].reshape(u0.shape), g[n:].reshape(u0.shape), gp
