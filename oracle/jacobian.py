"""Analytic Jacobian of the residual of scheme (2.20), as a SciPy sparse matrix (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The residual is F_u = (u1-u0)/dt - sum_a D_a[ c~_a (G_a mu) ] / h_a^2 and
F_v = (v1-v0)/dt + c nu / rho (Section 2, eq. NSOA-1).  Writing G_a for the face
difference, A_a for the face average and D_a for the face divergence along axis
a (all with the ghost rule of Section 2), the product rule gives

  J_uu = I/dt - sum_a D_a [ diag(G_a mu) A_a diag(c_u) + diag(A_a c) G_a (diag(mu_u) - gamma/2 L) ] / h_a^2
  J_uv =      - sum_a D_a [ diag(G_a mu) A_a diag(c_v) + diag(A_a c) G_a diag(mu_v) ] / h_a^2
  J_vv = I/dt + [ diag(nu c_v) + diag(c) (diag(nu_v) - gamma/2 L) ] / rho
  J_vu = diag(nu c_u + c nu_u) / rho

where L is the discrete Laplacian and mu_u, mu_v, nu_u, nu_v, c_u, c_v are the
pointwise partial derivatives with respect to the unknown state.  The Jacobian
is the matrix J_m of eq. hjacobi (Section 3.1).

Pin: central finite differences of oracle.scheme.residual (tests).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .params import Problem
from . import scheme


def _kron_axis(op1d, shape, axis):
    before = int(np.prod(shape[:axis])) if axis > 0 else 1
    after = int(np.prod(shape[axis + 1:])) if axis + 1 < len(shape) else 1
    return sp.kron(sp.identity(before, format="csr"),
                   sp.kron(op1d, sp.identity(after, format="csr"), format="csr"), format="csr")


def _face_diff_1d(n, bc):
    rows, cols, vals = [], [], []
    for f in range(n + 1):          # face f sits between cells f-1 and f
        left, right = f - 1, f
        if bc == "periodic":
            left %= n
            right %= n
        elif left < 0 or right >= n:
            continue                # Neumann boundary face: zero difference
        rows += [f, f]
        cols += [right, left]
        vals += [1.0, -1.0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, n))


def _face_avg_1d(n, bc):
    rows, cols, vals = [], [], []
    for f in range(n + 1):
        left, right = f - 1, f
        if bc == "periodic":
            left %= n
            right %= n
        else:
            left = min(max(left, 0), n - 1)
            right = min(max(right, 0), n - 1)
        rows += [f, f]
        cols += [left, right]
        vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, n))


def _face_div_1d(n):
    rows, cols, vals = [], [], []
    for i in range(n):
        rows += [i, i]
        cols += [i + 1, i]
        vals += [1.0, -1.0]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n + 1))


def operators(shape, prob: Problem):
    """Per-axis (G_a, A_a, D_a) on the flattened grid, plus the Laplacian L."""
    h = prob.spacing(shape)
    ops = []
    ncell = int(np.prod(shape))
    L = sp.csr_matrix((ncell, ncell))
    for a, n in enumerate(shape):
        fshape = list(shape)
        fshape[a] = n + 1
        G = _kron_axis(_face_diff_1d(n, prob.bc), shape, a)
        A = _kron_axis(_face_avg_1d(n, prob.bc), shape, a)
        # divergence maps faces (fshape) to cells; build it on the face grid
        D = _kron_axis(_face_div_1d(n), fshape, a)
        D = _restrict_rows_for_div(D, shape, fshape, a)
        ops.append((G, A, D, h[a]))
        L = L + (D @ G) / (h[a] * h[a])
    return ops, L.tocsr()


def _restrict_rows_for_div(D, shape, fshape, axis):
    """kron over the face grid gives an operator whose row space is indexed like
    the face grid with n along ``axis`` replaced by n (rows) — i.e. the cell grid.
    The construction above already has exactly prod(shape) rows; this checks it."""
    assert D.shape == (int(np.prod(shape)), int(np.prod(fshape)))
    return D


def g2_series_d1(x1, x0, S: int):
    """d/dx1 of g2_series: 1/2[f_x(z,s) + f_s(z,s) + f_x(1-z,s) - f_s(1-z,s)] with
    f_x = (1/x)(1 + sum r^{2m}/(2m+1)) and f_s = -(1/x) sum r^{2m-1}/(2m+1), r = s/x
    (term-by-term derivatives of the series of Lemma 2.2)."""
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
    return 0.5 * (fx1 + fs1 + fx2 - fs2)


def pointwise_derivatives(u1, v1, u0, v0, prob: Problem):
    """c, c_u, c_v and the pointwise parts mu_u, mu_v (= nu_u), nu_v of the
    derivative of G~^S with respect to (u1, v1)."""
    if prob.mobility == "midpoint":
        ub = 0.5 * (u1 + u0)
        vb = 0.5 * (v1 + v0)
        c = ub * (1 - ub) * (0.25 - vb * vb)
        cu = 0.5 * (1 - 2 * ub) * (0.25 - vb * vb)
        cv = -ub * (1 - ub) * vb
    elif prob.mobility == "average":
        c = 0.5 * (scheme.mobility(u1, v1) + scheme.mobility(u0, v0))
        cu = 0.5 * (1 - 2 * u1) * (0.25 - v1 * v1)
        cv = -u1 * (1 - u1) * v1
    elif prob.mobility == "explicit":
        c = scheme.mobility(u0, v0)
        cu = np.zeros_like(u1)
        cv = np.zeros_like(u1)
    else:
        raise ValueError(prob.mobility)
    dphi = g2_series_d1(u1 + v1, u0 + v0, prob.S)
    dpsi = g2_series_d1(u1 - v1, u0 - v0, prob.S)
    mu_u = -0.5 * prob.alpha + prob.theta * (dphi + dpsi)
    mu_v = prob.theta * (dphi - dpsi)
    nu_u = prob.theta * (dphi - dpsi)
    nu_v = -0.5 * prob.beta + prob.theta * (dphi + dpsi)
    return c, cu, cv, mu_u, mu_v, nu_u, nu_v


def jacobian(u1, v1, u0, v0, dt: float, prob: Problem):
    """dF/d(u1, v1) as a (2n x 2n) CSR matrix in the stacked order [u; v]."""
    shape = u1.shape
    n = int(np.prod(shape))
    ops, L = operators(shape, prob)
    mu, nu = scheme.discrete_variational_derivative(u1, v1, u0, v0, prob)
    c, cu, cv, mu_u, mu_v, nu_u, nu_v = pointwise_derivatives(u1, v1, u0, v0, prob)
    f = lambda a: a.ravel()
    dg = sp.diags
    I = sp.identity(n, format="csr")
    Juu = I / dt
    Juv = sp.csr_matrix((n, n))
    for G, A, D, ha in ops:
        gmu = G @ f(mu)
        ct = A @ f(c)
        Juu = Juu - D @ (dg(gmu) @ A @ dg(f(cu)) + dg(ct) @ G @ (dg(f(mu_u)) - 0.5 * prob.gamma * L)) / (ha * ha)
        Juv = Juv - D @ (dg(gmu) @ A @ dg(f(cv)) + dg(ct) @ G @ dg(f(mu_v))) / (ha * ha)
    Jvv = I / dt + (dg(f(nu * cv)) + dg(f(c)) @ (dg(f(nu_v)) - 0.5 * prob.gamma * L)) / prob.rho
    Jvu = dg(f(nu * cu + c * nu_u)) / prob.rho
    J = sp.bmat([[Juu, Juv], [Jvu, Jvv]], format="csr")
    J.sum_duplicates()
    return J


def jacobian_fd(u1, v1, u0, v0, dt, prob: Problem, eps=1e-7):
    """Dense central-difference Jacobian (tiny grids only; the P5 pin)."""
    shape = u1.shape
    n = int(np.prod(shape))
    X = np.concatenate([u1.ravel(), v1.ravel()])
    U0 = np.concatenate([u0.ravel(), v0.ravel()])
    J = np.zeros((2 * n, 2 * n))
    for k in range(2 * n):
        e = np.zeros(2 * n)
        step = eps * max(1.0, abs(X[k]))
        e[k] = step
        Fp = scheme.residual_vec(X + e, U0, dt, prob, shape)
        Fm = scheme.residual_vec(X - e, U0, dt, prob, shape)
        J[:, k] = (Fp - Fm) / (2 * step)
    return J
