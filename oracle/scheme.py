"""Discrete operators, energy and the residual of scheme (2.20) — vectorised NumPy, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Notation follows Section 2 of the paper.  Fields are arrays of shape (ny, nx)
(2D) or (nz, ny, nx) (3D); the cell (i, j[, k]) has centre ((i-1/2)dx, ...).
u1, v1 denote the unknown state at t_{n+1}; u0, v0 the state at t_n.

Pins (tests/test_oracle_*.py):
  f_series / g2_series : against the exact divided difference of Phi in 50-digit
                         arithmetic within the truncation bound of Lemma 2.2;
  laplacian, energy    : summation by parts (eq. summation), the DVD identities
                         for G1 and G3 (eq. DVD), closed forms on constant states
                         and single Fourier modes;
  residual             : F = 0 on constant states, the linearised single-mode
                         growth factor (a Crank–Nicolson symbol), mass
                         conservation, v = 0 invariance, Neumann(N) ==
                         periodic(2N) on mirrored data, 2D == 1D / 3D == 2D
                         reductions, and agreement with the independent loop
                         residual of oracle/scalar.py;
  the whole scheme     : second-order self-convergence in h and dt (Section 4.1 A).
"""
from __future__ import annotations

import numpy as np

from .params import Problem

# ---------------------------------------------------------------------------
# Free energy pieces (Section 1, eq. eq:2 and the split neq:01)
# ---------------------------------------------------------------------------


def Phi(z):
    """Phi(z) = z ln z + (1 - z) ln(1 - z), the ideal-mixing entropy (Section 1)."""
    z = np.asarray(z)
    return z * np.log(z) + (1.0 - z) * np.log(1.0 - z)


def mobility(u, v):
    """c(u, v) = u(1 - u)(1/4 - v^2), degenerate at pure phases (Section 1)."""
    return u * (1.0 - u) * (0.25 - v * v)


def local_energy_bulk(u, v, prob: Problem):
    """e1 + e2 of eq. neq:01: alpha/2 u(1-u) - beta/2 v^2 + theta(Phi(u+v)+Phi(u-v))."""
    return (0.5 * prob.alpha * u * (1.0 - u) - 0.5 * prob.beta * v * v
            + prob.theta * (Phi(u + v) + Phi(u - v)))


# ---------------------------------------------------------------------------
# The truncated divided difference (Lemma 2.2, eq. taylor / D2-1)
# ---------------------------------------------------------------------------


def f_series(x, sigma, S: int):
    """f_S(x, sigma) = ln x - sum_{m=1}^{S} (sigma/x)^{2m} / ((2m+1) 2m)  (eq. taylor).

    The exact f(x, sigma) = [(x+s)ln(x+s) - (x-s)ln(x-s)]/(2s) equals
    ln x + 1 - sum_m ...; the constant 1 is left out exactly as printed, because
    it cancels in the difference used by g2_series."""
    x = np.asarray(x)
    r2 = (np.asarray(sigma) / x) ** 2
    total = np.zeros_like(r2)
    power = np.ones_like(r2)
    for m in range(1, S + 1):
        power = power * r2
        total = total + power / ((2 * m + 1) * (2 * m))
    return np.log(x) - total


def g2_series(x1, x0, S: int):
    """One component phi^S (or psi^S) of G2^S for the variable p = u+v (or q = u-v).

    zeta = (x1+x0)/2, sigma = (x1-x0)/2 and phi^S = f_S(zeta, sigma) - f_S(1-zeta, sigma).
    The paper prints "+ f_S(1-zeta, -sigma)"; since f is even in sigma that sum
    would tend to ln zeta + ln(1-zeta) instead of Phi'(zeta) = ln zeta - ln(1-zeta),
    so the minus sign is taken (the approximation of the divided difference
    [Phi(x1)-Phi(x0)]/(x1-x0) of eq. D2)."""
    zeta = 0.5 * (x1 + x0)
    sigma = 0.5 * (x1 - x0)
    return f_series(zeta, sigma, S) - f_series(1.0 - zeta, sigma, S)


def g2_exact(x1, x0):
    """The exact divided difference [Phi(x1) - Phi(x0)] / (x1 - x0) of eq. D2
    (numerically unstable when x1 ~ x0, Section 2; used only where it is well
    conditioned or in extended precision)."""
    return (Phi(x1) - Phi(x0)) / (x1 - x0)


# ---------------------------------------------------------------------------
# Difference operators on the cell-centred grid (Section 2)
# ---------------------------------------------------------------------------


def _pad_mode(bc: str) -> str:
    # periodic: indices wrap; Neumann: ghost values copy the boundary cell
    # (phi_0 = phi_1, phi_{N+1} = phi_N, the discrete boundary rule of Section 2).
    if bc == "periodic":
        return "wrap"
    if bc == "neumann":
        return "edge"
    raise ValueError(f"unknown boundary condition {bc!r}")


def face_diff(phi, axis: int, bc: str):
    """Differences phi_i - phi_{i-1} on the n+1 faces i-1/2 (i = 0..n) along ``axis``,
    using the ghost rule; for Neumann the two boundary faces carry zero."""
    pad = [(0, 0)] * phi.ndim
    pad[axis] = (1, 1)
    return np.diff(np.pad(phi, pad, mode=_pad_mode(bc)), axis=axis)


def face_avg(phi, axis: int, bc: str):
    """(phi_{i-1} + phi_i)/2 on the n+1 faces along ``axis`` (the face mobility
    c~_{i+1/2} = (c_i + c_{i+1})/2 of Section 2)."""
    pad = [(0, 0)] * phi.ndim
    pad[axis] = (1, 1)
    p = np.pad(phi, pad, mode=_pad_mode(bc))
    lo = [slice(None)] * phi.ndim
    hi = [slice(None)] * phi.ndim
    lo[axis] = slice(0, -1)
    hi[axis] = slice(1, None)
    return 0.5 * (p[tuple(lo)] + p[tuple(hi)])


def _face_divergence(flux, axis: int):
    lo = [slice(None)] * flux.ndim
    hi = [slice(None)] * flux.ndim
    lo[axis] = slice(0, -1)
    hi[axis] = slice(1, None)
    return flux[tuple(hi)] - flux[tuple(lo)]


def laplacian(phi, h, bc: str):
    """Delta_h phi = sum over axes of D_a D_a phi (the 5-point / 7-point Laplacian)."""
    out = np.zeros_like(phi)
    for a in range(phi.ndim):
        out += _face_divergence(face_diff(phi, a, bc), a) / (h[a] * h[a])
    return out


def div_c_grad(c, phi, h, bc: str):
    """[nabla . c nabla phi]_h = sum_a D_a c~ D_a phi with face mobility the average
    of the two adjacent cell values (Section 2)."""
    out = np.zeros_like(phi)
    for a in range(phi.ndim):
        flux = face_avg(c, a, bc) * face_diff(phi, a, bc)
        out += _face_divergence(flux, a) / (h[a] * h[a])
    return out


# ---------------------------------------------------------------------------
# Scheme (2.20)
# ---------------------------------------------------------------------------


def operator_mobility(u1, v1, u0, v0, prob: Problem):
    """The cell mobility used inside the operator A~ of scheme (2.20).

    The paper writes c at level n but builds the scheme by the trapezoidal rule
    at the half-time level and claims second order in time; the reading taken
    here is the midpoint state c((u1+u0)/2, (v1+v0)/2).  The two alternatives are
    kept selectable for the time-order test."""
    if prob.mobility == "midpoint":
        return mobility(0.5 * (u1 + u0), 0.5 * (v1 + v0))
    if prob.mobility == "average":
        return 0.5 * (mobility(u1, v1) + mobility(u0, v0))
    if prob.mobility == "explicit":
        return mobility(u0, v0)
    raise ValueError(prob.mobility)


def discrete_variational_derivative(u1, v1, u0, v0, prob: Problem):
    """G~^S = G1 + G2^S + G3 (eqs. dvds-2, D2-1, dvds-1); returns (mu, nu).

    G1 = (-alpha/2 (u1+u0-1), -beta/2 (v1+v0))
    G2^S = (theta(phi^S + psi^S), theta(phi^S - psi^S)) with p = u+v, q = u-v
    G3 = (-gamma/2 (Delta u1 + Delta u0), -gamma/2 (Delta v1 + Delta v0))."""
    h = prob.spacing(u1.shape)
    phi = g2_series(u1 + v1, u0 + v0, prob.S)
    psi = g2_series(u1 - v1, u0 - v0, prob.S)
    mu = (-0.5 * prob.alpha * (u1 + u0 - 1.0) + prob.theta * (phi + psi)
          - 0.5 * prob.gamma * (laplacian(u1, h, prob.bc) + laplacian(u0, h, prob.bc)))
    nu = (-0.5 * prob.beta * (v1 + v0) + prob.theta * (phi - psi)
          - 0.5 * prob.gamma * (laplacian(v1, h, prob.bc) + laplacian(v0, h, prob.bc)))
    return mu, nu


def residual(u1, v1, u0, v0, dt: float, prob: Problem):
    """F(U1; U0, dt) of scheme (2.20): (U1 - U0)/dt + A~ G~^S = 0, i.e.

    F_u = (u1 - u0)/dt - [nabla . c nabla mu]_h
    F_v = (v1 - v0)/dt + c nu / rho.
    Returns (F_u, F_v) with the field shape."""
    h = prob.spacing(u1.shape)
    mu, nu = discrete_variational_derivative(u1, v1, u0, v0, prob)
    c = operator_mobility(u1, v1, u0, v0, prob)
    Fu = (u1 - u0) / dt - div_c_grad(c, mu, h, prob.bc)
    Fv = (v1 - v0) / dt + c * nu / prob.rho
    return Fu, Fv


def residual_vec(X, U0, dt, prob: Problem, shape):
    """Residual on the stacked vector X = [u.ravel(), v.ravel()]."""
    n = int(np.prod(shape))
    u1 = X[:n].reshape(shape)
    v1 = X[n:].reshape(shape)
    Fu, Fv = residual(u1, v1, U0[:n].reshape(shape), U0[n:].reshape(shape), dt, prob)
    return np.concatenate([Fu.ravel(), Fv.ravel()])


# ---------------------------------------------------------------------------
# Discrete energy and mass (eqs. relations, freeenergy)
# ---------------------------------------------------------------------------


def gradient_energy_density(phi, h, bc: str):
    """sum over axes of [(D^± phi)^2] = ((D^+ phi)^2 + (D^- phi)^2)/2 at each cell."""
    out = np.zeros_like(phi)
    for a in range(phi.ndim):
        fd = face_diff(phi, a, bc) / h[a]
        lo = [slice(None)] * phi.ndim
        hi = [slice(None)] * phi.ndim
        lo[a] = slice(0, -1)   # D^- at cell i is face i-1/2
        hi[a] = slice(1, None)  # D^+ at cell i is face i+1/2
        out += 0.5 * (fd[tuple(hi)] ** 2 + fd[tuple(lo)] ** 2)
    return out


def energy_density(u, v, prob: Problem):
    """[e~]_{ij} of eq. relations with the exact logarithmic Phi."""
    h = prob.spacing(u.shape)
    return (local_energy_bulk(u, v, prob)
            + 0.5 * prob.gamma * (gradient_energy_density(u, h, prob.bc)
                                  + gradient_energy_density(v, h, prob.bc)))


def cell_volume(shape, prob: Problem):
    return float(np.prod(prob.spacing(shape)))


def energy(u, v, prob: Problem) -> float:
    """E~ = <e~> = sum of e~ times the cell volume (eq. freeenergy)."""
    return float(np.sum(energy_density(u, v, prob)) * cell_volume(u.shape, prob))


def mass(u, prob: Problem) -> float:
    """M = sum of u times the cell volume (conserved by the flux form of F_u)."""
    return float(np.sum(u) * cell_volume(u.shape, prob))


def admissible(u, v) -> bool:
    """The admissible set of Section 2: u in (0,1), v in (-1/2,1/2), u +- v in (0,1)
    (the last two imply the first two)."""
    p = u + v
    q = u - v
    return bool(np.all(p > 0) and np.all(p < 1) and np.all(q > 0) and np.all(q < 1)
                and np.all(np.isfinite(u)) and np.all(np.isfinite(v)))
