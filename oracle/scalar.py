"""Cell-by-cell residual of scheme (2.20) written with explicit loops (pure Python floats).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

An independent second coding of the residual: no NumPy vector operations, no
ghost padding; each face of a cell is visited explicitly, and a Neumann boundary
face simply carries no flux (the ghost rule phi_0 = phi_1 of Section 2 makes
every boundary difference vanish).  Used on tiny grids (P6-style agreement with
the vectorised residual and a dense Newton solve) and on sampled cells of full
size grids.
"""
from __future__ import annotations

import math
from typing import Iterator, Optional, Sequence, Tuple

from .params import Problem


def _neighbours(cell: Tuple[int, ...], shape, bc: str) -> Iterator[Tuple[int, Optional[Tuple[int, ...]]]]:
    """Yield (axis, neighbour index or None) for the 2*d faces of ``cell``."""
    for a in range(len(shape)):
        for step in (-1, 1):
            j = cell[a] + step
            if 0 <= j < shape[a]:
                nb = list(cell)
                nb[a] = j
                yield a, tuple(nb)
            elif bc == "periodic":
                nb = list(cell)
                nb[a] = j % shape[a]
                yield a, tuple(nb)
            else:
                yield a, None


def _fS(x: float, s: float, S: int) -> float:
    r = s / x
    acc = 0.0
    for m in range(1, S + 1):
        acc += r ** (2 * m) / ((2 * m + 1) * (2 * m))
    return math.log(x) - acc


def _phiS(a1: float, a0: float, S: int) -> float:
    zeta = 0.5 * (a1 + a0)
    s = 0.5 * (a1 - a0)
    return _fS(zeta, s, S) - _fS(1.0 - zeta, s, S)


def _lap(f, cell, shape, h, bc) -> float:
    acc = 0.0
    for a, nb in _neighbours(cell, shape, bc):
        if nb is not None:
            acc += (f[nb] - f[cell]) / (h[a] * h[a])
    return acc


def _c(u1, v1, u0, v0, cell, prob: Problem) -> float:
    if prob.mobility == "midpoint":
        ub = 0.5 * (u1[cell] + u0[cell])
        vb = 0.5 * (v1[cell] + v0[cell])
        return ub * (1.0 - ub) * (0.25 - vb * vb)
    c1 = u1[cell] * (1.0 - u1[cell]) * (0.25 - v1[cell] ** 2)
    c0 = u0[cell] * (1.0 - u0[cell]) * (0.25 - v0[cell] ** 2)
    if prob.mobility == "average":
        return 0.5 * (c1 + c0)
    return c0


def _mu_nu(u1, v1, u0, v0, cell, shape, h, prob: Problem):
    phi = _phiS(u1[cell] + v1[cell], u0[cell] + v0[cell], prob.S)
    psi = _phiS(u1[cell] - v1[cell], u0[cell] - v0[cell], prob.S)
    mu = (-prob.alpha / 2 * (u1[cell] + u0[cell] - 1.0) + prob.theta * (phi + psi)
          - prob.gamma / 2 * (_lap(u1, cell, shape, h, prob.bc) + _lap(u0, cell, shape, h, prob.bc)))
    nu = (-prob.beta / 2 * (v1[cell] + v0[cell]) + prob.theta * (phi - psi)
          - prob.gamma / 2 * (_lap(v1, cell, shape, h, prob.bc) + _lap(v0, cell, shape, h, prob.bc)))
    return mu, nu


def residual_at(u1, v1, u0, v0, dt: float, prob: Problem, cell: Sequence[int]):
    """(F_u, F_v) of scheme (2.20) at one cell, from local reads only."""
    cell = tuple(int(c) for c in cell)
    shape = u1.shape
    h = prob.spacing(shape)
    mu_k, nu_k = _mu_nu(u1, v1, u0, v0, cell, shape, h, prob)
    c_k = _c(u1, v1, u0, v0, cell, prob)
    div = 0.0
    for a, nb in _neighbours(cell, shape, prob.bc):
        if nb is None:
            continue  # zero flux through a Neumann boundary face
        mu_n, _ = _mu_nu(u1, v1, u0, v0, nb, shape, h, prob)
        c_face = 0.5 * (c_k + _c(u1, v1, u0, v0, nb, prob))
        div += c_face * (mu_n - mu_k) / (h[a] * h[a])
    Fu = (u1[cell] - u0[cell]) / dt - div
    Fv = (v1[cell] - v0[cell]) / dt + c_k * nu_k / prob.rho
    return Fu, Fv


def residual_loops(u1, v1, u0, v0, dt: float, prob: Problem):
    """Residual on the whole grid by visiting every cell (tiny grids only)."""
    import numpy as np
    Fu = np.empty_like(u1)
    Fv = np.empty_like(v1)
    for cell in np.ndindex(*u1.shape):
        Fu[cell], Fv[cell] = residual_at(u1, v1, u0, v0, dt, prob, cell)
    return Fu, Fv
