"""Newton solve of one time step of scheme (2.20) with a sparse direct linear solve.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3.1: X_{m+1} = X_m + lambda_m S_m with X_0 = U^n, J_m S_m = -F(X_m),
stopping when ||F(X_{m+1})|| <= max(eps_r ||F(X_0)||, eps_a).  The oracle's linear
solve is exact (SuperLU), so the result is the root of F(.; U^n, dt) that the
Krylov–Schwarz path must reproduce up to its tolerances.

The paper names a line search from Dennis & Schnabel without details.  The
reading used on both sides: backtracking on f = ||F||^2/2 with the Armijo test
f(lambda) <= f(0) - 2 alpha lambda f(0) (alpha = 1e-4, slope of the Newton
direction), a quadratic model on the first backtrack and a cubic model after,
each new lambda clamped to [0.1, 0.5] times the previous one; a trial outside
the admissible set (p or q = u -+ v not in (0,1)) or with a non-finite residual
halves lambda; failure below lambda = 1e-8.

"NKS diverges" (Section 3.2) reads: the iteration limit is exceeded, the line
search fails, or the residual becomes non-finite.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse.linalg as spla

from .params import Problem
from . import scheme, jacobian


@dataclass
class NewtonOptions:
    rtol: float = 1e-8          # eps_r
    atol: float = 1e-13         # eps_a
    max_it: int = 50
    ls_alpha: float = 1e-4
    ls_min_lambda: float = 1e-8


@dataclass
class NewtonResult:
    converged: bool
    X: np.ndarray
    iterations: int
    fnorms: List[float] = field(default_factory=list)
    lambdas: List[float] = field(default_factory=list)
    reason: str = ""


def _admissible_vec(X, n):
    u = X[:n]
    v = X[n:]
    return scheme.admissible(u, v)


def line_search(residual_fn, X, S, F, n, opts: NewtonOptions):
    """Backtracking line search along S from X (the reading stated in the module doc).

    Returns (lambda, X_new, F_new) or None on failure."""
    f0 = 0.5 * float(F @ F)
    slope = -2.0 * f0
    lam = 1.0
    prev = None  # (lambda, f) of the last admissible trial that failed the test
    while lam >= opts.ls_min_lambda:
        Xt = X + lam * S
        if not _admissible_vec(Xt, n):
            lam *= 0.5
            continue
        Ft = residual_fn(Xt)
        if not np.all(np.isfinite(Ft)):
            lam *= 0.5
            continue
        ft = 0.5 * float(Ft @ Ft)
        if ft <= f0 + opts.ls_alpha * lam * slope:
            return lam, Xt, Ft
        if prev is None:
            new = -slope * lam * lam / (2.0 * (ft - f0 - slope * lam))
        else:
            lp, fp = prev
            t1 = ft - f0 - slope * lam
            t2 = fp - f0 - slope * lp
            a = (t1 / (lam * lam) - t2 / (lp * lp)) / (lam - lp)
            b = (-lp * t1 / (lam * lam) + lam * t2 / (lp * lp)) / (lam - lp)
            if a == 0.0:
                new = -slope / (2.0 * b)
            else:
                disc = b * b - 3.0 * a * slope
                new = (-b + math.sqrt(disc)) / (3.0 * a) if disc >= 0.0 else 0.5 * lam
        if not math.isfinite(new):
            new = 0.5 * lam
        new = min(max(new, 0.1 * lam), 0.5 * lam)
        prev = (lam, ft)
        lam = new
    return None


def solve_step(u0, v0, dt: float, prob: Problem, opts: Optional[NewtonOptions] = None,
               X_init=None, forcing=None) -> NewtonResult:
    """Solve F(U1; U0, dt) = 0 of scheme (2.20) from X_0 = U^n (or ``X_init``).

    ``forcing`` (a stacked [f_u, f_v] vector, default none) is subtracted from the
    residual: the manufactured-solution test solves F(U1; U0, dt) = f with the
    forcing of a chosen exact solution.  It does not depend on U1, so the Jacobian
    is unchanged."""
    opts = opts or NewtonOptions()
    shape = u0.shape
    n = int(np.prod(shape))
    U0 = np.concatenate([u0.ravel(), v0.ravel()])
    X = U0.copy() if X_init is None else np.array(X_init, dtype=np.float64)
    if forcing is None:
        rfun = lambda Y: scheme.residual_vec(Y, U0, dt, prob, shape)
    else:
        fvec = np.asarray(forcing, dtype=np.float64)
        rfun = lambda Y: scheme.residual_vec(Y, U0, dt, prob, shape) - fvec
    F = rfun(X)
    f_init = float(np.linalg.norm(F))
    res = NewtonResult(False, X, 0, [f_init], [])
    if not math.isfinite(f_init):
        res.reason = "nonfinite"
        return res
    tol = max(opts.rtol * f_init, opts.atol)
    if f_init <= tol:
        res.converged = True
        return res
    for it in range(1, opts.max_it + 1):
        J = jacobian.jacobian(X[:n].reshape(shape), X[n:].reshape(shape), u0, v0, dt, prob)
        lu = spla.splu(J.tocsc(), permc_spec="MMD_AT_PLUS_A")
        S = lu.solve(-F)
        ls = line_search(rfun, X, S, F, n, opts)
        if ls is None:
            res.reason = "line_search"
            res.iterations = it
            return res
        lam, X, F = ls
        fn = float(np.linalg.norm(F))
        res.X = X
        res.iterations = it
        res.fnorms.append(fn)
        res.lambdas.append(lam)
        if not math.isfinite(fn):
            res.reason = "nonfinite"
            return res
        if fn <= tol:
            res.converged = True
            return res
    res.reason = "max_it"
    return res
