"""Adaptive time stepping of Section 3.2 and the time-stepping driver of the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Prediction (eq. sencondt): dt~_n = max(dt_min, dt_max / sqrt(1 + eta X'_d(t_n)^2)),
X'_d = ||X^n - X^{n-1}|| / dt_{n-1}, and dt_0 = dt_min.  If the nonlinear solve
diverges, dt~_n := dt~_n / sqrt(2) and the solve restarts; eta doubles on every
divergence (the modification proposed at the end of Section 3.2).

Readings where the paper is silent: the norm is the plain Euclidean norm over
all unknowns (an h^d-weighted norm is selectable); retries are floored at
dt_min and a divergence at dt_min is reported as a failure with the state left
at the last accepted step; the retry uses dt~/sqrt(2) (eta's new value only
affects later predictions); eta never decreases.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .params import Problem
from . import scheme
from .newton import NewtonOptions, solve_step


def predict_dt(first: bool, diff_norm: float, dt_prev: float, eta: float,
               dt_min: float, dt_max: float) -> float:
    """eq. sencondt; the first step uses dt_min."""
    if first:
        return dt_min
    xd = diff_norm / dt_prev
    return max(dt_min, dt_max / math.sqrt(1.0 + eta * xd * xd))


def retry_dt(dt: float, dt_min: float) -> float:
    """The divergence retry dt~ / sqrt(2), floored at dt_min."""
    return max(dt / math.sqrt(2.0), dt_min)


def diff_norm(X, Xprev, shape, prob: Problem, weighted: bool = False) -> float:
    d = float(np.linalg.norm(X - Xprev))
    if weighted:
        d *= math.sqrt(scheme.cell_volume(shape, prob))
    return d


@dataclass
class StepRecord:
    t: float
    dt: float
    eta: float
    newton_its: int          # Newton iterations of all attempts of this step
    retries: int
    energy: float
    mass: float


class DivergedError(RuntimeError):
    pass


@dataclass
class Run:
    """The oracle's time-stepping state (U^n, U^{n-1}, dt_{n-1}, eta, t)."""
    prob: Problem
    u: np.ndarray
    v: np.ndarray
    adaptive: bool = True
    dt_fixed: float = 1e-3
    dt_min: float = 1e-4
    dt_max: float = 1e-1
    eta: float = 1e4
    newton: NewtonOptions = field(default_factory=NewtonOptions)
    weighted_norm: bool = False
    t: float = 0.0
    X_prev: Optional[np.ndarray] = None
    dt_prev: float = 0.0
    history: List[StepRecord] = field(default_factory=list)

    @property
    def X(self):
        return np.concatenate([self.u.ravel(), self.v.ravel()])

    def step(self, dt_override: Optional[float] = None) -> StepRecord:
        shape = self.u.shape
        n = self.u.size
        if dt_override is not None:
            dt = dt_override
        elif not self.adaptive:
            dt = self.dt_fixed
        else:
            first = self.X_prev is None
            dn = 0.0 if first else diff_norm(self.X, self.X_prev, shape, self.prob, self.weighted_norm)
            dt = predict_dt(first, dn, self.dt_prev, self.eta, self.dt_min, self.dt_max)
        its = 0
        retries = 0
        while True:
            res = solve_step(self.u, self.v, dt, self.prob, self.newton)
            its += res.iterations
            if res.converged:
                break
            if not self.adaptive or dt_override is not None:
                raise DivergedError(f"Newton failed at fixed dt={dt}: {res.reason}")
            self.eta *= 2.0
            if dt <= self.dt_min:
                raise DivergedError(f"Newton failed at dt_min={dt}: {res.reason}")
            dt = retry_dt(dt, self.dt_min)
            retries += 1
        X_old = self.X
        self.u = res.X[:n].reshape(shape).copy()
        self.v = res.X[n:].reshape(shape).copy()
        self.X_prev = X_old
        self.dt_prev = dt
        self.t += dt
        rec = StepRecord(self.t, dt, self.eta, its, retries,
                         scheme.energy(self.u, self.v, self.prob), scheme.mass(self.u, self.prob))
        self.history.append(rec)
        return rec
