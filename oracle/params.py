"""Problem parameters for the oracle (independent of the product's parameter struct)."""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Tuple


@dataclass(frozen=True)
class Problem:
    """Physical and discretisation parameters of system (1) on a box.

    Section 1: alpha, beta (pair interactions), theta (entropy), gamma (gradient
    energy), rho (density).  Section 4: the series order S (S=10 in the paper).
    ``bc`` is "periodic" or "neumann".  ``lengths`` are (Lx, Ly[, Lz]) and the grid
    shape follows the field arrays (x fastest, last axis).
    """
    alpha: float = 1.2
    beta: float = 1.2
    theta: float = 0.1
    gamma: float = 1e-3
    rho: float = 1.0
    S: int = 10
    bc: str = "periodic"
    lengths: Tuple[float, ...] = (1.0, 1.0)
    mobility: str = "midpoint"   # time level of c(u,v) inside the operator A

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)

    def spacing(self, shape):
        """Mesh sizes (h along axis 0, 1, ...) for a field of the given shape.

        Axis order follows the array: for a 2D (ny, nx) field this returns
        (hy, hx), where lengths are given as (Lx, Ly[, Lz])."""
        d = len(shape)
        L = tuple(self.lengths[:d]) if len(self.lengths) >= d else tuple(self.lengths) + (1.0,) * (d - len(self.lengths))
        # lengths are (Lx, Ly, Lz); array axes are (..., y, x)
        return tuple(L[d - 1 - a] / shape[a] for a in range(d))
