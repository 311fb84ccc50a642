"""Overlapping Schwarz preconditioners with subdomain ILU(0) — plain Python, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3.1: the domain is split into np non-overlapping boxes Omega_k, each
extended by delta cell layers to Omega_k^delta.  R_k^delta restricts a vector to
Omega_k^delta; A_k = R_k^delta J (R_k^delta)^T; inv(A_k) is approximated by an
incomplete LU factorisation.  Classical AS (eq. invM) sums (R_k^delta)^T inv(A_k)
R_k^delta; the left-restricted variant writes back only the owned part Omega_k,
the right-restricted variant restricts the input to the owned part.

Readings where the paper is silent (shared with the HIP path):
* split sizes: n cells into m parts of sizes floor(n/m) or floor(n/m)+1, the
  larger ones first; Neumann boxes are clipped at the domain boundary; periodic
  boxes wrap, and every periodic direction must have at least 2 parts with box
  length <= n-2 so no box touches itself across the wrap;
* unknown order inside Omega_k^delta: cells lexicographic with x fastest, and at
  each cell u before v (the interleaved X of Section 3.1);
* ILU(0) pattern: the structural stencil pattern of the Jacobian restricted to
  the box (u-row: u on the radius-2 diamond, v on the radius-1 star; v-row: v on
  the star and u at the cell), independent of numerically zero values.

Subdomain solvers (Table 2): ILU(0), ILU(k) on the level-of-fill pattern, and the
exact LU.  A second base pattern for ILU(0) and ILU(k), the "box" pattern: every
coupling between two box cells at most 2 apart along each axis, u and v both ways
(the nonzero structure a structured-grid sparse-matrix library allocates for a
stencil of width 2 that reaches the diagonal neighbours, explicit zeros included);
the paper does not state its ILU pattern, and this is the reading under which plain
ILU(0) converges as Table 2 reports.

Pins: textbook ILU(0) property (LU)_ij = A_ij on the pattern; ILU(0) equals the
exact LU when the pattern admits no fill; one subdomain with zero overlap and an
exact subdomain solve reproduces the global solve; ILU(k) levels equal the
fill-path characterisation (shortest path through lower-numbered vertices) and
(LU)_ij = A_ij on the level-k pattern; ILU(k) for k beyond the fill reaches the
exact LU (tests); on boxes at most 3 cells wide in x the box pattern holds all the
fill of the natural order, so its ILU(0) is the exact LU (tests).
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def split(n: int, parts: int) -> List[Tuple[int, int]]:
    """(start, length) of ``parts`` contiguous pieces of n cells."""
    base, rem = divmod(n, parts)
    out, s = [], 0
    for k in range(parts):
        ln = base + (1 if k < rem else 0)
        out.append((s, ln))
        s += ln
    return out


def stencil_offsets(dim: int, radius: int):
    """Offsets d with |d|_1 <= radius, in array-axis order (axis 0 slowest)."""
    rng = range(-radius, radius + 1)
    out = []
    for d in np.ndindex(*([2 * radius + 1] * dim)):
        off = tuple(int(x) - radius for x in d)
        if sum(abs(x) for x in off) <= radius:
            out.append(off)
    return out


def row_pattern(dim: int):
    """Structural Jacobian pattern: list of (row type, offset, column type), type 0 = u, 1 = v."""
    pat = []
    for off in stencil_offsets(dim, 2):
        pat.append((0, off, 0))
    for off in stencil_offsets(dim, 1):
        pat.append((0, off, 1))
    for off in stencil_offsets(dim, 1):
        pat.append((1, off, 1))
    pat.append((1, tuple([0] * dim), 0))
    return pat


@dataclass
class Subdomain:
    box_start: Tuple[int, ...]     # unwrapped start of Omega_k^delta (array-axis order)
    box_len: Tuple[int, ...]
    own_start: Tuple[int, ...]     # Omega_k, also unwrapped
    own_len: Tuple[int, ...]
    cells: List[Tuple[int, ...]]   # box coordinates of existing cells, lexicographic
    gcell: np.ndarray              # flat global cell index per entry of ``cells``
    owned: np.ndarray              # bool per entry of ``cells``

    def unknowns(self, ncell: int) -> np.ndarray:
        """Global indices (stacked [u; v] vector) in interleaved order u_c, v_c."""
        idx = np.empty(2 * len(self.cells), dtype=np.int64)
        idx[0::2] = self.gcell
        idx[1::2] = self.gcell + ncell
        return idx


def decompose(shape, parts, overlap: int, bc: str) -> List[Subdomain]:
    """Overlapping boxes Omega_k^delta of Section 3.1 (array-axis order for shape/parts)."""
    dim = len(shape)
    pieces = [split(shape[a], parts[a]) for a in range(dim)]
    if bc == "periodic":
        for a in range(dim):
            if parts[a] < 2:
                raise ValueError("periodic directions need at least 2 subdomains")
            longest = max(ln for _, ln in pieces[a]) + 2 * overlap
            if longest > shape[a] - 2:
                raise ValueError("overlapping box would touch itself across the periodic wrap")
    subs = []
    for combo in np.ndindex(*parts):
        own_start = tuple(pieces[a][combo[a]][0] for a in range(dim))
        own_len = tuple(pieces[a][combo[a]][1] for a in range(dim))
        box_start = tuple(s - overlap for s in own_start)
        box_len = tuple(l + 2 * overlap for l in own_len)
        cells, gcell, owned = [], [], []
        for b in np.ndindex(*box_len):
            g = [box_start[a] + b[a] for a in range(dim)]
            if bc == "periodic":
                g = [g[a] % shape[a] for a in range(dim)]
            elif any(g[a] < 0 or g[a] >= shape[a] for a in range(dim)):
                continue
            cells.append(tuple(b))
            gcell.append(int(np.ravel_multi_index(tuple(g), shape)))
            owned.append(all(overlap <= b[a] < overlap + own_len[a] for a in range(dim)))
        subs.append(Subdomain(box_start, box_len, own_start, own_len, cells,
                              np.array(gcell, dtype=np.int64), np.array(owned, dtype=bool)))
    return subs


def subdomain_matrix(J, sub: Subdomain, shape) -> Dict[int, Dict[int, float]]:
    """A_k = R_k^delta J (R_k^delta)^T on the structural pattern, as row -> {col: value}
    in the subdomain's interleaved order."""
    dim = len(shape)
    ncell = int(np.prod(shape))
    J = J.tocsr()
    J.sort_indices()
    local = {c: i for i, c in enumerate(sub.cells)}
    rows: Dict[int, Dict[int, float]] = {}
    for i, c in enumerate(sub.cells):
        for t in (0, 1):
            rows[2 * i + t] = {}

    def entry(grow, gcol):
        """J[grow, gcol] (zero when not stored), read from the CSR arrays."""
        lo, hi = J.indptr[grow], J.indptr[grow + 1]
        k = lo + int(np.searchsorted(J.indices[lo:hi], gcol))
        return float(J.data[k]) if k < hi and J.indices[k] == gcol else 0.0

    for rt, off, ct in row_pattern(dim):
        for i, c in enumerate(sub.cells):
            nb = tuple(c[a] + off[a] for a in range(dim))
            j = local.get(nb)
            if j is None:
                continue
            grow = int(sub.gcell[i]) + rt * ncell
            gcol = int(sub.gcell[j]) + ct * ncell
            rows[2 * i + rt][2 * j + ct] = entry(grow, gcol)
    return rows


def ilu0(rows: Dict[int, Dict[int, float]]):
    """Textbook ILU(0) (IKJ order) on the pattern of ``rows``.

    Returns a dict row -> {col: value} holding L (unit diagonal, entries col < row)
    and U (col >= row) in place, with (LU)_ij = A_ij for every (i, j) in the pattern."""
    return ilu_on_pattern(rows)


def box_pattern(rows: Dict[int, Dict[int, float]], sub: Subdomain, width: int = 2):
    """The rows of A_k extended by explicit zeros to the box pattern: entry (2i+t, 2j+t')
    for every pair of box cells i, j whose coordinates differ by at most ``width`` along
    every axis, and t, t' in {u, v}.  Values of A_k are kept."""
    local = {c: i for i, c in enumerate(sub.cells)}
    dim = len(sub.cells[0]) if sub.cells else 0
    out = {i: dict(r) for i, r in rows.items()}
    offs = list(np.ndindex(*([2 * width + 1] * dim)))
    for i, c in enumerate(sub.cells):
        for d in offs:
            j = local.get(tuple(c[a] + d[a] - width for a in range(dim)))
            if j is None:
                continue
            for t in (0, 1):
                for tc in (0, 1):
                    out[2 * i + t].setdefault(2 * j + tc, 0.0)
    return out


def fill_levels(rows: Dict[int, Dict[int, float]], k: int) -> Dict[int, Dict[int, int]]:
    """Level-of-fill pattern of ILU(k) (Table 2's ILU(1), ILU(2)): every entry of A has
    level 0; eliminating pivot p from row i creates or updates entry (i, j), j > p,
    with level lev(i, p) + lev(p, j) + 1, the smallest such value kept; entries of
    level above k are dropped.  Rows are processed in order, and the pivots of a row
    in increasing column order, including fill created earlier in the same row."""
    lev: Dict[int, Dict[int, int]] = {}
    for i in range(len(rows)):
        li = {j: 0 for j in rows[i]}
        heap = [p for p in li if p < i]       # pivots of row i, smallest first
        heapq.heapify(heap)
        while heap:
            p = heapq.heappop(heap)
            for j, lpj in lev[p].items():
                if j <= p:
                    continue
                new = li[p] + lpj + 1
                if new > k:
                    continue
                if j not in li:
                    li[j] = new
                    if j < i:
                        heapq.heappush(heap, j)
                elif new < li[j]:
                    li[j] = new
        lev[i] = li
    return lev


def iluk(rows: Dict[int, Dict[int, float]], k: int):
    """ILU(k): the IKJ elimination of ilu_on_pattern on the level-k pattern of
    fill_levels (fill entries start at zero).  k = 0 is ILU(0)."""
    lev = fill_levels(rows, k)
    a = {i: {j: rows[i].get(j, 0.0) for j in lev[i]} for i in rows}
    return ilu_on_pattern(a)


def ilu_on_pattern(rows: Dict[int, Dict[int, float]]):
    """Incomplete LU restricted to the pattern of ``rows`` (IKJ order): for each row i,
    for each k < i in the pattern, l_ik = a_ik / u_kk and a_ij -= l_ik u_kj for the
    j > k that are in row i's pattern; other updates are dropped."""
    a = {i: dict(r) for i, r in rows.items()}
    n = len(a)
    for i in range(n):
        ri = a[i]
        for k in sorted(c for c in ri if c < i):
            ri[k] = ri[k] / a[k][k]
            lik = ri[k]
            for j, ukj in a[k].items():
                if j > k and j in ri:
                    ri[j] -= lik * ukj
    return a


def shifted(rows, sigma):
    """A + sigma diag(A): the diagonal entries scaled by (1 + sigma).  Plain ILU(0) of the
    biharmonic-dominated u-block can produce pivots of either sign once the
    dt h^{-4} term dominates; the shifted matrix keeps them positive (a Manteuffel
    shift).  The preconditioner changes, the Newton root does not."""
    out = {i: dict(r) for i, r in rows.items()}
    for i in out:
        out[i][i] = out[i][i] * (1.0 + sigma)
    return out


def ilu_solve(fac, b):
    """Solve L U x = b with the factors of ilu0 (forward then backward substitution)."""
    n = len(fac)
    y = np.array(b, dtype=np.float64)
    for i in range(n):
        s = y[i]
        for j, v in fac[i].items():
            if j < i:
                s -= v * y[j]
        y[i] = s
    x = y
    for i in range(n - 1, -1, -1):
        s = x[i]
        for j, v in fac[i].items():
            if j > i:
                s -= v * x[j]
        x[i] = s / fac[i][i]
    return x


def to_dense(rows, n=None):
    n = n or len(rows)
    M = np.zeros((n, n))
    for i, r in rows.items():
        for j, v in r.items():
            M[i, j] = v
    return M


def to_sparse(rows, n=None):
    n = n or len(rows)
    r, c, v = [], [], []
    for i, row in rows.items():
        for j, x in row.items():
            r.append(i)
            c.append(j)
            v.append(x)
    return sp.csc_matrix((v, (r, c)), shape=(n, n))


class Schwarz:
    """Additive Schwarz preconditioner M^{-1} with a subdomain solver for inv(A_k).

    kind: "left" (restricted extension; the paper's choice), "right" (restricted
    restriction) or "classical" (eq. invM).  solver (Section 3.1 and Table 2):
    "ilu0"; "iluk" with ``level`` = k (ILU(1), ILU(2)); "iluk_box", ILU(k) whose level-0
    pattern is ``box_pattern`` (k = 0: ILU(0) on the box pattern); "lu", the exact subdomain
    solve (a sparse direct factorisation of A_k; the result does not depend on its
    ordering).  ``exact=True`` is the same as solver="lu"."""

    def __init__(self, J, shape, parts, overlap, bc, kind="left", exact=False, shift=0.0,
                 solver="ilu0", level=0):
        self.shape = tuple(shape)
        self.ncell = int(np.prod(shape))
        self.kind = kind
        self.subs = decompose(self.shape, parts, overlap, bc)
        self.factors = []
        self.solver = "lu" if exact else solver
        self.exact = self.solver == "lu"
        for sub in self.subs:
            rows = subdomain_matrix(J, sub, self.shape)
            if shift:
                rows = shifted(rows, shift)
            if self.solver == "lu":
                self.factors.append(spla.splu(to_sparse(rows)))
            elif self.solver == "iluk":
                self.factors.append(iluk(rows, level))
            elif self.solver == "iluk_box":
                self.factors.append(iluk(box_pattern(rows, sub), level))
            elif self.solver == "ilu0":
                self.factors.append(ilu0(rows))
            else:
                raise ValueError(f"unknown subdomain solver {solver!r}")

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        z = np.zeros_like(r)
        for sub, fac in zip(self.subs, self.factors):
            idx = sub.unknowns(self.ncell)
            own = np.repeat(sub.owned, 2)
            rk = r[idx].copy()
            if self.kind == "right":
                rk[~own] = 0.0
            xk = fac.solve(rk) if self.exact else ilu_solve(fac, rk)
            if self.kind == "left":
                z[idx[own]] += xk[own]
            else:
                z[idx] += xk
        return z
