"""Pins for the oracle's overlapping Schwarz preconditioners and textbook ILU(0)
(Section 3.1, eq. invM and the restricted variants)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from acch_inputs import perturbed_pair
from oracle import jacobian, schwarz
from oracle.params import Problem


def _J(shape, bc, seed=1, dt=1e-2):
    prob = Problem(bc=bc, lengths=(1.0, 1.0, 1.0)[:len(shape)])
    u1, v1, u0, v0 = perturbed_pair(shape, seed)
    return jacobian.jacobian(u1, v1, u0, v0, dt, prob)


def test_split_sizes():
    assert schwarz.split(10, 3) == [(0, 4), (4, 3), (7, 3)]
    assert schwarz.split(64, 2) == [(0, 32), (32, 32)]
    assert sum(l for _, l in schwarz.split(97, 8)) == 97


def test_pattern_counts():
    assert len(schwarz.row_pattern(2)) == 24
    assert len(schwarz.row_pattern(3)) == 40


@pytest.mark.parametrize("bc,parts,ov", [("periodic", (2, 2), 1), ("neumann", (2, 3), 2), ("neumann", (1, 1), 0)])
def test_ilu0_defining_property(bc, parts, ov):
    """(LU)_ij = A_ij for every (i, j) in the pattern of A_k (textbook ILU(0))."""
    shape = (12, 14)
    J = _J(shape, bc)
    for sub in schwarz.decompose(shape, parts, ov, bc)[:2]:
        rows = schwarz.subdomain_matrix(J, sub, shape)
        fac = schwarz.ilu0(rows)
        F = schwarz.to_dense(fac)
        L = np.tril(F, -1) + np.eye(len(F))
        U = np.triu(F)
        LU = L @ U
        A = schwarz.to_dense(rows)
        for i, r in rows.items():
            for j in r:
                assert abs(LU[i, j] - A[i, j]) <= 1e-13 * np.max(np.abs(A))


def test_ilu0_equals_lu_without_fill():
    """A tridiagonal matrix has no fill, so ILU(0) is its exact LU."""
    n = 12
    rng = np.random.default_rng(0)
    main = rng.uniform(4, 5, n)
    off1 = rng.uniform(-1, 1, n - 1)
    off2 = rng.uniform(-1, 1, n - 1)
    A = np.diag(main) + np.diag(off1, 1) + np.diag(off2, -1)
    rows = {i: {j: A[i, j] for j in range(max(0, i - 1), min(n, i + 2))} for i in range(n)}
    fac = schwarz.ilu0(rows)
    b = rng.standard_normal(n)
    assert np.allclose(schwarz.ilu_solve(fac, b), np.linalg.solve(A, b), rtol=1e-13, atol=1e-14)


def test_subdomain_matrix_is_restriction():
    """A_k equals the principal submatrix R J R^T of the global Jacobian."""
    shape = (10, 12)
    J = _J(shape, "periodic")
    sub = schwarz.decompose(shape, (2, 2), 1, "periodic")[3]
    idx = sub.unknowns(int(np.prod(shape)))
    want = J.toarray()[np.ix_(idx, idx)]
    got = schwarz.to_dense(schwarz.subdomain_matrix(J, sub, shape))
    assert np.array_equal(got, want)


def test_decomposition_owned_sets_partition():
    for bc, shape, parts, ov in [("periodic", (12, 16), (2, 4), 2), ("neumann", (9, 11), (3, 2), 1)]:
        subs = schwarz.decompose(shape, parts, ov, bc)
        owned = np.concatenate([s.gcell[s.owned] for s in subs])
        assert np.array_equal(np.sort(owned), np.arange(int(np.prod(shape))))


def test_periodic_box_must_not_wrap_onto_itself():
    with pytest.raises(ValueError):
        schwarz.decompose((8, 8), (1, 2), 1, "periodic")
    with pytest.raises(ValueError):
        schwarz.decompose((8, 8), (2, 2), 2, "periodic")


def test_single_exact_subdomain_is_the_inverse():
    """One Neumann subdomain without overlap and an exact subdomain solve: M^{-1} = J^{-1}."""
    shape = (6, 7)
    J = _J(shape, "neumann")
    P = schwarz.Schwarz(J, shape, (1, 1), 0, "neumann", kind="left", exact=True)
    r = np.random.default_rng(3).standard_normal(J.shape[0])
    assert np.allclose(P.apply(r), spla.spsolve(J.tocsc(), r), rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("kind", ["left", "right", "classical"])
def test_schwarz_variants_precondition_gmres(kind):
    """Each variant is a usable preconditioner: GMRES converges to the direct solution."""
    shape = (16, 16)
    J = _J(shape, "periodic", dt=5e-2)
    P = schwarz.Schwarz(J, shape, (2, 2), 1, "periodic", kind=kind)
    r = np.random.default_rng(4).standard_normal(J.shape[0])
    M = spla.LinearOperator(J.shape, matvec=P.apply)
    x, info = spla.gmres(J, r, M=M, rtol=1e-11, restart=30, maxiter=200)
    assert info == 0
    assert np.linalg.norm(J @ x - r) <= 1e-10 * np.linalg.norm(r)


def test_left_ras_writes_each_unknown_once():
    """Left-RAS with identity subdomain matrices is the identity map."""
    shape = (16, 18)
    n = 2 * int(np.prod(shape))
    I = sp.identity(n, format="csr")
    P = schwarz.Schwarz(I, shape, (2, 3), 2, "periodic", kind="left")
    r = np.random.default_rng(5).standard_normal(n)
    assert np.allclose(P.apply(r), r, rtol=0, atol=0)


def _fill_path_levels(rows, k):
    """Levels by the fill-path characterisation of ILU(k): entry (i, j) has level
    (length of the shortest path i -> j in the graph of A whose interior vertices are
    all numbered below min(i, j)) - 1, kept when <= k.  Breadth-first search per row."""
    n = len(rows)
    out = {}
    for i in range(n):
        li = {}
        for j in range(n):
            lim = min(i, j)
            seen = {i: 0}
            q = [i]
            found = None
            while q and found is None:
                nq = []
                for a in q:
                    for b in rows[a]:
                        if b == j:
                            found = seen[a] + 1
                            break
                        if b < lim and b not in seen:
                            seen[b] = seen[a] + 1
                            nq.append(b)
                    if found is not None:
                        break
                q = nq
            if found is not None and found - 1 <= k:
                li[j] = found - 1
        out[i] = li
    return out


@pytest.mark.parametrize("k", [1, 2, 3])
def test_iluk_levels_match_fill_paths(k):
    """Symbolic ILU(k) levels = the fill-path characterisation (brute force)."""
    shape = (6, 5)
    J = _J(shape, "neumann")
    sub = schwarz.decompose(shape, (1, 1), 0, "neumann")[0]
    rows = schwarz.subdomain_matrix(J, sub, shape)
    lev = schwarz.fill_levels(rows, k)
    ref = _fill_path_levels(rows, k)
    assert lev == ref


@pytest.mark.parametrize("k", [1, 2])
def test_iluk_defining_property(k):
    """(LU)_ij = A_ij for every (i, j) of the level-k pattern; outside the pattern L and U
    are zero; fill occurs (the pattern grows with k)."""
    shape = (12, 14)
    J = _J(shape, "neumann")
    sub = schwarz.decompose(shape, (2, 2), 1, "neumann")[1]
    rows = schwarz.subdomain_matrix(J, sub, shape)
    lev = schwarz.fill_levels(rows, k)
    assert sum(len(r) for r in lev.values()) > sum(len(r) for r in rows.values())
    F = schwarz.to_dense(schwarz.iluk(rows, k))
    n = len(F)
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    A = schwarz.to_dense(rows)
    LU = L @ U
    mask = np.zeros((n, n), dtype=bool)
    for i, r in lev.items():
        for j in r:
            mask[i, j] = True
    assert np.all(F[~mask] == 0.0)
    assert np.max(np.abs((LU - A)[mask])) <= 1e-12 * np.max(np.abs(A))


def test_iluk_zero_is_ilu0_and_full_level_is_exact_lu():
    shape = (10, 12)
    J = _J(shape, "periodic", dt=1e-3)
    sub = schwarz.decompose(shape, (2, 2), 1, "periodic")[0]
    rows = schwarz.subdomain_matrix(J, sub, shape)
    assert schwarz.iluk(rows, 0) == schwarz.ilu0(rows)
    n = len(rows)
    F = schwarz.to_dense(schwarz.iluk(rows, n))
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    A = schwarz.to_dense(rows)
    assert np.max(np.abs(L @ U - A)) <= 1e-12 * np.max(np.abs(A))


def test_box_pattern_extends_the_stencil_pattern():
    """The box pattern holds every entry of A_k (values kept) and adds zeros so that an
    interior cell's two rows couple to all 25 cells at Chebyshev distance <= 2, both
    types: 50 entries per row; no entry couples cells further apart."""
    shape = (12, 14)
    J = _J(shape, "neumann")
    sub = schwarz.decompose(shape, (2, 2), 1, "neumann")[0]
    rows = schwarz.subdomain_matrix(J, sub, shape)
    box = schwarz.box_pattern(rows, sub)
    for i, r in rows.items():
        for j, v in r.items():
            assert box[i][j] == v
    for i, r in box.items():
        ci = sub.cells[i // 2]
        for j, v in r.items():
            cj = sub.cells[j // 2]
            assert max(abs(ci[0] - cj[0]), abs(ci[1] - cj[1])) <= 2
            if j not in rows[i]:
                assert v == 0.0
    ci = sub.cells.index((4, 4))
    assert len(box[2 * ci]) == len(box[2 * ci + 1]) == 50


def test_box_ilu0_is_exact_lu_on_narrow_boxes():
    """On a box 3 cells wide every cell of rows y-2 .. y+2 is within distance 2 of a cell
    in row y, so the box pattern is the whole envelope of the natural order, which holds
    all LU fill: ILU(0) on it is the exact LU.  The same box with the width-1 pattern
    drops fill (control)."""
    shape = (9, 3)
    J = _J(shape, "neumann", dt=1e-3)
    sub = schwarz.decompose(shape, (1, 1), 0, "neumann")[0]
    rows = schwarz.subdomain_matrix(J, sub, shape)
    A = schwarz.to_dense(rows)
    b = np.random.default_rng(3).standard_normal(len(A))
    for width, exact in ((2, True), (1, False)):
        fac = schwarz.ilu0(schwarz.box_pattern(rows, sub, width))
        F = schwarz.to_dense(fac)
        L = np.tril(F, -1) + np.eye(len(F))
        err = np.max(np.abs(L @ np.triu(F) - A)) / np.max(np.abs(A))
        if exact:
            assert err <= 1e-13
            x = schwarz.ilu_solve(fac, b)
            assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.norm(x)
        else:
            assert err > 1e-10   # dropped fill, far above rounding


@pytest.mark.parametrize("k", [0, 1])
def test_box_iluk_defining_property(k):
    """ILU(k) on the box base pattern: (LU)_ij = A_ij on the level-k pattern of the box
    pattern, zero outside it."""
    shape = (12, 14)
    J = _J(shape, "periodic")
    sub = schwarz.decompose(shape, (2, 2), 1, "periodic")[3]
    rows = schwarz.box_pattern(schwarz.subdomain_matrix(J, sub, shape), sub)
    lev = schwarz.fill_levels(rows, k)
    F = schwarz.to_dense(schwarz.iluk(rows, k))
    n = len(F)
    L = np.tril(F, -1) + np.eye(n)
    A = schwarz.to_dense(rows)
    mask = np.zeros((n, n), dtype=bool)
    for i, r in lev.items():
        for j in r:
            mask[i, j] = True
    assert np.all(F[~mask] == 0.0)
    assert np.max(np.abs((L @ np.triu(F) - A)[mask])) <= 1e-12 * np.max(np.abs(A))


@pytest.mark.parametrize("solver,level", [("iluk", 1), ("iluk", 2), ("lu", 0), ("iluk_box", 0), ("iluk_box", 1)])
def test_subdomain_solvers_precondition_gmres(solver, level):
    """Left-RAS with each Table 2 subdomain solver drives GMRES to the direct solution;
    the exact subdomain LU solves A_k x = r_k to rounding."""
    shape = (16, 18)
    J = _J(shape, "neumann", dt=1e-3).tocsr()
    P = schwarz.Schwarz(J, shape, (2, 2), 1, "neumann", kind="left", solver=solver, level=level)
    b = np.random.default_rng(0).standard_normal(J.shape[0])
    M = spla.LinearOperator(J.shape, matvec=P.apply)
    x, info = spla.gmres(J, b, M=M, rtol=1e-12, atol=0.0, restart=60, maxiter=20)
    assert info == 0
    assert np.linalg.norm(x - spla.spsolve(J.tocsc(), b)) <= 1e-8 * np.linalg.norm(x)
    if solver == "lu":
        sub = P.subs[1]
        A = schwarz.to_dense(schwarz.subdomain_matrix(J, sub, shape))
        r = np.random.default_rng(1).standard_normal(len(A))
        assert np.linalg.norm(A @ P.factors[1].solve(r) - r) <= 1e-12 * np.linalg.norm(r) * np.linalg.cond(A)
