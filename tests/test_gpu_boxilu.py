"""GPU parity of the box-pattern ILU(0) subdomain solver (Section 3.1, Table 2's ILU(0)
under the box-pattern reading) against the oracle: every factor entry against the
oracle's textbook ILU(0) on the box pattern, M^{-1} r against the oracle's Schwarz
operator for the three variants, FP64 and FP32 factors, boxes up to the largest the
kernels take, and whole Newton steps against the oracle's roots."""
import math

import numpy as np
import pytest

from acch_inputs import perturbed_pair, random_ic
from oracle import controller, jacobian, newton, schwarz
from oracle.params import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2007_04560_amd import Solver  # noqa: E402

# (shape (ny, nx), bc, sub (x, y), overlap)
CASES = [((37, 29), "periodic", (2, 2), 1), ((45, 58), "neumann", (3, 2), 2), ((33, 17), "neumann", (1, 1), 0),
         ((26, 40), "periodic", (3, 2), 2)]

# lower and upper cells of the records, (dx, dy) in unknown order
LOWER = [(dx, -2) for dx in range(-2, 3)] + [(dx, -1) for dx in range(-2, 3)] + [(-2, 0), (-1, 0)]
UPPER = [(1, 0), (2, 0)] + [(dx, 1) for dx in range(-2, 3)] + [(dx, 2) for dx in range(-2, 3)]


def prob(bc):
    return Problem(bc=bc, alpha=1.2, beta=1.2, theta=0.1, gamma=1e-3, rho=1.0)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def vec(u, v):
    return np.concatenate([u.ravel(), v.ravel()])


def _setup(shape, bc, sub, ov, precision="fp64", kind="left", dt=2e-3, seed=31, shift=0.0):
    u1, v1, u0, v0 = perturbed_pair(shape, seed, amp=0.03)
    s = Solver(u0, v0, bc=bc, sub=sub, overlap=ov, subsolver="iluk_box", fill_level=0, precision=precision,
               schwarz=kind, ilu_shift=shift)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    s.factor()
    return s, jacobian.jacobian(u1, v1, u0, v0, dt, prob(bc))


@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
@pytest.mark.parametrize("shift", [0.0, 0.02])
def test_box_ilu0_factors_match_oracle(shape, bc, sub, ov, shift):
    """Each record slot equals the oracle's ILU(0) on the box pattern of A_k (+ shift
    diag(A_k)): L entries, U entries, the stored reciprocal pivots; zeros towards cells
    outside the grid; padding cells are identity rows."""
    s, Jo = _setup(shape, bc, sub, ov, shift=shift)
    info = s.info()
    bw, bh = info["box_w"], info["box_h"]
    rec = s.export_factors().cpu().numpy()
    assert rec.shape == (info["nsub"], bw * bh, 104)
    subs = schwarz.decompose(shape, (sub[1], sub[0]), ov, bc)
    worst, scale = 0.0, 0.0
    for k, sd in enumerate(subs):
        rows = schwarz.subdomain_matrix(Jo, sd, shape)
        if shift:
            rows = schwarz.shifted(rows, shift)
        fac = schwarz.iluk(schwarz.box_pattern(rows, sd), 0)
        local = {c: i for i, c in enumerate(sd.cells)}
        seen = np.zeros((bw * bh, 104), dtype=bool)
        for c, oi in local.items():
            by, bx = c
            cell = by * bw + bx
            want = np.zeros(104)
            for q, (dx, dy) in enumerate(LOWER):
                oj = local.get((by + dy, bx + dx))
                if oj is not None:
                    want[4 * q:4 * q + 4] = [fac[2 * oi].get(2 * oj, 0.0), fac[2 * oi].get(2 * oj + 1, 0.0),
                                             fac[2 * oi + 1].get(2 * oj, 0.0), fac[2 * oi + 1].get(2 * oj + 1, 0.0)]
            want[48] = fac[2 * oi + 1][2 * oi]
            for q, (dx, dy) in enumerate(UPPER):
                oj = local.get((by + dy, bx + dx))
                if oj is not None:
                    want[52 + 4 * q:56 + 4 * q] = [fac[2 * oi].get(2 * oj, 0.0), fac[2 * oi].get(2 * oj + 1, 0.0),
                                                   fac[2 * oi + 1].get(2 * oj, 0.0),
                                                   fac[2 * oi + 1].get(2 * oj + 1, 0.0)]
            want[100] = 1.0 / fac[2 * oi][2 * oi]
            want[101] = fac[2 * oi][2 * oi + 1]
            want[102] = 1.0 / fac[2 * oi + 1][2 * oi + 1]
            got = rec[k, cell]
            err = np.abs(got - want)
            rel = np.array([100, 102])
            err[rel] /= np.abs(want[rel])
            worst = max(worst, float(np.max(err)))
            scale = max(scale, float(np.max(np.abs(want))))
            seen[cell] = True
        # padding and cells outside the grid: identity rows
        for cell in range(bw * bh):
            if not seen[cell].any():
                ident = np.zeros(104)
                ident[100] = ident[102] = 1.0
                assert np.array_equal(rec[k, cell], ident), (k, cell)
    assert worst <= 1e-11 * max(scale, 1.0)


@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
@pytest.mark.parametrize("kind", ["left", "right", "classical"])
def test_box_ilu0_preconditioner_matches_oracle(shape, bc, sub, ov, kind):
    s, Jo = _setup(shape, bc, sub, ov, kind=kind)
    r = np.random.default_rng(7).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind=kind, solver="iluk_box", level=0).apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))


@pytest.mark.parametrize("shape,bc,sub,ov", CASES[:2])
def test_box_ilu0_mixed_precision(shape, bc, sub, ov):
    """FP32 records (the pivot rows of the elimination are read back in FP32): M^{-1} r
    within FP32 rounding of the FP64 oracle."""
    s, Jo = _setup(shape, bc, sub, ov, precision="mixed")
    r = np.random.default_rng(9).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", solver="iluk_box", level=0).apply(r)
    assert np.linalg.norm(z - zo) <= 1e-4 * np.linalg.norm(zo)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_box_ilu0_largest_boxes(precision):
    """Padded boxes 144 wide (48 cells per wavefront, the most the LDS stages take) and
    a ragged split; then a box 160 tall (the most rows of the LDS ring)."""
    for shape, sub, ov, bw, bh in (((30, 279), (2, 1), 2, 144, 34), ((315, 20), (1, 2), 1, 22, 160)):
        s, Jo = _setup(shape, "neumann", sub, ov, precision=precision, dt=1e-3)
        info = s.info()
        assert (info["box_w"], info["box_h"]) == (bw, bh)
        r = np.random.default_rng(10).standard_normal(Jo.shape[0])
        z = s.precondition(dev(r)).cpu().numpy()
        zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, "neumann", kind="left", solver="iluk_box",
                             level=0).apply(r)
        if precision == "fp64":
            assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))
        else:
            assert np.linalg.norm(z - zo) <= 1e-4 * np.linalg.norm(zo)
        s.close()


def test_box_ilu0_rejects_boxes_beyond_its_limits():
    u0, v0 = random_ic((24, 283), 0)
    with pytest.raises(Exception):   # 146 wide
        Solver(u0, v0, bc="neumann", sub=(2, 1), overlap=2, subsolver="iluk_box", fill_level=0)
    u0, v0 = random_ic((317, 20), 0)
    with pytest.raises(Exception):   # 161 tall
        Solver(u0, v0, bc="neumann", sub=(1, 2), overlap=1, subsolver="iluk_box", fill_level=0)


def _rel_l2(u, v, uo, vo):
    return math.sqrt(np.sum((u - uo) ** 2 + (v - vo) ** 2) / np.sum(uo ** 2 + vo ** 2))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_box_ilu0_steps_match_oracle(precision):
    """Four steps of the 64x64 periodic workload (2x2 subdomains, overlap 1) with plain
    (unshifted) box-pattern ILU(0): roots = the oracle's to 1e-10 per step, the same
    Newton counts, and fewer GMRES iterations than shifted stencil-pattern ILU(0)."""
    shape = (64, 64)
    u0, v0 = random_ic(shape, 0)
    kw = dict(bc="periodic", sub=(2, 2), overlap=1, dt_fixed=1e-3, newton_rtol=1e-12, newton_atol=1e-13,
              gmres_rtol=1e-12, precision=precision)
    s = Solver(u0, v0, subsolver="iluk_box", fill_level=0, **kw)
    s0 = Solver(u0, v0, ilu_shift=0.02, **kw)
    run = controller.Run(prob("periodic"), u0.copy(), v0.copy(), adaptive=False, dt_fixed=1e-3,
                         newton=newton.NewtonOptions(rtol=1e-12, atol=1e-13))
    its, its0 = 0, 0
    for k in range(4):
        info = s.step(1)[0]
        its += info["gmres_its"]
        its0 += s0.step(1)[0]["gmres_its"]
        rec = run.step()
        ug, vg = s.fields()
        assert _rel_l2(ug, vg, run.u, run.v) <= 1e-10, k
        assert info["newton_its"] == rec.newton_its
    assert its < its0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["left", "classical"])
def test_box_ilu0_one_wave_form_matches_oracle(precision, kind):
    """576 boxes of 6x6 cells (24x24 subdomains of a 96x96 periodic grid, overlap 1): at
    least two boxes per CU with at most 16 cells per wavefront, so the sweeps run one wave
    per box without barriers; M^{-1} r against the oracle."""
    shape, bc, sub, ov = (96, 96), "periodic", (24, 24), 1
    s, Jo = _setup(shape, bc, sub, ov, precision=precision, kind=kind)
    info = s.info()
    assert info["nsub"] == 576 and (info["box_w"], info["box_h"]) == (6, 6)
    r = np.random.default_rng(13).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind=kind, solver="iluk_box", level=0).apply(r)
    if precision == "fp64":
        assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))
    else:
        assert np.linalg.norm(z - zo) <= 1e-4 * np.linalg.norm(zo)


def test_box_ilu0_factor_blocks_of_128_rows():
    """A box 69 rows tall takes the 128-thread factorisation blocks: records and M^{-1} r
    against the oracle."""
    shape, bc, sub, ov = (130, 20), "neumann", (1, 2), 2
    s, Jo = _setup(shape, bc, sub, ov, dt=1e-3)
    assert s.info()["box_h"] == 69
    r = np.random.default_rng(14).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", solver="iluk_box", level=0).apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("shape,bc,sub,ov", [((12, 12), "periodic", (2, 2), 1), ((10, 14), "neumann", (2, 1), 2),
                                             ((9, 11), "neumann", (1, 1), 0)])
@pytest.mark.parametrize("kind", ["left", "right", "classical"])
def test_box_ilu0_transpose_is_the_transpose_of_the_oracle_operator(shape, bc, sub, ov, kind):
    """M^{-T} r with box-pattern ILU(0) (transposed records, U^T then L^T sweeps, the
    variant's restriction and extension exchanged) against the transpose of the oracle's
    M^{-1}, formed column by column."""
    s, Jo = _setup(shape, bc, sub, ov, kind=kind, dt=5e-3, seed=52)
    P = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind=kind, solver="iluk_box", level=0)
    n2 = Jo.shape[0]
    Minv = np.column_stack([P.apply(np.eye(n2)[:, k]) for k in range(n2)])
    r = np.random.default_rng(5).standard_normal(n2)
    z = s.precondition_transpose(dev(r)).cpu().numpy()
    assert _rel(z, Minv.T @ r) <= 1e-10


@pytest.mark.parametrize("shape,sub,ov", [((96, 96), (24, 24), 1), ((128, 128), (4, 4), 2)])
@pytest.mark.parametrize("kind", ["left", "classical"])
def test_box_ilu0_transpose_adjoint_identity(shape, sub, ov, kind):
    """<M^{-T} a, b> = <a, M^{-1} b> with the one-wave (576 boxes of 6x6) and the 256-thread
    (16 boxes of 36x36) sweep forms."""
    s, _ = _setup(shape, "periodic", sub, ov, kind=kind, dt=1e-3, seed=53)
    rng = np.random.default_rng(6)
    a = dev(rng.standard_normal(2 * shape[0] * shape[1]))
    b = dev(rng.standard_normal(2 * shape[0] * shape[1]))
    lhs = float(torch.dot(s.precondition_transpose(a), b))
    rhs = float(torch.dot(a, s.precondition(b)))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_box_ilu0_adjoint_step_matches_oracle():
    """One adjoint step (J^T solve preconditioned by the transposed box-pattern ILU(0)
    operator) against the oracle's sparse direct adjoint step."""
    from oracle import adjoint as oadj
    shape, bc = (36, 30), "neumann"
    u1, v1, u0, v0 = perturbed_pair(shape, 55, amp=0.03)
    dt = 2e-3
    s = Solver(u0, v0, bc=bc, sub=(3, 2), overlap=2, subsolver="iluk_box", fill_level=0, gmres_rtol=1e-13,
               gmres_max_restarts=30)
    g1 = np.random.default_rng(8).standard_normal(2 * u1.size)
    gprev, dp, its, _ = s.adjoint_step(dev(vec(u1, v1)), dev(vec(u0, v0)), dt, dev(g1))
    g0o, _, dpo = oadj.adjoint_step(u1, v1, u0, v0, dt, Problem(bc=bc), g1)
    assert its > 0
    assert _rel(gprev.cpu().numpy(), g0o) <= 1e-9


def _box32(u0, v0, precision="fp64", **kw):
    """The 512x512 box-pattern workload's Schwarz settings: 32x32 subdomains (1024 boxes of
    20x20 cells, one wave per box), overlap 2, unshifted ILU(0) on the box pattern."""
    return Solver(u0, v0, bc="periodic", sub=(32, 32), overlap=2, subsolver="iluk_box", fill_level=0,
                  ilu_shift=0.0, precision=precision, **kw)


def _box32_factored(precision, seed):
    shape = (512, 512)
    u0, v0 = random_ic(shape, 0)
    rng = np.random.default_rng(seed)
    u1 = u0 + 0.01 * rng.uniform(-1, 1, shape)
    v1 = v0 + 0.01 * rng.uniform(-1, 1, shape)
    s = _box32(u0, v0, precision)
    info = s.info()
    assert info["nsub"] == 1024 and (info["box_w"], info["box_h"]) == (20, 20)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), 1e-4)
    s.factor()
    return s, (u1, v1, u0, v0), rng


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_box32_workload_sampled_subdomains_match_oracle(precision):
    """At the full 512x512 size in the benchmark's launch configuration: M^{-1} r on the
    owned cells of sampled subdomains (the two corner boxes, which wrap, an edge box and an
    interior one) against the oracle's ILU(0) solve of each subdomain on its own; with the
    restricted extension an owned cell takes its value from its own box only."""
    s, (u1, v1, u0, v0), rng = _box32_factored(precision, 61)
    shape, n = u0.shape, u0.size
    r = rng.standard_normal(2 * n)
    z = s.precondition(dev(r)).cpu().numpy()
    J = jacobian.jacobian(u1, v1, u0, v0, 1e-4, prob("periodic")).tocsr()
    subs = schwarz.decompose(shape, (32, 32), 2, "periodic")
    for k in (0, 31, 529, 1023):
        sub = subs[k]
        fac = schwarz.iluk(schwarz.box_pattern(schwarz.subdomain_matrix(J, sub, shape), sub), 0)
        idx = sub.unknowns(n)
        own = np.repeat(sub.owned, 2)
        zk = schwarz.ilu_solve(fac, r[idx])[own]
        zg = z[idx[own]]
        if precision == "fp64":
            assert np.max(np.abs(zg - zk)) <= 1e-10 * np.max(np.abs(zk)), k
        else:
            assert np.linalg.norm(zg - zk) <= 1e-4 * np.linalg.norm(zk), k


def test_box32_workload_transpose_adjoint_identity():
    """The adjoint workload's transposed operator at 512x512 over 32x32 subdomains:
    <M^{-T} a, b> = <a, M^{-1} b>."""
    s, _, rng = _box32_factored("fp64", 62)
    a = dev(rng.standard_normal(2 * 512 * 512))
    b = dev(rng.standard_normal(2 * 512 * 512))
    lhs = float(torch.dot(s.precondition_transpose(a), b))
    rhs = float(torch.dot(a, s.precondition(b)))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_box32_workload_roots_at_sampled_steps():
    """The 512x512 box-pattern workload as the benchmark runs it (adaptive, tolerance 1e-8):
    at steps 1, 25 and 60 the oracle's residual of the GPU's new state, taken with the
    step's dt and the GPU's previous state, is at the Newton tolerance; mass is exact and
    the energy decreases."""
    from oracle import scheme
    shape = (512, 512)
    u0, v0 = random_ic(shape, 0)
    P = prob("periodic")
    s = _box32(u0, v0, adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1e4)
    M0 = scheme.mass(u0, P)
    done = 0
    for k in (1, 25, 60):
        if k - 1 > done:
            s.step(k - 1 - done)
        up, vp = s.fields()
        info = s.step(1)[0]
        done = k
        ug, vg = s.fields()
        Fu, Fv = scheme.residual(ug, vg, up, vp, info["dt"], P)
        F0u, F0v = scheme.residual(up, vp, up, vp, info["dt"], P)
        f1 = math.sqrt(np.sum(Fu ** 2 + Fv ** 2))
        f0 = math.sqrt(np.sum(F0u ** 2 + F0v ** 2))
        assert f1 <= 2e-8 * f0, (k, f1, f0)
        assert abs(scheme.mass(ug, P) - M0) <= 1e-12 * M0
        assert scheme.energy(ug, vg, P) < scheme.energy(up, vp, P)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["left", "right", "classical"])
def test_box_ilu0_wide_wavefronts(precision, kind):
    """Boxes 54 wide (18 cells on a wavefront, more than one wave's quads hold, so the
    256-thread sweeps): M^{-1} r against the oracle for the three variants."""
    shape, bc, sub, ov = (60, 100), "neumann", (2, 1), 2
    s, Jo = _setup(shape, bc, sub, ov, precision=precision, kind=kind)
    info = s.info()
    assert 16 < -(-info["box_w"] // 3) <= 32 and info["box_h"] >= 54   # 17 .. 32 cells on a wavefront
    r = np.random.default_rng(15).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind=kind, solver="iluk_box", level=0).apply(r)
    if precision == "fp64":
        assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))
    else:
        assert np.linalg.norm(z - zo) <= 1e-4 * np.linalg.norm(zo)


@pytest.mark.parametrize("kind", ["left", "classical"])
def test_box_ilu0_wide_wavefronts_transpose(kind):
    """<M^{-T} a, b> = <a, M^{-1} b> on 68 x 68 boxes (23 cells on a wavefront)."""
    s, _ = _setup((128, 128), "periodic", (2, 2), 2, kind=kind, dt=1e-3, seed=54)
    assert 16 < -(-s.info()["box_w"] // 3) <= 32
    rng = np.random.default_rng(16)
    a = dev(rng.standard_normal(2 * 128 * 128))
    b = dev(rng.standard_normal(2 * 128 * 128))
    lhs = float(torch.dot(s.precondition_transpose(a), b))
    rhs = float(torch.dot(a, s.precondition(b)))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)
