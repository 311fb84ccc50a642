"""GPU parity: every stage of the HIP path against the FP64 CPU oracle.

All inputs are seeded (acch_inputs); the oracle never sees GPU output except where a
test checks a property of it (a residual of the GPU's root, the ILU(0) defining
identity).  Tolerances: floating point only; kernels that evaluate the same
formula agree to ~1e-13 relative, whole steps to 1e-10 relative l2 per step.
"""
import math

import numpy as np
import pytest

from acch_inputs import perturbed_pair, random_ic
from oracle import controller, jacobian, newton, scalar, schwarz, scheme
from oracle.params import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2007_04560_amd import Solver  # noqa: E402

# 2D slot offsets of the Jacobian (include/acch.h): (row type, col type, dx, dy)
JSLOTS = ([(0, 0, dx, dy) for dx, dy in [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1), (-2, 0), (2, 0), (0, -2), (0, 2),
                                         (-1, -1), (1, -1), (-1, 1), (1, 1)]]
          + [(0, 1, dx, dy) for dx, dy in [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]]
          + [(1, 1, dx, dy) for dx, dy in [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]]
          + [(1, 0, 0, 0)])
# ILU factor slots (include/acch.h): (row type, col type, dx, dy); diagonal slots hold 1/U
FSLOTS = ([(0, 0, -1, 0), (0, 0, -2, 0), (0, 0, 1, -1), (0, 0, 0, -1), (0, 0, -1, -1), (0, 0, 0, -2),
           (0, 1, -1, 0), (0, 1, 0, -1), (1, 1, -1, 0), (1, 1, 0, -1), (1, 0, 0, 0),
           (0, 0, 0, 0), (0, 0, 1, 0), (0, 0, 2, 0), (0, 0, -1, 1), (0, 0, 0, 1), (0, 0, 1, 1), (0, 0, 0, 2),
           (0, 1, 0, 0), (0, 1, 1, 0), (0, 1, 0, 1), (1, 1, 0, 0), (1, 1, 1, 0), (1, 1, 0, 1)])
INV_DIAG = {11, 21}


def prob(bc, L=(1.0, 1.0), mobility="midpoint", **kw):
    base = dict(alpha=1.2, beta=1.2, theta=0.1, gamma=1e-3, rho=1.0)
    base.update(kw)
    return Problem(bc=bc, lengths=L, mobility=mobility, **base)


def solver(u0, v0, bc, L=(1.0, 1.0), mobility="midpoint", **kw):
    phys = {k: kw.pop(k) for k in ["alpha", "beta", "theta", "gamma", "rho"] if k in kw}
    return Solver(u0, v0, bc=bc, L=L, mobility=mobility, **phys, **kw)


def vec(u, v):
    return np.concatenate([u.ravel(), v.ravel()])


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


CASES = [((37, 29), "periodic", (2, 2), 1), ((64, 64), "periodic", (2, 2), 1), ((45, 100), "neumann", (3, 2), 2),
         ((33, 17), "neumann", (1, 1), 0)]


@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
@pytest.mark.parametrize("mob", ["midpoint", "average"])
def test_residual_matches_oracle(shape, bc, sub, ov, mob):
    u1, v1, u0, v0 = perturbed_pair(shape, 17, amp=0.03)
    kw = dict(alpha=4.0, beta=2.0, gamma=0.005, rho=0.001)
    L = (1.0, 1.3)
    P = prob(bc, L, mob, **kw)
    dt = 3e-3
    s = solver(u0, v0, bc, L, mob, sub=sub, overlap=ov, **kw)
    F, f2, bad = s.residual(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    Fu, Fv = scheme.residual(u1, v1, u0, v0, dt, P)
    want = vec(Fu, Fv)
    got = F.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert abs(f2 - want @ want) <= 1e-12 * (want @ want)
    assert bad == 0
    # an inadmissible cell is counted
    u1b = u1.copy()
    u1b[3, 4] = 1.2
    _, _, bad = s.residual(dev(vec(u1b, v1)), dev(vec(u0, v0)), dt)
    assert bad == 1


@pytest.mark.parametrize("shape,bc", [((37, 29), "periodic"), ((45, 100), "neumann")])
def test_energy_and_mass_match_oracle(shape, bc):
    u, v = random_ic(shape, 3)
    L = (1.0, 1.3)
    P = prob(bc, L, alpha=4.0, beta=2.0, gamma=0.005)
    sub = (2, 2)
    s = solver(u, v, bc, L, sub=sub, overlap=1, alpha=4.0, beta=2.0, gamma=0.005)
    E, M = s.energy()
    assert abs(E - scheme.energy(u, v, P)) <= 1e-13 * abs(scheme.energy(u, v, P))
    assert abs(M - scheme.mass(u, P)) <= 1e-14 * scheme.mass(u, P)


def oracle_slots(Jsp, shape, bc):
    """The oracle Jacobian rearranged into the 24-slot layout."""
    ny, nx = shape
    n = nx * ny
    J = Jsp.tocsr()
    out = np.zeros((24, ny, nx))
    for k, (rt, ct, dx, dy) in enumerate(JSLOTS):
        for y in range(ny):
            for x in range(nx):
                xx, yy = x + dx, y + dy
                if bc == "periodic":
                    xx %= nx
                    yy %= ny
                elif not (0 <= xx < nx and 0 <= yy < ny):
                    continue
                out[k, y, x] = J[rt * n + y * nx + x, ct * n + yy * nx + xx]
    return out


@pytest.mark.parametrize("shape,bc,sub,ov", CASES[:1] + CASES[2:])
@pytest.mark.parametrize("mob", ["midpoint", "average"])
def test_jacobian_and_spmv_match_oracle(shape, bc, sub, ov, mob):
    u1, v1, u0, v0 = perturbed_pair(shape, 23, amp=0.03)
    L = (1.0, 1.3)
    P = prob(bc, L, mob)
    dt = 2e-3
    s = solver(u0, v0, bc, L, mob, sub=sub, overlap=ov)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    got = s.export_jacobian().cpu().numpy()
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, P)
    want = oracle_slots(Jo, shape, bc)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    x = np.random.default_rng(4).standard_normal(2 * u1.size)
    y = s.apply_jacobian(dev(x)).cpu().numpy()
    yo = Jo @ x
    assert np.max(np.abs(y - yo)) <= 1e-12 * np.max(np.abs(yo))


def oracle_factor_slots(J, shape, bc, sub, ov, bw, bh, shift=0.0):
    subs = schwarz.decompose(shape, (sub[1], sub[0]), ov, bc)
    out = np.zeros((len(subs), 24, bh, bw))
    mask = np.zeros((len(subs), bh, bw), dtype=bool)
    for s_i, sd in enumerate(subs):
        rows = schwarz.subdomain_matrix(J, sd, shape)
        fac = schwarz.ilu0(schwarz.shifted(rows, shift) if shift else rows)
        index = {c: i for i, c in enumerate(sd.cells)}
        for i, (by, bx) in enumerate(sd.cells):
            mask[s_i, by, bx] = True
            for k, (rt, ct, dx, dy) in enumerate(FSLOTS):
                j = index.get((by + dy, bx + dx))
                if j is None:
                    continue
                val = fac[2 * i + rt].get(2 * j + ct, 0.0)
                out[s_i, k, by, bx] = 1.0 / val if k in INV_DIAG else val
    return out, mask, subs


@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
@pytest.mark.parametrize("shift", [0.0, 0.02])
def test_ilu_factors_and_preconditioner_match_oracle(shape, bc, sub, ov, shift):
    u1, v1, u0, v0 = perturbed_pair(shape, 31, amp=0.03)
    P = prob(bc)
    dt = 5e-3
    s = solver(u0, v0, bc, sub=sub, overlap=ov, ilu_shift=shift)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    s.factor()
    got = s.export_factors().cpu().numpy()
    info = s.info()
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, P)
    want, mask, subs = oracle_factor_slots(Jo, shape, bc, sub, ov, info["box_w"], info["box_h"], shift)
    m = np.broadcast_to(mask[:, None], want.shape)
    scale = np.max(np.abs(want[m]))
    assert np.max(np.abs(got[m] - want[m])) <= 1e-11 * scale
    r = np.random.default_rng(7).standard_normal(2 * u1.size)
    z = s.precondition(dev(r)).cpu().numpy()
    Pc = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", shift=shift)
    zo = Pc.apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))


@pytest.mark.parametrize("shape,bc,sub,ov", CASES[1:3])
def test_gmres_solves_the_newton_system(shape, bc, sub, ov):
    u1, v1, u0, v0 = perturbed_pair(shape, 41, amp=0.03)
    P = prob(bc)
    dt = 1e-3
    s = solver(u0, v0, bc, sub=sub, overlap=ov, gmres_rtol=1e-12, gmres_restart=30)
    X = dev(vec(u1, v1))
    Xn = dev(vec(u0, v0))
    F, _, _ = s.residual(X, Xn, dt)
    s.jacobian(X, Xn, dt)
    s.factor()
    S, its, res = s.gmres(F)
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, P)
    Fo = F.cpu().numpy()
    Sg = S.cpu().numpy()
    # the true linear residual, measured with the oracle's Jacobian
    assert np.linalg.norm(Jo @ Sg + Fo) <= 1e-10 * np.linalg.norm(Fo)
    import scipy.sparse.linalg as spla
    So = spla.spsolve(Jo.tocsc(), -Fo)
    assert np.linalg.norm(Sg - So) <= 1e-8 * np.linalg.norm(So)
    assert 1 <= its < 60


def _rel_l2(u, v, uo, vo):
    return math.sqrt(np.sum((u - uo) ** 2 + (v - vo) ** 2) / np.sum(uo ** 2 + vo ** 2))


def test_ten_fixed_steps_periodic64_match_oracle():
    """The 64x64 periodic workload: 10 steps at dt = 1e-3, 2x2 subdomains, overlap 1.
    Tight tolerances on both sides so that the per-step error measures the roots."""
    shape = (64, 64)
    u0, v0 = random_ic(shape, 0)
    P = prob("periodic")
    s = solver(u0, v0, "periodic", sub=(2, 2), overlap=1, dt_fixed=1e-3, newton_rtol=1e-12,
               newton_atol=1e-13, gmres_rtol=1e-12)
    run = controller.Run(P, u0.copy(), v0.copy(), adaptive=False, dt_fixed=1e-3,
                         newton=newton.NewtonOptions(rtol=1e-12, atol=1e-13))
    M0 = scheme.mass(u0, P)
    for k in range(10):
        info = s.step(1)[0]
        rec = run.step()
        ug, vg = s.fields()
        err = _rel_l2(ug, vg, run.u, run.v)
        assert err <= 1e-10, (k, err)
        assert abs(info["mass"] - M0) <= 1e-12 * M0
        assert abs(info["energy"] - rec.energy) <= 1e-10 * abs(rec.energy)
        # the same Newton path: every step takes as many Newton iterations as the oracle's
        assert info["newton_its"] == rec.newton_its, (k, info["newton_its"], rec.newton_its)


def test_ten_fixed_steps_default_tolerance_error_is_reported():
    """The same workload at the benchmark's Newton tolerance 1e-8: the per-step
    difference to the tight oracle root stays at the tolerance level."""
    shape = (64, 64)
    u0, v0 = random_ic(shape, 0)
    P = prob("periodic")
    s = solver(u0, v0, "periodic", sub=(2, 2), overlap=1, dt_fixed=1e-3)
    run = controller.Run(P, u0.copy(), v0.copy(), adaptive=False, dt_fixed=1e-3,
                         newton=newton.NewtonOptions(rtol=1e-12, atol=1e-13))
    run8 = controller.Run(P, u0.copy(), v0.copy(), adaptive=False, dt_fixed=1e-3,
                          newton=newton.NewtonOptions(rtol=1e-8, atol=1e-13))
    M0 = scheme.mass(u0, P)
    for k in range(10):
        info = s.step(1)[0]
        run.step()
        rec8 = run8.step()
        ug, vg = s.fields()
        assert _rel_l2(ug, vg, run.u, run.v) <= 1e-7
        assert abs(info["mass"] - M0) <= 1e-12 * M0
        # Newton iterations at the benchmark tolerance: the oracle's count at the same
        # tolerance (its linear solves are exact, the GPU's stop at xi_r = 1e-8)
        assert info["newton_its"] == rec8.newton_its, (k, info["newton_its"], rec8.newton_its)


def test_adaptive_neumann_steps_match_oracle():
    """Adaptive dt (eq. sencondt) on a Neumann grid: dt sequence and fields agree."""
    shape = (40, 48)
    u0, v0 = random_ic(shape, 5)
    P = prob("neumann")
    kw = dict(adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1.0)
    s = solver(u0, v0, "neumann", sub=(2, 3), overlap=2, newton_rtol=1e-12, newton_atol=1e-13,
               gmres_rtol=1e-12, **kw)
    run = controller.Run(P, u0.copy(), v0.copy(), adaptive=True, dt_min=1e-4, dt_max=1e-1, eta=1.0,
                         newton=newton.NewtonOptions(rtol=1e-12, atol=1e-13))
    for k in range(8):
        info = s.step(1)[0]
        rec = run.step()
        assert abs(info["dt"] - rec.dt) <= 1e-9 * rec.dt, (k, info["dt"], rec.dt)
        ug, vg = s.fields()
        assert _rel_l2(ug, vg, run.u, run.v) <= 1e-10
    assert run.history[-1].dt > 2e-4   # dt left dt_min


def test_periodic512_sampled_residual_and_root():
    """At the full 512x512 size: the residual kernel at sampled cells against the
    loop oracle, and one Newton solve whose root the vectorised oracle confirms."""
    shape = (512, 512)
    u0, v0 = random_ic(shape, 0)
    P = prob("periodic")
    s = solver(u0, v0, "periodic", sub=(8, 8), overlap=2, dt_fixed=1e-4, newton_rtol=1e-10, ilu_shift=0.02)
    rng = np.random.default_rng(99)
    u1 = u0 + 0.01 * rng.uniform(-1, 1, shape)
    v1 = v0 + 0.01 * rng.uniform(-1, 1, shape)
    F, _, _ = s.residual(dev(vec(u1, v1)), dev(vec(u0, v0)), 1e-4)
    Fg = F.cpu().numpy()
    n = u0.size
    for _ in range(40):
        y, x = int(rng.integers(512)), int(rng.integers(512))
        fu, fv = scalar.residual_at(u1, v1, u0, v0, 1e-4, P, (y, x))
        assert abs(Fg[y * 512 + x] - fu) <= 1e-12 * max(1.0, abs(fu)) * 1e3
        assert abs(Fg[n + y * 512 + x] - fv) <= 1e-12 * max(1.0, abs(fv)) * 1e3
    info = s.solve_step(1e-4)
    ug, vg = s.fields()
    Fu, Fv = scheme.residual(ug, vg, u0, v0, 1e-4, P)
    F0u, F0v = scheme.residual(u0, v0, u0, v0, 1e-4, P)
    f0 = math.sqrt(np.sum(F0u ** 2 + F0v ** 2))
    assert math.sqrt(np.sum(Fu ** 2 + Fv ** 2)) <= 1e-9 * f0
    assert abs(scheme.mass(ug, P) - scheme.mass(u0, P)) <= 1e-12 * scheme.mass(u0, P)
    assert scheme.energy(ug, vg, P) < scheme.energy(u0, v0, P)


def test_timing_modes_count_launches():
    """acch_timing: 1 times every launch of every class; 2 times one Schwarz launch in 16
    and nothing else, and does not change the result."""
    shape = (64, 64)
    u0, v0 = random_ic(shape, 3)
    out = {}
    for mode in (1, 2):
        s = solver(u0, v0, "periodic", sub=(2, 2), overlap=1, dt_fixed=1e-3)
        s.timing(mode)
        s.step(2)
        st = s.kernel_stats()
        out[mode] = (st, s.fields())
        s.close()
    full, sampled = out[1][0], out[2][0]
    n_ras = full["ras"][1]
    assert n_ras > 16 and full["spmv_dots"][1] > 0 and full["residual"][1] > 0
    assert sampled["ras"][1] == (n_ras + 15) // 16 and sampled["ras"][0] > 0
    assert all(v[1] == 0 for k, v in sampled.items() if k != "ras")
    for a, b in zip(out[1][1], out[2][1]):
        assert np.array_equal(a, b)


def test_errors_are_reported():
    shape = (16, 16)
    u0, v0 = random_ic(shape, 1)
    from paper_2007_04560_amd import AcchError
    bad = u0.copy()
    bad[0, 0] = 1.5
    with pytest.raises(AcchError) as e:
        solver(bad, v0, "periodic", sub=(2, 2), overlap=1)
    assert e.value.code == 2
    s = solver(u0, v0, "periodic", sub=(2, 2), overlap=1, dt_fixed=1e-3, newton_max_it=1, newton_rtol=1e-300,
               newton_atol=1e-300)
    with pytest.raises(AcchError) as e:
        s.step(1)
    assert e.value.code == 3
    ug, vg = s.fields()
    assert np.array_equal(ug, u0) and np.array_equal(vg, v0)


def test_wide_boxes_use_two_waves_and_match_oracle():
    """Boxes wider than 127 cells run the two-wave solve (lane hand-over through LDS)."""
    shape = (40, 262)
    u1, v1, u0, v0 = perturbed_pair(shape, 51, amp=0.03)
    P = prob("neumann")
    dt = 2e-4
    s = solver(u0, v0, "neumann", sub=(2, 1), overlap=2, ilu_shift=0.02)
    assert s.info()["box_w"] > 127
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    s.factor()
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, P)
    r = np.random.default_rng(8).standard_normal(2 * u1.size)
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (1, 2), 2, "neumann", kind="left", shift=0.02).apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))


@pytest.mark.parametrize("shape,bc,sub,ov,rows", [((140, 60), "neumann", (1, 2), 2, 64),
                                                   ((150, 60), "periodic", (2, 2), 2, 64),
                                                   ((270, 40), "neumann", (1, 2), 2, 128)])
def test_tall_boxes_switch_lane_rows_and_match_oracle(shape, bc, sub, ov, rows):
    """Boxes taller than the sweep's lanes (64 per wave): lane t takes row t and later
    row t + 64 NW, switching between two loop iterations of each sweep; M^{-1} against
    the oracle, M^{-T} through the adjoint identity."""
    u1, v1, u0, v0 = perturbed_pair(shape, 57, amp=0.03)
    P = prob(bc)
    dt = 5e-5   # a step size whose ILU(0) factors stay well scaled on these long boxes
    s = solver(u0, v0, bc, sub=sub, overlap=ov, ilu_shift=0.02)
    info = s.info()
    assert rows < info["box_h"] <= 2 * rows
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    s.factor()
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, P)
    rng = np.random.default_rng(9)
    r = rng.standard_normal(2 * u1.size)
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", shift=0.02).apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))
    a = dev(rng.standard_normal(2 * u1.size))
    b = dev(rng.standard_normal(2 * u1.size))
    lhs = float(torch.dot(s.precondition_transpose(a), b))
    rhs = float(torch.dot(a, s.precondition(b)))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


@pytest.mark.parametrize("shape,bc,sub,ov", [((64, 64), "periodic", (2, 2), 1), ((45, 100), "neumann", (3, 2), 2)])
def test_mixed_precision_preconditioner_close_to_fp64(shape, bc, sub, ov):
    """FP32 factors and solves: the preconditioner output is the FP64 one to FP32 accuracy."""
    u1, v1, u0, v0 = perturbed_pair(shape, 61, amp=0.03)
    P = prob(bc)
    dt = 1e-3
    out = {}
    for prec in ["fp64", "mixed"]:
        s = solver(u0, v0, bc, sub=sub, overlap=ov, ilu_shift=0.02, precision=prec)
        s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
        s.factor()
        r = np.random.default_rng(9).standard_normal(2 * u1.size)
        out[prec] = s.precondition(dev(r)).cpu().numpy()
    rel = np.max(np.abs(out["mixed"] - out["fp64"])) / np.max(np.abs(out["fp64"]))
    assert 1e-9 < rel < 1e-4


def test_mixed_precision_steps_match_fp64_oracle():
    """The FP32 preconditioner changes the iteration, not the root: 10 steps of the 64x64
    periodic workload in mixed precision match the FP64 oracle to 1e-10 per step."""
    shape = (64, 64)
    u0, v0 = random_ic(shape, 0)
    P = prob("periodic")
    s = solver(u0, v0, "periodic", sub=(2, 2), overlap=1, dt_fixed=1e-3, newton_rtol=1e-12,
               newton_atol=1e-13, gmres_rtol=1e-12, precision="mixed")
    run = controller.Run(P, u0.copy(), v0.copy(), adaptive=False, dt_fixed=1e-3,
                         newton=newton.NewtonOptions(rtol=1e-12, atol=1e-13))
    M0 = scheme.mass(u0, P)
    for k in range(10):
        info = s.step(1)[0]
        run.step()
        ug, vg = s.fields()
        assert _rel_l2(ug, vg, run.u, run.v) <= 1e-10, k
        assert abs(info["mass"] - M0) <= 1e-12 * M0


def test_zero_filled_params_through_the_c_abi():
    """A C caller that fills only the problem fields and zero-fills the rest gets the
    documented defaults: mass projection on (drift <= 1e-12), energy logged every step,
    factors reused; the steps match the oracle."""
    import ctypes
    import paper_2007_04560_amd as pkg
    lib = pkg.load_library()
    shape = (48, 40)
    u0, v0 = random_ic(shape, 3)
    p = pkg.Params()
    p.dim, p.n[0], p.n[1], p.bc = 2, shape[1], shape[0], 0
    p.alpha, p.beta, p.theta, p.gamma, p.rho = 1.2, 1.2, 0.1, 1e-3, 1.0
    p.dt_fixed, p.sub[0], p.sub[1], p.overlap = 1e-3, 2, 2, 1
    nb = ctypes.c_size_t()
    assert lib.acch_workspace_bytes(ctypes.byref(p), ctypes.byref(nb)) == 0
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    p.workspace = (ws.data_ptr() + 255) // 256 * 256
    p.workspace_bytes = nb.value
    p.stream = torch.cuda.current_stream().cuda_stream
    ctx = ctypes.c_void_p()
    uc, vc = np.ascontiguousarray(u0), np.ascontiguousarray(v0)
    assert lib.acch_create(ctypes.byref(p), uc.ctypes.data, vc.ctypes.data, ctypes.byref(ctx)) == 0
    try:
        info = (pkg.StepInfo * 4)()
        acc = ctypes.c_int()
        assert lib.acch_step(ctx, 4, info, ctypes.byref(acc)) == 0 and acc.value == 4
        P = prob("periodic")
        M0 = scheme.mass(u0, P)
        run = controller.Run(P, u0.copy(), v0.copy(), adaptive=False, dt_fixed=1e-3)
        for k in range(4):
            rec = run.step()
            assert math.isfinite(info[k].energy)
            assert abs(info[k].energy - rec.energy) <= 1e-7 * abs(rec.energy)
            assert abs(info[k].mass - M0) <= 1e-12 * M0
        ug, vg = np.empty(shape), np.empty(shape)
        assert lib.acch_get_fields(ctx, ug.ctypes.data, vg.ctypes.data) == 0
        assert _rel_l2(ug, vg, run.u, run.v) <= 1e-7
    finally:
        lib.acch_destroy(ctx)


def _oracle_root_check(ug, vg, up, vp, dt, P, tol):
    """The oracle residual at a GPU root, relative to the residual at the step's start."""
    Fu, Fv = scheme.residual(ug, vg, up, vp, dt, P)
    F0u, F0v = scheme.residual(up, vp, up, vp, dt, P)
    f1 = math.sqrt(np.sum(Fu ** 2 + Fv ** 2))
    f0 = math.sqrt(np.sum(F0u ** 2 + F0v ** 2))
    assert f1 <= tol * f0, (f1, f0)


def test_periodic512_workload_roots_at_sampled_steps():
    """The 512x512 periodic workload as the benchmark runs it (adaptive, tolerance 1e-8):
    at steps 1, 25 and 60 the oracle's residual of the GPU's new state, taken with the
    step's dt and the GPU's previous state, is at the Newton tolerance; mass is exact and
    the energy decreases."""
    shape = (512, 512)
    u0, v0 = random_ic(shape, 0)
    P = prob("periodic")
    s = solver(u0, v0, "periodic", sub=(8, 8), overlap=2, adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1e4,
               ilu_shift=0.02)
    M0 = scheme.mass(u0, P)
    done = 0
    for k in (1, 25, 60):
        if k - 1 > done:
            s.step(k - 1 - done)
        up, vp = s.fields()
        info = s.step(1)[0]
        done = k
        ug, vg = s.fields()
        _oracle_root_check(ug, vg, up, vp, info["dt"], P, 2e-8)
        assert abs(scheme.mass(ug, P) - M0) <= 1e-12 * M0
        assert scheme.energy(ug, vg, P) < scheme.energy(up, vp, P)


def test_neumann2048_setup_at_256_mixed():
    """The 2048^2 Neumann configuration's setup (FP32 subdomain factors and solves, 16x16
    subdomains, overlap 2, adaptive dt in [1e-4, 1e-1]) on the 256^2 grid where it
    converges, at the configuration's tolerance 1e-8: three steps whose mixed-precision
    roots the oracle's residual confirms, equal to the FP64 GPU run's roots to 1e-7 per
    step, with exact mass.  Neumann boxes need the larger shift 0.05 (with 0.02 the ILU(0)
    pivots of the boundary boxes change sign and GMRES stalls)."""
    shape = (256, 256)
    u0, v0 = random_ic(shape, 0)
    P = prob("neumann")
    kw = dict(sub=(16, 16), overlap=2, adaptive=True, dt_min=1e-4, dt_max=1e-1, eta0=1e4, ilu_shift=0.05,
              gmres_max_restarts=30)
    sm = solver(u0, v0, "neumann", precision="mixed", **kw)
    sd = solver(u0, v0, "neumann", precision="fp64", **kw)
    M0 = scheme.mass(u0, P)
    up, vp = u0, v0
    for k in range(3):
        im = sm.step(1)[0]
        idd = sd.step(1)[0]
        assert im["dt"] == idd["dt"]
        um, vm = sm.fields()
        ud, vd = sd.fields()
        _oracle_root_check(um, vm, up, vp, im["dt"], P, 2e-8)
        assert _rel_l2(um, vm, ud, vd) <= 1e-7
        assert abs(scheme.mass(um, P) - M0) <= 1e-12 * M0
        up, vp = um, vm
