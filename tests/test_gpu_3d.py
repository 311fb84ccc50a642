"""GPU parity of the 3D path (residual, energy, 40-slot Jacobian and its products,
3D subdomain ILU(0) / Schwarz and its transpose, whole steps, the adjoint step)
against the FP64 oracle, which is written for any dimension."""
import numpy as np
import pytest

from acch_inputs import perturbed_pair, random_ic
from oracle import adjoint as oadj
from oracle import controller, jacobian, newton, schwarz, scheme
from oracle.params import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2007_04560_amd import Solver, set_option  # noqa: E402

L3 = (1.0, 0.9, 1.1)
CASES = [((9, 10, 11), "periodic", (2, 2, 2), 1), ((8, 10, 12), "neumann", (2, 2, 3), 1),
         ((10, 9, 11), "neumann", (1, 2, 2), 2)]


def vec(u, v):
    return np.concatenate([u.ravel(), v.ravel()])


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def solver(u0, v0, bc, sub, ov, **kw):
    return Solver(u0, v0, bc=bc, L=L3, sub=sub, overlap=ov, **kw)


@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
def test_residual_energy_3d_match_oracle(shape, bc, sub, ov):
    u1, v1, u0, v0 = perturbed_pair(shape, 71, amp=0.03)
    P = Problem(bc=bc, lengths=L3)
    s = solver(u0, v0, bc, sub, ov)
    F, f2, bad = s.residual(dev(vec(u1, v1)), dev(vec(u0, v0)), 2e-3)
    Fu, Fv = scheme.residual(u1, v1, u0, v0, 2e-3, P)
    assert rel(F.cpu().numpy(), vec(Fu, Fv)) <= 1e-12
    assert bad == 0
    E, M = s.energy()
    assert abs(E - scheme.energy(u0, v0, P)) <= 1e-13 * abs(scheme.energy(u0, v0, P))
    assert abs(M - scheme.mass(u0, P)) <= 1e-14 * scheme.mass(u0, P)


@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
@pytest.mark.parametrize("mob", ["midpoint", "explicit"])
def test_jacobian_3d_products_match_oracle(shape, bc, sub, ov, mob):
    u1, v1, u0, v0 = perturbed_pair(shape, 72, amp=0.03)
    P = Problem(bc=bc, lengths=L3, mobility=mob)
    s = solver(u0, v0, bc, sub, ov, mobility=mob)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), 2e-3)
    Jo = jacobian.jacobian(u1, v1, u0, v0, 2e-3, P)
    x = np.random.default_rng(5).standard_normal(2 * u1.size)
    assert rel(s.apply_jacobian(dev(x)).cpu().numpy(), Jo @ x) <= 1e-12
    assert rel(s.apply_jacobian_transpose(dev(x)).cpu().numpy(), Jo.T @ x) <= 1e-12


@pytest.fixture(params=[1, 0], ids=["window", "boxbuffer"])
def window(request):
    """Both forms of the 3D apply: LDS window and whole box in device memory."""
    set_option("ras3d_window", request.param)
    yield request.param
    set_option("ras3d_window", 1)


@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_schwarz_3d_matches_oracle(shape, bc, sub, ov, precision, window):
    u1, v1, u0, v0 = perturbed_pair(shape, 73, amp=0.03)
    P = Problem(bc=bc, lengths=L3)
    s = solver(u0, v0, bc, sub, ov, ilu_shift=0.02, precision=precision)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), 2e-3)
    s.factor()
    Jo = jacobian.jacobian(u1, v1, u0, v0, 2e-3, P)
    Pc = schwarz.Schwarz(Jo, shape, (sub[2], sub[1], sub[0]), ov, bc, kind="left", shift=0.02)
    r = np.random.default_rng(6).standard_normal(2 * u1.size)
    z = s.precondition(dev(r)).cpu().numpy()
    zo = Pc.apply(r)
    assert rel(z, zo) <= (1e-10 if precision == "fp64" else 1e-4)
    # the transpose: <M^{-T} a, b> = <a, M^{-1} b>
    a = dev(np.random.default_rng(7).standard_normal(2 * u1.size))
    lhs = float(torch.dot(s.precondition_transpose(a), dev(r)))
    rhs = float(torch.dot(a, dev(z)))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_transpose_3d_is_the_transpose_of_the_oracle_operator():
    shape, bc, sub, ov = (4, 5, 6), "neumann", (2, 2, 1), 1
    u1, v1, u0, v0 = perturbed_pair(shape, 74, amp=0.03)
    s = solver(u0, v0, bc, sub, ov, ilu_shift=0.02)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), 2e-3)
    s.factor()
    Jo = jacobian.jacobian(u1, v1, u0, v0, 2e-3, Problem(bc=bc, lengths=L3))
    Pc = schwarz.Schwarz(Jo, shape, (sub[2], sub[1], sub[0]), ov, bc, kind="left", shift=0.02)
    n2 = 2 * u1.size
    Minv = np.column_stack([Pc.apply(np.eye(n2)[:, k]) for k in range(n2)])
    r = np.random.default_rng(8).standard_normal(n2)
    assert rel(s.precondition_transpose(dev(r)).cpu().numpy(), Minv.T @ r) <= 1e-10


@pytest.mark.parametrize("bc", ["neumann", "periodic"])
def test_steps_3d_match_oracle(bc, window):
    shape = (8, 9, 10) if bc == "neumann" else (9, 9, 10)
    sub = (2, 2, 2)
    u0, v0 = random_ic(shape, 75)
    s = solver(u0, v0, bc, sub, 1, dt_fixed=1e-3, ilu_shift=0.02, newton_rtol=1e-12, newton_atol=1e-13,
               gmres_rtol=1e-13, gmres_atol=1e-15, gmres_max_restarts=30)
    recs = s.step(3)
    run = controller.Run(Problem(bc=bc, lengths=L3), u0, v0, adaptive=False, dt_fixed=1e-3,
                         newton=newton.NewtonOptions(rtol=1e-12, atol=1e-11))
    for _ in range(3):
        run.step()
    u, v = s.fields()
    ref = vec(run.u, run.v)
    assert np.linalg.norm(vec(u, v) - ref) <= 1e-10 * np.linalg.norm(ref)
    assert abs(recs[-1]["mass"] - recs[0]["mass"]) <= 1e-12 * recs[0]["mass"]


def test_adjoint_step_and_energy_gradient_3d_match_oracle():
    shape, bc = (6, 7, 8), "neumann"
    u1, v1, u0, v0 = perturbed_pair(shape, 76, amp=0.03)
    P = Problem(bc=bc, lengths=L3)
    s = solver(u0, v0, bc, (2, 2, 2), 1, ilu_shift=0.02, gmres_rtol=1e-13, gmres_max_restarts=30)
    g1 = np.random.default_rng(9).standard_normal(2 * u1.size)
    gprev, dp, its, _ = s.adjoint_step(dev(vec(u1, v1)), dev(vec(u0, v0)), 2e-3, dev(g1))
    g0o, _, dpo = oadj.adjoint_step(u1, v1, u0, v0, 2e-3, P, g1)
    assert rel(gprev.cpu().numpy(), g0o) <= 1e-9
    for k, name in enumerate(oadj.PARAMS):
        assert abs(dp[k] - dpo[name]) <= 1e-9 * max(abs(dpo[name]), 1e-3 * np.max(np.abs(g0o))), name
    g, dpe = s.energy_gradient()
    gu, gv, gp = oadj.energy_gradient(u0, v0, P)
    assert rel(g.cpu().numpy(), vec(gu, gv)) <= 1e-12
    for k, name in enumerate(oadj.PARAMS):
        assert abs(dpe[k] - gp[name]) <= 1e-12 * abs(gp[name]), name


def test_final_energy_gradient_3d_matches_central_differences():
    """d(final energy)/d(v0, theta, gamma) on 16^3 through 4 fixed steps with one
    recomputed checkpoint segment, against central differences of the GPU forward."""
    from paper_2007_04560_amd.adjoint import final_energy
    shape = (16, 16, 16)
    u0, v0 = random_ic(shape, 77)
    kw = dict(bc="neumann", L=L3, sub=(2, 2, 2), overlap=1, adaptive=False, dt_fixed=2e-3, ilu_shift=0.02,
              newton_rtol=1e-12, newton_atol=1e-13, gmres_rtol=1e-13, gmres_atol=1e-15, gmres_max_restarts=30)
    p0 = np.array([1.2, 1.2, 0.1, 1e-3])
    nsteps = 4

    def energy(u, v, p):
        with Solver(u, v, **dict(zip(("alpha", "beta", "theta", "gamma"), p)), **kw) as s:
            s.step(nsteps)
            return s.energy()[0]

    params = torch.tensor(p0, requires_grad=True)
    tu = torch.tensor(u0, requires_grad=True)
    tv = torch.tensor(v0, requires_grad=True)
    E = final_energy(tu, tv, params, nsteps, checkpoint_every=2, **kw)
    E.backward()
    for k in (2, 3):
        h = 1e-6 * p0[k]
        pp, pm = p0.copy(), p0.copy()
        pp[k] += h
        pm[k] -= h
        fd = (energy(u0, v0, pp) - energy(u0, v0, pm)) / (2 * h)
        assert abs(float(params.grad[k]) - fd) <= 1e-6 * abs(fd), (k, float(params.grad[k]), fd)
    d = np.random.default_rng(12).uniform(-1, 1, shape)
    eps = 1e-5
    fd = (energy(u0, v0 + eps * d, p0) - energy(u0, v0 - eps * d, p0)) / (2 * eps)
    assert abs(float((tv.grad * torch.tensor(d)).sum()) - fd) <= 1e-6 * abs(fd)


def test_window_and_box_buffer_applies_agree_at_full_box_size(window):
    """A 34^3 box (32^3 with overlap 1, as in a 4x4x4 split of 128^3), about the largest
    the LDS window takes: both applies agree with each other on the same factors."""
    shape = (32, 32, 32)
    u1, v1, u0, v0 = perturbed_pair(shape, 78, amp=0.03)
    s = solver(u0, v0, "neumann", (1, 1, 1), 1, ilu_shift=0.02)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), 2e-3)
    s.factor()
    r = dev(np.random.default_rng(13).standard_normal(2 * u1.size))
    z = s.precondition(r).cpu().numpy()
    set_option("ras3d_window", 1 - window)
    z2 = s.precondition(r).cpu().numpy()
    assert rel(z, z2) <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-4)])
def test_window_apply_on_workload_sized_boxes_matches_oracle(precision, tol):
    """Boxes of 18^3 cells (16^3 owned, overlap 1): the box of the 128^3 workload's
    8x8x8 split, on a 32^3 grid split 2x2x2.  M^{-1} r of the windowed apply against the
    oracle's left-RAS with shifted ILU(0) on the same boxes."""
    shape = (32, 32, 32)
    u1, v1, u0, v0 = perturbed_pair(shape, 79, amp=0.03)
    s = Solver(u0, v0, bc="neumann", sub=(2, 2, 2), overlap=1, ilu_shift=0.02, precision=precision)
    assert s.info()["box_w"] == 18
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), 2e-3)
    s.factor()
    r = np.random.default_rng(14).standard_normal(2 * u1.size)
    z = s.precondition(dev(r)).cpu().numpy()
    Jo = jacobian.jacobian(u1, v1, u0, v0, 2e-3, Problem(bc="neumann", lengths=(1.0, 1.0, 1.0)))
    zo = schwarz.Schwarz(Jo, shape, (2, 2, 2), 1, "neumann", kind="left", shift=0.02).apply(r)
    if precision == "fp64":
        assert rel(z, zo) <= tol
    else:
        assert np.linalg.norm(z - zo) <= tol * np.linalg.norm(zo)


def test_neumann128_3d_first_newton_solve_root():
    """The 128^3 workload's first time step (dt_min = 1e-4, 8x8x8 subdomains, overlap 1):
    the GPU's Newton root leaves an oracle residual below 1e-9 of the initial one, and the
    mass of u is unchanged to 1e-12."""
    shape = (128, 128, 128)
    u0, v0 = random_ic(shape, 0)
    P = Problem(bc="neumann", lengths=(1.0, 1.0, 1.0))
    with Solver(u0, v0, bc="neumann", sub=(8, 8, 8), overlap=1, ilu_shift=0.02, newton_rtol=1e-11,
                gmres_rtol=1e-10) as s:
        info = s.solve_step(1e-4)
        ug, vg = s.fields()
    F0u, F0v = scheme.residual(u0, v0, u0, v0, 1e-4, P)
    Fu, Fv = scheme.residual(ug, vg, u0, v0, 1e-4, P)
    f0 = np.sqrt(np.sum(F0u ** 2) + np.sum(F0v ** 2))
    f1 = np.sqrt(np.sum(Fu ** 2) + np.sum(Fv ** 2))
    assert f1 <= 1e-9 * f0, (f1, f0, info)
    M0, M1 = scheme.mass(u0, P), scheme.mass(ug, P)
    assert abs(M1 - M0) <= 1e-12 * M0
    assert info["newton_its"] >= 2
