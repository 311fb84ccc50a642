"""GPU parity of the discrete adjoint (transposed Jacobian product, transposed
Schwarz operator, the step-back of the dt-frozen step map, the energy gradient and
the checkpointed autograd wrapper) against the FP64 oracle and against central
differences of the GPU forward run."""
import numpy as np
import pytest

from acch_inputs import perturbed_pair, random_ic
from oracle import adjoint as oadj
from oracle import jacobian, schwarz
from oracle.newton import NewtonOptions
from oracle.params import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2007_04560_amd import Solver  # noqa: E402
from paper_2007_04560_amd.adjoint import final_energy  # noqa: E402

PARAMS = ("alpha", "beta", "theta", "gamma")


def vec(u, v):
    return np.concatenate([u.ravel(), v.ravel()])


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("shape,bc,sub,ov", [((37, 29), "periodic", (2, 2), 1), ((45, 100), "neumann", (3, 2), 2)])
def test_jacobian_transpose_product_matches_oracle(shape, bc, sub, ov):
    u1, v1, u0, v0 = perturbed_pair(shape, 51, amp=0.03)
    dt = 2e-3
    s = Solver(u0, v0, bc=bc, sub=sub, overlap=ov)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    x = np.random.default_rng(3).standard_normal(2 * u1.size)
    y = s.apply_jacobian_transpose(dev(x)).cpu().numpy()
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, Problem(bc=bc))
    assert rel(y, Jo.T @ x) <= 1e-12


@pytest.mark.parametrize("shape,bc,sub,ov", [((12, 12), "periodic", (2, 2), 1), ((10, 14), "neumann", (2, 1), 2),
                                             ((9, 11), "neumann", (1, 1), 0)])
def test_preconditioner_transpose_is_the_transpose_of_the_oracle_operator(shape, bc, sub, ov):
    """M^{-T} r on the GPU against the transpose of the oracle's M^{-1}, formed column
    by column on a small grid."""
    u1, v1, u0, v0 = perturbed_pair(shape, 52, amp=0.03)
    dt = 5e-3
    s = Solver(u0, v0, bc=bc, sub=sub, overlap=ov, ilu_shift=0.02)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    s.factor()
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, Problem(bc=bc))
    Pc = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", shift=0.02)
    n2 = 2 * u1.size
    Minv = np.column_stack([Pc.apply(np.eye(n2)[:, k]) for k in range(n2)])
    r = np.random.default_rng(5).standard_normal(n2)
    z = s.precondition_transpose(dev(r)).cpu().numpy()
    assert rel(z, Minv.T @ r) <= 1e-10


@pytest.mark.parametrize("shape,bc,sub,ov", [((512, 512), "periodic", (8, 8), 2), ((300, 170), "neumann", (3, 2), 2),
                                             ((40, 262), "neumann", (2, 1), 2)])
def test_preconditioner_transpose_adjoint_identity(shape, bc, sub, ov):
    """<M^{-T} a, b> = <a, M^{-1} b> at full size (the forward operator is pinned to
    the oracle elsewhere).  The bound is rounding relative to |<z, b>| for sums
    whose operator norms reach 1e29 (ILU(0) growth on the large Neumann boxes)."""
    u1, v1, u0, v0 = perturbed_pair(shape, 53, amp=0.03)
    s = Solver(u0, v0, bc=bc, sub=sub, overlap=ov, ilu_shift=0.02)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), 1e-3)
    s.factor()
    rng = np.random.default_rng(6)
    a = dev(rng.standard_normal(2 * u1.size))
    b = dev(rng.standard_normal(2 * u1.size))
    lhs = float(torch.dot(s.precondition_transpose(a), b))
    rhs = float(torch.dot(a, s.precondition(b)))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


@pytest.mark.parametrize("bc,mob", [("periodic", "midpoint"), ("neumann", "average"), ("neumann", "explicit")])
def test_energy_gradient_matches_oracle(bc, mob):
    shape = (40, 56)
    u, v = random_ic(shape, 54)
    P = Problem(bc=bc, lengths=(1.0, 1.4), mobility=mob)
    s = Solver(u, v, bc=bc, L=(1.0, 1.4), mobility=mob, sub=(2, 2), overlap=1)
    g, dp = s.energy_gradient()
    gu, gv, gp = oadj.energy_gradient(u, v, P)
    assert rel(g.cpu().numpy(), vec(gu, gv)) <= 1e-12
    for k, name in enumerate(PARAMS):
        assert abs(dp[k] - gp[name]) <= 1e-12 * abs(gp[name]), name


@pytest.mark.parametrize("bc,mob,sub,ov", [("periodic", "midpoint", (2, 2), 1), ("neumann", "average", (3, 2), 2),
                                           ("neumann", "explicit", (2, 3), 1)])
def test_adjoint_step_matches_oracle(bc, mob, sub, ov):
    shape = (36, 30)
    u1, v1, u0, v0 = perturbed_pair(shape, 55, amp=0.03)
    dt = 2e-3
    P = Problem(bc=bc, mobility=mob)
    s = Solver(u0, v0, bc=bc, mobility=mob, sub=sub, overlap=ov, ilu_shift=0.02, gmres_rtol=1e-13,
               gmres_max_restarts=30)
    g1 = np.random.default_rng(8).standard_normal(2 * u1.size)
    gprev, dp, its, _ = s.adjoint_step(dev(vec(u1, v1)), dev(vec(u0, v0)), dt, dev(g1))
    g0o, _, dpo = oadj.adjoint_step(u1, v1, u0, v0, dt, P, g1)
    assert its > 0
    assert rel(gprev.cpu().numpy(), g0o) <= 1e-9
    for k, name in enumerate(PARAMS):
        assert abs(dp[k] - dpo[name]) <= 1e-9 * max(abs(dpo[name]), 1e-3 * np.max(np.abs(g0o))), name


def _tight(**kw):
    base = dict(newton_rtol=1e-12, newton_atol=1e-13, gmres_rtol=1e-13, gmres_atol=1e-15, gmres_max_restarts=30,
                ilu_shift=0.02)
    base.update(kw)
    return base


def test_final_energy_gradient_matches_oracle_adjoint():
    """Autograd through 7 adaptive steps (checkpoints every 3: three recomputed
    segments) against the oracle's adjoint with the same step sizes."""
    shape = (24, 24)
    u0, v0 = random_ic(shape, 56)
    kw = _tight(bc="periodic", sub=(2, 2), overlap=1, adaptive=True, dt_min=1e-4, dt_max=2e-3, eta0=1e-4)
    params = torch.tensor([1.2, 1.2, 0.1, 1e-3], dtype=torch.float64, requires_grad=True)
    tu = torch.tensor(u0, requires_grad=True)
    tv = torch.tensor(v0, requires_grad=True)
    E = final_energy(tu, tv, params, 7, checkpoint_every=3, **kw)
    E.backward()
    with Solver(u0, v0, alpha=1.2, beta=1.2, theta=0.1, gamma=1e-3, **kw) as s:
        dts = [r["dt"] for r in s.step(7)]
    assert len(set(dts)) > 1   # the controller did change dt
    P = Problem(bc="periodic")
    Eo, gu, gv, gp = oadj.gradient(u0, v0, dts, P, NewtonOptions(rtol=1e-12, atol=1e-11))
    assert abs(float(E.detach()) - Eo) <= 1e-10 * abs(Eo)
    assert rel(tu.grad.numpy(), gu) <= 1e-7
    assert rel(tv.grad.numpy(), gv) <= 1e-7
    for k, name in enumerate(PARAMS):
        assert abs(float(params.grad[k]) - gp[name]) <= 1e-7 * abs(gp[name]), name


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_final_energy_gradient_matches_central_differences(precision):
    """Fixed dt (so the step map is the one differentiated): directional derivatives
    in v0 and u0 and the four parameter derivatives against central differences of
    the GPU forward run, relative error <= 1e-6."""
    shape = (20, 16)
    u0, v0 = random_ic(shape, 57)
    kw = _tight(bc="neumann", sub=(2, 2), overlap=1, adaptive=False, dt_fixed=2e-3, precision=precision)
    p0 = np.array([1.2, 1.2, 0.1, 2e-3])
    nsteps = 6

    def energy(u, v, p):
        with Solver(u, v, **dict(zip(PARAMS, p)), **kw) as s:
            s.step(nsteps)
            return s.energy()[0]

    params = torch.tensor(p0, requires_grad=True)
    tu = torch.tensor(u0, requires_grad=True)
    tv = torch.tensor(v0, requires_grad=True)
    E = final_energy(tu, tv, params, nsteps, checkpoint_every=5, **kw)
    E.backward()
    for k, name in enumerate(PARAMS):
        h = 1e-6 * p0[k]
        pp, pm = p0.copy(), p0.copy()
        pp[k] += h
        pm[k] -= h
        fd = (energy(u0, v0, pp) - energy(u0, v0, pm)) / (2 * h)
        assert abs(float(params.grad[k]) - fd) <= 1e-6 * abs(fd), (name, float(params.grad[k]), fd)
    d = np.random.default_rng(9).uniform(-1, 1, shape)
    eps = 1e-5
    fd = (energy(u0, v0 + eps * d, p0) - energy(u0, v0 - eps * d, p0)) / (2 * eps)
    assert abs(float((tv.grad * torch.tensor(d)).sum()) - fd) <= 1e-6 * abs(fd)
    fd = (energy(u0 + eps * d, v0, p0) - energy(u0 - eps * d, v0, p0)) / (2 * eps)
    assert abs(float((tu.grad * torch.tensor(d)).sum()) - fd) <= 1e-6 * abs(fd)
