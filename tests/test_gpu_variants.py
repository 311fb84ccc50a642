"""GPU parity of the Schwarz variants (Section 3.1, left- and right-restricted and
classical additive Schwarz): the preconditioner, its transpose and whole steps
against the FP64 oracle."""
import numpy as np
import pytest

from acch_inputs import perturbed_pair, random_ic
from oracle import controller, jacobian, newton, schwarz
from oracle.params import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2007_04560_amd import AcchError, Solver  # noqa: E402

KINDS = ["left", "right", "classical"]
CASES = [((37, 29), "periodic", (2, 2), 1), ((45, 100), "neumann", (3, 2), 2), ((64, 64), "periodic", (4, 2), 2)]


def vec(u, v):
    return np.concatenate([u.ravel(), v.ravel()])


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_variant_preconditioner_matches_oracle(kind, shape, bc, sub, ov, precision):
    u1, v1, u0, v0 = perturbed_pair(shape, 61, amp=0.03)
    dt = 5e-3
    s = Solver(u0, v0, bc=bc, sub=sub, overlap=ov, ilu_shift=0.02, schwarz=kind, precision=precision)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    s.factor()
    r = np.random.default_rng(9).standard_normal(2 * u1.size)
    z = s.precondition(dev(r)).cpu().numpy()
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, Problem(bc=bc))
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind=kind, shift=0.02).apply(r)
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert np.max(np.abs(z - zo)) <= tol * np.max(np.abs(zo))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("shape,bc,sub,ov", [((12, 12), "periodic", (2, 2), 1), ((10, 14), "neumann", (2, 1), 2)])
def test_variant_transpose_is_the_transpose(kind, shape, bc, sub, ov):
    u1, v1, u0, v0 = perturbed_pair(shape, 62, amp=0.03)
    dt = 5e-3
    s = Solver(u0, v0, bc=bc, sub=sub, overlap=ov, ilu_shift=0.02, schwarz=kind)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    s.factor()
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, Problem(bc=bc))
    Pc = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind=kind, shift=0.02)
    n2 = 2 * u1.size
    Minv = np.column_stack([Pc.apply(np.eye(n2)[:, k]) for k in range(n2)])
    r = np.random.default_rng(10).standard_normal(n2)
    z = s.precondition_transpose(dev(r)).cpu().numpy()
    assert np.max(np.abs(z - Minv.T @ r)) <= 1e-10 * np.max(np.abs(Minv.T @ r))


@pytest.mark.parametrize("kind", ["right", "classical"])
def test_variant_steps_match_oracle(kind):
    shape = (40, 40)
    u0, v0 = random_ic(shape, 63)
    s = Solver(u0, v0, bc="periodic", sub=(2, 2), overlap=1, schwarz=kind, dt_fixed=1e-3, ilu_shift=0.02,
               newton_rtol=1e-12, newton_atol=1e-13, gmres_rtol=1e-13, gmres_atol=1e-15, gmres_max_restarts=30)
    recs = s.step(3)
    assert all(r["gmres_its"] > 0 for r in recs)
    run = controller.Run(Problem(bc="periodic"), u0, v0, adaptive=False, dt_fixed=1e-3,
                         newton=newton.NewtonOptions(rtol=1e-12, atol=1e-11))
    for _ in range(3):
        run.step()
    u, v = s.fields()
    ref = vec(run.u, run.v)
    assert np.linalg.norm(vec(u, v) - ref) <= 1e-10 * np.linalg.norm(ref)


def test_variant_needs_narrow_overlap():
    u0, v0 = random_ic((30, 30), 64)
    with pytest.raises(AcchError):
        Solver(u0, v0, bc="neumann", sub=(10, 10), overlap=4, schwarz="classical")


@pytest.mark.parametrize("shape,bc,sub", [((37, 29), "periodic", (2, 2)), ((45, 100), "neumann", (3, 2))])
def test_classical_without_overlap_matches_oracle(shape, bc, sub):
    """Classical AS with delta = 0 (Table 3's first column): non-overlapping boxes, each
    subdomain's ILU(0) solve added on its own cells."""
    u1, v1, u0, v0 = perturbed_pair(shape, 65, amp=0.03)
    s = Solver(u0, v0, bc=bc, sub=sub, overlap=0, ilu_shift=0.02, schwarz="classical")
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), 5e-3)
    s.factor()
    r = np.random.default_rng(11).standard_normal(2 * u1.size)
    z = s.precondition(dev(r)).cpu().numpy()
    Jo = jacobian.jacobian(u1, v1, u0, v0, 5e-3, Problem(bc=bc))
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), 0, bc, kind="classical", shift=0.02).apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))
    # with no overlap the three variants are one operator
    zl = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), 0, bc, kind="left", shift=0.02).apply(r)
    assert np.max(np.abs(zl - zo)) <= 1e-14 * np.max(np.abs(zo))


@pytest.mark.parametrize("shape,bc,sub,ov", [((9, 10, 11), "periodic", (2, 2, 2), 1),
                                             ((8, 10, 12), "neumann", (2, 2, 3), 1),
                                             ((10, 9, 11), "neumann", (1, 2, 2), 2),
                                             ((8, 10, 12), "neumann", (2, 2, 2), 0)])
@pytest.mark.parametrize("kind", ["right", "classical"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_variant_preconditioner_3d_matches_oracle(shape, bc, sub, ov, kind, precision):
    """The 3D right-restricted and classical variants (box sweeps, then the sum over the
    boxes of each cell) against the oracle."""
    L3 = (1.0, 0.9, 1.1)
    u1, v1, u0, v0 = perturbed_pair(shape, 66, amp=0.03)
    s = Solver(u0, v0, bc=bc, L=L3, sub=sub, overlap=ov, ilu_shift=0.02, schwarz=kind, precision=precision)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), 2e-3)
    s.factor()
    r = np.random.default_rng(12).standard_normal(2 * u1.size)
    z = s.precondition(dev(r)).cpu().numpy()
    Jo = jacobian.jacobian(u1, v1, u0, v0, 2e-3, Problem(bc=bc, lengths=L3))
    zo = schwarz.Schwarz(Jo, shape, (sub[2], sub[1], sub[0]), ov, bc, kind=kind, shift=0.02).apply(r)
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert np.max(np.abs(z - zo)) <= tol * np.max(np.abs(zo))


@pytest.mark.parametrize("kind", ["right", "classical"])
def test_variant_steps_3d_match_oracle(kind):
    shape, bc = (8, 9, 10), "neumann"
    L3 = (1.0, 0.9, 1.1)
    u0, v0 = random_ic(shape, 67)
    s = Solver(u0, v0, bc=bc, L=L3, sub=(2, 2, 2), overlap=1, schwarz=kind, dt_fixed=1e-3, ilu_shift=0.02,
               newton_rtol=1e-12, newton_atol=1e-13, gmres_rtol=1e-13, gmres_atol=1e-15, gmres_max_restarts=30)
    recs = s.step(3)
    run = controller.Run(Problem(bc=bc, lengths=L3), u0, v0, adaptive=False, dt_fixed=1e-3,
                         newton=newton.NewtonOptions(rtol=1e-12, atol=1e-11))
    for _ in range(3):
        run.step()
    u, v = s.fields()
    ref = vec(run.u, run.v)
    assert np.linalg.norm(vec(u, v) - ref) <= 1e-10 * np.linalg.norm(ref)
    assert abs(recs[-1]["mass"] - recs[0]["mass"]) <= 1e-12 * recs[0]["mass"]
    with pytest.raises(AcchError):
        s.precondition_transpose(dev(np.zeros(2 * u0.size)))
