"""The paper's long adaptive 2D run (Section 4.2: alpha 4, beta 2, gamma 5e-3, theta 0.1,
rho 1e-3, u0 = 0.55 + 0.05 U(-1,1), dt in [1e-4, 10], eta = 1e4) on small grids: the
first adaptive steps against the FP64 oracle, then a few hundred steps for the
properties the paper reports for it (monotone energy, conserved mass, dt leaving
dt_min)."""
import numpy as np
import pytest

from acch_inputs import random_ic
from oracle import controller, newton
from oracle.params import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2007_04560_amd import Solver  # noqa: E402

PHYS = dict(alpha=4.0, beta=2.0, gamma=0.005, theta=0.1, rho=0.001)
CTRL = dict(adaptive=True, dt_min=1e-4, dt_max=10.0, eta0=1e4)


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_long_run_first_steps_match_oracle(bc):
    shape = (24, 28)
    u0, v0 = random_ic(shape, 21, u_mean=0.55)
    s = Solver(u0, v0, bc=bc, sub=(2, 2), overlap=2, ilu_shift=0.02, newton_rtol=1e-12, newton_atol=1e-13,
               gmres_rtol=1e-12, gmres_atol=1e-15, gmres_max_restarts=30, **PHYS, **CTRL)
    run = controller.Run(Problem(bc=bc, **PHYS), u0.copy(), v0.copy(), adaptive=True, dt_min=1e-4, dt_max=10.0,
                         eta=1e4, newton=newton.NewtonOptions(rtol=1e-12, atol=1e-13))
    for k in range(6):
        info = s.step(1)[0]
        rec = run.step()
        assert abs(info["dt"] - rec.dt) <= 1e-9 * rec.dt, (k, info["dt"], rec.dt)
        u, v = s.fields()
        ref = np.concatenate([run.u.ravel(), run.v.ravel()])
        assert np.linalg.norm(np.concatenate([u.ravel(), v.ravel()]) - ref) <= 1e-10 * np.linalg.norm(ref), k


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_long_run_energy_mass_and_step_growth(bc):
    shape = (32, 32)
    u0, v0 = random_ic(shape, 22, u_mean=0.55)
    s = Solver(u0, v0, bc=bc, sub=(2, 2), overlap=2, ilu_shift=0.02, **PHYS, **CTRL)
    E0, M0 = s.energy()
    recs = []
    for _ in range(4):
        recs += s.step(100)
    E = [E0] + [r["energy"] for r in recs]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(E, E[1:])), "energy increased"
    assert all(abs(r["mass"] - M0) <= 1e-12 * M0 for r in recs)
    dts = [r["dt"] for r in recs]
    assert min(dts) >= 1e-4 * (1 - 1e-12) and max(dts) <= 10.0
    assert max(dts) > 4e-4, "dt never left dt_min"
    ts = [r["t"] for r in recs]
    assert all(b > a for a, b in zip(ts, ts[1:]))


def test_long_run_with_plain_box_pattern_ilu0_leaves_small_steps():
    """The 128x128 periodic long run (8x8 subdomains, overlap 1, the late-time tolerance
    eps_a = 1e-6) with plain (unshifted) ILU(0) on the box pattern: 2000 steps with the
    energy non-increasing and the mass conserved at every step, and dt growing past 1e-2.
    Over the same 2000 steps shifted ILU(0) on the stencil pattern stays at dt <= 1.2e-3:
    GMRES fails as dt grows, and every failure doubles eta."""
    shape = (128, 128)
    u0, v0 = random_ic(shape, 0, u_mean=0.55)
    s = Solver(u0, v0, bc="periodic", sub=(8, 8), overlap=1, subsolver="iluk_box", fill_level=0, ilu_shift=0.0,
               newton_atol=1e-6, **PHYS, **CTRL)
    E0, M0 = s.energy()
    recs = []
    for _ in range(20):
        recs += s.step(100)
    E = [E0] + [r["energy"] for r in recs]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(E, E[1:])), "energy increased"
    assert all(abs(r["mass"] - M0) <= 1e-12 * M0 for r in recs)
    assert max(r["dt"] for r in recs) > 1e-2
