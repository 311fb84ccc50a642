"""GPU parity of the ILU(k) and exact-LU subdomain solvers (Section 3.1, Table 2)
against the oracle: the band factors against the oracle's textbook ILU(k) on the
level-of-fill pattern, M^{-1} r against the oracle's Schwarz operator with the same
subdomain solver (the exact LU there is a sparse direct factorisation of A_k), and
whole Newton steps against the oracle's roots."""
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
CASES = [((37, 29), "periodic", (2, 2), 1), ((45, 58), "neumann", (3, 2), 2), ((33, 17), "neumann", (1, 1), 0)]


def prob(bc):
    return Problem(bc=bc, alpha=1.2, beta=1.2, theta=0.1, gamma=1e-3, rho=1.0)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def vec(u, v):
    return np.concatenate([u.ravel(), v.ravel()])


def _setup(shape, bc, sub, ov, subsolver, level=0, precision="fp64", schwarz_kind="left", dt=2e-3, seed=31):
    u1, v1, u0, v0 = perturbed_pair(shape, seed, amp=0.03)
    s = Solver(u0, v0, bc=bc, sub=sub, overlap=ov, subsolver=subsolver, fill_level=level, precision=precision,
               schwarz=schwarz_kind)
    s.jacobian(dev(vec(u1, v1)), dev(vec(u0, v0)), dt)
    s.factor()
    Jo = jacobian.jacobian(u1, v1, u0, v0, dt, prob(bc))
    return s, Jo


@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
@pytest.mark.parametrize("subsolver,level", [("iluk", 1), ("iluk", 2), ("iluk_box", 1), ("iluk_box", 2)])
def test_iluk_band_factors_match_oracle(shape, bc, sub, ov, subsolver, level):
    """Every entry of the GPU's ILU(k) factors (band storage) equals the oracle's
    textbook ILU(k) on the level-k pattern (of the stencil or of the box base
    pattern), and the band is zero off that pattern."""
    s, Jo = _setup(shape, bc, sub, ov, subsolver, level)
    band = s.export_band().cpu().numpy()
    info = s.info()
    bw = info["box_w"]
    kl = 4 * bw + (5 if subsolver == "iluk_box" else 0)
    assert band.shape[2] == 2 * kl + 1
    subs = schwarz.decompose(shape, (sub[1], sub[0]), ov, bc)
    worst, scale = 0.0, 0.0
    for k, sd in enumerate(subs):
        rows = schwarz.subdomain_matrix(Jo, sd, shape)
        if subsolver == "iluk_box":
            rows = schwarz.box_pattern(rows, sd)
        fac = schwarz.iluk(rows, level)
        seen = np.zeros(band.shape[1:], dtype=bool)
        for i, (by, bx) in enumerate(sd.cells):
            for t in (0, 1):
                R = 2 * (by * bw + bx) + t
                for jcol, val in fac[2 * i + t].items():
                    cj = sd.cells[jcol // 2]
                    C = 2 * (cj[0] * bw + cj[1]) + jcol % 2
                    want = 1.0 / val if C == R else val
                    got = band[k, R, C - R + kl]
                    worst = max(worst, abs(got - want) / max(abs(want), 1e-300) if C == R else abs(got - want))
                    scale = max(scale, abs(val))
                    seen[R, C - R + kl] = True
                # off the pattern the row of a grid cell holds zeros
                row = band[k, R].copy()
                row[seen[R]] = 0.0
                assert np.all(row == 0.0), (k, R)
    assert worst <= 1e-11 * max(scale, 1.0)


@pytest.mark.parametrize("shape,bc,sub,ov", CASES)
@pytest.mark.parametrize("subsolver,level", [("iluk", 1), ("iluk", 2), ("lu", 0), ("iluk_box", 0), ("iluk_box", 2)])
def test_band_preconditioner_matches_oracle(shape, bc, sub, ov, subsolver, level):
    s, Jo = _setup(shape, bc, sub, ov, subsolver, level)
    r = np.random.default_rng(7).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    P = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", solver=subsolver, level=level)
    zo = P.apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))


@pytest.mark.parametrize("kind", ["right", "classical"])
@pytest.mark.parametrize("subsolver,level", [("iluk", 2), ("lu", 0), ("iluk_box", 0)])
def test_band_preconditioner_variants_match_oracle(kind, subsolver, level):
    shape, bc, sub, ov = (45, 58), "neumann", (3, 2), 2
    s, Jo = _setup(shape, bc, sub, ov, subsolver, level, schwarz_kind=kind)
    r = np.random.default_rng(8).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    P = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind=kind, solver=subsolver, level=level)
    zo = P.apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))


@pytest.mark.parametrize("subsolver,level", [("iluk", 2), ("lu", 0), ("iluk_box", 0)])
def test_band_mixed_precision_preconditioner(subsolver, level):
    """FP32 band factors: M^{-1} r within FP32 rounding (amplified by the box matrices'
    conditioning) of the FP64 oracle."""
    shape, bc, sub, ov = (45, 58), "neumann", (3, 2), 2
    s, Jo = _setup(shape, bc, sub, ov, subsolver, level, precision="mixed")
    r = np.random.default_rng(9).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", solver=subsolver, level=level).apply(r)
    assert np.linalg.norm(z - zo) <= 1e-4 * np.linalg.norm(zo)


@pytest.mark.parametrize("subsolver", ["lu", "iluk"])
def test_widest_band_box(subsolver):
    """Padded boxes 55 cells wide (the largest register window of the factorisation)
    and 44 tall, ragged Neumann split."""
    shape, bc, sub, ov = (80, 101), "neumann", (2, 2), 2
    s, Jo = _setup(shape, bc, sub, ov, subsolver, 1, dt=1e-3)
    assert s.info()["box_w"] == 55
    r = np.random.default_rng(10).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", solver=subsolver, level=1).apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))


def test_widest_box_pattern_box():
    """The box base pattern widens the band by 5 diagonals: padded boxes 54 cells wide
    take the largest register window (kl = 221), ragged Neumann split (ILU(1) on the
    box pattern; its ILU(0) has kernels of its own)."""
    shape, bc, sub, ov = (80, 99), "neumann", (2, 2), 2
    s, Jo = _setup(shape, bc, sub, ov, "iluk_box", 1, dt=1e-3)
    assert s.info()["box_w"] == 54
    r = np.random.default_rng(12).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", solver="iluk_box", level=1).apply(r)
    assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))


def test_box_pattern_rejects_boxes_wider_than_its_window():
    u0, v0 = random_ic((24, 101), 0)
    with pytest.raises(Exception):
        Solver(u0, v0, bc="neumann", sub=(2, 1), overlap=2, subsolver="iluk_box", fill_level=1)
    Solver(u0, v0, bc="neumann", sub=(2, 1), overlap=2, subsolver="iluk", fill_level=1).close()


def _rel_l2(u, v, uo, vo):
    return math.sqrt(np.sum((u - uo) ** 2 + (v - vo) ** 2) / np.sum(uo ** 2 + vo ** 2))


@pytest.mark.parametrize("subsolver,level", [("iluk", 1), ("iluk", 2), ("lu", 0), ("iluk_box", 0)])
def test_steps_with_band_subsolvers_match_oracle(subsolver, level):
    """Four steps of the 64x64 periodic workload (2x2 subdomains, overlap 1) with each
    subdomain solver: roots = the oracle's to 1e-10 per step, the same Newton counts,
    and fewer GMRES iterations than with ILU(0)."""
    shape = (64, 64)
    u0, v0 = random_ic(shape, 0)
    kw = dict(bc="periodic", sub=(2, 2), overlap=1, dt_fixed=1e-3, newton_rtol=1e-12, newton_atol=1e-13,
              gmres_rtol=1e-12)
    s = Solver(u0, v0, subsolver=subsolver, fill_level=level, **kw)
    s0 = Solver(u0, v0, **kw)
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


# box widths whose register windows take 6, 8, 10, 11, 12 and 13 tiles of 16 (the smallest
# nr with 16 nr >= 4 bw + 1); two subdomains along x, overlap 2, Neumann
@pytest.mark.parametrize("bw,nr", [(22, 6), (30, 8), (38, 10), (42, 11), (46, 12), (50, 13)])
@pytest.mark.parametrize("subsolver,level,precision", [("lu", 0, "fp64"), ("iluk", 1, "fp64"), ("lu", 0, "mixed")])
def test_band_window_sizes_match_oracle(bw, nr, subsolver, level, precision):
    """M^{-1} r with each register-window size of the band factorisation (FP32 factors
    are eliminated in FP32) against the oracle's Schwarz operator with the same
    subdomain solver."""
    ov = 2
    shape, bc, sub = (24, 2 * (bw - 2 * ov)), "neumann", (2, 1)
    assert 16 * nr >= 4 * bw + 1 > 16 * (nr - 1)
    s, Jo = _setup(shape, bc, sub, ov, subsolver, level, precision=precision, dt=1e-3)
    assert s.info()["box_w"] == bw
    r = np.random.default_rng(11).standard_normal(Jo.shape[0])
    z = s.precondition(dev(r)).cpu().numpy()
    zo = schwarz.Schwarz(Jo, shape, (sub[1], sub[0]), ov, bc, kind="left", solver=subsolver, level=level).apply(r)
    if precision == "fp64":
        assert np.max(np.abs(z - zo)) <= 1e-10 * np.max(np.abs(zo))
    else:
        assert np.linalg.norm(z - zo) <= 1e-4 * np.linalg.norm(zo)
