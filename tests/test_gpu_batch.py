"""GPU tests of the batched driver: every instance of a batch must follow its own
single-instance run (same kernels, same operation order per instance), with and
without the recorded graphs and in mixed precision, and match the FP64 oracle."""
import numpy as np
import pytest

from acch_inputs import random_ic
from oracle import controller, newton
from oracle.params import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2007_04560_amd import AcchError, BatchSolver, Solver  # noqa: E402
from paper_2007_04560_amd.batch import autotune, parts_for, with_boxes  # noqa: E402

COMMON = dict(dt_fixed=1e-3, overlap=1, ilu_shift=0.02, newton_rtol=1e-8, gmres_rtol=1e-8)


def instances():
    """Uneven instances: sizes, boundaries, parameters and subdomain counts differ."""
    spec = [((24, 24), "periodic", 0.10, 1e-3, (2, 2)), ((40, 32), "neumann", 0.09, 2e-3, (2, 3)),
            ((33, 47), "periodic", 0.12, 5e-4, (3, 2)), ((16, 20), "neumann", 0.11, 1.5e-3, (1, 1)),
            ((48, 48), "periodic", 0.08, 8e-4, (3, 3)), ((20, 36), "neumann", 0.1, 1e-3, (2, 1))]
    fields, params = [], []
    for k, (shape, bc, theta, gamma, sub) in enumerate(spec):
        fields.append(random_ic(shape, 300 + k))
        params.append(dict(bc=bc, theta=theta, gamma=gamma, sub=sub))
    return fields, params


def single_runs(fields, params, nsteps, **common):
    out = []
    for (u, v), p in zip(fields, params):
        kw = dict(common)
        kw.update(p)
        with Solver(u, v, **kw) as s:
            recs = s.step(nsteps)
            out.append((s.fields(), sum(r["newton_its"] for r in recs), sum(r["gmres_its"] for r in recs)))
    return out


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_single_instance_runs(graph, precision):
    fields, params = instances()
    nsteps = 3
    ref = single_runs(fields, params, nsteps, precision=precision, **COMMON)
    with BatchSolver(fields, params, graph=graph, precision=precision, **COMMON) as b:
        nit, git = b.step(nsteps)
        for i, ((u, v), n_it, g_it) in enumerate(ref):
            ub, vb = b.fields(i)
            scale = max(np.max(np.abs(u)), np.max(np.abs(v)))
            assert max(np.max(np.abs(ub - u)), np.max(np.abs(vb - v))) <= 1e-13 * scale, i
            assert nit[i] == n_it and git[i] == g_it, (i, nit[i], n_it, git[i], g_it)
        c = b.counters()
        assert (c["graph_launches"] > 0) == graph


def test_batched_preconditioner_equals_each_instance():
    """One launch over all subdomains of all instances = each instance's own M^{-1}."""
    fields, params = instances()
    with BatchSolver(fields, params, **COMMON) as b:
        b.step(1)
        info = b.info()
        r = np.random.default_rng(11).standard_normal(2 * info["ncell"])
        z = b.precondition(torch.as_tensor(r).cuda())
        b.stream.synchronize()
        z = z.cpu().numpy()
    for i, ((u, v), p) in enumerate(zip(fields, params)):
        kw = dict(COMMON)
        kw.update(p)
        n2 = 2 * u.size
        xo = info["xoff"][i]
        with Solver(u, v, **kw) as s:
            s.step(1)
            zi = s.precondition(torch.as_tensor(r[xo:xo + n2]).cuda()).cpu().numpy()
        assert np.max(np.abs(z[xo:xo + n2] - zi)) <= 1e-13 * np.max(np.abs(zi)), i


BOX = dict(COMMON, ilu_shift=0.0, subsolver="iluk_box", fill_level=0)


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_box_pattern_batch_matches_single_instance_runs(graph, precision):
    """Batches with ILU(0) on the box pattern (its own factorisation and sweep kernels, one
    launch each over all boxes of all instances, padded to a common box): each instance
    follows its own single-instance run, with the same Newton and GMRES counts."""
    fields, params = instances()
    nsteps = 3
    ref = single_runs(fields, params, nsteps, precision=precision, **BOX)
    with BatchSolver(fields, params, graph=graph, precision=precision, **BOX) as b:
        nit, git = b.step(nsteps)
        for i, ((u, v), n_it, g_it) in enumerate(ref):
            ub, vb = b.fields(i)
            scale = max(np.max(np.abs(u)), np.max(np.abs(v)))
            assert max(np.max(np.abs(ub - u)), np.max(np.abs(vb - v))) <= 1e-13 * scale, i
            assert nit[i] == n_it and git[i] == g_it, (i, nit[i], n_it, git[i], g_it)
        assert (b.counters()["graph_launches"] > 0) == graph


def test_box_pattern_batched_preconditioner_equals_each_instance():
    fields, params = instances()
    with BatchSolver(fields, params, **BOX) as b:
        b.step(1)
        info = b.info()
        r = np.random.default_rng(12).standard_normal(2 * info["ncell"])
        z = b.precondition(torch.as_tensor(r).cuda())
        b.stream.synchronize()
        z = z.cpu().numpy()
    for i, ((u, v), p) in enumerate(zip(fields, params)):
        kw = dict(BOX)
        kw.update(p)
        n2 = 2 * u.size
        xo = info["xoff"][i]
        with Solver(u, v, **kw) as s:
            s.step(1)
            zi = s.precondition(torch.as_tensor(r[xo:xo + n2]).cuda()).cpu().numpy()
        assert np.max(np.abs(z[xo:xo + n2] - zi)) <= 1e-13 * np.max(np.abs(zi)), i


@pytest.mark.parametrize("pattern", ["stencil", "box"])
def test_batch_matches_oracle(pattern):
    fields, params = instances()
    fields, params = fields[:2], params[:2]
    tight = dict(COMMON if pattern == "stencil" else BOX, newton_rtol=1e-12, newton_atol=1e-13, gmres_rtol=1e-13,
                 gmres_atol=1e-15, gmres_max_restarts=30)
    with BatchSolver(fields, params, **tight) as b:
        b.step(2)
        E, M = b.energy()
        for i, ((u0, v0), p) in enumerate(zip(fields, params)):
            P = Problem(bc=p["bc"], theta=p["theta"], gamma=p["gamma"])
            run = controller.Run(P, u0, v0, adaptive=False, dt_fixed=1e-3,
                                 newton=newton.NewtonOptions(rtol=1e-12, atol=1e-11))
            run.step()
            run.step()
            ub, vb = b.fields(i)
            ref = np.concatenate([run.u.ravel(), run.v.ravel()])
            got = np.concatenate([ub.ravel(), vb.ravel()])
            assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref), i
            assert abs(M[i] - np.sum(u0) / u0.size) <= 1e-12 * M[i]


def test_batch_rejects_bad_configurations():
    fields, params = instances()
    with pytest.raises(AcchError):
        BatchSolver(fields[:2], [dict(params[0], adaptive=True), params[1]], **COMMON)
    with pytest.raises(AcchError):
        BatchSolver(fields[:2], [params[0], dict(params[1], overlap=2)], **COMMON)
    with pytest.raises(AcchError):   # ILU(k >= 1) has no batched kernels
        BatchSolver(fields[:2], params[:2], **dict(BOX, fill_level=1))
    with pytest.raises(AcchError):   # one subdomain solver for all instances
        BatchSolver(fields[:2], [params[0], dict(params[1], subsolver="iluk_box")], **COMMON)


def test_autotuner_picks_a_measured_box():
    fields = [random_ic((n, n), 400 + n) for n in (32, 48, 64)]
    params = [dict(bc="periodic") for _ in fields]
    assert parts_for(64, 32, 1, True) == 2 and parts_for(48, 64, 1, True) == 2
    best, timings = autotune(fields, params, boxes=(16, 32), steps=1, **COMMON)
    assert best in (16, 32) and set(timings) == {16, 32}
    subs = with_boxes([u.shape for u, _ in fields], params, best, 1)
    with BatchSolver(fields, subs, **COMMON) as b:
        nit, _ = b.step(1)
        assert np.all(nit >= 1)
