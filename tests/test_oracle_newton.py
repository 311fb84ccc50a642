"""Pins for the oracle's Newton step (Section 3.1), line search, controller
(Section 3.2), energy law (Theorem 2.3) and the scheme's convergence order (Section 4.1 A)."""
import math

import numpy as np
import pytest

from acch_inputs import perturbed_pair, random_ic, smooth_ic_2d
import scipy.sparse.linalg as spla

from oracle import controller, jacobian, newton, scalar, scheme
from oracle.params import Problem


def _dense_newton_loops(u0, v0, dt, prob, tol=1e-13, max_it=30):
    """Newton on the loop residual with a dense finite-difference Jacobian."""
    shape = u0.shape
    n = u0.size

    def F(X):
        Fu, Fv = scalar.residual_loops(X[:n].reshape(shape), X[n:].reshape(shape), u0, v0, dt, prob)
        return np.concatenate([Fu.ravel(), Fv.ravel()])

    X = np.concatenate([u0.ravel(), v0.ravel()])
    for _ in range(max_it):
        Fx = F(X)
        if np.linalg.norm(Fx) < tol:
            break
        J = np.zeros((2 * n, 2 * n))
        for k in range(2 * n):
            e = np.zeros(2 * n)
            e[k] = 1e-7
            J[:, k] = (F(X + e) - F(X - e)) / 2e-7
        X = X - np.linalg.solve(J, Fx)
    return X


@pytest.mark.parametrize("shape,bc", [((4, 4), "periodic"), ((3, 4), "neumann"), ((3, 3, 3), "neumann")])
def test_newton_root_matches_dense_loop_newton(shape, bc):
    prob = Problem(bc=bc, lengths=(1.0, 1.0, 1.0)[:len(shape)], gamma=0.01)
    u0, v0 = random_ic(shape, 4)
    dt = 0.05
    res = newton.solve_step(u0, v0, dt, prob, newton.NewtonOptions(rtol=1e-15, atol=1e-13))
    assert res.converged
    X2 = _dense_newton_loops(u0, v0, dt, prob)
    assert np.max(np.abs(res.X - X2)) <= 1e-13 * np.max(np.abs(X2))


def test_newton_step_properties():
    shape = (16, 16)
    prob = Problem(bc="periodic")
    u0, v0 = random_ic(shape, 0)
    res = newton.solve_step(u0, v0, 1e-3, prob, newton.NewtonOptions(rtol=1e-12))
    assert res.converged and 1 <= res.iterations <= 6
    n = u0.size
    u1 = res.X[:n].reshape(shape)
    v1 = res.X[n:].reshape(shape)
    assert abs(scheme.mass(u1, prob) - scheme.mass(u0, prob)) < 1e-15
    assert scheme.energy(u1, v1, prob) < scheme.energy(u0, v0, prob)
    # quadratic convergence: the last ratio is tiny
    f = res.fnorms
    assert f[-1] < 1e-12 * f[0]


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
def test_energy_law_identity(bc):
    """E(U1) - E(U0) + dt <G~ . A~ G~^S> = dt <G~ . F(U1)> (from eqs. DVD and NSOA-1) and,
    for S = 10, Theorem 2.3's dissipation -<G~ . A~ G~^S> <= 1/4 <R . A~ R>."""
    shape = (12, 10)
    prob = Problem(bc=bc, lengths=(1.0, 0.9), alpha=4.0, beta=2.0, gamma=0.005, rho=0.001)
    h = prob.spacing(shape)
    u0, v0 = random_ic(shape, 3, u_mean=0.55)
    dt = 0.01
    res = newton.solve_step(u0, v0, dt, prob, newton.NewtonOptions(rtol=1e-10))
    n = u0.size
    u1 = res.X[:n].reshape(shape)
    v1 = res.X[n:].reshape(shape)
    vol = scheme.cell_volume(shape, prob)
    mu_s, nu_s = scheme.discrete_variational_derivative(u1, v1, u0, v0, prob)
    phi = scheme.g2_exact(u1 + v1, u0 + v0)
    psi = scheme.g2_exact(u1 - v1, u0 - v0)
    G1u = -0.5 * prob.alpha * (u1 + u0 - 1)
    G1v = -0.5 * prob.beta * (v1 + v0)
    G3u = -0.5 * prob.gamma * (scheme.laplacian(u1, h, bc) + scheme.laplacian(u0, h, bc))
    G3v = -0.5 * prob.gamma * (scheme.laplacian(v1, h, bc) + scheme.laplacian(v0, h, bc))
    Gu = G1u + prob.theta * (phi + psi) + G3u
    Gv = G1v + prob.theta * (phi - psi) + G3v
    c = scheme.operator_mobility(u1, v1, u0, v0, prob)
    AGu = -scheme.div_c_grad(c, mu_s, h, bc)
    AGv = c * nu_s / prob.rho
    Fu, Fv = scheme.residual(u1, v1, u0, v0, dt, prob)
    dE = scheme.energy(u1, v1, prob) - scheme.energy(u0, v0, prob)
    diss = vol * np.sum(Gu * AGu + Gv * AGv)
    work = vol * np.sum(Gu * Fu + Gv * Fv)
    assert abs(dE + dt * diss - dt * work) < 1e-10 * abs(dE)
    assert dE < 0
    Ru, Rv = Gu - mu_s, Gv - nu_s
    ARu = -scheme.div_c_grad(c, Ru, h, bc)
    bound = 0.25 * vol * np.sum(Ru * ARu + Rv * c * Rv / prob.rho)
    assert -diss <= bound + 1e-12 * abs(diss)


def _newton_direction(shape, seed, dt, prob):
    u0, v0 = random_ic(shape, seed)
    U0 = np.concatenate([u0.ravel(), v0.ravel()])
    rfun = lambda Y: scheme.residual_vec(Y, U0, dt, prob, shape)
    F = rfun(U0)
    J = jacobian.jacobian(u0, v0, u0, v0, dt, prob)
    S = spla.spsolve(J.tocsc(), -F)
    return U0, F, S, rfun


def test_line_search_backtracks_and_respects_admissibility():
    """A step that leaves the admissible set at full length: lambda halves (without
    evaluating F) until the trial is admissible, every evaluated trial is admissible,
    each later lambda lies in [0.1, 0.5] times the previous one, and the accepted
    point passes the sufficient-decrease test."""
    shape = (8, 8)
    prob = Problem(bc="periodic")
    X, F, SN, rfun = _newton_direction(shape, 1, 0.01, prob)
    n = X.size // 2
    S = 1024.0 * SN                       # far beyond the admissible set at lambda = 1
    assert not scheme.admissible((X + S)[:n], (X + S)[n:])
    m = 0                                 # first admissible power of two, found directly
    while not scheme.admissible((X + S / 2 ** m)[:n], (X + S / 2 ** m)[n:]):
        m += 1
    assert m >= 2
    k = int(np.argmax(np.abs(S)))
    trials = []

    def logged(Y):
        assert scheme.admissible(Y[:n], Y[n:])
        trials.append((Y[k] - X[k]) / S[k])
        return rfun(Y)

    out = newton.line_search(logged, X, S, F, n, newton.NewtonOptions())
    assert out is not None
    lam, Xt, Ft = out
    assert trials[0] == pytest.approx(2.0 ** -m, rel=1e-12)
    for a, b in zip(trials, trials[1:]):
        assert 0.1 * a * (1 - 1e-12) <= b <= 0.5 * a * (1 + 1e-12)
    assert lam == pytest.approx(trials[-1], rel=1e-12)
    assert scheme.admissible(Xt[:n], Xt[n:])
    assert 0.5 * Ft @ Ft <= 0.5 * F @ F * (1 - 2e-4 * lam)


def _atan_trials(x0):
    """Trial lambdas of the line search on F(x) = atan(x) along the Newton step
    S = -atan(x0)(1 + x0^2), with the values f(lambda) = atan(x0 + lambda S)^2 / 2."""
    F = lambda X: np.array([math.atan(X[0])])
    X = np.array([x0])
    S = np.array([-math.atan(x0) * (1.0 + x0 * x0)])
    trials = []

    def logged(Y):
        trials.append(((Y[0] - x0) / S[0], 0.5 * math.atan(Y[0]) ** 2))
        return F(Y)

    out = newton.line_search(logged, X, S, F(X), 0, newton.NewtonOptions())
    return out, trials, 0.5 * math.atan(x0) ** 2


def test_line_search_quadratic_backtrack_on_atan():
    """From x0 = 2 the full Newton step overshoots; the next trial is the minimiser of
    the parabola through f(0), the Newton slope f'(0) = -2 f(0) and f(1), which passes.
    The expected lambda was computed by hand from that parabola:
    f(0) = atan(2)^2/2 = 0.61285..., f(1) = atan(2 - 5 atan 2)^2/2 = 0.83873...,
    lambda = 2 f(0) / (2 (f(1) - f(0) + 2 f(0))) = 0.42221028..."""
    out, trials, f0 = _atan_trials(2.0)
    assert out is not None
    assert [t for t, _ in trials][0] == 1.0
    assert len(trials) == 2
    lam = trials[1][0]
    assert lam == pytest.approx(0.422210284908187, rel=1e-12)
    # the same point as the stationary point of the interpolating parabola, found by
    # fitting q(t) = f0 + g t + c t^2 to the data with a least-squares solve
    g = -2.0 * f0
    c = np.linalg.lstsq(np.array([[1.0]]), np.array([trials[0][1] - f0 - g]), rcond=None)[0][0]
    assert lam == pytest.approx(-g / (2.0 * c), rel=1e-12)
    assert out[0] == lam


def test_line_search_upper_clamp_on_atan():
    """Just inside Newton's 2-cycle of atan (x0 = 1.39173520..., the cycle point being
    the root of 2x = atan(x)(1 + x^2), 1.39174520...) the full step lands almost on
    -x0: f(1) is below f(0) by less than the Armijo margin, so the step fails, and the
    parabola's minimiser f(0)/(f(0) + f(1)) = 0.50000294... is clamped to 0.5."""
    out, trials, f0 = _atan_trials(1.3917352002707346)
    assert out is not None
    lams = [t for t, _ in trials]
    assert lams[0] == 1.0 and f0 * (1 - 2e-4) < trials[0][1] < f0
    assert lams[1] == 0.5
    assert out[0] == 0.5


def test_line_search_cubic_backtracks_on_atan():
    """From x0 = 10 the quadratic trial fails too; the later trials minimise the cubic
    f(0) + f'(0) t + b t^2 + a t^3 through the last two trials (a, b from a 2x2 solve,
    the minimum taken where the cubic's second derivative is positive), each clamped to
    [0.1, 0.5] times the previous lambda.  Hand-computed sequence:
    1, 0.46956306999, 0.17085943160, 0.06468572070 (accepted)."""
    out, trials, f0 = _atan_trials(10.0)
    assert out is not None
    lams = [t for t, _ in trials]
    want = [1.0, 0.4695630699888559, 0.17085943160316305, 0.06468572069667183]
    assert len(lams) == len(want)
    for got, w in zip(lams, want):
        assert got == pytest.approx(w, rel=1e-10)
    g = -2.0 * f0
    for i in range(2, len(trials)):
        (l1, f1), (l2, f2) = trials[i - 2], trials[i - 1]
        a, b = np.linalg.solve(np.array([[l1 ** 3, l1 ** 2], [l2 ** 3, l2 ** 2]]),
                               np.array([f1 - f0 - g * l1, f2 - f0 - g * l2]))
        roots = np.roots([3 * a, 2 * b, g])
        mins = [r.real for r in roots if abs(r.imag) < 1e-14 and 6 * a * r.real + 2 * b > 0]
        assert len(mins) == 1
        expect = min(max(mins[0], 0.1 * l2), 0.5 * l2)
        assert lams[i] == pytest.approx(expect, rel=1e-10)
    assert out[0] == lams[-1]
    f_acc = trials[-1][1]
    assert f_acc <= f0 * (1 - 2e-4 * lams[-1])


def test_controller_prediction_table():
    """eq. sencondt with dt_0 = dt_min."""
    assert controller.predict_dt(True, 5.0, 1.0, 1e4, 1e-4, 0.1) == 1e-4
    cases = [(0.0, 1e-3, 1e4, 0.1), (1e-3, 1e-3, 1e4, 0.1 / math.sqrt(1 + 1e4)),
             (1.0, 1e-4, 1e4, 1e-4), (0.02, 0.01, 100.0, 0.1 / math.sqrt(1 + 100 * 4))]
    for dn, dtp, eta, want in cases:
        assert abs(controller.predict_dt(False, dn, dtp, eta, 1e-4, 0.1) - want) < 1e-15
    assert controller.retry_dt(1e-3, 1e-4) == pytest.approx(1e-3 / math.sqrt(2))
    assert controller.retry_dt(1.2e-4, 1e-4) == 1e-4


def test_controller_retries_and_eta_doubling():
    """Forcing every attempt to diverge (one Newton iteration allowed, impossible
    tolerance) walks dt down by sqrt(2) to dt_min, doubling eta each time, then fails."""
    shape = (8, 8)
    prob = Problem(bc="periodic")
    u, v = random_ic(shape, 2)
    run = controller.Run(prob, u.copy(), v.copy(), adaptive=True, dt_min=1e-4, dt_max=1e-1, eta=1e4,
                         newton=newton.NewtonOptions(rtol=0.0, atol=0.0, max_it=1))
    run.X_prev = run.X + 1e-4
    run.dt_prev = 1e-4
    dt0 = controller.predict_dt(False, np.linalg.norm(np.full(2 * u.size, 1e-4)), 1e-4, 1e4, 1e-4, 1e-1)
    expect_retries = 0
    dt = dt0
    while dt > 1e-4:
        dt = controller.retry_dt(dt, 1e-4)
        expect_retries += 1
    with pytest.raises(controller.DivergedError):
        run.step()
    assert run.eta == 1e4 * 2 ** (expect_retries + 1)
    assert np.array_equal(run.u, u) and np.array_equal(run.v, v)


def test_adaptive_run_grows_dt_and_dissipates_energy():
    shape = (16, 16)
    prob = Problem(bc="neumann")
    u, v = random_ic(shape, 5)
    # eta = 1: with the plain 2-norm X'_d is about 30 here, so dt leaves dt_min at once
    run = controller.Run(prob, u, v, adaptive=True, dt_min=1e-4, dt_max=1e-1, eta=1.0)
    E = [scheme.energy(u, v, prob)]
    for _ in range(12):
        E.append(run.step().energy)
    dts = [r.dt for r in run.history]
    assert dts[0] == 1e-4 and max(dts) > 10 * dts[0]
    assert all(E[i + 1] <= E[i] + 1e-14 for i in range(len(E) - 1))
    m0 = scheme.mass(u, prob)
    assert abs(run.history[-1].mass - m0) < 1e-14


def _restrict(f):
    return 0.25 * (f[0::2, 0::2] + f[1::2, 0::2] + f[0::2, 1::2] + f[1::2, 1::2])


def _run_fixed(n, dt, T, prob):
    u, v = smooth_ic_2d(n, n)
    run = controller.Run(prob, u, v, adaptive=False, dt_fixed=dt,
                         newton=newton.NewtonOptions(rtol=1e-12, atol=1e-10))
    for _ in range(int(round(T / dt))):
        run.step()
    return run.u, run.v


@pytest.mark.slow
def test_second_order_in_time_and_space():
    """Self-convergence on the smooth data of Section 4.1 A: successive differences
    shrink by about 4 when dt (or h) halves; the explicit mobility reading is only
    first order in time."""
    prob = Problem(bc="periodic", alpha=4.0, beta=2.0, gamma=0.005, theta=0.1, rho=0.001)
    T = 0.008
    sols = [_run_fixed(16, T / k, T, prob) for k in (2, 4, 8)]
    d = [np.sqrt(np.sum((sols[i][0] - sols[i + 1][0]) ** 2 + (sols[i][1] - sols[i + 1][1]) ** 2))
         for i in range(2)]
    order_t = math.log2(d[0] / d[1])
    assert 1.8 < order_t < 2.3
    pe = prob.with_(mobility="explicit")
    sols = [_run_fixed(16, T / k, T, pe) for k in (2, 4, 8)]
    d = [np.sqrt(np.sum((sols[i][0] - sols[i + 1][0]) ** 2 + (sols[i][1] - sols[i + 1][1]) ** 2))
         for i in range(2)]
    assert math.log2(d[0] / d[1]) < 1.4
    T = 0.004
    s = [_run_fixed(n, T / 8, T, prob) for n in (16, 32, 64)]
    e1 = np.sqrt(np.mean((s[0][0] - _restrict(s[1][0])) ** 2 + (s[0][1] - _restrict(s[1][1])) ** 2))
    e2 = np.sqrt(np.mean((s[1][0] - _restrict(s[2][0])) ** 2 + (s[1][1] - _restrict(s[2][1])) ** 2))
    assert 1.7 < math.log2(e1 / e2) < 2.4
