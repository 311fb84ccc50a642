"""Gradient of the final discrete energy of a run of scheme (2.20) by the discrete
adjoint of the time-step map, as a ``torch.autograd.Function``.

The loss is E~(U^N), the discrete energy (eqs. relations, freeenergy) after N
accepted steps from (u0, v0), with the accepted step sizes held fixed (the
dependence of the adaptive controller's dt on the state is not differentiated).
Forward: the steps run in libacch; the accepted dt sequence is recorded and the
state is checkpointed (host copies) every ``checkpoint_every`` steps.  Backward:
from the last segment to the first, the segment's states are recomputed from its
checkpoint with the recorded step sizes (acch_solve_step), then acch_adjoint_step
walks back through it:
  J_n^T lambda_n = g_{n+1},  g_n = -(dF_n/dU^n)^T lambda_n,  dE/dp -= lambda_n . dF_n/dp.
Every step of that runs in the HIP library; this module only schedules the calls.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from .binding import Solver

PARAM_NAMES = ("alpha", "beta", "theta", "gamma")


def _run_forward(u0: np.ndarray, v0: np.ndarray, nsteps: int, checkpoint_every: int, kw: Dict):
    s = Solver(u0, v0, **kw)
    ckpts: List[Tuple[int, np.ndarray, np.ndarray]] = [(0, u0.copy(), v0.copy())]
    dts: List[float] = []
    for k in range(nsteps):
        if k > 0 and k % checkpoint_every == 0:
            u, v = s.fields()
            ckpts.append((k, u, v))
        rec = s.step(1)[0]
        dts.append(float(rec["dt"]))
    return s, ckpts, dts


def _state(s: Solver, u: np.ndarray, v: np.ndarray):
    return s.vector(np.concatenate([u.ravel(), v.ravel()]))


class FinalEnergy:
    """``FinalEnergy.apply(u0, v0, params, nsteps, checkpoint_every, solver_kw)`` with
    u0, v0 float64 tensors of the grid shape (ny, nx) and params a float64 tensor
    (alpha, beta, theta, gamma); returns E~(U^N) as a 0-d float64 tensor."""

    _fn = None

    @classmethod
    def apply(cls, *args):
        if cls._fn is None:
            cls._fn = _make_function()
        return cls._fn.apply(*args)


def _make_function():
    import torch

    class _FinalEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, u0, v0, params, nsteps: int, checkpoint_every: int, solver_kw: Dict):
            if nsteps < 1 or checkpoint_every < 1:
                raise ValueError("nsteps and checkpoint_every must be positive")
            kw = dict(solver_kw)
            kw.update(dict(zip(PARAM_NAMES, params.detach().cpu().double().tolist())))
            u0n = u0.detach().cpu().double().numpy()
            v0n = v0.detach().cpu().double().numpy()
            s, ckpts, dts = _run_forward(u0n, v0n, nsteps, checkpoint_every, kw)
            E, _ = s.energy()
            uN, vN = s.fields()
            ctx.solver = s
            ctx.ckpts = ckpts
            ctx.dts = dts
            ctx.final = (uN, vN)
            ctx.shape = u0n.shape
            ctx.out_device = u0.device
            return torch.tensor(E, dtype=torch.float64, device=u0.device)

        @staticmethod
        def backward(ctx, gE):
            s: Solver = ctx.solver
            n = int(np.prod(ctx.shape))
            g, dp = s.energy_gradient(_state(s, *ctx.final))
            bounds = [c[0] for c in ctx.ckpts] + [len(ctx.dts)]
            for seg in range(len(ctx.ckpts) - 1, -1, -1):
                k0, u, v = ctx.ckpts[seg]
                k1 = bounds[seg + 1]
                s.set_fields(u, v)
                states = [_state(s, u, v)]
                for k in range(k0, k1):
                    s.solve_step(ctx.dts[k])
                    states.append(_state(s, *s.fields()))
                for k in range(k1 - 1, k0 - 1, -1):
                    g, dp, _, _ = s.adjoint_step(states[k + 1 - k0], states[k - k0], ctx.dts[k], g, dp)
            s.close()
            scale = gE.detach().to(torch.float64).cpu()
            gu = (g[:n].reshape(ctx.shape).to(ctx.out_device) * scale.to(ctx.out_device))
            gv = (g[n:].reshape(ctx.shape).to(ctx.out_device) * scale.to(ctx.out_device))
            gp = torch.tensor(dp, dtype=torch.float64) * scale
            return gu, gv, gp.to(ctx.out_device), None, None, None

    return _FinalEnergy


def final_energy(u0, v0, params, nsteps: int, checkpoint_every: int = 5, **solver_kw):
    """E~(U^N) after nsteps accepted steps, differentiable in u0, v0 and params =
    (alpha, beta, theta, gamma).  solver_kw are Solver options other than the four
    parameters (grid, boundary, subdomains, tolerances, dt control ...)."""
    for k in PARAM_NAMES:
        if k in solver_kw:
            raise ValueError(f"{k} is passed in params")
    return FinalEnergy.apply(u0, v0, params, nsteps, checkpoint_every, solver_kw)
