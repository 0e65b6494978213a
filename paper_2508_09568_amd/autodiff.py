"""Differentiable rollouts of the bunch update for inverse / initial-state problems.

`rollout(U0, bunch, nbr, dt, dx, nsteps, checkpoint_every)` advances U0 (owned cells and
faces; guards are refilled every step) by `nsteps` updates at fixed time steps and is a
torch.autograd.Function: the backward pass recomputes each segment of `checkpoint_every`
steps from its stored checkpoint and runs the library's adjoint (mhd_bunch_adjoint) step
by step in reverse.  Memory: nsteps/checkpoint_every + checkpoint_every states.
"""
from __future__ import annotations

import torch


def _step(bunch, U, nbr, dt, dx):
    """One update: guards refilled from owned values, then advanced; returns (U_in with
    guards, U_out with zero guards)."""
    Ug = U.clone()
    bunch.fill_guards(Ug, nbr)
    Uo = torch.zeros_like(U)
    bunch.update(Ug, Uo, dt, dx)
    return Ug, Uo


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, bunch, nbr, dt_seq, dx, k):
        n = dt_seq.shape[0]
        ckpt = []
        U = U0.detach()
        for s in range(n):
            if s % k == 0:
                ckpt.append(U)
            _, U = _step(bunch, U, nbr, dt_seq[s], dx)
        ctx.bunch, ctx.nbr, ctx.dx, ctx.k = bunch, nbr, dx, k
        ctx.dt_seq = dt_seq
        ctx.ckpt = ckpt
        return U

    @staticmethod
    def backward(ctx, lam):
        bunch, nbr, dx, k, dt_seq = ctx.bunch, ctx.nbr, ctx.dx, ctx.k, ctx.dt_seq
        n = dt_seq.shape[0]
        lam = lam.contiguous().clone()
        for seg in reversed(range(len(ctx.ckpt))):
            s0 = seg * k
            s1 = min(n, s0 + k)
            # recompute the inputs (guards filled) of the steps of this segment
            ins = []
            U = ctx.ckpt[seg]
            for s in range(s0, s1):
                Ug, U = _step(bunch, U, nbr, dt_seq[s], dx)
                ins.append(Ug)
            for s in reversed(range(s0, s1)):
                out = torch.empty_like(lam)
                bunch.adjoint(ins[s - s0], lam, out, dt_seq[s], dx)
                lam = out
            del ins
        ctx.ckpt = None
        return lam, None, None, None, None, None


def rollout(U0, bunch, nbr, dt_seq, dx, checkpoint_every=5):
    """Differentiable `len(dt_seq)`-step rollout of U0.

    U0: state tensor (owned entries meaningful); bunch: binding.Bunch with
    adjoint_bind(nbr_host) done; nbr: (P, 27) int32 device neighbour table; dt_seq:
    (nsteps, P) float64 device tensor of per-patch time steps; dx: (P, 3) float64 device."""
    return _Rollout.apply(U0, bunch, nbr, dt_seq, dx, int(checkpoint_every))
