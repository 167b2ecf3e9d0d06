"""Full-waveform-inversion misfit as a torch.autograd.Function.

The forward pass builds a solver for the given per-cell material, runs the
library's `dgt_fwi_gradient` (forward run, checkpointed reversal with the
reversed chain, FP64 gradient accumulation) and returns the misfit; the backward
pass scales the gradient the library computed.  Argument marshalling only: every
step runs in the library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import dgtile as D


@dataclass
class FwiSetup:
    mesh: D.Mesh
    degree: int
    dt: float
    shots_xy: np.ndarray            # [nshots, 2]
    rec_xy: np.ndarray              # [nrec, 2]
    nsteps: int
    observed: torch.Tensor          # [nshots, nsteps, nrec, 2] FP64 on the GPU
    time_order: int = 4
    precision: int = 0              # 0 FP64 state, 1 FP32 state (gradient in FP64 either way)
    nsnap: int = 32
    mode: int = 1                   # 0 untiled, 1 tiled
    tile_size: int = 128
    splits: tuple = (13,)
    schedule: int = 0
    free_sides: int = 0xF           # the adjoint needs free-surface (or periodic) boundaries
    f0: float = 5.0
    t0: float = 0.2
    amp: float = 1.0
    last: dict = field(default_factory=dict)


def make_solver(setup: FwiSetup, lam, mu, rho) -> D.Solver:
    s = D.Solver(setup.mesh, lam, mu, rho, degree=setup.degree, flux=0, time_order=setup.time_order,
                 precision=setup.precision, free_sides=setup.free_sides, dt=setup.dt)
    xy = np.asarray(setup.shots_xy, np.float64).reshape(-1, 2)
    s.set_shots(len(xy), xy, setup.f0, setup.t0, setup.amp)
    if setup.mode == 1:
        s.inspect(setup.tile_size, partition=1, splits=setup.splits)
        s.set_schedule(setup.schedule)
    return s


class FWIMisfit(torch.autograd.Function):
    """J(lam, mu, rho) = 1/2 sum over shots, steps and receivers of |r - d|^2."""

    @staticmethod
    def forward(ctx, lam, mu, rho, setup: FwiSetup):
        host = [t.detach().to("cpu", torch.float64).numpy() for t in (lam, mu, rho)]
        s = make_solver(setup, *host)
        J, gl, gm, gr = s.fwi_gradient(setup.rec_xy, setup.nsteps, setup.observed, setup.nsnap, setup.mode)
        setup.last = dict(misfit=J)
        ctx.save_for_backward(gl.to(lam.device, lam.dtype), gm.to(mu.device, mu.dtype), gr.to(rho.device, rho.dtype))
        return torch.tensor(J, dtype=torch.float64, device=lam.device)

    @staticmethod
    def backward(ctx, gJ):
        gl, gm, gr = ctx.saved_tensors
        return gJ * gl, gJ * gm, gJ * gr, None


def misfit(lam, mu, rho, setup: FwiSetup):
    return FWIMisfit.apply(lam, mu, rho, setup)
