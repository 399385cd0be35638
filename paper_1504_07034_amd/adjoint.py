"""Gradients of a flow objective through the LBRS time loop.

The objective is J = sum of rho(x, T)^2 over the cells whose centres lie in a
window, after T fixed-speed D2Q4 steps on a periodic domain, as a function of
the initial density rho0 of a gas at rest with p = rho^gamma/gamma.  The lattice
speed is frozen at lambda*(U0)/cfl of the reference (unperturbed) initial state
so that the step map is smooth and dt is fixed.

`LBRSFunction` wraps the library's checkpointed sweeps in torch.autograd:
forward  -- lbrs_isentropic_to_cons, lbrs_init, lbrs_forward_checkpointed
            (population snapshots every `segment` ~ sqrt(T) steps) and
            lbrs_window_objective (J and dJ/df^T);
backward -- lbrs_backward_checkpointed (per segment: recompute with a U^n
            tape, then reverse adjoint steps), lbrs_adjoint_init and
            lbrs_isentropic_to_cons_adjoint.
Memory: ceil(T/segment) population sets plus `segment` moment sets.

With `store_all` the forward sweep keeps every step's moments instead
(lbrs_forward_taped: T moment sets, 32 B per cell and step -- 250 GiB for
2048^2 cells and 2000 steps, which the device's HBM holds) and the backward
sweep runs straight through that tape (lbrs_backward_taped): no recompute.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import lbrs


def window_range(n: int, lo: float, hi: float, x0: float = 0.0, x1: float = 1.0):
    """Index range [i0, i1) of the cells whose centres lie in the closed [lo, hi]."""
    dx = (x1 - x0) / n
    c = x0 + (np.arange(n) + 0.5) * dx
    idx = np.nonzero((c >= lo) & (c <= hi))[0]
    if idx.size == 0:
        raise ValueError("empty window")
    return int(idx[0]), int(idx[-1]) + 1


@dataclass
class GradientSpec:
    n: int                      # cells per side, domain [0,1]^2, periodic
    steps: int                  # T
    window: tuple = (0.7, 0.8)  # closed square [lo, hi]^2 of cell centres
    gamma: float = 1.4
    omega: float = 1.0
    cfl: float = 0.5
    layout: int = lbrs.LBRS_LAYOUT_ROWS
    segment: int | None = None  # checkpoint spacing; default ceil(sqrt(T)), rounded up to a
                                # multiple of the steps per launch
    lam: float | None = None    # frozen lattice speed; set by prepare()
    tile: tuple | None = None   # (rows_per_tile, waves_per_block, alternate) of the step kernel
    fuse: int = 1               # steps per launch of the plain forward steps (1 to 4)
    store_all: bool | None = False  # keep every step's moments (None: if they fit)

    def params(self, mode, lam_user=0.0):
        return lbrs.make_params(lbrs.LBRS_D2Q4, self.n, self.n, (0.0, 1.0, 0.0, 1.0), self.gamma,
                                self.omega, self.cfl, (1, 1, 1, 1), mode, lam_user, self.layout)

    @property
    def seg(self) -> int:
        if self.segment:
            return self.segment
        f = max(1, self.fuse)
        return min(self.steps, math.ceil(math.ceil(math.sqrt(self.steps)) / f) * f)


class GradientRunner:
    """Device buffers and the library context for one GradientSpec."""

    def __init__(self, spec: GradientSpec, rho_ref: torch.Tensor):
        self.spec = spec
        n = spec.n
        dev = rho_ref.device
        # frozen lattice speed of the reference state (the library computes it)
        probe = lbrs.Sim(lbrs.LBRS_D2Q4, n, n, gamma=spec.gamma, omega=spec.omega, cfl=spec.cfl,
                         bc=(1, 1, 1, 1), lambda_mode=lbrs.LBRS_LAMBDA_FROZEN_INIT,
                         layout=spec.layout, device=dev)
        U = torch.empty((4, n, n), dtype=torch.float64, device=dev)
        lbrs.lbrs_isentropic_to_cons(probe.p, rho_ref.contiguous(), U)
        probe.init(U)
        spec.lam = probe.state()["lambda"]
        probe.close()
        del probe
        self.sim = lbrs.Sim(lbrs.LBRS_D2Q4, n, n, gamma=spec.gamma, omega=spec.omega, cfl=spec.cfl,
                            bc=(1, 1, 1, 1), lambda_mode=lbrs.LBRS_LAMBDA_USER,
                            lambda_user=spec.lam, layout=spec.layout, device=dev)
        if spec.tile is not None:
            self.sim.set_tile(*spec.tile)
        self.sim.set_fusion(spec.fuse)
        fcount = 16 * n * n
        tape_all = spec.steps * 4 * n * n
        if spec.store_all is None:
            # every step's moments if they fit beside the buffers below with
            # 2 GiB to spare
            torch.cuda.empty_cache()
            free, _ = torch.cuda.mem_get_info(dev)
            self.store_all = 8 * (tape_all + 4 * fcount) + (2 << 30) <= free
        else:
            self.store_all = bool(spec.store_all)
        self.tape = None
        if self.store_all:
            self.ckpt = None
            try:
                self.tape = torch.empty(tape_all, dtype=torch.float64, device=dev)
            except torch.cuda.OutOfMemoryError:
                if spec.store_all:
                    raise
                self.store_all = False  # automatic choice: fall back to checkpoints
                torch.cuda.empty_cache()
        self._seg = None
        if not self.store_all:
            self._alloc_segments()
        self.fbar = torch.empty(fcount, dtype=torch.float64, device=dev)
        self.work = torch.empty(fcount, dtype=torch.float64, device=dev)
        self.U0 = torch.empty((4, n, n), dtype=torch.float64, device=dev)
        self.J = torch.zeros(1, dtype=torch.float64, device=dev)
        self.win = window_range(n, *spec.window)

    def _alloc_segments(self):
        """Checkpoints and the segment tape for the spec's segment length."""
        spec, n = self.spec, self.spec.n
        if self._seg == spec.seg:
            return
        dev = self.sim.device
        self.ckpt = self.tape = None
        nck = math.ceil(spec.steps / spec.seg)
        self.ckpt = torch.empty(nck * 16 * n * n, dtype=torch.float64, device=dev)
        self.tape = torch.empty(spec.seg * 4 * n * n, dtype=torch.float64, device=dev)
        self._seg = spec.seg

    def forward(self, rho0: torch.Tensor, keep: bool = True) -> torch.Tensor:
        s, sim = self.spec, self.sim
        lbrs.lbrs_isentropic_to_cons(sim.p, rho0.contiguous(), self.U0)
        sim.init(self.U0)
        if keep and self.store_all:
            lbrs.lbrs_forward_taped(sim.ctx, s.steps, self.tape)
        elif keep:
            lbrs.lbrs_forward_checkpointed(sim.ctx, s.steps, s.seg, self.ckpt)
        else:
            sim.step(s.steps)
        i0, i1 = self.win
        lbrs.lbrs_window_objective(sim.ctx, i0, i1, i0, i1, self.J, self.fbar)
        return self.J.clone()

    def backward(self, rho0: torch.Tensor) -> torch.Tensor:
        s, sim = self.spec, self.sim
        if self.store_all:
            lbrs.lbrs_backward_taped(sim.ctx, s.steps, self.tape, self.fbar, self.work)
        else:
            lbrs.lbrs_backward_checkpointed(sim.ctx, s.steps, s.seg, self.ckpt, self.tape,
                                            self.fbar, self.work)
        Ubar0 = torch.empty_like(self.U0)
        lbrs.lbrs_adjoint_init(sim.ctx, self.fbar, self.U0, Ubar0)
        rbar = torch.empty_like(rho0)
        lbrs.lbrs_isentropic_to_cons_adjoint(sim.p, rho0.contiguous(), Ubar0, rbar)
        return rbar

    def tune(self, rho0: torch.Tensor, steps: int = 10) -> dict:
        """Autotune the step kernel's launch shape on this runner's problem
        (from the initial state of rho0; the caller's results are unaffected)."""
        from . import autotune
        lbrs.lbrs_isentropic_to_cons(self.sim.p, rho0.contiguous(), self.U0)
        self.sim.init(self.U0)
        best = autotune.tune(self.sim, steps=steps, use_cache=False)
        self.spec.tile = (best["rows"], best["wpb"], best["alt"])
        self.spec.fuse = best["fuse"]
        if not self.store_all:
            self._alloc_segments()  # the default segment follows the steps per launch
        return best

    def close(self):
        self.sim.close()
        self.ckpt = self.tape = self.fbar = self.work = None


class LBRSFunction(torch.autograd.Function):
    """J(rho0) with a hand-written adjoint: J.backward() gives dJ/drho0."""

    @staticmethod
    def forward(ctx, rho0: torch.Tensor, runner: GradientRunner):
        J = runner.forward(rho0, keep=True)
        ctx.runner = runner
        ctx.save_for_backward(rho0)
        return J[0]

    @staticmethod
    def backward(ctx, gJ):
        (rho0,) = ctx.saved_tensors
        g = ctx.runner.backward(rho0)
        return gJ * g, None
