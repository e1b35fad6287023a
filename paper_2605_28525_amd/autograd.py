"""Differentiable rollout of the sparse-grid MPM step (torch.autograd.Function).

Forward: `steps` explicit steps from an initial state whose velocity is v0,
with Young's modulus E and friction angle phi, keeping a copy of the state
every `checkpoint` steps.  Backward: for each checkpoint segment, last first,
the segment is recomputed from its checkpoint on the library's tape (every
step's input state, and its build and grids in one tape slot per step), then
the hand-written adjoint transfers run step by step in reverse over the tape.
Gradients: dL/dE, dL/dphi (per degree) and dL/dv0 (in the initial particle
order).

The library reorders particles every step, and a recomputed segment need not
repeat the first pass's order: the compact block order follows the hash slots
that concurrent insertions claim, and the particles are stored block by block.
Adjoints are carried across segment boundaries by particle id.
"""
from __future__ import annotations

import torch

from . import mpm as M


class Rollout:
    """Holds an adjoint-enabled context and the initial state of one workload."""

    def __init__(self, w, steps: int, checkpoint: int = 50, block_capacity: int = 0, device="cuda"):
        self.w = w
        self.steps = int(steps)
        self.K = int(checkpoint)
        self.params = M.params_from_workload(w, block_capacity=block_capacity, flags=M.MPM_FLAG_ADJOINT)
        self.ctx = M.mpm_create(self.params)
        M.mpm_tape_reserve(self.ctx, self.K)
        self.init = M.ParticleSet.from_arrays(w.state(), device=device)
        self.dim, self.n = w.dim, w.n
        self.device = device
        self.nu = float(w.nu)
        self.dt = float(w.dt)
        self._bufs = [M.ParticleSet(w.dim, w.n, device) for _ in range(2)]
        self._bars = [M.ParticleSet(w.dim, w.n, device, zero=False) for _ in range(2)]
        self._pool = []   # states of one recomputed segment, allocated on first use
        self.param_bar = torch.zeros(2, dtype=torch.float32, device=device)
        self._arange = torch.arange(self.n, dtype=torch.long, device=device)
        self.checkpoints = []

    def close(self):
        if self.ctx:
            M.mpm_destroy(self.ctx)
            self.ctx = None

    def set_material(self, E: float, phi: float):
        M.mpm_set_material(self.ctx, float(E), self.nu, float(phi), self.dt)

    def run_forward(self, v0: torch.Tensor, E: float, phi: float, keep_checkpoints=True):
        """Returns the final ParticleSet (positions in a permuted order, ids carried)."""
        self.set_material(E, phi)
        a, b = self._bufs
        a.copy_(self.init)
        a.v.copy_(v0)
        a.id.copy_(torch.arange(self.n, dtype=torch.int32, device=self.device))
        self.checkpoints = []
        for s0 in range(0, self.steps, self.K):
            if keep_checkpoints:
                self.checkpoints.append(M.ParticleSet(self.dim, self.n, self.device).copy_(a))
            k = min(self.K, self.steps - s0)
            M.mpm_step(self.ctx, a.view(), b.view(), k)
            if k % 2 == 1:
                a, b = b, a
        self._bufs = [a, b]
        return a

    def backward(self, checkpoints, final_ids: torch.Tensor, x_bar: torch.Tensor, E: float, phi: float):
        """x_bar: dL/dx of the final state of the forward pass that kept
        `checkpoints` (same order as `final_ids`).  The material of that pass is
        set again, so other forward passes on this Rollout in between do not
        change the result.  Returns (dL/dE, dL/dphi, dL/dv0)."""
        if len(checkpoints) != (self.steps + self.K - 1) // self.K:
            raise ValueError("checkpoint list does not cover the rollout")
        self.set_material(E, phi)
        self.param_bar.zero_()
        bar_ids = final_ids.clone()
        bar, spare = self._bars
        for key in ("v", "C", "F", "tau"):
            getattr(bar, key).zero_()
        bar.x.copy_(x_bar)
        while len(self._pool) < self.K + 1:
            self._pool.append(M.ParticleSet(self.dim, self.n, self.device, zero=False))
        nseg = len(checkpoints)
        for si in range(nseg - 1, -1, -1):
            s0 = si * self.K
            k = min(self.K, self.steps - s0)
            states = self._pool[:k + 1]
            states[0].copy_(checkpoints[si])
            views = [st.view() for st in states]
            M.mpm_tape_forward(self.ctx, views)
            # align the incoming adjoint with the recomputed end state by id
            # (always applied, so that no host sync decides whether to)
            inv = torch.empty_like(bar_ids, dtype=torch.long)
            inv[bar_ids.long()] = self._arange
            perm = inv[states[-1].id.long()]
            for key in ("x", "v", "C", "F", "tau"):
                getattr(bar, key).copy_(getattr(bar, key)[:, perm])
            # every field of the input adjoint is overwritten; the result is in bar
            M.mpm_tape_adjoint(self.ctx, views, bar.view(), spare.view(), self.param_bar)
            bar_ids = states[0].id.clone()
        # the initial state is in the caller's order (ids 0..n-1)
        inv = torch.empty_like(bar_ids, dtype=torch.long)
        inv[bar_ids.long()] = self._arange
        v0_bar = bar.v[:, inv].clone()
        self._bars = [bar, spare]
        pb = self.param_bar.detach().cpu()
        return float(pb[0]), float(pb[1]), v0_bar


class _RolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, phi, v0, roll: Rollout):
        final = roll.run_forward(v0.detach(), float(E), float(phi))
        ctx.roll = roll
        # run_forward allocates a fresh checkpoint list every call and the final
        # state lives in buffers the next forward pass overwrites: keep the list,
        # the ids and the material of this pass, not the buffers
        ctx.checkpoints = roll.checkpoints
        ctx.material = (float(E), float(phi))
        ctx.ids = final.id.clone()
        # positions returned in the caller's particle order
        inv = torch.empty_like(ctx.ids, dtype=torch.long)
        inv[ctx.ids.long()] = torch.arange(roll.n, device=roll.device)
        ctx.inv = inv
        return final.x[:, inv].clone()

    @staticmethod
    def backward(ctx, grad_x):
        roll = ctx.roll
        # grad_x is in caller order; bring it to the final state's order
        x_bar = grad_x[:, ctx.ids.long()].contiguous()
        gE, gphi, gv0 = roll.backward(ctx.checkpoints, ctx.ids, x_bar, *ctx.material)
        dev = grad_x.device
        return (torch.tensor(gE, dtype=torch.float64, device=dev), torch.tensor(gphi, dtype=torch.float64, device=dev),
                gv0, None)


def rollout(E: torch.Tensor, phi: torch.Tensor, v0: torch.Tensor, roll: Rollout) -> torch.Tensor:
    """Final positions (d, n) in the caller's particle order, differentiable with
    respect to E, phi (degrees) and v0 (d, n)."""
    return _RolloutFn.apply(E, phi, v0, roll)
