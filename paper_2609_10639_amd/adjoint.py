"""Differentiable VLBM rollout on the GPU with the library's hand-written adjoint.

`rollout(W0, solver, nsteps)` maps the initial conserved field W0 (FP64 device
tensor, (D+2, ny, nx)) to W after `nsteps` frozen-link-speed steps (the solver
must be created with retarget_every = 0 and c_fixed).  Its backward pass runs
the adjoint step of the library (vlbm_raw_adjoint_step) in reverse order.

Memory: the states are kept with two-level (square-root) checkpointing, the
binomial schedule of revolve restricted to two levels: the forward pass stores
every K-th state (K = ceil(sqrt(nsteps)) by default); the backward pass
replays one segment of K steps at a time from its checkpoint into a segment
buffer and runs the adjoint steps of that segment backwards.  Cost: one extra
forward replay of every step; storage: about 2 sqrt(nsteps) states.

Only argument marshalling and the checkpoint schedule live here; every step of
the forward and adjoint computation runs in the library's HIP kernels.
"""
import math

import torch


class _State:
    __slots__ = ("f", "norms")

    def __init__(self, f, norms):
        self.f = f
        self.norms = norms


class Rollout:
    """Checkpointed forward/adjoint driver for one Solver (frozen link speed)."""

    def __init__(self, solver, nsteps, checkpoint_every=None):
        if solver.params.get("retarget_every", 1) != 0:
            raise ValueError("the differentiable rollout needs a frozen link speed (retarget_every=0)")
        self.s = solver
        self.nsteps = int(nsteps)
        self.K = int(checkpoint_every) if checkpoint_every else max(1, math.ceil(math.sqrt(max(self.nsteps, 1))))

    def _new(self):
        return _State(self.s.new_populations(), self.s.new_norms())

    def _step(self, a, b):
        self.s.raw_step(a.f, a.norms, b.f, b.norms)

    def forward(self, W0):
        """Returns W_N and the checkpoints (state n for n = 0, K, 2K, ...)."""
        s = self.s
        cur, nxt = self._new(), self._new()
        s.raw_init(W0, cur.f, cur.norms)
        checkpoints = {}
        for n in range(self.nsteps):
            if n % self.K == 0:
                checkpoints[n] = _State(cur.f.clone(), cur.norms.clone())
            self._step(cur, nxt)
            cur, nxt = nxt, cur
        WN = torch.empty((s.NK,) + s.shape, dtype=torch.float64, device="cuda")
        s.raw_moments(cur.f, WN)
        return WN, checkpoints

    def backward(self, W0, checkpoints, WN_bar):
        s = self.s
        lam, lam2 = s.new_populations(), s.new_populations()
        s.raw_moments_adjoint(WN_bar.contiguous(), lam)
        seg = [self._new() for _ in range(self.K)]
        for start in sorted(checkpoints, reverse=True):
            end = min(start + self.K, self.nsteps)
            ck = checkpoints[start]
            seg[0].f.copy_(ck.f)
            seg[0].norms.copy_(ck.norms)
            for n in range(start, end - 1):
                self._step(seg[n - start], seg[n - start + 1])
            for n in range(end - 1, start - 1, -1):
                st = seg[n - start]
                s.raw_adjoint_step(st.f, st.norms, lam, lam2)
                lam, lam2 = lam2, lam
        W0bar = torch.empty((s.NK,) + s.shape, dtype=torch.float64, device="cuda")
        s.raw_init_adjoint(W0.contiguous(), lam, W0bar)
        return W0bar


class _RolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, W0, runner):
        W0 = W0.detach().contiguous()
        WN, checkpoints = runner.forward(W0)
        ctx.runner = runner
        ctx.checkpoints = checkpoints
        ctx.save_for_backward(W0)
        return WN

    @staticmethod
    def backward(ctx, WN_bar):
        (W0,) = ctx.saved_tensors
        W0bar = ctx.runner.backward(W0, ctx.checkpoints, WN_bar.to(torch.float64))
        ctx.checkpoints = None
        return W0bar, None


def rollout(W0, solver, nsteps, checkpoint_every=None):
    """Differentiable W0 -> W(nsteps) for a frozen-link-speed Solver."""
    return _RolloutFn.apply(W0, Rollout(solver, nsteps, checkpoint_every))
