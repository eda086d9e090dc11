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
forward replay of every step; storage: about 2 sqrt(nsteps) states (3 sqrt(nsteps)
with overlap).

Overlap (default): the replay of the next segment (the one before, in time)
runs on a second HIP stream of default priority, through a second library
context, into the other of two segment buffers, while the adjoint steps of the
current segment run on the solver's stream.  Events order the two: an adjoint
segment waits for its replay, and a replay into a buffer waits for the adjoint
segment that last read it.  The kernels and their inputs are the same, so the
gradient is bit for bit that of the serial schedule.

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

    def __init__(self, solver, nsteps, checkpoint_every=None, overlap=True):
        if solver.params.get("retarget_every", 1) != 0:
            raise ValueError("the differentiable rollout needs a frozen link speed (retarget_every=0)")
        self.s = solver
        self.nsteps = int(nsteps)
        self.K = int(checkpoint_every) if checkpoint_every else max(1, math.ceil(math.sqrt(max(self.nsteps, 1))))
        self.overlap = bool(overlap)

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

    def _side_solver(self):
        # one side stream and context per solver, kept on it across rollouts
        side = getattr(self.s, "_rollout_side", None)
        if side is None:
            from .solver import Solver
            stream = torch.cuda.Stream()   # default priority
            side = (stream, Solver(stream=stream, **dict(self.s.params)))
            self.s._rollout_side = side
        return side

    def backward(self, W0, checkpoints, WN_bar):
        starts = sorted(checkpoints, reverse=True)
        if self.overlap and len(starts) > 1 and self.K > 1:
            return self._backward_overlapped(W0, checkpoints, starts, WN_bar)
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

    def _backward_overlapped(self, W0, checkpoints, starts, WN_bar):
        s = self.s
        side, s2 = self._side_solver()
        main = s.stream
        lam, lam2 = s.new_populations(), s.new_populations()
        s.raw_moments_adjoint(WN_bar.contiguous(), lam)
        sets = [[self._new() for _ in range(self.K)] for _ in range(2)]
        ready = [torch.cuda.Event() for _ in range(2)]
        free = [None, None]   # event: the adjoint segment that last read the buffer is done
        side.wait_stream(main)   # checkpoints, buffers and lam are ready on the solver's stream

        def replay(b, start):
            end = min(start + self.K, self.nsteps)
            seg = sets[b]
            with torch.cuda.stream(side):
                if free[b] is not None:
                    side.wait_event(free[b])
                ck = checkpoints[start]
                seg[0].f.copy_(ck.f)
                seg[0].norms.copy_(ck.norms)
                for n in range(start, end - 1):
                    a, c = seg[n - start], seg[n - start + 1]
                    s2.raw_step(a.f, a.norms, c.f, c.norms)
                ready[b].record(side)

        replay(0, starts[0])
        for i, start in enumerate(starts):
            b = i % 2
            if i + 1 < len(starts):
                replay(1 - b, starts[i + 1])
            main.wait_event(ready[b])
            end = min(start + self.K, self.nsteps)
            seg = sets[b]
            for n in range(end - 1, start - 1, -1):
                st = seg[n - start]
                s.raw_adjoint_step(st.f, st.norms, lam, lam2)
                lam, lam2 = lam2, lam
            ev = torch.cuda.Event()
            ev.record(main)
            free[b] = ev
        main.wait_stream(side)
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


def rollout(W0, solver, nsteps, checkpoint_every=None, overlap=True):
    """Differentiable W0 -> W(nsteps) for a frozen-link-speed Solver."""
    return _RolloutFn.apply(W0, Rollout(solver, nsteps, checkpoint_every, overlap))
