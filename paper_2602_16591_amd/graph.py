"""One compute call of a plan captured into a HIP graph and replayed.

The compute entry points only enqueue kernels: no allocation, no host synchronisation and no
memset nodes (the work buffers are cleared by the kernels that consume them), so the call,
captured once with torch.cuda.CUDAGraph on the caller's stream, replays as a single graph
launch. Inputs are copied into the captured input buffers before a replay; the outputs are
the captured output buffers, overwritten by every replay.
"""
from __future__ import annotations


class CapturedCompute:
    """plan.compute(pos, q, **kw) as a replayable graph (plan: Plan or BatchPlan).

    Stage timing of the plan must be off while capturing (events would be captured too)."""

    def __init__(self, plan, pos, q, **kw):
        import torch
        self.plan = plan
        self.pos = pos.detach().clone()
        self.q = q.detach().clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plan.compute(self.pos, self.q, **kw)   # a plain run first, outside the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.outputs = plan.compute(self.pos, self.q, **kw)
        torch.cuda.synchronize()

    def __call__(self, pos=None, q=None):
        """Replays the graph on the current stream (after copying new inputs, if given) and
        returns the output tensors (phi, vec, energy)."""
        if pos is not None:
            self.pos.copy_(pos)
        if q is not None:
            self.q.copy_(q)
        self.graph.replay()
        return self.outputs
