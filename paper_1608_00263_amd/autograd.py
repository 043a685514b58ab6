"""PyTorch autograd binding of the adjoint gradient.

The loss is the sample cross entropy of Eqs. (ae) and (5),
L(theta) = ln S - (1/k) sum_i ln p_theta(x_i), for a circuit whose
parametrised gates are rotations exp(-i theta_j G_j / 2) (Sec. V): the
forward runs the circuit on the GPU and evaluates the cross entropy; the
backward runs the library's adjoint pass on the output state the forward
left behind, so the state is computed once per step.  For a unitary circuit
S = 1, so the gradient is that of -(1/k) sum ln p_theta(x_i).

Argument marshalling only: both passes are calls of the C library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import sv


class _Stamp:
    """Which forward's output state the module's GPU state holds: the
    generation number of that forward, or None once anything else (a later
    forward's backward, an uncomputation) has changed the contents."""

    def __init__(self):
        self.last = 0        # generation of the most recent forward
        self.ready = None    # generation whose output the state holds


class _CircuitCrossEntropy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, circ, state, samples, checkpoint_c, stamp):
        c = circ.with_theta(theta.detach().to("cpu", torch.float64).numpy())
        args = sv.CircuitArgs(c)   # marshalled once for both passes
        stamp.last += 1
        stamp.ready = None
        if checkpoint_c > 0:
            # the forward pass of the adjoint, keeping its state copies
            state.forward_checkpoints(c, checkpoint_c, args=args)
        else:
            state.apply(c, "auto", from_zero=True, args=args)
        ce, _, zeros = state.cross_entropy(samples)
        if zeros:
            raise sv.SVError(sv.SV_ESTATE, "a sample has probability 0 under the circuit")
        stamp.ready = stamp.last
        ctx.gen = stamp.last
        ctx.stamp = stamp
        ctx.circ = c
        ctx.args = args
        ctx.state = state
        ctx.samples = samples
        ctx.checkpoint_c = checkpoint_c
        ctx.theta_meta = (theta.dtype, theta.device)
        return torch.tensor(ce, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        # the forward state (and its checkpoints) is reused only while the
        # handle still holds this forward's output (no later forward, no
        # earlier backward, which uncomputes it); otherwise the backward
        # recomputes it from |0..0>
        ready = ctx.stamp.ready == ctx.gen
        ctx.stamp.ready = None
        _, grad = ctx.state.backward(ctx.circ, ctx.samples, checkpoint_c=ctx.checkpoint_c,
                                     state_ready=ready, args=ctx.args)
        dtype, device = ctx.theta_meta
        gt = torch.from_numpy(np.asarray(grad, dtype=np.float64)).to(device=device, dtype=dtype)
        return g.to(device=device, dtype=dtype) * gt, None, None, None, None, None


class CircuitCrossEntropy(torch.nn.Module):
    """theta -> L(theta) on fixed samples, differentiable by the adjoint method.

    circ: a parametrised circuit (its theta is replaced by the input);
    samples: uint64 bit-strings; checkpoint_c: the backward pass reuses the
    forward state while the module's state still holds that forward's output
    (after another forward or backward it is recomputed); with c > 0 the
    forward also keeps a state copy every c cycles, which bounds the drift of
    the uncomputation.  The module owns one GPU state of the circuit's size.
    """

    def __init__(self, circ, samples, dtype: str = "c64", checkpoint_c: int = 0):
        super().__init__()
        self.circ = circ
        self.samples = np.ascontiguousarray(samples, dtype=np.uint64)
        self.checkpoint_c = int(checkpoint_c)
        self.state = sv.State(circ.n, dtype)
        self._stamp = _Stamp()

    def forward(self, theta: torch.Tensor) -> torch.Tensor:
        if theta.numel() != self.circ.nparams:
            raise ValueError("theta has %d entries, the circuit %d parameters"
                             % (theta.numel(), self.circ.nparams))
        return _CircuitCrossEntropy.apply(theta, self.circ, self.state, self.samples, self.checkpoint_c,
                                          self._stamp)

    def close(self):
        self.state.close()
