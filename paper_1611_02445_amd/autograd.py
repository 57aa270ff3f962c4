"""Gradient of the mean fluid x-velocity after T steps, with checkpointing.

Forward map (one fused step of the library): s_t = C(S s_{t-1}, F), with S the
pull streaming with bounce-back and C the local LBGK + Guo collision.  The loss
is L = (1/N_fluid) sum_fluid u_x(s_T).  The reverse sweep runs the library's
adjoint kernels:

    seed(s_{T-1})                    -> eta_T,      grad_g  = ...
    step(s_{t-2}, eta_t), t = T..2   -> eta_{t-1},  grad_g += ...
    final(eta_1)                     -> lambda_0 = dL/ds_0

It needs the states s_{T-1}, ..., s_0 in decreasing order.  The forward pass
keeps every K-th state (checkpoints s_0, s_K, s_2K, ...); the backward pass
recomputes one segment of K states at a time from its checkpoint into a ring
of K buffers and consumes it from the top, so the extra work is one forward
step per adjoint step and the memory is ceil(T/K) + K lattices.

This module only orders library calls; every step, adjoint step, conversion
and reduction runs in the HIP library.
"""
import math

import torch

from .lattice import Lattice


class CheckpointedAdjoint:
    """Forward run with checkpoints and the matching reverse sweep on a Lattice
    (FP64 storage, quasi-compressible model)."""

    def __init__(self, lat: Lattice, T: int, K: int):
        if T < 1:
            raise ValueError("T must be >= 1")
        if K < 1:
            raise ValueError("K must be >= 1")
        self.lat, self.T, self.K = lat, int(T), int(min(K, T))
        self.n_ckpt = math.ceil(self.T / self.K)
        self.ckpt = [lat.new_state() for _ in range(self.n_ckpt)]  # s_0, s_K, ...
        self.ring = [lat.new_state() for _ in range(self.K)]
        self.tmp = [lat.new_state(), lat.new_state()]
        self.eta = [lat.new_adjoint(), lat.new_adjoint()]
        self.lam0 = lat.new_adjoint()
        self.grad = lat.new_grad()
        self.forward_steps = 0
        self.recompute_steps = 0

    def memory_bytes(self):
        s = self.lat.sizes
        return ((self.n_ckpt + self.K + 2) * s.state_bytes + 3 * s.adjoint_bytes + s.grad_force_bytes)

    def forward(self, f0_dense=None):
        """Load s_0 (dense FP64 [19,nz,ny,nx], or the current lattice when None),
        run T steps and return the loss."""
        lat = self.lat
        if f0_dense is not None:
            lat.set_state(f0_dense, self.ckpt[0])
        else:
            self.ckpt[0].copy_(lat.current_state())
        cur = self.ckpt[0]
        spare = 0
        for t in range(1, self.T + 1):
            if t % self.K == 0 and t < self.T:
                nxt = self.ckpt[t // self.K]
            else:
                nxt = self.tmp[spare]
                spare ^= 1
            lat.step_buf(cur, nxt)
            cur = nxt
        self.forward_steps += self.T
        self.sT = cur
        _, _, sums = lat.macroscopic(state=cur, fields=False)
        return sums[7] / sums[4]

    def _segment(self, j):
        """Recompute s_{jK} .. s_{jK + len - 1} into the ring; returns len."""
        lat = self.lat
        start = j * self.K
        length = min(self.K, self.T - start)
        self.ring[0].copy_(self.ckpt[j])
        for r in range(1, length):
            lat.step_buf(self.ring[r - 1], self.ring[r])
        self.recompute_steps += length - 1
        return length

    def backward(self):
        """Reverse sweep; returns (dL/ds0 dense [19,...], dL/dg dense [3,...])."""
        lat = self.lat
        e_cur, e_nxt = self.eta
        # states needed, in order: s_{T-1} (seed), s_{T-2}, ..., s_0 (steps t = T..2)
        first = True
        for j in range(self.n_ckpt - 1, -1, -1):
            length = self._segment(j)
            for r in range(length - 1, -1, -1):
                s = self.ring[r]
                if first:
                    lat.adjoint_seed(s, e_cur, self.grad)
                    first = False
                else:
                    lat.adjoint_step(s, e_cur, e_nxt, self.grad)
                    e_cur, e_nxt = e_nxt, e_cur
        lat.adjoint_final(e_cur, self.lam0)
        g_f0 = lat.get_state(self.lam0)
        g_g = lat.tiles_to_dense(self.grad, 3, 0)
        return g_f0, g_g


class MeanVelocityLoss(torch.autograd.Function):
    """L(f0, g) = mean fluid x-velocity after T steps from the initial
    distributions f0 [19,nz,ny,nx] under the body-force field g [3,nz,ny,nx]
    (both FP64 on the device, padded box).  Backward returns dL/df0 and dL/dg
    from the hand-written adjoint with checkpoints every K steps."""

    @staticmethod
    def forward(ctx, f0, g, lat, T, K):
        lat.set_force(g.detach())
        run = CheckpointedAdjoint(lat, T, K)
        loss = run.forward(f0.detach())
        ctx.run = run
        return torch.tensor(loss, dtype=torch.float64, device=f0.device)

    @staticmethod
    def backward(ctx, grad_out):
        g_f0, g_g = ctx.run.backward()
        scale = grad_out.to(torch.float64)
        ctx.run = None
        return g_f0 * scale, g_g * scale, None, None, None


def mean_velocity_loss(f0, g, lat, T, K):
    return MeanVelocityLoss.apply(f0, g, lat, T, K)
