"""Gradient of the mean fluid x-velocity after T steps, with checkpointing.

Forward map (one fused step of the library): s_t = C(S s_{t-1}, F), with S the
pull streaming with bounce-back and C the local LBGK + Guo collision.  The loss
is L = (1/N_fluid) sum_fluid u_x(s_T).  The reverse sweep runs the library's
adjoint kernels:

    seed(s_{T-1})                    -> eta_T,      grad_g  = ...
    step(s_{t-2}, eta_t), t = T..2   -> eta_{t-1},  grad_g += ...
    final(eta_1)                     -> lambda_0 = dL/ds_0

It needs the states s_{T-1}, ..., s_0 in decreasing order.  The forward pass
keeps every K-th state (checkpoints s_0, s_K, s_2K, ...).  With one level the
backward pass recomputes one segment of K states at a time from its
checkpoint into a ring of buffers and consumes it from the top: one extra
forward step per adjoint step, ceil(T/K) + K + 1 lattices.  With a second
level (K2 < K) each segment is first re-run once keeping every K2-th state,
and then each sub-segment of K2 states is recomputed into the ring: about two
extra forward steps per adjoint step, ceil(T/K) + ceil(K/K2) + K2 lattices.
``plan_checkpoints`` picks (K, K2) with the least recomputation that fits a
lattice budget.

This module only orders library calls; every step, adjoint step, conversion
and reduction runs in the HIP library.
"""
import math

import torch

from .lattice import Lattice


def _recompute_cost(T, K, K2):
    """Forward steps re-run by the backward pass for checkpoint intervals
    (K, K2); K2 = None for one level."""
    def segment(length):
        if K2 is None:
            return length - 1
        n2 = math.ceil(length / K2)
        # one pass to the last second-level checkpoint, then each sub-segment
        return (n2 - 1) * K2 + (length - n2)
    cost = (T // K) * segment(K)
    if T % K:
        cost += segment(T % K)
    return cost


def lattices_needed(T, K, K2=None):
    """Forward-state lattices held at once (checkpoints, second-level
    checkpoints, ring and two step buffers), for T steps."""
    K = min(K, T)
    n1 = math.ceil(T / K)
    if K2 is None or K2 >= K:
        return n1 + (K - 1) + 2
    return n1 + (math.ceil(K / K2) - 1) + (K2 - 1) + 2


def plan_checkpoints(T, max_lattices):
    """(K, K2) for T adjoint steps within max_lattices forward lattices: one
    level when it fits (the smallest K that fits, i.e. the least recompute),
    else two levels with the least recompute.  Raises when even two levels do
    not fit."""
    T = int(T)
    for K in range(1, T + 1):
        if lattices_needed(T, K) <= max_lattices:
            return K, None
    best = None
    for K in range(2, T + 1):
        n1 = math.ceil(T / K)
        if n1 + 2 > max_lattices:
            continue
        for K2 in range(1, min(K, max_lattices)):
            if lattices_needed(T, K, K2) > max_lattices:
                continue
            c = _recompute_cost(T, K, K2)
            if best is None or c < best[0]:
                best = (c, K, K2)
    if best is None:
        raise ValueError(f"{T} adjoint steps do not fit in {max_lattices} lattices")
    return best[1], best[2]


class CheckpointedAdjoint:
    """Forward run with checkpoints and the matching reverse sweep on a Lattice
    (FP64 or FP32 storage, quasi-compressible model)."""

    def __init__(self, lat: Lattice, T: int, K: int, K2=None):
        if T < 1:
            raise ValueError("T must be >= 1")
        if K < 1 or (K2 is not None and K2 < 1):
            raise ValueError("checkpoint intervals must be >= 1")
        self.lat, self.T, self.K = lat, int(T), int(min(K, T))
        self.K2 = None if K2 is None or K2 >= self.K else int(K2)
        self.n_ckpt = math.ceil(self.T / self.K)
        self.ckpt = [lat.new_state() for _ in range(self.n_ckpt)]  # s_0, s_K, ...
        inner = self.K if self.K2 is None else self.K2
        # ring slot 0 is always a checkpoint buffer (first or second level)
        self.ring = [lat.new_state() for _ in range(inner - 1)]
        self.ckpt2 = [] if self.K2 is None else [lat.new_state() for _ in range(math.ceil(self.K / self.K2) - 1)]
        self.tmp = [lat.new_state(), lat.new_state()]
        self.eta = [lat.new_adjoint(), lat.new_adjoint()]
        self.grad = lat.new_grad()
        self.forward_steps = 0
        self.recompute_steps = 0

    @classmethod
    def within_memory(cls, lat: Lattice, T: int, free_bytes=None, reserve_bytes=4 << 30):
        """Sized to the device memory that is free now (less reserve_bytes):
        the checkpoint intervals come from plan_checkpoints."""
        if free_bytes is None:
            free_bytes, _ = torch.cuda.mem_get_info(lat.device)
        s = lat.sizes
        avail = free_bytes - reserve_bytes - 2 * s.adjoint_bytes - s.grad_force_bytes
        K, K2 = plan_checkpoints(T, max(int(avail // max(s.state_bytes, 1)), 0))
        return cls(lat, T, K, K2)

    def lattices(self):
        return len(self.ckpt) + len(self.ckpt2) + len(self.ring) + len(self.tmp)

    def memory_bytes(self):
        s = self.lat.sizes
        return self.lattices() * s.state_bytes + 2 * s.adjoint_bytes + s.grad_force_bytes

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

    def _ring(self, first, length):
        """Recompute the `length` states that start at buffer `first` into
        the ring; returns the buffers in time order."""
        bufs = [first] + self.ring[:length - 1]
        for r in range(1, length):
            self.lat.step_buf(bufs[r - 1], bufs[r])
        self.recompute_steps += length - 1
        return bufs

    def _states_reversed(self):
        """s_{T-1}, s_{T-2}, ..., s_0 (buffers valid until the next item)."""
        lat = self.lat
        for j in range(self.n_ckpt - 1, -1, -1):
            length = min(self.K, self.T - j * self.K)
            if self.K2 is None:
                yield from reversed(self._ring(self.ckpt[j], length))
                continue
            n2 = math.ceil(length / self.K2)
            level2 = [self.ckpt[j]] + self.ckpt2[:n2 - 1]
            cur, spare = self.ckpt[j], 0
            for r in range(1, (n2 - 1) * self.K2 + 1):
                if r % self.K2 == 0:
                    nxt = level2[r // self.K2]
                else:
                    nxt = self.tmp[spare]
                    spare ^= 1
                lat.step_buf(cur, nxt)
                cur = nxt
            self.recompute_steps += (n2 - 1) * self.K2
            for m in range(n2 - 1, -1, -1):
                yield from reversed(self._ring(level2[m], min(self.K2, length - m * self.K2)))

    def backward(self, dense=True):
        """Reverse sweep; returns (dL/ds0 dense [19,...], dL/dg dense [3,...]),
        or with dense=False the library's own buffers: the adjoint lattice
        holding dL/ds0 and the FP64 tile-order gradient [n_tiles, 3, 64]."""
        lat = self.lat
        e_cur, e_nxt = self.eta
        # states needed, in order: s_{T-1} (seed), s_{T-2}, ..., s_0 (steps t = T..2)
        first = True
        for s in self._states_reversed():
            if first:
                lat.adjoint_seed(s, e_cur, self.grad)
                first = False
            else:
                lat.adjoint_step(s, e_cur, e_nxt, self.grad)
                e_cur, e_nxt = e_nxt, e_cur
        lat.adjoint_final(e_cur, e_nxt)
        if not dense:
            return e_nxt, self.grad.view(-1, 3, 64)
        g_f0 = lat.adjoint_get(e_nxt)
        g_g = lat.tiles_to_dense(self.grad, 3, 0)
        return g_f0, g_g


class MeanVelocityLoss(torch.autograd.Function):
    """L(f0, g) = mean fluid x-velocity after T steps from the initial
    distributions f0 [19,nz,ny,nx] under the body-force field g [3,nz,ny,nx]
    (both FP64 on the device, padded box).  Backward returns dL/df0 and dL/dg
    from the hand-written adjoint with checkpoints every K steps (and every
    K2 steps inside a segment when K2 is given)."""

    @staticmethod
    def forward(ctx, f0, g, lat, T, K, K2=None):
        lat.set_force(g.detach())
        run = CheckpointedAdjoint(lat, T, K, K2)
        loss = run.forward(f0.detach())
        ctx.run = run
        return torch.tensor(loss, dtype=torch.float64, device=f0.device)

    @staticmethod
    def backward(ctx, grad_out):
        g_f0, g_g = ctx.run.backward()
        scale = grad_out.to(torch.float64)
        ctx.run = None
        return g_f0 * scale, g_g * scale, None, None, None, None


def mean_velocity_loss(f0, g, lat, T, K, K2=None):
    return MeanVelocityLoss.apply(f0, g, lat, T, K, K2)
