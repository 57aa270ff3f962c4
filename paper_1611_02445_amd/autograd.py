"""Gradient of the mean fluid x-velocity after T steps, with checkpointing.

Forward map (one fused step of the library): s_t = C(S s_{t-1}, F), with S the
pull streaming with bounce-back and C the local collision of the lattice's
model (LBGK or LBMRT, either equilibrium) with Guo forcing.  The loss is
L = (1/N_fluid) sum_fluid u_x(s_T).  The reverse sweep runs the library's
adjoint kernels:

    seed(s_{T-1})                    -> eta_T,      grad_g  = ...
    step(s_{t-2}, eta_t), t = T..2   -> eta_{t-1},  grad_g += ...
    final(eta_1)                     -> lambda_0 = dL/ds_0

It needs the states s_{T-1}, ..., s_0 in decreasing order.  The forward pass
keeps every K-th state (checkpoints s_0, s_K, s_2K, ...).  With one level the
backward pass recomputes one segment of K states at a time from its
checkpoint into a ring of buffers and consumes it from the top: one extra
forward step per adjoint step, ceil(T/K) + K + 1 lattices.  Each further level
(intervals K > K2 > K3 ...) first re-runs a segment once keeping every
K2-th state and then treats each sub-segment the same way, down to a ring of
the last interval: about one more forward step per adjoint step per level,
for ceil(T/K) + ceil(K/K2) + ... + K_last lattices.  ``plan_checkpoints``
picks the intervals with the least recomputation that fit a lattice budget.

This module only orders library calls; every step, adjoint step, conversion
and reduction runs in the HIP library.
"""
import functools
import math

import torch

from .lattice import Lattice


def _intervals(T, K, inner):
    """Normalised checkpoint intervals: K capped at T, then each inner interval
    strictly below the previous one (others dropped)."""
    out = [int(min(K, T))]
    for k in inner:
        if k is None:
            continue
        if k < 1:
            raise ValueError("checkpoint intervals must be >= 1")
        if k < out[-1]:
            out.append(int(k))
    return out


@functools.lru_cache(maxsize=None)
def _segment_cost(length, inner):
    """Forward steps re-run to hand out the `length` states of a segment, given
    the inner intervals below its level (a tuple; empty = ring)."""
    if not inner:
        return length - 1
    K = inner[0]
    n = math.ceil(length / K)
    cost = (n - 1) * K  # one pass to the segment's last inner checkpoint
    full = length // K
    cost += full * _segment_cost(K, inner[1:])
    if length % K:
        cost += _segment_cost(length % K, inner[1:])
    return cost


def _recompute_cost(T, K, *inner):
    """Forward steps re-run by the backward pass for checkpoint intervals
    (K, K2, ...); no inner interval (or None) = one level."""
    iv = _intervals(T, K, inner)
    K, rest = iv[0], tuple(iv[1:])
    cost = (T // K) * _segment_cost(K, rest)
    if T % K:
        cost += _segment_cost(T % K, rest)
    return cost


def lattices_needed(T, K, *inner):
    """Forward-state lattices held at once (checkpoints of every level, the
    ring and two step buffers), for T steps."""
    iv = _intervals(T, K, inner)
    n = math.ceil(T / iv[0])
    for a, b in zip(iv[:-1], iv[1:]):
        n += math.ceil(a / b) - 1
    return n + (iv[-1] - 1) + 2


def plan_checkpoints(T, max_lattices, max_levels=3):
    """Checkpoint intervals (a tuple K, K2, ...) for T adjoint steps within
    max_lattices forward lattices, with the fewest levels that fit and, among
    those, the least recomputation.  Raises when max_levels do not fit."""
    T, M = int(T), int(max_lattices)
    for K in range(1, T + 1):  # one level: the smallest K that fits
        if lattices_needed(T, K) <= M:
            return (K,)
    if max_levels < 2:
        raise ValueError(f"{T} adjoint steps do not fit in {M} lattices with one level")
    best = None
    # every K for moderate T; for long horizons the K that start a new count
    # of checkpoints (the search would otherwise take T * M cost evaluations)
    ks = range(2, T + 1) if T <= 20000 else sorted({math.ceil(T / n) for n in range(1, M + 1)})
    for K in ks:
        if K < 2 or math.ceil(T / K) + 2 > M:
            continue
        for K2 in range(1, min(K, M)):
            if lattices_needed(T, K, K2) <= M:
                c = _recompute_cost(T, K, K2)
                if best is None or c < best[0]:
                    best = (c, (K, K2))
    if best is not None:
        return best[1]
    if max_levels >= 3:
        ks = sorted({math.ceil(T / n) for n in range(1, M + 1)})
        for K in ks:
            if K < 3 or math.ceil(T / K) + 2 > M:
                continue
            for K2 in sorted({math.ceil(K / n) for n in range(2, M + 1)}):
                if K2 < 2 or K2 >= K:
                    continue
                for K3 in range(1, min(K2, M)):
                    if lattices_needed(T, K, K2, K3) <= M:
                        c = _recompute_cost(T, K, K2, K3)
                        if best is None or c < best[0]:
                            best = (c, (K, K2, K3))
        if best is not None:
            return best[1]
    raise ValueError(f"{T} adjoint steps do not fit in {M} lattices with {max_levels} levels")


class CheckpointedAdjoint:
    """Forward run with checkpoints and the matching reverse sweep on a Lattice
    (FP64 or FP32 storage, any collision model).  Intervals: K for the
    forward checkpoints, then optional inner intervals K2 > K3 > ..."""

    def __init__(self, lat: Lattice, T: int, K: int, *inner):
        if T < 1:
            raise ValueError("T must be >= 1")
        if K < 1:
            raise ValueError("checkpoint intervals must be >= 1")
        self.lat, self.T = lat, int(T)
        self.intervals = _intervals(self.T, K, inner)
        self.K = self.intervals[0]
        self.K2 = self.intervals[1] if len(self.intervals) > 1 else None
        self.n_ckpt = math.ceil(self.T / self.K)
        self.ckpt = [lat.new_state() for _ in range(self.n_ckpt)]  # s_0, s_K, ...
        # inner level j keeps ceil(K_{j-1}/K_j) - 1 states besides its parent's
        self.inner_ckpt = [[lat.new_state() for _ in range(math.ceil(a / b) - 1)]
                           for a, b in zip(self.intervals[:-1], self.intervals[1:])]
        # ring slot 0 is always a checkpoint buffer of the level above
        self.ring = [lat.new_state() for _ in range(self.intervals[-1] - 1)]
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
        return cls(lat, T, *plan_checkpoints(T, max(int(avail // max(s.state_bytes, 1)), 0)))

    def lattices(self):
        return len(self.ckpt) + sum(len(b) for b in self.inner_ckpt) + len(self.ring) + len(self.tmp)

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

    def _segment_reversed(self, first, length, level):
        """The `length` states of a segment starting with the state in buffer
        `first`, last first; `level` indexes the inner intervals."""
        if level + 1 >= len(self.intervals):
            yield from reversed(self._ring(first, length))
            return
        K = self.intervals[level + 1]
        n = math.ceil(length / K)
        keep = [first] + self.inner_ckpt[level][:n - 1]
        cur, spare = first, 0
        for r in range(1, (n - 1) * K + 1):
            if r % K == 0:
                nxt = keep[r // K]
            else:
                nxt = self.tmp[spare]
                spare ^= 1
            self.lat.step_buf(cur, nxt)
            cur = nxt
        self.recompute_steps += (n - 1) * K
        for m in range(n - 1, -1, -1):
            yield from self._segment_reversed(keep[m], min(K, length - m * K), level + 1)

    def _states_reversed(self):
        """s_{T-1}, s_{T-2}, ..., s_0 (buffers valid until the next item)."""
        for j in range(self.n_ckpt - 1, -1, -1):
            yield from self._segment_reversed(self.ckpt[j], min(self.K, self.T - j * self.K), 0)

    def backward(self, dense=True):
        """Reverse sweep; returns (dL/ds0 dense [19,...], dL/dg dense [3,...]),
        or with dense=False the library's own buffers: the adjoint lattice
        holding dL/ds0 and the FP64 gradient in per-node-field order (one
        entry per fluid node and component; lattice.field_to_dense)."""
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
            return e_nxt, self.grad
        g_f0 = lat.adjoint_get(e_nxt)
        g_g = lat.field_to_dense(self.grad, 0)
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
