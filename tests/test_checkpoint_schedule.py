"""Host logic of the checkpointed reverse sweep: with a stand-in lattice whose
buffers only carry a time index, the sweep must hand the adjoint kernels
s_{T-1}, s_{T-2}, ..., s_0 in that order, never read a buffer that a later
recomputation has overwritten, re-run exactly the planned number of steps and
hold no more lattices than planned."""
import math

import pytest

from paper_1611_02445_amd.autograd import CheckpointedAdjoint, _recompute_cost, lattices_needed, plan_checkpoints


class Buf:
    def __init__(self, pool):
        self.t = None
        pool.append(self)

    def copy_(self, other):
        self.t = other.t


class FakeSizes:
    state_bytes = 1
    adjoint_bytes = 1
    grad_force_bytes = 1


class FakeLattice:
    """Records the library calls the sweep makes."""

    def __init__(self):
        self.states, self.adj = [], []
        self.cur = None
        self.seen = []
        self.steps = 0
        self.sizes = FakeSizes()

    def new_state(self):
        return Buf(self.states)

    def new_adjoint(self):
        return Buf(self.adj)

    def new_grad(self):
        return object()

    def current_state(self):
        return self.cur

    def set_state(self, f0, buf):
        buf.t = 0

    def step_buf(self, src, dst):
        assert src is not dst and src.t is not None
        dst.t = src.t + 1
        self.steps += 1

    def macroscopic(self, state=None, fields=False):
        return None, None, [0, 0, 0, 0, 1.0, 0, 0, 0.0]

    def adjoint_seed(self, s, e, g):
        self.seen.append(s.t)
        e.t = s.t + 1

    def adjoint_step(self, s, e_in, e_out, g):
        assert e_in is not e_out
        assert e_in.t == s.t + 2  # eta_{t} with s = s_{t-2}
        self.seen.append(s.t)
        e_out.t = s.t + 1

    def adjoint_final(self, e, out):
        assert e.t == 1 and out is not e
        out.t = 0

    def adjoint_get(self, buf):
        return buf.t

    def field_to_dense(self, buf, dtype=0):
        return None


@pytest.mark.parametrize("T,iv", [(1, (1,)), (7, (3,)), (12, (5,)), (12, (12,)), (23, (5, 2)), (40, (10, 3)),
                                  (41, (10, 4)), (2000, (100, 10)), (9, (4, 8)), (60, (20, 6, 2)), (61, (17, 5, 3)),
                                  (2000, (200, 30, 6)), (10, (10, 3, 1))])
def test_sweep_order_and_cost(T, iv):
    lat = FakeLattice()
    run = CheckpointedAdjoint(lat, T, *iv)
    run.forward(object())
    assert lat.steps == T and run.sT.t == T
    lat.steps = 0
    lam0, _ = run.backward()
    assert lat.seen == list(range(T - 1, -1, -1))
    assert lam0 == 0
    assert run.recompute_steps == lat.steps == _recompute_cost(T, *run.intervals)
    assert len(lat.states) == run.lattices() == lattices_needed(T, *iv)
    assert len(lat.adj) == 2
    if len(run.intervals) == 1:
        assert run.recompute_steps == T - run.n_ckpt


def _brute_best(T, budget, levels):
    if levels == 1:
        return min((_recompute_cost(T, k), (k,)) for k in range(1, T + 1) if lattices_needed(T, k) <= budget)
    return min((_recompute_cost(T, k, k2), (k, k2)) for k in range(2, T + 1) for k2 in range(1, k)
               if lattices_needed(T, k, k2) <= budget)


@pytest.mark.parametrize("T,budget", [(2000, 100), (2000, 45), (2000, 40), (50, 12), (10, 8)])
def test_plan_fits_and_is_no_worse_than_neighbours(T, budget):
    iv = plan_checkpoints(T, budget)
    assert lattices_needed(T, *iv) <= budget
    cost = _recompute_cost(T, *iv)
    if any(lattices_needed(T, k) <= budget for k in range(1, T + 1)):
        assert len(iv) == 1 and cost == _brute_best(T, budget, 1)[0]
    else:
        assert len(iv) == 2 and cost == _brute_best(T, budget, 2)[0]


def test_plan_three_levels_when_two_do_not_fit():
    T, budget = 2000, 30  # two levels need at least 38 lattices here
    with pytest.raises(ValueError):
        plan_checkpoints(T, budget, max_levels=2)
    iv = plan_checkpoints(T, budget)
    assert len(iv) == 3 and lattices_needed(T, *iv) <= budget
    assert _recompute_cost(T, *iv) <= 3 * T


def test_plan_rejects_impossible_budget():
    with pytest.raises(ValueError):
        plan_checkpoints(10, 4)


def test_one_level_cost_closed_form():
    for T in (1, 5, 17, 100):
        for K in (1, 2, 3, 7, 100):
            assert _recompute_cost(T, min(K, T)) == T - math.ceil(T / min(K, T))
