"""Device tile orders (``lbm_tile_order``, host only): every order is a
permutation of the kept tiles, and each has the structure it is chosen for.
Within a step the tiles are updated independently (Section 3.1, Alg. 2), so
the order is free; the GPU tests check that results do not depend on it."""
import numpy as np
import pytest

from paper_1611_02445_amd import inputs as I
from paper_1611_02445_amd._abi import LbmError
from paper_1611_02445_amd.lattice import Tiling


def _tile_coords(t, perm):
    return t.arrays()["tile_xyz"][perm] // 4


def _dense(ntx, nty, ntz):
    return Tiling(np.zeros((4 * ntz, 4 * nty, 4 * ntx), np.uint8), 7)


@pytest.mark.parametrize("order", range(6))
def test_every_order_is_a_permutation_of_the_kept_tiles(order):
    s, _ = I.sphere_pack((40, 28, 52), 0.5, 2.0, 6.0, seed=3)
    t = Tiling(s, 7)
    assert 0 < t.n_tiles < t.tx * t.ty * t.tz  # some tiles are dropped
    p = t.device_order(order)
    assert p.dtype == np.int32 and np.array_equal(np.sort(p), np.arange(t.n_tiles))


def test_default_is_morton_and_order_one_is_discovery():
    s, _ = I.sphere_pack((32, 24, 40), 0.5, 2.0, 5.0, seed=14)
    t = Tiling(s, 7)
    assert np.array_equal(t.device_order(0), t.device_order(4))
    assert np.array_equal(t.device_order(1), np.arange(t.n_tiles))


@pytest.mark.parametrize("order", [4, 5])
@pytest.mark.parametrize("level", [1, 2])
def test_aligned_runs_of_both_curves_fill_cubes(order, level):
    """On a dense 16^3-tile box, every aligned run of 8^level consecutive
    device tiles fills a cube of edge 2^level (both curves recurse by octants)."""
    t = _dense(16, 16, 16)
    c = _tile_coords(t, t.device_order(order))
    n, e = 8 ** level, 2 ** level
    for k in range(0, len(c), n):
        blk = c[k:k + n]
        lo = blk.min(0)
        assert np.all(lo % e == 0) and np.all(blk.max(0) - lo == e - 1)
        assert len({tuple(v) for v in blk}) == n


def test_morton_key_is_the_bit_interleave():
    t = _dense(8, 4, 2)  # non-cubic grid
    c = _tile_coords(t, t.device_order(4))

    def key(x, y, z):
        k = 0
        for b in range(4):
            k |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
        return k

    keys = [key(*v) for v in c]
    assert keys == sorted(keys)


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_hilbert_steps_are_face_neighbours(n):
    """A Hilbert curve over a dense 2^b cube starts at the origin and every
    step moves to a face neighbour (Morton does not: it jumps)."""
    t = _dense(n, n, n)
    c = _tile_coords(t, t.device_order(5))
    assert tuple(c[0]) == (0, 0, 0)
    steps = np.abs(np.diff(c, axis=0)).sum(1)
    assert np.all(steps == 1)
    m = _tile_coords(t, t.device_order(4))
    assert np.abs(np.diff(m, axis=0)).sum(1).max() > 1


def test_hilbert_on_a_clipped_grid_keeps_most_steps_adjacent():
    """On a grid that is not a power-of-two cube the curve is clipped; the
    order is still a permutation and most consecutive tiles still touch."""
    t = _dense(6, 5, 3)
    c = _tile_coords(t, t.device_order(5))
    assert len({tuple(v) for v in c}) == 90
    steps = np.abs(np.diff(c, axis=0)).sum(1)
    assert np.mean(steps == 1) > 0.8


@pytest.mark.parametrize("order,S", [(2, 4), (3, 8)])
def test_slabs_keep_z_innermost_within_a_slab(order, S):
    t = _dense(3, 2, 9)  # the last slab is ragged
    c = _tile_coords(t, t.device_order(order))
    keys = [(z // S, y, x, z % S) for x, y, z in c]
    assert keys == sorted(keys)


def test_all_solid_box_has_an_empty_order():
    t = Tiling(np.ones((8, 8, 8), np.uint8), 7)
    assert t.n_tiles == 0
    for o in range(6):
        assert t.device_order(o).shape == (0,)


@pytest.mark.parametrize("order", [-1, 6])
def test_orders_outside_the_range_are_rejected(order):
    t = _dense(2, 2, 2)
    with pytest.raises(LbmError, match="LBM_E_INVAL.*order"):
        t.device_order(order)


def test_null_arguments_are_rejected_and_leave_the_output_untouched():
    import ctypes
    from paper_1611_02445_amd._abi import call
    t = _dense(2, 2, 2)
    perm = np.full(t.n_tiles, -7, dtype=np.int32)
    with pytest.raises(LbmError, match="LBM_E_INVAL"):
        call("lbm_tile_order", None, 0, perm.ctypes.data_as(ctypes.c_void_p))
    with pytest.raises(LbmError, match="LBM_E_INVAL.*NULL"):
        call("lbm_tile_order", t._ptr, 0, None)
    with pytest.raises(LbmError, match="LBM_E_INVAL"):
        call("lbm_tile_order", t._ptr, 9, perm.ctypes.data_as(ctypes.c_void_p))
    assert np.all(perm == -7)
