"""The library's host tiler (lbm_build_tiles) against the oracle tiler:
bit-exact tables on random and structured bitmaps (no GPU needed)."""
import numpy as np
import pytest

from oracle import tiles_ref as T
from paper_1611_02445_amd import inputs as I
from paper_1611_02445_amd._abi import LbmError
from paper_1611_02445_amd.lattice import Tiling


def _same(solid, periodic):
    a = Tiling(solid, periodic)
    t = a.arrays()
    r = T.build_tiles(solid, periodic)
    for k in ("tile_map", "tile_xyz", "nbr", "fluid_mask"):
        assert np.array_equal(t[k], r[k]), k
    assert (a.nx, a.ny, a.nz) == (r["nx"], r["ny"], r["nz"])
    assert a.n_tiles == r["n_tiles"] and a.n_fluid == r["n_fluid"]
    assert a.eta_t == r["eta_t"]


@pytest.mark.parametrize("seed", range(8))
def test_random_bitmaps(seed):
    rng = np.random.default_rng(seed)
    periodic = int(rng.integers(0, 8))
    shape = []
    for bit, ax in ((4, 0), (2, 1), (1, 2)):
        n = int(rng.integers(1, 6)) * 4 if periodic & bit else int(rng.integers(1, 23))
        shape.append(n)
    s = I.random_bitmap(tuple(shape), float(rng.uniform(0, 1)), seed)
    _same(s, periodic)


def test_structured_geometries():
    _same(I.square_channel(32), 7)
    _same(I.plane_channel(8, 10, 4), 5)
    sp, _ = I.sphere_pack((40, 36, 44), 0.4, 4.0, 12.0, seed=2)
    _same(sp, 7)
    _same(sp, 0)
    _same(np.ones((5, 5, 5), np.uint8), 0)
    _same(np.zeros((4, 4, 4), np.uint8), 7)
    one = np.ones((9, 10, 11), np.uint8)
    one[8, 9, 10] = 0
    _same(one, 0)


def test_invalid_arguments():
    with pytest.raises(LbmError, match="LBM_E_INVAL"):
        Tiling(np.zeros((4, 4, 6), np.uint8), 1)  # periodic x of length 6
    with pytest.raises(LbmError, match="LBM_E_INVAL"):
        Tiling(np.zeros((4, 4, 4), np.uint8), 8)
