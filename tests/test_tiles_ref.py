"""Pins of the oracle tiler (Alg. 1) against the paper's worked examples and a
brute-force definition."""
import json
import os

import numpy as np
import pytest

from oracle import tiles_ref as T
from paper_1611_02445_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def _channel_tiles(side, oy, oz):
    """Square channel along x (periodic x), cross-section side x side with its
    corner at (oy, oz) inside a box padded by the tiler."""
    s = I.channel_cross_section(side, oy, oz, length=4, box=side + 8)
    r = T.build_tiles(s, periodic=1)
    return r


def test_fig6_worked_example():
    g = _load("fig6_square_channel_8x8.json")
    counts = {}
    etas = []
    for oy in range(4):
        for oz in range(4):
            r = _channel_tiles(g["side"], oy, oz)
            n_cross = r["n_tiles"]  # one tile along x (length 4)
            counts[n_cross] = counts.get(n_cross, 0) + 1
            etas.append(r["eta_t"])
            assert r["eta_t"] == pytest.approx(g["eta_t"][str(n_cross)], abs=1e-15)
    assert {str(k): v for k, v in counts.items()} == g["tile_counts"]
    assert np.mean(etas) == pytest.approx(g["mean_eta_t"], abs=1e-15)
    assert round(np.mean(etas), 2) == g["mean_eta_t_printed"]


def test_side_tile_plus_one_same_utilisation():
    facts = _load("tiling_facts.json")
    side = facts["side_tile_plus_one"]["side"]
    etas = {_channel_tiles(side, oy, oz)["eta_t"] for oy in range(4) for oz in range(4)}
    assert len(etas) == 1


def test_side_equal_tile_reaches_one():
    side = _load("tiling_facts.json")["side_equal_tile"]["side"]
    assert max(_channel_tiles(side, oy, oz)["eta_t"] for oy in range(4) for oz in range(4)) == 1.0


def test_lowest_utilisation_at_side_4k_plus_2():
    # read as the worst tiling of each side (the mean is flat between m = 0 and 1)
    m = _load("tiling_facts.json")["lowest_mod"]["m"]
    for k in (2, 3, 5):
        worst = []
        for r in range(4):
            side = 4 * k + r
            worst.append(min(_channel_tiles(side, oy, oz)["eta_t"] for oy in range(4) for oz in range(4)))
        assert int(np.argmin(worst)) == m


def test_padding_count():
    f = _load("tiling_facts.json")["padding"]
    nx, ny, nz = f["shape_xyz"]
    pz, py, px = T.padded_shape((nz, ny, nx), periodic=0)
    assert (px, py, pz) == tuple(f["padded_xyz"])
    assert px * py * pz == f["padded_nodes"]
    assert round(px * py * pz / 1e5) / 10 == f["printed_nodes"] / 1e6


def test_overhead_example():
    f = _load("tiling_facts.json")["overhead_example"]
    eta = f["eta_t"]
    assert round((1 - eta) / eta, 1) == f["delta_printed"]


@pytest.mark.parametrize("seed,shape,frac,periodic", [
    (0, (5, 6, 7), 0.5, 0), (1, (8, 8, 8), 0.9, 7), (2, (4, 9, 12), 0.3, 5), (3, (12, 4, 5), 0.97, 2),
    (4, (8, 12, 4), 0.0, 7), (5, (7, 7, 7), 1.0, 0)])
def test_vectorised_matches_bruteforce(seed, shape, frac, periodic):
    s = I.random_bitmap(shape, frac, seed)
    # periodic axes must be multiples of 4
    for bit, ax in ((1, 2), (2, 1), (4, 0)):
        if periodic & bit and shape[ax] % 4:
            pytest.skip("periodic axis not a multiple of 4")
    r = T.build_tiles(s, periodic)
    b = T.build_tiles_bruteforce(s, periodic)
    assert np.array_equal(r["tile_map"], b["tile_map"])
    assert [tuple(v) for v in r["tile_xyz"]] == [tuple(v) for v in b["tile_xyz"]]
    assert [int(m) for m in r["fluid_mask"]] == list(b["fluid_mask"])
    assert r["nbr"].tolist() == b["nbr"]
    assert r["n_fluid"] == int((T.pad(s, periodic) == 0).sum())


def test_periodic_axis_must_be_multiple_of_four():
    with pytest.raises(ValueError):
        T.build_tiles(np.zeros((4, 4, 6), dtype=np.uint8), periodic=1)


def test_single_fluid_node_and_all_solid():
    s = np.ones((9, 9, 9), dtype=np.uint8)
    r = T.build_tiles(s)
    assert r["n_tiles"] == 0 and r["n_fluid"] == 0
    s[5, 6, 7] = 0
    r = T.build_tiles(s)
    assert r["n_tiles"] == 1
    assert r["tile_xyz"].tolist() == [[4, 4, 4]]
    assert int(r["fluid_mask"][0]) == 1 << (3 + 4 * 2 + 16 * 1)
    assert r["nbr"][0, 13] == 0 and (r["nbr"][0] == -1).sum() == 26


def test_table6_sphere_arrays_tile_utilisation():
    """Tile utilisation of random sphere arrays (diameter 40, 192^3) against the
    printed row, for the porosities where the placement rule does not matter
    much (0.9 down to 0.3; the rule is unstated)."""
    import json
    import os
    from paper_1611_02445_amd import inputs as I
    with open(os.path.join(os.path.dirname(__file__), "golden", "table6_spheres_tile_utilisation.json")) as fh:
        g = json.load(fh)
    r = g["sphere_diameter"] / 2.0
    for p, eta_paper in zip(g["porosity"], g["tile_utilisation"]):
        solid, _ = I.sphere_pack(tuple(g["box"]), p, r, r, seed=11, periodic=True)
        t = T.build_tiles(solid, 7)
        eta = t["n_fluid"] / (64.0 * t["n_tiles"])
        assert abs((solid == 0).mean() - p) <= 0.01
        if p >= 0.3:
            assert abs(eta - eta_paper) <= 0.02, (p, eta, eta_paper)
        else:
            assert eta_paper <= eta <= eta_paper + 0.05, (p, eta, eta_paper)
