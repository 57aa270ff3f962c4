"""The propagation-only kernels of the paper's intra-tile layout study
(Section 3.3, Eqs. 11-13; Table 5) on a fully fluid box: kind 3 (XYZ for every
direction) moves the same bytes as the library's own propagation-only kernel,
and kinds 4-6 are that kernel conjugated by their per-direction slot maps."""
import numpy as np
import pytest

import oracle as O

from helpers import log, new_lattice, perturbed_state

pytestmark = pytest.mark.gpu

# the maps, written out from Eqs. 11-13 (x, y, z in 0..3 inside the tile)
XYZ = [x + 4 * y + 16 * z for z in range(4) for y in range(4) for x in range(4)]
YXZ = [y + 4 * x + 16 * z for z in range(4) for y in range(4) for x in range(4)]
ZIG = [2 * (x + 3 * y + (4 if x == 3 else 0) * (3 - y)) + (z % 2) + 16 * (z & 2)
       for z in range(4) for y in range(4) for x in range(4)]
# D3Q19 directions by name: E 1, W 3, NE 7, NW 8, SW 9, SE 10, ET 11, EB 12, WT 13, WB 14
YXZ_DIRS = (1, 3, 11, 12, 8, 9, 13, 14)
ZIG_DIRS = (7, 10)
KINDS = {3: (False, False), 4: (False, True), 5: (True, False), 6: (True, True), 7: "face"}
# the face-major order (kind 7): x slowest, y slowest
XSLOW = [y + 4 * z + 16 * x for z in range(4) for y in range(4) for x in range(4)]
YSLOW = [x + 4 * z + 16 * y for z in range(4) for y in range(4) for x in range(4)]
DT = {"f64": "float64", "f32": "float32", "f16s": "float16"}


def _slot_maps(kind):
    """maps[i][n] = slot of node n (x + 4y + 16z) in direction i's block."""
    maps = np.array([XYZ] * 19)
    if KINDS[kind] == "face":
        for i in (1, 3):  # E, W
            maps[i] = XSLOW
        for i in (2, 4, 7, 8, 9, 10):  # N, S and the xy edges
            maps[i] = YSLOW
        return maps
    yxz, zig = KINDS[kind]
    for i in range(19):
        if yxz and i in YXZ_DIRS:
            maps[i] = YXZ
        if zig and i in ZIG_DIRS:
            maps[i] = ZIG
    return maps


def _blocks(buf, lat, storage):
    import torch
    return buf.view(getattr(torch, DT[storage]))[:lat.n_tiles * 19 * 64].view(lat.n_tiles, 19, 64)


def test_maps_are_permutations():
    for m in (XYZ, YXZ, ZIG, XSLOW, YSLOW):
        assert sorted(m) == list(range(64))
    # under the face-major order the x = 3 face (read by the east neighbour
    # for E) and the y = 3 face (read by the north neighbour for N) are the
    # last 16 slots: one 128-byte line in FP64
    assert sorted(XSLOW[3 + 4 * y + 16 * z] for y in range(4) for z in range(4)) == list(range(48, 64))
    assert sorted(YSLOW[x + 12 + 16 * z] for x in range(4) for z in range(4)) == list(range(48, 64))
    # zigzagNE keeps the two z-neighbours z = 2k, 2k+1 of a column side by side
    for x in range(4):
        for y in range(4):
            assert ZIG[x + 4 * y + 16] == ZIG[x + 4 * y] + 1


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("periodic", [0, 5])
def test_layout_kinds_conjugate_the_propagation(storage, periodic):
    import torch
    solid = np.zeros((12, 16, 20), np.uint8)  # z, y, x: 3 x 4 x 5 full tiles
    lat = new_lattice(solid, 0.8, periodic, storage=storage)
    lat.init()
    f0 = perturbed_state(solid, 31)
    lat.set_state(torch.from_numpy(f0))
    a = lat.current_state()
    b2, b3 = lat.new_state(), lat.new_state()
    lat.calib_step(2, a, b2)
    lat.calib_step(3, a, b3)
    torch.cuda.synchronize()
    assert torch.equal(b2, b3)
    if storage == "f64":
        assert np.array_equal(lat.get_state(b3).cpu().numpy(), O.pull(f0, solid, periodic=periodic))
    ref = _blocks(b3, lat, storage).cpu().numpy()
    src = _blocks(a, lat, storage).cpu().numpy()
    for kind in (4, 5, 6, 7):
        maps = _slot_maps(kind)
        a_l = lat.new_state()
        out = lat.new_state()
        perm = np.empty_like(src)
        for i in range(19):
            perm[:, i, maps[i]] = src[:, i, :]
        _blocks(a_l, lat, storage).copy_(torch.from_numpy(perm))
        lat.calib_step(kind, a_l, out)
        got_l = _blocks(out, lat, storage).cpu().numpy()
        got = np.stack([got_l[:, i, maps[i]] for i in range(19)], axis=1)
        log(f"[case] layout kind {kind} {storage} periodic={periodic}")
        assert np.array_equal(np.ascontiguousarray(got).view(np.uint8), np.ascontiguousarray(ref).view(np.uint8))


def test_layout_kinds_need_full_tiles():
    from paper_1611_02445_amd._abi import LbmError
    solid = np.zeros((8, 8, 8), np.uint8)
    solid[3, 3, 3] = 1
    lat = new_lattice(solid, 0.8, 7)
    lat.init()
    b = lat.new_state()
    with pytest.raises(LbmError):
        lat.calib_step(4, lat.current_state(), b)
    with pytest.raises(LbmError):
        lat.calib_step(7, lat.current_state(), b)
    with pytest.raises(LbmError):
        lat.calib_step(8, lat.current_state(), b)
