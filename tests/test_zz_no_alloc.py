"""lbm_macroscopic_noalloc, the entry point for callers that cannot allocate
device memory, against lbm_macroscopic_buf, the entry point it mirrors: the
same fields and sums bitwise, on two calls in a row (the second on a context
with fewer tiles, so the library's static scratch still holds the first
call's partials beyond the ones the second reads), and the size limit."""
import ctypes

import numpy as np
import pytest

from paper_1611_02445_amd import _abi
from paper_1611_02445_amd import inputs as I
from paper_1611_02445_amd.lattice import _vp

from helpers import log, new_lattice

pytestmark = pytest.mark.gpu

MAX_TILES = 262144  # LBM_NOALLOC_MAX_TILES


def _both(lat, state=None):
    """(fields, sums) from lbm_macroscopic_buf and from lbm_macroscopic_noalloc,
    each into fresh buffers filled with NaN first."""
    import torch
    out = []
    for name in ("lbm_macroscopic_buf", "lbm_macroscopic_noalloc"):
        rho = torch.full(lat.dense_shape, float("nan"), dtype=torch.float64, device=lat.device)
        u = torch.full((3,) + lat.dense_shape, float("nan"), dtype=torch.float64, device=lat.device)
        sums = (ctypes.c_double * 8)()
        rc = getattr(_abi.lib(), name)(lat.ctx, _vp(state), _vp(rho), _vp(u), sums)
        out.append((rc, rho.cpu().numpy(), u.cpu().numpy(), np.array(sums[:])))
    return out


def _check_equal(lat, label, state=None):
    (rc0, r0, u0, s0), (rc1, r1, u1, s1) = _both(lat, state)
    log(f"[case] {label}: tiles={lat.n_tiles} rc={rc0},{rc1} mass={s1[0]:.15e} max|u|={s1[5]:.3e}")
    assert rc0 == 0 and rc1 == 0
    assert np.array_equal(r0, r1) and np.array_equal(u0, u1)
    assert np.array_equal(s0, s1)
    assert s1[4] == lat.n_fluid


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_noalloc_matches_buffered_on_two_calls(storage):
    import torch
    big, _ = I.sphere_pack((64, 48, 56), 0.45, 3.0, 7.0, seed=91)
    small, _ = I.sphere_pack((20, 16, 12), 0.6, 2.0, 3.0, seed=92)
    a = new_lattice(big, 0.7, 7, storage=storage)
    b = new_lattice(small, 0.9, 7, storage=storage, model="inc")
    assert b.n_tiles < a.n_tiles
    for lat, g in ((a, (1e-5, 0.0, 2e-6)), (b, (0.0, 3e-6, 0.0))):
        lat.init()
        lat.set_force(g)
        lat.step(25)
    _check_equal(a, f"{storage} first call")
    _check_equal(b, f"{storage} second call, fewer tiles")
    # any lattice buffer of the context, and the first context again
    _check_equal(b, f"{storage} other lattice", state=b.state_a if b.current_state() is b.state_b else b.state_b)
    _check_equal(a, f"{storage} first context again")


def test_noalloc_keeps_the_numeric_checks():
    big, _ = I.sphere_pack((16, 16, 16), 0.6, 2.0, 4.0, seed=93)
    lat = new_lattice(big, 0.8, 7, check_u_max=True)
    lat.init(u0=(0.06, 0.0, 0.0))
    (rc0, _, _, s0), (rc1, _, _, s1) = _both(lat)
    assert rc0 == rc1 == _abi.STATUS_CODE["LBM_E_NUMERIC"]
    assert np.array_equal(s0, s1)


def test_noalloc_rejects_more_tiles_than_its_scratch():
    # a fully fluid box of 65 x 64 x 64 tiles: 266,240 > 262,144
    solid = np.zeros((256, 256, 260), np.uint8)
    lat = new_lattice(solid, 0.8, 7 & ~1, storage="f16s")
    assert lat.n_tiles == 65 * 64 * 64 > MAX_TILES
    sums = (ctypes.c_double * 8)()
    rc = _abi.lib().lbm_macroscopic_noalloc(lat.ctx, None, None, None, sums)
    log(f"[case] noalloc over the limit: rc={rc} {_abi.lib().lbm_last_error().decode()}")
    assert rc == _abi.STATUS_CODE["LBM_E_RANGE"]
    assert b"static scratch" in _abi.lib().lbm_last_error()
