"""The compressibility limit as a runtime check: the paper keeps the largest
macroscopic speed at u_max <= 0.05 (Section 2.2).  With check_u_max set, the
synchronising macroscopic calls fill their outputs and then report
LBM_E_NUMERIC when max |u| exceeds it; without it they only report it in
sums[5]."""
import ctypes

import numpy as np
import pytest

from paper_1611_02445_amd import _abi
from paper_1611_02445_amd import inputs as I

from helpers import log, new_lattice

pytestmark = pytest.mark.gpu


def _raw_macroscopic(lat):
    """lbm_macroscopic through the C ABI: (status, sums)."""
    sums = (ctypes.c_double * 8)()
    rc = _abi.lib().lbm_macroscopic(lat.ctx, None, None, sums)
    return rc, np.array(sums[:])


@pytest.mark.parametrize("model", ["qc", "inc", "mrt-qc"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_u_max_limit(model, storage):
    s, _ = I.sphere_pack((16, 16, 16), 0.6, 2.0, 4.0, seed=61)
    # a state at rest speed 0.06 > 0.05 along x: rejected with the check on
    lat = new_lattice(s, 0.8, 7, model=model, storage=storage, check_u_max=True)
    lat.init(u0=(0.06, 0.0, 0.0))
    rc, sums = _raw_macroscopic(lat)
    log(f"[case] {storage} {model} u0=0.06 check on: rc={rc} max|u|={sums[5]:.6f}")
    assert rc == _abi.STATUS_CODE["LBM_E_NUMERIC"]
    assert b"compressibility" in _abi.lib().lbm_last_error()
    # the outputs are filled before the status is returned
    assert abs(sums[5] - 0.06) < 1e-3 and sums[4] == lat.n_fluid and sums[6] == 0
    with pytest.raises(_abi.LbmError, match="LBM_E_NUMERIC"):
        lat.permeability(1e-6)
    # each component below the limit, the speed above it: the check is on |u|
    lat.init(u0=(0.03, 0.03, 0.03))
    rc, sums = _raw_macroscopic(lat)
    assert rc == _abi.STATUS_CODE["LBM_E_NUMERIC"] and sums[5] > 0.05
    # below the limit the same calls succeed
    lat.init(u0=(0.04, 0.0, 0.0))
    rc, sums = _raw_macroscopic(lat)
    assert rc == 0 and abs(sums[5] - 0.04) < 1e-3
    lat.step(10)
    assert _raw_macroscopic(lat)[0] == 0
    # without the check 0.06 is reported, not rejected
    off = new_lattice(s, 0.8, 7, model=model, storage=storage)
    off.init(u0=(0.06, 0.0, 0.0))
    rc, sums = _raw_macroscopic(off)
    assert rc == 0 and abs(sums[5] - 0.06) < 1e-3


def test_u_max_limit_trips_during_a_run():
    """A body force accelerating a fully fluid periodic box from rest: the
    speed after n steps is (n - 1/2) g exactly (free acceleration), so the
    check passes up to the step that crosses 0.05 and fails after it."""
    g = 1e-3
    lat = new_lattice(np.zeros((8, 8, 8), np.uint8), 0.8, 7, check_u_max=True)
    lat.init()
    lat.set_force((g, 0.0, 0.0))
    lat.step(50)  # u = 0.0495
    rc, sums = _raw_macroscopic(lat)
    assert rc == 0 and abs(sums[5] - 0.0495) < 1e-12
    lat.step(1)  # u = 0.0505
    rc, sums = _raw_macroscopic(lat)
    assert rc == _abi.STATUS_CODE["LBM_E_NUMERIC"] and abs(sums[5] - 0.0505) < 1e-12
