"""Per-node fields (the force density and the force gradient) stored one
entry per fluid node and component: the round trip through lbm_set_force and
lbm_field_to_dense is exact (default, discovery and Hilbert tile orders), pad
entries are zero, and a per-node force gives the oracle's step on partly
solid tiles for every storage type."""
import numpy as np
import pytest

import oracle as O
from paper_1611_02445_amd import inputs as I

from helpers import log, new_lattice, padded, perturbed_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order", [0, 1, 5])
@pytest.mark.parametrize("storage,dtype", [("f64", 0), ("f32", 1), ("f16s", 1)])
def test_force_field_round_trip(storage, dtype, order):
    import torch
    s, _ = I.sphere_pack((20, 24, 16), 0.45, 2.0, 5.0, seed=71)
    sp = padded(s, 7)
    rng = np.random.default_rng(72)
    g = rng.normal(0.0, 1e-5, (3,) + sp.shape)
    lat = new_lattice(s, 0.8, 7, storage=storage, rho0=1.25, tile_order=order)
    lat.set_force(torch.from_numpy(g).cuda())
    back = lat.field_to_dense(lat.force_buf, dtype).cpu().numpy()
    ref = 1.25 * g
    if dtype == 1:
        ref = ref.astype(np.float32).astype(np.float64)
    ref[:, sp == 1] = 0.0
    assert np.array_equal(back, ref)
    # every byte of the buffer is either a fluid node's entry or a zero pad
    n_entries = lat.sizes.force_bytes // (8 if dtype == 0 else 4)
    assert n_entries % 16 == 0 and n_entries >= 3 * lat.n_fluid
    raw = lat.force_buf.view(torch.float64 if dtype == 0 else torch.float32)[:n_entries].cpu().numpy()
    assert np.count_nonzero(raw) == np.count_nonzero(ref)
    assert np.array_equal(np.sort(raw[raw != 0]), np.sort(ref[ref != 0].astype(raw.dtype)))


@pytest.mark.parametrize("storage,model", [("f64", "qc"), ("f64", "mrt-inc"), ("f32", "qc"), ("f16s", "inc")])
def test_per_node_force_step_against_oracle(storage, model):
    import torch
    tau, steps = 0.75, 40
    s, _ = I.sphere_pack((16, 20, 24), 0.5, 2.0, 4.0, seed=73)
    sp = padded(s, 7)
    f0 = perturbed_state(sp, 74)
    rng = np.random.default_rng(75)
    g = rng.normal(2e-5, 5e-6, (3,) + sp.shape)
    g[:, sp == 1] = 0.0
    lat = new_lattice(s, tau, 7, storage=storage, model=model)
    lat.init()
    lat.set_state(torch.from_numpy(f0))
    lat.set_force(torch.from_numpy(g).cuda())
    lat.step(steps)
    got = lat.get_state().cpu().numpy()
    ref = O.run(f0, sp, tau, steps, force=g, periodic=7, model=O.MODELS[model])
    fl = sp == 0
    c, w, _ = O.lattice()
    if storage == "f64":
        err = np.max(np.abs(got[:, fl] - ref[:, fl]) / np.abs(ref[:, fl]))
        log(f"[case] per-node force {storage} {model}: max rel err {err:.2e}")
        assert err <= 1e-12
    else:
        d = np.abs(ref - w[:, None, None, None])[:, fl].max()
        err = np.abs(got[:, fl] - ref[:, fl]).max()
        bound = steps * 2.0 ** -24 * d * 8 if storage == "f32" else steps * 2.0 ** -10 * d
        log(f"[case] per-node force {storage} {model}: max |df| {err:.2e}, bound {bound:.2e}")
        assert err <= bound
