"""lbm_step_graphed: replays of a captured 32-step HIP graph give bitwise the
states of plain launches, from either lattice parity, across changes of the
kernel arguments (recapture), with eager work and synchronisation between the
replays; stochastic FP16 rounding is refused."""
import numpy as np
import pytest

from paper_1611_02445_amd import inputs as I

from helpers import log, new_lattice, padded, perturbed_state

pytestmark = pytest.mark.gpu


def _pair(solid, storage, **kw):
    import torch
    lats = []
    f0 = perturbed_state(padded(solid, 7), 5)
    for _ in range(2):
        lat = new_lattice(solid, 0.8, 7, storage=storage, **kw)
        lat.init()
        lat.set_state(torch.from_numpy(f0))
        lat.set_force((1e-5, 0.0, 0.0))
        lats.append(lat)
    return lats


@pytest.mark.parametrize("storage,rounding", [("f64", "stochastic"), ("f32", "stochastic"), ("f16s", "nearest")])
def test_graph_replays_match_plain_launches(storage, rounding):
    import torch
    solid, _ = I.sphere_pack((24, 20, 28), 0.5, 2.0, 4.0, seed=9)
    plain, graphed = _pair(solid, storage, f16_rounding=rounding)
    # counts chosen to cover: no full chunk, one chunk, chunks + remainder, an odd
    # start parity, and a recapture after the force changes
    for k, n in enumerate((5, 32, 70, 1, 64, 33, 96)):
        if k == 4:
            for lat in (plain, graphed):
                lat.set_force((2e-5, -1e-6, 0.0))
        plain.step(n)
        graphed.step(n, graphed=True)
        torch.cuda.synchronize()
        a, b = plain.get_state(), graphed.get_state()
        log(f"[case] graph {storage} call {k} n={n}")
        assert torch.equal(a, b)
        assert (plain.current_state_ptr() == plain.state_a.data_ptr()) == \
            (graphed.current_state_ptr() == graphed.state_a.data_ptr())
        _ = (a.sum() * 2).item()  # eager work between the replays


def test_graph_refuses_stochastic_fp16_and_handles_empty():
    from paper_1611_02445_amd._abi import LbmError
    solid, _ = I.sphere_pack((16, 16, 16), 0.5, 2.0, 4.0, seed=9)
    lat = new_lattice(solid, 0.8, 7, storage="f16s")
    lat.init()
    with pytest.raises(LbmError, match="UNSUPPORTED"):
        lat.step(64, graphed=True)
    empty = new_lattice(np.ones((8, 8, 8), np.uint8), 0.8, 7)
    empty.init()
    empty.step(65, graphed=True)


@pytest.mark.parametrize("model", ["mrt-qc", "inc"])
def test_graph_with_open_boundaries_and_other_models(model):
    """Boundary masks and the model are captured with the kernel arguments;
    removing the boundaries triggers a recapture."""
    import torch
    solid = np.zeros((8, 12, 32), np.uint8)
    solid[:, 0, :] = 1
    solid[:, -1, :] = 1
    bt = np.zeros_like(solid)
    bt[:, 1:-1, 0] = 1
    bt[:, 1:-1, -1] = 2
    lats = []
    for _ in range(2):
        lat = new_lattice(solid, 0.8, 4, model=model)
        lat.init()
        lat.set_boundaries(bt, u_in=(0.02, 0.0, 0.0))
        lats.append(lat)
    plain, graphed = lats
    for k, n in enumerate((40, 64, 3, 70)):
        if k == 2:
            for lat in lats:
                lat.set_boundaries(None)
        plain.step(n)
        graphed.step(n, graphed=True)
        torch.cuda.synchronize()
        log(f"[case] graph {model} with boundaries call {k} n={n}")
        assert torch.equal(plain.get_state(), graphed.get_state())
