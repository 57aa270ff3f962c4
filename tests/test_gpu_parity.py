"""GPU parity: the fused tiled step (HIP) against the dense FP64 oracle, node by
node.  Bar: |f_gpu - f_oracle| <= 1e-12 |f_oracle| for every distribution of
every fluid node (the FP64 tolerance of the method's statement), rho likewise.
Velocity is a difference of distributions (u ~ 1e-5 from f ~ 0.03), so its
bound is the one the f bound implies: |du_a| <= 1e-12 sum_i |c_ia| f_i / rho,
about 1e-12 / 3 at rho ~ 1."""
import numpy as np
import pytest

import oracle as O
from paper_1611_02445_amd import inputs as I

from helpers import log, new_lattice, padded, perturbed_state, rel_err_f

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _run_case(name, solid, periodic, tau, steps, g=(0.0, 0.0, 0.0), model="qc", seed=None, tpw=0, field=None):
    import torch
    log(f"[case] {name} shape={solid.shape} periodic={periodic} tau={tau} steps={steps} model={model} tpw={tpw}")
    sp = padded(solid, periodic)
    lat = new_lattice(solid, tau, periodic, model=model, tiles_per_wg=tpw)
    lat.init()
    if seed is not None:
        f0 = perturbed_state(sp, seed)
        lat.set_state(torch.from_numpy(f0))
    else:
        f0 = O.init(sp, model=O.MODELS[model])
    if field is not None:
        lat.set_force(torch.from_numpy(field))
        force = field  # oracle takes F = rho0 g with rho0 = 1
    else:
        lat.set_force(g)
        force = np.array(g, dtype=np.float64)
    lat.step(steps)
    torch.cuda.synchronize()
    fg = lat.get_state().cpu().numpy()
    fo = O.run(f0, sp, tau, steps, force=force, periodic=periodic, model=O.MODELS[model])
    err = rel_err_f(fg, fo, sp)
    log(f"   f rel err {err:.3e}  tiles={lat.n_tiles} fluid={lat.n_fluid}")
    assert err <= TOL
    # never written: solid slots stay 0
    assert np.all(fg[:, sp == 1] == 0.0)
    return lat, sp, fg, fo, force


def test_fully_fluid_periodic_random_state():
    s = I.fluid_box(16, 12, 8)
    _run_case("fluid-box", s, 7, 0.7, 60, g=(1e-5, -3e-6, 2e-6), seed=1)


def test_square_duct_config_500_steps():
    # 32^3 square duct, tau 0.8, g_x 1e-6, 500 steps (the Poiseuille configuration)
    lat, sp, fg, fo, force = _run_case("duct32", I.square_channel(32), 7, 0.8, 500, g=(1e-6, 0, 0))
    rho_g, u_g, sums = lat.macroscopic()
    rho_o, u_o = O.macroscopic(fo, sp, force=force)
    fl = sp == 0
    rho_g = rho_g.cpu().numpy()
    u_g = u_g.cpu().numpy()
    assert np.max(np.abs(rho_g[fl] - rho_o[fl]) / rho_o[fl]) <= TOL
    c, _, _ = O.lattice()
    for a in range(3):
        bound = TOL * np.tensordot(np.abs(c[:, a]), fo, axes=1)[fl] / rho_o[fl]
        assert np.all(np.abs(u_g[a][fl] - u_o[a][fl]) <= bound)
    assert np.all(rho_g[~fl] == 0) and np.all(u_g[:, ~fl] == 0)
    so = O.sums(fo, sp, force=force)
    assert abs(sums[0] - so[0]) <= 1e-13 * so[0]
    assert np.max(np.abs(sums[1:4] - so[1:4])) <= 1e-10 * abs(so[1])
    assert sums[4] == so[4] and sums[6] == 0
    m0 = O.sums(O.init(sp), sp)[0]
    assert abs(sums[0] - m0) / m0 <= 1e-13


def test_sphere_pack_crop_200_steps():
    # 64^3 periodic crop of the 256^3 random sphere pack (porosity 0.4, r 4..12)
    s, _ = I.sphere_pack((64, 64, 64), 0.4, 4.0, 12.0, seed=2)
    _run_case("spheres64", s, 7, 0.7, 200, g=(1e-6, 0, 0))


def test_ragged_nonperiodic_box_with_empty_tiles():
    s, _ = I.sphere_pack((21, 18, 27), 0.5, 2.0, 5.0, seed=7, periodic=False)
    s[:, :, :9] = 1  # a slab of dropped tiles
    _run_case("ragged", s, 0, 0.9, 80, g=(2e-5, 1e-5, 0), seed=3)


def test_mixed_periodicity_random_bitmap():
    s = I.random_bitmap((12, 16, 10), 0.35, seed=5)
    _run_case("bitmap-pyz", s, 6, 0.62, 40, g=(0, 1e-5, -1e-5), seed=4)


def test_incompressible_model():
    s, _ = I.sphere_pack((16, 16, 16), 0.6, 2.0, 4.0, seed=8)
    _run_case("incompressible", s, 7, 0.75, 100, g=(1e-5, 0, 0), model="inc", seed=5)


@pytest.mark.parametrize("model", ["mrt-qc", "mrt-inc"])
def test_multiple_relaxation_times(model):
    s, _ = I.sphere_pack((20, 16, 24), 0.55, 2.0, 4.5, seed=12)
    _run_case(model, s, 7, 0.68, 100, g=(1e-5, -2e-6, 3e-6), model=model, seed=6)


def test_multiple_relaxation_times_ragged_nonperiodic():
    s, _ = I.sphere_pack((21, 18, 27), 0.5, 2.0, 5.0, seed=13, periodic=False)
    _run_case("mrt-ragged", s, 0, 0.9, 60, g=(2e-5, 1e-5, 0), model="mrt-qc", seed=7)


def test_per_node_force_field():
    s, _ = I.sphere_pack((16, 20, 12), 0.5, 2.0, 4.0, seed=9)
    sp = padded(s, 7)
    rng = np.random.default_rng(6)
    field = np.zeros((3,) + sp.shape)
    field[0] = rng.normal(1e-6, 1e-7, sp.shape)
    field[1] = rng.normal(0, 1e-7, sp.shape)
    field[:, sp == 1] = 0
    _run_case("force-field", s, 7, 0.8, 50, field=field, seed=6)


@pytest.mark.parametrize("tpw", [1, 2, 8])
def test_tiles_per_workgroup_bitwise_identical(tpw):
    import torch
    s, _ = I.sphere_pack((24, 24, 24), 0.5, 2.0, 5.0, seed=10)
    ref = new_lattice(s, 0.7, 7, tiles_per_wg=4)
    ref.init()
    ref.set_force((1e-5, 0, 0))
    ref.step(20)
    alt = new_lattice(s, 0.7, 7, tiles_per_wg=tpw)
    alt.init()
    alt.set_force((1e-5, 0, 0))
    alt.step(20)
    torch.cuda.synchronize()
    assert torch.equal(ref.get_state(), alt.get_state())


def test_rest_state_and_source_untouched():
    import torch
    s, _ = I.sphere_pack((20, 20, 20), 0.5, 2.0, 5.0, seed=11)
    lat = new_lattice(s, 0.8, 7)
    lat.init()
    lat.set_force((0, 0, 0))
    f0 = lat.get_state().clone()
    lat.step(300)
    assert torch.max(torch.abs(lat.get_state() - f0)).item() <= 1e-15
    # one step must leave its source lattice bit-identical
    lat.set_force((1e-5, 0, 0))
    src = lat.current_state().clone()
    lat.step(1)
    torch.cuda.synchronize()
    assert torch.equal(src, lat.state_a if lat.current_state() is lat.state_b else lat.state_b)


def test_all_solid_and_single_node():
    import torch
    lat = new_lattice(np.ones((8, 8, 8), np.uint8), 0.8, 0)
    assert lat.n_tiles == 0
    lat.init()
    lat.step(3)
    _, _, sums = lat.macroscopic(fields=False)
    assert np.all(sums == 0)
    s = np.ones((9, 9, 9), np.uint8)
    s[4, 5, 6] = 0
    _run_case("single-node", s, 0, 0.8, 10, g=(1e-5, 0, 0), seed=7)


def test_calibration_kernels():
    import torch
    s, _ = I.sphere_pack((16, 16, 16), 0.5, 2.0, 4.0, seed=12)
    sp = padded(s, 7)
    lat = new_lattice(s, 0.8, 7)
    lat.init()
    f0 = perturbed_state(sp, 13)
    lat.set_state(torch.from_numpy(f0))
    src = lat.current_state()
    dst = lat.new_state()
    dst.zero_()
    lat.calib_step(1, src, dst)
    assert torch.equal(lat.get_state(dst), lat.get_state(src))
    lat.calib_step(2, src, dst)
    g = lat.get_state(dst).cpu().numpy()
    assert np.array_equal(g, O.pull(f0, sp, periodic=7))


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_tile_order_buffers_follow_the_listed_order(order):
    """Row d of a tile-order buffer belongs to the tile that lbm_tile_order
    lists d-th for the context's order."""
    import torch
    s, _ = I.sphere_pack((32, 24, 40), 0.5, 2.0, 5.0, seed=14)
    lat = new_lattice(s, 0.7, 7, tile_order=order)
    perm = lat.tiling.device_order(order)
    n = lat.n_tiles
    buf = np.repeat(perm.astype(np.float64) + 1.0, 64).reshape(n, 1, 64)
    dense = lat.tiles_to_dense(torch.from_numpy(buf).cuda(), 1)[0].cpu().numpy()
    tmap = lat.tiling.arrays()["tile_map"]
    want = np.repeat(np.repeat(np.repeat(tmap + 1.0, 4, 0), 4, 1), 4, 2)
    assert s.shape == dense.shape
    want[s != 0] = 0.0  # solid nodes, in kept tiles too, read 0
    assert np.array_equal(dense, want)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
@pytest.mark.parametrize("storage", ["f64", "f16s"])
def test_tile_order_bitwise_identical(order, storage):
    """The device tile order changes only where tiles live and when they run."""
    import torch
    s, _ = I.sphere_pack((32, 24, 40), 0.5, 2.0, 5.0, seed=14)
    res = []
    for o in (1, order):
        lat = new_lattice(s, 0.7, 7, storage=storage, tile_order=o)
        lat.init()
        lat.set_force((1e-5, 0, 0))
        lat.step(15)
        res.append((lat.get_state(), lat.macroscopic()[2]))
    torch.cuda.synchronize()
    assert torch.equal(res[0][0], res[1][0])
    # counts and max are order-free; FP64 sums are reduced in device tile order
    assert np.array_equal(res[0][1][[4, 5, 6]], res[1][1][[4, 5, 6]])
    assert abs(res[0][1][0] - res[1][1][0]) <= 1e-14 * res[0][1][0]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_wide_offsets_bitwise_identical(storage):
    """The 64-bit-offset kernels (used when a lattice exceeds 4 GiB) give the
    same bits as the 32-bit ones: forced on a small sphere pack."""
    import torch
    s, _ = I.sphere_pack((24, 20, 16), 0.5, 2.0, 4.0, seed=71)
    log(f"[case] wide offsets {storage}")
    out = []
    for wide in (False, True):
        lat = new_lattice(s, 0.7, 7, storage=storage, wide_offsets=wide)
        lat.init()
        lat.set_force((1e-5, 2e-6, 0.0))
        lat.step(40)
        out.append(lat.get_state().cpu().numpy())
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_wide_offsets_adjoint_bitwise_identical(storage):
    import torch
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    s, _ = I.sphere_pack((16, 20, 24), 0.5, 2.0, 4.0, seed=72)
    res = []
    for wide in (False, True):
        lat = new_lattice(s, 0.8, 7, storage=storage, wide_offsets=wide)
        lat.init()
        lat.set_force((1e-5, 0.0, 0.0))
        run = CheckpointedAdjoint(lat, 9, 4)
        L = run.forward(None)
        gs, gg = run.backward()
        res.append((L, gs.cpu().numpy(), gg.cpu().numpy()))
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1]) and np.array_equal(res[0][2], res[1][2])


def _random_cases(n, seed):
    """Seeded random small geometries: each axis 5..20 nodes, periodic axes
    rounded to whole tiles, solid fraction 0.1..0.9 (down to tiles with a
    single fluid node), every model, tau and force."""
    rng = np.random.default_rng(seed)
    models = ["qc", "inc", "mrt-qc", "mrt-inc"]
    for k in range(n):
        periodic = int(rng.integers(0, 8))
        dims = []
        for axis in range(3):  # x, y, z -> bits 1, 2, 4
            d = int(rng.integers(5, 21))
            if periodic >> axis & 1:
                d = max(4, d // 4 * 4)
            dims.append(d)
        nx, ny, nz = dims
        solid = I.random_bitmap((nz, ny, nx), float(rng.uniform(0.1, 0.9)), seed=int(rng.integers(1 << 30)))
        yield (k, solid, periodic, float(rng.uniform(0.55, 1.4)), models[k % 4],
               tuple(float(v) for v in rng.normal(0, 1e-5, 3)), int(rng.integers(1 << 30)))


@pytest.mark.parametrize("case", list(_random_cases(16, 2024)), ids=lambda c: f"rand{c[0]}")
def test_random_geometries(case):
    """Random geometries exercise unusual tile masks (single fluid nodes,
    checkerboards, empty neighbours) in every model; FP64 bar."""
    k, solid, periodic, tau, model, g, seed = case
    if (solid == 0).sum() == 0:
        pytest.skip("no fluid node")
    _run_case(f"random{k}", solid, periodic, tau, 25, g=g, model=model, seed=seed % 1000)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_walk_direction_leaves_results_bitwise_unchanged(storage):
    """Consecutive launches walk the tiles in opposite directions (the parity
    of a per-context launch counter).  A context whose counter is one ahead,
    so that every one of its launches walks the other way, must produce the
    same lattice and the same adjoint bit for bit: the direction only changes
    when a tile runs."""
    import torch
    s, _ = I.sphere_pack((32, 24, 40), 0.5, 2.0, 5.0, seed=21)
    states, grads = [], []
    for shifted in (False, True):
        lat = new_lattice(s, 0.7, 7, storage=storage)
        lat.init()
        lat.set_force((1e-5, 0, 0))
        if shifted:  # one launch into a scratch lattice: the counter moves, the state does not
            lat.step_buf(lat.current_state(), lat.new_state())
            junk = (lat.new_adjoint(), lat.new_adjoint(), lat.new_grad())
            lat.adjoint_step(lat.current_state(), junk[0], junk[1], junk[2])
        lat.step(15)
        states.append(lat.get_state())
        sb, ei, eo, gr = lat.current_state(), lat.new_adjoint(), lat.new_adjoint(), lat.new_grad()
        lat.adjoint_seed(sb, ei, gr)
        for _ in range(5):
            lat.adjoint_step(sb, ei, eo, gr)
            ei, eo = eo, ei
        grads.append((lat.adjoint_get(ei), gr.clone()))
    torch.cuda.synchronize()
    assert torch.equal(states[0], states[1])
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])
