"""GPU adjoint: the library's reverse-sweep kernels (driven with checkpoints)
against the oracle's discrete adjoint, the reverse gather against the forward
gather (dot products), the autograd entry point, and central finite
differences of the GPU forward at the full 128^3 sphere-pack size."""
import numpy as np
import pytest

import oracle as O
from paper_1611_02445_amd import inputs as I

from helpers import elementwise_err, log, new_lattice, padded, perturbed_state

# FP64 adjoint against the oracle's, entry by entry: within 1e-11 relative
# for every entry above 1e-3 of the largest one, within 1e-14 of the largest
# below that.  An entry is a sum of contributions as large as the largest
# entries, so its FP64 rounding is absolute, a few ulp of the largest values
# (max-normalised differences of ~1e-15 after 12 steps); a floor at 1e-6 of
# the largest entry would ask for less than one ulp of it (3e-17 of it was
# seen on a near-zero entry).
F64_TOL, F64_FLOOR = 1e-11, 1e-3

pytestmark = pytest.mark.gpu


def _force_field(sp, seed, mean=1e-5, std=1e-6):
    rng = np.random.default_rng(seed)
    g = np.zeros((3,) + sp.shape)
    g[0] = rng.normal(mean, std, sp.shape)
    g[1] = rng.normal(0.0, std, sp.shape)
    g[:, sp == 1] = 0.0
    return g


@pytest.mark.parametrize("periodic,K,model", [(7, 5, "qc"), (0, 3, "qc"), (5, 12, "qc"), (7, 5, "inc"),
                                               (0, 3, "inc"), (7, 5, "mrt-qc"), (0, 3, "mrt-inc")])
def test_adjoint_matches_oracle(periodic, K, model):
    import torch
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    tau, T = 0.8, 12
    s, _ = I.sphere_pack((12, 16, 12), 0.55, 2.0, 3.5, seed=21, periodic=bool(periodic & 1))
    sp = padded(s, periodic)
    f0 = perturbed_state(sp, 3)
    g = _force_field(sp, 4)
    log(f"[case] adjoint vs oracle periodic={periodic} K={K} T={T} model={model}")
    Lo, gs_o, gF_o = O.adjoint(f0, sp, tau, g, T, periodic=periodic, model=O.MODELS[model])
    lat = new_lattice(s, tau, periodic, model=model)
    lat.set_force(torch.from_numpy(g).cuda())
    run = CheckpointedAdjoint(lat, T, K)
    L = run.forward(torch.from_numpy(f0))
    gs, gg = run.backward()
    gs, gg = gs.cpu().numpy(), gg.cpu().numpy()
    fl = sp == 0
    # L is a mean of u_x, a difference of distributions: the FP64 bar on f
    # (1e-12 relative) bounds it by 1e-12 times the mean of sum |c_x| f / rho
    c, _, _ = O.lattice()
    fT = O.run(f0, sp, tau, T, force=g, periodic=periodic, model=O.MODELS[model])
    scale = (np.tensordot(np.abs(c[:, 0]).astype(float), fT, axes=1)[fl] / fT.sum(0)[fl]).mean()
    log(f"   L {L:.12e} vs {Lo:.12e} (bound {1e-12 * scale:.1e})")
    assert abs(L - Lo) <= 1e-12 * scale
    es = elementwise_err(gs, gs_o, fl, F64_FLOOR)
    eg = elementwise_err(gg, gF_o, fl, F64_FLOOR)
    log(f"   per-entry dL/ds0 err {es:.2e}  dL/dg err {eg:.2e}")
    assert es <= F64_TOL and eg <= F64_TOL
    assert np.all(gs[:, ~fl] == 0) and np.all(gg[:, ~fl] == 0)
    assert run.recompute_steps == T - run.n_ckpt


def test_reverse_gather_is_transpose_of_pull():
    """<S v, w> = <v, S^T w>: S from the propagation-only kernel, S^T from the
    adjoint's final reverse gather."""
    import torch
    s, _ = I.sphere_pack((16, 16, 16), 0.5, 2.0, 4.0, seed=31)
    sp = padded(s, 7)
    fl = (sp == 0)[None]
    rng = np.random.default_rng(5)
    v = rng.normal(size=(19,) + sp.shape) * fl
    w = rng.normal(size=(19,) + sp.shape) * fl
    lat = new_lattice(s, 0.8, 7)
    a, b = lat.new_state(), lat.new_state()
    lat.set_state(torch.from_numpy(v), a)
    lat.calib_step(2, a, b)
    Sv = lat.get_state(b).cpu().numpy()
    lat.set_state(torch.from_numpy(w), a)
    lat.adjoint_final(a, b)
    STw = lat.get_state(b).cpu().numpy()
    lhs, rhs = np.sum(Sv * w), np.sum(v * STw)
    assert abs(lhs - rhs) <= 1e-13 * np.sum(np.abs(Sv * w))
    assert np.array_equal(Sv, O.pull(v, sp, periodic=7))
    assert np.allclose(STw, O.pull_transpose(w, sp, periodic=7), rtol=0, atol=1e-14)


def test_autograd_function():
    import torch
    from paper_1611_02445_amd.autograd import mean_velocity_loss
    tau, T, K = 0.7, 10, 4
    s, _ = I.sphere_pack((12, 12, 16), 0.6, 2.0, 3.5, seed=41)
    sp = padded(s, 7)
    f0 = perturbed_state(sp, 6)
    g = _force_field(sp, 7)
    Lo, gs_o, gF_o = O.adjoint(f0, sp, tau, g, T, periodic=7)
    lat = new_lattice(s, tau, 7)
    f0_t = torch.from_numpy(f0).cuda().requires_grad_(True)
    g_t = torch.from_numpy(g).cuda().requires_grad_(True)
    L = mean_velocity_loss(f0_t, g_t, lat, T, K)
    (3.0 * L).backward()
    fl = sp == 0
    assert abs(L.item() - Lo) <= 1e-12 * abs(Lo)
    assert elementwise_err(f0_t.grad.cpu().numpy(), 3 * gs_o, fl, F64_FLOOR) <= F64_TOL
    assert elementwise_err(g_t.grad.cpu().numpy(), 3 * gF_o, fl, F64_FLOOR) <= F64_TOL


@pytest.mark.parametrize("model", ["qc", "mrt-qc"])
def test_adjoint_full_size_finite_differences(model):
    """128^3 periodic sphere pack, porosity 0.5, radius U[4,12), tau 0.8,
    T = 2000, checkpoints every 100 steps, per-node g_x ~ N(1e-6, 1e-7).
    Central differences of the GPU forward: g_x at 32 random fluid nodes and
    f_i(0) at the same 32 nodes, direction i cycling through all 19."""
    import torch
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    tau, T, K = 0.8, 2000, 100
    s, n_sph = I.sphere_pack((128, 128, 128), 0.5, 4.0, 12.0, seed=4)
    sp = padded(s, 7)
    rng = np.random.default_rng(40)
    g = np.zeros((3,) + sp.shape)
    g[0] = rng.normal(1e-6, 1e-7, sp.shape)
    g[:, sp == 1] = 0.0
    log(f"[case] adjoint 128^3 spheres={n_sph} T={T} K={K} model={model}")
    lat = new_lattice(s, tau, 7, model=model)
    lat.init()
    f0 = lat.get_state()
    g_t = torch.from_numpy(g).cuda()
    lat.set_force(g_t)
    run = CheckpointedAdjoint(lat, T, K)
    L0 = run.forward(f0)
    gs, gg = run.backward()
    gs, gg = gs.cpu().numpy(), gg.cpu().numpy()

    def loss(f_init, gf):
        lat.set_force(gf)
        lat.set_state(f_init)
        lat.step(T)
        _, _, sums = lat.macroscopic(fields=False)
        return sums[7] / sums[4]

    fluid = np.flatnonzero(sp.ravel() == 0)
    nodes = rng.choice(fluid, 8, replace=False)
    nodes = np.concatenate([nodes, rng.choice(np.setdiff1d(fluid, nodes), 24, replace=False)])
    worst = 0.0
    gmax = np.abs(gg[0]).max()
    for n in nodes:
        eps = 1e-5
        gp = g_t.clone()
        gm = g_t.clone()
        gp.view(3, -1)[0, n] += eps
        gm.view(3, -1)[0, n] -= eps
        fd = (loss(f0, gp) - loss(f0, gm)) / (2 * eps)
        ad = gg.reshape(3, -1)[0, n]
        rel = abs(fd - ad) / max(abs(fd), 1e-3 * gmax)
        worst = max(worst, rel)
        log(f"   g node {n}: fd {fd:.10e} adjoint {ad:.10e} rel {rel:.2e}")
        assert rel <= 1e-6
    lat.set_force(g_t)
    smax = np.abs(gs).max()

    def loss_f(n, i, e):
        f = f0.clone()
        f.view(19, -1)[i, n] += e
        return loss(f, g_t)

    worst_f = 0.0
    for k, n in enumerate(nodes):
        i = k % 19
        # The f0 gradients are ~1e-11..1e-10, so the loss changes by only
        # ~1e-14 per 1e-3 of perturbation, and the FP64 rounding of the
        # perturbed forward runs (a different rounding path from the
        # perturbation on) is ~1e-7 of that change: the error of a difference
        # quotient falls with the step.  L depends on f through rho = sum f
        # and j / rho, so its Taylor coefficients scale with 1 / rho ~ 1 and
        # the six-point central difference (error ~ 36 eps^6 relative) at
        # eps = 5e-3 is far below the bound while dividing the rounding noise
        # by ~4 against a four-point difference at eps = 1e-3.
        eps = 5e-3
        fd = (45 * (loss_f(n, i, eps) - loss_f(n, i, -eps)) - 9 * (loss_f(n, i, 2 * eps) - loss_f(n, i, -2 * eps))
              + (loss_f(n, i, 3 * eps) - loss_f(n, i, -3 * eps))) / (60 * eps)
        ad = gs.reshape(19, -1)[i, n]
        rel = abs(fd - ad) / max(abs(fd), 1e-3 * smax)
        worst_f = max(worst_f, rel)
        log(f"   f node {n} i {i}: fd {fd:.10e} adjoint {ad:.10e} rel {rel:.2e}")
        assert rel <= 1e-6
    log(f"   L {L0:.6e}; worst g rel err {worst:.2e}; worst f0 rel err {worst_f:.2e}")


# FP32 storage and arithmetic (gradients still summed in FP64).  Each adjoint
# step evaluates every value with O(Q) FP32 operations, so its rounding is a
# few Q * 2^-24 of the largest adjoint value; over T steps the errors add up:
# bound T * Q * 2^-24 * 8 relative to the largest gradient entry.
F32_EPS = 2.0 ** -24


@pytest.mark.parametrize("periodic,K,K2,model", [(7, 5, None, "qc"), (0, 6, 2, "qc"), (7, 4, None, "inc"),
                                                  (7, 4, None, "mrt-qc"), (0, 6, 2, "mrt-inc")])
def test_adjoint_f32_matches_oracle(periodic, K, K2, model):
    import torch
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    tau, T = 0.8, 12
    s, _ = I.sphere_pack((12, 16, 12), 0.55, 2.0, 3.5, seed=22, periodic=bool(periodic & 1))
    sp = padded(s, periodic)
    f0 = perturbed_state(sp, 5)
    g = _force_field(sp, 6)
    log(f"[case] f32 adjoint vs oracle periodic={periodic} K={K} K2={K2} T={T} model={model}")
    Lo, gs_o, gF_o = O.adjoint(f0, sp, tau, g, T, periodic=periodic, model=O.MODELS[model])
    lat = new_lattice(s, tau, periodic, storage="f32", model=model)
    lat.set_force(torch.from_numpy(g).cuda())
    run = CheckpointedAdjoint(lat, T, K, K2)
    L = run.forward(torch.from_numpy(f0))
    gs, gg = run.backward()
    gs, gg = gs.cpu().numpy(), gg.cpu().numpy()
    fl = sp == 0
    tol = T * 19 * F32_EPS * 8
    es = np.max(np.abs(gs[:, fl] - gs_o[:, fl])) / np.abs(gs_o[:, fl]).max()
    eg = np.max(np.abs(gg[:, fl] - gF_o[:, fl])) / np.abs(gF_o[:, fl]).max()
    # the loss is a mean of u_x; each u_x carries at most the same relative
    # rounding bound times max|u|
    mi = O.MODELS[model]
    _, u = O.macroscopic(O.run(f0, sp, tau, T, force=g, periodic=periodic, model=mi), sp, force=g, model=mi)
    umax = np.abs(u[:, fl]).max()
    # per entry: the same relative bound with an absolute floor at 1e-2 of the
    # largest entry (FP32 rounding of a node's adjoint values scales with the
    # largest values that node combines, not with each entry)
    es_e = elementwise_err(gs, gs_o, fl, 1e-2)
    eg_e = elementwise_err(gg, gF_o, fl, 1e-2)
    log(f"   L {L:.9e} vs {Lo:.9e} (tol {tol * umax:.2e});  dL/ds0 err {es:.2e} (per entry {es_e:.2e})  "
        f"dL/dg err {eg:.2e} (per entry {eg_e:.2e})  tol {tol:.2e}")
    assert abs(L - Lo) <= tol * umax
    assert es <= tol and eg <= tol
    assert es_e <= tol and eg_e <= tol
    assert np.all(gs[:, ~fl] == 0) and np.all(gg[:, ~fl] == 0)


def test_reverse_gather_is_transpose_of_pull_f32():
    """FP32 adjoint lattices: the reverse gather and the propagation-only
    kernel move values without arithmetic, so both match the oracle's S and
    S^T exactly on FP32-representable inputs."""
    import torch
    s, _ = I.sphere_pack((16, 16, 16), 0.5, 2.0, 4.0, seed=32)
    sp = padded(s, 7)
    fl = (sp == 0)[None]
    rng = np.random.default_rng(8)
    v = (rng.normal(size=(19,) + sp.shape) * fl).astype(np.float32).astype(np.float64)
    w = (rng.normal(size=(19,) + sp.shape) * fl).astype(np.float32).astype(np.float64)
    lat = new_lattice(s, 0.8, 7, storage="f32")
    a, b = lat.new_adjoint(), lat.new_adjoint()
    lat.adjoint_set(torch.from_numpy(v), a)
    assert np.array_equal(lat.adjoint_get(a).cpu().numpy(), v)
    lat.calib_step(2, a, b)
    assert np.array_equal(lat.adjoint_get(b).cpu().numpy(), O.pull(v, sp, periodic=7))
    lat.adjoint_set(torch.from_numpy(w), a)
    lat.adjoint_final(a, b)
    assert np.array_equal(lat.adjoint_get(b).cpu().numpy(), O.pull_transpose(w, sp, periodic=7))


def test_multi_level_schedules_are_bitwise_one_level():
    """The schedule only changes which forward states are recomputed when;
    the kernels are deterministic, so the gradients are bitwise equal."""
    import torch
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    tau, T = 0.7, 29
    s, _ = I.sphere_pack((16, 16, 20), 0.5, 2.0, 4.0, seed=51)
    sp = padded(s, 7)
    f0 = torch.from_numpy(perturbed_state(sp, 9))
    g = torch.from_numpy(_force_field(sp, 10)).cuda()
    out = []
    for iv in ((5,), (29,), (10, 3), (12, 5), (15, 6, 2)):
        lat = new_lattice(s, tau, 7)
        lat.set_force(g)
        run = CheckpointedAdjoint(lat, T, *iv)
        L = run.forward(f0)
        gs, gg = run.backward()
        out.append((L, gs.cpu().numpy(), gg.cpu().numpy()))
    for L, gs, gg in out[1:]:
        assert L == out[0][0]
        assert np.array_equal(gs, out[0][1]) and np.array_equal(gg, out[0][2])


def test_adjoint_f32_against_f64_sphere_pack():
    """64^3 sphere pack, T = 300: FP32 gradients against the FP64 library
    adjoint (itself pinned to the oracle above), same relative bound."""
    import torch
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    tau, T, K = 0.8, 300, 20
    s, _ = I.sphere_pack((64, 64, 64), 0.5, 3.0, 8.0, seed=61)
    sp = padded(s, 7)
    g = torch.from_numpy(_force_field(sp, 11, mean=1e-6, std=1e-7)).cuda()
    res = {}
    for st in ("f64", "f32"):
        lat = new_lattice(s, tau, 7, storage=st)
        lat.set_force(g)
        lat.init()
        run = CheckpointedAdjoint(lat, T, K)
        L = run.forward(None)
        gs, gg = run.backward()
        res[st] = (L, gs.cpu().numpy(), gg.cpu().numpy())
    fl = sp == 0
    tol = T * 19 * F32_EPS * 8
    es = np.max(np.abs(res["f32"][1][:, fl] - res["f64"][1][:, fl])) / np.abs(res["f64"][1][:, fl]).max()
    eg = np.max(np.abs(res["f32"][2][:, fl] - res["f64"][2][:, fl])) / np.abs(res["f64"][2][:, fl]).max()
    eL = abs(res["f32"][0] - res["f64"][0]) / abs(res["f64"][0])
    log(f"   64^3 T={T}: L rel {eL:.2e}  dL/ds0 err {es:.2e}  dL/dg err {eg:.2e}  tol {tol:.2e}")
    assert es <= tol and eg <= tol
    assert eL <= 1e-3


@pytest.mark.parametrize("storage,model", [("f64", "qc"), ("f32", "qc"), ("f64", "mrt-qc")])
def test_adjoint_independent_of_launch_configuration(storage, model):
    """Tile order, tiles per workgroup and 64-bit offsets change where tiles
    live and when they run, not what an adjoint step computes per node: the
    gradients are bitwise equal (the loss, an FP64 sum in tile order, to the
    last bits).  The library's own choice (one tile per workgroup for the
    FP64 LBMRT adjoint, four otherwise) is one of the configurations."""
    import torch
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    tau, T = 0.75, 17
    s, _ = I.sphere_pack((20, 16, 24), 0.5, 2.0, 4.0, seed=61)
    sp = padded(s, 7)
    f0 = torch.from_numpy(perturbed_state(sp, 12))
    g = torch.from_numpy(_force_field(sp, 13)).cuda()
    out = []
    for kw in (dict(), dict(tiles_per_wg=4), dict(tile_order=1), dict(tile_order=2), dict(tile_order=3),
               dict(tile_order=5), dict(tile_order=4, tiles_per_wg=1), dict(tiles_per_wg=8), dict(wide_offsets=True)):
        lat = new_lattice(s, tau, 7, storage=storage, model=model, **kw)
        lat.set_force(g)
        run = CheckpointedAdjoint(lat, T, 6)
        L = run.forward(f0)
        gs, gg = run.backward()
        log(f"[case] adjoint {storage} {model} {kw}: L {L:.15e}")
        out.append((L, gs.cpu().numpy(), gg.cpu().numpy()))
    for L, gs, gg in out[1:]:
        assert abs(L - out[0][0]) <= 1e-14 * abs(out[0][0])
        assert np.array_equal(gs, out[0][1]) and np.array_equal(gg, out[0][2])


def test_adjoint_refuses_what_it_does_not_differentiate():
    from paper_1611_02445_amd._abi import LbmError
    s, _ = I.sphere_pack((12, 12, 12), 0.55, 2.0, 3.5, seed=23)
    lat = new_lattice(s, 0.8, 7, storage="f16s")
    lat.init()
    with pytest.raises(LbmError, match="UNSUPPORTED"):
        lat.adjoint_seed(lat.current_state(), lat.new_state(), lat.new_grad())
    lat = new_lattice(s, 0.8, 7)
    lat.init()
    types = np.zeros(padded(s, 7).shape, np.uint8)
    lat.set_boundaries(types, u_in=(0.01, 0.0, 0.0))
    with pytest.raises(LbmError, match="UNSUPPORTED"):
        lat.adjoint_seed(lat.current_state(), lat.new_adjoint(), lat.new_grad())


def _random_adjoint_cases(n, seed):
    rng = np.random.default_rng(seed)
    models = ["qc", "inc", "mrt-qc", "mrt-inc"]
    for k in range(n):
        periodic = int(rng.integers(0, 8))
        dims = []
        for axis in range(3):
            d = int(rng.integers(5, 17))
            if periodic >> axis & 1:
                d = max(4, d // 4 * 4)
            dims.append(d)
        nx, ny, nz = dims
        solid = I.random_bitmap((nz, ny, nx), float(rng.uniform(0.1, 0.7)), seed=int(rng.integers(1 << 30)))
        yield (k, solid, periodic, float(rng.uniform(0.6, 1.2)), models[k % 4], int(rng.integers(2, 8)),
               int(rng.integers(1 << 30)))


@pytest.mark.parametrize("case", list(_random_adjoint_cases(8, 77)), ids=lambda c: f"rand{c[0]}")
def test_adjoint_random_geometries(case):
    import torch
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    k, s, periodic, tau, model, K, seed = case
    if (s == 0).sum() == 0:
        pytest.skip("no fluid node")
    T = 9
    sp = padded(s, periodic)
    f0 = perturbed_state(sp, seed % 1000)
    g = _force_field(sp, seed % 997)
    log(f"[case] adjoint random{k} shape={s.shape} periodic={periodic} tau={tau:.2f} model={model} K={K}")
    Lo, gs_o, gF_o = O.adjoint(f0, sp, tau, g, T, periodic=periodic, model=O.MODELS[model])
    lat = new_lattice(s, tau, periodic, model=model)
    lat.set_force(torch.from_numpy(g).cuda())
    run = CheckpointedAdjoint(lat, T, K)
    run.forward(torch.from_numpy(f0))
    gs, gg = run.backward()
    gs, gg = gs.cpu().numpy(), gg.cpu().numpy()
    fl = sp == 0
    es = elementwise_err(gs, gs_o, fl, F64_FLOOR)
    eg = elementwise_err(gg, gF_o, fl, F64_FLOOR)
    log(f"   per-entry dL/ds0 err {es:.2e}  dL/dg err {eg:.2e}")
    assert es <= F64_TOL and eg <= F64_TOL
