"""Reduced-precision storage (FP32 shifted, FP16 shifted with a power-of-two
scale; FP32 arithmetic) against the FP64 oracle and the GPU FP64 result.

Tolerances follow from the storage formats.  A stored value is the shifted
d_i = f_i - w_i rho0 (|d_i| ~ 1e-3..1e-2 here), rounded once per step:
  FP32: relative 2^-24 of d_i per step, so after n steps the error in f_i is
        below n * 2^-24 * max|d| (plus FP32 arithmetic of the same order);
  FP16: h = fp16(2^k d) has an 11-bit significand: the error per step is
        below one ulp, 2^-10 * |d| (stochastic rounding, the default) or half
        an ulp (nearest-even), i.e. ~1e-6 here.
The target for both is |k - k_64| / k_64 <= 1e-3 on the permeability;
velocity errors are reported."""
import numpy as np
import pytest

import oracle as O
from paper_1611_02445_amd import inputs as I

from helpers import log, new_lattice, padded, perturbed_state

pytestmark = pytest.mark.gpu


def _run(solid, tau, periodic, storage, steps, g, f0=None, **kw):
    import torch
    lat = new_lattice(solid, tau, periodic, storage=storage, **kw)
    lat.init()
    if f0 is not None:
        lat.set_state(torch.from_numpy(f0))
    lat.set_force(g)
    lat.step(steps)
    return lat


@pytest.mark.parametrize("storage,model", [("f32", "qc"), ("f16s", "qc"), ("f32", "inc"), ("f16s", "inc"),
                                           ("f32u", "qc"), ("f32", "mrt-qc"), ("f16s", "mrt-qc"),
                                           ("f32", "mrt-inc")])
def test_reduced_storage_against_oracle(storage, model):
    tau, steps, g = 0.7, 100, (1e-5, 2e-6, 0.0)
    s, _ = I.sphere_pack((24, 24, 24), 0.5, 2.0, 5.0, seed=51)
    sp = padded(s, 7)
    f0 = perturbed_state(sp, 8, amp=0.01)
    kw = dict(model=model)
    if storage == "f32u":  # FP32 of f itself: rounding relative to |f|, not |f - w rho0|
        kw["f32_unshifted"] = True
    lat = _run(s, tau, 7, "f32" if storage == "f32u" else storage, steps, g, f0=f0, **kw)
    got = lat.get_state().cpu().numpy()
    ref = O.run(f0, sp, tau, steps, force=np.array(g), periodic=7, model=O.MODELS[model])
    fl = sp == 0
    c, w, _ = O.lattice()
    shift = 0.0 if storage == "f32u" else 1.0
    d = np.abs(ref - shift * w[:, None, None, None])[:, fl].max()
    err = np.abs(got[:, fl] - ref[:, fl]).max()
    bound = steps * 2.0 ** -24 * d * 8 if storage in ("f32", "f32u") else steps * 2.0 ** -10 * d
    log(f"[case] {storage} {model}: max |df| {err:.3e}, bound {bound:.3e}, max|d| {d:.3e}")
    assert err <= bound


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_rest_state_exact(storage):
    import torch
    s, _ = I.sphere_pack((16, 16, 16), 0.5, 2.0, 4.0, seed=52)
    lat = _run(s, 0.8, 7, storage, 200, (0.0, 0.0, 0.0))
    f0 = _run(s, 0.8, 7, storage, 0, (0.0, 0.0, 0.0)).get_state()
    assert torch.equal(lat.get_state(), f0)
    raw = lat.current_state()
    # shifted storage of a rest state is exactly zero in every slot
    assert int(torch.count_nonzero(raw)) == 0


def test_fp16_overflow_is_reported():
    import torch
    from paper_1611_02445_amd._abi import LbmError
    s, _ = I.sphere_pack((16, 16, 16), 0.5, 2.0, 4.0, seed=53)
    sp = padded(s, 7)
    f0 = perturbed_state(sp, 9, amp=0.2)
    lat = new_lattice(s, 0.8, 7, storage="f16s", f16_log2_scale=30)  # 2^30 * 0.05 > 65504
    lat.init()
    lat.set_state(torch.from_numpy(f0))
    with pytest.raises(LbmError, match="LBM_E_NUMERIC"):
        lat.macroscopic(fields=False)


def test_vessel_tree_512_storage_variants():
    """The 512^3 vessel network (about 5% fluid), tau 0.6, g_x 1e-5: FP64
    checked node by node against the oracle on sampled nodes; FP32 and FP16
    storage against FP64 after 20000 steps."""
    import torch
    tau, g, steps = 0.6, 1e-5, 20000
    s, L0 = I.vessel_tree(n=512)
    sp = padded(s, 7)
    log(f"[case] vessel512 L0={L0:.1f} fluid={1 - s.mean():.4f}")
    lat64 = _run(s, tau, 7, "f64", steps - 1, (g, 0.0, 0.0))
    prev = lat64.get_state().cpu().numpy()
    lat64.step(1)
    rng = np.random.default_rng(1)
    nodes = rng.choice(np.flatnonzero(sp.ravel() == 0), 2048, replace=False)
    cur = lat64.get_state().view(19, -1)[:, torch.from_numpy(nodes).cuda()].cpu().numpy()
    ref = O.step_nodes(prev, sp, tau, nodes, force=[g, 0, 0], periodic=7)
    e64 = np.max(np.abs(cur.T - ref) / np.abs(ref))
    del prev, cur
    torch.cuda.empty_cache()
    _, u64, s64 = lat64.macroscopic()
    k64 = lat64.permeability(g)
    log(f"   f64: tiles={lat64.n_tiles} eta_t={lat64.tiling.eta_t:.3f} k={k64:.6e} sampled err {e64:.2e}")
    assert e64 <= 1e-12
    nrm = torch.linalg.vector_norm(u64).item()
    for st, rounding in (("f32", "stochastic"), ("f16s", "stochastic"), ("f16s", "nearest")):
        lat = _run(s, tau, 7, st, steps, (g, 0.0, 0.0), f16_rounding=rounding)
        _, u, sums = lat.macroscopic()
        k = lat.permeability(g)
        du = torch.linalg.vector_norm(u - u64).item() / nrm
        dk = abs(k - k64) / abs(k64)
        dm = (sums[0] - s64[0]) / s64[0]
        log(f"   {st} ({rounding}): k={k:.6e} |dk|/k={dk:.2e} |du|/|u|={du:.2e} mass drift {dm:.2e}")
        if rounding == "stochastic":
            assert dk <= 1e-3
        del lat
