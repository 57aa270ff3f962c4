#!/usr/bin/env python3
"""Throughput of the fused tiled D3Q19 step on one MI355X.

Workload: a 256^3 periodic box of randomly placed, overlapping solid spheres
(radius uniform in [4, 12), seeded centres) added until the porosity is 0.4;
FP64 storage and arithmetic, LBGK tau = 0.7, uniform body force g_x = 1e-6,
4^3 tiles with all-solid tiles skipped.  A step is one fused
collide-and-stream update of every fluid node (one kernel launch); the timed
region holds exactly --steps steps with the lattice resident in HBM, after
--warmup untimed steps and ~200 ms of streaming work that brings an idle GPU
to its working clocks.

Prints one JSON line: MFLUPS (million fluid-node updates per second), the
roofline of the step kernel (algorithmic bytes per launch / average launch
time, against 8 TB/s and against the copy bandwidth the streaming probes
measure first), the CPU oracle timed on a bounded sample of the same
workload (all host threads and one), permeability after the run, and the
FP32 / FP16-shifted storage variants with their errors against the FP64
result, stated on a fixed run of --error-steps steps from rest.
"""
import argparse
import json
import os
import re
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "MFLUPS + % HBM roofline, FP64 vs FP32/FP16 storage at stated error; adjoint MFLUPS"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {"f64": 2 * 19 * 8, "f32": 2 * 19 * 4, "f32u": 2 * 19 * 4, "f16s": 2 * 19 * 2}
PROFILE_DIR = os.path.join(HERE, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counter_traffic(kernel_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    kernel (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or
    None when there is none or the kernel source changed since it was taken."""
    path = os.path.join(PROFILE_DIR, f"counters_{kernel_tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    from paper_1611_02445_amd.profiling import kernel_source_hash
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def build_case(args):
    from paper_1611_02445_amd import inputs
    t0 = time.time()
    solid, n_sph = inputs.sphere_pack((args.n, args.n, args.n), args.porosity, 4.0, 12.0, seed=args.seed)
    log(f"[bench] geometry {args.n}^3 spheres={n_sph} porosity={1 - solid.mean():.4f} ({time.time() - t0:.1f}s)")
    return solid


def bring_to_clock(torch, ms=200.0):
    """About `ms` of streaming-probe copies on scratch buffers, synchronised,
    right before a timed region.  A GPU that has idled (host work between
    measurements) starts a step run at lower clocks: the first ~30 FP64 steps
    after a lattice is created run at 430-442 us, settling to 413 by step ~40,
    while after 200 ms of streaming they run at 413-417 from the first one.
    A simulation runs ~10^5 steps at the working clocks, so the timed region
    starts there."""
    import ctypes
    from paper_1611_02445_amd import _abi
    a = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(10):
            _abi.call("lbm_stream_probe", ctypes.c_void_p(st.cuda_stream), 3, ctypes.c_void_p(a.data_ptr()),
                      ctypes.c_void_p(b.data_ptr()), a.numel() * 8, 65536, 256)
        torch.cuda.synchronize()
    del a, b


def time_storage(solid, storage, args, torch, want_state=False, model="qc"):
    from paper_1611_02445_amd.lattice import Lattice
    # "f32u": FP32 storage of f itself (the paper's form), an ablation of the shift
    # check_u_max: every macroscopic call of the run fails if the compressibility
    # limit u_max <= 0.05 (Section 2.2) is exceeded
    lat = Lattice(solid, args.tau, periodic=7, storage="f32" if storage == "f32u" else storage, model=model,
                  tiles_per_wg=args.tpw, tile_order=args.order, f32_unshifted=storage == "f32u", check_u_max=True)
    lat.init()
    lat.set_force((args.g, 0.0, 0.0))
    log(f"[bench] {storage}: tiles={lat.n_tiles} fluid={lat.n_fluid} eta_t={lat.tiling.eta_t:.4f}")
    torch.cuda.synchronize()
    bring_to_clock(torch)
    lat.step(args.warmup)
    stream = lat.stream
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    lat.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    # per-launch spread over a fixed number of separately timed launches (the
    # paper times every launch separately), whatever --steps is
    nlaunch = 500
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(nlaunch + 1)]
    evs[0].record(stream)
    for k in range(nlaunch):
        lat.step(1)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(nlaunch)])
    steps_done = args.warmup + args.steps + nlaunch
    k = lat.permeability(args.g)
    _, _, sums = lat.macroscopic(fields=False)
    out = dict(lat=lat, wall=wall, gpu_ms=gpu_ms, per=per, steps_done=steps_done, k=k, sums=sums)
    if want_state:
        out["u"] = lat.macroscopic()[1]
    return out


def time_calib(solid, args, torch, kernel=None, launches=None, lat=None, storage="f64"):
    """The paper's measurement kernels (Section 4.1) on the same tiles,
    storage and launch shape as the step: "read/write only" (rw) and
    "propagation only" (prop)."""
    from paper_1611_02445_amd.lattice import Lattice
    kernel = kernel or args.kernel
    launches = launches or args.steps
    kind = 1 if kernel == "rw" else 2
    if lat is None:
        lat = Lattice(solid, args.tau, periodic=7, storage=storage, tiles_per_wg=args.tpw, tile_order=args.order)
        lat.init()
    a, b = lat.new_state(), lat.new_state()
    a.copy_(lat.current_state())
    for _ in range(args.warmup):
        lat.calib_step(kind, a, b)
        a, b = b, a
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(lat.stream)
    for _ in range(launches):
        lat.calib_step(kind, a, b)
        a, b = b, a
    ev1.record(lat.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / launches
    nf = lat.n_fluid
    gbs = BYTES_PER_UPDATE[storage] * nf / (ms / 1e3) / 1e9
    log(f"[bench] {kernel}-only {storage}: {nf / (ms / 1e3) / 1e6:.1f} MFLUPS, {ms * 1e3:.1f} us, {gbs:.0f} GB/s")
    return {"kernel": kernel, "ms_per_launch": ms, "MFLUPS": nf / (ms / 1e3) / 1e6, "GBs": gbs,
            "frac": gbs / HBM_PEAK_GBS, "fluid_nodes": nf, "tiles": lat.n_tiles}


def time_adjoint(args, torch):
    """Adjoint throughput on the 128^3 periodic sphere pack (porosity 0.5,
    radius U[4,12), seed 4), FP64, tau 0.8, per-node g_x ~ N(1e-6, 1e-7),
    T steps with checkpoints every K: MFLUPS of the reverse sweep with and
    without the forward recomputation it needs."""
    from paper_1611_02445_amd import inputs
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    from paper_1611_02445_amd.lattice import Lattice
    solid, _ = inputs.sphere_pack((128, 128, 128), 0.5, 4.0, 12.0, seed=4)
    lat = Lattice(solid, 0.8, periodic=7, tiles_per_wg=args.tpw, tile_order=args.order)
    rng = np.random.default_rng(40)
    g = torch.zeros((3,) + lat.dense_shape, dtype=torch.float64)
    g[0] = torch.from_numpy(rng.normal(1e-6, 1e-7, lat.dense_shape))
    lat.set_force(g.cuda())
    lat.init()
    T, K = args.adj_steps, args.adj_k
    run = CheckpointedAdjoint(lat, T, K)
    run.forward(None)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(lat.stream)
    run.backward()
    ev[1].record(lat.stream)
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[1])
    # the adjoint kernels alone: T sweeps over ring buffers already filled
    e_in, e_out = run.eta
    s = run.ring[0]
    ev[2].record(lat.stream)
    lat.adjoint_seed(s, e_in, run.grad)
    for _ in range(T - 1):
        lat.adjoint_step(s, e_in, e_out, run.grad)
        e_in, e_out = e_out, e_in
    ev[3].record(lat.stream)
    torch.cuda.synchronize()
    kern_ms = ev[2].elapsed_time(ev[3])
    nf = lat.n_fluid
    out = {"workload": "128^3 sphere pack porosity 0.5, FP64, tau 0.8, per-node g_x ~ N(1e-6,1e-7)",
           "T": T, "K": K, "fluid_nodes": nf, "memory_GB": round(run.memory_bytes() / 1e9, 2),
           "MFLUPS_adjoint_kernels": round(nf * T / (kern_ms / 1e3) / 1e6, 1),
           "MFLUPS_backward_incl_recompute": round(nf * T / (total_ms / 1e3) / 1e6, 1),
           "recompute_steps": run.recompute_steps,
           # two gathered lattices and one written, the force density read,
           # the FP64 gradient read and written
           "bytes_per_fluid_update_adjoint": 3 * 19 * 8 + 3 * 8 + 2 * 3 * 8}
    ms = kern_ms / T
    out["adjoint_hbm_frac"] = round(out["bytes_per_fluid_update_adjoint"] * nf / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    log(f"[bench] adjoint: {out['MFLUPS_adjoint_kernels']} MFLUPS kernels, "
        f"{out['MFLUPS_backward_incl_recompute']} MFLUPS incl. recompute")
    del run, lat
    # the adjoint kernels of the other collision models on the same pack
    # (200 reverse steps over one recomputed state each)
    other = {}
    for model in ("inc", "mrt-qc", "mrt-inc"):
        lm = Lattice(solid, 0.8, periodic=7, model=model, tiles_per_wg=args.tpw, tile_order=args.order)
        lm.set_force(g.cuda())
        lm.init()
        s_buf, e_in, e_out, grad = lm.current_state(), lm.new_adjoint(), lm.new_adjoint(), lm.new_grad()
        lm.adjoint_seed(s_buf, e_in, grad)
        for _ in range(10):
            lm.adjoint_step(s_buf, e_in, e_out, grad)
            e_in, e_out = e_out, e_in
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lm.stream)
        for _ in range(200):
            lm.adjoint_step(s_buf, e_in, e_out, grad)
            e_in, e_out = e_out, e_in
        e1.record(lm.stream)
        torch.cuda.synchronize()
        other[model] = round(lm.n_fluid * 200 / (e0.elapsed_time(e1) / 1e3) / 1e6, 1)
        del lm, e_in, e_out, grad
    out["MFLUPS_adjoint_step_other_models"] = other
    log(f"[bench] adjoint step, other models: {other}")
    return out


def time_vessel(args, torch, steps=500):
    """The 512^3 synthetic vessel network (binary tree of capsules, about 5%
    fluid, mirrored into loops through periodic x; tau 0.6, g_x 1e-5): step
    MFLUPS of FP64, FP32 and FP16-shifted storage on the sparsest geometry."""
    from paper_1611_02445_amd import inputs
    from paper_1611_02445_amd.lattice import Lattice
    t0 = time.time()
    solid, L0 = inputs.vessel_tree(n=512)
    out = {"workload": "512^3 vessel network, radius 24 x 0.8 per level, 8 levels, ~5% fluid; tau 0.6, g_x 1e-5",
           "fluid_fraction": round(float((solid == 0).mean()), 5), "steps": steps}
    log(f"[bench] vessel 512^3: fluid {out['fluid_fraction']:.4f} ({time.time() - t0:.1f}s)")
    for st in ("f64", "f32", "f16s"):
        lat = Lattice(solid, 0.6, periodic=7, storage=st, tiles_per_wg=args.tpw, tile_order=args.order,
                      check_u_max=True)
        lat.init()
        lat.set_force((1e-5, 0.0, 0.0))
        lat.step(20)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(lat.stream)
        lat.step(steps)
        ev1.record(lat.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        out.update(tiles=lat.n_tiles, tile_grid=lat.tiling.tx * lat.tiling.ty * lat.tiling.tz,
                   fluid_nodes=lat.n_fluid, eta_t=round(lat.tiling.eta_t, 4))
        out[st] = {"MFLUPS": round(lat.n_fluid / (ms / 1e3) / 1e6, 1), "us_per_step": round(ms * 1e3, 2),
                   "hbm_frac": round(BYTES_PER_UPDATE[st] * lat.n_fluid / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"[bench] vessel {st}: {out[st]['MFLUPS']} MFLUPS")
        lat.macroscopic(fields=False)  # u_max check
        del lat
        torch.cuda.empty_cache()
    return out


def time_pack1024(args, torch):
    """The 1024x512x512 periodic sphere pack (porosity 0.2, radius U[6,16),
    seed 5), FP32-shifted storage, tau 0.65, g_x 1e-5: 8000 forward steps, then
    2000 more with checkpoints sized to the free HBM and the adjoint of those
    2000; then FP64 against FP32 permeability on the 256^3 crop at the origin
    (treated as periodic) after 10000 steps each."""
    from paper_1611_02445_amd import inputs
    from paper_1611_02445_amd.autograd import CheckpointedAdjoint
    from paper_1611_02445_amd.lattice import Lattice
    tau, g, T = 0.65, 1e-5, 2000
    t0 = time.time()
    solid, n_sph = inputs.sphere_pack((512, 512, 1024), 0.2, 6.0, 16.0, seed=5)
    log(f"[bench] pack1024: spheres={n_sph} porosity={1 - solid.mean():.4f} ({time.time() - t0:.1f}s)")
    lat = Lattice(solid, tau, periodic=7, storage="f32", tiles_per_wg=args.tpw, tile_order=args.order)
    lat.init()
    lat.set_force((g, 0.0, 0.0))
    nf = lat.n_fluid
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    lat.step(20)
    torch.cuda.synchronize()
    ev[0].record(lat.stream)
    lat.step(8000 - 20)
    ev[1].record(lat.stream)
    torch.cuda.synchronize()
    fwd_ms = ev[0].elapsed_time(ev[1]) / (8000 - 20)
    run = CheckpointedAdjoint.within_memory(lat, T)
    ev[2].record(lat.stream)
    L = run.forward(None)
    ev[3].record(lat.stream)
    run.backward(dense=False)
    ev[4].record(lat.stream)
    torch.cuda.synchronize()
    ckpt_fwd_ms = ev[2].elapsed_time(ev[3])
    back_ms = ev[3].elapsed_time(ev[4])
    e_in, e_out = run.eta
    s = run.ckpt[0]
    ev[5].record(lat.stream)
    lat.adjoint_seed(s, e_in, run.grad)
    for _ in range(T - 1):
        lat.adjoint_step(s, e_in, e_out, run.grad)
        e_in, e_out = e_out, e_in
    ev[6].record(lat.stream)
    torch.cuda.synchronize()
    kern_ms = ev[5].elapsed_time(ev[6])
    out = {"workload": "1024x512x512 periodic sphere pack, porosity 0.2, radius U[6,16), seed 5; "
                       "FP32-shifted storage, tau 0.65, g_x 1e-5; 10000 forward steps, adjoint of the last 2000",
           "tiles": lat.n_tiles, "fluid_nodes": nf, "eta_t": round(lat.tiling.eta_t, 4),
           "state_GB": round(lat.sizes.state_bytes / 1e9, 3),
           "forward_MFLUPS": round(nf / (fwd_ms / 1e3) / 1e6, 1),
           "forward_hbm_frac": round(BYTES_PER_UPDATE["f32"] * nf / (fwd_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
           "checkpointed_forward_MFLUPS": round(nf * T / (ckpt_fwd_ms / 1e3) / 1e6, 1),
           "adjoint_T": T, "checkpoint_intervals": run.intervals, "lattices": run.lattices(),
           "memory_GB": round(run.memory_bytes() / 1e9, 1), "recompute_steps": run.recompute_steps,
           "MFLUPS_adjoint_kernels": round(nf * T / (kern_ms / 1e3) / 1e6, 1),
           "MFLUPS_backward_incl_recompute": round(nf * T / (back_ms / 1e3) / 1e6, 1),
           # uniform force here: no force field to read
           "bytes_per_fluid_update_adjoint": 3 * 19 * 4 + 2 * 3 * 8,
           "loss": L}
    out["adjoint_hbm_frac"] = round(out["bytes_per_fluid_update_adjoint"] * nf / (kern_ms / T / 1e3) / 1e9
                                    / HBM_PEAK_GBS, 4)
    log(f"[bench] pack1024: forward {out['forward_MFLUPS']} MFLUPS, adjoint {out['MFLUPS_adjoint_kernels']} "
        f"MFLUPS kernels, {out['MFLUPS_backward_incl_recompute']} incl. recompute (intervals {run.intervals})")
    del run, lat
    torch.cuda.empty_cache()
    crop = np.ascontiguousarray(solid[:256, :256, :256])
    k = {}
    for st in ("f64", "f32"):
        lc = Lattice(crop, tau, periodic=7, storage=st)
        lc.init()
        lc.set_force((g, 0.0, 0.0))
        lc.step(10000)
        k[st] = lc.permeability(g)
        del lc
    out["crop256_permeability_f64"] = k["f64"]
    out["crop256_permeability_f32"] = k["f32"]
    out["crop256_rel_permeability_err"] = abs(k["f32"] - k["f64"]) / abs(k["f64"])
    log(f"[bench] pack1024 crop: dk/k {out['crop256_rel_permeability_err']:.2e}")
    return out


def _time_calib_kind(lat, kind, torch, launches=200, warmup=10):
    a, b = lat.new_state(), lat.new_state()
    a.copy_(lat.current_state())
    for _ in range(warmup):
        lat.calib_step(kind, a, b)
        a, b = b, a
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(lat.stream)
    for _ in range(launches):
        lat.calib_step(kind, a, b)
        a, b = b, a
    ev1.record(lat.stream)
    torch.cuda.synchronize()
    del a, b
    return ev0.elapsed_time(ev1) / launches


def sweep_layouts(args, torch):
    """The paper's intra-tile layout study (Section 3.3, Eqs. 11-13; Table 5):
    the propagation-only kernel with the per-direction slot maps XYZ, XYZ +
    zigzagNE, XYZ + YXZ and all three, and a face-major order for 128-byte
    lines, against the read/write-only kernel, on
    fully fluid boxes with bounce-back walls (the paper's 100^3 cavity, 25^3
    tiles, and a 256^3 one that no cache holds)."""
    from paper_1611_02445_amd.lattice import Lattice
    names = {1: "rw only", 3: "XYZ", 4: "XYZ + zigzagNE", 5: "XYZ + YXZ", 6: "all three", 7: "face-major"}
    rows = []
    for n in (100, 256):
        for st in ("f64", "f32"):
            lat = Lattice(np.zeros((n, n, n), np.uint8), 0.7, periodic=0, storage=st, tiles_per_wg=args.tpw,
                          tile_order=args.order)
            lat.init()
            for kind in (3, 4, 5, 6, 7, 1):
                ms = _time_calib_kind(lat, kind, torch, launches=max(10, min(200, args.steps)),
                                      warmup=max(2, min(10, args.warmup)))
                mf = lat.n_fluid / (ms / 1e3) / 1e6
                rows.append({"box": n, "storage": st, "layout": names[kind], "kind": kind, "us": round(ms * 1e3, 2),
                             "MFLUPS": round(mf, 1),
                             "bw_util": round(mf * 1e6 * BYTES_PER_UPDATE[st] / (HBM_PEAK_GBS * 1e9), 4)})
                log(f"[bench] layouts {n}^3 {st} {names[kind]}: {ms * 1e3:.1f} us, {mf:.0f} MFLUPS, "
                    f"{rows[-1]['bw_util']:.3f}")
            del lat
            torch.cuda.empty_cache()
    return rows


def time_small_grid(args, torch):
    """The 32^3 square duct (walls on the y and z faces, periodic in x; tau
    0.8, g_x 1e-6), FP64, 2000 steps: plain launches against replays of the
    32-step HIP graph (lbm_step_graphed).  A step of this grid takes about as
    long as launching it."""
    from paper_1611_02445_amd import inputs
    from paper_1611_02445_amd.lattice import Lattice
    solid = inputs.square_channel(32)
    out = {"workload": "square duct 32^3, FP64, 2000 steps"}
    for graphed in (False, True):
        lat = Lattice(solid, 0.8, periodic=1)
        lat.init()
        lat.set_force((1e-6, 0.0, 0.0))
        lat.step(64, graphed=graphed)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(lat.stream)
        lat.step(2000, graphed=graphed)
        ev1.record(lat.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = ev0.elapsed_time(ev1)
        key = "graphed" if graphed else "plain"
        out[key] = {"MFLUPS": round(lat.n_fluid * 2000 / (ms / 1e3) / 1e6, 1), "us_per_step": round(ms / 2, 3),
                    "wall_us_per_step": round(wall * 1e6 / 2000, 2)}
        del lat
    log(f"[bench] duct 32^3: plain {out['plain']['MFLUPS']} MFLUPS, graphed {out['graphed']['MFLUPS']} MFLUPS")
    return out


def sweep_cavity(args, torch):
    """The paper's dense-geometry study (Section 4.2, Table 3 and the cavity3D
    figures): lid-driven b^3 cavities (bounce-back walls, the top fluid layer
    a velocity node moving at 0.05 along x; the LBMRT kernels without the
    lid, which drives them unstable), every kernel (the
    read/write-only and propagation-only kernels, LBGK and LBMRT in both
    equilibria) in FP64 and FP32, from b = 20 up; per kernel the best MFLUPS,
    the b it was reached at, and the largest case."""
    from paper_1611_02445_amd.lattice import Lattice, Tiling
    sizes = (20, 32, 48, 64, 80, 100, 101, 102, 103, 128, 160, 192, 224, 252, 320, 384)
    kernels = ("rw", "prop", "inc", "qc", "mrt-inc", "mrt-qc")
    rows = []
    for b in sizes:
        tiling = Tiling(np.zeros((b, b, b), np.uint8), 0)
        steps = int(min(2000, max(50, 4e8 / b ** 3)))
        row = {"b": b, "nodes": b ** 3, "eta_t": round(tiling.eta_t, 4), "steps": steps}
        for st in ("f64", "f32"):
            for k in kernels:
                lat = Lattice(None, 0.7, periodic=0, storage=st, model=k if k not in ("rw", "prop") else "qc",
                              tiling=tiling)
                lat.init()
                if k in ("inc", "qc"):  # LBMRT under this lid grows unstable; walls only
                    lid = np.zeros(lat.dense_shape, np.uint8)
                    lid[b - 1, :b, :b] = 11  # velocity node rebuilding c_z = -1
                    lat.set_boundaries(lid, u_in=(0.05, 0.0, 0.0))
                if k in ("rw", "prop"):
                    ms = _time_calib_kind(lat, 1 if k == "rw" else 2, torch, launches=steps, warmup=10)
                else:
                    lat.step(10)
                    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    ev0.record(lat.stream)
                    lat.step(steps)
                    ev1.record(lat.stream)
                    torch.cuda.synchronize()
                    ms = ev0.elapsed_time(ev1) / steps
                row[f"MFLUPS_{st}_{k}"] = round(lat.n_fluid / (ms / 1e3) / 1e6, 1)
                del lat
        torch.cuda.empty_cache()
        log(f"[bench] cavity {b}^3: f64 rw {row['MFLUPS_f64_rw']} prop {row['MFLUPS_f64_prop']} "
            f"qc {row['MFLUPS_f64_qc']} mrt-qc {row['MFLUPS_f64_mrt-qc']} | f32 qc {row['MFLUPS_f32_qc']} MFLUPS")
        rows.append(row)
    summary = {}
    for key in rows[0]:
        if not key.startswith("MFLUPS_"):
            continue
        best = max(rows, key=lambda r: r[key])
        bpn = BYTES_PER_UPDATE[key.split("_")[1]]
        summary[key[7:]] = {"max_MFLUPS": best[key], "b_at_max": best["b"], "largest_case": rows[-1][key],
                            "bw_util_at_max": round(best[key] * 1e6 * bpn / (HBM_PEAK_GBS * 1e9), 4)}
    return {"rows": rows, "summary": summary}


def sweep_sphere_arrays(args, torch):
    """Random sphere arrays of diameter 40 in a 192^3 periodic box at the nine
    porosities of the paper's sparse-geometry table (Section 4.6, Table 6):
    tile utilisation and MFLUPS of the step (FP64 and FP32, both models)."""
    from paper_1611_02445_amd import inputs
    from paper_1611_02445_amd.lattice import Lattice
    rows = []
    for p in (1.0, 0.9, 0.8, 0.7, 0.6, 0.5, 0.4, 0.3, 0.2, 0.1):
        if p == 1.0:  # the dense normaliser: a fully fluid box with bounce-back walls
            solid = np.zeros((192, 192, 192), np.uint8)
        else:
            solid, _ = inputs.sphere_pack((192, 192, 192), p, 20.0, 20.0, seed=11)
        row = {"porosity": p}
        per = 0 if p == 1.0 else 7
        lat = Lattice(solid, 0.7, periodic=per, storage="f64")
        lat.init()
        for kind, name in ((1, "rw"), (2, "prop")):
            row[f"MFLUPS_f64_{name}"] = round(lat.n_fluid / (_time_calib_kind(lat, kind, torch, 500) / 1e3) / 1e6, 1)
        del lat
        for st in ("f64", "f32"):
            for model in ("inc", "qc", "mrt-inc", "mrt-qc"):
                lat = Lattice(solid, 0.7, periodic=per, storage=st, model=model)
                lat.init()
                lat.set_force((1e-6, 0.0, 0.0))
                lat.step(args.warmup)
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record(lat.stream)
                lat.step(500)
                ev1.record(lat.stream)
                torch.cuda.synchronize()
                row["eta_t"] = round(lat.tiling.eta_t, 4)
                row["fluid_nodes"] = lat.n_fluid
                row[f"MFLUPS_{st}_{model}"] = round(lat.n_fluid * 500 / (ev0.elapsed_time(ev1) / 1e3) / 1e6, 1)
                del lat
        log(f"[bench] spheres192 porosity {p}: eta_t {row['eta_t']} f64 qc {row['MFLUPS_f64_qc']} "
            f"f32 qc {row['MFLUPS_f32_qc']} MFLUPS")
        rows.append(row)
    # the paper's Fig. 12: each kernel's MFLUPS over its dense-box MFLUPS
    # against tile utilisation, and the slope alpha of the line through
    # (1, 1) that fits it: normalised ~ 1 - alpha (1 - eta_t)
    dense, sparse = rows[0], rows[1:]
    fits = {}
    for key in dense:
        if not key.startswith("MFLUPS_"):
            continue
        x = np.array([1.0 - r["eta_t"] for r in sparse])
        y = np.array([1.0 - r[key] / dense[key] for r in sparse])
        for r in sparse:
            r["norm_" + key[7:]] = round(r[key] / dense[key], 4)
        fits[key[7:]] = round(float((x * y).sum() / (x * x).sum()), 4)
    return {"rows": rows, "alpha": fits}


def sweep_channels(args, torch):
    """The paper's propagation study (Section 4.4, Eqs. 17-19) on this GPU:
    fully fluid rectangular channels of ~2^24 nodes (walls by bounce-back),
    from 4 x 4 x L to 256 x 256 x 256, timed with the propagation-only kernel.
    eta_f / eta_e = common tile faces / edges per tile."""
    from paper_1611_02445_amd.lattice import Lattice
    N = 1 << 24
    rows = []
    sides = (4, 8, 16, 32, 64, 128, 256)
    for a in sides:
        for b in sides:
            if b < a:
                continue
            c = max(4, (N // (a * b)) // 4 * 4)
            if c < b:
                continue
            A, B, C = a // 4, b // 4, c // 4
            T = A * B * C
            eta_f = ((A - 1) * B * C + A * (B - 1) * C + A * B * (C - 1)) / T
            eta_e = ((A - 1) * (B - 1) * C + (A - 1) * B * (C - 1) + A * (B - 1) * (C - 1)) / T
            solid = np.zeros((c, b, a), dtype=np.uint8)
            lat = Lattice(solid, 0.7, periodic=0)
            lat.init()
            x, y = lat.new_state(), lat.new_state()
            x.copy_(lat.current_state())
            for _ in range(10):
                lat.calib_step(2, x, y)
                x, y = y, x
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(lat.stream)
            for _ in range(100):
                lat.calib_step(2, x, y)
                x, y = y, x
            ev1.record(lat.stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / 100
            mf = lat.n_fluid / (ms / 1e3) / 1e6
            rows.append({"dims": [a, b, c], "eta_f": round(eta_f, 4), "eta_e": round(eta_e, 4),
                         "MFLUPS": round(mf, 1),
                         "bw_util": round(mf * 1e6 * BYTES_PER_UPDATE["f64"] / (HBM_PEAK_GBS * 1e9), 4)})
            log(f"[bench] channel {a}x{b}x{c}: eta_f {eta_f:.3f} eta_e {eta_e:.3f} "
                f"{mf:.0f} MFLUPS, {rows[-1]['bw_util']:.3f}")
            del lat, x, y
    X = np.array([[1.0, r["eta_f"], r["eta_e"]] for r in rows])
    yv = np.array([r["bw_util"] for r in rows])
    coef = np.linalg.lstsq(X, yv, rcond=None)[0]
    return {"rows": rows, "plane_fit": {"bw_util_at_0": round(float(coef[0]), 4),
                                        "per_face": round(float(coef[1]), 5), "per_edge": round(float(coef[2]), 5)}}


def fp64_state_bytes(solid, args):
    import ctypes
    from paper_1611_02445_amd import _abi
    from paper_1611_02445_amd.lattice import Tiling
    t = Tiling(solid, 7)
    p = _abi.Params(tau=args.tau, rho0=1.0, storage=0, model=0, f16_log2_scale=20)
    sz = _abi.Sizes()
    _abi.call("lbm_required_bytes", t._ptr, ctypes.byref(p), ctypes.byref(sz))
    return sz.state_bytes


def probe_ceiling(nbytes, torch, launches=10):
    """What the GPU sustains for plain streaming over one lattice's bytes: the
    library's read-only, write-only and copy probes (16-byte non-temporal
    accesses) over a sweep of workgroup counts and sizes; the best rate of
    each (copy counted as bytes read + bytes written)."""
    import ctypes
    from paper_1611_02445_amd import _abi
    n = nbytes // 16 * 16
    a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    pa, pb = ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr())
    best = {}
    rows = []
    for kind, name, moved in ((1, "read", n), (2, "write", n), (3, "copy", 2 * n)):
        for threads in (256, 512, 1024):
            for blocks in (2048, 8192, 32768, 65536, 131072, 262144):
                def go():
                    _abi.call("lbm_stream_probe", sp, kind, pa, pb, n, blocks, threads)
                for _ in range(3):
                    go()
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record(stream)
                for _ in range(launches):
                    go()
                ev1.record(stream)
                torch.cuda.synchronize()
                ms = ev0.elapsed_time(ev1) / launches
                gbs = moved / (ms / 1e3) / 1e9
                rows.append((name, threads, blocks, round(ms * 1e3, 2), round(gbs, 1)))
                if gbs > best.get(name, {}).get("GBs", 0.0):
                    best[name] = {"GBs": round(gbs, 1), "us": round(ms * 1e3, 2), "threads": threads,
                                  "blocks": blocks}
    del a, b
    for name in ("read", "write", "copy"):
        log(f"[bench] probe {name}: {best[name]['GBs']:.0f} GB/s ({best[name]['threads']} x {best[name]['blocks']})")
    return {"bytes": n, "best": best, "peak_frac": {k: round(v["GBs"] / HBM_PEAK_GBS, 4) for k, v in best.items()},
            "sweep": rows}


def error_run(solid, args, torch, variants):
    """The stated error of the reduced-precision storage types: FP64 and each
    variant run from rest for --error-steps steps on the same geometry
    (tau, g_x as the timed run); permeability and velocity of each against
    the FP64 run, whose step the parity tests hold to the oracle node by
    node.  The FP64 permeability at half the steps shows how close the run
    is to steady flow."""
    from paper_1611_02445_amd.lattice import Lattice
    n = args.error_steps
    out = {"steps": n, "reference": "GPU FP64 on the same run (node-by-node oracle parity is tested)"}
    u64 = None
    for st in ["f64"] + [v for v in variants if v != "f64"]:
        lat = Lattice(solid, args.tau, periodic=7, storage="f32" if st == "f32u" else st,
                      tiles_per_wg=args.tpw, tile_order=args.order, f32_unshifted=st == "f32u", check_u_max=True)
        lat.init()
        lat.set_force((args.g, 0.0, 0.0))
        lat.step(n // 2)
        k_half = lat.permeability(args.g)
        lat.step(n - n // 2)
        k = lat.permeability(args.g)
        _, u, sums = lat.macroscopic()
        if u64 is None:
            u64, k64, m64 = u, k, sums[0]
            out["f64"] = {"permeability": k, "permeability_at_half_steps": k_half,
                          "rel_change_over_second_half": abs(k - k_half) / abs(k), "u_max": sums[5]}
            log(f"[bench] error run f64: k {k:.6e} (half-way {k_half:.6e})")
        else:
            du = torch.linalg.vector_norm(u - u64).item() / torch.linalg.vector_norm(u64).item()
            dk = abs(k - k64) / abs(k64)
            out[st] = {"permeability": k, "rel_permeability_err_vs_f64": dk, "rel_l2_velocity_vs_f64": du,
                       "mass_drift": (sums[0] - m64) / m64, "u_max": sums[5]}
            log(f"[bench] error run {st}: |dk|/k {dk:.2e}, |du|/|u| {du:.2e}")
            del u
        del lat
        torch.cuda.empty_cache()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(solid, args, seconds, max_steps=200):
    """The oracle as it stands, dense FP64 steps of the same geometry, for about
    `seconds` of CPU time: (MFLUPS, steps, seconds used, threads, fluid nodes)."""
    import oracle as O
    from oracle import tiles_ref
    sp = tiles_ref.pad(solid, 7)
    f = O.init(sp)
    nf = int((sp == 0).sum())
    O.step(f[:, :4, :4, :4], sp[:4, :4, :4], args.tau)  # load + build
    steps, t_used = 0, 0.0
    while (t_used < seconds or steps == 0) and steps < max_steps:
        t0 = time.perf_counter()
        f = O.step(f, sp, args.tau, force=[args.g, 0.0, 0.0], periodic=7)
        t_used += time.perf_counter() - t0
        steps += 1
    return nf * steps / t_used / 1e6, steps, t_used, O.num_threads(), nf


def cpu_baseline(solid, args):
    """The oracle as it stands, on the same geometry, for a bounded number of
    steps (about --cpu-seconds of CPU work) on all host threads, then on one
    thread (a child process with OMP_NUM_THREADS=1, about --cpu-seconds-one)."""
    import subprocess
    mf, steps, t_used, threads, nf = _oracle_sample(solid, args, args.cpu_seconds)
    out = dict(value=mf, unit="MFLUPS", cores=threads, kind="oracle",
               sample=f"{steps} dense FP64 steps of the same {args.n}^3 sphere pack ({nf} fluid nodes), "
                      f"{t_used:.1f} s", cpu_model=_cpu_model(), host_cpus=os.cpu_count())
    if args.cpu_seconds_one > 0:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-one-core-leg", "--n", str(args.n),
               "--porosity", str(args.porosity), "--seed", str(args.seed), "--tau", str(args.tau),
               "--g", str(args.g), "--cpu-seconds", str(args.cpu_seconds_one)]
        r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
            out["one_core"] = one
        else:
            out["one_core"] = {"error": r.stderr.strip()[-300:]}
    return out


def one_core_leg(args):
    """Child process of cpu_baseline: the oracle on one thread."""
    solid = build_case(args)
    mf, steps, t_used, threads, nf = _oracle_sample(solid, args, args.cpu_seconds)
    print(json.dumps(dict(value=mf, unit="MFLUPS", cores=threads, kind="oracle",
                          sample=f"{steps} dense FP64 steps of the same {args.n}^3 sphere pack ({nf} fluid nodes), "
                                 f"{t_used:.1f} s on one thread")), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="box edge (nodes)")
    ap.add_argument("--porosity", type=float, default=0.4)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--tau", type=float, default=0.7)
    ap.add_argument("--g", type=float, default=1e-6)
    ap.add_argument("--tpw", type=int, default=0, help="tiles per workgroup (0 = library default)")
    ap.add_argument("--order", type=int, default=0, help="device tile order (0 = library default)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-seconds-one", type=float, default=10.0,
                    help="seconds of the one-thread oracle sample (0 = skip it)")
    ap.add_argument("--cpu-one-core-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--error-steps", type=int, default=10000,
                    help="steps of the fixed run the storage variants' errors are stated on (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceiling", dest="ceiling", action="store_false",
                    help="skip the streaming-probe sweep (the measured bandwidth ceiling)")
    ap.add_argument("--variants", default="f32,f16s,f32u",
                    help="extra storage variants ('' for none); f32u = FP32 without the shift (ablation)")
    ap.add_argument("--kernel", default="step", choices=["step", "rw", "prop"],
                    help="time the fused step, or the paper's read/write-only (rw) or propagation-only (prop) kernel")
    ap.add_argument("--adj-steps", type=int, default=2000, help="adjoint horizon T (0 = skip the adjoint)")
    ap.add_argument("--adj-k", type=int, default=100, help="adjoint checkpoint interval K")
    ap.add_argument("--pack1024", action="store_true",
                    help="also run the 1024x512x512 FP32 forward + adjoint workload (about 2 minutes)")
    ap.add_argument("--vessel", action="store_true",
                    help="also time the step on the 512^3 vessel network (about 5% fluid)")
    ap.add_argument("--sweep192", action="store_true",
                    help="also time the step on 192^3 random sphere arrays at porosities 0.9..0.1")
    ap.add_argument("--sweep-cavity", action="store_true",
                    help="also time every kernel on dense b^3 boxes (the paper's cavity3D study, Table 3)")
    ap.add_argument("--layouts", action="store_true",
                    help="also time the paper's intra-tile layout study (propagation-only kernel, Table 5)")
    ap.add_argument("--sweep-channels", action="store_true",
                    help="also time the propagation-only kernel on rectangular channels (the paper's Eqs. 17-19 study)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration)")
    args = ap.parse_args()
    if args.cpu_one_core_leg:
        one_core_leg(args)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calib:
        # a plain device copy of known size: the counter calibration, and the
        # practical read+write bandwidth of the part
        n = args.copy_calib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(5):
            b.copy_(a)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / 5
        print(json.dumps({"copy_calib_bytes": n * 8, "launches": 6, "ms_per_copy": ms,
                          "read_plus_write_GBs": 2 * n * 8 / (ms / 1e3) / 1e9}), flush=True)
        return
    solid = build_case(args)
    if args.kernel != "step":
        print(json.dumps(time_calib(solid, args, torch)), flush=True)
        return

    # the streaming ceiling over one FP64 lattice's bytes (it also brings the
    # GPU to its working clocks before the timed step)
    ceiling = probe_ceiling(fp64_state_bytes(solid, args), torch) if args.ceiling else None
    r = time_storage(solid, "f64", args, torch)
    lat = r["lat"]
    nf = lat.n_fluid
    ms_per_step = r["gpu_ms"] / args.steps
    mflups = nf * args.steps / (r["gpu_ms"] / 1e3) / 1e6
    launch_s = ms_per_step / 1e3
    alg_bytes = BYTES_PER_UPDATE["f64"] * nf
    achieved = alg_bytes / launch_s / 1e9
    traffic = counter_traffic("step_f64_spheres256")
    log(f"[bench] f64: {mflups:.1f} MFLUPS, {ms_per_step * 1e3:.1f} us/step, {achieved:.0f} GB/s algorithmic")

    result = {
        "metric": METRIC,
        "value": round(mflups, 2),
        "unit": "MFLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"random overlapping sphere pack {args.n}^3 periodic, porosity {args.porosity}, "
                        f"radius U[4,12), seed {args.seed}; D3Q19 LBGK quasi-compressible, tau {args.tau}, "
                        f"g_x {args.g}, 4^3 tiles, all-solid tiles skipped",
            "box": [args.n, args.n, args.n],
            "tiles": lat.n_tiles,
            "fluid_nodes": nf,
            "eta_t": round(lat.tiling.eta_t, 6),
            "porosity": round(float((solid == 0).mean()), 6),
            "storage": "f64",
            "workgroups": lat.info()["grid_blocks"],
            "tiles_per_workgroup": -(-lat.n_tiles // lat.info()["grid_blocks"]),
            "tile_order": {0: "morton", 1: "discovery", 2: "slabs4", 3: "slabs8", 4: "morton", 5: "hilbert"}[args.order],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic / launch_s / 1e9, 1),
            "kernel": "k_step<f64, quasi-compressible>",
            "bytes_per_fluid_update": BYTES_PER_UPDATE["f64"],
        },
        "launch_ms": {"min": round(float(r["per"].min()), 4), "mean": round(float(r["per"].mean()), 4),
                      "max": round(float(r["per"].max()), 4)},
        "wall_ms_per_step": round(r["wall"] * 1e3 / args.steps, 6),
        "permeability": r["k"],
        "steps_total": r["steps_done"],
        "mass": r["sums"][0],
        "u_max": r["sums"][5],
    }
    if traffic is not None:
        result["roofline"]["traffic_bytes_per_fluid_update"] = round(traffic / nf, 1)
    if ceiling is not None:
        # the best plain copy over the same number of bytes: the practical
        # ceiling for equal read and write traffic
        result["roofline"]["ceiling_GBs"] = ceiling["best"]["copy"]["GBs"]
        result["roofline"]["frac_of_ceiling"] = round(achieved / ceiling["best"]["copy"]["GBs"], 4)
        result["bandwidth_probe"] = ceiling
    # the paper's measurement kernels on the same tiles: what this layout
    # sustains without any gather (read/write only) and the gather alone
    result["paper_kernels"] = {}
    for kname in ("rw", "prop"):
        c = time_calib(solid, args, torch, kernel=kname, launches=min(args.steps, 500), lat=lat)
        result["paper_kernels"]["read_write_only" if kname == "rw" else "propagation_only"] = {
            "MFLUPS": round(c["MFLUPS"], 1), "ms_per_launch": round(c["ms_per_launch"], 6),
            "hbm_frac_algorithmic": round(c["frac"], 4)}

    variants = {}
    for st in [v for v in args.variants.split(",") if v]:
        rv = time_storage(solid, st, args, torch)
        ms = rv["gpu_ms"] / args.steps
        mf = nf * args.steps / (rv["gpu_ms"] / 1e3) / 1e6
        tr = counter_traffic(f"step_{st}_spheres256")
        variants[st] = {"MFLUPS": round(mf, 2), "ms_per_step": round(ms, 6),
                        "launch_ms_mean": round(float(rv["per"].mean()), 4),
                        "traffic_GBs": None if tr is None else round(tr / (ms / 1e3) / 1e9, 1),
                        "gain_over_f64": round(mf / mflups, 3),
                        "hbm_frac": round(BYTES_PER_UPDATE[st] * nf / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        "bytes_per_fluid_update": BYTES_PER_UPDATE[st]}
        log(f"[bench] {st}: {mf:.1f} MFLUPS (x{mf / mflups:.2f})")
        del rv
        if st in BYTES_PER_UPDATE and st != "f32u":
            # what the same layout sustains with no collision (propagation
            # only) and with no gather either (read/write only)
            for kname in ("rw", "prop"):
                c = time_calib(solid, args, torch, kernel=kname, launches=min(args.steps, 500), storage=st)
                variants[st]["read_write_only_ms" if kname == "rw" else "propagation_only_ms"] = \
                    round(c["ms_per_launch"], 6)
    if variants and args.error_steps > 0:
        # the stated error of each storage type: a fixed run from rest,
        # independent of --steps
        err = error_run(solid, args, torch, list(variants))
        result["error_run"] = err
        for st in variants:
            variants[st].update({k: err[st][k] for k in ("rel_permeability_err_vs_f64", "rel_l2_velocity_vs_f64",
                                                         "mass_drift")})
            variants[st]["error_steps"] = err["steps"]
    if variants:
        result["variants"] = variants
    # the paper's LBMRT kernels: multiple relaxation times, same tiles and bytes
    mrt = {}
    for st in ("f64", "f32"):
        a2 = argparse.Namespace(**vars(args))
        a2.steps = min(args.steps, 1000)
        rm = time_storage(solid, st, a2, torch, model="mrt-qc")
        ms = rm["gpu_ms"] / a2.steps
        mf = nf * a2.steps / (rm["gpu_ms"] / 1e3) / 1e6
        mrt[st] = {"MFLUPS": round(mf, 2), "ms_per_step": round(ms, 6),
                   "hbm_frac": round(BYTES_PER_UPDATE[st] * nf / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                   "permeability": rm["k"]}
        log(f"[bench] mrt {st}: {mf:.1f} MFLUPS")
        del rm
    result["mrt_quasi_compressible"] = mrt
    del r, lat
    torch.cuda.empty_cache()
    result["small_grid"] = time_small_grid(args, torch)
    if args.adj_steps > 0:
        result["adjoint"] = time_adjoint(args, torch)
        torch.cuda.empty_cache()
    if args.pack1024:
        result["pack1024"] = time_pack1024(args, torch)
        torch.cuda.empty_cache()
    if args.vessel:
        result["vessel512"] = time_vessel(args, torch)
        torch.cuda.empty_cache()
    if args.sweep192:
        result["sphere_arrays_192"] = sweep_sphere_arrays(args, torch)
        torch.cuda.empty_cache()
    if args.sweep_cavity:
        result["cavity"] = sweep_cavity(args, torch)
        torch.cuda.empty_cache()
    if args.layouts:
        result["layouts"] = sweep_layouts(args, torch)
        torch.cuda.empty_cache()
    if args.sweep_channels:
        result["channels_propagation"] = sweep_channels(args, torch)
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(solid, args)
        log(f"[bench] cpu baseline {result['cpu_baseline']['value']:.2f} MFLUPS on {result['cpu_baseline']['cores']} threads")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
