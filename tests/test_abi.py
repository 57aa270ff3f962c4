"""The C ABI: the library loads, exports every declared entry point, and
rejects invalid arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1611_02445_amd import _abi
from paper_1611_02445_amd.lattice import Tiling

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_binding_list():
    assert declared_functions() == sorted(_abi.EXPORTS)


def test_every_export_has_a_ctypes_signature():
    L = _abi.lib()
    for name in _abi.EXPORTS:
        fn = getattr(L, name)
        assert fn.argtypes is not None, name


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_abi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert _abi.lib().lbm_version().decode().startswith("tiledlbm")


def _params(**kw):
    p = dict(tau=0.8, rho0=1.0, storage=0, model=0, f16_log2_scale=20, tiles_per_wg=0, f16_rounding=0)
    p.update(kw)
    return _abi.Params(**p)


@pytest.mark.parametrize("bad", [dict(tau=0.5), dict(tau=0.3), dict(tau=float("nan")), dict(rho0=0.0),
                                 dict(storage=3), dict(model=4), dict(f16_log2_scale=31), dict(tiles_per_wg=3),
                                 dict(f16_rounding=2), dict(tile_order=6), dict(wide_offsets=2),
                                 dict(f32_unshifted=2), dict(f32_unshifted=1, storage=0),
                                 dict(check_u_max=2), dict(check_u_max=-1)])
def test_parameter_validation(bad):
    t = Tiling(np.zeros((8, 8, 8), np.uint8), 7)
    sz = _abi.Sizes()
    rc = _abi.lib().lbm_required_bytes(t._ptr, ctypes.byref(_params(**bad)), ctypes.byref(sz))
    assert rc == -1
    assert _abi.lib().lbm_last_error()
    ctx = ctypes.c_void_p()
    rc = _abi.lib().lbm_create(t._ptr, ctypes.byref(_params(**bad)), None, None, None, None, None, ctypes.byref(ctx))
    assert rc == -1 and not ctx.value


def test_required_bytes():
    t = Tiling(np.zeros((8, 12, 16), np.uint8), 7)
    assert t.n_tiles == 2 * 3 * 4
    for storage, nd, na in ((0, 8, 8), (1, 4, 4), (2, 2, 4)):
        sz = _abi.Sizes()
        _abi.call("lbm_required_bytes", t._ptr, ctypes.byref(_params(storage=storage)), ctypes.byref(sz))
        assert sz.state_bytes == 24 * 19 * 64 * nd
        assert sz.adjoint_bytes == (sz.state_bytes if storage != 2 else 0)
        assert sz.force_bytes == 24 * 3 * 64 * na
        assert sz.grad_force_bytes == 24 * 3 * 64 * 8
        assert sz.dense_nodes == 8 * 12 * 16
        assert sz.table_bytes >= 24 * (16 + 20 * (8 + 4 + 8) + 16)


def test_null_arguments():
    assert _abi.lib().lbm_build_tiles(None, 4, 4, 4, 0, None) == -1
    assert _abi.lib().lbm_step(None, 1) == -1
    assert _abi.lib().lbm_macroscopic(None, None, None, None) == -1


def test_boundary_buffer_size():
    t = Tiling(np.zeros((8, 12, 16), np.uint8), 7)
    sz = _abi.Sizes()
    _abi.call("lbm_required_bytes", t._ptr, ctypes.byref(_params()), ctypes.byref(sz))
    assert sz.bc_bytes == 24 * 72


def test_create_rejects_inconsistent_tiles():
    """Table checks run before any device memory is touched: the dummy
    buffer addresses below are never dereferenced."""
    dummy = [ctypes.c_void_p(4096 * (k + 1)) for k in range(4)]
    for field, value in (("n_fluid", 1), ("nbr", 99)):
        t = Tiling(np.zeros((8, 8, 8), np.uint8), 7)
        if field == "n_fluid":
            t._ptr.contents.n_fluid += value
        else:
            t._ptr.contents.nbr[0] = value
        ctx = ctypes.c_void_p()
        rc = _abi.lib().lbm_create(t._ptr, ctypes.byref(_params()), *dummy, None, ctypes.byref(ctx))
        assert rc == -1 and not ctx.value
        assert field.encode() in _abi.lib().lbm_last_error() or b"neighbour" in _abi.lib().lbm_last_error()


def test_compressibility_limit_is_the_papers():
    """The u_max check compares against 0.05 (Section 2.2), exported as
    LBM_U_MAX, and is off unless asked for."""
    text = open(HEADER).read()
    m = re.search(r"#define\s+LBM_U_MAX\s+([0-9.eE+-]+)", text)
    assert m and float(m.group(1)) == 0.05
    assert _abi.Params().check_u_max == 0
    t = Tiling(np.zeros((8, 8, 8), np.uint8), 7)
    sz = _abi.Sizes()
    assert _abi.lib().lbm_required_bytes(t._ptr, ctypes.byref(_params(check_u_max=1)), ctypes.byref(sz)) == 0


@pytest.mark.parametrize("kind,nbytes,blocks,threads", [(0, 1024, 64, 256), (4, 1024, 64, 256), (3, 1000, 64, 256),
                                                        (3, 0, 64, 256), (3, 1024, 0, 256), (3, 1024, 1 << 21, 256),
                                                        (3, 1024, 64, 100), (3, 1024, 64, 2048)])
def test_stream_probe_validation(kind, nbytes, blocks, threads):
    """Arguments are checked before anything is launched: the addresses below
    are never dereferenced."""
    src, dst = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)
    assert _abi.lib().lbm_stream_probe(None, kind, src, dst, nbytes, blocks, threads) == -1
    assert _abi.lib().lbm_last_error().startswith(b"lbm_stream_probe")


def test_stream_probe_rejects_overlap_and_misalignment():
    base = 1 << 20
    L = _abi.lib()
    assert L.lbm_stream_probe(None, 3, ctypes.c_void_p(base), ctypes.c_void_p(base + 512), 1024, 8, 64) == -1
    assert b"overlap" in L.lbm_last_error()
    assert L.lbm_stream_probe(None, 3, ctypes.c_void_p(base + 8), ctypes.c_void_p(1 << 30), 1024, 8, 64) == -1
    assert b"aligned" in L.lbm_last_error()
    assert L.lbm_stream_probe(None, 1, None, ctypes.c_void_p(1 << 30), 1024, 8, 64) == -1


def test_field_to_dense_validation():
    L = _abi.lib()
    assert L.lbm_field_to_dense(None, None, 0, None) == -1


def test_field_and_lattice_sizes_follow_the_fluid_slots():
    """Partly solid tiles: a lattice holds 19 k values per tile and a per-node
    field 3 k entries, each padded (128-byte lines; 16 entries)."""
    rng = np.random.default_rng(81)
    solid = (rng.random((12, 16, 20)) < 0.6).astype(np.uint8)
    t = Tiling(solid, 7)
    k = np.array([bin(int(m)).count("1") for m in t.arrays()["fluid_mask"]])
    for storage, nd, na in ((0, 8, 8), (1, 4, 4), (2, 2, 4)):
        sz = _abi.Sizes()
        _abi.call("lbm_required_bytes", t._ptr, ctypes.byref(_params(storage=storage)), ctypes.byref(sz))
        fe = int(((3 * k + 15) // 16 * 16).sum())
        assert sz.force_bytes == fe * na and sz.grad_force_bytes == fe * 8
        if storage != 2:
            L = 128 // nd
            assert sz.state_bytes == int(((19 * k + L - 1) // L * L).sum()) * nd
        else:  # FP16 keeps whole 64-slot blocks per kept tile
            assert sz.state_bytes == t.n_tiles * 19 * 64 * 2
