"""Python face of the C ABI: a host tiling and a device lattice.

PyTorch only provides device memory and the stream; every computation runs in
the HIP library (see include/lbm.h for the meaning of each call).
"""
import ctypes

import numpy as np

from . import _abi
from ._abi import call


def _vp(x):
    """void* of a torch tensor, an int address or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    return ctypes.c_void_p(x.data_ptr())


class Tiling:
    """Result of ``lbm_build_tiles`` (Alg. 1), held in library-owned host memory."""

    def __init__(self, solid, periodic=0):
        s = np.ascontiguousarray(solid, dtype=np.uint8)
        if s.ndim != 3:
            raise ValueError("solid must be a [nz, ny, nx] array")
        nz, ny, nx = s.shape
        ptr = ctypes.POINTER(_abi.Tiles)()
        call("lbm_build_tiles", s.ctypes.data_as(ctypes.c_void_p), nx, ny, nz, int(periodic), ctypes.byref(ptr))
        self._ptr = ptr
        self._free = _abi.lib().lbm_tiles_free
        self.shape_in = s.shape

    def __del__(self):
        # at interpreter shutdown module globals may already be gone: the
        # library handle is kept on the object
        p = getattr(self, "_ptr", None)
        free = getattr(self, "_free", None)
        if p and free is not None:
            free(p)
            self._ptr = None

    @property
    def t(self):
        return self._ptr.contents

    def __getattr__(self, name):
        if name in ("nx", "ny", "nz", "tx", "ty", "tz", "periodic", "n_tiles", "n_fluid", "eta_t"):
            return getattr(self._ptr.contents, name)
        raise AttributeError(name)

    @property
    def dense_shape(self):
        return (self.nz, self.ny, self.nx)

    def device_order(self, order=0):
        """``lbm_tile_order``: the discovery-order tile numbers in the order a
        context created with ``tile_order=order`` stores and processes them."""
        perm = np.empty(self.n_tiles, dtype=np.int32)
        call("lbm_tile_order", self._ptr, int(order), perm.ctypes.data_as(ctypes.c_void_p))
        return perm

    def arrays(self):
        """Copies of the tables as numpy arrays."""
        t = self.t
        n = t.n_tiles

        def grab(p, count, dt):
            if count == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(p, shape=(count,)).astype(dt, copy=True)

        return dict(
            tile_map=grab(t.tile_map, t.tx * t.ty * t.tz, np.int32).reshape(t.tz, t.ty, t.tx),
            tile_xyz=grab(t.tile_xyz, 3 * n, np.int32).reshape(n, 3),
            nbr=grab(t.nbr, 27 * n, np.int32).reshape(n, 27),
            fluid_mask=grab(t.fluid_mask, n, np.uint64),
        )


class Lattice:
    """A tiled D3Q19 lattice on one GPU: two lattices (A/B), the device tables
    and the reduction scratch, all allocated as torch tensors."""

    def __init__(self, solid, tau, periodic=0, rho0=1.0, storage="f64", model="qc", f16_log2_scale=20,
                 tiles_per_wg=0, device="cuda", tiling=None, stream=None, f16_rounding="stochastic",
                 tile_order=0, wide_offsets=False, f32_unshifted=False, check_u_max=False):
        import torch

        self.torch = torch
        self.tiling = tiling if tiling is not None else Tiling(solid, periodic)
        self.device = torch.device(device)
        self.params = _abi.Params(tau=float(tau), rho0=float(rho0), storage=_abi.STORAGE[storage],
                                  model=_abi.MODEL[model], f16_log2_scale=int(f16_log2_scale),
                                  tiles_per_wg=int(tiles_per_wg),
                                  f16_rounding={"stochastic": 0, "nearest": 1}[f16_rounding],
                                  tile_order=int(tile_order), wide_offsets=int(bool(wide_offsets)),
                                  f32_unshifted=int(bool(f32_unshifted)),
                                  check_u_max=int(bool(check_u_max)))
        self.storage = storage
        self.tau = float(tau)
        self.rho0 = float(rho0)
        sz = _abi.Sizes()
        call("lbm_required_bytes", self.tiling._ptr, ctypes.byref(self.params), ctypes.byref(sz))
        self.sizes = sz

        def buf(n):
            return torch.empty(max(int(n), 1), dtype=torch.uint8, device=self.device)

        self.state_a = buf(sz.state_bytes)
        self.state_b = buf(sz.state_bytes)
        self.tables = buf(sz.table_bytes)
        self.scratch = buf(sz.scratch_bytes)
        self.force_buf = None
        self.bc_buf = None
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        call("lbm_create", self.tiling._ptr, ctypes.byref(self.params), _vp(self.state_a), _vp(self.state_b),
             _vp(self.tables), _vp(self.scratch), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        self.ctx = ctx
        self._destroy = _abi.lib().lbm_destroy

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        destroy = getattr(self, "_destroy", None)
        if ctx and destroy is not None:
            destroy(ctx)
            self.ctx = None

    # -- sizes ---------------------------------------------------------------
    @property
    def n_tiles(self):
        return self.tiling.n_tiles

    @property
    def n_fluid(self):
        return self.tiling.n_fluid

    @property
    def dense_shape(self):
        return self.tiling.dense_shape

    def new_state(self):
        """An extra lattice buffer (e.g. a checkpoint slot)."""
        return self.torch.empty(max(self.sizes.state_bytes, 1), dtype=self.torch.uint8, device=self.device)

    def new_adjoint(self):
        return self.torch.empty(max(self.sizes.adjoint_bytes, 1), dtype=self.torch.uint8, device=self.device)

    def new_grad(self):
        return self.torch.zeros(max(self.sizes.grad_force_bytes // 8, 1), dtype=self.torch.float64,
                                device=self.device)

    # -- forward -------------------------------------------------------------
    def init(self, rho0=None, u0=(0.0, 0.0, 0.0)):
        call("lbm_init", self.ctx, float(self.rho0 if rho0 is None else rho0), *map(float, u0))

    def set_force(self, g):
        """g: a 3-vector (uniform body acceleration) or a float64 tensor
        [3, nz, ny, nx] on the device (per node)."""
        torch = self.torch
        if isinstance(g, torch.Tensor):
            g = g.to(device=self.device, dtype=torch.float64).contiguous()
            if tuple(g.shape) != (3,) + self.dense_shape:
                raise ValueError(f"force field must have shape {(3,) + self.dense_shape}")
            if self.force_buf is None:
                self.force_buf = torch.empty(max(self.sizes.force_bytes, 1), dtype=torch.uint8, device=self.device)
            call("lbm_set_force", self.ctx, 0.0, 0.0, 0.0, _vp(g), _vp(self.force_buf))
            self._force_src = g
        else:
            gx, gy, gz = map(float, g)
            call("lbm_set_force", self.ctx, gx, gy, gz, None, None)

    def set_boundaries(self, types, u_in=(0.0, 0.0, 0.0), rho_out=1.0):
        """Open boundaries: types is a uint8 array over the padded box
        [nz, ny, nx] of node codes (0 none; 1..12: axis (code-1)//4, and
        (code-1)%4 = 0 velocity node rebuilding c_a = +1, 1 pressure node
        rebuilding c_a = -1, 2 velocity c_a = -1, 3 pressure c_a = +1; 1 and 2
        are the x inlet and outlet).  Velocity nodes get u_in, pressure nodes
        rho_out.  None removes them."""
        if types is None:
            call("lbm_set_boundaries", self.ctx, None, 0.0, 0.0, 0.0, 1.0, None)
            return
        t = np.ascontiguousarray(types, dtype=np.uint8)
        if t.shape != self.dense_shape:
            raise ValueError(f"boundary types must have shape {self.dense_shape}")
        if self.bc_buf is None:
            self.bc_buf = self.torch.empty(max(self.sizes.bc_bytes, 1), dtype=self.torch.uint8, device=self.device)
        call("lbm_set_boundaries", self.ctx, t.ctypes.data_as(ctypes.c_void_p), *map(float, u_in), float(rho_out),
             _vp(self.bc_buf))

    def step(self, n=1, graphed=False):
        """n steps; graphed=True replays a captured HIP graph of 32 steps
        (same results, less launch overhead on small grids)."""
        call("lbm_step_graphed" if graphed else "lbm_step", self.ctx, int(n))

    def step_buf(self, src, dst):
        call("lbm_step_buf", self.ctx, _vp(src), _vp(dst))

    def calib_step(self, kind, src, dst):
        call("lbm_calib_step", self.ctx, int(kind), _vp(src), _vp(dst))

    def current_state_ptr(self):
        p = ctypes.c_void_p()
        call("lbm_current_state", self.ctx, ctypes.byref(p))
        return p.value

    def current_state(self):
        """The tensor (A or B) holding the current lattice."""
        p = self.current_state_ptr()
        return self.state_a if p == self.state_a.data_ptr() else self.state_b

    # -- outputs -------------------------------------------------------------
    def macroscopic(self, state=None, fields=True):
        """(rho [nz,ny,nx], u [3,nz,ny,nx], sums[8]) as FP64; fields=False
        returns (None, None, sums)."""
        torch = self.torch
        rho = u = None
        if fields:
            rho = torch.empty(self.dense_shape, dtype=torch.float64, device=self.device)
            u = torch.empty((3,) + self.dense_shape, dtype=torch.float64, device=self.device)
        sums = (ctypes.c_double * 8)()
        call("lbm_macroscopic_buf", self.ctx, _vp(state), _vp(rho), _vp(u), sums)
        return rho, u, np.array(sums[:])

    def permeability(self, g_x):
        k = ctypes.c_double()
        call("lbm_permeability", self.ctx, float(g_x), ctypes.byref(k))
        return k.value

    def get_state(self, state=None):
        torch = self.torch
        out = torch.empty((19,) + self.dense_shape, dtype=torch.float64, device=self.device)
        call("lbm_get_state", self.ctx, _vp(state), _vp(out))
        return out

    def set_state(self, f_dense, state=None):
        torch = self.torch
        f = torch.as_tensor(f_dense).to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(f.shape) != (19,) + self.dense_shape:
            raise ValueError(f"state must have shape {(19,) + self.dense_shape}")
        call("lbm_set_state", self.ctx, _vp(f), _vp(state))
        self.stream.synchronize()

    def field_to_dense(self, field_buf, dtype=0):
        """A per-node field (force density, force gradient) as a dense FP64
        [3, nz, ny, nx] tensor."""
        torch = self.torch
        out = torch.empty((3,) + self.dense_shape, dtype=torch.float64, device=self.device)
        call("lbm_field_to_dense", self.ctx, _vp(field_buf), int(dtype), _vp(out))
        return out

    def tiles_to_dense(self, tile_buf, ncomp, dtype=0):
        torch = self.torch
        out = torch.empty((ncomp,) + self.dense_shape, dtype=torch.float64, device=self.device)
        call("lbm_tiles_to_dense", self.ctx, _vp(tile_buf), int(ncomp), int(dtype), _vp(out))
        return out

    # -- adjoint -------------------------------------------------------------
    def adjoint_seed(self, s_Tm1, eta_T, grad):
        call("lbm_adjoint_seed", self.ctx, _vp(s_Tm1), _vp(eta_T), _vp(grad))

    def adjoint_step(self, s_tm2, eta_t, eta_tm1, grad):
        call("lbm_adjoint_step", self.ctx, _vp(s_tm2), _vp(eta_t), _vp(eta_tm1), _vp(grad))

    def adjoint_final(self, eta_1, lambda_0):
        call("lbm_adjoint_final", self.ctx, _vp(eta_1), _vp(lambda_0))

    def adjoint_get(self, adj):
        """Dense FP64 [19, nz, ny, nx] copy of an adjoint lattice."""
        torch = self.torch
        out = torch.empty((19,) + self.dense_shape, dtype=torch.float64, device=self.device)
        call("lbm_adjoint_get", self.ctx, _vp(adj), _vp(out))
        return out

    def adjoint_set(self, dense, adj):
        torch = self.torch
        v = torch.as_tensor(dense).to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(v.shape) != (19,) + self.dense_shape:
            raise ValueError(f"adjoint lattice must have shape {(19,) + self.dense_shape}")
        call("lbm_adjoint_set", self.ctx, _vp(v), _vp(adj))
        self.stream.synchronize()

    def info(self):
        n_t, n_f, st, gb = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        call("lbm_info", self.ctx, ctypes.byref(n_t), ctypes.byref(n_f), ctypes.byref(st), ctypes.byref(gb))
        return dict(n_tiles=n_t.value, n_fluid=n_f.value, storage=st.value, grid_blocks=gb.value)
