"""CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

The arithmetic lives in ``lbm_oracle.c`` (a dense D3Q19 LBGK or
multiple-relaxation-time step with pull streaming and halfway bounce-back, Guo
forcing, macroscopic fields and a discrete adjoint) and in ``tiles_ref.py`` (the tiling of Alg. 1).  This module
builds the C file with gcc and wraps it with numpy arrays; the reductions
(mass, momentum, permeability) are numpy sums over the oracle's fields.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import tiles_ref  # noqa: F401  (re-export)

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

Q = 19
_lib = None


def build(force=False):
    """Compile the oracle with gcc: -O2, OpenMP, no FMA contraction, no fast-math."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_lattice.argtypes = [P, P, P]
        L.oracle_feq.argtypes = [i32, f64, P, P]
        L.oracle_guo.argtypes = [f64, P, P, P]
        L.oracle_collide_node.argtypes = [i32, P, P, f64, P]
        L.oracle_init.argtypes = [P, P, i32, i32, i32, i32, f64, f64, f64, f64]
        L.oracle_step.argtypes = [P, P, P, i32, i32, i32, i32, i32, f64, P, f64, f64, f64]
        L.oracle_run.argtypes = [P, P, P, i32, i32, i32, i32, i32, f64, P, f64, f64, f64, i32]
        L.oracle_step_nodes.argtypes = [P, P, i32, i32, i32, i32, i32, f64, P, f64, f64, f64, P, i64, P]
        L.oracle_macroscopic.argtypes = [P, P, i32, i32, i32, i32, P, f64, f64, f64, P, P]
        L.oracle_pull.argtypes = [P, P, P, i32, i32, i32, i32]
        L.oracle_pull_transpose.argtypes = [P, P, P, i32, i32, i32, i32]
        L.oracle_collide_jt_node.argtypes = [i32, P, P, f64, P, P, P]
        L.oracle_loss_ux.argtypes = [i32, P, P, i32, i32, i32, P, P, P]
        L.oracle_loss_ux.restype = f64
        L.oracle_adjoint.argtypes = [i32, P, P, i32, i32, i32, i32, f64, P, i32, P, P]
        L.oracle_adjoint.restype = f64
        L.oracle_mrt_matrix.argtypes = [P, P]
        L.oracle_mrt_rates.argtypes = [f64, P]
        L.oracle_set_mrt_ghost_rates.argtypes = [P]
        L.oracle_collide_mrt_rates.argtypes = [i32, P, P, P, P]
        L.oracle_zou_he.argtypes = [i32, i32, P, f64, P, P]
        L.oracle_run_bc.argtypes = [P, P, P, i32, i32, i32, i32, i32, f64, P, f64, f64, f64, i32, P, P, f64]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def num_threads():
    return int(lib().oracle_num_threads())


def lattice():
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q, dtype=np.float64)
    opp = np.zeros(Q, dtype=np.int32)
    lib().oracle_lattice(_p(c), _p(w), _p(opp))
    return c, w, opp


def feq(rho, u, model=0):
    out = np.zeros(Q)
    lib().oracle_feq(model, float(rho), _p(_f64(u)), _p(out))
    return out


def guo(tau, u, F):
    out = np.zeros(Q)
    lib().oracle_guo(float(tau), _p(_f64(u)), _p(_f64(F)), _p(out))
    return out


MODELS = {"qc": 0, "inc": 1, "mrt-qc": 2, "mrt-inc": 3}


def mrt_matrix():
    """(M, M^-1): the D3Q19 moment matrix (rows = moments) and its inverse."""
    M = np.zeros((Q, Q))
    Minv = np.zeros((Q, Q))
    lib().oracle_mrt_matrix(_p(M), _p(Minv))
    return M, Minv


def mrt_rates(tau):
    s = np.zeros(Q)
    lib().oracle_mrt_rates(float(tau), _p(s))
    return s


class mrt_ghost_rates:
    """Context manager: run the multiple-relaxation-time operator with the
    rates (s_e, s_eps, s_q, s_pi, s_m) instead of the table's, restoring the
    table on exit."""

    def __init__(self, s_e=1.19, s_eps=1.4, s_q=1.2, s_pi=1.4, s_m=1.98):
        self.r = np.array([s_e, s_eps, s_q, s_pi, s_m], dtype=np.float64)

    def __enter__(self):
        lib().oracle_set_mrt_ghost_rates(_p(self.r))
        return self

    def __exit__(self, *exc):
        lib().oracle_set_mrt_ghost_rates(None)
        return False


def collide_mrt_rates(fin, F, s, model=2):
    """The multiple-relaxation-time operator with caller-given rates s[19]."""
    out = np.zeros(Q)
    lib().oracle_collide_mrt_rates(model, _p(_f64(fin)), _p(_f64(F)), _p(_f64(s)), _p(out))
    return out


def zou_he(f, btype, u_in=(0.0, 0.0, 0.0), rho_out=1.0, F=(0.0, 0.0, 0.0), model=0):
    """The populations of one node after the open-boundary rebuild.  btype
    1..12: axis (btype-1)//4; (btype-1)%4 = 0 velocity node with unknowns
    c_a = +1, 1 pressure node c_a = -1, 2 velocity c_a = -1, 3 pressure
    c_a = +1 (1 and 2: the x inlet and outlet)."""
    out = _f64(f).copy()
    lib().oracle_zou_he(int(btype), int(model), _p(_f64(u_in)), float(rho_out), _p(_f64(F)), _p(out))
    return out


def run_bc(f, solid, tau, nsteps, btype, u_in=(0.0, 0.0, 0.0), rho_out=1.0, force=None, periodic=0, model=0):
    """nsteps steps with open boundaries: btype [nz,ny,nx] uint8 (0 none,
    else a code of zou_he: velocity nodes get u_in, pressure nodes rho_out)."""
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    fa = _f64(f).copy()
    scratch = np.zeros_like(fa)
    keep, fp, fx, fy, fz = _force_args(force)
    bt = _u8(btype)
    lib().oracle_run_bc(_p(fa), _p(scratch), _p(solid), nx, ny, nz, periodic, model, tau, fp, fx, fy, fz,
                        int(nsteps), _p(bt), _p(_f64(u_in)), float(rho_out))
    return fa


def collide_node(fin, F, tau, model=0):
    out = np.zeros(Q)
    lib().oracle_collide_node(model, _p(_f64(fin)), _p(_f64(F)), float(tau), _p(out))
    return out


def collide_jt_node(fin, F, tau, lam, model=0):
    eta = np.zeros(Q)
    gF = np.zeros(3)
    lib().oracle_collide_jt_node(int(model), _p(_f64(fin)), _p(_f64(F)), float(tau), _p(_f64(lam)), _p(eta),
                                 _p(gF))
    return eta, gF


def _force_args(force):
    """force: None, a 3-vector (uniform) or a [3,nz,ny,nx] field."""
    if force is None:
        return None, None, 0.0, 0.0, 0.0
    f = np.asarray(force, dtype=np.float64)
    if f.ndim == 1:
        return None, None, float(f[0]), float(f[1]), float(f[2])
    f = _f64(f)
    return f, _p(f), 0.0, 0.0, 0.0


def init(solid, rho0=1.0, u0=(0.0, 0.0, 0.0), model=0):
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    f = np.zeros((Q, nz, ny, nx))
    lib().oracle_init(_p(f), _p(solid), nx, ny, nz, model, rho0, *map(float, u0))
    return f


def step(f, solid, tau, force=None, periodic=0, model=0):
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    fa = _f64(f)
    fb = np.zeros_like(fa)
    keep, fp, fx, fy, fz = _force_args(force)
    lib().oracle_step(_p(fa), _p(fb), _p(solid), nx, ny, nz, periodic, model, tau, fp, fx, fy, fz)
    return fb


def run(f, solid, tau, nsteps, force=None, periodic=0, model=0):
    """nsteps steps; returns the new state (the input is not modified)."""
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    fa = _f64(f).copy()
    scratch = np.zeros_like(fa)
    keep, fp, fx, fy, fz = _force_args(force)
    lib().oracle_run(_p(fa), _p(scratch), _p(solid), nx, ny, nz, periodic, model, tau, fp, fx, fy, fz,
                     int(nsteps))
    return fa


def step_nodes(f, solid, tau, nodes, force=None, periodic=0, model=0):
    """One-step update of the listed flat node indices: returns [len(nodes), 19]."""
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    fa = _f64(f)
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros((nodes.size, Q))
    keep, fp, fx, fy, fz = _force_args(force)
    lib().oracle_step_nodes(_p(fa), _p(solid), nx, ny, nz, periodic, model, tau, fp, fx, fy, fz, _p(nodes),
                            nodes.size, _p(out))
    return out


def macroscopic(f, solid, force=None, model=0):
    """(rho [nz,ny,nx], u [3,nz,ny,nx]) from a stored post-collision state."""
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    fa = _f64(f)
    rho = np.zeros((nz, ny, nx))
    u = np.zeros((3, nz, ny, nx))
    keep, fp, fx, fy, fz = _force_args(force)
    lib().oracle_macroscopic(_p(fa), _p(solid), nx, ny, nz, model, fp, fx, fy, fz, _p(rho), _p(u))
    return rho, u


def sums(f, solid, force=None, model=0):
    """FP64 totals {mass, mom_x, mom_y, mom_z, n_fluid} (numpy pairwise sums)."""
    rho, u = macroscopic(f, solid, force, model)
    fl = _u8(solid) == 0
    r = rho[fl]
    return np.array([r.sum(), (r * u[0][fl]).sum(), (r * u[1][fl]).sum(), (r * u[2][fl]).sum(),
                     float(fl.sum())])


def permeability(f, solid, tau, g_x, rho0=1.0, force=None, model=0):
    """Darcy permeability k = nu * q / g_x with the superficial flux
    q = sum_fluid rho u_x / (rho0 * N_box); nu = (tau - 1/2)/3."""
    rho, u = macroscopic(f, solid, force, model)
    fl = _u8(solid) == 0
    nu = (tau - 0.5) / 3.0
    q = (rho[fl] * u[0][fl]).sum() / (rho0 * solid.size)
    return nu * q / g_x


def pull(s, solid, periodic=0):
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    s = _f64(s)
    g = np.zeros_like(s)
    lib().oracle_pull(_p(s), _p(g), _p(solid), nx, ny, nz, periodic)
    return g


def pull_transpose(mu, solid, periodic=0):
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    mu = _f64(mu)
    out = np.zeros_like(mu)
    lib().oracle_pull_transpose(_p(mu), _p(out), _p(solid), nx, ny, nz, periodic)
    return out


def loss_ux(s, solid, force_field=None, model=0):
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    s = _f64(s)
    ff = None if force_field is None else _f64(force_field)
    return lib().oracle_loss_ux(int(model), _p(s), _p(solid), nx, ny, nz, _p(ff), None, None)


def adjoint(s0, solid, tau, force_field, T, periodic=0, model=0):
    """Returns (L, dL/ds0 [19,...], dL/dF [3,...]) for L = mean u_x at step T."""
    solid = _u8(solid)
    nz, ny, nx = solid.shape
    s0 = _f64(s0)
    ff = _f64(force_field)
    gs = np.zeros_like(s0)
    gF = np.zeros_like(ff)
    L = lib().oracle_adjoint(int(model), _p(s0), _p(solid), nx, ny, nz, periodic, tau, _p(ff), int(T), _p(gs),
                             _p(gF))
    if not np.isfinite(L):
        raise MemoryError("oracle_adjoint: allocation failed")
    return L, gs, gF
