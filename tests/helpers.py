"""Shared helpers of the GPU parity tests: run the same seeded case through the
HIP library and through the oracle on the padded box."""
import sys

import numpy as np

import oracle as O
from oracle import tiles_ref as T


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def padded(solid, periodic):
    return T.pad(solid, periodic)


def perturbed_state(solid_p, seed, amp=0.01, rho0=1.0):
    """feq(rho0, 0) times (1 + amp U(-1,1)) at fluid nodes (oracle feq)."""
    rng = np.random.default_rng(seed)
    f = O.init(solid_p, rho0=rho0)
    f *= 1.0 + amp * (2.0 * rng.random(f.shape) - 1.0)
    f[:, solid_p == 1] = 0.0
    return f


def rel_err_f(gpu, ora, solid_p):
    fl = solid_p == 0
    g = gpu[:, fl]
    o = ora[:, fl]
    return float(np.max(np.abs(g - o) / np.abs(o))) if o.size else 0.0


def new_lattice(solid, tau, periodic, **kw):
    from paper_1611_02445_amd.lattice import Lattice
    return Lattice(solid, tau, periodic=periodic, **kw)


def elementwise_err(got, ref, mask, floor):
    """Largest |got - ref| / max(|ref|, floor * max|ref|) over the entries of
    the masked nodes (mask over the last three axes): a relative bound on
    every entry, with an absolute floor for entries near zero."""
    g = got[..., mask]
    r = ref[..., mask]
    if r.size == 0:
        return 0.0
    den = np.maximum(np.abs(r), floor * np.abs(r).max())
    return float(np.max(np.abs(g - r) / den))
