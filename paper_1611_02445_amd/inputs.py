"""Seeded synthetic inputs: solid/fluid bitmaps and random perturbation fields.

This module holds no lattice-Boltzmann arithmetic.  It produces geometries
shaped like the paper's workloads (random arrangements of spheres, Section 4.6;
channels, Section 3.3; a branching vessel network standing in for the medical
geometries of Sections 4.7-4.8) and plain random fields.  Every array is a
``uint8`` bitmap indexed ``[z, y, x]`` with 1 = solid.
"""
import math

import numpy as np


def fluid_box(nx, ny, nz):
    return np.zeros((nz, ny, nx), dtype=np.uint8)


def square_channel(n=32, length=None):
    """Square duct along x: solid where y or z is on the box boundary."""
    nx = n if length is None else length
    s = np.zeros((n, n, nx), dtype=np.uint8)
    s[0, :, :] = 1
    s[-1, :, :] = 1
    s[:, 0, :] = 1
    s[:, -1, :] = 1
    return s


def plane_channel(nx, H, nz):
    """Channel between two walls normal to y: H fluid rows, one solid row on
    each side (ny = H + 2)."""
    s = np.zeros((nz, H + 2, nx), dtype=np.uint8)
    s[:, 0, :] = 1
    s[:, -1, :] = 1
    return s


def channel_cross_section(side, offset_y, offset_z, length=4, box=None, round_=False):
    """A channel along x with a square (or circular) side x side cross-section
    whose lower corner sits at (offset_y, offset_z) in a box of edge ``box``."""
    box = box or (side + 8)
    s = np.ones((box, box, length), dtype=np.uint8)
    if round_:
        r = side / 2.0
        cy, cz = offset_y + r - 0.5, offset_z + r - 0.5
        yy, zz = np.meshgrid(np.arange(box), np.arange(box), indexing="xy")
        inside = (yy - cy) ** 2 + (zz - cz) ** 2 <= r * r
        s[inside, :] = 0
    else:
        s[offset_z:offset_z + side, offset_y:offset_y + side, :] = 0
    return s


def random_bitmap(shape, solid_fraction, seed):
    rng = np.random.default_rng(seed)
    return (rng.random(shape) < solid_fraction).astype(np.uint8)


def sphere_pack(shape, porosity, rmin, rmax, seed, periodic=True, max_spheres=10_000_000):
    """Randomly placed, freely overlapping solid spheres (a Boolean model).

    Spheres with centres uniform in the box and radii uniform in [rmin, rmax)
    are added one at a time until the fluid fraction drops to ``porosity`` or
    below.  A node is solid when its (minimum-image, if periodic) distance to a
    centre is at most the radius.  Returns (bitmap, number of spheres)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    solid = np.zeros(shape, dtype=np.uint8)
    total = solid.size
    n_solid = 0
    count = 0
    dims = np.array([nx, ny, nz], dtype=np.float64)
    while 1.0 - n_solid / total > porosity and count < max_spheres:
        c = rng.uniform(0.0, 1.0, 3) * dims
        r = rng.uniform(rmin, rmax)
        count += 1
        ranges = []
        for a, n in enumerate((nx, ny, nz)):
            lo = int(math.floor(c[a] - r))
            hi = int(math.ceil(c[a] + r))
            idx = np.arange(lo, hi + 1)
            if periodic:
                idx_w = idx % n
                keep = np.ones(idx.size, dtype=bool)
            else:
                keep = (idx >= 0) & (idx < n)
                idx_w = idx
            ranges.append((idx[keep], idx_w[keep]))
        (xs, xw), (ys, yw), (zs, zw) = ranges
        if xs.size == 0 or ys.size == 0 or zs.size == 0:
            continue
        d2 = ((zs[:, None, None] - c[2]) ** 2 + (ys[None, :, None] - c[1]) ** 2
              + (xs[None, None, :] - c[0]) ** 2)
        inside = d2 <= r * r
        if periodic and (2 * r + 2 >= min(nx, ny, nz)):
            raise ValueError("sphere too large for the periodic box")
        ix = np.ix_(zw, yw, xw)
        sub = solid[ix]
        new = inside & (sub == 0)
        n_solid += int(new.sum())
        sub[inside] = 1
        solid[ix] = sub
    return solid, count


def _capsule_stamp(fluid, p0, p1, r):
    """Mark as fluid every node within distance r of the segment p0-p1
    (coordinates x, y, z; nodes outside the box are ignored)."""
    nz, ny, nx = fluid.shape
    lo = np.floor(np.minimum(p0, p1) - r).astype(int)
    hi = np.ceil(np.maximum(p0, p1) + r).astype(int)
    lo = np.maximum(lo, 0)
    hi = np.minimum(hi, np.array([nx - 1, ny - 1, nz - 1]))
    if np.any(hi < lo):
        return
    xs = np.arange(lo[0], hi[0] + 1)
    ys = np.arange(lo[1], hi[1] + 1)
    zs = np.arange(lo[2], hi[2] + 1)
    d = p1 - p0
    L2 = float(d @ d)
    X = xs[None, None, :] - p0[0]
    Y = ys[None, :, None] - p0[1]
    Z = zs[:, None, None] - p0[2]
    if L2 > 0:
        t = np.clip((X * d[0] + Y * d[1] + Z * d[2]) / L2, 0.0, 1.0)
    else:
        t = np.zeros_like(X + Y + Z, dtype=np.float64)
    dist2 = (X - t * d[0]) ** 2 + (Y - t * d[1]) ** 2 + (Z - t * d[2]) ** 2
    sub = fluid[zs[0]:zs[-1] + 1, ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1]
    sub |= dist2 <= r * r


def vessel_tree(n=512, root_radius=24.0, ratio=0.8, levels=8, fluid_target=0.05, seed=3, length0=None):
    """A seeded binary branching network of tubes, mirrored into a loop.

    Half tree (x < n/2): a root tube of radius R0 starts at (0, n/2, n/2)
    heading +x; a segment of level k has radius R0 ratio^k and length
    L0 ratio^k and ends in two children turned by +-theta (theta uniform in
    20..45 degrees) in a random plane through the parent axis.  A segment that
    would leave the half box is reflected back in (its end point is mirrored
    at the wall it crosses and its direction flipped there).  The leaves are
    extended along +x to the mid-plane x = n/2 - 1/2 and the half is mirrored
    (x -> n-1-x), so the network closes into loops through the periodic x
    boundary.  L0 is bisected so that the fluid fraction is close to
    ``fluid_target`` (unless ``length0`` is given).  Returns the bitmap
    (1 = solid) and the L0 used."""
    half = n // 2

    def build(L0):
        rng = np.random.default_rng(seed)
        fluid = np.zeros((n, n, half), dtype=bool)
        stack = [(np.array([0.0, n / 2.0, n / 2.0]), np.array([1.0, 0.0, 0.0]), 0)]
        while stack:
            p, d, k = stack.pop()
            r = root_radius * ratio ** k
            L = L0 * ratio ** k
            q = p + L * d
            d = d.copy()
            lo = np.array([0.0, r + 1.0, r + 1.0])
            hi = np.array([half - 0.5, n - r - 2.0, n - r - 2.0])
            for a in range(3):
                if q[a] > hi[a]:
                    q[a] = max(lo[a], 2 * hi[a] - q[a])
                    d[a] = -abs(d[a])
                elif q[a] < lo[a]:
                    q[a] = min(hi[a], 2 * lo[a] - q[a])
                    d[a] = abs(d[a])
            _capsule_stamp(fluid, p, q, r)
            if k + 1 < levels:
                v = rng.normal(size=3)
                v -= (v @ d) * d
                v /= np.linalg.norm(v)
                for sgn in (1.0, -1.0):
                    th = math.radians(rng.uniform(20.0, 45.0))
                    nd = math.cos(th) * d + sgn * math.sin(th) * v
                    nd /= np.linalg.norm(nd)
                    stack.append((q, nd, k + 1))
            else:
                _capsule_stamp(fluid, q, np.array([half - 0.5, q[1], q[2]]), r)
        return np.concatenate([fluid, fluid[:, :, ::-1]], axis=2)

    if length0 is not None:
        geo = build(length0)
        return (~geo).astype(np.uint8), float(length0)
    lo_L, hi_L = 0.05 * n, 2.0 * n
    geo, L0 = None, None
    for _ in range(14):
        mid = 0.5 * (lo_L + hi_L)
        g = build(mid)
        frac = g.mean()
        geo, L0 = g, mid
        if abs(frac - fluid_target) <= 0.002 * fluid_target * 10:
            break
        if frac < fluid_target:
            lo_L = mid
        else:
            hi_L = mid
    return (~geo).astype(np.uint8), float(L0)


def perturbation(shape, seed, amplitude=1.0):
    """Uniform random factors in [-amplitude, amplitude) of the given shape."""
    rng = np.random.default_rng(seed)
    return amplitude * (2.0 * rng.random(shape) - 1.0)


def normal_field(shape, mean, std, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(mean, std, size=shape)
