"""Independent numpy tiler -- TEST INFRASTRUCTURE ONLY (the oracle of the host
tiling step).  Only tests, the smoke check and the benchmark's CPU-baseline leg
may import it.

Follows the paper's tiling description (Section 3.1, Alg. 1):

* the box is covered from node (0,0,0) by a uniform grid of a^3 tiles (a = 4);
  a box edge that is not a multiple of a is extended with solid nodes;
* tiles holding at least one non-solid node are kept, numbered in the order the
  scan finds them (z outer, then y, then x innermost);
* a dense tile grid ("tileMap") holds each kept tile's number, or -1;
* the coordinates of each kept tile's corner are listed ("nonEmptyTiles").

Our reading of what the paper leaves open:

* the loop bounds of Alg. 1 are read as tile indices 0..ceil(N/a)-1 with node
  coordinate a*t + n;
* periodic axes are not padded (padding would change the period), so they must
  already be multiples of a;
* the per-tile node-type block is a 64-bit fluid mask, bit x + 4y + 16z;
* the 3x3x3 neighbourhood of a tile (the window the kernel copies from the
  tile map, Section 3.4) is listed per tile with k = (dx+1) + 3(dy+1) + 9(dz+1),
  wrapping on periodic axes, -1 for an all-solid or outside tile.
"""
import numpy as np

A = 4


def padded_shape(shape, periodic):
    """Padded (nz, ny, nx).  periodic bit0 = x, bit1 = y, bit2 = z."""
    nz, ny, nx = shape
    out = []
    for axis_bit, n in ((4, nz), (2, ny), (1, nx)):
        if periodic & axis_bit:
            if n % A:
                raise ValueError("periodic axis length must be a multiple of 4")
            out.append(n)
        else:
            out.append(-(-n // A) * A)
    return tuple(out)


def pad(solid, periodic):
    """Extend non-periodic axes with solid nodes up to a multiple of 4."""
    solid = np.asarray(solid, dtype=np.uint8)
    pz, py, px = padded_shape(solid.shape, periodic)
    out = np.ones((pz, py, px), dtype=np.uint8)
    out[: solid.shape[0], : solid.shape[1], : solid.shape[2]] = solid
    return out


def build_tiles(solid, periodic=0):
    """Returns a dict with padded dims, tile grid dims, tile_map [tz,ty,tx],
    tile_xyz [n,3] (corner node x,y,z), nbr [n,27], fluid_mask [n] (uint64),
    n_fluid and eta_t (Eq. 14)."""
    p = pad(solid, periodic)
    nz, ny, nx = p.shape
    tz, ty, tx = nz // A, ny // A, nx // A
    fluid = p == 0
    # blocks[tz, ty, tx, z, y, x]
    blocks = fluid.reshape(tz, A, ty, A, tx, A).transpose(0, 2, 4, 1, 3, 5)
    bits = (np.uint64(1) << np.arange(64, dtype=np.uint64)).reshape(A, A, A)
    masks = (blocks.astype(np.uint64) * bits).sum(axis=(3, 4, 5), dtype=np.uint64)
    keep = masks != 0
    # np.nonzero on a C-ordered (tz,ty,tx) grid lists z outer, then y, then x
    kz, ky, kx = np.nonzero(keep)
    n_tiles = kz.size
    tile_map = np.full((tz, ty, tx), -1, dtype=np.int32)
    tile_map[kz, ky, kx] = np.arange(n_tiles, dtype=np.int32)
    tile_xyz = np.stack([kx * A, ky * A, kz * A], axis=1).astype(np.int32)
    fluid_mask = masks[kz, ky, kx].astype(np.uint64)
    nbr = np.full((n_tiles, 27), -1, dtype=np.int32)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                k = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
                cx, cy, cz = kx + dx, ky + dy, kz + dz
                ok = np.ones(n_tiles, dtype=bool)
                for c, n, bit in ((cx, tx, 1), (cy, ty, 2), (cz, tz, 4)):
                    if periodic & bit:
                        c %= n
                    else:
                        ok &= (c >= 0) & (c < n)
                idx = np.where(ok)[0]
                nbr[idx, k] = tile_map[cz[idx], cy[idx], cx[idx]]
    n_fluid = int(fluid.sum())
    eta_t = n_fluid / (n_tiles * A ** 3) if n_tiles else 0.0
    return dict(nx=nx, ny=ny, nz=nz, tx=tx, ty=ty, tz=tz, periodic=periodic, n_tiles=n_tiles,
                n_fluid=n_fluid, eta_t=eta_t, tile_map=tile_map, tile_xyz=tile_xyz, nbr=nbr,
                fluid_mask=fluid_mask, padded=p)


def build_tiles_bruteforce(solid, periodic=0):
    """The same definition in plain Python loops, for tiny inputs."""
    p = pad(solid, periodic)
    nz, ny, nx = p.shape
    tz, ty, tx = nz // A, ny // A, nx // A
    order, masks = [], []
    tile_map = -np.ones((tz, ty, tx), dtype=np.int64)
    for z0 in range(tz):
        for y0 in range(ty):
            for x0 in range(tx):
                m = 0
                for z in range(A):
                    for y in range(A):
                        for x in range(A):
                            if p[A * z0 + z, A * y0 + y, A * x0 + x] == 0:
                                m |= 1 << (x + A * y + A * A * z)
                if m:
                    tile_map[z0, y0, x0] = len(order)
                    order.append((A * x0, A * y0, A * z0))
                    masks.append(m)
    nbr = []
    for (x0, y0, z0) in order:
        row = []
        for k in range(27):
            d = (k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1)
            c = [x0 // A + d[0], y0 // A + d[1], z0 // A + d[2]]
            ok = True
            for a, n in enumerate((tx, ty, tz)):
                if c[a] < 0 or c[a] >= n:
                    if periodic >> a & 1:
                        c[a] %= n
                    else:
                        ok = False
            row.append(int(tile_map[c[2], c[1], c[0]]) if ok else -1)
        nbr.append(row)
    return dict(tile_map=tile_map, tile_xyz=order, fluid_mask=masks, nbr=nbr)
