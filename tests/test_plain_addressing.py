"""The address algebra of the FP16 (whole 64-slot block) gather, on the CPU.

A lane's source slot for direction i is lane + C_r, where r is the region of
the tile (self or a face or edge neighbour) its upstream node falls in and
C_r a per-wave constant.  The kernel forms it without a per-region select as
lane + C_00 + (M_a & (C_a - C_00)) [+ (M_b & (C_b - C_00))
+ (M_a & M_b & (C_ab - C_a - C_b + C_00))], with M_a the all-ones mask of the
lanes whose shifted node leaves the tile along axis a, in unsigned 32-bit
wrap-around arithmetic.  This checks that identity for every D3Q19 direction
(pull and reverse shifts), every lane and random 32-bit constants; the GPU
parity tests check the kernel itself."""
import numpy as np

M32 = 0xFFFFFFFF
CX = [0, 1, 0, -1, 0, 0, 0, 1, -1, -1, 1, 1, 1, -1, -1, 0, 0, 0, 0]
CY = [0, 0, 1, 0, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, 1, -1, -1]
CZ = [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1]


def _crossing(shift, lane):
    """Per axis, 1 when the lane's node plus the shift leaves the 4^3 tile."""
    node = (lane & 3, (lane >> 2) & 3, lane >> 4)
    return tuple(int(not 0 <= n + s <= 3) for n, s in zip(node, shift))


def test_masked_form_equals_region_select():
    rng = np.random.default_rng(5)
    for _ in range(50):
        const = {}  # C_r per region flags (bx, by, bz), random 32-bit values
        for bx in (0, 1):
            for by in (0, 1):
                for bz in (0, 1):
                    const[(bx, by, bz)] = int(rng.integers(0, 2 ** 32))
        for i in range(1, 19):
            for sign in (-1, 1):
                shift = (sign * CX[i], sign * CY[i], sign * CZ[i])
                axes = [a for a in range(3) if shift[a] != 0]
                assert 1 <= len(axes) <= 2  # D3Q19 has no corner directions
                f1 = tuple(int(a == axes[0]) for a in range(3))
                c00, c1 = const[(0, 0, 0)], const[f1]
                for lane in range(64):
                    cross = _crossing(shift, lane)
                    ref = (lane + const[cross]) & M32
                    m1 = M32 if cross[axes[0]] else 0
                    e = (lane + c00 + (m1 & ((c1 - c00) & M32))) & M32
                    if len(axes) == 2:
                        f2 = tuple(int(a == axes[1]) for a in range(3))
                        f12 = tuple(x | y for x, y in zip(f1, f2))
                        c2, c12 = const[f2], const[f12]
                        m2 = M32 if cross[axes[1]] else 0
                        e = (e + (m2 & ((c2 - c00) & M32)) + ((m1 & m2) & ((c12 - c1 - c2 + c00) & M32))) & M32
                    assert e == ref, (i, sign, lane)
