// Host tiler: Alg. 1 of the paper (Section 3.1) plus the per-tile fluid masks
// and the 3x3x3 neighbour window the kernel needs (Section 3.4).
//
// One pass over the tile grid in z, y, x order builds the 64-bit fluid mask of
// each tile and numbers the tiles that hold a non-solid node in the order they
// are found; a second pass fills the 27-entry neighbour rows from the dense
// tile map, wrapping periodic axes.  O(box) time and memory.
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"

namespace tlbm {

static thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

void clear_error() { g_error.clear(); }

}  // namespace tlbm

using namespace tlbm;

extern "C" const char *lbm_last_error(void) { return g_error.c_str(); }

extern "C" const char *lbm_version(void) { return "tiledlbm-gfx950 0.1"; }

extern "C" void lbm_tiles_free(lbm_tiles *t) {
    if (!t) return;
    free(t->tile_map);
    free(t->tile_xyz);
    free(t->nbr);
    free(t->fluid_mask);
    free(t);
}

extern "C" int lbm_build_tiles(const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz, int32_t periodic,
                               lbm_tiles **out) {
    clear_error();
    if (!solid || !out) return fail(LBM_E_INVAL, "lbm_build_tiles: NULL argument");
    *out = nullptr;
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(LBM_E_INVAL, "lbm_build_tiles: box dims must be > 0");
    if (periodic & ~7) return fail(LBM_E_INVAL, "lbm_build_tiles: unknown periodic bits 0x%x", periodic);
    const int32_t in_dim[3] = {nx, ny, nz};
    int64_t pad[3];
    for (int a = 0; a < 3; ++a) {
        if ((periodic >> a) & 1) {
            if (in_dim[a] % 4)
                return fail(LBM_E_INVAL, "lbm_build_tiles: periodic axis %c has length %d, not a multiple of 4",
                            "xyz"[a], in_dim[a]);
            pad[a] = in_dim[a];
        } else {
            pad[a] = ((int64_t)in_dim[a] + 3) / 4 * 4;
        }
        if (pad[a] > INT32_MAX) return fail(LBM_E_RANGE, "lbm_build_tiles: padded axis too long");
    }
    const int64_t tx = pad[0] / 4, ty = pad[1] / 4, tz = pad[2] / 4;
    const int64_t n_grid = tx * ty * tz;

    lbm_tiles *t = (lbm_tiles *)calloc(1, sizeof(lbm_tiles));
    if (!t) return fail(LBM_E_NOMEM, "lbm_build_tiles: out of host memory");
    t->nx = (int32_t)pad[0];
    t->ny = (int32_t)pad[1];
    t->nz = (int32_t)pad[2];
    t->tx = (int32_t)tx;
    t->ty = (int32_t)ty;
    t->tz = (int32_t)tz;
    t->periodic = periodic;
    t->tile_map = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_grid);
    if (!t->tile_map) {
        lbm_tiles_free(t);
        return fail(LBM_E_NOMEM, "lbm_build_tiles: out of host memory");
    }

    // pass 1: masks in discovery order (z outer, y, x inner)
    std::vector<uint64_t> masks;
    std::vector<int32_t> corners;
    int64_t n_fluid = 0;
    const size_t sx = 1, sy = (size_t)nx, sz = (size_t)nx * (size_t)ny;
    // pass 1 grows the two lists: an allocation failure there is reported,
    // not thrown through the C interface
    try {
        for (int64_t bz = 0; bz < tz; ++bz)
            for (int64_t by = 0; by < ty; ++by)
                for (int64_t bx = 0; bx < tx; ++bx) {
                    uint64_t m = 0;
                    for (int z = 0; z < 4; ++z) {
                        const int64_t Z = 4 * bz + z;
                        if (Z >= nz) continue;  // padding: solid
                        for (int y = 0; y < 4; ++y) {
                            const int64_t Y = 4 * by + y;
                            if (Y >= ny) continue;
                            const uint8_t *row = solid + (size_t)Z * sz + (size_t)Y * sy;
                            for (int x = 0; x < 4; ++x) {
                                const int64_t X = 4 * bx + x;
                                if (X >= nx) continue;
                                if (!row[(size_t)X * sx]) m |= 1ull << (x + 4 * y + 16 * z);
                            }
                        }
                    }
                    const int64_t g = bx + tx * (by + ty * bz);
                    if (m) {
                        if ((int64_t)masks.size() >= INT32_MAX) {
                            lbm_tiles_free(t);
                            return fail(LBM_E_RANGE, "lbm_build_tiles: more than INT32_MAX non-empty tiles");
                        }
                        t->tile_map[g] = (int32_t)masks.size();
                        masks.push_back(m);
                        corners.push_back((int32_t)(4 * bx));
                        corners.push_back((int32_t)(4 * by));
                        corners.push_back((int32_t)(4 * bz));
                        n_fluid += __builtin_popcountll(m);
                    } else {
                        t->tile_map[g] = -1;
                    }
                }
    } catch (const std::bad_alloc &) {
        lbm_tiles_free(t);
        return fail(LBM_E_NOMEM, "lbm_build_tiles: out of host memory");
    }
    const int64_t n = (int64_t)masks.size();
    t->n_tiles = (int32_t)n;
    t->n_fluid = n_fluid;
    t->eta_t = n ? (double)n_fluid / (64.0 * (double)n) : 0.0;
    t->fluid_mask = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    t->tile_xyz = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(n ? n : 1));
    t->nbr = (int32_t *)malloc(sizeof(int32_t) * 27 * (size_t)(n ? n : 1));
    if (!t->fluid_mask || !t->tile_xyz || !t->nbr) {
        lbm_tiles_free(t);
        return fail(LBM_E_NOMEM, "lbm_build_tiles: out of host memory");
    }
    if (n) {
        memcpy(t->fluid_mask, masks.data(), sizeof(uint64_t) * (size_t)n);
        memcpy(t->tile_xyz, corners.data(), sizeof(int32_t) * 3 * (size_t)n);
    }

    // pass 2: neighbour rows
    const int64_t tdim[3] = {tx, ty, tz};
    for (int64_t i = 0; i < n; ++i) {
        const int64_t c[3] = {t->tile_xyz[3 * i] / 4, t->tile_xyz[3 * i + 1] / 4, t->tile_xyz[3 * i + 2] / 4};
        for (int k = 0; k < 27; ++k) {
            const int d[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
            int64_t p[3];
            bool inside = true;
            for (int a = 0; a < 3; ++a) {
                p[a] = c[a] + d[a];
                if (p[a] < 0 || p[a] >= tdim[a]) {
                    if ((periodic >> a) & 1)
                        p[a] = (p[a] + tdim[a]) % tdim[a];
                    else
                        inside = false;
                }
            }
            t->nbr[27 * i + k] = inside ? t->tile_map[p[0] + tx * (p[1] + ty * p[2])] : -1;
        }
    }
    *out = t;
    return LBM_OK;
}
