// Shared definitions of the tiled LBM library: error reporting, the D3Q19
// velocity set as compile-time tables, and the device-side table layout.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "lbm.h"

namespace tlbm {

// ---------------------------------------------------------------------------
// errors: a thread-local message behind lbm_last_error()
// ---------------------------------------------------------------------------
int fail(int code, const char *fmt, ...);
void clear_error();

// ---------------------------------------------------------------------------
// D3Q19 (Section 2.2, Fig. 1 caption; weights listed after Eq. 4).
// 0 rest; 1..6 E N W S T B; 7..18 NE NW SW SE ET EB WT WB NT NB ST SB.
// ---------------------------------------------------------------------------
constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, 0, -1, 0, 0, 0, 1, -1, -1, 1, 1, 1, -1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 1, 0, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};

constexpr int opposite(int i) {
    for (int j = 0; j < Q; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) return j;
    return -1;
}
constexpr double weight(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// lane n = x + 4y + 16z inside a tile (the XYZ map of Eq. 11)
constexpr int TILE = 64;

// ---------------------------------------------------------------------------
// device table layout inside the caller's `tables` buffer
//   [0]            uint64 fluid mask per tile
//   [nbr_off]      int32 [n_tiles][32]: the 27 neighbours, padded with -1
//   [xyz_off]      int32 [n_tiles][4]:  corner x, y, z, 0
// ---------------------------------------------------------------------------
constexpr int NBR_STRIDE = 32;
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
struct TableLayout {
    size_t mask_off, nbr_off, xyz_off, total;
    explicit TableLayout(int64_t n_tiles) {
        mask_off = 0;
        nbr_off = align_up(mask_off + (size_t)n_tiles * 8, 256);
        xyz_off = align_up(nbr_off + (size_t)n_tiles * NBR_STRIDE * 4, 256);
        total = align_up(xyz_off + (size_t)n_tiles * 16, 256);
    }
};

struct DevTables {
    const uint64_t *mask;
    const int32_t *nbr;
    const int32_t *xyz;
};

// reduction scratch: per-tile partials of 8 doubles + the final 8
constexpr int NSUM = 8;

}  // namespace tlbm
