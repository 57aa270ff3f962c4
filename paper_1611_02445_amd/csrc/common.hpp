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

// multiple relaxation times: moment k of direction i, the D3Q19 basis of
// d'Humieres, Ginzburg, Krafczyk, Lallemand and Luo (2002) written as
// polynomials of c (rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx,
// p_ww, pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z); the rows are orthogonal
constexpr int mrt_coef(int k, int i) {
    const int cx = CX[i], cy = CY[i], cz = CZ[i];
    const int c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return cx;
    case 4: return (5 * c2 - 9) * cx;
    case 5: return cy;
    case 6: return (5 * c2 - 9) * cy;
    case 7: return cz;
    case 8: return (5 * c2 - 9) * cz;
    case 9: return 3 * cx * cx - c2;
    case 10: return (3 * cx * cx - c2) * (3 * c2 - 5);
    case 11: return cy * cy - cz * cz;
    case 12: return (cy * cy - cz * cz) * (3 * c2 - 5);
    case 13: return cx * cy;
    case 14: return cy * cz;
    case 15: return cx * cz;
    case 16: return (cy * cy - cz * cz) * cx;
    case 17: return (cz * cz - cx * cx) * cy;
    default: return (cx * cx - cy * cy) * cz;
    }
}
constexpr int mrt_norm(int k) {
    int n = 0;
    for (int i = 0; i < Q; ++i) n += mrt_coef(k, i) * mrt_coef(k, i);
    return n;
}
// the same as a table, evaluated by the compiler
struct MrtTable {
    int c[Q][Q];
    int n[Q];
};
constexpr MrtTable make_mrt_table() {
    MrtTable t{};
    for (int k = 0; k < Q; ++k) {
        for (int i = 0; i < Q; ++i) t.c[k][i] = mrt_coef(k, i);
        t.n[k] = mrt_norm(k);
    }
    return t;
}
constexpr MrtTable MRT = make_mrt_table();
// relaxation rate of moment k; 0 marks the conserved moments (rho, j), whose
// non-equilibrium part vanishes; -1 marks the viscous moments (rate 1/tau)
constexpr double mrt_rate(int k) {
    switch (k) {
    case 0: case 3: case 5: case 7: return 0.0;
    case 1: return 1.19;
    case 2: case 10: case 12: return 1.4;
    case 4: case 6: case 8: return 1.2;
    case 16: case 17: case 18: return 1.98;
    default: return -1.0;
    }
}

// Opposite directions pair up (9 pairs, the lower index first); every moment
// row is either even or odd under c -> -c (the scalar and tensor moments even,
// the vector ones odd)
constexpr int pair_first(int p) {
    int n = 0;
    for (int i = 1; i < Q; ++i) {
        if (opposite(i) < i) continue;
        if (n == p) return i;
        ++n;
    }
    return -1;
}
constexpr int NPAIR = 9;
constexpr bool mrt_row_odd(int k) {
    for (int i = 1; i < Q; ++i)
        if (mrt_coef(k, i) != -mrt_coef(k, opposite(i))) return false;
    return true;
}

// lane n = x + 4y + 16z inside a tile (the XYZ map of Eq. 11)
constexpr int TILE = 64;

// ---------------------------------------------------------------------------
// lattice layout
//   runs  (FP64, FP32): tile t with k fluid nodes owns one contiguous run of
//         19*k values, direction i at base[t] + i*k + slot, slot = number of
//         fluid nodes of the tile below the node; the run is padded to whole
//         128-byte lines
//   plain (FP16): tile t owns 19 blocks of 64 values at t*19*64 + i*64 + n;
//         a block is exactly one 128-byte line
// ---------------------------------------------------------------------------
inline size_t storage_size(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32 ? 4 : 2); }
// Per-node fields with three components (the force density and its
// gradient) are kept per fluid slot as well: tile t owns 3*k entries at
// fbase[t] + c*k + slot (c = x, y, z), padded to a multiple of FIELD_PAD
// entries (128 bytes of FP64, 64 of FP32).
constexpr uint64_t FIELD_PAD = 16;
inline uint64_t field_elems(uint64_t mask) {
    const uint64_t k = (uint64_t)__builtin_popcountll(mask);
    return (3 * k + FIELD_PAD - 1) / FIELD_PAD * FIELD_PAD;
}
inline bool runs_layout(int storage) { return storage != LBM_F16S; }
inline uint64_t run_elems(uint64_t mask, int storage) {
    const uint64_t L = 128 / storage_size(storage);
    const uint64_t k = (uint64_t)__builtin_popcountll(mask);
    return (Q * k + L - 1) / L * L;
}

// ---------------------------------------------------------------------------
// device table layout inside the caller's `tables` buffer
//   [rec_off]    TileRec per tile: fluid mask, element offset of its data
//   [nbm_off]    uint64 [n_tiles][20]: fluid masks of the 19 tiles a D3Q19
//                step reads from (the tile itself, 6 face and 12 edge
//                neighbours; corners are never needed), 0 for a missing one
//   [nbb32_off]  uint32 [n_tiles][20]: element offsets of the same 19 tiles
//   [nbb64_off]  uint64 [n_tiles][20]: the same offsets in 64 bits
//   [xyz_off]    int32  [n_tiles][4]: corner x, y, z, 0
//   [fld_off]    uint64 [n_tiles]: entry offset of the tile's per-node field run
// The neighbourhood is gathered once on the host, so a wave reads it with a
// few wide scalar loads instead of chasing 19 tile numbers.
// ---------------------------------------------------------------------------
struct TileRec {
    uint64_t mask;
    uint64_t base;
};
constexpr int NB_STRIDE = 20;
// slot of neighbour k = (dx+1) + 3(dy+1) + 9(dz+1) in a neighbourhood row,
// -1 for the 8 corners
constexpr int nb_slot(int k) {
    int slot = 0;
    for (int j = 0; j < 27; ++j) {
        const int nz = (j % 3 != 1) + ((j / 3) % 3 != 1) + (j / 9 != 1);
        if (nz == 3) {
            if (j == k) return -1;
            continue;
        }
        if (j == k) return slot;
        ++slot;
    }
    return -1;
}
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
struct TableLayout {
    size_t rec_off, nbm_off, nbb32_off, nbb64_off, xyz_off, fld_off, total;
    explicit TableLayout(int64_t n_tiles) {
        const size_t n = (size_t)n_tiles;
        rec_off = 0;
        nbm_off = align_up(rec_off + n * sizeof(TileRec), 256);
        nbb32_off = align_up(nbm_off + n * NB_STRIDE * 8, 256);
        nbb64_off = align_up(nbb32_off + n * NB_STRIDE * 4, 256);
        xyz_off = align_up(nbb64_off + n * NB_STRIDE * 8, 256);
        fld_off = align_up(xyz_off + n * 16, 256);
        total = align_up(fld_off + n * 8, 256);
    }
};

struct DevTables {
    const TileRec *rec;
    const uint64_t *nbm;
    const uint32_t *nbb32;
    const uint64_t *nbb64;
    const int32_t *xyz;
    const uint64_t *fbase;
};

// reduction scratch: per-tile partials of 8 doubles + the final 8
constexpr int NSUM = 8;

}  // namespace tlbm
