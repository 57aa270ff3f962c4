// C ABI entry points: parameter validation, buffer sizing, table upload,
// lattice ping-pong and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace tlbm;

// A replayable chunk of steps: GRAPH_STEPS launches captured once from one
// lattice parity with the kernel arguments in P.
constexpr int32_t GRAPH_STEPS = 32;
struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Phys P{};
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

struct lbm_ctx {
    lbm_params params;
    int32_t nx, ny, nz, periodic;
    int32_t n_tiles;
    int64_t n_fluid;
    void *a, *b;        // the two lattices
    int cur;            // 0: a is current, 1: b is current
    void *tables;
    uint32_t adj_launches = 0;  // adjoint step launches so far
    double *scratch;    // [n_tiles][8] partials + [8] final
    hipStream_t stream;
    Launch L;
    Launch LA;          // the adjoint kernels' launch shape
    Phys P;
    size_t state_bytes;
    int device;
    std::vector<int32_t> corner;  // [n_tiles][3] tile corners in device order (host copy)
    StepGraph graphs[2];          // lbm_step_graphed, by starting parity
    hipStream_t capture = nullptr;  // private stream the graphs are captured on
    double *noalloc = nullptr;      // this device's copy of noalloc_scratch (lbm_macroscopic_noalloc)
    hipError_t noalloc_err = hipSuccess;
    ~lbm_ctx() {
        graphs[0].release();
        graphs[1].release();
        if (capture) (void)hipStreamDestroy(capture);
    }
};

namespace {

size_t arith_size(int storage) { return storage == LBM_F64 ? 8 : 4; }

// entries of one per-node field (force density or its gradient)
uint64_t field_entries(const lbm_tiles *t) {
    uint64_t e = 0;
    for (int64_t i = 0; i < t->n_tiles; ++i) e += field_elems(t->fluid_mask[i]);
    return e;
}

// elements of one lattice of the given storage
uint64_t lattice_elems(const lbm_tiles *t, int storage) {
    if (!runs_layout(storage)) return (uint64_t)t->n_tiles * Q * TILE;
    uint64_t e = 0;
    for (int64_t i = 0; i < t->n_tiles; ++i) e += run_elems(t->fluid_mask[i], storage);
    return e;
}

int check_params(const lbm_params *p) {
    if (!p) return fail(LBM_E_INVAL, "NULL params");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_E_INVAL, "tau must be > 1/2 (got %g)", p->tau);
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return fail(LBM_E_INVAL, "rho0 must be > 0 (got %g)", p->rho0);
    if (p->storage < LBM_F64 || p->storage > LBM_F16S) return fail(LBM_E_INVAL, "unknown storage %d", p->storage);
    if (p->model < LBM_QUASI_COMPRESSIBLE || p->model > LBM_MRT_INCOMPRESSIBLE)
        return fail(LBM_E_INVAL, "unknown model %d", p->model);
    if (p->f16_log2_scale < 0 || p->f16_log2_scale > 30)
        return fail(LBM_E_INVAL, "f16_log2_scale must be in [0, 30] (got %d)", p->f16_log2_scale);
    const int tpw = p->tiles_per_wg;
    if (!(tpw == 0 || tpw == 1 || tpw == 2 || tpw == 4 || tpw == 8))
        return fail(LBM_E_INVAL, "tiles_per_wg must be 0, 1, 2, 4 or 8 (got %d)", tpw);
    if (p->tile_order < 0 || p->tile_order > 5)
        return fail(LBM_E_INVAL, "tile_order must be in 0..5 (got %d)", p->tile_order);
    if (p->wide_offsets != 0 && p->wide_offsets != 1)
        return fail(LBM_E_INVAL, "wide_offsets must be 0 or 1 (got %d)", p->wide_offsets);
    if (p->f32_unshifted != 0 && p->f32_unshifted != 1)
        return fail(LBM_E_INVAL, "f32_unshifted must be 0 or 1 (got %d)", p->f32_unshifted);
    if (p->f32_unshifted && p->storage != LBM_F32)
        return fail(LBM_E_INVAL, "f32_unshifted applies to FP32 storage only");
    if (p->f16_rounding != 0 && p->f16_rounding != 1)
        return fail(LBM_E_INVAL, "f16_rounding must be 0 (stochastic) or 1 (nearest) (got %d)", p->f16_rounding);
    if (p->check_u_max != 0 && p->check_u_max != 1)
        return fail(LBM_E_INVAL, "check_u_max must be 0 or 1 (got %d)", p->check_u_max);
    return LBM_OK;
}

int check_tiles(const lbm_tiles *t) {
    if (!t) return fail(LBM_E_INVAL, "NULL tiles");
    if (t->n_tiles < 0) return fail(LBM_E_INVAL, "negative tile count");
    if (t->n_tiles > 0 && (!t->nbr || !t->fluid_mask || !t->tile_xyz))
        return fail(LBM_E_INVAL, "tiles without tables");
    return LBM_OK;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// runs f, turning a failed host allocation into LBM_E_NOMEM rather than
// letting the exception unwind through the C interface
template <class F>
int no_throw(const char *what, F &&f) {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return fail(LBM_E_NOMEM, "%s: out of host memory", what);
    }
}

// tiles (waves) per workgroup when the caller leaves it to the library: 4 was
// the fastest of 1, 2, 4, 8 for every storage type on the sphere packs
constexpr int DEFAULT_TPW = 4;
// device tile order when the caller leaves it to the library: Morton (the
// Hilbert order ties it, discovery order and the slabs trail)
constexpr int DEFAULT_TILE_ORDER = 4;

// spread the bits of a 21-bit integer three apart (Morton interleave)
uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
}

// Position of (x, y, z) along a 3-D Hilbert curve over a 2^b cube, after
// J. Skilling, "Programming the Hilbert curve" (AIP Conf. Proc. 707, 2004):
// the coordinates are turned, bit plane by bit plane from the top, into the
// "transposed" index (undoing the curve's rotations and reflections, then a
// Gray code), whose bits, taken plane by plane, are the index.
uint64_t hilbert3(uint32_t x, uint32_t y, uint32_t z, int b) {
    uint32_t X[3] = {x, y, z};
    for (uint32_t q = 1u << (b - 1); q > 1; q >>= 1) {
        const uint32_t low = q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & q) {
                X[0] ^= low;
            } else {
                const uint32_t swap = (X[0] ^ X[i]) & low;
                X[0] ^= swap;
                X[i] ^= swap;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t flip = 0;
    for (uint32_t q = 1u << (b - 1); q > 1; q >>= 1)
        if (X[2] & q) flip ^= q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= flip;
    uint64_t h = 0;
    for (int k = b - 1; k >= 0; --k)
        h = (h << 3) | ((X[0] >> k & 1u) << 2) | ((X[1] >> k & 1u) << 1) | (X[2] >> k & 1u);
    return h;
}

// Order in which the device stores and processes the kept tiles (a
// permutation of the discovery order).  Consecutive device tiles run at the
// same time on one XCD, so an order that keeps the six face neighbours close
// lets the partially shared neighbour lines be found in that XCD's L2.
//   1 discovery (z outer, y, x inner), 2/3 slabs of 4/8 tile planes with z
//   innermost inside a slab, 4 Morton (bit-interleaved tile coordinates),
//   5 Hilbert (no jumps between consecutive tiles of the curve)
void processing_order(const lbm_tiles *t, int order, std::vector<int32_t> &perm) {
    const int64_t n = t->n_tiles;
    perm.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    if (order == 1) return;
    std::vector<uint64_t> key((size_t)n);
    const uint64_t TX = (uint64_t)t->tx, TY = (uint64_t)t->ty;
    // bits per coordinate of the Hilbert cube (a key of 3 b bits; past 21 it
    // wraps, which leaves the sort a permutation, only a less local one)
    int hb = 1;
    while ((1ull << hb) < std::max<uint64_t>(std::max<uint64_t>(TX, TY), (uint64_t)t->tz)) ++hb;
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t x = (uint64_t)(t->tile_xyz[3 * i] / 4), y = (uint64_t)(t->tile_xyz[3 * i + 1] / 4),
                       z = (uint64_t)(t->tile_xyz[3 * i + 2] / 4);
        if (order == 2 || order == 3) {
            const uint64_t S = order == 2 ? 4 : 8;
            key[i] = (((z / S) * TY + y) * TX + x) * S + (z % S);
        } else if (order == 5) {
            key[i] = hilbert3((uint32_t)x, (uint32_t)y, (uint32_t)z, hb);
        } else {
            key[i] = spread3(x) | spread3(y) << 1 | spread3(z) << 2;
        }
    }
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
}

// Reduction scratch of lbm_macroscopic_noalloc: the per-tile partials and
// the final sums of up to LBM_NOALLOC_MAX_TILES tiles.  Host code never uses
// this name as an address (on the host it is only a handle to the symbol):
// each device's copy is looked up once with hipGetSymbolAddress and that
// pointer is what the kernels get.
static __device__ __align__(256) double noalloc_scratch[((size_t)LBM_NOALLOC_MAX_TILES + 1) * NSUM];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mutex;
double *noalloc_ptr[NOALLOC_MAX_DEVICES];

// the address of the current device's copy of noalloc_scratch, looked up on
// the first call for that device (the caller has that device current)
hipError_t noalloc_lookup(int device, double **out) {
    *out = nullptr;
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(noalloc_mutex);
    if (!noalloc_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        noalloc_ptr[device] = reinterpret_cast<double *>(p);
    }
    *out = noalloc_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" int lbm_tile_order(const lbm_tiles *tiles, int32_t order, int32_t *perm) {
    clear_error();
    int rc;
    if ((rc = check_tiles(tiles))) return rc;
    if (order < 0 || order > 5) return fail(LBM_E_INVAL, "lbm_tile_order: order must be in 0..5 (got %d)", order);
    if (!perm) return fail(LBM_E_INVAL, "lbm_tile_order: NULL output");
    return no_throw("lbm_tile_order", [&]() -> int {
        std::vector<int32_t> p;
        processing_order(tiles, order == 0 ? DEFAULT_TILE_ORDER : order, p);
        std::copy(p.begin(), p.end(), perm);
        return LBM_OK;
    });
}

extern "C" int lbm_required_bytes(const lbm_tiles *tiles, const lbm_params *params, lbm_sizes *out) {
    clear_error();
    int rc;
    if ((rc = check_tiles(tiles)) || (rc = check_params(params))) return rc;
    if (!out) return fail(LBM_E_INVAL, "NULL output");
    const size_t n = (size_t)tiles->n_tiles;
    out->state_bytes = lattice_elems(tiles, params->storage) * storage_size(params->storage);
    out->table_bytes = TableLayout((int64_t)n).total;
    out->scratch_bytes = (n + 1) * NSUM * sizeof(double);
    const size_t fe = field_entries(tiles);
    out->force_bytes = fe * arith_size(params->storage);
    // the adjoint lattice has the layout and element type of the state (runs);
    // FP16 storage has no adjoint
    out->adjoint_bytes = params->storage == LBM_F16S ? 0 : out->state_bytes;
    out->grad_force_bytes = fe * sizeof(double);
    out->bc_bytes = n * 9 * sizeof(uint64_t);
    out->dense_nodes = (size_t)tiles->nx * (size_t)tiles->ny * (size_t)tiles->nz;
    return LBM_OK;
}

extern "C" int lbm_create(const lbm_tiles *tiles, const lbm_params *params, void *state_a, void *state_b,
                          void *tables, void *scratch, void *hip_stream, lbm_ctx **out) {
    clear_error();
    int rc;
    if ((rc = check_tiles(tiles)) || (rc = check_params(params))) return rc;
    if (!out) return fail(LBM_E_INVAL, "NULL output");
    *out = nullptr;
    const int64_t n = tiles->n_tiles;
    if (n > 0 && (!state_a || !state_b || !tables || !scratch))
        return fail(LBM_E_INVAL, "lbm_create: NULL device buffer");
    if (n > 0 && state_a == state_b) return fail(LBM_E_INVAL, "lbm_create: the two lattices must differ");
    // Validate every table entry the kernels will index with.
    int64_t fluid = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (tiles->fluid_mask[i] == 0) return fail(LBM_E_INVAL, "lbm_create: kept tile %lld has no fluid node", (long long)i);
        fluid += __builtin_popcountll(tiles->fluid_mask[i]);
        for (int k = 0; k < 27; ++k) {
            const int32_t v = tiles->nbr[27 * i + k];
            if (v < -1 || v >= n) return fail(LBM_E_INVAL, "lbm_create: neighbour index %d out of range", v);
        }
        if (tiles->nbr[27 * i + 13] != (int32_t)i) return fail(LBM_E_INVAL, "lbm_create: tile %lld is not its own centre neighbour", (long long)i);
        for (int a = 0; a < 3; ++a) {
            const int32_t c = tiles->tile_xyz[3 * i + a];
            const int32_t lim = a == 0 ? tiles->nx : (a == 1 ? tiles->ny : tiles->nz);
            if (c < 0 || c % 4 || c + 4 > lim) return fail(LBM_E_INVAL, "lbm_create: tile corner out of the box");
        }
    }
    // n_fluid normalises the adjoint loss and decides which measurement
    // kernels may address a lattice as whole tiles: it must be the masks' count
    if (fluid != tiles->n_fluid)
        return fail(LBM_E_INVAL, "lbm_create: n_fluid %lld does not match the %lld fluid nodes of the masks",
                    (long long)tiles->n_fluid, (long long)fluid);
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_E_NOMEM, "lbm_create: out of host memory");
    c->params = *params;
    if (c->params.tiles_per_wg == 0) c->params.tiles_per_wg = DEFAULT_TPW;
    if (c->params.tile_order == 0) c->params.tile_order = DEFAULT_TILE_ORDER;
    c->nx = tiles->nx;
    c->ny = tiles->ny;
    c->nz = tiles->nz;
    c->periodic = tiles->periodic;
    c->n_tiles = (int32_t)n;
    c->n_fluid = tiles->n_fluid;
    c->a = state_a;
    c->b = state_b;
    c->cur = 0;
    c->tables = tables;
    c->scratch = reinterpret_cast<double *>(scratch);
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->state_bytes = lattice_elems(tiles, params->storage) * storage_size(params->storage);
    if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
    // set-up for lbm_macroscopic_noalloc, once per device with the context's
    // device current; a failure is reported by that entry point only
    c->noalloc_err = c->device >= 0 ? noalloc_lookup(c->device, &c->noalloc) : hipErrorNoDevice;

    const TableLayout lay(n);
    if (n > 0) try {
        // device tile d holds discovery tile perm[d]; neighbour numbers are
        // translated with the inverse permutation
        std::vector<int32_t> perm, inv;
        processing_order(tiles, c->params.tile_order, perm);
        inv.assign((size_t)n, 0);
        for (int64_t d = 0; d < n; ++d) inv[perm[d]] = (int32_t)d;
        std::vector<unsigned char> host(lay.total, 0);
        c->corner.assign((size_t)n * 3, 0);
        TileRec *rec = reinterpret_cast<TileRec *>(host.data() + lay.rec_off);
        uint64_t *nbm = reinterpret_cast<uint64_t *>(host.data() + lay.nbm_off);
        uint32_t *nbb32 = reinterpret_cast<uint32_t *>(host.data() + lay.nbb32_off);
        uint64_t *nbb64 = reinterpret_cast<uint64_t *>(host.data() + lay.nbb64_off);
        int32_t *xyz = reinterpret_cast<int32_t *>(host.data() + lay.xyz_off);
        uint64_t *fbase = reinterpret_cast<uint64_t *>(host.data() + lay.fld_off);
        uint64_t next = 0, next_field = 0;
        for (int64_t d = 0; d < n; ++d) {
            const int64_t i = perm[d];
            rec[d].mask = tiles->fluid_mask[i];
            if (runs_layout(params->storage)) {
                rec[d].base = next;
                next += run_elems(tiles->fluid_mask[i], params->storage);
            } else {
                rec[d].base = (uint64_t)d * Q * TILE;
            }
            fbase[d] = next_field;
            next_field += field_elems(tiles->fluid_mask[i]);
            for (int a = 0; a < 3; ++a) xyz[4 * d + a] = tiles->tile_xyz[3 * i + a];
            for (int a = 0; a < 3; ++a) c->corner[3 * d + a] = tiles->tile_xyz[3 * i + a];
            xyz[4 * d + 3] = 0;
        }
        // neighbourhood rows (needs every tile's record first)
        for (int64_t d = 0; d < n; ++d) {
            const int64_t i = perm[d];
            for (int k = 0; k < 27; ++k) {
                const int s = nb_slot(k);
                if (s < 0) continue;
                const int32_t v = tiles->nbr[27 * i + k];
                const TileRec r = v < 0 ? TileRec{0, 0} : rec[inv[v]];
                nbm[NB_STRIDE * d + s] = r.mask;
                nbb32[NB_STRIDE * d + s] = (uint32_t)r.base;
                nbb64[NB_STRIDE * d + s] = r.base;
            }
        }
        hipError_t e = hipMemcpyAsync(tables, host.data(), lay.total, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "lbm_create: table upload");
        }
    } catch (const std::bad_alloc &) {
        delete c;
        return fail(LBM_E_NOMEM, "lbm_create: out of host memory");
    }
    const unsigned char *tb = reinterpret_cast<const unsigned char *>(tables);
    c->L.stream = c->stream;
    c->L.n_tiles = (int)n;
    c->L.tpw = c->params.tiles_per_wg;
    c->L.grid = (int)((n + c->L.tpw - 1) / c->L.tpw);
    c->L.tb.rec = reinterpret_cast<const TileRec *>(tb + lay.rec_off);
    c->L.tb.nbm = reinterpret_cast<const uint64_t *>(tb + lay.nbm_off);
    c->L.tb.nbb32 = reinterpret_cast<const uint32_t *>(tb + lay.nbb32_off);
    c->L.tb.nbb64 = reinterpret_cast<const uint64_t *>(tb + lay.nbb64_off);
    c->L.tb.xyz = reinterpret_cast<const int32_t *>(tb + lay.xyz_off);
    c->L.tb.fbase = reinterpret_cast<const uint64_t *>(tb + lay.fld_off);
    // every byte offset into a lattice (an adjoint lattice has the layout and
    // size of the state) must fit 32 bits for the 32-bit kernels
    c->L.off32 = c->state_bytes <= (size_t)UINT32_MAX && !c->params.wide_offsets;
    // The FP64 LBMRT adjoint steps hold 2 waves per SIMD (194-250 VGPRs); with
    // one tile per workgroup instead of four they run 4-5% faster on a 128^3
    // sphere pack, while the LBGK adjoint kernels are fastest at four.  Applies
    // only when the caller left the workgroup size to the library.
    c->LA = c->L;
    if (params->tiles_per_wg == 0 && params->storage == LBM_F64 && params->model >= LBM_MRT_QUASI_COMPRESSIBLE) {
        c->LA.tpw = 1;
        c->LA.grid = (int)n;
    }

    Phys &P = c->P;
    P = Phys{};
    P.storage = params->storage;
    P.model = params->model;
    P.omega = 1.0 / params->tau;
    P.kg = 1.0 - 1.0 / (2.0 * params->tau);
    P.rho0 = params->rho0;
    // reduced storage holds f_i - w_i rho0 unless FP32 is asked to store f_i
    P.rho_base = (params->storage == LBM_F64 || params->f32_unshifted) ? 0.0 : params->rho0;
    P.field = nullptr;
    P.scale = params->storage == LBM_F16S ? std::ldexp(1.0f, params->f16_log2_scale) : 1.0f;
    P.inv_scale = 1.0f / P.scale;
    P.inv_nfluid = c->n_fluid > 0 ? 1.0 / (double)c->n_fluid : 0.0;
    P.f16_stochastic = params->storage == LBM_F16S && params->f16_rounding == 0;
    P.launch_counter = 0;
    *out = c;
    return LBM_OK;
}

extern "C" int lbm_destroy(lbm_ctx *c) {
    delete c;
    return LBM_OK;
}

static void *cur_state(lbm_ctx *c) { return c->cur ? c->b : c->a; }

#define CHECK_CTX(c)                                                      \
    do {                                                                  \
        clear_error();                                                    \
        if (!(c)) return fail(LBM_E_INVAL, "NULL context");               \
    } while (0)

static int launched(hipError_t e, const char *what) { return e == hipSuccess ? LBM_OK : hip_fail(e, what); }

extern "C" int lbm_init(lbm_ctx *c, double rho0, double ux, double uy, double uz) {
    CHECK_CTX(c);
    if (!(rho0 > 0.0) || !std::isfinite(rho0)) return fail(LBM_E_INVAL, "lbm_init: rho0 must be > 0");
    Phys P = c->P;
    P.rho0 = rho0;  // initial density; the storage shift stays at the context's rho0
    c->cur = 0;
    return launched(launch_init(c->L, P, c->a, c->b, ux, uy, uz), "lbm_init");
}

extern "C" int lbm_set_force(lbm_ctx *c, double gx, double gy, double gz, const double *g_dense_dev, void *g_tile_buf) {
    CHECK_CTX(c);
    if (!g_dense_dev) {
        if (!std::isfinite(gx) || !std::isfinite(gy) || !std::isfinite(gz))
            return fail(LBM_E_INVAL, "lbm_set_force: non-finite force");
        c->P.field = nullptr;
        c->P.F[0] = c->params.rho0 * gx;
        c->P.F[1] = c->params.rho0 * gy;
        c->P.F[2] = c->params.rho0 * gz;
        return LBM_OK;
    }
    if (!g_tile_buf && c->n_tiles > 0) return fail(LBM_E_INVAL, "lbm_set_force: field given without a tile buffer");
    hipError_t e = launch_force_to_tiles(c->L, c->P, g_dense_dev, g_tile_buf, c->nx, c->ny, c->nz);
    if (e != hipSuccess) return hip_fail(e, "lbm_set_force");
    c->P.field = g_tile_buf;
    c->P.F[0] = c->P.F[1] = c->P.F[2] = 0.0;
    return LBM_OK;
}

extern "C" int lbm_set_boundaries(lbm_ctx *c, const uint8_t *type_host, double ux, double uy, double uz,
                                  double rho_out, void *bc_tile_buf) {
    CHECK_CTX(c);
    if (!type_host) {
        c->P.bc = nullptr;
        return LBM_OK;
    }
    if (!std::isfinite(ux) || !std::isfinite(uy) || !std::isfinite(uz) || !std::isfinite(rho_out) || !(rho_out > 0))
        return fail(LBM_E_INVAL, "lbm_set_boundaries: non-finite velocity or non-positive density");
    if (!(std::fabs(ux) < 1.0 && std::fabs(uy) < 1.0 && std::fabs(uz) < 1.0))
        return fail(LBM_E_INVAL, "lbm_set_boundaries: every velocity component must be below 1 in magnitude");
    if (c->n_tiles > 0 && !bc_tile_buf) return fail(LBM_E_INVAL, "lbm_set_boundaries: NULL tile buffer");
    const size_t nx = (size_t)c->nx, ny = (size_t)c->ny, nz = (size_t)c->nz;
    // every flagged node must be a fluid node of a kept tile
    size_t flagged = 0;
    for (size_t n = 0; n < nx * ny * nz; ++n) {
        if (type_host[n] > 12) return fail(LBM_E_INVAL, "lbm_set_boundaries: node code %d is not in 0..12", type_host[n]);
        flagged += type_host[n] != 0;
    }
    return no_throw("lbm_set_boundaries", [&]() -> int {
        // per tile: the mask of its boundary nodes, then their 64 codes
        std::vector<uint64_t> masks((size_t)c->n_tiles * 9, 0);
        size_t found = 0;
        for (int64_t d = 0; d < c->n_tiles; ++d) {
            const size_t x0 = (size_t)c->corner[3 * d], y0 = (size_t)c->corner[3 * d + 1],
                         z0 = (size_t)c->corner[3 * d + 2];
            uint8_t *codes = reinterpret_cast<uint8_t *>(&masks[9 * d + 1]);
            for (int lane = 0; lane < TILE; ++lane) {
                const size_t x = x0 + (lane & 3), y = y0 + ((lane >> 2) & 3), z = z0 + (lane >> 4);
                const uint8_t t = type_host[x + nx * (y + ny * z)];
                if (t) masks[9 * d] |= 1ull << lane;
                codes[lane] = t;
                found += t != 0;
            }
        }
        if (found != flagged)
            return fail(LBM_E_INVAL, "lbm_set_boundaries: %zu flagged nodes lie in dropped tiles", flagged - found);
        // ... and fluid inside its tile
        std::vector<TileRec> rec((size_t)c->n_tiles);
        hipError_t e = hipMemcpyAsync(rec.data(), c->L.tb.rec, rec.size() * sizeof(TileRec), hipMemcpyDeviceToHost,
                                      c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(e, "lbm_set_boundaries: reading tile masks");
        for (int64_t d = 0; d < c->n_tiles; ++d)
            if (masks[9 * d] & ~rec[d].mask) return fail(LBM_E_INVAL, "lbm_set_boundaries: a flagged node is solid");
        if (c->n_tiles > 0) {
            e = hipMemcpyAsync(bc_tile_buf, masks.data(), masks.size() * sizeof(uint64_t), hipMemcpyHostToDevice,
                               c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) return hip_fail(e, "lbm_set_boundaries: upload");
        }
        c->P.bc = reinterpret_cast<const uint64_t *>(bc_tile_buf);
        c->P.bc_u[0] = ux;
        c->P.bc_u[1] = uy;
        c->P.bc_u[2] = uz;
        c->P.bc_rho = rho_out;
        return LBM_OK;
    });
}

extern "C" int lbm_step(lbm_ctx *c, int32_t n) {
    CHECK_CTX(c);
    if (n < 0) return fail(LBM_E_INVAL, "lbm_step: negative step count");
    for (int32_t s = 0; s < n; ++s) {
        void *src = cur_state(c);
        void *dst = c->cur ? c->a : c->b;
        hipError_t e = launch_step(c->L, c->P, src, dst);
        if (e != hipSuccess) return hip_fail(e, "lbm_step");
        c->P.launch_counter++;
        c->cur ^= 1;
    }
    return LBM_OK;
}

// Capture GRAPH_STEPS steps from the current lattice with the kernel
// arguments P, on the context's private stream (the caller's stream is not
// put into capture mode).
static int capture_steps(lbm_ctx *c, StepGraph &g, const Phys &P) {
    g.release();
    hipError_t e = hipSuccess;
    if (!c->capture) e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "lbm_step_graphed: capture stream");
    Launch L = c->L;
    L.stream = c->capture;
    e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "lbm_step_graphed: begin capture");
    void *x = cur_state(c), *y = c->cur ? c->a : c->b;
    for (int32_t s = 0; s < GRAPH_STEPS && e == hipSuccess; ++s) {
        // the launch counter's parity sets the direction a step walks the
        // tiles in (its other use, stochastic rounding, is not graphed)
        Phys Ps = P;
        Ps.launch_counter = (uint32_t)s;
        e = launch_step(L, Ps, x, y);
        std::swap(x, y);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e_end = hipStreamEndCapture(c->capture, &graph);  // always leave capture mode
    if (e == hipSuccess) e = e_end;
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        g.exec = nullptr;
        return hip_fail(e, "lbm_step_graphed: capture");
    }
    g.graph = graph;
    g.P = P;
    return LBM_OK;
}

extern "C" int lbm_step_graphed(lbm_ctx *c, int32_t n) {
    CHECK_CTX(c);
    if (n < 0) return fail(LBM_E_INVAL, "lbm_step_graphed: negative step count");
    if (c->P.storage == LBM_F16S && c->P.f16_stochastic)
        return fail(LBM_E_UNSUPPORTED, "lbm_step_graphed: stochastic FP16 rounding draws new bits every launch, "
                                       "which a replayed graph would repeat");
    const int32_t chunks = c->n_tiles > 0 ? n / GRAPH_STEPS : 0;
    if (chunks > 0) {
        // the captured arguments: everything but the launch counter, which
        // only stochastic rounding reads
        Phys key = c->P;
        key.launch_counter = 0;
        StepGraph &g = c->graphs[c->cur];
        if (!g.exec || std::memcmp(&g.P, &key, sizeof(Phys)) != 0) {
            const int rc = capture_steps(c, g, key);
            if (rc) return rc;
        }
        for (int32_t k = 0; k < chunks; ++k) {
            const hipError_t e = hipGraphLaunch(g.exec, c->stream);
            if (e != hipSuccess) return hip_fail(e, "lbm_step_graphed: launch");
        }
        // an even number of steps: the same lattice is current again
        c->P.launch_counter += (uint32_t)(chunks * GRAPH_STEPS);
    }
    return lbm_step(c, n - chunks * GRAPH_STEPS);
}

extern "C" int lbm_step_buf(lbm_ctx *c, const void *src, void *dst) {
    CHECK_CTX(c);
    if (c->n_tiles > 0 && (!src || !dst)) return fail(LBM_E_INVAL, "lbm_step_buf: NULL lattice");
    if (src == dst && c->n_tiles > 0) return fail(LBM_E_INVAL, "lbm_step_buf: src and dst must differ");
    const int rc = launched(launch_step(c->L, c->P, src, dst), "lbm_step_buf");
    c->P.launch_counter++;
    return rc;
}

extern "C" int lbm_current_state(lbm_ctx *c, void **state) {
    CHECK_CTX(c);
    if (!state) return fail(LBM_E_INVAL, "NULL output");
    *state = cur_state(c);
    return LBM_OK;
}

// the checks a synchronising macroscopic call applies to its reduced sums:
// non-finite values always, the compressibility limit u_max <= 0.05
// (Section 2.2) when the context asks for it
static int check_sums(const lbm_ctx *c, const double *sums, const char *what) {
    if (sums[6] > 0.0) return fail(LBM_E_NUMERIC, "%s: %.0f fluid nodes with non-finite values", what, sums[6]);
    if (c->params.check_u_max && sums[5] > LBM_U_MAX)
        return fail(LBM_E_NUMERIC, "%s: max |u| = %.6g exceeds the compressibility limit %g", what, sums[5], LBM_U_MAX);
    return LBM_OK;
}

// the macroscopic fields and reduced sums of a lattice, with the per-tile
// partials and the final sums in `partials` ([n_tiles + 1][8] doubles)
static int macroscopic_into(lbm_ctx *c, const void *state, double *rho_dev, double *u_dev, double sums[8],
                            double *partials) {
    if (!state) state = cur_state(c);
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    hipError_t e = hipSuccess;
    if (rho_dev) e = launch_fill(c->stream, rho_dev, N);
    if (e == hipSuccess && u_dev) e = launch_fill(c->stream, u_dev, 3 * N);
    double *final_ = partials + (size_t)c->n_tiles * NSUM;
    if (c->n_tiles == 0) {
        for (int k = 0; k < NSUM; ++k) sums[k] = 0.0;
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        return launched(e, "lbm_macroscopic");
    }
    if (e == hipSuccess) e = launch_macro(c->L, c->P, state, rho_dev, u_dev, c->nx, c->ny, c->nz, partials);
    if (e == hipSuccess) e = launch_reduce(c->stream, partials, c->n_tiles, final_);
    if (e == hipSuccess) e = hipMemcpyAsync(sums, final_, NSUM * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_macroscopic");
    return check_sums(c, sums, "lbm_macroscopic");
}

extern "C" int lbm_macroscopic_buf(lbm_ctx *c, const void *state, double *rho_dev, double *u_dev, double sums[8]) {
    CHECK_CTX(c);
    if (!sums) return fail(LBM_E_INVAL, "lbm_macroscopic: NULL sums");
    return macroscopic_into(c, state, rho_dev, u_dev, sums, c->scratch);
}

extern "C" int lbm_macroscopic_noalloc(lbm_ctx *c, const void *state, double *rho_dev, double *u_dev, double sums[8]) {
    CHECK_CTX(c);
    if (!sums) return fail(LBM_E_INVAL, "lbm_macroscopic_noalloc: NULL sums");
    if (c->n_tiles > LBM_NOALLOC_MAX_TILES)
        return fail(LBM_E_RANGE, "lbm_macroscopic_noalloc: %d kept tiles exceed the %d of the static scratch "
                                 "(use lbm_macroscopic_buf)", c->n_tiles, LBM_NOALLOC_MAX_TILES);
    if (!c->noalloc)
        return fail(LBM_E_HIP, "lbm_macroscopic_noalloc: static scratch unavailable on device %d: %s", c->device,
                    hipGetErrorString(c->noalloc_err));
    return macroscopic_into(c, state, rho_dev, u_dev, sums, c->noalloc);
}

extern "C" int lbm_macroscopic(lbm_ctx *c, double *rho_dev, double *u_dev, double sums[8]) {
    CHECK_CTX(c);
    return lbm_macroscopic_buf(c, cur_state(c), rho_dev, u_dev, sums);
}

extern "C" int lbm_permeability(lbm_ctx *c, double g_x, double *k) {
    CHECK_CTX(c);
    if (!k) return fail(LBM_E_INVAL, "NULL output");
    if (g_x == 0.0) return fail(LBM_E_INVAL, "lbm_permeability: g_x must be nonzero");
    double s[8];
    const int rc = lbm_macroscopic(c, nullptr, nullptr, s);
    if (rc) return rc;
    const double nu = (c->params.tau - 0.5) / 3.0;
    const double nbox = (double)c->nx * (double)c->ny * (double)c->nz;
    *k = nu * (s[1] / (c->params.rho0 * nbox)) / g_x;
    return LBM_OK;
}

extern "C" int lbm_get_state(lbm_ctx *c, const void *state, double *f_dense_dev) {
    CHECK_CTX(c);
    if (!f_dense_dev) return fail(LBM_E_INVAL, "lbm_get_state: NULL output");
    if (!state) state = cur_state(c);
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    hipError_t e = launch_fill(c->stream, f_dense_dev, Q * N);
    if (e == hipSuccess) e = launch_get_state(c->L, c->P, state, f_dense_dev, c->nx, c->ny, c->nz);
    return launched(e, "lbm_get_state");
}

extern "C" int lbm_set_state(lbm_ctx *c, const double *f_dense_dev, void *state) {
    CHECK_CTX(c);
    if (!f_dense_dev) return fail(LBM_E_INVAL, "lbm_set_state: NULL input");
    if (!state) state = cur_state(c);
    return launched(launch_set_state(c->L, c->P, f_dense_dev, state, c->nx, c->ny, c->nz), "lbm_set_state");
}

extern "C" int lbm_tiles_to_dense(lbm_ctx *c, const void *tile_buf, int32_t ncomp, int32_t dtype, double *dense_dev) {
    CHECK_CTX(c);
    if (!tile_buf || !dense_dev) return fail(LBM_E_INVAL, "lbm_tiles_to_dense: NULL buffer");
    if (ncomp <= 0 || ncomp > 64) return fail(LBM_E_INVAL, "lbm_tiles_to_dense: ncomp must be in 1..64");
    if (dtype != 0 && dtype != 1) return fail(LBM_E_INVAL, "lbm_tiles_to_dense: dtype must be 0 (f64) or 1 (f32)");
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    hipError_t e = launch_fill(c->stream, dense_dev, (size_t)ncomp * N);
    if (e == hipSuccess) e = launch_tiles_to_dense(c->L, tile_buf, ncomp, dtype, dense_dev, c->nx, c->ny, c->nz);
    return launched(e, "lbm_tiles_to_dense");
}

extern "C" int lbm_field_to_dense(lbm_ctx *c, const void *field_buf, int32_t dtype, double *dense_dev) {
    CHECK_CTX(c);
    if (!dense_dev || (!field_buf && c->n_tiles > 0)) return fail(LBM_E_INVAL, "lbm_field_to_dense: NULL buffer");
    if (dtype != 0 && dtype != 1) return fail(LBM_E_INVAL, "lbm_field_to_dense: dtype must be 0 (f64) or 1 (f32)");
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    hipError_t e = launch_fill(c->stream, dense_dev, 3 * N);
    if (e == hipSuccess) e = launch_field_to_dense(c->L, field_buf, dtype, dense_dev, c->nx, c->ny, c->nz);
    return launched(e, "lbm_field_to_dense");
}

static int adjoint_supported(lbm_ctx *c) {
    if (c->params.storage == LBM_F16S) return fail(LBM_E_UNSUPPORTED, "adjoint: built for FP64 and FP32 storage only");
    if (c->P.bc) return fail(LBM_E_UNSUPPORTED, "adjoint: not built for open boundaries");
    return LBM_OK;
}

// adjoint lattices hold unshifted values: the state codec with no shift
static Phys unshifted(const lbm_ctx *c) {
    Phys P = c->P;
    P.rho_base = 0.0;
    return P;
}

extern "C" int lbm_adjoint_get(lbm_ctx *c, const void *adj, double *dense_dev) {
    CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc) return rc;
    if (!dense_dev || (!adj && c->n_tiles > 0)) return fail(LBM_E_INVAL, "lbm_adjoint_get: NULL buffer");
    const size_t N = (size_t)c->nx * c->ny * c->nz;
    hipError_t e = launch_fill(c->stream, dense_dev, Q * N);
    if (e == hipSuccess) e = launch_get_state(c->L, unshifted(c), adj, dense_dev, c->nx, c->ny, c->nz);
    return launched(e, "lbm_adjoint_get");
}

extern "C" int lbm_adjoint_set(lbm_ctx *c, const double *dense_dev, void *adj) {
    CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc) return rc;
    if (!dense_dev || (!adj && c->n_tiles > 0)) return fail(LBM_E_INVAL, "lbm_adjoint_set: NULL buffer");
    return launched(launch_set_state(c->L, unshifted(c), dense_dev, adj, c->nx, c->ny, c->nz), "lbm_adjoint_set");
}

extern "C" int lbm_adjoint_seed(lbm_ctx *c, const void *s_Tm1, void *eta_T, double *grad_g_tile) {
    CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc) return rc;
    if (c->n_tiles > 0 && (!s_Tm1 || !eta_T || !grad_g_tile)) return fail(LBM_E_INVAL, "lbm_adjoint_seed: NULL buffer");
    return launched(launch_adjoint_seed(c->LA, c->P, s_Tm1, eta_T, grad_g_tile), "lbm_adjoint_seed");
}

extern "C" int lbm_adjoint_step(lbm_ctx *c, const void *s_tm2, const void *eta_t, void *eta_tm1, double *grad_g_tile) {
    CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc) return rc;
    if (c->n_tiles > 0 && (!s_tm2 || !eta_t || !eta_tm1 || !grad_g_tile))
        return fail(LBM_E_INVAL, "lbm_adjoint_step: NULL buffer");
    if (eta_t == eta_tm1 && c->n_tiles > 0) return fail(LBM_E_INVAL, "lbm_adjoint_step: eta buffers must differ");
    Phys P = c->P;  // the counter's parity sets the direction the launch walks the tiles in
    P.launch_counter = c->adj_launches++;
    return launched(launch_adjoint_step(c->LA, P, s_tm2, eta_t, eta_tm1, grad_g_tile), "lbm_adjoint_step");
}

extern "C" int lbm_adjoint_final(lbm_ctx *c, const void *eta_1, void *lambda_0) {
    CHECK_CTX(c);
    int rc = adjoint_supported(c);
    if (rc) return rc;
    if (c->n_tiles > 0 && (!eta_1 || !lambda_0)) return fail(LBM_E_INVAL, "lbm_adjoint_final: NULL buffer");
    if (eta_1 == lambda_0 && c->n_tiles > 0) return fail(LBM_E_INVAL, "lbm_adjoint_final: buffers must differ");
    return launched(launch_adjoint_final(c->LA, c->P, eta_1, lambda_0), "lbm_adjoint_final");
}

extern "C" int lbm_calib_step(lbm_ctx *c, int32_t kind, const void *src, void *dst) {
    CHECK_CTX(c);
    if (kind < 1 || kind > 7) return fail(LBM_E_INVAL, "lbm_calib_step: kind must be 1 to 7");
    // the layout study addresses the plain 64-slot blocks, which coincide
    // with the lattice's own bytes only when every kept tile is full
    if (kind >= 3 && c->n_fluid != (int64_t)TILE * c->n_tiles)
        return fail(LBM_E_UNSUPPORTED, "lbm_calib_step: kinds 3-7 need every kept tile entirely fluid");
    if (c->n_tiles > 0 && (!src || !dst || src == dst)) return fail(LBM_E_INVAL, "lbm_calib_step: bad lattices");
    return launched(launch_calib(c->L, kind, c->params.storage, src, dst), "lbm_calib_step");
}

extern "C" int lbm_stream_probe(void *hip_stream, int32_t kind, const void *src, void *dst, size_t bytes,
                                int32_t blocks, int32_t threads) {
    clear_error();
    if (kind < 1 || kind > 3) return fail(LBM_E_INVAL, "lbm_stream_probe: kind must be 1 (read), 2 (write) or 3 (copy)");
    if (bytes == 0 || bytes % 16) return fail(LBM_E_INVAL, "lbm_stream_probe: bytes must be a positive multiple of 16");
    if (blocks < 1 || blocks > (1 << 20)) return fail(LBM_E_INVAL, "lbm_stream_probe: blocks must be in 1..2^20");
    if (!(threads == 64 || threads == 128 || threads == 256 || threads == 512 || threads == 1024))
        return fail(LBM_E_INVAL, "lbm_stream_probe: threads must be 64, 128, 256, 512 or 1024");
    if ((kind != 2 && !src) || !dst) return fail(LBM_E_INVAL, "lbm_stream_probe: NULL buffer");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
        return fail(LBM_E_INVAL, "lbm_stream_probe: buffers must be 16-byte aligned");
    if (kind == 3) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
        if (a < b + bytes && b < a + bytes) return fail(LBM_E_INVAL, "lbm_stream_probe: src and dst overlap");
    }
    return launched(launch_probe(reinterpret_cast<hipStream_t>(hip_stream), kind, src, dst, bytes, blocks, threads),
                    "lbm_stream_probe");
}

extern "C" int lbm_info(lbm_ctx *c, int32_t *n_tiles, int64_t *n_fluid, int32_t *storage, int32_t *grid_blocks) {
    CHECK_CTX(c);
    if (n_tiles) *n_tiles = c->n_tiles;
    if (n_fluid) *n_fluid = c->n_fluid;
    if (storage) *storage = c->params.storage;
    if (grid_blocks) *grid_blocks = c->L.grid;
    return LBM_OK;
}
