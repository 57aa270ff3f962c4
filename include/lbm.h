/*
 * lbm.h -- C ABI of the tiled sparse-geometry D3Q19 lattice-Boltzmann library
 * for AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Tomczak & Szafran, "A new GPU implementation for
 * lattice-Boltzmann simulations on sparse geometries": the box is covered by
 * 4x4x4-node tiles, all-solid tiles are dropped (Section 3.1, Alg. 1), and one
 * fused kernel per time step gathers the 19 distributions of every fluid node
 * from its upstream neighbours (pull streaming), replaces reads from solid
 * neighbours by bounce-back, collides with LBGK and stores the result in a
 * second lattice (Section 3.4, Alg. 2; Eq. 2, 3, 5, 7).  A body force (Guo
 * forcing), periodic axes, reduced-precision storage and a discrete adjoint
 * are additions described with each entry point.
 *
 * Conventions used throughout:
 *   - dense arrays are indexed [..][z][y][x] with x fastest, over the PADDED
 *     box (nx, ny, nz of lbm_tiles);
 *   - D3Q19 directions: 0 rest; 1 E(+x) 2 N(+y) 3 W(-x) 4 S(-y) 5 T(+z)
 *     6 B(-z); 7 NE 8 NW 9 SW 10 SE 11 ET 12 EB 13 WT 14 WB 15 NT 16 NB 17 ST
 *     18 SB (e_3 = W as in the paper's Fig. 1);
 *   - inside a tile, node (x,y,z) in 0..3 has lane/bit n = x + 4y + 16z
 *     (the XYZ map, Eq. 11);
 *   - tile-order buffers are [n_tiles][components][64], tiles in the
 *     context's device order (tile_order; lbm_tile_order lists it); lbm_tiles_to_dense converts;
 *   - per-node fields (the force density and its gradient) hold one entry per
 *     fluid node and component: tile t's run of 3k entries (k fluid nodes),
 *     component c of the node with rank r among the tile's fluid nodes (in
 *     node order n = x + 4y + 16z) at entry c*k + r, padded to a multiple of
 *     16 entries, tiles in device order; lbm_field_to_dense converts;
 *   - device pointers are plain HIP device addresses owned by the caller; the
 *     library allocates no device buffers (lbm_step_graphed alone creates a
 *     private stream and executable graphs, held by the context until
 *     lbm_destroy);
 *   - a context is not thread-safe: one host thread at a time may call into
 *     it; distinct contexts are independent;
 *   - every call returns an lbm_status; on failure lbm_last_error() gives a
 *     thread-local message.  Nothing crosses the ABI as a C++ exception.
 *   - kernel launches are asynchronous on the context's stream; errors of a
 *     launch itself are returned by the launching call, faults inside a kernel
 *     surface at the next synchronising call (lbm_macroscopic*).
 */
#ifndef TILED_LBM_H
#define TILED_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_E_INVAL = -1,       /* bad argument (NULL, tau <= 1/2, bad dims, ...) */
    LBM_E_NOMEM = -2,       /* host allocation failed */
    LBM_E_RANGE = -3,       /* a count does not fit the index types */
    LBM_E_HIP = -4,         /* a HIP runtime call or launch failed */
    LBM_E_STATE = -5,       /* call not valid in the context's current state */
    LBM_E_UNSUPPORTED = -6, /* option combination not built */
    LBM_E_NUMERIC = -7      /* a checking call found non-finite values, or a fluid speed above the
                               compressibility limit when that check is on (check_u_max) */
} lbm_status;

typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2 } lbm_storage;
/* Collision models: bit 0 picks the equilibrium and velocity (Eq. 3 and 5,
 * or Eq. 4 and 6), bit 1 the operator: single relaxation time (LBGK, Eq. 2
 * and 7) or multiple relaxation times (the paper's LBMRT; D3Q19 moment basis
 * and rates of d'Humieres et al. 2002, viscous moments relaxed at 1/tau, Guo
 * forcing in moment space). */
typedef enum {
    LBM_QUASI_COMPRESSIBLE = 0,
    LBM_INCOMPRESSIBLE = 1,
    LBM_MRT_QUASI_COMPRESSIBLE = 2,
    LBM_MRT_INCOMPRESSIBLE = 3
} lbm_model;
enum { LBM_PX = 1, LBM_PY = 2, LBM_PZ = 4 }; /* periodic-axis bits */

/* ------------------------------------------------------------------------
 * Tiling (host only; no device is touched).
 * ------------------------------------------------------------------------ */

/* Result of lbm_build_tiles.  Host memory owned by the library; release with
 * lbm_tiles_free. */
typedef struct lbm_tiles {
    int32_t nx, ny, nz;     /* padded box: each non-periodic axis rounded up to a multiple of 4 */
    int32_t tx, ty, tz;     /* tile grid = padded box / 4 */
    int32_t periodic;       /* LBM_PX | LBM_PY | LBM_PZ */
    int32_t n_tiles;        /* kept (non-empty) tiles */
    int64_t n_fluid;        /* non-solid nodes: the MFLUPS numerator */
    double eta_t;           /* average tile utilisation n_fluid / (64 n_tiles), Eq. 14 */
    int32_t *tile_map;      /* [tz][ty][tx]: tile number or -1 for an all-solid tile ("tileMap") */
    int32_t *tile_xyz;      /* [n_tiles][3]: corner node (x,y,z) of each kept tile, in the
                               order the scan finds them: z outer, y, x inner ("nonEmptyTiles") */
    int32_t *nbr;           /* [n_tiles][27]: tile number of the neighbour at offset (dx,dy,dz),
                               k = (dx+1) + 3(dy+1) + 9(dz+1); 13 is the tile itself; -1 when
                               all-solid or outside a non-periodic axis; periodic axes wrap */
    uint64_t *fluid_mask;   /* [n_tiles]: bit x+4y+16z set for a non-solid node ("nodeType") */
} lbm_tiles;

/* Tile a geometry (Section 3.1, Alg. 1; the tile map and neighbourhood of
 * Section 3.4).
 *   solid    host [nz][ny][nx] bytes, nonzero = solid; read only
 *   nx,ny,nz box size in nodes (> 0)
 *   periodic LBM_P* bits; a periodic axis must have a length that is a
 *            multiple of 4 (padding would change the period) -> LBM_E_INVAL
 *   out      receives a new lbm_tiles
 * Non-periodic axes are extended with solid nodes up to a multiple of 4.
 * Returns LBM_E_RANGE if the tile count exceeds INT32_MAX. */
int lbm_build_tiles(const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz, int32_t periodic,
                    lbm_tiles **out);
void lbm_tiles_free(lbm_tiles *tiles);

/* Device order of the kept tiles.  Within a step every tile reads only the
 * previous lattice and writes only its own nodes (Section 3.1, Alg. 2), so the
 * order in which tiles are stored and processed changes no result.  Host
 * only; no GPU is touched.
 *   tiles  from lbm_build_tiles; read only
 *   order  as lbm_params.tile_order, 0..5 (0 = the library default, Morton)
 *   perm   host int32[n_tiles], caller-owned, written: a context created with
 *          this order stores and processes tile tiles->tile_xyz[perm[d]] as its
 *          d-th tile, so row d of a tile-order buffer belongs to that tile
 * Returns LBM_E_INVAL for a NULL pointer, a malformed tiling or an order
 * outside 0..5; perm is then untouched. */
int lbm_tile_order(const lbm_tiles *tiles, int32_t order, int32_t *perm);

/* ------------------------------------------------------------------------
 * Context and device buffers.
 * ------------------------------------------------------------------------ */
typedef struct lbm_params {
    double tau;             /* LBGK relaxation time (Eq. 2), > 1/2; nu = (tau - 1/2)/3 */
    double rho0;            /* reference density: F = rho0 * g, shift of reduced storage */
    int32_t storage;        /* lbm_storage */
    int32_t model;          /* lbm_model */
    int32_t f16_log2_scale; /* LBM_F16S: stored h = fp16(2^k (f_i - w_i rho0)), k in [0, 30] */
    int32_t tiles_per_wg;   /* tiles (wave64s) per workgroup: 1, 2, 4 or 8; 0 = default */
    int32_t f16_rounding;   /* LBM_F16S stores: 0 = stochastic (unbiased; default), 1 = nearest-even.
                               Stochastic rounding uses gfx950's stochastic-rounding conversion
                               with bits from a counter-based hash of (tile corner, node,
                               direction, launch counter): results are reproducible for the same
                               sequence of launches and do not depend on tile_order. */
    int32_t tile_order;     /* order in which the device stores and processes the kept tiles:
                               0 = library default (Morton), 1 = discovery order, 2 / 3 = slabs of
                               4 / 8 tile planes with z innermost, 4 = Morton (z-order of the tile
                               coordinates), 5 = Hilbert (a curve whose consecutive tiles are
                               always face neighbours).  Only the device layout changes; every dense input
                               and output is the same for all orders (FP64 sums may differ in the
                               last bits: their summation order follows the tiles). */
    int32_t wide_offsets;   /* 0 = 32-bit lattice offsets whenever every byte offset of a lattice
                               fits 32 bits (else 64-bit), 1 = always 64-bit.  Results are
                               identical; 1 exists to exercise the large-lattice kernels on
                               small inputs. */
    int32_t f32_unshifted;  /* LBM_F32 only: 1 stores f_i itself instead of f_i - w_i rho0 (the
                               paper's FP32 storage; kept as an ablation of the shift), 0 =
                               shifted (default).  Must be 0 for other storage types. */
    int32_t check_u_max;    /* 1 = lbm_macroscopic, lbm_macroscopic_buf, lbm_macroscopic_noalloc
                               and lbm_permeability return LBM_E_NUMERIC (after filling their outputs)
                               when the largest fluid speed max |u| exceeds LBM_U_MAX = 0.05, the
                               bound on the macroscopic velocity that keeps the compressibility
                               error of the quasi-compressible model small (Section 2.2);
                               0 = no check (default). */
} lbm_params;

/* The compressibility limit checked when lbm_params.check_u_max is set. */
#define LBM_U_MAX 0.05

typedef struct lbm_sizes {
    size_t state_bytes;      /* one lattice: per tile 19*k values (k fluid nodes) padded to whole
                                128-byte lines (FP64, FP32); n_tiles * 19 * 64 * 2 (FP16) */
    size_t table_bytes;      /* device copy of the tiling tables */
    size_t scratch_bytes;    /* reduction scratch */
    size_t force_bytes;      /* per-node force field: sum over tiles of 3k padded to 16 entries,
                                times sizeof(arith) (FP64 storage: 8, else 4) */
    size_t adjoint_bytes;    /* one adjoint lattice: state_bytes (FP64, FP32), 0 for FP16 */
    size_t grad_force_bytes; /* force gradient, FP64, same entries as the force field: entries * 8 */
    size_t bc_bytes;         /* open boundaries: n_tiles * 72 (node mask + 64 node codes) */
    size_t dense_nodes;      /* nx * ny * nz of the padded box */
} lbm_sizes;

typedef struct lbm_ctx lbm_ctx;

/* Buffer sizes for a tiling and parameter set.  All pointers required. */
int lbm_required_bytes(const lbm_tiles *tiles, const lbm_params *params, lbm_sizes *out);

/* Create a context.
 *   state_a, state_b  two device lattices of state_bytes each ("two copies of
 *                     f_i", Section 3.1); a step reads one and writes the other
 *   tables            device buffer of table_bytes; filled here from `tiles`
 *   scratch           device buffer of scratch_bytes
 *   hip_stream        hipStream_t the context launches on (NULL = default stream)
 * The tables are copied to the device and the stream is synchronised before
 * returning, so `tiles` may be freed afterwards.  Parameters are validated
 * (LBM_E_INVAL): tau > 1/2, rho0 > 0, known storage and model, f16 scale in
 * [0,30], tiles_per_wg in {0,1,2,4,8}, f16_rounding in {0,1}, tile_order in
 * 0..5, wide_offsets in {0,1}, f32_unshifted in {0,1} (1 only with LBM_F32),
 * check_u_max in {0,1};
 * the tables are checked (every neighbour index
 * in [-1, n_tiles), each tile its own centre neighbour, no empty kept tile). */
int lbm_create(const lbm_tiles *tiles, const lbm_params *params, void *state_a, void *state_b,
               void *tables, void *scratch, void *hip_stream, lbm_ctx **out);
int lbm_destroy(lbm_ctx *ctx);

/* f_i = feq_i(rho0, u0) (Eq. 3 or 4) at every fluid node of both lattices, 0 at
 * solid nodes; the current lattice becomes state_a. */
int lbm_init(lbm_ctx *ctx, double rho0, double ux, double uy, double uz);

/* Body acceleration g; the force density is F = rho0 * g (Guo forcing).
 * With g_dense_dev == NULL the force is uniform (gx, gy, gz).  Otherwise
 * g_dense_dev is a device FP64 field [3][nz][ny][nx] that is converted into
 * g_tile_buf (force_bytes, caller-owned, must outlive its use) and used from
 * then on; gx, gy, gz are ignored. */
int lbm_set_force(lbm_ctx *ctx, double gx, double gy, double gz, const double *g_dense_dev,
                  void *g_tile_buf);

/* Open boundaries (the paper's Zou-He velocity inlet and constant-pressure
 * outlet, Section 2.2) on faces normal to any axis.
 *   type_host  host [nz][ny][nx] bytes over the padded box: 0 none, else a
 *              code 1..12 with axis a = (code-1)/4 (0 x, 1 y, 2 z) and
 *              r = (code-1)%4:
 *                r = 0 velocity node, the populations with c_a = +1 are
 *                      rebuilt (the domain lies at +a: an inlet on a low face),
 *                r = 1 pressure node, c_a = -1 rebuilt (an outlet on a high face),
 *                r = 2 velocity node, c_a = -1 rebuilt,
 *                r = 3 pressure node, c_a = +1 rebuilt;
 *              a velocity node gets velocity (ux, uy, uz), a pressure node
 *              density rho_out and tangential velocity 0 (codes 1 and 2 are
 *              the x inlet and outlet); NULL removes all open boundaries
 *   bc_tile_buf  device buffer of bc_bytes (caller-owned, must outlive its use)
 * The rebuild follows the gather (which bounces back at the missing
 * upstream nodes) and precedes the collision; with a body force it targets the
 * momentum rho u - F/2 so that the collision's velocity is the prescribed
 * one.  Flagged nodes must be fluid, codes at most 12 and every velocity
 * component below 1 in magnitude (else LBM_E_INVAL).  Synchronises. */
int lbm_set_boundaries(lbm_ctx *ctx, const uint8_t *type_host, double ux, double uy, double uz, double rho_out,
                       void *bc_tile_buf);

/* n fused collide-and-stream steps on the context's stream, alternating the
 * two lattices (Alg. 2).  Asynchronous. */
int lbm_step(lbm_ctx *ctx, int32_t n);

/* The same n steps as lbm_step, bitwise, launched as replays of a HIP graph
 * of 32 steps (the remainder n mod 32 as plain launches): for small grids,
 * where launching a kernel costs as much as running it.  The graph is
 * captured on first use from either lattice parity (on a private stream of
 * the context) and captured again whenever a kernel argument has changed
 * since (force, boundaries, parameters).  Asynchronous on the context's
 * stream.  LBM_E_UNSUPPORTED for FP16 storage with stochastic rounding,
 * whose random bits change with every launch. */
int lbm_step_graphed(lbm_ctx *ctx, int32_t n);

/* One step from lattice `src` to lattice `dst` (any caller buffers of
 * state_bytes, e.g. checkpoint slots; src != dst).  Does not change which
 * lattice is current. */
int lbm_step_buf(lbm_ctx *ctx, const void *src, void *dst);

/* Pointer to the current lattice (the one the last step wrote). */
int lbm_current_state(lbm_ctx *ctx, void **state);

/* Density and velocity of the current lattice: rho = sum f*_i and
 * u = (sum c_i f*_i - F/2) / rho (incompressible: without the division),
 * i.e. the velocity the last collision used.
 *   rho_dev  device FP64 [nz][ny][nx] or NULL; 0 at solid and dropped nodes
 *   u_dev    device FP64 [3][nz][ny][nx] or NULL
 *   sums     host double[8]: total mass sum rho, momentum sum rho u (x, y, z),
 *            fluid node count, max |u|, number of fluid nodes with a
 *            non-finite rho or u, and sum u_x (the adjoint's loss is
 *            sums[7] / sums[4], the mean x-velocity over fluid nodes).
 *            Reduced in FP64 in a fixed order (bitwise reproducible).
 * Synchronises the stream.  Returns LBM_E_NUMERIC (after filling sums and the
 * fields) when a non-finite value was found, or, with check_u_max set, when
 * sums[5] = max |u| exceeds LBM_U_MAX. */
int lbm_macroscopic(lbm_ctx *ctx, double *rho_dev, double *u_dev, double sums[8]);
/* The same for any lattice buffer of the context. */
int lbm_macroscopic_buf(lbm_ctx *ctx, const void *state, double *rho_dev, double *u_dev, double sums[8]);

/* lbm_macroscopic_buf for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the per-tile partial sums go to a library-owned device array
 * instead of the context's scratch buffer, so this call needs no scratch and
 * calls no hipMalloc, hipFree or allocating library routine.
 *   state, rho_dev, u_dev, sums   as for lbm_macroscopic_buf (state NULL =
 *                                 current lattice; rho_dev, u_dev may be NULL)
 * The array holds the partials of at most LBM_NOALLOC_MAX_TILES kept tiles
 * ((LBM_NOALLOC_MAX_TILES + 1) * 8 doubles, 16 MiB); it is part of the
 * library's device code, so every GPU the library runs on holds its own copy
 * until the process ends.  A context with more kept tiles gets LBM_E_RANGE
 * (use lbm_macroscopic_buf).  Results are bitwise those of
 * lbm_macroscopic_buf (same kernels, same reduction order), and the same
 * LBM_E_NUMERIC checks apply.  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (from other streams, host
 * threads or contexts) race and must be serialised by the caller.  The array
 * keeps the last call's partials; nothing in it has to start at zero, since
 * a call writes every entry it reads.  Synchronises the stream. */
#define LBM_NOALLOC_MAX_TILES 262144
int lbm_macroscopic_noalloc(lbm_ctx *ctx, const void *state, double *rho_dev, double *u_dev, double sums[8]);

/* Darcy permeability of the current lattice along x: k = nu * q / g_x with the
 * superficial flux q = sum rho u_x / (rho0 * nx*ny*nz).  Synchronises. */
int lbm_permeability(lbm_ctx *ctx, double g_x, double *k);

/* Dense FP64 copy of a lattice: f_dense_dev [19][nz][ny][nx] (device),
 * decoded from reduced storage; 0 at solid and dropped nodes.  state == NULL
 * means the current lattice. */
int lbm_get_state(lbm_ctx *ctx, const void *state, double *f_dense_dev);
/* Load a lattice from a dense FP64 array (encoded into the storage type;
 * solid slots are set to 0).  state == NULL means the current lattice. */
int lbm_set_state(lbm_ctx *ctx, const double *f_dense_dev, void *state);

/* A per-node field (force density or force gradient; see the conventions)
 * of FP64 (dtype 0) or FP32 (dtype 1) to a dense FP64 [3][nz][ny][nx] device
 * array (0 at solid and dropped nodes). */
int lbm_field_to_dense(lbm_ctx *ctx, const void *field_buf, int32_t dtype, double *dense_dev);

/* Tile-order buffer [n_tiles][ncomp][64] of FP64 (dtype 0) or FP32 (dtype 1)
 * to a dense FP64 [ncomp][nz][ny][nx] device array (0 outside kept tiles). */
int lbm_tiles_to_dense(lbm_ctx *ctx, const void *tile_buf, int32_t ncomp, int32_t dtype, double *dense_dev);

/* ------------------------------------------------------------------------
 * Discrete adjoint of the fused step (an addition: the paper has no adjoint;
 * the forward operator is the one of Alg. 2 with Eq. 2, 3, 5, 7 and Guo
 * forcing).  Every model (LBGK and LBMRT, quasi-compressible Eq. 3 and 5 or
 * incompressible Eq. 4 and 6); FP64 storage with FP64 arithmetic, or FP32
 * storage with FP32 arithmetic.  FP16 storage and open boundaries return
 * LBM_E_UNSUPPORTED; NULL buffers return LBM_E_INVAL.
 *
 * Forward: s_t = C(S s_{t-1}, F), S = pull streaming with bounce-back,
 * C = the model's local collision with Guo forcing.  Loss L = (1/N_fluid) sum_fluid u_x(s_T),
 * u_x from the stored lattice as lbm_macroscopic defines it for the model.
 * The adjoint lattices hold eta_t = J_t^T lambda_t (J_t = dC/dg at
 * g_t = S s_{t-1}, lambda_t = dL/ds_t); lambda_{t-1} = S^T eta_t is formed
 * on the fly by a reverse gather.  Gradients with respect to the body
 * acceleration g are accumulated in FP64 per-node-field order (one entry
 * per fluid node and component, see the conventions; lbm_field_to_dense).
 * The backward sweep is:
 *     lbm_adjoint_seed(s_{T-1})                      -> eta_T,  gF  = ...
 *     lbm_adjoint_step(s_{t-2}, eta_t) for t=T..2   -> eta_{t-1}, gF += ...
 *     lbm_adjoint_final(eta_1)                        -> lambda_0 = dL/ds_0
 * An adjoint lattice (adjoint_bytes, caller-owned device memory) has the
 * layout and element type of the state but holds unshifted values: the
 * shift of reduced storage is a constant, so dL/dd = dL/df.  Forward states
 * are the context's own lattices or buffers of state_bytes.  All calls are
 * asynchronous on the context's stream.
 * ------------------------------------------------------------------------ */
/* Seed: from the forward state s_{T-1}, write eta_T and OVERWRITE
 * grad_g_tile (grad_force_bytes, FP64, device) with the step-T contribution
 * plus the direct dL/dg. */
int lbm_adjoint_seed(lbm_ctx *ctx, const void *s_Tm1, void *eta_T, double *grad_g_tile);
/* One reverse step: from eta_t and the forward state s_{t-2}, write eta_{t-1}
 * (eta_t != eta_tm1, else LBM_E_INVAL) and ADD the step's contribution to
 * grad_g_tile. */
int lbm_adjoint_step(lbm_ctx *ctx, const void *s_tm2, const void *eta_t, void *eta_tm1, double *grad_g_tile);
/* Final reverse gather: lambda_0 = S^T eta_1 = dL/ds_0 into another adjoint
 * lattice (eta_1 != lambda_0). */
int lbm_adjoint_final(lbm_ctx *ctx, const void *eta_1, void *lambda_0);
/* Dense FP64 copy [19][nz][ny][nx] (device) of an adjoint lattice, and the
 * reverse; 0 at solid and dropped nodes / solid slots set to 0. */
int lbm_adjoint_get(lbm_ctx *ctx, const void *adj, double *dense_dev);
int lbm_adjoint_set(lbm_ctx *ctx, const double *dense_dev, void *adj);

/* ------------------------------------------------------------------------
 * Measurement kernels (the paper's "read/write only" and "propagation only"
 * kernels, Section 4.1): same tiles and launch shape as a step, kind 1 reads
 * and writes each node's own 19 values, kind 2 performs the full gather and
 * bounce-back and stores the gathered values without collision.
 * Kinds 3-6 are the propagation-only kernel of the paper's intra-tile layout
 * study (Section 3.3, Eqs. 11-13, Table 5): each direction's 64-slot block
 * orders the tile's nodes by the XYZ map (x + 4y + 16z), the YXZ map
 * (y + 4x + 16z) or the zigzagNE map; kind 3 uses XYZ for every direction,
 * kind 4 adds zigzagNE for NE and SE, kind 5 YXZ for E, W, ET, EB, NW, SW,
 * WT and WB, kind 6 both.  Kind 7 (not the paper's) is a face-major order for
 * 128-byte lines: y + 4z + 16x for E and W, x + 4z + 16y for N, S, NE, NW,
 * SW and SE, XYZ for the rest, so that each face a neighbour reads is one
 * contiguous run.  src and dst are read and written in that layout
 * (not the library's state layout, except for kind 3, whose bytes equal it).
 * Kinds 3-7 need every kept tile entirely fluid (else LBM_E_UNSUPPORTED), where
 * the layouts occupy the same bytes as a state lattice.
 * src != dst, both state lattices of this context (else LBM_E_INVAL).
 * ------------------------------------------------------------------------ */
int lbm_calib_step(lbm_ctx *ctx, int32_t kind, const void *src, void *dst);

/* Bandwidth probes: plain streaming kernels that measure what the GPU
 * sustains, the practical ceiling read beside the nominal HBM peak (the
 * paper sets its GPU's measured copy bandwidth beside the peak, Section 4.1).
 *   kind 1 read only: reads `bytes` of src; dst receives at most 4 bytes,
 *          and only when the data hash to one fixed value (which keeps the
 *          loads), so it needs 16 writable bytes
 *   kind 2 write only: writes zeros over `bytes` of dst; src may be NULL
 *   kind 3 copy: dst = src over `bytes`; the ranges must not overlap
 * 16-byte non-temporal loads and stores, four in flight per thread, grid-stride
 * over the buffer with `blocks` workgroups (1 .. 2^20) of `threads` threads
 * (64, 128, 256, 512 or 1024).  bytes must be a positive multiple of 16 and
 * both buffers 16-byte aligned (else LBM_E_INVAL).  Needs no context;
 * asynchronous on hip_stream (NULL = the default stream). */
int lbm_stream_probe(void *hip_stream, int32_t kind, const void *src, void *dst, size_t bytes, int32_t blocks,
                     int32_t threads);

/* Counts of the current context (any pointer may be NULL). */
int lbm_info(lbm_ctx *ctx, int32_t *n_tiles, int64_t *n_fluid, int32_t *storage, int32_t *grid_blocks);

const char *lbm_last_error(void);
const char *lbm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TILED_LBM_H */
