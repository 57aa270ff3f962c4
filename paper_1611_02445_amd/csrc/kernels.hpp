// Host-side launch interface of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace tlbm {

// physics and storage parameters of a launch
struct Phys {
    int storage;       // lbm_storage
    int model;         // lbm_model
    double omega;      // 1/tau
    double kg;         // 1 - 1/(2 tau), Guo source prefactor
    double rho0;       // reference density (force density F = rho0 g)
    double rho_base;   // shift of the stored values: 0 for FP64, rho0 for reduced storage
    double F[3];       // uniform force density (used when field == nullptr)
    const void *field; // per-node force density of the arithmetic type (per fluid slot), or null
    float scale;       // FP16: 2^k; 1 otherwise
    float inv_scale;
    double inv_nfluid; // 1 / N_fluid (adjoint loss normalisation)
    int f16_stochastic;       // FP16 stores with stochastic rounding
    uint32_t launch_counter;  // step launches so far (seeds the rounding bits)
    const uint64_t *bc;       // open boundaries: [n_tiles][9] node mask + 64 node codes, or null
    double bc_u[3];           // velocity of the velocity nodes
    double bc_rho;            // density of the pressure nodes
};

struct Launch {
    hipStream_t stream;
    int n_tiles;
    int tpw;          // tiles (waves) per workgroup
    int grid;         // workgroups
    DevTables tb;
    bool off32;       // every lattice byte offset fits in 32 bits
};

hipError_t launch_step(const Launch &L, const Phys &P, const void *src, void *dst);
hipError_t launch_calib(const Launch &L, int kind, int storage, const void *src, void *dst);
hipError_t launch_init(const Launch &L, const Phys &P, void *a, void *b, double ux, double uy, double uz);
hipError_t launch_fill(hipStream_t s, double *p, size_t n);
hipError_t launch_macro(const Launch &L, const Phys &P, const void *state, double *rho, double *u, int nx, int ny,
                        int nz, double *partials);
hipError_t launch_reduce(hipStream_t s, const double *partials, int n_tiles, double *out);
hipError_t launch_get_state(const Launch &L, const Phys &P, const void *state, double *dense, int nx, int ny, int nz);
hipError_t launch_set_state(const Launch &L, const Phys &P, const double *dense, void *state, int nx, int ny, int nz);
hipError_t launch_force_to_tiles(const Launch &L, const Phys &P, const double *g_dense, void *tile_buf, int nx,
                                 int ny, int nz);
hipError_t launch_field_to_dense(const Launch &L, const void *field, int dtype, double *dense, int nx, int ny,
                                 int nz);
hipError_t launch_tiles_to_dense(const Launch &L, const void *tile_buf, int ncomp, int dtype, double *dense, int nx,
                                 int ny, int nz);
hipError_t launch_adjoint_seed(const Launch &L, const Phys &P, const void *s_prev, void *eta, double *grad);
hipError_t launch_adjoint_step(const Launch &L, const Phys &P, const void *s_prev2, const void *eta_in,
                               void *eta_out, double *grad);
hipError_t launch_probe(hipStream_t s, int kind, const void *src, void *dst, size_t bytes, int blocks, int threads);
hipError_t launch_adjoint_final(const Launch &L, const Phys &P, const void *eta_in, void *lambda_out);

}  // namespace tlbm
