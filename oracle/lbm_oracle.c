/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, dense FP64 reference of the D3Q19 lattice-Boltzmann scheme
 * that the tiled GPU path computes.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library; the product
 * path never calls it.  It shares no source, header or table with the GPU
 * library: the lattice table below is typed in here from the paper's
 * description of D3Q19 (Section 2.2, Fig. 1 caption and the weights listed
 * after Eq. 4).
 *
 * What is computed (all on a dense box, node index x + nx*(y + ny*z),
 * distributions stored as f[i][node]):
 *
 *   - streaming in pull form (Sections 2.3 and 3.4: every node gathers f_i
 *     from the node it came from; Alg. 2), with halfway bounce-back at solid or
 *     missing neighbours (Section 3.4: no propagation from or to solid nodes;
 *     Section 2.2: walls are bounce-back),
 *   - LBGK collision (Eq. 2 and Eq. 7) with the quasi-compressible equilibrium
 *     (Eq. 3) and velocity (Eq. 5), or the incompressible pair (Eq. 4, Eq. 6),
 *   - a body force.  The paper drives its flows by boundaries only, so the
 *     forcing is our reading: Guo, Zheng and Shi (2002) -- velocity shifted by
 *     F/2 and a second-order source term.
 *   - a discrete adjoint (reverse mode) of T steps for the loss
 *     "mean x-velocity over fluid nodes", storing every state, for every
 *     collision model,
 *   - the multiple-relaxation-time operator the paper names for its LBMRT
 *     kernels (Section 2.2; no matrix given): the D3Q19 moment basis and
 *     relaxation rates of d'Humieres et al. (2002), both equilibria,
 *   - the Zou-He velocity inlet and constant-pressure outlet the paper
 *     names for its open boundaries (Section 2.2), on faces normal to any
 *     axis.
 *
 * Parity unpinned: the rates of the moments eps and pi (1.4, 1.4).  They
 * act below the Navier-Stokes level on moments that are even in every
 * velocity component a plane or sound-wave test excites, so no transport
 * coefficient or closed form fixes them; they are the cited paper's values.
 * The shear rate (1/tau), the energy rate (1.19, through the bulk
 * viscosity) and the q and m rates (1.2, 1.98, through the wall slip of
 * halfway bounce-back in plane Poiseuille flow) are pinned.
 *
 * Arithmetic is plain C in double precision with the operations written in
 * the order of the formulas; build without FMA contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* threads the OpenMP loops use (1 without OpenMP) */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* D3Q19 velocities.  0 = rest; 1..6 axis directions E N W S T B (e_3 = W =
 * (-1,0,0) as the Fig. 1 caption fixes); 7..18 the twelve edge directions. */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0},
    {1, 0, 1}, {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1},
    {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};

/* weights: 1/3 rest, 1/18 axis, 1/36 edge (the list after Eq. 4) */
static double WT(int i) {
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* opposite direction: the one whose velocity is -c_i (found by search, not a
 * typed-in table) */
static int OPP(int i) {
    for (int j = 0; j < Q; ++j)
        if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2])
            return j;
    return -1;
}

/* ------------------------------------------------------------------ */
/* lattice export (for invariant tests)                                */
/* ------------------------------------------------------------------ */
void oracle_lattice(int32_t *c /*[19][3]*/, double *w /*[19]*/, int32_t *opp /*[19]*/) {
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = CV[i][a];
        w[i] = WT(i);
        opp[i] = OPP(i);
    }
}

/* ------------------------------------------------------------------ */
/* local pieces: equilibrium, forcing term, collision                  */
/* ------------------------------------------------------------------ */

/* Models: bit 0 selects the equilibrium and velocity (0 quasi-compressible,
 * Eq. 3 and 5; 1 incompressible, Eq. 4 and 6), bit 1 the collision operator
 * (0 single relaxation time, Eq. 2 and 7; 1 multiple relaxation times). */
static int incompressible(int model) { return model & 1; }
static int multi_relaxation(int model) { return (model >> 1) & 1; }

/* Eq. 3 (quasi-compressible) or Eq. 4 (incompressible),
 * c_s^2 = 1/3 so 1/c_s^2 = 3, 1/(2 c_s^4) = 4.5, 1/(2 c_s^2) = 1.5 */
static double feq_i(int model, int i, double rho, const double u[3]) {
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
    if (!incompressible(model)) return WT(i) * rho * (1.0 + poly);
    return WT(i) * (rho + poly);
}

/* Guo forcing source: (1 - 1/(2 tau)) w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)] */
static double guo_i(int i, double tau, const double u[3], const double F[3]) {
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    double cF = CV[i][0] * F[0] + CV[i][1] * F[1] + CV[i][2] * F[2];
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    return (1.0 - 1.0 / (2.0 * tau)) * WT(i) * (3.0 * (cF - uF) + 9.0 * cu * cF);
}

/* density and velocity of the gathered (pre-collision) values:
 * rho = sum f; u = (sum c f + F/2) / rho  (Eq. 5 with Guo's half-force shift),
 * incompressible: u = sum c f + F/2 (Eq. 6) */
static void moments(int model, const double fin[Q], const double F[3], double *rho, double u[3]) {
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        r += fin[i];
        for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * fin[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = !incompressible(model) ? (j[a] + 0.5 * F[a]) / r : (j[a] + 0.5 * F[a]);
}

/* ------------------------------------------------------------------ */
/* multiple relaxation times (the LBMRT kernels of Sections 2.2 and    */
/* 4.6; the paper names the operator but gives no matrix): the D3Q19   */
/* moment basis of d'Humieres, Ginzburg, Krafczyk, Lallemand and Luo    */
/* (2002), each moment a polynomial in the velocity c:                  */
/*   rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww,    */
/*   pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z                             */
/* ------------------------------------------------------------------ */
static double mrt_row(int k, int i) {
    const double cx = CV[i][0], cy = CV[i][1], cz = CV[i][2];
    const double c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return cx;
    case 4: return (5.0 * c2 - 9.0) * cx;
    case 5: return cy;
    case 6: return (5.0 * c2 - 9.0) * cy;
    case 7: return cz;
    case 8: return (5.0 * c2 - 9.0) * cz;
    case 9: return 3.0 * cx * cx - c2;
    case 10: return (3.0 * cx * cx - c2) * (3.0 * c2 - 5.0);
    case 11: return cy * cy - cz * cz;
    case 12: return (cy * cy - cz * cz) * (3.0 * c2 - 5.0);
    case 13: return cx * cy;
    case 14: return cy * cz;
    case 15: return cx * cz;
    case 16: return (cy * cy - cz * cz) * cx;
    case 17: return (cz * cz - cx * cx) * cy;
    default: return (cx * cx - cy * cy) * cz;
    }
}

/* relaxation rates of the same paper; the viscous moments relax at 1/tau
 * (so nu = (tau - 1/2)/3 as for the single-time operator); the rates of the
 * conserved moments (rho, j) do not enter */
static const double GHOST_DEFAULT[5] = {1.19, 1.4, 1.2, 1.4, 1.98};
static double GHOST[5] = {1.19, 1.4, 1.2, 1.4, 1.98}; /* e, eps, q, pi, m */
static void mrt_rates(double tau, double s[Q]) {
    const double sv = 1.0 / tau;
    const double e = GHOST[0], ep = GHOST[1], q = GHOST[2], pi = GHOST[3], m = GHOST[4];
    const double r[Q] = {0.0, e, ep, 0.0, q, 0.0, q, 0.0, q, sv, pi, sv, pi, sv, sv, sv, m, m, m};
    for (int k = 0; k < Q; ++k) s[k] = r[k];
}

/* Test hook: the rates of the e, eps, q, pi and m moments used by every
 * later step and adjoint of the multiple-relaxation-time operator (NULL
 * restores the table above).  Lets the tests check closed forms that depend
 * on these rates at more than one value; not thread-safe against a running
 * step. */
void oracle_set_mrt_ghost_rates(const double *r /*[5] or NULL*/) {
    for (int k = 0; k < 5; ++k) GHOST[k] = r ? r[k] : GHOST_DEFAULT[k];
}

/* M (rows k, columns i) and its inverse by Gauss-Jordan elimination, built
 * once when the library is loaded (before any threaded loop can use them) */
static double MRT_M[Q][Q], MRT_MINV[Q][Q];
__attribute__((constructor)) static void mrt_init(void) {
    double a[Q][2 * Q];
    for (int k = 0; k < Q; ++k)
        for (int i = 0; i < Q; ++i) {
            MRT_M[k][i] = mrt_row(k, i);
            a[k][i] = MRT_M[k][i];
            a[k][Q + i] = (k == i) ? 1.0 : 0.0;
        }
    for (int col = 0; col < Q; ++col) {
        int piv = col;
        for (int r = col + 1; r < Q; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        for (int c = 0; c < 2 * Q; ++c) {
            double t = a[col][c];
            a[col][c] = a[piv][c];
            a[piv][c] = t;
        }
        const double p = a[col][col];
        for (int c = 0; c < 2 * Q; ++c) a[col][c] /= p;
        for (int r = 0; r < Q; ++r) {
            if (r == col) continue;
            const double m = a[r][col];
            if (m != 0.0)
                for (int c = 0; c < 2 * Q; ++c) a[r][c] -= m * a[col][c];
        }
    }
    for (int i = 0; i < Q; ++i)
        for (int k = 0; k < Q; ++k) MRT_MINV[i][k] = a[i][Q + k];
}

/* Guo source without its (1 - 1/(2 tau)) factor: w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)] */
static double guo_raw_i(int i, const double u[3], const double F[3]) {
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    double cF = CV[i][0] * F[0] + CV[i][1] * F[1] + CV[i][2] * F[2];
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    return WT(i) * (3.0 * (cF - uF) + 9.0 * cu * cF);
}

/* m = M f, m_eq = M f_eq, m* = m - S (m - m_eq) + (I - S/2) M Fbar,
 * f* = M^-1 m*  (Guo forcing carried into moment space) */
static void collide_mrt_rates(int model, const double fin[Q], const double F[3], const double s[Q], double fout[Q]) {
    double rho, u[3], fe[Q], fb[Q], m[Q], meq[Q], mf[Q], ms[Q];
    moments(model, fin, F, &rho, u);
    for (int i = 0; i < Q; ++i) {
        fe[i] = feq_i(model, i, rho, u);
        fb[i] = guo_raw_i(i, u, F);
    }
    for (int k = 0; k < Q; ++k) {
        m[k] = meq[k] = mf[k] = 0.0;
        for (int i = 0; i < Q; ++i) {
            m[k] += MRT_M[k][i] * fin[i];
            meq[k] += MRT_M[k][i] * fe[i];
            mf[k] += MRT_M[k][i] * fb[i];
        }
        ms[k] = m[k] - s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * s[k]) * mf[k];
    }
    for (int i = 0; i < Q; ++i) {
        fout[i] = 0.0;
        for (int k = 0; k < Q; ++k) fout[i] += MRT_MINV[i][k] * ms[k];
    }
}

/* Eq. 7 with the source: f*_i = f_i - (f_i - feq_i)/tau + S_i, or the
 * multiple-relaxation-time operator */
static void collide(int model, const double fin[Q], const double F[3], double tau, double fout[Q]) {
    if (multi_relaxation(model)) {
        double s[Q];
        mrt_rates(tau, s);
        collide_mrt_rates(model, fin, F, s, fout);
        return;
    }
    double rho, u[3];
    moments(model, fin, F, &rho, u);
    for (int i = 0; i < Q; ++i)
        fout[i] = fin[i] - (fin[i] - feq_i(model, i, rho, u)) / tau + guo_i(i, tau, u, F);
}

/* exports for the tests: the moment matrix, its inverse, the rates, and the
 * operator with caller-given rates */
void oracle_mrt_matrix(double *M /*[19][19]*/, double *Minv /*[19][19]*/) {
    for (int k = 0; k < Q; ++k)
        for (int i = 0; i < Q; ++i) {
            M[k * Q + i] = MRT_M[k][i];
            Minv[k * Q + i] = MRT_MINV[k][i];
        }
}

void oracle_mrt_rates(double tau, double *s /*[19]*/) { mrt_rates(tau, s); }

void oracle_collide_mrt_rates(int32_t model, const double *fin, const double *F, const double *s, double *fout) {
    collide_mrt_rates(model, fin, F, s, fout);
}

void oracle_feq(int32_t model, double rho, const double *u, double *feq /*[19]*/) {
    for (int i = 0; i < Q; ++i) feq[i] = feq_i(model, i, rho, u);
}

void oracle_guo(double tau, const double *u, const double *F, double *S /*[19]*/) {
    for (int i = 0; i < Q; ++i) S[i] = guo_i(i, tau, u, F);
}

void oracle_collide_node(int32_t model, const double *fin, const double *F, double tau, double *fout) {
    collide(model, fin, F, tau, fout);
}

/* ------------------------------------------------------------------ */
/* geometry helpers                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    int nx, ny, nz, periodic; /* periodic: bit0 x, bit1 y, bit2 z */
    const uint8_t *solid;     /* 1 = solid */
} box_t;

/* node index of (x,y,z) displaced by d; -1 when it leaves the box along a
 * non-periodic axis.  Periodic axes wrap modulo the box size. */
static long shifted(const box_t *b, int x, int y, int z, int dx, int dy, int dz) {
    int p[3] = {x + dx, y + dy, z + dz};
    int n[3] = {b->nx, b->ny, b->nz};
    for (int a = 0; a < 3; ++a) {
        if (p[a] < 0 || p[a] >= n[a]) {
            if (!(b->periodic >> a & 1)) return -1;
            p[a] = ((p[a] % n[a]) + n[a]) % n[a];
        }
    }
    return (long)p[0] + (long)b->nx * ((long)p[1] + (long)b->ny * (long)p[2]);
}

static int is_fluid(const box_t *b, long idx) { return idx >= 0 && !b->solid[idx]; }

static void force_at(const double *field, long N, long idx, double fx, double fy, double fz, double F[3]) {
    if (field) {
        F[0] = field[idx];
        F[1] = field[N + idx];
        F[2] = field[2 * N + idx];
    } else {
        F[0] = fx;
        F[1] = fy;
        F[2] = fz;
    }
}

/* pull with halfway bounce-back for one fluid node:
 * fin_i(x) = s_i(x - c_i) if x - c_i is fluid, otherwise s_opp(i)(x) */
static void gather(const box_t *b, const double *s, long N, int x, int y, int z, double fin[Q]) {
    long self = (long)x + (long)b->nx * ((long)y + (long)b->ny * (long)z);
    for (int i = 0; i < Q; ++i) {
        long src = shifted(b, x, y, z, -CV[i][0], -CV[i][1], -CV[i][2]);
        if (is_fluid(b, src))
            fin[i] = s[(long)i * N + src];
        else
            fin[i] = s[(long)OPP(i) * N + self];
    }
}

/* ------------------------------------------------------------------ */
/* open boundaries (the paper's Zou-He velocity inlet and constant-     */
/* pressure outlet, Section 2.2) on faces normal to an axis: after the   */
/* gather, the populations that enter through the face are rebuilt so    */
/* that the node has the prescribed velocity (velocity node) or density  */
/* (pressure node).                                                       */
/* Code c = 1..12: axis a = (c-1)/4 (x, y, z); r = (c-1)%4 gives the kind */
/* and the sign n = c_a of the unknown populations:                       */
/*   r = 0 velocity, n = +1 (the domain lies at +a: an inlet on the low   */
/*         face); r = 1 pressure, n = -1 (an outlet on the high face);    */
/*   r = 2 velocity, n = -1;  r = 3 pressure, n = +1.                     */
/* Codes 1 and 2 are the x inlet and x outlet.                            */
/* With a body force the rebuilt momentum is J = rho u - F/2, so that    */
/* the collision's velocity (J + F/2)/rho is the prescribed one; a        */
/* pressure node's tangential velocity is 0.                              */
/* Unknown i (c_ia = n) from its opposite, Zou and He's bounce-back of   */
/* the non-equilibrium part with the tangential-momentum correction of   */
/* Hecht and Harting (2010):                                              */
/*   f_i = f_opp(i) + 6 w_i (c_i . J) - sum_{t != a} c_it N_t,           */
/*   N_t = 1/2 sum_{c_a = 0} c_t f - J_t / 3                             */
/* ------------------------------------------------------------------ */
typedef struct {
    const uint8_t *type; /* [N] 0 none, else a code 1..12; NULL = no open boundaries */
    double u[3];         /* velocity of the velocity nodes */
    double rho_out;      /* density of the pressure nodes */
} bc_t;

static void zou_he(int code, int model, const double u_in[3], double rho_out, const double F[3], double f[Q]) {
    const int a = (code - 1) / 4, r = (code - 1) % 4;
    const int velocity = (r == 0 || r == 2);
    const int n = (r == 0 || r == 3) ? 1 : -1; /* c_a of the unknown populations */
    double s_tan = 0.0, s_known = 0.0, t[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        if (CV[i][a] == 0) {
            s_tan += f[i];
            for (int b = 0; b < 3; ++b) t[b] += CV[i][b] * f[i];
        } else if (CV[i][a] == -n) {
            s_known += f[i]; /* the populations leaving through the face */
        }
    }
    double J[3];
    if (velocity) {
        if (!incompressible(model)) {
            const double rho = (s_tan + 2.0 * s_known - 0.5 * n * F[a]) / (1.0 - n * u_in[a]);
            for (int b = 0; b < 3; ++b) J[b] = rho * u_in[b] - 0.5 * F[b];
        } else {
            for (int b = 0; b < 3; ++b) J[b] = u_in[b] - 0.5 * F[b];
        }
    } else {
        /* sum f = rho_out and sum c_a f = J_a fix the normal momentum */
        for (int b = 0; b < 3; ++b) J[b] = -0.5 * F[b];
        J[a] = n * (rho_out - s_tan - 2.0 * s_known);
    }
    double N[3];
    for (int b = 0; b < 3; ++b) N[b] = (b == a) ? 0.0 : 0.5 * t[b] - J[b] / 3.0;
    for (int i = 0; i < Q; ++i) {
        if (CV[i][a] != n) continue;
        const double cJ = CV[i][0] * J[0] + CV[i][1] * J[1] + CV[i][2] * J[2];
        f[i] = f[OPP(i)] + 6.0 * WT(i) * cJ - CV[i][0] * N[0] - CV[i][1] * N[1] - CV[i][2] * N[2];
    }
}

/* exported for the tests: the rebuilt populations of one node */
void oracle_zou_he(int32_t type, int32_t model, const double *u_in, double rho_out, const double *F, double *f) {
    zou_he(type, model, u_in, rho_out, F, f);
}

/* ------------------------------------------------------------------ */
/* initial state, one step, macroscopic fields                         */
/* ------------------------------------------------------------------ */

/* f_i = feq_i(rho0, u0) at fluid nodes, 0 at solid nodes */
void oracle_init(double *f, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz, int32_t model,
                 double rho0, double ux, double uy, double uz) {
    long N = (long)nx * ny * nz;
    double u[3] = {ux, uy, uz};
    for (int i = 0; i < Q; ++i) {
        double v = feq_i(model, i, rho0, u);
        for (long n = 0; n < N; ++n) f[(long)i * N + n] = solid[n] ? 0.0 : v;
    }
}

/* one time step: fb = C(S fa), with open boundaries when bc->type is set.
 * Solid nodes are neither read (bounce-back replaces the read) nor written.
 * force: NULL for the uniform (fx,fy,fz), otherwise a per-node field [3][N]. */
static void step_bc(const double *fa, double *fb, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz,
                    int32_t periodic, int32_t model, double tau, const double *force, double fx, double fy,
                    double fz, const bc_t *bc) {
    box_t b = {nx, ny, nz, periodic, solid};
    long N = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long idx = (long)x + (long)nx * ((long)y + (long)ny * (long)z);
                if (solid[idx]) continue;
                double fin[Q], fout[Q], F[3];
                gather(&b, fa, N, x, y, z, fin);
                force_at(force, N, idx, fx, fy, fz, F);
                if (bc && bc->type && bc->type[idx]) zou_he(bc->type[idx], model, bc->u, bc->rho_out, F, fin);
                collide(model, fin, F, tau, fout);
                for (int i = 0; i < Q; ++i) fb[(long)i * N + idx] = fout[i];
            }
}

void oracle_step(const double *fa, double *fb, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz,
                 int32_t periodic, int32_t model, double tau, const double *force, double fx, double fy,
                 double fz) {
    step_bc(fa, fb, solid, nx, ny, nz, periodic, model, tau, force, fx, fy, fz, NULL);
}

/* n steps with open boundaries (type [N]: 0 none, 1 velocity inlet, 2 pressure outlet) */
void oracle_run_bc(double *f, double *scratch, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz,
                   int32_t periodic, int32_t model, double tau, const double *force, double fx, double fy,
                   double fz, int32_t nsteps, const uint8_t *type, const double *u_in, double rho_out) {
    bc_t bc = {type, {u_in[0], u_in[1], u_in[2]}, rho_out};
    long N = (long)nx * ny * nz;
    double *a = f, *b = scratch;
    for (int s = 0; s < nsteps; ++s) {
        step_bc(a, b, solid, nx, ny, nz, periodic, model, tau, force, fx, fy, fz, &bc);
        double *t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * (size_t)Q * (size_t)N);
}

/* n steps, ping-ponging between f (in/out) and a scratch array of the same size */
void oracle_run(double *f, double *scratch, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz,
                int32_t periodic, int32_t model, double tau, const double *force, double fx, double fy,
                double fz, int32_t nsteps) {
    long N = (long)nx * ny * nz;
    double *a = f, *b = scratch;
    for (int s = 0; s < nsteps; ++s) {
        oracle_step(a, b, solid, nx, ny, nz, periodic, model, tau, force, fx, fy, fz);
        double *t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * (size_t)Q * (size_t)N);
}

/* update only the listed nodes (one step from fa), out[k][19]; used to check a
 * large GPU run node by node.  A listed solid node yields zeros. */
void oracle_step_nodes(const double *fa, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz,
                       int32_t periodic, int32_t model, double tau, const double *force, double fx, double fy,
                       double fz, const int64_t *nodes, int64_t count, double *out) {
    box_t b = {nx, ny, nz, periodic, solid};
    long N = (long)nx * ny * nz;
    for (int64_t k = 0; k < count; ++k) {
        long idx = nodes[k];
        double *o = out + k * Q;
        if (solid[idx]) {
            for (int i = 0; i < Q; ++i) o[i] = 0.0;
            continue;
        }
        int x = (int)(idx % nx), y = (int)((idx / nx) % ny), z = (int)(idx / ((long)nx * ny));
        double fin[Q], F[3];
        gather(&b, fa, N, x, y, z, fin);
        force_at(force, N, idx, fx, fy, fz, F);
        collide(model, fin, F, tau, o);
    }
}

/* density and velocity from a stored post-collision state:
 * rho = sum f*, u = (sum c f* - F/2)/rho (the velocity the collision used);
 * incompressible: u = sum c f* - F/2.  Zero at solid nodes. */
void oracle_macroscopic(const double *f, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz, int32_t model,
                        const double *force, double fx, double fy, double fz, double *rho, double *u) {
    long N = (long)nx * ny * nz;
    for (long n = 0; n < N; ++n) {
        if (solid[n]) {
            rho[n] = 0.0;
            u[n] = u[N + n] = u[2 * N + n] = 0.0;
            continue;
        }
        double r = 0.0, j[3] = {0.0, 0.0, 0.0}, F[3];
        for (int i = 0; i < Q; ++i) {
            double v = f[(long)i * N + n];
            r += v;
            for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * v;
        }
        force_at(force, N, n, fx, fy, fz, F);
        rho[n] = r;
        for (int a = 0; a < 3; ++a)
            u[(long)a * N + n] = !incompressible(model) ? (j[a] - 0.5 * F[a]) / r : (j[a] - 0.5 * F[a]);
    }
}

/* ------------------------------------------------------------------ */
/* discrete adjoint                                                    */
/* ------------------------------------------------------------------ */
/* The forward map is s_t = C(S s_{t-1}, F): S the pull with bounce-back,
 * C the local collision.  For a scalar loss L(s_T, F):
 *     lambda_T      = dL/ds_T
 *     eta_t         = J_t^T lambda_t,   J_t = dC/dg at g_t = S s_{t-1}
 *     dL/dF        += (dC/dF)^T lambda_t
 *     lambda_{t-1}  = S^T eta_t
 * and dL/ds_0 = lambda_0.  Provided for every model: the single-relaxation-
 * time ones (quasi-compressible, Eq. 3 and 5; incompressible, Eq. 4 and 6)
 * and the multiple-relaxation-time operator with either equilibrium. */

/* S as an operator on a whole field: g = S s (solid nodes of g set to 0) */
void oracle_pull(const double *s, double *g, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz,
                 int32_t periodic) {
    box_t b = {nx, ny, nz, periodic, solid};
    long N = (long)nx * ny * nz;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long idx = (long)x + (long)nx * ((long)y + (long)ny * (long)z);
                double fin[Q];
                if (solid[idx]) {
                    for (int i = 0; i < Q; ++i) g[(long)i * N + idx] = 0.0;
                    continue;
                }
                gather(&b, s, N, x, y, z, fin);
                for (int i = 0; i < Q; ++i) g[(long)i * N + idx] = fin[i];
            }
}

/* S^T: every slot s_j(y) that S copies somewhere collects what was sent there.
 * Written as a scatter that follows S read by read, so that it is the
 * transpose by construction: for each fluid x and each i, the value mu_i(x)
 * is added back to the slot S read it from. */
void oracle_pull_transpose(const double *mu, double *out, const uint8_t *solid, int32_t nx, int32_t ny,
                           int32_t nz, int32_t periodic) {
    box_t b = {nx, ny, nz, periodic, solid};
    long N = (long)nx * ny * nz;
    memset(out, 0, sizeof(double) * (size_t)Q * (size_t)N);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long idx = (long)x + (long)nx * ((long)y + (long)ny * (long)z);
                if (solid[idx]) continue;
                for (int i = 0; i < Q; ++i) {
                    long src = shifted(&b, x, y, z, -CV[i][0], -CV[i][1], -CV[i][2]);
                    if (is_fluid(&b, src))
                        out[(long)i * N + src] += mu[(long)i * N + idx];
                    else
                        out[(long)OPP(i) * N + idx] += mu[(long)i * N + idx];
                }
            }
}

/* derivatives of the single-relaxation-time collision at one node (model 0
 * quasi-compressible, 1 incompressible).
 * Returns (J^T lam)_j in eta[19] and (dC/dF)^T lam in gF[3].
 *   dC_i/dg_j = (1 - 1/tau) delta_ij + (1/tau) dfeq_i/dg_j + dS_i/dg_j
 *   dfeq_i/dg_j = dfeq_i/drho + dfeq_i/du . du/dg_j
 * quasi-compressible (Eq. 3, u = (j + F/2)/rho, Eq. 5):
 *   du/dg_j = (c_j - u)/rho,  du/dF = I/(2 rho)
 *   dfeq_i/drho = w_i (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
 *   dfeq_i/du   = w_i rho (3 c_i + 9 (c_i.u) c_i - 3 u)
 * incompressible (Eq. 4, u = j + F/2, Eq. 6):
 *   du/dg_j = c_j,  du/dF = I/2
 *   dfeq_i/drho = w_i
 *   dfeq_i/du   = w_i (3 c_i + 9 (c_i.u) c_i - 3 u)
 * both:
 *   dS_i/du     = (1 - 1/(2tau)) w_i (9 (c_i.F) c_i - 3 F)
 *   dS_i/dF|_u  = (1 - 1/(2tau)) w_i (3 (c_i - u) + 9 (c_i.u) c_i) */
/* the same for the multiple-relaxation-time operator (models 2 and 3):
 *   f* = f - R (f - feq) + (I - R/2) G,   R = M^-1 S M,
 *   G_i = w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)]  (the raw Guo source)
 * so with mu = R^T lam and nu = (I - R/2)^T lam
 *   (J^T lam)_j = lam_j - mu_j + sum_i mu_i dfeq_i/dg_j + sum_i nu_i dG_i/dg_j
 *   (dC/dF)^T lam = sum_i mu_i dfeq_i/du du/dF + sum_i nu_i (dG_i/dF|_u + dG_i/du du/dF)
 * with dG_i/du = w_i (9 (c_i.F) c_i - 3 F), dG_i/dF|_u = w_i (3 (c_i - u) + 9 (c_i.u) c_i)
 * and feq, u of the model's equilibrium (Eq. 3, 5 or Eq. 4, 6). */
static void collide_jt_mrt(int model, const double *fin, const double *F, double tau, const double *lam,
                           double *eta, double *gF) {
    const int inc = incompressible(model);
    double s[Q], R[Q][Q], mu[Q], nu[Q], rho, u[3];
    mrt_rates(tau, s);
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) {
            R[i][j] = 0.0;
            for (int k = 0; k < Q; ++k) R[i][j] += MRT_MINV[i][k] * s[k] * MRT_M[k][j];
        }
    for (int j = 0; j < Q; ++j) {
        mu[j] = 0.0;
        for (int i = 0; i < Q; ++i) mu[j] += R[i][j] * lam[i];
        nu[j] = lam[j] - 0.5 * mu[j];
    }
    moments(model, fin, F, &rho, u);
    double A = 0.0, V[3] = {0.0, 0.0, 0.0}, D[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        double c[3] = {(double)CV[i][0], (double)CV[i][1], (double)CV[i][2]};
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        double cF = c[0] * F[0] + c[1] * F[1] + c[2] * F[2];
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        A += mu[i] * (inc ? WT(i) : WT(i) * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        for (int a = 0; a < 3; ++a) {
            double dfeq_du = WT(i) * (inc ? 1.0 : rho) * (3.0 * c[a] + 9.0 * cu * c[a] - 3.0 * u[a]);
            double dG_du = WT(i) * (9.0 * cF * c[a] - 3.0 * F[a]);
            V[a] += mu[i] * dfeq_du + nu[i] * dG_du;
            D[a] += nu[i] * WT(i) * (3.0 * (c[a] - u[a]) + 9.0 * cu * c[a]);
        }
    }
    for (int j = 0; j < Q; ++j) {
        double cj_u = 0.0;
        for (int a = 0; a < 3; ++a) cj_u += V[a] * (inc ? CV[j][a] : (CV[j][a] - u[a]) / rho);
        eta[j] = lam[j] - mu[j] + A + cj_u;
    }
    for (int a = 0; a < 3; ++a) gF[a] = V[a] / (inc ? 2.0 : 2.0 * rho) + D[a];
}

void oracle_collide_jt_node(int32_t model, const double *fin, const double *F, double tau, const double *lam,
                            double *eta, double *gF) {
    if (multi_relaxation(model)) {
        collide_jt_mrt(model, fin, F, tau, lam, eta, gF);
        return;
    }
    const int inc = model == 1;
    double rho, u[3];
    moments(model, fin, F, &rho, u);
    double k = 1.0 - 1.0 / (2.0 * tau);
    double A = 0.0, V[3] = {0.0, 0.0, 0.0}, D[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        double c[3] = {(double)CV[i][0], (double)CV[i][1], (double)CV[i][2]};
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        double cF = c[0] * F[0] + c[1] * F[1] + c[2] * F[2];
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double dfeq_drho = inc ? WT(i) : WT(i) * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        A += lam[i] * dfeq_drho / tau;
        for (int a = 0; a < 3; ++a) {
            double dfeq_du = WT(i) * (inc ? 1.0 : rho) * (3.0 * c[a] + 9.0 * cu * c[a] - 3.0 * u[a]);
            double dS_du = k * WT(i) * (9.0 * cF * c[a] - 3.0 * F[a]);
            V[a] += lam[i] * (dfeq_du / tau + dS_du);
            D[a] += lam[i] * k * WT(i) * (3.0 * (c[a] - u[a]) + 9.0 * cu * c[a]);
        }
    }
    for (int j = 0; j < Q; ++j) {
        double cj_u = 0.0;
        for (int a = 0; a < 3; ++a) cj_u += V[a] * (inc ? CV[j][a] : (CV[j][a] - u[a]) / rho);
        eta[j] = (1.0 - 1.0 / tau) * lam[j] + A + cj_u;
    }
    for (int a = 0; a < 3; ++a) gF[a] = V[a] / (inc ? 2.0 : 2.0 * rho) + D[a];
}

/* loss L = (1/N_f) sum_fluid u_x(s) with u_x = (sum c_x s - F_x/2)/rho
 * (models 0, 2) or sum c_x s - F_x/2 (models 1, 3).  When lam != NULL also
 * returns dL/ds in lam[19][N] and adds dL/dF_x to gF. */
double oracle_loss_ux(int32_t model, const double *s, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz,
                      const double *force, double *lam, double *gF) {
    const int inc = incompressible(model);
    long N = (long)nx * ny * nz, nf = 0;
    for (long n = 0; n < N; ++n) nf += !solid[n];
    double L = 0.0;
    for (long n = 0; n < N; ++n) {
        if (solid[n]) {
            if (lam)
                for (int i = 0; i < Q; ++i) lam[(long)i * N + n] = 0.0;
            continue;
        }
        double r = 0.0, jx = 0.0;
        for (int i = 0; i < Q; ++i) {
            r += s[(long)i * N + n];
            jx += CV[i][0] * s[(long)i * N + n];
        }
        double Fx = force ? force[n] : 0.0;
        double ux = inc ? jx - 0.5 * Fx : (jx - 0.5 * Fx) / r;
        L += ux;
        if (lam) {
            for (int i = 0; i < Q; ++i)
                lam[(long)i * N + n] = (inc ? CV[i][0] : (CV[i][0] - ux) / r) / (double)nf;
            if (gF) gF[n] += -0.5 / (inc ? 1.0 : r) / (double)nf;
        }
    }
    return L / (double)nf;
}

/* Full reverse-mode run: T forward steps from s0 with the per-node force field
 * F[3][N], loss = mean u_x at step T.  Writes dL/ds0 [19][N] and dL/dF [3][N];
 * returns L.  Keeps all T+1 states (small boxes only).  Returns NaN on
 * allocation failure. */
double oracle_adjoint(int32_t model, const double *s0, const uint8_t *solid, int32_t nx, int32_t ny, int32_t nz,
                      int32_t periodic, double tau, const double *force, int32_t T, double *grad_s0,
                      double *grad_F) {
    long N = (long)nx * ny * nz;
    size_t SZ = (size_t)Q * (size_t)N;
    double *states = (double *)malloc(sizeof(double) * SZ * (size_t)(T + 1));
    double *lam = (double *)malloc(sizeof(double) * SZ);
    double *eta = (double *)malloc(sizeof(double) * SZ);
    double *g = (double *)malloc(sizeof(double) * SZ);
    if (!states || !lam || !eta || !g) {
        free(states); free(lam); free(eta); free(g);
        return 0.0 / 0.0;
    }
    memcpy(states, s0, sizeof(double) * SZ);
    for (int t = 1; t <= T; ++t)
        oracle_step(states + (size_t)(t - 1) * SZ, states + (size_t)t * SZ, solid, nx, ny, nz, periodic, model, tau,
                    force, 0.0, 0.0, 0.0);
    for (int a = 0; a < 3; ++a)
        for (long n = 0; n < N; ++n) grad_F[(long)a * N + n] = 0.0;
    double L = oracle_loss_ux(model, states + (size_t)T * SZ, solid, nx, ny, nz, force, lam, grad_F);
    for (int t = T; t >= 1; --t) {
        oracle_pull(states + (size_t)(t - 1) * SZ, g, solid, nx, ny, nz, periodic);
        memset(eta, 0, sizeof(double) * SZ);
        for (long n = 0; n < N; ++n) {
            if (solid[n]) continue;
            double fin[Q], l[Q], e[Q], F[3], dF[3];
            for (int i = 0; i < Q; ++i) {
                fin[i] = g[(long)i * N + n];
                l[i] = lam[(long)i * N + n];
            }
            force_at(force, N, n, 0.0, 0.0, 0.0, F);
            oracle_collide_jt_node(model, fin, F, tau, l, e, dF);
            for (int i = 0; i < Q; ++i) eta[(long)i * N + n] = e[i];
            for (int a = 0; a < 3; ++a) grad_F[(long)a * N + n] += dF[a];
        }
        oracle_pull_transpose(eta, lam, solid, nx, ny, nz, periodic);
    }
    memcpy(grad_s0, lam, sizeof(double) * SZ);
    free(states); free(lam); free(eta); free(g);
    return L;
}
