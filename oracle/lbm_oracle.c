/*
 * FP64 CPU oracle for the fused time step of the improved 3D thermal
 * multiphase lattice Boltzmann model of Li, Yu & Luo (arXiv:2201.06039):
 * a D3Q19 MRT pseudopotential lattice (Sec. II, Eqs. (1)-(10), Peng-Robinson
 * EOS of Eq. (49)) coupled to a D3Q7 MRT temperature lattice (Sec. III C,
 * Eqs. (37)-(45)) whose phase-change source, Eq. (18), uses the local
 * temperature gradient of Eq. (45) and the local velocity divergence of
 * Eq. (48).  As an option the temperature lattice is D3Q19 with the BGK
 * collision of Eq. (19) and the gradient of Eq. (36) (Sec. III B, Sec. V).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library: every table
 * here is built from the paper's definitions, the D3Q19 moment matrix is
 * assembled from its monomial rows and inverted by Gauss-Jordan elimination,
 * and every transform is a plain dense matrix-vector product.
 *
 * Structure: whole-grid passes with no fusion, in the order
 *   macro (rho, T, psi)  ->  stencil (F_m, grad rho)  ->  collide (both
 *   lattices)  ->  stream (+ boundary rules).
 * Everything is double precision.  Readings of points the paper leaves open
 * are marked "Reading:" where they are applied.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Measurement build (ORC_FP32): the same source evaluated in single
 * precision -- every double below, parameters and exported arguments
 * included, becomes a float, and floating constants are single precision
 * (gcc -fsingle-precision-constant).  It measures how far a plain FP32
 * evaluation of the scheme drifts from the FP64 one; the FP64 build is the
 * oracle. */
#ifdef ORC_FP32
#define double float
#define sqrt sqrtf
#define fabs fabsf
#endif

#define Q19 19
#define Q7 7

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EUNSTABLE = -4 };

/* Parameters of one simulation; field meaning follows the paper's symbols. */
typedef struct orc_params {
    int nx, ny, nz;
    int bc_z;              /* 0: periodic in z; 1: bounce-back wall below z=0, open top;
                              2: bounce-back walls below z=0 and above z=nz-1 (closed box) */
    double a, b, R;        /* Peng-Robinson constants, Eq. (49) */
    double acentric;       /* omega in Eq. (49) */
    double G;              /* interaction strength, Eq. (7)-(8) */
    double sigma;          /* mechanical-stability constant in S_4, Eq. (9) */
    double tau_e, tau_v, tau_q, tau_pi;   /* Eq. (6) */
    double cV;             /* specific heat at constant volume, Eq. (18) */
    double d;              /* D3Q7 weight parameter, w0 = 1-d, w1..6 = d/6 */
    int kappa_mode;        /* 0: constant conductivity lambda; 1: constant chi */
    double kappa;          /* lambda or chi, per kappa_mode */
    double vs_q, vs_pi;    /* varsigma_q, varsigma_pi of Eq. (43) */
    double grav[3];        /* gravitational acceleration in F_b = (rho - rho_ave) g */
    double T_wall_patch;   /* bottom wall temperature inside the heated patch */
    double T_wall;         /* bottom wall temperature outside the patch */
    double patch_radius;   /* radius of the heated patch, centred in x-y */
    double T_top;          /* Dirichlet temperature of the open top */
    int thermal;           /* 1: temperature lattice evolves; 0: held fixed */
    int bc_T_shell;        /* 1: outer layer of nodes held at T_shell (Sec. IV A) */
    double T_shell;        /* temperature of that layer */
    int thermal_bgk;       /* 1: BGK temperature collision of Eq. (19) instead of the MRT one */
    int thermal_lattice;   /* 0: D3Q7 (Sec. III B); 1: D3Q19 with the standard weights, BGK only */
    int divu_mode;         /* 0: Eq. (48) at every node; 1: isotropic finite differences of u at
                              interior nodes, Eq. (48) at the layers next to a wall or the open top */
    int freeze_flow;       /* pin hook only (no counterpart in the product): 1 keeps the density
                              populations fixed and takes u = 0 and div u = 0 in Eq. (18), so the
                              temperature lattice evolves by conduction through a frozen rho(x) */
    int wet_mode;          /* bottom wall wettability: 0 neutral (the solid node mirrors the fluid
                              node above it); 1 virtual density rho_w = phi rho_ave - drho, after
                              Li, Luo, Kang & Chen (Phys. Rev. E 90, 053301, 2014) */
    double wet_phi;        /* wet_mode 1, outside the patch: rho_w = wet_phi * rho_ave */
    double wet_phi_in;     /* wet_mode 1, inside the patch: rho_w = wet_phi_in * rho_ave - wet_drho */
    double wet_drho;
    double wet_square;     /* patch: the square of this side centred at ((nx-1)/2, (ny-1)/2); 0: none */
    double wet_disc;       /* patch: the disc of this diameter centred there; 0: none */
} orc_params;

typedef struct orc_sim {
    orc_params p;
    long nn;
    double M[Q19][Q19], Minv[Q19][Q19];
    double N[Q7][Q7], Ninv[Q7][Q7];
    double omega[Q19];   /* omega(|e_alpha|^2) of Eq. (7) */
    int QT;              /* velocities of the temperature lattice: 7 or 19 */
    const int (*ET)[3];  /* their components */
    double wT[Q19];      /* equilibrium weights of the temperature lattice, Eq. (22) */
    double csT2;         /* c_sT^2: d/3 for D3Q7, 1/3 for D3Q19 */
    double Tc;           /* critical temperature implied by a, b, R */
    double *f, *g, *phi_prev;   /* state at time t (post-streaming) */
    double *fs, *gp;            /* post-collision f* and g+ */
    double *fn, *gn;            /* streamed state for t+1 */
    double *rho, *T, *psi;
    double *Fm, *grho;          /* 3 components, component-major */
    double *rho_w, *psi_w;      /* virtual density and psi of the solid layer below z = 0 (wet_mode 1) */
    double *uall;               /* u of Eq. (10) at every node (divu_mode 1), component-major */
    double rho_ave;             /* average density used by the next step's buoyancy */
    int status;
} orc_sim;

/* ---------------------------------------------------------------------------
 * Lattices.
 * ------------------------------------------------------------------------- */

/* Sec. II, Eq. (2): the 19 velocities in the paper's column order, c = 1. */
static const int E19[Q19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
    {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* Sec. III B, Eq. (21): the D3Q7 velocities. */
static const int E7[Q7][3] = {{0, 0, 0}, {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},
                              {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* Sec. III C, Eq. (38): the D3Q7 transformation matrix as printed. */
static const double N_PRINTED[Q7][Q7] = {
    {1, 1, 1, 1, 1, 1, 1},   {0, 1, -1, 0, 0, 0, 0},  {0, 0, 0, 1, -1, 0, 0},
    {0, 0, 0, 0, 0, 1, -1},  {0, 1, 1, 1, 1, 1, 1},   {0, 1, 1, -1, -1, 0, 0},
    {0, 1, 1, 0, 0, -1, -1}};

/* Row k of the D3Q19 transformation matrix M is the monomial p_k(e).
 * Reading: the paper defers M to its Ref. [37]; the rows used here are the raw
 * velocity monomials whose equilibria are exactly the list in Eq. (5), and
 * whose grouping m1+m11+m13 = sum e_x|e|^2 f (and cyclic) is the one Eq. (46)
 * relies on. */
static double moment_poly(int k, const int e[3]) {
    const double x = e[0], y = e[1], z = e[2];
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x + y * y + z * z;
    case 5: return 2.0 * x * x - y * y - z * z;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * x * y;
    case 11: return x * y * y;
    case 12: return x * x * z;
    case 13: return x * z * z;
    case 14: return y * y * z;
    case 15: return y * z * z;
    case 16: return x * x * y * y;
    case 17: return x * x * z * z;
    case 18: return y * y * z * z;
    }
    return 0.0;
}

/* Gauss-Jordan inversion with partial pivoting of an n x n row-major matrix. */
static int gauss_jordan_inverse(int n, const double *A, double *Ainv) {
    double *W = (double *)malloc(sizeof(double) * n * 2 * n);
    if (!W) return ORC_ENOMEM;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            W[r * 2 * n + c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(W[r * 2 * n + col]) > fabs(W[piv * 2 * n + col])) piv = r;
        if (fabs(W[piv * 2 * n + col]) < 1e-12) { free(W); return ORC_EINVAL; }
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = W[col * 2 * n + c];
                W[col * 2 * n + c] = W[piv * 2 * n + c];
                W[piv * 2 * n + c] = t;
            }
        const double inv = 1.0 / W[col * 2 * n + col];
        for (int c = 0; c < 2 * n; ++c) W[col * 2 * n + c] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double fac = W[r * 2 * n + col];
            if (fac == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) W[r * 2 * n + c] -= fac * W[col * 2 * n + c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r * n + c] = W[r * 2 * n + n + c];
    free(W);
    return ORC_OK;
}

static int build_tables(orc_sim *s) {
    for (int k = 0; k < Q19; ++k)
        for (int a = 0; a < Q19; ++a) s->M[k][a] = moment_poly(k, E19[a]);
    int rc = gauss_jordan_inverse(Q19, &s->M[0][0], &s->Minv[0][0]);
    if (rc) return rc;
    memcpy(s->N, N_PRINTED, sizeof(N_PRINTED));
    rc = gauss_jordan_inverse(Q7, &s->N[0][0], &s->Ninv[0][0]);
    if (rc) return rc;
    /* Eq. (7): omega(1) = 1/6, omega(2) = 1/12 for D3Q19. */
    for (int a = 0; a < Q19; ++a) {
        const int e2 = E19[a][0] * E19[a][0] + E19[a][1] * E19[a][1] + E19[a][2] * E19[a][2];
        s->omega[a] = e2 == 1 ? 1.0 / 6.0 : (e2 == 2 ? 1.0 / 12.0 : 0.0);
    }
    if (s->p.thermal_lattice == 0) {
        /* Sec. III B, Eq. (22): w0 = 1 - d, w1..6 = d/6, c_sT^2 = d/3. */
        s->QT = Q7;
        s->ET = E7;
        s->wT[0] = 1.0 - s->p.d;
        for (int a = 1; a < Q7; ++a) s->wT[a] = s->p.d / 6.0;
        s->csT2 = s->p.d / 3.0;
    } else {
        /* Sec. III B: on D3Q19 the weights are the standard ones, 1/3 at
         * rest, 1/18 along the axes and 1/36 along the diagonals, and
         * c_sT^2 = c_s^2 = 1/3. */
        s->QT = Q19;
        s->ET = E19;
        for (int a = 0; a < Q19; ++a) {
            const int e2 = E19[a][0] * E19[a][0] + E19[a][1] * E19[a][1] + E19[a][2] * E19[a][2];
            s->wT[a] = e2 == 0 ? 1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
        s->csT2 = 1.0 / 3.0;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Thermodynamics.
 * ------------------------------------------------------------------------- */

/* Sec. IV A: a = 0.45724 R^2 Tc^2/pc and b = 0.0778 R Tc/pc give
 * Tc = (0.0778/0.45724) a/(b R). */
static double critical_temperature(const orc_params *p) {
    if (p->a == 0.0 || p->b == 0.0 || p->R == 0.0) return 0.0;
    return 0.0778 / 0.45724 * p->a / (p->b * p->R);
}

/* Eq. (49): Peng-Robinson equation of state. */
static double p_eos(const orc_params *p, double Tc, double rho, double T) {
    double attraction = 0.0;
    if (p->a != 0.0) {
        const double w = p->acentric;
        const double kappa = 0.37464 + 1.54226 * w - 0.26992 * w * w;
        const double root = 1.0 + kappa * (1.0 - sqrt(T / Tc));
        const double vartheta = root * root;
        attraction = p->a * vartheta * rho * rho / (1.0 + 2.0 * p->b * rho - p->b * p->b * rho * rho);
    }
    return rho * p->R * T / (1.0 - p->b * rho) - attraction;
}

/* Eq. (8) squared: psi^2 = 2 [p_EOS - rho c_s^2] / (G c^2), with c = 1. */
static double psi_squared(const orc_params *p, double Tc, double rho, double T) {
    const double cs2 = 1.0 / 3.0, c = 1.0;
    return 2.0 * (p_eos(p, Tc, rho, T) - rho * cs2) / (p->G * c * c);
}

/* ---------------------------------------------------------------------------
 * Node-level pieces of the collision, exported for unit pins.
 * ------------------------------------------------------------------------- */

/* Eq. (5): equilibrium moments. */
static void equilibrium_moments(double rho, const double u[3], double meq[Q19]) {
    const double cs2 = 1.0 / 3.0;
    const double ux = u[0], uy = u[1], uz = u[2];
    const double usq = ux * ux + uy * uy + uz * uz;
    const double varphi = rho * cs2 * cs2 * (1.0 - 1.5 * usq);
    meq[0] = rho;
    meq[1] = rho * ux;
    meq[2] = rho * uy;
    meq[3] = rho * uz;
    meq[4] = rho + rho * usq;
    meq[5] = rho * (2.0 * ux * ux - uy * uy - uz * uz);
    meq[6] = rho * (uy * uy - uz * uz);
    meq[7] = rho * ux * uy;
    meq[8] = rho * ux * uz;
    meq[9] = rho * uy * uz;
    meq[10] = rho * cs2 * uy + rho * ux * ux * uy;
    meq[11] = rho * cs2 * ux + rho * uy * uy * ux;
    meq[12] = rho * cs2 * uz + rho * ux * ux * uz;
    meq[13] = rho * cs2 * ux + rho * uz * uz * ux;
    meq[14] = rho * cs2 * uz + rho * uy * uy * uz;
    meq[15] = rho * cs2 * uy + rho * uz * uz * uy;
    meq[16] = varphi + rho * cs2 * (ux * ux + uy * uy);
    meq[17] = varphi + rho * cs2 * (ux * ux + uz * uz);
    meq[18] = varphi + rho * cs2 * (uy * uy + uz * uz);
}

/* Eq. (9): forcing moments.  F is the total force; Fm the interaction force
 * of Eq. (7), which alone enters the sigma term of S_4. */
static void forcing_moments(const orc_params *p, const double F[3], const double Fm[3],
                            const double u[3], double psi, double S[Q19]) {
    const double cs2 = 1.0 / 3.0, dt = 1.0;
    const double Fx = F[0], Fy = F[1], Fz = F[2];
    const double ux = u[0], uy = u[1], uz = u[2];
    const double Fm2 = Fm[0] * Fm[0] + Fm[1] * Fm[1] + Fm[2] * Fm[2];
    const double Fu = Fx * ux + Fy * uy + Fz * uz;
    S[0] = 0.0;
    S[1] = Fx;
    S[2] = Fy;
    S[3] = Fz;
    S[4] = 2.0 * Fu + 6.0 * p->sigma * Fm2 / (psi * psi * dt * (p->tau_e - 0.5));
    S[5] = 2.0 * (2.0 * Fx * ux - Fy * uy - Fz * uz);
    S[6] = 2.0 * (Fy * uy - Fz * uz);
    S[7] = Fx * uy + Fy * ux;
    S[8] = Fx * uz + Fz * ux;
    S[9] = Fy * uz + Fz * uy;
    S[10] = cs2 * Fy;
    S[11] = cs2 * Fx;
    S[12] = cs2 * Fz;
    S[13] = cs2 * Fx;
    S[14] = cs2 * Fz;
    S[15] = cs2 * Fy;
    S[16] = 2.0 * cs2 * (ux * Fx + uy * Fy);
    S[17] = 2.0 * cs2 * (ux * Fx + uz * Fz);
    S[18] = 2.0 * cs2 * (uy * Fy + uz * Fz);
}

/* Eq. (6): diagonal of Lambda. */
static void relaxation_rates(const orc_params *p, double lam[Q19]) {
    for (int k = 0; k < 4; ++k) lam[k] = 1.0;
    lam[4] = 1.0 / p->tau_e;
    for (int k = 5; k <= 9; ++k) lam[k] = 1.0 / p->tau_v;
    for (int k = 10; k <= 15; ++k) lam[k] = 1.0 / p->tau_q;
    for (int k = 16; k <= 18; ++k) lam[k] = 1.0 / p->tau_pi;
}

/* ---------------------------------------------------------------------------
 * Geometry.
 * ------------------------------------------------------------------------- */

static long node_index(const orc_params *p, int x, int y, int z) {
    return ((long)z * p->ny + y) * p->nx + x;
}

/* Index of the node x + e used by the interaction-force and density-gradient
 * stencils.  x and y are periodic.  In z: periodic, or, with walls,
 * Reading: a solid node below z = 0 carries the virtual density and
 * temperature of the fluid node directly above it (neutral wetting), and a
 * node above the open top copies the top layer. */
static long stencil_neighbour(const orc_params *p, int x, int y, int z, const int e[3]) {
    const int xn = ((x + e[0]) % p->nx + p->nx) % p->nx;
    const int yn = ((y + e[1]) % p->ny + p->ny) % p->ny;
    int zn = z + e[2];
    if (p->bc_z == 0) {
        zn = (zn % p->nz + p->nz) % p->nz;
    } else {
        if (zn < 0) zn = 0;
        if (zn > p->nz - 1) zn = p->nz - 1;
    }
    return node_index(p, xn, yn, zn);
}

/* Reading: wall temperature of the heated patch (a disc centred in x-y). */
static double bottom_wall_temperature(const orc_params *p, int x, int y) {
    const double cx = 0.5 * (p->nx - 1), cy = 0.5 * (p->ny - 1);
    const double r2 = (x - cx) * (x - cx) + (y - cy) * (y - cy);
    return r2 <= p->patch_radius * p->patch_radius ? p->T_wall_patch : p->T_wall;
}

/* ---------------------------------------------------------------------------
 * Whole-grid passes.
 * ------------------------------------------------------------------------- */

/* Whether bottom-wall node (x, y) lies in the wettability patch: the centred
 * square or the centred disc. */
static int in_wet_patch(const orc_params *p, int x, int y) {
    const double cx = 0.5 * (p->nx - 1), cy = 0.5 * (p->ny - 1), h = 0.5 * p->wet_square;
    const double dx = x - cx, dy = y - cy, r = 0.5 * p->wet_disc;
    const int in_square = p->wet_square > 0.0 && fabs(dx) <= h && fabs(dy) <= h;
    const int in_disc = p->wet_disc > 0.0 && dx * dx + dy * dy <= r * r;
    return in_square || in_disc;
}

/* Wettability of the bottom wall (Sec. IV B-C; the paper takes its scheme
 * from its Ref. [52], which is not reproduced here).  Reading: the virtual-
 * density scheme of Li, Luo, Kang & Chen (2014).  A solid node x_s of the
 * layer below z = 0 carries the virtual density
 *   rho_w = phi * rho_ave - drho,
 *   rho_ave = sum_a w_a rho(x_s + e_a) s(x_s + e_a) / sum_a w_a s(x_s + e_a),
 * phi > 1 wetting, phi < 1 or drho > 0 non-wetting (that paper's improved
 * scheme takes phi = 1, drho > 0 for non-wetting walls; at the density ratio
 * of 0.86 T_c, rho_l/rho_g = 17, a drho above ~0.1 drives the vapour density
 * at the wall to zero, so phi < 1 is the usable form here),
 * s = 1 on fluid nodes: the five neighbours with e_z = +1 (weights 1/18 for
 * (0,0,1), 1/36 for the four diagonals).  Its psi is Eq. (8) at rho_w and the
 * temperature of the fluid node above it (reading).  The density gradient
 * and the force of Eq. (7) at the fluid layer see these virtual values. */
static void pass_wall_density(orc_sim *s) {
    const orc_params *p = &s->p;
    int bad = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(| : bad)
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            double num = 0.0, den = 0.0;
            for (int a = 1; a < Q19; ++a) {
                if (E19[a][2] != 1) continue;
                const double w = (E19[a][0] == 0 && E19[a][1] == 0) ? 1.0 / 18.0 : 1.0 / 36.0;
                const int xn = ((x + E19[a][0]) % p->nx + p->nx) % p->nx;
                const int yn = ((y + E19[a][1]) % p->ny + p->ny) % p->ny;
                num += w * s->rho[node_index(p, xn, yn, 0)];
                den += w;
            }
            const double rho_ave = num / den;
            const double rw = in_wet_patch(p, x, y) ? p->wet_phi_in * rho_ave - p->wet_drho : p->wet_phi * rho_ave;
            const double p2 = psi_squared(p, s->Tc, rw, s->T[node_index(p, x, y, 0)]);
            if (!(rw > 0.0) || !(p2 >= 0.0)) bad = 1;
            s->rho_w[(long)y * p->nx + x] = rw;
            s->psi_w[(long)y * p->nx + x] = sqrt(p2 > 0.0 ? p2 : 0.0);
        }
    if (bad) s->status = ORC_EUNSTABLE;
}

/* Eq. (10) rho = sum f, Eq. (20) T = sum g, Eq. (8) psi. */
static void pass_macro(orc_sim *s) {
    const long nn = s->nn;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long i = 0; i < nn; ++i) {
        double rho = 0.0, T = 0.0;
        for (int a = 0; a < Q19; ++a) rho += s->f[a * nn + i];
        for (int a = 0; a < s->QT; ++a) T += s->g[a * nn + i];
        const double p2 = psi_squared(&s->p, s->Tc, rho, T);
        if (!(rho > 0.0) || !(p2 >= 0.0) || !(T == T)) bad = 1;
        s->rho[i] = rho;
        s->T[i] = T;
        s->psi[i] = sqrt(p2 > 0.0 ? p2 : 0.0);
    }
    if (bad) s->status = ORC_EUNSTABLE;
    if (s->p.bc_z != 0 && s->p.wet_mode == 1) pass_wall_density(s);
}

/* Eq. (7) interaction force, and the isotropic gradient of rho with the same
 * weights.  Reading: the paper cites, but does not print, the isotropic
 * finite-difference gradient; it is taken as sum omega(|e|^2) rho(x+e) e. */
static void pass_stencil(orc_sim *s) {
    const orc_params *p = &s->p;
    const long nn = s->nn;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const long i = node_index(p, x, y, z);
                double sp[3] = {0, 0, 0}, sr[3] = {0, 0, 0};
                for (int a = 1; a < Q19; ++a) {
                    const long j = stencil_neighbour(p, x, y, z, E19[a]);
                    double pj = s->psi[j], rj = s->rho[j];
                    if (p->bc_z != 0 && p->wet_mode == 1 && z + E19[a][2] < 0) {
                        const long k = j % ((long)p->nx * p->ny);  /* (x + e_x, y + e_y) of the solid layer */
                        pj = s->psi_w[k];
                        rj = s->rho_w[k];
                    }
                    for (int c = 0; c < 3; ++c) {
                        sp[c] += s->omega[a] * pj * E19[a][c];
                        sr[c] += s->omega[a] * rj * E19[a][c];
                    }
                }
                for (int c = 0; c < 3; ++c) {
                    s->Fm[c * nn + i] = -p->G * s->psi[i] * sp[c];
                    s->grho[c * nn + i] = sr[c];
                }
            }
}

/* Total force: F = F_m + F_b with the buoyancy F_b = (rho - rho_ave) g. */
static void total_force(const orc_sim *s, long i, double F[3], double Fm[3]) {
    for (int c = 0; c < 3; ++c) {
        Fm[c] = s->Fm[c * s->nn + i];
        F[c] = Fm[c] + (s->rho[i] - s->rho_ave) * s->p.grav[c];
    }
}

/* Eq. (10): u = (sum e f + dt F / 2) / rho. */
static void velocity(const orc_sim *s, long i, const double F[3], double u[3]) {
    const long nn = s->nn;
    for (int c = 0; c < 3; ++c) {
        double j = 0.0;
        for (int a = 0; a < Q19; ++a) j += E19[a][c] * s->f[a * nn + i];
        u[c] = (j + 0.5 * F[c]) / s->rho[i];
    }
}

/* Collision of both lattices at every node. */
/* Constant-temperature boundary of the D^2-law test (Sec. IV A).  Reading:
 * the outermost layer of nodes of the (otherwise periodic) box is a thermal
 * reservoir at T_shell; its temperature populations are w T_shell before and
 * after every collision. */
static int in_shell(const orc_params *p, int x, int y, int z) {
    return p->bc_T_shell && (x == 0 || x == p->nx - 1 || y == 0 || y == p->ny - 1 || z == 0 || z == p->nz - 1);
}

static void pass_collide(orc_sim *s) {
    const orc_params *p = &s->p;
    const long nn = s->nn;
    const double cs2 = 1.0 / 3.0, dt = 1.0;
    const double csT2 = s->csT2;      /* Eq. (22): c_sT^2 = d/3 (D3Q7) or 1/3 (D3Q19) */
    const int QT = s->QT;
    double lam[Q19];
    relaxation_rates(p, lam);
    if (p->divu_mode == 1) {
        /* u(t) of Eq. (10) at every node, for the finite-difference divergence. */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < nn; ++i) {
            double F[3], Fm[3], u[3];
            total_force(s, i, F, Fm);
            velocity(s, i, F, u);
            for (int c = 0; c < 3; ++c) s->uall[c * nn + i] = u[c];
        }
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nn; ++i) {
        const double rho = s->rho[i];
        double F[3], Fm[3], u[3];
        total_force(s, i, F, Fm);
        velocity(s, i, F, u);
        if (p->freeze_flow)
            for (int c = 0; c < 3; ++c) u[c] = 0.0;

        /* Eq. (3): m* = m - Lambda (m - m_eq) + dt (I - Lambda/2) S. */
        double fl[Q19], m[Q19], meq[Q19], S[Q19], ms[Q19];
        for (int a = 0; a < Q19; ++a) fl[a] = s->f[a * nn + i];
        for (int k = 0; k < Q19; ++k) {
            m[k] = 0.0;
            for (int a = 0; a < Q19; ++a) m[k] += s->M[k][a] * fl[a];
        }
        equilibrium_moments(rho, u, meq);
        forcing_moments(p, F, Fm, u, s->psi[i], S);
        for (int k = 0; k < Q19; ++k)
            ms[k] = m[k] - lam[k] * (m[k] - meq[k]) + dt * (1.0 - 0.5 * lam[k]) * S[k];
        /* Eq. (4): f* = M^-1 m*. */
        for (int a = 0; a < Q19; ++a) {
            double acc = 0.0;
            for (int k = 0; k < Q19; ++k) acc += s->Minv[a][k] * ms[k];
            s->fs[a * nn + i] = acc;
        }

        if (!p->thermal) continue;
        if (p->bc_T_shell) {
            const int x = (int)(i % p->nx), y = (int)((i / p->nx) % p->ny), z = (int)(i / ((long)p->nx * p->ny));
            if (in_shell(p, x, y, z)) {
                for (int a = 0; a < QT; ++a) s->gp[a * nn + i] = s->wT[a] * p->T_shell;
                continue;
            }
        }

        /* Eq. (48): local velocity divergence from the non-equilibrium part
         * of m_4 (reading: applied at every node, pre-collision m_4). */
        const double Fu = F[0] * u[0] + F[1] * u[1] + F[2] * u[2];
        double divu = (-(m[4] - meq[4]) / (p->tau_e * dt) + (1.0 - 1.0 / (2.0 * p->tau_e)) * S[4] - 2.0 * Fu)
                      / (2.0 * rho * cs2);
        if (p->divu_mode == 1) {
            /* The practice Eq. (48) replaces (Sec. III C): the isotropic
             * finite-difference divergence sum omega(|e|^2) e . u(x + e) of
             * u(t) at interior nodes; the layers next to a wall or the open
             * top keep Eq. (48). */
            const int x = (int)(i % p->nx), y = (int)((i / p->nx) % p->ny), z = (int)(i / ((long)p->nx * p->ny));
            if (p->bc_z == 0 || (z > 0 && z < p->nz - 1)) {
                double acc = 0.0;
                for (int a = 1; a < Q19; ++a) {
                    const long j = stencil_neighbour(p, x, y, z, E19[a]);
                    for (int c = 0; c < 3; ++c) acc += s->omega[a] * E19[a][c] * s->uall[c * nn + j];
                }
                divu = acc;
            }
        }
        if (p->freeze_flow) divu = 0.0;

        const double T = s->T[i];
        /* chi = lambda/(rho cV) (constant lambda) or given; chi = (vs_T - 0.5) c_sT^2 dt. */
        const double chi = p->kappa_mode == 0 ? p->kappa / (rho * p->cV) : p->kappa;
        const double vsT = 0.5 + chi / (csT2 * dt);

        double gl[Q19], gradT[3];
        for (int a = 0; a < QT; ++a) gl[a] = s->g[a * nn + i];
        double n[Q7], neq[Q7];
        if (QT == Q7) {
            /* Eq. (38): n = N g; Eq. (42): n_eq. */
            for (int k = 0; k < Q7; ++k) {
                n[k] = 0.0;
                for (int a = 0; a < Q7; ++a) n[k] += s->N[k][a] * gl[a];
            }
            neq[0] = T; neq[1] = 0.0; neq[2] = 0.0; neq[3] = 0.0;
            neq[4] = 3.0 * csT2 * T; neq[5] = 0.0; neq[6] = 0.0;
            /* Eq. (45): local temperature gradient. */
            for (int c = 0; c < 3; ++c) gradT[c] = -(n[1 + c] - neq[1 + c]) / (vsT * csT2 * dt);
        } else {
            /* Eq. (36): grad T = -sum e (g - w T) / (tau_g c_sT^2 dt), tau_g = vs_T. */
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int a = 0; a < Q19; ++a) acc += E19[a][c] * (gl[a] - s->wT[a] * T);
                gradT[c] = -acc / (vsT * csT2 * dt);
            }
        }

        /* Eq. (18) with (dp/dT)_rho ~ rho R/(1 - b rho) (Sec. IV A); c_V constant. */
        const double rhocV = rho * p->cV;
        double adv = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double grad_rhocV = p->cV * s->grho[c * nn + i];
            adv += (chi * grad_rhocV / rhocV - u[c]) * gradT[c];
        }
        const double dpdT = rho * p->R / (1.0 - p->b * rho);
        const double phis = adv - T / rhocV * dpdT * divu;

        if (QT == Q7) {
            /* Eq. (39) with Gamma of Eq. (43). */
            double ns[Q7];
            double Gam[Q7] = {1.0, 1.0 / vsT, 1.0 / vsT, 1.0 / vsT, 1.0 / p->vs_q, 1.0 / p->vs_pi, 1.0 / p->vs_pi};
            if (p->thermal_bgk) {
                /* Eq. (19): g <- g - (g - w T)/tau_g + Q with tau_g = varsigma_T; in
                 * moment space every non-conserved moment relaxes at 1/tau_g. */
                for (int k = 1; k < Q7; ++k) Gam[k] = 1.0 / vsT;
            }
            for (int k = 0; k < Q7; ++k) ns[k] = n[k] - Gam[k] * (n[k] - neq[k]);
            /* Eqs. (23)-(24) with C_alpha = w_alpha phi_s, and Eq. (40). */
            for (int a = 0; a < Q7; ++a) {
                double acc = 0.0;
                for (int k = 0; k < Q7; ++k) acc += s->Ninv[a][k] * ns[k];
                const double Q = 1.5 * s->wT[a] * phis - 0.5 * s->wT[a] * s->phi_prev[i];
                s->gp[a * nn + i] = acc + dt * Q;
            }
        } else {
            /* Eq. (19) in population space with g_eq = w T (Eq. (20)) and the
             * source of Eqs. (23)-(24), C_alpha = w_alpha phi_s. */
            for (int a = 0; a < Q19; ++a) {
                const double geq = s->wT[a] * T;
                const double Q = 1.5 * s->wT[a] * phis - 0.5 * s->wT[a] * s->phi_prev[i];
                s->gp[a * nn + i] = gl[a] - (gl[a] - geq) / vsT + dt * Q;
            }
        }
        s->phi_prev[i] = phis;
    }
}

/* The velocity opposite to e_a; the D3Q7 velocities are the first seven of
 * D3Q19 in the same order, so one rule serves both lattices. */
static int opposite19(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }

/* Eq. (4) and Eq. (40): f(x + e, t + 1) = f*(x, t), g(x + e, t + 1) = g+(x, t),
 * periodic in x and y.  With walls: Eq. (50) halfway bounce-back of f and
 * Eq. (51) anti-bounce-back of g at the bottom.  Reading for the open top:
 * the unknown incoming f at the top layer are copied from the layer below
 * (zero gradient) and g obeys Eq. (51) with T_top. */
static void pass_stream(orc_sim *s) {
    const orc_params *p = &s->p;
    const long nn = s->nn;
    const int walls = p->bc_z != 0;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const long i = node_index(p, x, y, z);
                for (int a = 0; a < Q19 && !p->freeze_flow; ++a) {
                    const int xd = ((x + E19[a][0]) % p->nx + p->nx) % p->nx;
                    const int yd = ((y + E19[a][1]) % p->ny + p->ny) % p->ny;
                    int zd = z + E19[a][2];
                    if (!walls) {
                        zd = (zd % p->nz + p->nz) % p->nz;
                    } else if (zd < 0) {
                        s->fn[opposite19(a) * nn + i] = s->fs[a * nn + i];
                        continue;
                    } else if (zd > p->nz - 1) {
                        /* bc_z 2: Eq. (50) bounce-back at the top wall too; bc_z 1: leaves the domain */
                        if (p->bc_z == 2) s->fn[opposite19(a) * nn + i] = s->fs[a * nn + i];
                        continue;
                    }
                    s->fn[a * nn + node_index(p, xd, yd, zd)] = s->fs[a * nn + i];
                }
                if (!p->thermal) continue;
                for (int a = 0; a < s->QT; ++a) {
                    const int xd = ((x + s->ET[a][0]) % p->nx + p->nx) % p->nx;
                    const int yd = ((y + s->ET[a][1]) % p->ny + p->ny) % p->ny;
                    int zd = z + s->ET[a][2];
                    if (!walls) {
                        zd = (zd % p->nz + p->nz) % p->nz;
                    } else if (zd < 0) {
                        const double Tw = bottom_wall_temperature(p, x, y);
                        s->gn[opposite19(a) * nn + i] = -s->gp[a * nn + i] + 2.0 * s->wT[a] * Tw;
                        continue;
                    } else if (zd > p->nz - 1) {
                        s->gn[opposite19(a) * nn + i] = -s->gp[a * nn + i] + 2.0 * s->wT[a] * p->T_top;
                        continue;
                    }
                    s->gn[a * nn + node_index(p, xd, yd, zd)] = s->gp[a * nn + i];
                }
            }
    if (p->thermal && p->bc_T_shell) {
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x)
                    if (in_shell(p, x, y, z))
                        for (int a = 0; a < s->QT; ++a) s->gn[a * nn + node_index(p, x, y, z)] = s->wT[a] * p->T_shell;
    }
    if (p->bc_z == 1 && !p->freeze_flow) {
        const int zt = p->nz - 1;
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x)
                for (int a = 0; a < Q19; ++a)
                    if (E19[a][2] < 0)
                        s->fn[a * nn + node_index(p, x, y, zt)] = s->fn[a * nn + node_index(p, x, y, zt - 1)];
    }
    double *t;
    if (!p->freeze_flow) { t = s->f; s->f = s->fn; s->fn = t; }
    if (p->thermal) { t = s->g; s->g = s->gn; s->gn = t; }
}

/* Mean density over the grid, summed in node order. */
static double mean_density(const orc_sim *s) {
    double acc = 0.0;
    for (long i = 0; i < s->nn; ++i) acc += s->rho[i];
    return acc / (double)s->nn;
}

/* ---------------------------------------------------------------------------
 * Exported API.
 * ------------------------------------------------------------------------- */

void orc_destroy(orc_sim *s) {
    if (!s) return;
    free(s->f); free(s->g); free(s->phi_prev); free(s->fs); free(s->gp);
    free(s->fn); free(s->gn); free(s->rho); free(s->T); free(s->psi);
    free(s->Fm); free(s->grho); free(s->uall); free(s->rho_w); free(s->psi_w);
    free(s);
}

int orc_create(const orc_params *p, orc_sim **out) {
    *out = NULL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return ORC_EINVAL;
    if (p->bc_z < 0 || p->bc_z > 2) return ORC_EINVAL;
    if (p->bc_z != 0 && p->nz < 3) return ORC_EINVAL;
    if (p->wet_mode != 0 && (p->wet_mode != 1 || p->bc_z == 0 || !(p->wet_phi > 0.0) || !(p->wet_phi_in > 0.0) ||
                             !(p->wet_drho >= 0.0) || !(p->wet_square >= 0.0) || !(p->wet_disc >= 0.0)))
        return ORC_EINVAL;
    if (p->bc_T_shell && (p->bc_z != 0 || !p->thermal || !(p->T_shell > 0.0))) return ORC_EINVAL;
    if (p->thermal_bgk != 0 && p->thermal_bgk != 1) return ORC_EINVAL;
    /* Reading: the paper gives relaxation rates for the D3Q7 moments only,
     * so the D3Q19 temperature lattice takes the BGK collision. */
    if (p->thermal_lattice != 0 && (p->thermal_lattice != 1 || !p->thermal_bgk)) return ORC_EINVAL;
    if (p->divu_mode != 0 && p->divu_mode != 1) return ORC_EINVAL;
    if (p->tau_e <= 0.5 || p->tau_v <= 0.5 || p->tau_q <= 0.5 || p->tau_pi <= 0.5) return ORC_EINVAL;
    if (p->vs_q <= 0.5 || p->vs_pi <= 0.5 || p->G == 0.0 || p->cV <= 0.0) return ORC_EINVAL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!s) return ORC_ENOMEM;
    s->p = *p;
    s->nn = (long)p->nx * p->ny * p->nz;
    s->Tc = critical_temperature(p);
    const long nn = s->nn;
    s->f = calloc(Q19 * nn, sizeof(double));
    s->fs = calloc(Q19 * nn, sizeof(double));
    s->fn = calloc(Q19 * nn, sizeof(double));
    const long qt = p->thermal_lattice ? Q19 : Q7;
    s->g = calloc(qt * nn, sizeof(double));
    s->gp = calloc(qt * nn, sizeof(double));
    s->gn = calloc(qt * nn, sizeof(double));
    s->phi_prev = calloc(nn, sizeof(double));
    s->rho = calloc(nn, sizeof(double));
    s->T = calloc(nn, sizeof(double));
    s->psi = calloc(nn, sizeof(double));
    s->Fm = calloc(3 * nn, sizeof(double));
    s->grho = calloc(3 * nn, sizeof(double));
    s->uall = calloc(p->divu_mode ? 3 * nn : 1, sizeof(double));
    s->rho_w = calloc((long)p->nx * p->ny, sizeof(double));
    s->psi_w = calloc((long)p->nx * p->ny, sizeof(double));
    if (!s->f || !s->fs || !s->fn || !s->g || !s->gp || !s->gn || !s->phi_prev || !s->rho || !s->T ||
        !s->psi || !s->Fm || !s->grho || !s->uall || !s->rho_w || !s->psi_w) {
        orc_destroy(s);
        return ORC_ENOMEM;
    }
    int rc = build_tables(s);
    if (rc) { orc_destroy(s); return rc; }
    *out = s;
    return ORC_OK;
}

/* Initial populations: f = M^-1 m_eq(rho0, u0), g = w T0, phi_s(t - dt) = 0.
 * The average density for the first step's buoyancy is the initial mean. */
int orc_init_fields(orc_sim *s, const double *rho, const double *ux, const double *uy, const double *uz,
                    const double *T) {
    const long nn = s->nn;
    for (long i = 0; i < nn; ++i) {
        if (!(rho[i] > 0.0) || !(T[i] > 0.0) || !(psi_squared(&s->p, s->Tc, rho[i], T[i]) >= 0.0))
            return ORC_EINVAL;
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nn; ++i) {
        const double u[3] = {ux[i], uy[i], uz[i]};
        double meq[Q19];
        equilibrium_moments(rho[i], u, meq);
        for (int a = 0; a < Q19; ++a) {
            double acc = 0.0;
            for (int k = 0; k < Q19; ++k) acc += s->Minv[a][k] * meq[k];
            s->f[a * nn + i] = acc;
        }
        for (int a = 0; a < s->QT; ++a) s->g[a * nn + i] = s->wT[a] * T[i];
        s->phi_prev[i] = 0.0;
    }
    s->status = ORC_OK;
    pass_macro(s);
    s->rho_ave = mean_density(s);
    return s->status;
}

/* n time steps.  The buoyancy of step t uses the mean density at t - 1
 * (reading; for a closed or periodic domain it equals the current mean up to
 * rounding, since mass is conserved). */
int orc_step(orc_sim *s, int nsteps) {
    for (int k = 0; k < nsteps; ++k) {
        pass_macro(s);
        if (s->status) return s->status;
        const double next_rho_ave = mean_density(s);
        pass_stencil(s);
        pass_collide(s);
        pass_stream(s);
        s->rho_ave = next_rho_ave;
    }
    return s->status;
}

/* rho, u of Eq. (10) with the total force, and T, at the current time. */
int orc_get_rho_u_T(orc_sim *s, double *rho, double *ux, double *uy, double *uz, double *T) {
    pass_macro(s);
    pass_stencil(s);
    const long nn = s->nn;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nn; ++i) {
        double F[3], Fm[3], u[3];
        total_force(s, i, F, Fm);
        velocity(s, i, F, u);
        rho[i] = s->rho[i];
        ux[i] = u[0];
        uy[i] = u[1];
        uz[i] = u[2];
        T[i] = s->T[i];
    }
    return s->status;
}

/* Raw state: f (19 x nn), g (7 or 19 x nn), phi_s history (nn), average density. */
void orc_get_state(const orc_sim *s, double *f, double *g, double *phi_prev, double *rho_ave) {
    memcpy(f, s->f, sizeof(double) * Q19 * s->nn);
    memcpy(g, s->g, sizeof(double) * s->QT * s->nn);
    memcpy(phi_prev, s->phi_prev, sizeof(double) * s->nn);
    *rho_ave = s->rho_ave;
}

void orc_set_state(orc_sim *s, const double *f, const double *g, const double *phi_prev, double rho_ave) {
    memcpy(s->f, f, sizeof(double) * Q19 * s->nn);
    memcpy(s->g, g, sizeof(double) * s->QT * s->nn);
    memcpy(s->phi_prev, phi_prev, sizeof(double) * s->nn);
    s->rho_ave = rho_ave;
    s->status = ORC_OK;
}

/* Total mass sum rho and sum T over the grid. */
void orc_reduce(orc_sim *s, double *mass, double *energy) {
    pass_macro(s);
    double m = 0.0, e = 0.0;
    for (long i = 0; i < s->nn; ++i) { m += s->rho[i]; e += s->T[i]; }
    *mass = m;
    *energy = e;
}

/* --- unit hooks used by the pins ------------------------------------------ */

void orc_tables(const orc_params *p, double *M, double *Minv, double *N, double *Ninv, int *e19, int *e7,
                double *omega, double *wT) {
    orc_sim s;
    memset(&s, 0, sizeof(s));
    s.p = *p;
    build_tables(&s);
    memcpy(M, s.M, sizeof(s.M));
    memcpy(Minv, s.Minv, sizeof(s.Minv));
    memcpy(N, s.N, sizeof(s.N));
    memcpy(Ninv, s.Ninv, sizeof(s.Ninv));
    memcpy(e19, E19, sizeof(E19));
    memcpy(e7, E7, sizeof(E7));
    memcpy(omega, s.omega, sizeof(s.omega));
    memcpy(wT, s.wT, sizeof(double) * s.QT);
}

double orc_critical_temperature(const orc_params *p) { return critical_temperature(p); }

double orc_p_eos(const orc_params *p, double rho, double T) { return p_eos(p, critical_temperature(p), rho, T); }

double orc_psi_squared(const orc_params *p, double rho, double T) {
    return psi_squared(p, critical_temperature(p), rho, T);
}

void orc_equilibrium_moments(double rho, const double *u, double *meq) { equilibrium_moments(rho, u, meq); }

void orc_forcing_moments(const orc_params *p, const double *F, const double *Fm, const double *u, double psi,
                         double *S) {
    forcing_moments(p, F, Fm, u, psi, S);
}

double orc_rho_ave(const orc_sim *s) { return s->rho_ave; }

/* Threads an OpenMP parallel region of the oracle uses (for reporting). */
int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following parallel regions of the calling thread; n <= 0
 * restores the number OpenMP started with. */
void orc_set_threads(int n) {
#ifdef _OPENMP
    static int initial = 0;
    if (!initial) initial = omp_get_max_threads();
    omp_set_num_threads(n > 0 ? n : initial);
#else
    (void)n;
#endif
}
