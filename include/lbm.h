/*
 * liblbm -- C-ABI of the MI355X (gfx950) implementation of the fused time step
 * of the improved 3D thermal multiphase lattice Boltzmann model of Li, Yu &
 * Luo, "Improved three-dimensional thermal multiphase lattice Boltzmann model
 * for liquid-vapor phase change" (arXiv:2201.06039):
 *
 *   - D3Q19 MRT pseudopotential lattice for density and velocity
 *     (Sec. II, Eqs. (1)-(10)) with the Peng-Robinson EOS (Sec. IV A, Eq. (49));
 *   - D3Q7 MRT lattice for temperature (Sec. III C, Eqs. (37)-(43)) whose
 *     source phi_s (Sec. III A, Eq. (18)) uses the local temperature gradient
 *     of Eq. (45) and the local velocity divergence of Eq. (48); as options
 *     the BGK collision of Eq. (19) with the gradient of Eq. (36), on D3Q7 or
 *     on a D3Q19 temperature lattice (Sec. III B);
 *   - halfway bounce-back (Eq. (50)) and anti-bounce-back (Eq. (51)) at a
 *     bottom wall, an open top, and buoyancy F_b = (rho - rho_ave) g (Sec. IV C).
 *
 * Conventions shared by every call:
 *   - Lattice units: delta_t = delta_x = c = 1.
 *   - Node index i = x + nx * (y + ny * z); host field arrays are double
 *     precision, structure of arrays, length nx*ny*nz, owned by the caller.
 *     The library copies them and never keeps a host pointer.
 *   - Device memory: the caller allocates one arena of lbm_arena_bytes() bytes
 *     (for example a torch.uint8 CUDA tensor) and keeps it alive until
 *     lbm_destroy().  The library never allocates device memory itself.
 *   - All device work is enqueued on the stream passed to lbm_create()
 *     (a hipStream_t; NULL means the default stream).  Calls that return host
 *     data synchronise that stream; lbm_step() does not.
 *   - A handle is not thread-safe.
 *   - Every int-returning call returns an LBM_* status below.
 *     lbm_strerror() gives a static description.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define LBM_OK 0
#define LBM_EINVAL (-1)    /* invalid argument or parameter                    */
#define LBM_ENOMEM (-2)    /* arena too small                                  */
#define LBM_EHIP (-3)      /* HIP runtime error                                */
#define LBM_EUNSTABLE (-4) /* a step produced rho <= 0, psi^2 < 0 or NaN       */
#define LBM_ESTATE (-5)    /* call out of order (e.g. step before init)        */
#define LBM_ESCRATCH (-6)  /* grid too large for lbm_reduce_static's scratch   */

/* Boundary in z (x and y are always periodic). */
#define LBM_BC_PERIODIC 0
/* Halfway bounce-back wall below z = 0 (Eq. (50)) with anti-bounce-back
 * Dirichlet temperature (Eq. (51)); open top at z = nz-1 whose unknown f are
 * copied from the layer below and whose g obey Eq. (51) with T_top. */
#define LBM_BC_WALL_BOTTOM_OPEN_TOP 1
/* Closed box (Sec. IV C): halfway bounce-back walls below z = 0 and above
 * z = nz-1 (Eq. (50)); anti-bounce-back Dirichlet temperature (Eq. (51)) at
 * the bottom (T_wall, T_wall_patch) and at the top (T_top). */
#define LBM_BC_WALLS 2

/* Wettability of the bottom wall (walls only; the top wall and the open top
 * see a copy of the top fluid layer).  NEUTRAL: a solid node below z = 0
 * carries the density and temperature of the fluid node above it.
 * VIRTUAL_DENSITY: the virtual-density scheme of Li, Luo, Kang & Chen
 * (Phys. Rev. E 90, 053301, 2014) standing in for the paper's Ref. [52]: a
 * solid node carries rho_w = phi rho_ave - drho, rho_ave the weighted mean of
 * its five fluid neighbours (weights 1/18 and 1/36 of Eq. (5)), and psi of
 * Eq. (8) at rho_w and the temperature of the fluid node above it; phi =
 * wet_phi_in, drho = wet_drho inside the patch -- a square of side
 * wet_square centred at ((nx-1)/2, (ny-1)/2) (Sec. IV C's patterned wall)
 * and a disc of diameter wet_disc centred there (a contact line pinned on
 * its rim stands in for Sec. IV B's hysteresis window), either or both;
 * membership decided in FP64 -- phi = wet_phi, drho = 0 elsewhere.  phi > 1 wets (contact angle below 90 degrees), phi < 1 or
 * drho > 0 does not.  Adds one launch per step. */
#define LBM_WET_NEUTRAL 0
#define LBM_WET_VIRTUAL_DENSITY 1

/* Thermal conductivity mode of Eq. (17): chi = lambda/(rho c_V). */
#define LBM_KAPPA_CONST_LAMBDA 0 /* kappa is lambda; chi varies with rho per node */
#define LBM_KAPPA_CONST_CHI 1    /* kappa is chi itself                           */

/* Temperature lattice (Sec. III B). */
#define LBM_THERMAL_D3Q7 0  /* Eq. (21); weights 1 - d, d/6; c_sT^2 = d/3          */
#define LBM_THERMAL_D3Q19 1 /* the D3Q19 velocities of Eq. (2) with the standard   */
                            /* weights 1/3, 1/18, 1/36 and c_sT^2 = 1/3; BGK only */
                            /* (thermal_bgk = 1); storage F32, F64 or F16; not in */
                            /* batches                                            */

/* Velocity divergence in the source term of Eq. (18) (Sec. III C). */
#define LBM_DIVU_LOCAL 0 /* Eq. (48) at every node, from the non-equilibrium m_4 */
#define LBM_DIVU_FD 1    /* the practice Eq. (48) replaces: isotropic finite     */
                         /* differences sum omega(|e|^2) e . u(x + e) of u(t) of */
                         /* Eq. (10) at interior nodes, Eq. (48) at the layers   */
                         /* next to a wall or the open top.  Each step first     */
                         /* writes u at every node into the staging region (a   */
                         /* velocity pass: one more launch of the step's shape). */
                         /* Built for storage F32, F64 and F16, and copies whose */
                         /* two halves (planes below and above the split) each   */
                         /* stay under 4 GiB (lbm_step returns EINVAL            */
                         /* otherwise); not in batches                           */

/* Storage format of the populations.
 *   F32, F64: the populations f, g themselves; arithmetic in the same type.
 *   F16, BF16, F32_DEV: deviations from the rest equilibrium of a per-node
 *     reference, e = (f_alpha - w_alpha rho_r) s and r = (g_alpha - w_alpha T_r) s,
 *     with w_alpha the weights of Eq. (5) at u = 0 (1/3, 1/18, 1/36) and of
 *     the temperature lattice (1 - d, d/6 on D3Q7), in the storage type.  rho_r and T_r are
 *     the node's density and temperature one step earlier, stored as two more
 *     planes (FP16 for F16, FP32 for BF16 and F32_DEV); s = 1024 for F16
 *     (keeps small deviations out of the subnormal range), 1 otherwise.
 *     Arithmetic is FP32.  The moments are formed from e and the references
 *     directly, so the rest part (the O(rho) bulk of every population) is
 *     never rounded to the storage type: only deviations are.  Accuracy of
 *     these formats is a property of the workload (it is measured against
 *     the FP64 evolution, not assumed). */
#define LBM_STORE_F32 0
#define LBM_STORE_F64 1
#define LBM_STORE_F16 2
#define LBM_STORE_BF16 3
#define LBM_STORE_F32_DEV 4

/* Problem statement.  Field names are the paper's symbols. */
typedef struct lbm_params {
    int nx, ny, nz;          /* grid; nx, ny, nz >= 1 (nz >= 3 with walls)      */
    int bc_z;                /* LBM_BC_*                                       */
    double a, b, R;          /* Peng-Robinson constants, Eq. (49)              */
    double acentric;         /* acentric factor omega of Eq. (49)              */
    double G;                /* interaction strength of Eqs. (7)-(8), != 0     */
    double sigma;            /* constant of the S_4 term of Eq. (9)            */
    double tau_e, tau_v, tau_q, tau_pi; /* relaxation times of Eq. (6), > 1/2  */
    double cV;               /* specific heat at constant volume, > 0          */
    double d;                /* D3Q7 weights w0 = 1-d, w1..6 = d/6, 0 < d < 1  */
    int kappa_mode;          /* LBM_KAPPA_*                                    */
    double kappa;            /* lambda or chi, > 0                             */
    double vs_q, vs_pi;      /* varsigma_q, varsigma_pi of Eq. (43), > 1/2      */
    double g[3];             /* gravity in F_b = (rho - rho_ave) g             */
    double T_wall_patch;     /* wall temperature inside the heated disc        */
    double T_wall;           /* wall temperature outside it                    */
    double patch_radius;     /* disc radius, centred at ((nx-1)/2, (ny-1)/2)   */
    double T_top;            /* Dirichlet temperature of the open top          */
    int thermal;             /* 1: temperature lattice evolves; 0: held fixed  */
    int storage;             /* LBM_STORE_*                                    */
    int bc_T_shell;          /* 1: constant-temperature boundary of Sec. IV A:  */
                             /* the outer layer of nodes (x, y or z at 0 or at */
                             /* n-1) is a reservoir at T_shell -- it emits     */
                             /* w T_shell without collision and every g        */
                             /* streamed into it is replaced by w T_shell, so  */
                             /* its T is T_shell after every step.  Needs      */
                             /* bc_z = LBM_BC_PERIODIC and thermal = 1.  The   */
                             /* density lattice stays periodic.                */
    double T_shell;          /* reservoir temperature, > 0 when bc_T_shell     */
    int thermal_bgk;         /* 0: MRT temperature collision, Eqs. (37)-(43);  */
                             /* 1: BGK, Eq. (19): one relaxation time          */
                             /* tau_g = 1/2 + chi/c_sT^2 for every moment (the */
                             /* MRT one with varsigma_q = varsigma_pi = tau_g),*/
                             /* grad T from Eq. (36)                           */
    int thermal_lattice;     /* LBM_THERMAL_*; D3Q19 stores 19 g planes        */
                             /* instead of 7 (38 population planes, not 26)   */
    int divu_mode;           /* LBM_DIVU_*                                     */
    int wet_mode;            /* LBM_WET_* (walls only)                         */
    double wet_phi;          /* > 0: phi outside the square                    */
    double wet_phi_in;       /* > 0: phi inside the square                     */
    double wet_drho;         /* >= 0: drho inside the square                   */
    double wet_square;       /* >= 0: side of the centred square (0: none)     */
    double wet_disc;         /* >= 0: diameter of the centred disc (0: none)   */
} lbm_params;

typedef struct lbm_handle lbm_handle;

/* Device bytes the arena must hold for these parameters (0 if invalid).
 * Layout: two copies (ping-pong) of the 19 + QT population planes (and, for
 * the deviation formats, the rho_r and T_r planes), the phi_s history plane
 * (FP32, FP64 for F64 storage), six FP64 staging planes for init and readout,
 * block partial sums and a few scalars, each region 256-byte aligned.
 * 0 also when nx*ny*nz times the element size reaches 2^32 bytes, or one
 * x-y plane of two elements a node does.  Grids whose population copy halves
 * exceed 4 GiB are addressed with 64-bit plain pointers instead of buffer
 * resources (same results). */
size_t lbm_arena_bytes(const lbm_params *p);

/* Validate p, derive the constants (T_c from a, b, R as in Sec. IV A; c_sT^2 =
 * d/3), carve the caller-owned arena and bind the HIP stream.
 * EINVAL: bad parameter or NULL pointer; ENOMEM: arena_bytes too small or
 * dev_arena not 256-byte aligned.  On success *out owns host memory only. */
int lbm_create(const lbm_params *p, void *dev_arena, size_t arena_bytes, void *hip_stream, lbm_handle **out);

/* Initial state (t = 0): f = M^-1 m_eq(rho, u) with Eq. (5), g = w T
 * (Sec. III C), phi_s(t - dt) = 0; rho_ave of the buoyancy is the initial mean.
 * EINVAL if rho <= 0, T <= 0 or psi^2 < 0 (Eq. (8)) at any node, or a NULL
 * pointer.  Synchronises the stream. */
int lbm_init_fields(lbm_handle *h, const double *rho, const double *ux, const double *uy, const double *uz,
                    const double *T);

/* Enqueue n >= 0 fused time steps (Eq. (1)-(10) collide + stream of f,
 * Eq. (37)-(45), (48), (18), (23)-(24) of g) without blocking.  Step t uses the
 * mean density at t - 1 in F_b.  ESTATE before lbm_init_fields.  On a
 * non-NULL stream that is not being captured, pairs of steps are replays of
 * a HIP graph of two steps, captured at the first use and kept until the
 * launch shape changes; on the NULL stream, or while the caller captures the
 * stream, the launches are enqueued directly. */
int lbm_step(lbm_handle *h, int n);

/* rho (Eq. (10)), u = (sum e f + F/2)/rho with the total force F (Eq. (10)),
 * and T (Eq. (20)) at the current time, as FP64 host arrays of nx*ny*nz.
 * Synchronises the stream; returns EUNSTABLE if any step since the last
 * check saw rho <= 0, psi^2 < 0 or NaN (the arrays are still written). */
int lbm_get_rho_u_T(lbm_handle *h, double *rho, double *ux, double *uy, double *uz, double *T);

/* FP64 sums of rho and T over the grid.  Synchronises; may return EUNSTABLE. */
int lbm_reduce(lbm_handle *h, double *mass, double *energy);

/* For callers that cannot allocate device memory or touch the arena's
 * scratch (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): lbm_reduce with its partial sums and results in a
 * static device array of the library (16 MiB on each GPU it runs on, held
 * until the process ends) instead of the arena.  Allocates nothing; same
 * kernels, same summation order, same results as lbm_reduce.  Up to
 * 268,434,432 nodes (2^20 - 4 blocks of 256): ESCRATCH beyond.  All handles
 * on one GPU share the array: calls that overlap on one GPU (other threads,
 * other streams) race.  Synchronises the handle's stream; may return
 * EUNSTABLE; ESTATE before init. */
int lbm_reduce_static(lbm_handle *h, double *mass, double *energy);

/* Size of the raw checkpoint: header, the stored planes (f, g and, for the
 * deviation formats, rho_r and T_r, in the storage format), phi_s history,
 * rho_ave. */
size_t lbm_state_bytes(const lbm_handle *h);

/* Copy the raw state to/from a host buffer of lbm_state_bytes() bytes.
 * Restoring and stepping reproduces the uninterrupted run bit for bit.
 * EINVAL on a size, header or grid mismatch.  Both synchronise. */
int lbm_get_state(lbm_handle *h, void *host_buf, size_t bytes);
int lbm_set_state(lbm_handle *h, const void *host_buf, size_t bytes);

/* Launch shape of the fused step kernel: an x-y tile of tile_x * tile_y
 * nodes per workgroup marching over chunk_z planes (each thread updates one
 * node per plane, chunk_z nodes in all).  Supported tiles:
 * 64x4, 32x8, 64x8, 32x16, 128x4 (F64 storage: 64x4 and 32x8 only);
 * chunk_z >= 1 (values above nz are clamped to nz).  EINVAL otherwise.
 * The result of a step does not depend on the launch shape. */
int lbm_set_launch(lbm_handle *h, int tile_x, int tile_y, int chunk_z);
int lbm_get_launch(const lbm_handle *h, int *tile_x, int *tile_y, int *chunk_z, int *workgroups);

/* Number of kernel launches lbm_step() enqueues per time step: 1, plus 1
 * when gravity needs the rho_ave reduction, plus 1 with LBM_DIVU_FD. */
int lbm_launches_per_step(const lbm_handle *h);

/* Release host resources; the arena stays with the caller.  NULL-safe. */
void lbm_destroy(lbm_handle *h);

/* Static description of a status code. */
const char *lbm_strerror(int status);

/* ---------------------------------------------------------------------------
 * Batches: many independent lattices (each its own lbm_params: grid, EOS
 * constants, temperatures, relaxation times) advanced together, one launch
 * per time step for all of them.  Each lattice follows exactly the time step
 * of a single lattice (the calls above), and its results are bitwise those of
 * a single lattice run with the same tile shape.  The launch is persistent: a
 * fixed grid of workgroups takes (lattice, tile, z-chunk) items from a device
 * work counter, largest lattices first, so lattices of uneven size share the
 * GPU.  On a non-NULL stream, lbm_batch_step() replays a captured HIP graph of
 * two steps.
 *
 * Restrictions (EINVAL otherwise): 1 <= ncases <= 65536, every lattice valid
 * for lbm_create, the same `storage` for all, bc_z = LBM_BC_PERIODIC, no
 * gravity (g = 0; the reservoir boundary bc_T_shell is allowed), the D3Q7
 * temperature lattice.
 * --------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

/* Device bytes of a batch arena for these lattices (0 if invalid): each
 * lattice's two population copies, phi_s plane and scalars, plus one set of
 * staging planes and partial sums sized for the largest lattice, the work
 * list and its counter, per-lattice step descriptors, and a copy of every
 * phi_s plane for lbm_batch_autotune(). */
size_t lbm_batch_arena_bytes(const lbm_params *cases, int ncases);

/* Carve the caller-owned arena (256-byte aligned) and bind the stream.  The
 * launch starts at the default tile of the largest lattice's format.
 * EINVAL / ENOMEM as for lbm_create. */
int lbm_batch_create(const lbm_params *cases, int ncases, void *dev_arena, size_t arena_bytes, void *hip_stream,
                     lbm_batch **out);

/* Initial state of lattice c (0 <= c < ncases) from FP64 host fields, as
 * lbm_init_fields.  Every lattice must be initialised before lbm_batch_step. */
int lbm_batch_init_case(lbm_batch *b, int c, const double *rho, const double *ux, const double *uy,
                        const double *uz, const double *T);

/* Enqueue n >= 0 time steps of every lattice without blocking.  ESTATE if a
 * lattice is not initialised. */
int lbm_batch_step(lbm_batch *b, int n);

/* Readout and sums of lattice c, as lbm_get_rho_u_T and lbm_reduce
 * (EUNSTABLE reports a problem in lattice c since its last check). */
int lbm_batch_get_rho_u_T(lbm_batch *b, int c, double *rho, double *ux, double *uy, double *uz, double *T);
int lbm_batch_reduce(lbm_batch *b, int c, double *mass, double *energy);

/* Launch shape: tile (as lbm_set_launch, shared by all lattices), z-chunk
 * length (clamped to each lattice's nz) and the number of persistent
 * workgroups (0: two per compute unit's worth of resident 256-thread groups;
 * at most the number of work items is used).  tile_x = tile_y = 0 selects
 * fitted tiles: 512-thread workgroups, each lattice with its own tile of
 * 256..512 nodes (whole x rows, exactly nx wide, for lattices up to 128
 * wide; otherwise, or where it fits better, a multiple of 4 from 64 up to
 * below nx) chosen to leave the fewest thread slots idle on its nx x ny
 * planes (not with FP64 storage).  Results do not depend on
 * the launch.  EINVAL for unsupported shapes. */
int lbm_batch_set_launch(lbm_batch *b, int tile_x, int tile_y, int chunk_z, int workgroups);
int lbm_batch_get_launch(const lbm_batch *b, int *tile_x, int *tile_y, int *chunk_z, int *workgroups, int *items);

/* The tile lattice c (0 <= c < ncases) runs with under the current launch,
 * and the threads of its workgroups (tile_x * tile_y, or 512 with fitted
 * tiles).  EINVAL for a bad index or NULL output. */
int lbm_batch_case_tile(const lbm_batch *b, int c, int *tile_x, int *tile_y, int *threads);

/* The fitted tile a batch gives a lattice with these parameters (launch tile
 * 0 x 0, above), computed on the host without a device: its workgroups have
 * 512 threads.  EINVAL for invalid parameters, FP64 storage or NULL output. */
int lbm_fitted_tile(const lbm_params *p, int *tile_x, int *tile_y);

/* Autotuner: times `steps` launches of each candidate launch shape (every
 * supported tile and fitted tiles, chunks of 8, 16, 32, 64 and 128 planes --
 * the nodes each thread updates --, one and two persistent
 * groups per compute unit) on the current state, keeps the fastest, and
 * restores the state (the timed launches only write the idle population copy
 * and the phi_s planes, which are put back).  *best_ms receives its time per
 * step.  Synchronises the stream. */
int lbm_batch_autotune(lbm_batch *b, int steps, double *best_ms);

/* Release host resources (graphs included); the arena stays with the caller. */
void lbm_batch_destroy(lbm_batch *b);

/* ---------------------------------------------------------------------------
 * Measurement aid (not part of the model): copy `bytes` bytes (a multiple of
 * 16; both pointers 16-byte aligned device memory, not overlapping) with a
 * plain streaming kernel (one 16-byte non-temporal load and store a
 * thread), enqueued on the stream
 * without blocking.  Its rate is the practical HBM ceiling the step kernels
 * are compared with, and its known traffic calibrates the hardware counters.
 * EINVAL on a bad argument.
 * --------------------------------------------------------------------------- */
int lbm_copy_probe(const void *src, void *dst, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
