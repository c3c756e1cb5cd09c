// Host side of liblbm: parameter validation, arena carving, launches and the
// C-ABI declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "lbm.h"
#include "lbm_kernels.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxChunk = 1 << 20;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct TileShape {
    int tx, ty;
};
constexpr TileShape kTiles[] = {{64, 4}, {32, 8}, {64, 8}, {32, 16}, {128, 4}};

struct Layout {
    size_t nn, stride, es, rs, cs, planes;
    size_t npop;   // population planes: 19 + velocities of the temperature lattice
    int qt;        // 7 (D3Q7) or 19 (D3Q19)
    size_t off_pop[2], off_phi, off_stage, off_part, off_scal, off_wall, total;
    size_t max_partials;
};

bool valid_storage(int s) {
    return s == LBM_STORE_F32 || s == LBM_STORE_F64 || s == LBM_STORE_F16 || s == LBM_STORE_BF16 ||
           s == LBM_STORE_F32_DEV;
}

// Bytes of one stored population value.
size_t element_bytes(int s) {
    if (s == LBM_STORE_F64) return 8;
    if (s == LBM_STORE_F16 || s == LBM_STORE_BF16) return 2;
    return 4;
}

// Velocities of the temperature lattice.
int thermal_q(const lbm_params *p) { return p->thermal_lattice == LBM_THERMAL_D3Q19 ? 19 : 7; }

// Planes per copy: 19 + QT populations, plus rho_r and T_r for the deviation
// formats (FP16 for F16, FP32 for BF16 and F32_DEV).
size_t planes_of(int s, int qt) { return 19 + qt + ((s == LBM_STORE_F32 || s == LBM_STORE_F64) ? 0 : 2); }
size_t reference_bytes(int s) { return s == LBM_STORE_F64 ? 8 : (s == LBM_STORE_F16 ? 2 : 4); }

bool valid_params(const lbm_params *p) {
    if (!p) return false;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
    if (!valid_storage(p->storage)) return false;
    // Node indices and element offsets are 32-bit: nx*ny*nz elements of a plane must span under 4 GiB.
    // Byte offsets inside an x-y plane are 32-bit too (in the paired layout a node takes two elements).
    if ((size_t)p->nx * p->ny * p->nz * element_bytes(p->storage) >= (size_t)1 << 32) return false;
    if ((size_t)p->nx * p->ny * 2 * (element_bytes(p->storage) > 4 ? element_bytes(p->storage) : 4) >= (size_t)1 << 32)
        return false;
    if (p->bc_z != LBM_BC_PERIODIC && p->bc_z != LBM_BC_WALL_BOTTOM_OPEN_TOP && p->bc_z != LBM_BC_WALLS) return false;
    if (p->bc_z != LBM_BC_PERIODIC && p->nz < 3) return false;
    if (p->wet_mode != LBM_WET_NEUTRAL && p->wet_mode != LBM_WET_VIRTUAL_DENSITY) return false;
    if (p->wet_mode == LBM_WET_VIRTUAL_DENSITY &&
        (p->bc_z == LBM_BC_PERIODIC || !(p->wet_phi > 0.0) || !(p->wet_phi_in > 0.0) || !(p->wet_drho >= 0.0) ||
         !(p->wet_square >= 0.0) || !(p->wet_disc >= 0.0)))
        return false;
    if (!(p->tau_e > 0.5) || !(p->tau_v > 0.5) || !(p->tau_q > 0.5) || !(p->tau_pi > 0.5)) return false;
    if (!(p->vs_q > 0.5) || !(p->vs_pi > 0.5)) return false;
    if (p->G == 0.0 || !(p->cV > 0.0) || !(p->kappa > 0.0)) return false;
    if (!(p->d > 0.0 && p->d < 1.0)) return false;
    if (p->kappa_mode != LBM_KAPPA_CONST_LAMBDA && p->kappa_mode != LBM_KAPPA_CONST_CHI) return false;
    if (p->a != 0.0 && !(p->b > 0.0 && p->R > 0.0)) return false;
    if (p->a < 0.0 || p->b < 0.0 || p->R < 0.0) return false;
    if (p->thermal != 0 && p->thermal != 1) return false;
    if (p->bc_T_shell != 0 && p->bc_T_shell != 1) return false;
    if (p->thermal_bgk != 0 && p->thermal_bgk != 1) return false;
    // The paper gives relaxation rates for the D3Q7 moments only: the D3Q19
    // temperature lattice takes the BGK collision.
    if (p->thermal_lattice != LBM_THERMAL_D3Q7 && p->thermal_lattice != LBM_THERMAL_D3Q19) return false;
    if (p->divu_mode != LBM_DIVU_LOCAL && p->divu_mode != LBM_DIVU_FD) return false;
    if (p->divu_mode == LBM_DIVU_FD && (p->storage == LBM_STORE_BF16 || p->storage == LBM_STORE_F32_DEV))
        return false;
    if (p->thermal_lattice == LBM_THERMAL_D3Q19 &&
        (!p->thermal_bgk || p->storage == LBM_STORE_BF16 || p->storage == LBM_STORE_F32_DEV))
        return false;
    if (p->bc_T_shell && (p->bc_z != LBM_BC_PERIODIC || !p->thermal || !(p->T_shell > 0.0))) return false;
    return true;
}

size_t max_workgroups(const lbm_params *p) {
    size_t best = 0;
    for (const TileShape &t : kTiles) {
        const size_t nb = (size_t)((p->nx + t.tx - 1) / t.tx) * ((p->ny + t.ty - 1) / t.ty) * p->nz;
        if (nb > best) best = nb;
    }
    const size_t nn = (size_t)p->nx * p->ny * p->nz;
    const size_t sum_blocks = (nn + 255) / 256;
    return best > sum_blocks ? best : sum_blocks;
}

size_t copy_bytes(const Layout &L) { return L.stride * (L.npop * L.es + (L.planes - L.npop) * L.rs); }

// Physical planes of a copy, as stored: the plain layout (FP64) has the npop
// population planes; the paired layout (2- and 4-byte elements) has npop / 2
// planes of population pairs, then (deviation formats) one pair plane of
// references as wide as the populations, or two planes of wider ones.
bool paired(const Layout &L) { return L.es == 2 || L.es == 4; }
bool refs_in_pair(const Layout &L) { return L.planes == L.npop + 2 && L.rs == L.es; }
size_t phys_planes(const Layout &L) {
    if (!paired(L)) return L.planes;
    return L.npop / 2 + (L.planes == L.npop + 2 ? (refs_in_pair(L) ? 1 : 2) : 0);
}
size_t plane_offset(const Layout &L, size_t k) {
    const size_t np = L.npop;
    if (paired(L)) {
        if (k < np / 2 || refs_in_pair(L)) return k * L.stride * 2 * L.es;
        return np * L.stride * L.es + (k - np / 2) * L.stride * L.rs;
    }
    return k < np ? k * L.stride * L.es : np * L.stride * L.es + (k - np) * L.stride * L.rs;
}
size_t plane_bytes(const Layout &L, size_t k) {
    if (paired(L)) return (k < L.npop / 2 || refs_in_pair(L)) ? L.nn * 2 * L.es : L.nn * L.rs;
    return L.nn * (k < L.npop ? L.es : L.rs);
}

// Elements between consecutive population planes.  On large grids the
// planes are not left a power of two apart: the 14 to 26 planes a wavefront
// streams at once would then start at the same offset modulo the HBM
// interleave, and at 512^3 (2^27 nodes) a pad of 32832 elements measured 2%
// (FP16) and 10% (FP32) faster than none; pads near 64 K elements measured
// slower.  Small lattices (the batch) keep the plain stride.
constexpr size_t kPlanePad = 32832;

size_t plane_stride(size_t nn) {
    const size_t s = align_up(nn, 128);
    return nn >= ((size_t)1 << 22) ? s + kPlanePad : s;
}

Layout make_layout(const lbm_params *p) {
    Layout L;
    L.nn = (size_t)p->nx * p->ny * p->nz;
    L.es = element_bytes(p->storage);
    L.cs = p->storage == LBM_STORE_F64 ? 8 : 4;
    L.rs = reference_bytes(p->storage);
    L.qt = thermal_q(p);
    L.npop = 19 + L.qt;
    L.planes = planes_of(p->storage, L.qt);
    L.stride = plane_stride(L.nn);
    // Each ping-pong copy holds its planes contiguously, `stride` elements
    // apart: f_0..f_18, g_0..g_{QT-1}, then (deviation formats) rho_r and T_r.
    size_t off = 0;
    for (int k = 0; k < 2; ++k) {
        L.off_pop[k] = off;
        off = align_up(off + copy_bytes(L), kAlign);
    }
    L.off_phi = off;
    off = align_up(off + L.stride * L.cs, kAlign);
    L.off_stage = off;
    off = align_up(off + 6 * L.nn * sizeof(double), kAlign);
    L.max_partials = max_workgroups(p);
    L.off_part = off;
    off = align_up(off + 2 * L.max_partials * sizeof(double), kAlign);
    L.off_scal = off;
    off = align_up(off + 64 * sizeof(double), kAlign);
    // virtual density and psi of the solid layer below a bottom wall (walls only)
    L.off_wall = off;
    if (p->bc_z != LBM_BC_PERIODIC) off = align_up(off + 2 * (size_t)p->nx * p->ny * sizeof(double), kAlign);
    L.total = off;
    return L;
}

// Squared radius of the wettability disc (0: none), for k_wall_density.
double disc_r2(const lbm_params &p) { return 0.25 * p.wet_disc * p.wet_disc; }

template <typename C>
lbm::Phys<C> make_phys(const lbm_params *p) {
    lbm::Phys<C> P;
    const double w = p->acentric;
    const double Tc = (p->a != 0.0) ? 0.0778 / 0.45724 * p->a / (p->b * p->R) : 1.0;
    P.a = (C)p->a;
    P.b = (C)p->b;
    P.R = (C)p->R;
    P.kap = (C)(0.37464 + 1.54226 * w - 0.26992 * w * w);
    P.inv_Tc = (C)(1.0 / Tc);
    P.two_over_Gc2 = (C)(2.0 / p->G);
    P.negG = (C)(-p->G);
    P.sig6 = (C)(6.0 * p->sigma / (p->tau_e - 0.5));
    P.lam_e = (C)(1.0 / p->tau_e);
    P.lam_v = (C)(1.0 / p->tau_v);
    P.lam_q = (C)(1.0 / p->tau_q);
    P.lam_pi = (C)(1.0 / p->tau_pi);
    P.divu_a = (C)(1.0 / p->tau_e);
    P.divu_b = (C)(1.0 - 1.0 / (2.0 * p->tau_e));
    P.cV = (C)p->cV;
    P.inv_cV = (C)(1.0 / p->cV);
    if (thermal_q(p) == 7) {
        // Sec. III B, Eq. (22): w0 = 1 - d, w1..6 = d/6, c_sT^2 = d/3.
        P.wT0 = (C)(1.0 - p->d);
        P.wT1 = (C)(p->d / 6.0);
        P.csT2 = (C)(p->d / 3.0);
        P.inv_csT2 = (C)(3.0 / p->d);
    } else {
        // D3Q19: the standard weights and c_sT^2 = c_s^2 = 1/3.
        P.wT0 = (C)(1.0 / 3.0);
        P.wT1 = (C)(1.0 / 18.0);
        P.csT2 = (C)(1.0 / 3.0);
        P.inv_csT2 = (C)3.0;
    }
    P.d = (C)p->d;
    P.kappa = (C)p->kappa;
    P.gam_q = (C)(1.0 / p->vs_q);
    P.gam_pi = (C)(1.0 / p->vs_pi);
    P.gx = (C)p->g[0];
    P.gy = (C)p->g[1];
    P.gz = (C)p->g[2];
    P.kappa_mode = p->kappa_mode;
    P.thermal = p->thermal;
    P.shell = p->bc_T_shell;
    P.thermal_bgk = p->thermal_bgk;
    P.T_shell = (C)p->T_shell;
    P.attract = p->a != 0.0;
    P.gravity = (p->g[0] != 0.0 || p->g[1] != 0.0 || p->g[2] != 0.0);
    P.T_patch = p->T_wall_patch;
    P.T_wall = p->T_wall;
    P.patch_r2 = p->patch_radius * p->patch_radius;
    P.T_top = p->T_top;
    P.cx = 0.5 * (p->nx - 1);
    P.cy = 0.5 * (p->ny - 1);
    P.top_wall = p->bc_z == LBM_BC_WALLS;
    P.wet = p->bc_z != LBM_BC_PERIODIC && p->wet_mode == LBM_WET_VIRTUAL_DENSITY;
    P.wet_phi = p->wet_phi;
    P.wet_phi_in = p->wet_phi_in;
    P.wet_drho = p->wet_drho;
    P.wet_square = p->wet_square;
    return P;
}

struct StateHeader {
    char magic[8];
    int32_t version, nx, ny, nz, storage, planes;
    uint64_t nn, es, cs;
};
constexpr int32_t kStateVersion = 3;

// Calls fn with a value of the format type of `storage` for a temperature
// lattice of QT velocities.
template <int QT, typename Fn>
int with_format_q(int storage, Fn &&fn) {
    switch (storage) {
    case LBM_STORE_F32: return fn(lbm::Fmt<lbm::StoreF32, QT>{});
    case LBM_STORE_F64: return fn(lbm::Fmt<lbm::StoreF64, QT>{});
    case LBM_STORE_F16: return fn(lbm::Fmt<lbm::StoreF16, QT>{});
    }
    if constexpr (QT == 7) {  // the comparison formats are built for D3Q7 only
        if (storage == LBM_STORE_BF16) return fn(lbm::Fmt<lbm::StoreBF16, QT>{});
        if (storage == LBM_STORE_F32_DEV) return fn(lbm::Fmt<lbm::StoreF32Dev, QT>{});
    }
    return LBM_EINVAL;
}

// The same for a lattice's own storage format and temperature lattice.
template <typename Fn>
int with_format(const lbm_params &p, Fn &&fn) {
    if (thermal_q(&p) == 19) return with_format_q<19>(p.storage, fn);
    return with_format_q<7>(p.storage, fn);
}

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch of lbm_reduce_static, the allocation-free variant of
// lbm_reduce: its per-block partial sums of rho and T ([kScratchResults, ...))
// and its two results ([0] mass, [1] energy) live in this file-scope device
// array instead of the handle's arena.  Each GPU the library runs on holds
// its own copy until the process ends.  Host code never names `scratch` in a
// launch or a copy (on the host that name is not a device address): the
// address of each device's copy is looked up once, with that device current,
// at the first lbm_create on it, and kept in scratch_ptr[device].  Every call
// writes the entries it reads (nothing must start at zero); calls that
// overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
constexpr size_t kScratchDoubles = (size_t)1 << 21;  // 16 MiB a device
constexpr size_t kScratchResults = 8;                // results first, partial sums after them
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double *scratch_ptr[kMaxDevices];

// The address of `device`'s copy of the scratch array (the device is current).
int scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return LBM_EHIP;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptr[device]) return LBM_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_EHIP;
    scratch_ptr[device] = (double *)ptr;
    return LBM_OK;
}

double *scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    return scratch_ptr[device];
}

}  // namespace

struct lbm_handle {
    lbm_params p;
    Layout L;
    hipStream_t stream;
    // Device regions: a lattice of its own has them all in its arena; the
    // lattices of a batch share the staging planes and partial sums.
    char *r_pop[2], *r_phi, *r_scal;
    double *r_wall;   // walls: rho_w and psi_w of the solid layer (null for periodic grids)
    double *r_stage, *r_part;
    int cur;          // which population copy holds the state
    int initialized;
    int tile_x, tile_y, chunk_z;
    int workgroups;
    int device;               // HIP device current at lbm_create (the arena's)
    hipGraphExec_t exec[2];   // two steps starting from copy 0 / copy 1 (lbm_step on a stream)
    unsigned *status() { return (unsigned *)(r_scal + 8 * sizeof(double)); }
    double *rho_ave() { return (double *)r_scal; }
    double *mass() { return (double *)(r_scal + sizeof(double)); }
    double *energy() { return (double *)(r_scal + 2 * sizeof(double)); }
    double *stage() { return r_stage; }
    double *partials() { return r_part; }
    void *pop(int k) { return r_pop[k]; }
    void *phi() { return r_phi; }
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EHIP; }

// Default launch shape (measured on MI355X): 64x8 tiles where the rows are
// long enough (their halo is 29% of the tile against 52% for 128x4 or 64x4;
// FP32 at 128^3 / 192^3 / 256^3 / the 256x256x384 pool: 1-13% faster than
// 128x4 tiles, FP16 2-4% faster than 32x16 except at 128^3; at 512^3 16-bit
// storage runs 2% faster in whole 128-node rows), and chunks of up to 64
// planes; the z halo of a chunk is read twice, so chunks are kept long
// (64 planes: 2-3% faster than 32 at 512^3 and on the pool) unless the grid
// would then give fewer workgroups than the 256 compute units.
bool buffer_path(const Layout &L);

void set_default_launch(lbm_handle *h) {
    const int nx = h->p.nx, ny = h->p.ny, nz = h->p.nz;
    const bool half = h->L.es == 2;
    if (nx >= 64) {
        h->tile_x = 64;
        h->tile_y = 8;
    } else if (nx > 32) {
        h->tile_x = 64;
        h->tile_y = 4;
    } else {
        h->tile_x = 32;
        h->tile_y = 8;
    }
    if (h->L.qt == 19 && nx > 32) {
        // D3Q19 temperature lattice (measured at 128^3): FP32 holds its 38
        // populations per node without spilling only in 256-thread tiles;
        // FP16 runs best with whole 128-node rows.
        h->tile_x = (half && nx >= 96) ? 128 : 64;
        h->tile_y = 4;
    }
    if (h->p.storage == LBM_STORE_F64 && h->tile_x * h->tile_y != 256) {
        h->tile_x = nx > 32 ? 64 : 32;
        h->tile_y = nx > 32 ? 4 : 8;
    }
    const long tiles = (long)((nx + h->tile_x - 1) / h->tile_x) * ((ny + h->tile_y - 1) / h->tile_y);
    // Chunk depth: the one that minimises the waves of workgroups times the
    // planes each workgroup marches (plus 3 for the pipeline's start), with
    // as many workgroups in flight as the 256 compute units hold: one of 512
    // threads each, or two of 256 (one where a 256-thread step needs more
    // than 256 registers a lane: the D3Q19 temperature lattice, FP64).  This takes the longest chunks at about one workgroup
    // per compute unit where the tiles divide the grid well (512^3: whole
    // 512-plane columns, -2% against chunks of 64 planes; the 256x256x384
    // wall grid: 192 planes, -9% FP16, -10% FP32) and avoids a partial
    // last wave where they do not (200x200x100: 20 planes, 500 workgroups,
    // rather than 39 planes and 300).  Grids on the plain-pointer path in 4-
    // or 8-byte storage stop at 64 planes (512^3 FP32: 6.46 ms with 64, 6.63
    // ms with 256, 6.67 ms with 512).
    const bool one_per_cu = h->tile_x * h->tile_y >= 512 || h->L.qt == 19 || h->p.storage == LBM_STORE_F64;
    const long resident = one_per_cu ? 256L : 512L;
    const long cap = (!half && !buffer_path(h->L)) ? (nz < 64 ? nz : 64) : nz;
    long cz = 1;
    double best = 1e300;
    for (long c = 1; c <= cap; ++c) {
        const long wg = tiles * ((nz + c - 1) / c);
        const double cost = (double)((wg + resident - 1) / resident) * (double)(c + 3);
        if (cost <= best) {
            best = cost;
            cz = c;
        }
    }
    h->chunk_z = (int)cz;
}

int workgroups_for(const lbm_handle *h, int tx, int ty, int cz) {
    const long n = (long)((h->p.nx + tx - 1) / tx) * ((h->p.ny + ty - 1) / ty) * ((h->p.nz + cz - 1) / cz);
    return (int)n;
}

// The buffer-resource path addresses each half of a copy's planes (split at
// plane 14; 20 with the D3Q19 temperature lattice) with 32-bit offsets.
size_t split_low_bytes(const Layout &L) {
    const size_t split = L.qt == 19 ? lbm::PopLayout<19>::kSplit : lbm::PopLayout<7>::kSplit;
    return split * L.stride * L.es;
}
bool buffer_path(const Layout &L) {
    const size_t lo = split_low_bytes(L);
    const size_t hi = copy_bytes(L) - lo;
    return lo <= 0xFFFFFFFFull && hi <= 0xFFFFFFFFull;
}
// Record counts of the two buffer resources of a copy (unused with plain pointers).
void set_buffer_extents(const Layout &L, unsigned &lo, unsigned &hi) {
    lo = hi = 0;
    if (!buffer_path(L)) return;
    lo = (unsigned)split_low_bytes(L);
    hi = (unsigned)(copy_bytes(L) - split_low_bytes(L));
}

template <typename ST, int TX, int TY, bool WALLS>
int launch_step_t(lbm_handle *h, const lbm::StepArgs<ST> &A, int nb) {
    if (buffer_path(h->L))
        hipLaunchKernelGGL((lbm::k_step<ST, TX, TY, WALLS, true, false>), dim3(nb), dim3(TX * TY), 0, h->stream, A);
    else
        hipLaunchKernelGGL((lbm::k_step<ST, TX, TY, WALLS, false, false>), dim3(nb), dim3(TX * TY), 0, h->stream, A);
    return hip_status(hipGetLastError());
}

// The finite-difference divergence is built for the FP32, FP64 and FP16
// formats, 256-thread tiles and the buffer-resource path (checked when the
// parameters and the launch shape are set).
template <typename ST>
constexpr bool fd_built() {
    return !std::is_same<typename ST::T, __bf16>::value && !(ST::kDev && sizeof(typename ST::T) == 4);
}

// A step with the finite-difference divergence is two launches of the same
// shape: the velocity pass (u(t) of every node into the staging region) and
// the step that reads it.
template <typename ST, int TX, int TY, bool WALLS>
int launch_fd_t(lbm_handle *h, const lbm::StepArgs<ST> &A, int nb) {
    hipLaunchKernelGGL((lbm::k_velocity_pass<ST, TX, TY, WALLS, true>), dim3(nb), dim3(TX * TY), 0, h->stream, A);
    hipLaunchKernelGGL((lbm::k_step<ST, TX, TY, WALLS, true, true>), dim3(nb), dim3(TX * TY), 0, h->stream, A);
    return hip_status(hipGetLastError());
}

template <typename ST, bool WALLS>
int launch_step_fd(lbm_handle *h, const lbm::StepArgs<ST> &A, int nb) {
    if constexpr (fd_built<ST>()) {
        if (!buffer_path(h->L)) return LBM_EINVAL;
        const int tx = h->tile_x, ty = h->tile_y;
        if (tx == 64 && ty == 4) return launch_fd_t<ST, 64, 4, WALLS>(h, A, nb);
        if (tx == 32 && ty == 8) return launch_fd_t<ST, 32, 8, WALLS>(h, A, nb);
        if constexpr (sizeof(typename ST::C) == 4) {
            if (tx == 64 && ty == 8) return launch_fd_t<ST, 64, 8, WALLS>(h, A, nb);
            if (tx == 32 && ty == 16) return launch_fd_t<ST, 32, 16, WALLS>(h, A, nb);
            if (tx == 128 && ty == 4) return launch_fd_t<ST, 128, 4, WALLS>(h, A, nb);
        }
        return LBM_EINVAL;
    } else {
        return LBM_EINVAL;
    }
}

// FP32-arithmetic formats instantiate every tile shape; the FP64 build (used
// to check the kernel against the FP64 oracle) only the two 256-thread tiles,
// which fit its registers without spilling.
template <typename ST, bool WALLS>
int launch_step_tile(lbm_handle *h, const lbm::StepArgs<ST> &A, int nb) {
    if (h->p.divu_mode == LBM_DIVU_FD) return launch_step_fd<ST, WALLS>(h, A, nb);
    const int tx = h->tile_x, ty = h->tile_y;
    if (tx == 64 && ty == 4) return launch_step_t<ST, 64, 4, WALLS>(h, A, nb);
    if (tx == 32 && ty == 8) return launch_step_t<ST, 32, 8, WALLS>(h, A, nb);
    if constexpr (sizeof(typename ST::C) == 4) {
        if (tx == 64 && ty == 8) return launch_step_t<ST, 64, 8, WALLS>(h, A, nb);
        if (tx == 32 && ty == 16) return launch_step_t<ST, 32, 16, WALLS>(h, A, nb);
        if (tx == 128 && ty == 4) return launch_step_t<ST, 128, 4, WALLS>(h, A, nb);
    }
    return LBM_EINVAL;
}

template <typename ST>
int step_once(lbm_handle *h) {
    using T = typename ST::T;
    using C = typename ST::C;
    lbm::StepArgs<ST> A;
    const int c = h->cur, n = 1 - c;
    A.pop_in = (const T *)h->pop(c);
    A.pop_out = (T *)h->pop(n);
    A.phi = (C *)h->phi();
    A.rho_ave = h->rho_ave();
    A.partials = h->partials();
    A.status = h->status();
    A.stride = h->L.stride;
    set_buffer_extents(h->L, A.buf_lo_bytes, A.buf_hi_bytes);
    A.nx = h->p.nx;
    A.ny = h->p.ny;
    A.nz = h->p.nz;
    A.ntx = (h->p.nx + h->tile_x - 1) / h->tile_x;
    A.nty = (h->p.ny + h->tile_y - 1) / h->tile_y;
    A.tile_x = h->tile_x;
    A.tile_y = h->tile_y;
    A.cz = h->chunk_z;
    A.P = make_phys<C>(&h->p);
    A.wall = h->r_wall;
    // u(t) planes of the finite-difference divergence: the staging region
    // (six FP64 planes) holds the three planes in the compute type.
    A.uout = (C *)h->stage();
    A.ustage = A.uout;
    A.unn = h->L.nn;
    const int nb = h->workgroups;
    if (A.P.wet) {
        // virtual density of the wall's solid layer from the state at time t
        const size_t nxy = (size_t)h->p.nx * h->p.ny;
        hipLaunchKernelGGL(lbm::k_wall_density<ST>, dim3((unsigned)((nxy + 255) / 256)), dim3(256), 0, h->stream,
                           (const T *)h->pop(c), h->L.stride, h->p.nx, h->p.ny, make_phys<double>(&h->p),
                           disc_r2(h->p), h->r_wall, h->status());
    }
    int rc = h->p.bc_z != LBM_BC_PERIODIC ? launch_step_tile<ST, true>(h, A, nb) : launch_step_tile<ST, false>(h, A, nb);
    if (rc) return rc;
    if (A.P.gravity) {
        hipLaunchKernelGGL(lbm::k_finish, dim3(1), dim3(256), 0, h->stream, (const double *)h->partials(), nb, 1, 0,
                           1.0 / (double)h->L.nn, h->rho_ave());
        rc = hip_status(hipGetLastError());
        if (rc) return rc;
    }
    h->cur = n;
    return LBM_OK;
}

// Captured graphs of two steps (from copy `from` back to it).  They hold the
// launch shape, so lbm_set_launch drops them.
void drop_step_graphs(lbm_handle *h) {
    for (int k = 0; k < 2; ++k) {
        if (h->exec[k]) (void)hipGraphExecDestroy(h->exec[k]);
        h->exec[k] = nullptr;
    }
}

int step_graph(lbm_handle *h, int from) {
    if (h->exec[from]) return LBM_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return LBM_EHIP;
    int rc = LBM_OK;
    for (int k = 0; k < 2 && !rc; ++k)
        rc = with_format(h->p, [&](auto fmt) { return step_once<decltype(fmt)>(h); });
    const hipError_t e = hipStreamEndCapture(h->stream, &g);
    h->cur = from;  // capture launches nothing; the two steps end where they began
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : LBM_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&h->exec[from], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) h->exec[from] = nullptr;
    return hip_status(ei);
}

// Sum rho and T of the current state into mass/energy (and optionally rho_ave).
template <typename ST>
int reduce_state(lbm_handle *h, bool set_rho_ave) {
    using T = typename ST::T;
    const size_t nn = h->L.nn;
    const int nb = (int)((nn + 255) / 256);
    hipLaunchKernelGGL(lbm::k_sum<ST>, dim3(nb), dim3(256), 0, h->stream, (const T *)h->pop(h->cur), h->L.stride, nn,
                       h->partials());
    hipLaunchKernelGGL(lbm::k_finish, dim3(1), dim3(256), 0, h->stream, (const double *)h->partials(), nb, 2, 0, 1.0,
                       h->mass());
    hipLaunchKernelGGL(lbm::k_finish, dim3(1), dim3(256), 0, h->stream, (const double *)h->partials(), nb, 2, 1, 1.0,
                       h->energy());
    if (set_rho_ave)
        hipLaunchKernelGGL(lbm::k_finish, dim3(1), dim3(256), 0, h->stream, (const double *)h->partials(), nb, 2, 0,
                           1.0 / (double)nn, h->rho_ave());
    return hip_status(hipGetLastError());
}

int check_status(lbm_handle *h, unsigned *out) {
    unsigned st = 0;
    hipError_t e = hipMemcpyAsync(&st, h->status(), sizeof(unsigned), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return LBM_EHIP;
    *out = st;
    return LBM_OK;
}

int clear_status(lbm_handle *h) {
    return hip_status(hipMemsetAsync(h->status(), 0, sizeof(unsigned), h->stream));
}

}  // namespace

extern "C" {

size_t lbm_arena_bytes(const lbm_params *p) {
    if (!valid_params(p)) return 0;
    return make_layout(p).total;
}

int lbm_create(const lbm_params *p, void *dev_arena, size_t arena_bytes, void *hip_stream, lbm_handle **out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!valid_params(p) || !dev_arena) return LBM_EINVAL;
    const Layout L = make_layout(p);
    if (arena_bytes < L.total || ((uintptr_t)dev_arena % kAlign) != 0) return LBM_ENOMEM;
    lbm_handle *h = (lbm_handle *)calloc(1, sizeof(lbm_handle));
    if (!h) return LBM_ENOMEM;
    h->p = *p;
    h->L = L;
    h->stream = (hipStream_t)hip_stream;
    char *arena = (char *)dev_arena;
    h->r_pop[0] = arena + L.off_pop[0];
    h->r_pop[1] = arena + L.off_pop[1];
    h->r_phi = arena + L.off_phi;
    h->r_scal = arena + L.off_scal;
    h->r_stage = (double *)(arena + L.off_stage);
    h->r_part = (double *)(arena + L.off_part);
    h->r_wall = p->bc_z != LBM_BC_PERIODIC ? (double *)(arena + L.off_wall) : nullptr;
    h->cur = 0;
    h->initialized = 0;
    set_default_launch(h);
    h->workgroups = workgroups_for(h, h->tile_x, h->tile_y, h->chunk_z);
    int rc = hip_status(hipGetDevice(&h->device));
    if (!rc) rc = scratch_setup(h->device);
    if (!rc) rc = clear_status(h);
    if (rc) {
        free(h);
        return rc;
    }
    *out = h;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Initial state into population copy `copy` (which then holds the state).
int init_state(lbm_handle *h, const double *rho, const double *ux, const double *uy, const double *uz,
               const double *T, int copy) {
    const size_t nn = h->L.nn, bytes = nn * sizeof(double);
    double *st = h->stage();
    const double *src[5] = {rho, ux, uy, uz, T};
    for (int k = 0; k < 5; ++k) {
        hipError_t e = hipMemcpyAsync(st + k * nn, src[k], bytes, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) return LBM_EHIP;
    }
    int rc = clear_status(h);
    if (rc) return rc;
    const lbm::Phys<double> P = make_phys<double>(&h->p);
    const int nb = (int)((nn + 255) / 256);
    h->cur = copy;
    rc = with_format(h->p, [&](auto fmt) {
        using ST = decltype(fmt);
        hipLaunchKernelGGL(lbm::k_init<ST>, dim3(nb), dim3(256), 0, h->stream, (const double *)st, nn,
                           (typename ST::T *)h->pop(copy), (typename ST::C *)h->phi(), h->L.stride, P, h->status());
        return reduce_state<ST>(h, true);
    });
    if (rc) return rc;
    unsigned s = 0;
    rc = check_status(h, &s);
    if (rc) return rc;
    if (s & 2u) {
        h->initialized = 0;
        clear_status(h);
        return LBM_EINVAL;
    }
    h->initialized = 1;
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_init_fields(lbm_handle *h, const double *rho, const double *ux, const double *uy, const double *uz,
                    const double *T) {
    if (!h || !rho || !ux || !uy || !uz || !T) return LBM_EINVAL;
    return init_state(h, rho, ux, uy, uz, T, 0);
}

int lbm_step(lbm_handle *h, int n) {
    if (!h || n < 0) return LBM_EINVAL;
    if (!h->initialized) return LBM_ESTATE;
    if (h->stream && n >= 2) {
        // Pairs of steps as graph replays, unless the caller is capturing
        // this stream itself (then the launches go into the caller's graph).
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(h->stream, &cs) != hipSuccess) return LBM_EHIP;
        if (cs == hipStreamCaptureStatusNone) {
            for (; n >= 2; n -= 2) {
                int rc = step_graph(h, h->cur);
                if (!rc) rc = hip_status(hipGraphLaunch(h->exec[h->cur], h->stream));
                if (rc) return rc;
            }
        }
    }
    for (int k = 0; k < n; ++k) {
        const int rc = with_format(h->p, [&](auto fmt) { return step_once<decltype(fmt)>(h); });
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_get_rho_u_T(lbm_handle *h, double *rho, double *ux, double *uy, double *uz, double *T) {
    if (!h || !rho || !ux || !uy || !uz || !T) return LBM_EINVAL;
    if (!h->initialized) return LBM_ESTATE;
    const size_t nn = h->L.nn;
    const int nb = (int)((nn + 255) / 256);
    const lbm::Phys<double> P = make_phys<double>(&h->p);
    double *st = h->stage();
    const int walls = h->p.bc_z != LBM_BC_PERIODIC;
    const lbm::Phys<double> Pw = make_phys<double>(&h->p);
    const int lrc = with_format(h->p, [&](auto fmt) {
        using ST = decltype(fmt);
        const typename ST::T *pop = (const typename ST::T *)h->pop(h->cur);
        if (Pw.wet) {
            const size_t nxy = (size_t)h->p.nx * h->p.ny;
            hipLaunchKernelGGL(lbm::k_wall_density<ST>, dim3((unsigned)((nxy + 255) / 256)), dim3(256), 0, h->stream,
                               pop, h->L.stride, h->p.nx, h->p.ny, Pw, disc_r2(h->p), h->r_wall, h->status());
        }
        hipLaunchKernelGGL(lbm::k_macro<ST>, dim3(nb), dim3(256), 0, h->stream, pop, h->L.stride, nn, P, st);
        hipLaunchKernelGGL(lbm::k_velocity<ST>, dim3(nb), dim3(256), 0, h->stream, pop, h->L.stride, h->p.nx, h->p.ny,
                           h->p.nz, walls, P, (const double *)h->rho_ave(), (const double *)(Pw.wet ? h->r_wall : nullptr),
                           st);
        return hip_status(hipGetLastError());
    });
    if (lrc) return lrc;
    double *dst[5] = {rho, ux, uy, uz, T};
    for (int k = 0; k < 5; ++k) {
        if (hipMemcpyAsync(dst[k], st + k * nn, nn * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
            return LBM_EHIP;
    }
    unsigned s = 0;
    const int rc = check_status(h, &s);
    if (rc) return rc;
    if (s & 1u) {
        clear_status(h);
        return LBM_EUNSTABLE;
    }
    return LBM_OK;
}

int lbm_reduce(lbm_handle *h, double *mass, double *energy) {
    if (!h || !mass || !energy) return LBM_EINVAL;
    if (!h->initialized) return LBM_ESTATE;
    int rc = with_format(h->p, [&](auto fmt) { return reduce_state<decltype(fmt)>(h, false); });
    if (rc) return rc;
    double me[2];
    if (hipMemcpyAsync(me, h->mass(), 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return LBM_EHIP;
    unsigned s = 0;
    rc = check_status(h, &s);
    if (rc) return rc;
    *mass = me[0];
    *energy = me[1];
    if (s & 1u) {
        clear_status(h);
        return LBM_EUNSTABLE;
    }
    return LBM_OK;
}

int lbm_reduce_static(lbm_handle *h, double *mass, double *energy) {
    if (!h || !mass || !energy) return LBM_EINVAL;
    const size_t nb = (h->L.nn + 255) / 256;
    if (2 * nb > kScratchDoubles - kScratchResults) return LBM_ESCRATCH;
    if (!h->initialized) return LBM_ESTATE;
    double *sp = scratch_of(h->device);
    if (!sp) return LBM_EHIP;
    // The kernels and block order of lbm_reduce, with the static scratch in
    // place of the arena's partial sums and scalars.
    int rc = with_format(h->p, [&](auto fmt) {
        using ST = decltype(fmt);
        hipLaunchKernelGGL(lbm::k_sum<ST>, dim3((unsigned)nb), dim3(256), 0, h->stream,
                           (const typename ST::T *)h->pop(h->cur), h->L.stride, h->L.nn, sp + kScratchResults);
        hipLaunchKernelGGL(lbm::k_finish, dim3(1), dim3(256), 0, h->stream, (const double *)(sp + kScratchResults),
                           (int)nb, 2, 0, 1.0, sp);
        hipLaunchKernelGGL(lbm::k_finish, dim3(1), dim3(256), 0, h->stream, (const double *)(sp + kScratchResults),
                           (int)nb, 2, 1, 1.0, sp + 1);
        return hip_status(hipGetLastError());
    });
    if (rc) return rc;
    double me[2];
    if (hipMemcpyAsync(me, sp, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess) return LBM_EHIP;
    unsigned s = 0;
    rc = check_status(h, &s);
    if (rc) return rc;
    *mass = me[0];
    *energy = me[1];
    if (s & 1u) {
        clear_status(h);
        return LBM_EUNSTABLE;
    }
    return LBM_OK;
}

size_t lbm_state_bytes(const lbm_handle *h) {
    if (!h) return 0;
    const size_t nn = h->L.nn;
    size_t planes = 0;
    for (size_t a = 0; a < phys_planes(h->L); ++a) planes += plane_bytes(h->L, a);
    return sizeof(StateHeader) + planes + nn * h->L.cs + sizeof(double);
}

int lbm_get_state(lbm_handle *h, void *host_buf, size_t bytes) {
    if (!h || !host_buf || bytes != lbm_state_bytes(h)) return LBM_EINVAL;
    if (!h->initialized) return LBM_ESTATE;
    StateHeader hd;
    memset(&hd, 0, sizeof(hd));
    memcpy(hd.magic, "LBMSTAT1", 8);
    hd.version = kStateVersion;
    hd.planes = (int32_t)phys_planes(h->L);
    hd.nx = h->p.nx;
    hd.ny = h->p.ny;
    hd.nz = h->p.nz;
    hd.storage = h->p.storage;
    hd.nn = h->L.nn;
    hd.es = h->L.es;
    hd.cs = h->L.cs;
    char *out = (char *)host_buf;
    memcpy(out, &hd, sizeof(hd));
    out += sizeof(hd);
    for (size_t a = 0; a < phys_planes(h->L); ++a) {
        const size_t bytes = plane_bytes(h->L, a);
        if (hipMemcpyAsync(out, (char *)h->pop(h->cur) + plane_offset(h->L, a), bytes, hipMemcpyDeviceToHost,
                           h->stream) != hipSuccess)
            return LBM_EHIP;
        out += bytes;
    }
    if (hipMemcpyAsync(out, h->phi(), h->L.nn * h->L.cs, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return LBM_EHIP;
    out += h->L.nn * h->L.cs;
    if (hipMemcpyAsync(out, h->rho_ave(), sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return LBM_EHIP;
    unsigned s = 0;
    const int rc = check_status(h, &s);
    if (rc) return rc;
    if (s & 1u) {
        clear_status(h);
        return LBM_EUNSTABLE;
    }
    return LBM_OK;
}

int lbm_set_state(lbm_handle *h, const void *host_buf, size_t bytes) {
    if (!h || !host_buf || bytes != lbm_state_bytes(h)) return LBM_EINVAL;
    StateHeader hd;
    memcpy(&hd, host_buf, sizeof(hd));
    if (memcmp(hd.magic, "LBMSTAT1", 8) != 0 || hd.version != kStateVersion || hd.nx != h->p.nx ||
        hd.ny != h->p.ny || hd.nz != h->p.nz || hd.storage != h->p.storage || hd.planes != (int32_t)phys_planes(h->L) ||
        hd.nn != h->L.nn || hd.es != h->L.es || hd.cs != h->L.cs)
        return LBM_EINVAL;
    const char *in = (const char *)host_buf + sizeof(hd);
    h->cur = 0;
    for (size_t a = 0; a < phys_planes(h->L); ++a) {
        const size_t bytes = plane_bytes(h->L, a);
        if (hipMemcpyAsync((char *)h->pop(0) + plane_offset(h->L, a), in, bytes, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess)
            return LBM_EHIP;
        in += bytes;
    }
    if (hipMemcpyAsync(h->phi(), in, h->L.nn * h->L.cs, hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return LBM_EHIP;
    in += h->L.nn * h->L.cs;
    if (hipMemcpyAsync(h->rho_ave(), in, sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return LBM_EHIP;
    int rc = clear_status(h);
    if (rc) return rc;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBM_EHIP;
    h->initialized = 1;
    return LBM_OK;
}

int lbm_set_launch(lbm_handle *h, int tile_x, int tile_y, int chunk_z) {
    if (!h || chunk_z < 1 || chunk_z > kMaxChunk) return LBM_EINVAL;
    bool ok = false;
    for (const TileShape &t : kTiles) ok = ok || (t.tx == tile_x && t.ty == tile_y);
    if (h->p.storage == LBM_STORE_F64) ok = ok && tile_x * tile_y == 256;
    if (!ok) return LBM_EINVAL;
    const int cz = chunk_z > h->p.nz ? h->p.nz : chunk_z;
    const int nb = workgroups_for(h, tile_x, tile_y, cz);
    if ((size_t)nb > h->L.max_partials) return LBM_EINVAL;
    h->tile_x = tile_x;
    h->tile_y = tile_y;
    h->chunk_z = cz;
    h->workgroups = nb;
    drop_step_graphs(h);
    return LBM_OK;
}

int lbm_get_launch(const lbm_handle *h, int *tile_x, int *tile_y, int *chunk_z, int *workgroups) {
    if (!h || !tile_x || !tile_y || !chunk_z || !workgroups) return LBM_EINVAL;
    *tile_x = h->tile_x;
    *tile_y = h->tile_y;
    *chunk_z = h->chunk_z;
    *workgroups = h->workgroups;
    return LBM_OK;
}

int lbm_launches_per_step(const lbm_handle *h) {
    if (!h) return 0;
    return ((h->p.g[0] != 0.0 || h->p.g[1] != 0.0 || h->p.g[2] != 0.0) ? 2 : 1) +
           (h->p.divu_mode == LBM_DIVU_FD ? 1 : 0) +
           ((h->p.bc_z != LBM_BC_PERIODIC && h->p.wet_mode == LBM_WET_VIRTUAL_DENSITY) ? 1 : 0);
}

void lbm_destroy(lbm_handle *h) {
    if (!h) return;
    drop_step_graphs(h);
    free(h);
}

const char *lbm_strerror(int status) {
    switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "arena too small or misaligned";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_EUNSTABLE: return "unstable state (rho <= 0, psi^2 < 0 or NaN)";
    case LBM_ESTATE: return "call out of order";
    case LBM_ESCRATCH: return "grid larger than the static scratch of lbm_reduce_static";
    }
    return "unknown status";
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent lattices.
// ---------------------------------------------------------------------------

struct lbm_batch {
    int n;
    int storage;
    hipStream_t stream;
    lbm_handle *cases;     // per-lattice handles (regions inside the batch arena)
    int *order;            // lattices by decreasing node count (work-list order)
    // shared device regions
    char *d_desc;          // StepArgs of every lattice
    unsigned *d_item_case, *d_first_item, *d_queue;
    char *d_phi_backup;    // copy of all phi_s planes (autotuner)
    size_t max_items;
    int cus;               // compute units of the device
    // launch
    int tile_x, tile_y, chunk_z, workgroups;
    unsigned n_items;
    unsigned bin_start[lbm::kXcds + 1];  // item ranges of the XCDs
    int cur;               // population copy holding the state of every lattice
    hipGraphExec_t exec[2];  // two steps starting from copy 0 / copy 1
};

namespace {

constexpr size_t kDescBytes = sizeof(lbm::StepArgs<lbm::StoreF64>) > sizeof(lbm::StepArgs<lbm::StoreF32>)
                                  ? sizeof(lbm::StepArgs<lbm::StoreF64>)
                                  : sizeof(lbm::StepArgs<lbm::StoreF32>);

bool valid_batch(const lbm_params *cases, int n) {
    if (!cases || n < 1 || n > 65536) return false;
    for (int c = 0; c < n; ++c) {
        const lbm_params *p = cases + c;
        if (!valid_params(p) || p->storage != cases[0].storage || p->bc_z != LBM_BC_PERIODIC) return false;
        if (p->g[0] != 0.0 || p->g[1] != 0.0 || p->g[2] != 0.0) return false;
        if (p->thermal_lattice != LBM_THERMAL_D3Q7) return false;  // the batched kernel is built for D3Q7
        if (p->divu_mode != LBM_DIVU_LOCAL) return false;          // and for the local divergence
    }
    return true;
}

// Per-lattice regions: two copies, phi_s, scalars.
size_t case_bytes(const Layout &L) {
    return 2 * align_up(copy_bytes(L), kAlign) + align_up(L.stride * L.cs, kAlign) + align_up(64 * sizeof(double), kAlign);
}

struct BatchLayout {
    size_t off_stage, off_part, off_queue, off_desc, off_item_case, off_first, off_phi_backup, off_cases, total;
    size_t max_items;
};

BatchLayout make_batch_layout(const lbm_params *cases, int n) {
    BatchLayout B;
    size_t max_nn = 0, max_part = 0, items = 0, phi = 0, lat = 0;
    for (int c = 0; c < n; ++c) {
        const Layout L = make_layout(cases + c);
        max_nn = L.nn > max_nn ? L.nn : max_nn;
        max_part = L.max_partials > max_part ? L.max_partials : max_part;
        items += max_workgroups(cases + c);
        phi += align_up(L.stride * L.cs, kAlign);
        lat += case_bytes(L);
    }
    size_t off = 0;
    B.off_stage = off;
    off = align_up(off + 6 * max_nn * sizeof(double), kAlign);
    B.off_part = off;
    off = align_up(off + 2 * max_part * sizeof(double), kAlign);
    B.off_queue = off;
    off = align_up(off + (lbm::kXcds + 1) * sizeof(unsigned), kAlign);
    B.off_desc = off;
    off = align_up(off + (size_t)n * kDescBytes, kAlign);
    B.off_item_case = off;
    off = align_up(off + items * sizeof(unsigned), kAlign);
    B.off_first = off;
    off = align_up(off + (size_t)n * sizeof(unsigned), kAlign);
    B.off_phi_backup = off;
    off = align_up(off + phi, kAlign);
    B.off_cases = off;
    off += lat;
    B.total = off;
    B.max_items = items;
    return B;
}

void drop_graphs(lbm_batch *b) {
    for (int k = 0; k < 2; ++k) {
        if (b->exec[k]) hipGraphExecDestroy(b->exec[k]);
        b->exec[k] = nullptr;
    }
}

// tile_x = tile_y = 0 asks for fitted tiles: each lattice its own shape,
// in 512-thread workgroups (not for FP64, whose step fits 256 threads only).
constexpr int kFitThreads = 512;

bool tile_supported(int storage, int tx, int ty) {
    if (tx == 0 && ty == 0) return storage != LBM_STORE_F64;
    bool ok = false;
    for (const TileShape &t : kTiles) ok = ok || (t.tx == tx && t.ty == ty);
    return ok && (storage != LBM_STORE_F64 || tx * ty == 256);
}

// The fitted tile of a lattice: of the shapes with 256..512 nodes whose
// extended tile fits the kernel's LDS ring (kFitNodes) and that span whole x
// rows (exactly nx wide) or are 4k wide with 64 <= width < nx, the one that
// leaves the fewest of its workgroups' 512 thread slots idle; shapes within
// 2% of it go to the smaller halo (the two halo rows only for whole-row
// tiles, whose x neighbours are their own columns), then to the wider tile.
// Its tile count stays within the lattice's share of the work list.
// Measured on the 256-lattice batch (L = 24..96): any 4k width 3.26 ms,
// widths from 32 3.02 ms, whole rows rounded up to 4k 2.90 ms per step
// (32 x 16 tiles: 3.41 ms) -- narrow tiles cost more in coalescing than
// their fit saves.
constexpr int kFitMinWidth = 64;
constexpr double kFitTolerance = 0.02;

TileShape fitted_tile(const lbm_params &p) {
    const size_t bound = max_workgroups(&p);
    TileShape best{32, 16};
    double be = -1.0;
    int bh = 1 << 30;
    std::vector<int> widths;
    if (p.nx >= 2 && p.nx <= 128) widths.push_back(p.nx);
    for (int tx = kFitMinWidth; tx <= 128 && tx < p.nx; tx += 4) widths.push_back(tx);
    for (int tx : widths) {
        for (int ty = 1; ty <= 256; ++ty) {
            const int nt = tx * ty;
            if (nt > kFitThreads || nt < 256 || (tx + 2) * (ty + 2) > lbm::kFitNodes) continue;
            const size_t tiles = (size_t)((p.nx + tx - 1) / tx) * (size_t)((p.ny + ty - 1) / ty);
            if (tiles * (size_t)p.nz > bound) continue;
            const double e = (double)p.nx * p.ny / ((double)tiles * kFitThreads);
            const int halo = tx == p.nx ? 2 * tx : 2 * (tx + ty) + 4;
            const bool better =
                e > be + kFitTolerance || (e > be - kFitTolerance && (halo < bh || (halo == bh && tx > best.tx)));
            if (better) {
                best = TileShape{tx, ty};
                be = e > be ? e : be;
                bh = halo;
            }
        }
    }
    return best;
}

// The tile lattice c runs with under the batch's launch.
TileShape case_tile(const lbm_batch *b, int c) {
    return b->tile_x ? TileShape{b->tile_x, b->tile_y} : fitted_tile(b->cases[c].p);
}

// Work list and step descriptors for the current launch shape.  Lattices
// are dealt to the XCDs largest first, each to the XCD with the least work so
// far (nodes, idle tile slots included); every XCD's items are contiguous.
template <typename ST>
int build_batch_tables(lbm_batch *b) {
    std::vector<lbm::StepArgs<ST>> desc(b->n);
    std::vector<unsigned> first(b->n), item_case;
    std::vector<int> bin_of(b->n);
    item_case.reserve(b->max_items);
    {
        double load[lbm::kXcds] = {0};
        for (int k = 0; k < b->n; ++k) {
            const int c = b->order[k];
            const lbm_params &p = b->cases[c].p;
            const TileShape t = case_tile(b, c);
            const double slots = (double)((p.nx + t.tx - 1) / t.tx) * ((p.ny + t.ty - 1) / t.ty) *
                                 (b->tile_x ? t.tx * t.ty : kFitThreads) * p.nz;
            int best = 0;
            for (int x = 1; x < lbm::kXcds; ++x)
                if (load[x] < load[best]) best = x;
            load[best] += slots;
            bin_of[c] = best;
        }
    }
    for (int x = 0; x <= lbm::kXcds; ++x) b->bin_start[x] = 0;
    for (int pass = 0; pass < lbm::kXcds; ++pass)
    for (int k = 0; k < b->n; ++k) {
        const int c = b->order[k];
        if (bin_of[c] != pass) continue;
        lbm_handle *h = b->cases + c;
        lbm::StepArgs<ST> A;
        A.pop_in = (const typename ST::T *)h->pop(0);
        A.pop_out = (typename ST::T *)h->pop(1);
        A.phi = (typename ST::C *)h->phi();
        A.rho_ave = h->rho_ave();
        A.partials = h->partials();
        A.status = h->status();
        A.stride = h->L.stride;
        set_buffer_extents(h->L, A.buf_lo_bytes, A.buf_hi_bytes);
        A.wall = nullptr;    // batches are periodic
        A.ustage = nullptr;  // batches run the local divergence of Eq. (48)
        A.uout = nullptr;
        A.unn = 0;
        A.nx = h->p.nx;
        A.ny = h->p.ny;
        A.nz = h->p.nz;
        const TileShape t = case_tile(b, c);
        A.ntx = (h->p.nx + t.tx - 1) / t.tx;
        A.nty = (h->p.ny + t.ty - 1) / t.ty;
        A.tile_x = t.tx;
        A.tile_y = t.ty;
        A.cz = b->chunk_z < h->p.nz ? b->chunk_z : h->p.nz;
        A.P = make_phys<typename ST::C>(&h->p);
        desc[c] = A;
        const unsigned items = (unsigned)(A.ntx * A.nty * ((h->p.nz + A.cz - 1) / A.cz));
        first[c] = (unsigned)item_case.size();
        for (unsigned i = 0; i < items; ++i) item_case.push_back((unsigned)c);
        b->bin_start[pass + 1] = (unsigned)item_case.size();
    }
    for (int x = 1; x <= lbm::kXcds; ++x)
        if (b->bin_start[x] < b->bin_start[x - 1]) b->bin_start[x] = b->bin_start[x - 1];
    if (item_case.size() > b->max_items) return LBM_EINVAL;
    b->n_items = (unsigned)item_case.size();
    hipError_t e = hipMemcpyAsync(b->d_desc, desc.data(), desc.size() * sizeof(desc[0]), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_item_case, item_case.data(), item_case.size() * sizeof(unsigned),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_first_item, first.data(), first.size() * sizeof(unsigned), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // the host vectors go out of scope
    return hip_status(e);
}

int default_batch_workgroups(const lbm_batch *b, int tx, int ty) {
    // Two waves per SIMD fit the step kernel's registers: 8 waves per compute unit.
    const int threads = tx * ty > 0 ? tx * ty : kFitThreads;
    const int per_cu = (8 * 64) / threads > 0 ? (8 * 64) / threads : 1;
    return b->cus * per_cu;
}

template <typename ST, int TX, int TY, bool FIT = false>
int launch_batch_t(lbm_batch *b, int parity, int grid) {
    lbm::BatchQueue Q;
    Q.item_case = b->d_item_case;
    Q.first_item = b->d_first_item;
    Q.queue = b->d_queue;
    for (int x = 0; x <= lbm::kXcds; ++x) Q.bin_start[x] = b->bin_start[x];
    const lbm::StepArgs<ST> *d = (const lbm::StepArgs<ST> *)b->d_desc;
    bool buf = true;
    for (int c = 0; c < b->n; ++c) buf = buf && buffer_path(b->cases[c].L);
    if (buf)
        hipLaunchKernelGGL((lbm::k_step_batch<ST, TX, TY, true, FIT>), dim3(grid), dim3(TX * TY), 0, b->stream, d, Q,
                           parity);
    else
        hipLaunchKernelGGL((lbm::k_step_batch<ST, TX, TY, false, FIT>), dim3(grid), dim3(TX * TY), 0, b->stream, d,
                           Q, parity);
    return hip_status(hipGetLastError());
}

template <typename ST>
int launch_batch(lbm_batch *b, int parity) {
    const int tx = b->tile_x, ty = b->tile_y;
    int grid = b->workgroups > 0 ? b->workgroups : default_batch_workgroups(b, tx, ty);
    if ((unsigned)grid > b->n_items) grid = (int)b->n_items;
    if (grid < 1) grid = 1;
    if (tx == 64 && ty == 4) return launch_batch_t<ST, 64, 4>(b, parity, grid);
    if (tx == 32 && ty == 8) return launch_batch_t<ST, 32, 8>(b, parity, grid);
    if constexpr (sizeof(typename ST::C) == 4) {
        if (tx == 0 && ty == 0) return launch_batch_t<ST, 32, 16, true>(b, parity, grid);  // fitted tiles
        if (tx == 64 && ty == 8) return launch_batch_t<ST, 64, 8>(b, parity, grid);
        if (tx == 32 && ty == 16) return launch_batch_t<ST, 32, 16>(b, parity, grid);
        if (tx == 128 && ty == 4) return launch_batch_t<ST, 128, 4>(b, parity, grid);
    }
    return LBM_EINVAL;
}

int batch_launch_one(lbm_batch *b, int parity) {
    return with_format_q<7>(b->storage, [&](auto fmt) { return launch_batch<decltype(fmt)>(b, parity); });
}

int batch_tables(lbm_batch *b) {
    drop_graphs(b);
    return with_format_q<7>(b->storage, [&](auto fmt) { return build_batch_tables<decltype(fmt)>(b); });
}

// Graph of two steps starting from population copy `from`.
int batch_graph(lbm_batch *b, int from) {
    if (b->exec[from]) return LBM_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return LBM_EHIP;
    int rc = batch_launch_one(b, from);
    if (!rc) rc = batch_launch_one(b, 1 - from);
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc || e != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return rc ? rc : LBM_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&b->exec[from], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    return hip_status(ei);
}

}  // namespace

extern "C" {

size_t lbm_batch_arena_bytes(const lbm_params *cases, int ncases) {
    if (!valid_batch(cases, ncases)) return 0;
    return make_batch_layout(cases, ncases).total;
}

int lbm_batch_create(const lbm_params *cases, int ncases, void *dev_arena, size_t arena_bytes, void *hip_stream,
                     lbm_batch **out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!valid_batch(cases, ncases) || !dev_arena) return LBM_EINVAL;
    const BatchLayout B = make_batch_layout(cases, ncases);
    if (arena_bytes < B.total || ((uintptr_t)dev_arena % kAlign) != 0) return LBM_ENOMEM;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return LBM_EHIP;
    lbm_batch *b = new lbm_batch();
    b->n = ncases;
    b->storage = cases[0].storage;
    b->stream = (hipStream_t)hip_stream;
    b->cases = new lbm_handle[ncases]();
    b->order = new int[ncases];
    b->cus = cus;
    char *arena = (char *)dev_arena;
    b->d_desc = arena + B.off_desc;
    b->d_item_case = (unsigned *)(arena + B.off_item_case);
    b->d_first_item = (unsigned *)(arena + B.off_first);
    b->d_queue = (unsigned *)(arena + B.off_queue);
    b->d_phi_backup = arena + B.off_phi_backup;
    b->max_items = B.max_items;
    b->exec[0] = b->exec[1] = nullptr;
    size_t off = B.off_cases;
    size_t largest = 0;
    for (int c = 0; c < ncases; ++c) {
        lbm_handle *h = b->cases + c;
        h->p = cases[c];
        h->L = make_layout(cases + c);
        h->stream = b->stream;
        h->r_pop[0] = arena + off;
        h->r_pop[1] = h->r_pop[0] + align_up(copy_bytes(h->L), kAlign);
        h->r_phi = h->r_pop[1] + align_up(copy_bytes(h->L), kAlign);
        h->r_scal = h->r_phi + align_up(h->L.stride * h->L.cs, kAlign);
        h->r_stage = (double *)(arena + B.off_stage);
        h->r_part = (double *)(arena + B.off_part);
        off += case_bytes(h->L);
        h->cur = 0;
        h->initialized = 0;
        b->order[c] = c;
        if (h->L.nn > b->cases[largest].L.nn) largest = c;
    }
    // Largest lattices first: the long items start early and the small ones fill the tail.
    std::sort(b->order, b->order + ncases, [&](int a, int c) {
        return b->cases[a].L.nn != b->cases[c].L.nn ? b->cases[a].L.nn > b->cases[c].L.nn : a < c;
    });
    set_default_launch(b->cases + largest);
    b->tile_x = b->cases[largest].tile_x;
    b->tile_y = b->cases[largest].tile_y;
    b->chunk_z = 16;
    b->workgroups = 0;
    b->cur = 0;
    int rc = hip_status(hipMemsetAsync(b->d_queue, 0, (lbm::kXcds + 1) * sizeof(unsigned), b->stream));
    for (int c = 0; c < ncases && !rc; ++c) rc = clear_status(b->cases + c);
    if (!rc) rc = batch_tables(b);
    if (rc) {
        lbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_init_case(lbm_batch *b, int c, const double *rho, const double *ux, const double *uy,
                        const double *uz, const double *T) {
    if (!b || c < 0 || c >= b->n || !rho || !ux || !uy || !uz || !T) return LBM_EINVAL;
    return init_state(b->cases + c, rho, ux, uy, uz, T, b->cur);
}

int lbm_batch_step(lbm_batch *b, int n) {
    if (!b || n < 0) return LBM_EINVAL;
    for (int c = 0; c < b->n; ++c)
        if (!b->cases[c].initialized) return LBM_ESTATE;
    int rc = LBM_OK;
    if (b->stream) {
        // pairs of steps as graph replays
        for (; n >= 2 && !rc; n -= 2) {
            rc = batch_graph(b, b->cur);
            if (!rc) rc = hip_status(hipGraphLaunch(b->exec[b->cur], b->stream));
        }
    }
    for (; n > 0 && !rc; --n) {
        rc = batch_launch_one(b, b->cur);
        if (!rc) b->cur = 1 - b->cur;
    }
    for (int c = 0; c < b->n; ++c) b->cases[c].cur = b->cur;
    return rc;
}

int lbm_batch_get_rho_u_T(lbm_batch *b, int c, double *rho, double *ux, double *uy, double *uz, double *T) {
    if (!b || c < 0 || c >= b->n) return LBM_EINVAL;
    return lbm_get_rho_u_T(b->cases + c, rho, ux, uy, uz, T);
}

int lbm_batch_reduce(lbm_batch *b, int c, double *mass, double *energy) {
    if (!b || c < 0 || c >= b->n) return LBM_EINVAL;
    return lbm_reduce(b->cases + c, mass, energy);
}

int lbm_batch_set_launch(lbm_batch *b, int tile_x, int tile_y, int chunk_z, int workgroups) {
    if (!b || chunk_z < 1 || chunk_z > kMaxChunk || workgroups < 0) return LBM_EINVAL;
    if (!tile_supported(b->storage, tile_x, tile_y)) return LBM_EINVAL;
    const int tx = b->tile_x, ty = b->tile_y, cz = b->chunk_z, wg = b->workgroups;
    b->tile_x = tile_x;
    b->tile_y = tile_y;
    b->chunk_z = chunk_z;
    b->workgroups = workgroups;
    const int rc = batch_tables(b);
    if (rc) {
        b->tile_x = tx;
        b->tile_y = ty;
        b->chunk_z = cz;
        b->workgroups = wg;
        batch_tables(b);
    }
    return rc;
}

int lbm_batch_case_tile(const lbm_batch *b, int c, int *tile_x, int *tile_y, int *threads) {
    if (!b || c < 0 || c >= b->n || !tile_x || !tile_y || !threads) return LBM_EINVAL;
    const TileShape t = case_tile(b, c);
    *tile_x = t.tx;
    *tile_y = t.ty;
    *threads = b->tile_x ? t.tx * t.ty : kFitThreads;
    return LBM_OK;
}
int lbm_fitted_tile(const lbm_params *p, int *tile_x, int *tile_y) {
    if (!p || !tile_x || !tile_y || !valid_params(p) || p->storage == LBM_STORE_F64) return LBM_EINVAL;
    const TileShape t = fitted_tile(*p);
    *tile_x = t.tx;
    *tile_y = t.ty;
    return LBM_OK;
}

int lbm_batch_get_launch(const lbm_batch *b, int *tile_x, int *tile_y, int *chunk_z, int *workgroups, int *items) {
    if (!b || !tile_x || !tile_y || !chunk_z || !workgroups || !items) return LBM_EINVAL;
    *tile_x = b->tile_x;
    *tile_y = b->tile_y;
    *chunk_z = b->chunk_z;
    int grid = b->workgroups > 0 ? b->workgroups : default_batch_workgroups(b, b->tile_x, b->tile_y);
    if ((unsigned)grid > b->n_items) grid = (int)b->n_items;
    *workgroups = grid;
    *items = (int)b->n_items;
    return LBM_OK;
}

int lbm_batch_autotune(lbm_batch *b, int steps, double *best_ms) {
    if (!b || steps < 1 || !best_ms) return LBM_EINVAL;
    for (int c = 0; c < b->n; ++c)
        if (!b->cases[c].initialized) return LBM_ESTATE;
    // Status words as they stand (an instability flagged by earlier steps is
    // reported after the sweep too; flags raised by the timed launches are not).
    std::vector<unsigned> status(b->n, 0u);
    for (int c = 0; c < b->n; ++c)
        if (hipMemcpyAsync(&status[c], b->cases[c].status(), sizeof(unsigned), hipMemcpyDeviceToHost, b->stream) !=
            hipSuccess)
            return LBM_EHIP;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EHIP;
    // keep every phi_s plane: the timed launches update them in place
    size_t off = 0;
    for (int c = 0; c < b->n; ++c) {
        const size_t bytes = b->cases[c].L.nn * b->cases[c].L.cs;
        if (hipMemcpyAsync(b->d_phi_backup + off, b->cases[c].phi(), bytes, hipMemcpyDeviceToDevice, b->stream) !=
            hipSuccess)
            return LBM_EHIP;
        off += align_up(b->cases[c].L.stride * b->cases[c].L.cs, kAlign);
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LBM_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return LBM_EHIP;
    }
    const int chunks[] = {8, 16, 32, 64, 128};
    double best = 1e30;
    int bt[4] = {b->tile_x, b->tile_y, b->chunk_z, b->workgroups};
    int rc = LBM_OK;
    std::vector<TileShape> shapes(std::begin(kTiles), std::end(kTiles));
    shapes.push_back(TileShape{0, 0});  // fitted tiles
    for (const TileShape &t : shapes) {
        if (!tile_supported(b->storage, t.tx, t.ty)) continue;
        for (int cz : chunks) {
            for (int mult = 1; mult <= 2 && !rc; ++mult) {
                b->tile_x = t.tx;
                b->tile_y = t.ty;
                b->chunk_z = cz;
                b->workgroups = mult * default_batch_workgroups(b, t.tx, t.ty);
                rc = batch_tables(b);
                if (!rc) rc = batch_launch_one(b, b->cur);  // warm-up
                if (!rc) rc = hip_status(hipEventRecord(e0, b->stream));
                for (int k = 0; k < steps && !rc; ++k) rc = batch_launch_one(b, b->cur);
                if (!rc) rc = hip_status(hipEventRecord(e1, b->stream));
                if (!rc) rc = hip_status(hipEventSynchronize(e1));
                float ms = 0.0f;
                if (!rc) rc = hip_status(hipEventElapsedTime(&ms, e0, e1));
                if (!rc && ms / steps < best) {
                    best = ms / steps;
                    bt[0] = t.tx;
                    bt[1] = t.ty;
                    bt[2] = cz;
                    bt[3] = b->workgroups;
                }
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    // Restore phi_s and the status words whatever happened in the sweep (the
    // first error is the one returned), and install the fastest shape.
    off = 0;
    for (int c = 0; c < b->n; ++c) {
        const size_t bytes = b->cases[c].L.nn * b->cases[c].L.cs;
        int r = hip_status(
            hipMemcpyAsync(b->cases[c].phi(), b->d_phi_backup + off, bytes, hipMemcpyDeviceToDevice, b->stream));
        if (!r)
            r = hip_status(hipMemcpyAsync(b->cases[c].status(), &status[c], sizeof(unsigned), hipMemcpyHostToDevice,
                                          b->stream));
        if (!rc) rc = r;
        off += align_up(b->cases[c].L.stride * b->cases[c].L.cs, kAlign);
    }
    b->tile_x = bt[0];
    b->tile_y = bt[1];
    b->chunk_z = bt[2];
    b->workgroups = bt[3];
    const int rc2 = batch_tables(b);
    if (!rc) rc = rc2;
    const int rc3 = hip_status(hipStreamSynchronize(b->stream));  // the status copies read `status`
    if (!rc) rc = rc3;
    *best_ms = best;
    return rc;
}

void lbm_batch_destroy(lbm_batch *b) {
    if (!b) return;
    drop_graphs(b);
    delete[] b->cases;
    delete[] b->order;
    delete b;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Measurement aid: a plain streaming copy, one 16-byte element per thread
// with non-temporal loads and stores (of the forms measured on MI355X --
// grid-stride loops, several elements a thread, temporal accesses, the
// runtime's device-to-device copy -- the fastest: 6.1-6.5 TB/s on 2 GiB),
// the practical HBM ceiling the step kernels are compared with.
// ---------------------------------------------------------------------------

namespace {

__global__ void __launch_bounds__(256) k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 v;
    v.x = __builtin_nontemporal_load(&src[i].x);
    v.y = __builtin_nontemporal_load(&src[i].y);
    v.z = __builtin_nontemporal_load(&src[i].z);
    v.w = __builtin_nontemporal_load(&src[i].w);
    __builtin_nontemporal_store(v.x, &dst[i].x);
    __builtin_nontemporal_store(v.y, &dst[i].y);
    __builtin_nontemporal_store(v.z, &dst[i].z);
    __builtin_nontemporal_store(v.w, &dst[i].w);
}

}  // namespace

extern "C" int lbm_copy_probe(const void *src, void *dst, size_t bytes, void *hip_stream) {
    if (!src || !dst || bytes == 0 || bytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
        return LBM_EINVAL;
    const size_t n = bytes / 16;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return LBM_EINVAL;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, (const uint4 *)src,
                       (uint4 *)dst, n);
    return hip_status(hipGetLastError());
}
