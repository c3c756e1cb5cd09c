// Host side of liblbm: parameter validation, arena carving, launches and the
// C-ABI declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

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
    size_t off_pop[2], off_phi, off_stage, off_part, off_scal, total;
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

// Planes per copy: 26 populations, plus rho_r and T_r for the deviation
// formats (FP16 for F16, FP32 for BF16 and F32_DEV).
size_t planes_of(int s) { return (s == LBM_STORE_F32 || s == LBM_STORE_F64) ? 26 : 28; }
size_t reference_bytes(int s) { return s == LBM_STORE_F64 ? 8 : (s == LBM_STORE_F16 ? 2 : 4); }

bool valid_params(const lbm_params *p) {
    if (!p) return false;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
    if (!valid_storage(p->storage)) return false;
    // node byte offsets inside a plane must fit in 32 bits
    if ((size_t)p->nx * p->ny * p->nz * element_bytes(p->storage) >= (size_t)1 << 32) return false;
    if (p->bc_z != LBM_BC_PERIODIC && p->bc_z != LBM_BC_WALL_BOTTOM_OPEN_TOP) return false;
    if (p->bc_z == LBM_BC_WALL_BOTTOM_OPEN_TOP && p->nz < 3) return false;
    if (!(p->tau_e > 0.5) || !(p->tau_v > 0.5) || !(p->tau_q > 0.5) || !(p->tau_pi > 0.5)) return false;
    if (!(p->vs_q > 0.5) || !(p->vs_pi > 0.5)) return false;
    if (p->G == 0.0 || !(p->cV > 0.0) || !(p->kappa > 0.0)) return false;
    if (!(p->d > 0.0 && p->d < 1.0)) return false;
    if (p->kappa_mode != LBM_KAPPA_CONST_LAMBDA && p->kappa_mode != LBM_KAPPA_CONST_CHI) return false;
    if (p->a != 0.0 && !(p->b > 0.0 && p->R > 0.0)) return false;
    if (p->a < 0.0 || p->b < 0.0 || p->R < 0.0) return false;
    if (p->thermal != 0 && p->thermal != 1) return false;
    if (p->bc_T_shell != 0 && p->bc_T_shell != 1) return false;
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

size_t copy_bytes(const Layout &L) { return L.stride * (26 * L.es + (L.planes - 26) * L.rs); }

// Byte offset of plane a (0..25 populations, 26..27 references) in a copy.
size_t plane_offset(const Layout &L, size_t a) {
    return a < 26 ? a * L.stride * L.es : 26 * L.stride * L.es + (a - 26) * L.stride * L.rs;
}
size_t plane_bytes(const Layout &L, size_t a) { return L.nn * (a < 26 ? L.es : L.rs); }

Layout make_layout(const lbm_params *p) {
    Layout L;
    L.nn = (size_t)p->nx * p->ny * p->nz;
    L.es = element_bytes(p->storage);
    L.cs = p->storage == LBM_STORE_F64 ? 8 : 4;
    L.rs = reference_bytes(p->storage);
    L.planes = planes_of(p->storage);
    L.stride = align_up(L.nn, 128);
    // Each ping-pong copy holds its planes contiguously, `stride` elements
    // apart: f_0..f_18, g_0..g_6, then (deviation formats) rho_r and T_r.
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
    L.total = off;
    return L;
}

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
    P.wT0 = (C)(1.0 - p->d);
    P.wT1 = (C)(p->d / 6.0);
    P.csT2 = (C)(p->d / 3.0);
    P.inv_csT2 = (C)(3.0 / p->d);
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
    P.T_shell = (C)p->T_shell;
    P.attract = p->a != 0.0;
    P.gravity = (p->g[0] != 0.0 || p->g[1] != 0.0 || p->g[2] != 0.0);
    P.T_patch = p->T_wall_patch;
    P.T_wall = p->T_wall;
    P.patch_r2 = p->patch_radius * p->patch_radius;
    P.T_top = p->T_top;
    P.cx = 0.5 * (p->nx - 1);
    P.cy = 0.5 * (p->ny - 1);
    return P;
}

struct StateHeader {
    char magic[8];
    int32_t version, nx, ny, nz, storage, planes;
    uint64_t nn, es, cs;
};
constexpr int32_t kStateVersion = 2;

// Calls fn with a value of the storage-format type of `storage`.
template <typename Fn>
int with_format(int storage, Fn &&fn) {
    switch (storage) {
    case LBM_STORE_F32: return fn(lbm::StoreF32{});
    case LBM_STORE_F64: return fn(lbm::StoreF64{});
    case LBM_STORE_F16: return fn(lbm::StoreF16{});
    case LBM_STORE_BF16: return fn(lbm::StoreBF16{});
    case LBM_STORE_F32_DEV: return fn(lbm::StoreF32Dev{});
    }
    return LBM_EINVAL;
}

}  // namespace

struct lbm_handle {
    lbm_params p;
    Layout L;
    hipStream_t stream;
    char *arena;
    int cur;          // which population copy holds the state
    int initialized;
    int tile_x, tile_y, chunk_z;
    int workgroups;
    unsigned *status() { return (unsigned *)(arena + L.off_scal + 8 * sizeof(double)); }
    double *rho_ave() { return (double *)(arena + L.off_scal); }
    double *mass() { return (double *)(arena + L.off_scal + sizeof(double)); }
    double *energy() { return (double *)(arena + L.off_scal + 2 * sizeof(double)); }
    double *stage() { return (double *)(arena + L.off_stage); }
    double *partials() { return (double *)(arena + L.off_part); }
    void *pop(int k) { return arena + L.off_pop[k]; }
    void *phi() { return arena + L.off_phi; }
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EHIP; }

// Default launch shape (measured on MI355X): tiles as wide as the rows allow
// (128 nodes: whole 512-byte rows, and the x halo wraps inside the tile when
// nx = 128), 4 rows, and chunks of 16-32 planes; the z halo of a chunk is read
// twice, so chunks are kept long unless the grid would then give fewer
// workgroups than the 256 compute units.
void set_default_launch(lbm_handle *h) {
    const int nx = h->p.nx, ny = h->p.ny, nz = h->p.nz;
    const bool half = h->L.es == 2;
    if (half && nx >= 64) {
        // 16-bit storage: the kernel is bound by instruction issue more than
        // by the row length, and 64x8 tiles recompute fewer halo nodes.
        h->tile_x = 64;
        h->tile_y = 8;
    } else if (nx >= 96) {
        h->tile_x = 128;
        h->tile_y = 4;
    } else if (nx > 32) {
        h->tile_x = 64;
        h->tile_y = 4;
    } else {
        h->tile_x = 32;
        h->tile_y = 8;
    }
    if (h->p.storage == LBM_STORE_F64 && h->tile_x * h->tile_y != 256) {
        h->tile_x = nx > 32 ? 64 : 32;
        h->tile_y = nx > 32 ? 4 : 8;
    }
    const long tiles = (long)((nx + h->tile_x - 1) / h->tile_x) * ((ny + h->tile_y - 1) / h->tile_y);
    long cz = (long)nz * tiles / 256;
    if (cz > 32) cz = 32;
    if (cz < 4) cz = 4;
    if (cz > nz) cz = nz;
    h->chunk_z = (int)cz;
}

int workgroups_for(const lbm_handle *h, int tx, int ty, int cz) {
    const long n = (long)((h->p.nx + tx - 1) / tx) * ((h->p.ny + ty - 1) / ty) * ((h->p.nz + cz - 1) / cz);
    return (int)n;
}

// The buffer-resource path addresses each half of a copy's planes (split at
// plane 14) with 32-bit offsets.
bool buffer_path(const Layout &L) {
    const size_t lo = (size_t)lbm::kSplitPlane * L.stride * L.es;
    const size_t hi = copy_bytes(L) - lo;
    return lo <= 0xFFFFFFFFull && hi <= 0xFFFFFFFFull;
}

template <typename ST, int TX, int TY, bool WALLS>
int launch_step_t(lbm_handle *h, const lbm::StepArgs<ST> &A, int nb) {
    if (buffer_path(h->L))
        hipLaunchKernelGGL((lbm::k_step<ST, TX, TY, WALLS, true>), dim3(nb), dim3(TX * TY), 0, h->stream, A);
    else
        hipLaunchKernelGGL((lbm::k_step<ST, TX, TY, WALLS, false>), dim3(nb), dim3(TX * TY), 0, h->stream, A);
    return hip_status(hipGetLastError());
}

// FP32-arithmetic formats instantiate every tile shape; the FP64 build (used
// to check the kernel against the FP64 oracle) only the two 256-thread tiles,
// which fit its registers without spilling.
template <typename ST, bool WALLS>
int launch_step_tile(lbm_handle *h, const lbm::StepArgs<ST> &A, int nb) {
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
    A.nx = h->p.nx;
    A.ny = h->p.ny;
    A.nz = h->p.nz;
    A.ntx = (h->p.nx + h->tile_x - 1) / h->tile_x;
    A.nty = (h->p.ny + h->tile_y - 1) / h->tile_y;
    A.cz = h->chunk_z;
    A.P = make_phys<C>(&h->p);
    const int nb = h->workgroups;
    int rc = h->p.bc_z == LBM_BC_WALL_BOTTOM_OPEN_TOP ? launch_step_tile<ST, true>(h, A, nb)
                                                      : launch_step_tile<ST, false>(h, A, nb);
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
    h->arena = (char *)dev_arena;
    h->cur = 0;
    h->initialized = 0;
    set_default_launch(h);
    h->workgroups = workgroups_for(h, h->tile_x, h->tile_y, h->chunk_z);
    int rc = clear_status(h);
    if (rc) {
        free(h);
        return rc;
    }
    *out = h;
    return LBM_OK;
}

int lbm_init_fields(lbm_handle *h, const double *rho, const double *ux, const double *uy, const double *uz,
                    const double *T) {
    if (!h || !rho || !ux || !uy || !uz || !T) return LBM_EINVAL;
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
    h->cur = 0;
    rc = with_format(h->p.storage, [&](auto fmt) {
        using ST = decltype(fmt);
        hipLaunchKernelGGL(lbm::k_init<ST>, dim3(nb), dim3(256), 0, h->stream, (const double *)st, nn,
                           (typename ST::T *)h->pop(0), (typename ST::C *)h->phi(), h->L.stride, P, h->status());
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

int lbm_step(lbm_handle *h, int n) {
    if (!h || n < 0) return LBM_EINVAL;
    if (!h->initialized) return LBM_ESTATE;
    for (int k = 0; k < n; ++k) {
        const int rc = with_format(h->p.storage, [&](auto fmt) { return step_once<decltype(fmt)>(h); });
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
    const int walls = h->p.bc_z == LBM_BC_WALL_BOTTOM_OPEN_TOP;
    const int lrc = with_format(h->p.storage, [&](auto fmt) {
        using ST = decltype(fmt);
        const typename ST::T *pop = (const typename ST::T *)h->pop(h->cur);
        hipLaunchKernelGGL(lbm::k_macro<ST>, dim3(nb), dim3(256), 0, h->stream, pop, h->L.stride, nn, P, st);
        hipLaunchKernelGGL(lbm::k_velocity<ST>, dim3(nb), dim3(256), 0, h->stream, pop, h->L.stride, h->p.nx, h->p.ny,
                           h->p.nz, walls, P, (const double *)h->rho_ave(), st);
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
    int rc = with_format(h->p.storage, [&](auto fmt) { return reduce_state<decltype(fmt)>(h, false); });
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

size_t lbm_state_bytes(const lbm_handle *h) {
    if (!h) return 0;
    const size_t nn = h->L.nn;
    size_t planes = 0;
    for (size_t a = 0; a < h->L.planes; ++a) planes += plane_bytes(h->L, a);
    return sizeof(StateHeader) + planes + nn * h->L.cs + sizeof(double);
}

int lbm_get_state(lbm_handle *h, void *host_buf, size_t bytes) {
    if (!h || !host_buf || bytes != lbm_state_bytes(h)) return LBM_EINVAL;
    if (!h->initialized) return LBM_ESTATE;
    StateHeader hd;
    memset(&hd, 0, sizeof(hd));
    memcpy(hd.magic, "LBMSTAT1", 8);
    hd.version = kStateVersion;
    hd.planes = (int32_t)h->L.planes;
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
    for (size_t a = 0; a < h->L.planes; ++a) {
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
        hd.ny != h->p.ny || hd.nz != h->p.nz || hd.storage != h->p.storage || hd.planes != (int32_t)h->L.planes ||
        hd.nn != h->L.nn || hd.es != h->L.es || hd.cs != h->L.cs)
        return LBM_EINVAL;
    const char *in = (const char *)host_buf + sizeof(hd);
    h->cur = 0;
    for (size_t a = 0; a < h->L.planes; ++a) {
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
    return (h->p.g[0] != 0.0 || h->p.g[1] != 0.0 || h->p.g[2] != 0.0) ? 2 : 1;
}

void lbm_destroy(lbm_handle *h) { free(h); }

const char *lbm_strerror(int status) {
    switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "arena too small or misaligned";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_EUNSTABLE: return "unstable state (rho <= 0, psi^2 < 0 or NaN)";
    case LBM_ESTATE: return "call out of order";
    }
    return "unknown status";
}

}  // extern "C"
