// Device code of liblbm for gfx950 (MI355X): the fused D3Q19 + D3Q7 time step
// of Li, Yu & Luo (arXiv:2201.06039) and its helper kernels.  The temperature
// lattice may also be D3Q19 (standard weights, BGK collision of Eq. (19)).
//
// State layout in HBM (structure of arrays, x fastest), two ping-pong copies
// (D3Q7 temperature lattice; D3Q19: g on planes 19..37, references 38, 39):
//   plane  0..18   D3Q19 populations f_alpha at time t (post-streaming)
//   plane 19..25   D3Q7 populations g_alpha
//   plane 26, 27   (deviation storage only) per-node references rho_r, T_r
// plus one phi_s(t - dt) plane (Eq. (23) history) updated in place.
//
// Storage formats.  Plain FP32/FP64 store the populations themselves.  The
// deviation formats (FP16, BF16, and FP32 for comparison) store
//   e_alpha = (f_alpha - w_alpha rho_r) * scale,   r_alpha = (g_alpha - w_alpha T_r) * scale
// where rho_r, T_r are the density and temperature of the node one step
// earlier rounded to the storage type, written by the node itself.  A node's
// moments are formed from e and the reference directly (rho = rho_r + sum e,
// rho u = sum e_alpha e_alpha), so the O(rho) rest part never enters a
// rounded difference.  Push streaming writes the value for node y encoded
// against y's new reference, which the writer reads from the LDS ring.
//
// The fused step kernel assigns each workgroup an x-y tile of TX*TY nodes and
// a chunk of z planes.  It marches up the chunk: for plane z+1 it computes
// rho, T and psi of the tile plus a one-node halo into a 4-plane LDS ring, so
// the 18-neighbour force of Eq. (7) and the density gradient at plane z read
// same-time-level values from LDS.  Halo nodes are recomputed from their own
// populations (an extra read served mostly by L2), which keeps the whole step
// in one launch with one read and one write of the state per node.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

// Sec. II, Eq. (2): D3Q19 velocity components, alpha = 0..18.
constexpr int kE19X[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kE19Y[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kE19Z[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
// Sec. III B, Eq. (21): the D3Q7 velocities are the first seven of Eq. (2)
// in the same order, so the temperature lattice (D3Q7 or D3Q19) indexes
// kE19* directly.
constexpr bool d3q7_is_head_of_d3q19() {
    constexpr int e7[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (int a = 0; a < 7; ++a)
        if (e7[a][0] != kE19X[a] || e7[a][1] != kE19Y[a] || e7[a][2] != kE19Z[a]) return false;
    return true;
}
static_assert(d3q7_is_head_of_d3q19(), "D3Q7 velocity order");

__host__ __device__ constexpr int opposite(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }

// Rest weights of the D3Q19 equilibrium: w0 = 1/3, axis 1/18, diagonal 1/36.
__host__ __device__ constexpr double w19(int a) { return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

template <typename C>
struct Num;
template <>
struct Num<float> {
    __device__ static float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
};
template <>
struct Num<double> {
    __device__ static double rcp(double x) { return 1.0 / x; }
    __device__ static double sqrt(double x) { return ::sqrt(x); }
};

// Constants of the model in the compute type, derived on the host.
template <typename C>
struct Phys {
    C a, b, R;            // Eq. (49)
    C kap;                // 0.37464 + 1.54226 w - 0.26992 w^2
    C inv_Tc;             // 1/T_c, T_c = (0.0778/0.45724) a/(b R)
    C two_over_Gc2;       // psi^2 = 2 (p - rho c_s^2)/(G c^2), Eq. (8)
    C negG;               // F_m = -G psi sum(...), Eq. (7)
    C sig6;               // 6 sigma/(tau_e - 1/2), Eq. (9)
    C lam_e, lam_v, lam_q, lam_pi;  // Eq. (6)
    C divu_a, divu_b;     // Eq. (48): 1/tau_e and 1 - 1/(2 tau_e)
    C cV, inv_cV;
    C wT0, wT1;           // D3Q7 weights
    C csT2, inv_csT2, d;  // c_sT^2 = d/3
    C kappa;              // lambda or chi
    C gam_q, gam_pi;      // 1/varsigma_q, 1/varsigma_pi
    C gx, gy, gz;         // gravity
    int kappa_mode;       // 0: constant lambda, 1: constant chi
    int thermal;          // temperature lattice evolves
    int shell;            // outer layer of nodes held at T_shell (periodic grids only)
    int thermal_bgk;      // single relaxation time for the temperature lattice, Eq. (19)
    C T_shell;
    int attract;          // a != 0
    int gravity;          // g != 0
    int top_wall;         // walls: bounce-back at the top too (closed box) instead of the open top
    int wet;              // walls: virtual density of the solid layer below z = 0 from the wall buffer
    double T_patch, T_wall, patch_r2, T_top, cx, cy;  // walls (decisions in FP64)
    double wet_phi, wet_phi_in, wet_drho, wet_square;  // virtual-density scheme of the bottom wall
};

// psi^2 of Eq. (8) with the Peng-Robinson pressure of Eq. (49).  rho, T and
// psi of a node are evaluated in several inlined copies (its own tile and the
// halo of its neighbours' tiles); contraction into FMA is off here so that
// every copy rounds identically and the result never depends on the tiling.
template <typename C>
__device__ __forceinline__ C psi_squared(const Phys<C> &P, C rho, C T) {
#pragma clang fp contract(off)
    C attraction = C(0);
    if (P.attract) {
        const C root = C(1) + P.kap * (C(1) - Num<C>::sqrt(T * P.inv_Tc));
        attraction = P.a * root * root * rho * rho * Num<C>::rcp(C(1) + C(2) * P.b * rho - P.b * P.b * rho * rho);
    }
    const C p = rho * P.R * T * Num<C>::rcp(C(1) - P.b * rho) - attraction;
    return P.two_over_Gc2 * (p - rho * C(1.0 / 3.0));
}

template <typename C>
__device__ __forceinline__ C sum19(const C *f) {
    return f[0] + (((f[1] + f[2]) + (f[3] + f[4])) + (f[5] + f[6])) +
           (((f[7] + f[8]) + (f[9] + f[10])) + ((f[11] + f[12]) + (f[13] + f[14])) +
            ((f[15] + f[16]) + (f[17] + f[18])));
}

template <typename C>
__device__ __forceinline__ C sum7(const C *g) {
    return g[0] + ((g[1] + g[2]) + (g[3] + g[4]) + (g[5] + g[6]));
}

// T = sum g over the QT velocities of the temperature lattice.
template <int QT, typename C>
__device__ __forceinline__ C sum_T(const C *g) {
    if constexpr (QT == 7) return sum7(g);
    else return sum19(g);
}

// m = M f for the raw monomial basis (1, e, |e|^2, 2ex^2-ey^2-ez^2, ey^2-ez^2,
// exey, exez, eyez, ex^2ey, exey^2, ex^2ez, exez^2, ey^2ez, eyez^2, ex^2ey^2,
// ex^2ez^2, ey^2ez^2), evaluated with pair sums and differences.  m[0] is not
// formed (it is rho).  With `rho` given, m[4], m[16..18] are returned as
// deviations from the rest equilibrium w rho (m4 - rho = q - f0 with q the
// sum of the twelve diagonal populations, m16..18 - rho/9), which avoids
// differences of O(rho) numbers.
template <typename C, bool DEV = false>
__device__ __forceinline__ void moments19(const C *f, C *m, C rho = C(0)) {
    const C a1 = f[1] + f[2], d1 = f[1] - f[2];
    const C a3 = f[3] + f[4], d3 = f[3] - f[4];
    const C a5 = f[5] + f[6], d5 = f[5] - f[6];
    const C s78 = f[7] + f[8], d78 = f[7] - f[8], s910 = f[9] + f[10], d910 = f[9] - f[10];
    const C s1112 = f[11] + f[12], d1112 = f[11] - f[12], s1314 = f[13] + f[14], d1314 = f[13] - f[14];
    const C s1516 = f[15] + f[16], d1516 = f[15] - f[16], s1718 = f[17] + f[18], d1718 = f[17] - f[18];
    m[16] = s78 + s910;
    m[17] = s1112 + s1314;
    m[18] = s1516 + s1718;
    m[7] = s78 - s910;
    m[8] = s1112 - s1314;
    m[9] = s1516 - s1718;
    m[10] = d78 - d910;
    m[11] = d78 + d910;
    m[12] = d1112 - d1314;
    m[13] = d1112 + d1314;
    m[14] = d1516 - d1718;
    m[15] = d1516 + d1718;
    m[1] = d1 + m[11] + m[13];
    m[2] = d3 + m[10] + m[15];
    m[3] = d5 + m[12] + m[14];
    const C A = a1 + a3 + a5;
    m[5] = C(2) * a1 - a3 - a5 + m[16] + m[17] - C(2) * m[18];
    m[6] = a3 - a5 + m[16] - m[17];
    if (DEV) {
        m[4] = (m[16] + m[17] + m[18]) - f[0];
        const C r9 = rho * C(1.0 / 9.0);
        m[16] -= r9;
        m[17] -= r9;
        m[18] -= r9;
    } else {
        m[4] = A + C(2) * (m[16] + m[17] + m[18]);
    }
}

// f = M^-1 m, the exact inverse of moments19 (m[0] = rho included).
template <typename C>
__device__ __forceinline__ void populations19(const C *m, C *f) {
    const C q = m[16] + m[17] + m[18];
    const C A = m[4] - C(2) * q;
    const C a1 = (m[5] + A - m[16] - m[17] + C(2) * m[18]) * C(1.0 / 3.0);
    const C b35 = m[6] - m[16] + m[17];
    const C r35 = A - a1;
    const C a3 = C(0.5) * (r35 + b35), a5 = C(0.5) * (r35 - b35);
    const C d1 = m[1] - m[11] - m[13];
    const C d3 = m[2] - m[10] - m[15];
    const C d5 = m[3] - m[12] - m[14];
    f[0] = m[0] - A - q;
    f[1] = C(0.5) * (a1 + d1);
    f[2] = C(0.5) * (a1 - d1);
    f[3] = C(0.5) * (a3 + d3);
    f[4] = C(0.5) * (a3 - d3);
    f[5] = C(0.5) * (a5 + d5);
    f[6] = C(0.5) * (a5 - d5);
    const C s78 = C(0.5) * (m[16] + m[7]), s910 = C(0.5) * (m[16] - m[7]);
    const C d78 = C(0.5) * (m[10] + m[11]), d910 = C(0.5) * (m[11] - m[10]);
    f[7] = C(0.5) * (s78 + d78);
    f[8] = C(0.5) * (s78 - d78);
    f[9] = C(0.5) * (s910 + d910);
    f[10] = C(0.5) * (s910 - d910);
    const C s1112 = C(0.5) * (m[17] + m[8]), s1314 = C(0.5) * (m[17] - m[8]);
    const C d1112 = C(0.5) * (m[12] + m[13]), d1314 = C(0.5) * (m[13] - m[12]);
    f[11] = C(0.5) * (s1112 + d1112);
    f[12] = C(0.5) * (s1112 - d1112);
    f[13] = C(0.5) * (s1314 + d1314);
    f[14] = C(0.5) * (s1314 - d1314);
    const C s1516 = C(0.5) * (m[18] + m[9]), s1718 = C(0.5) * (m[18] - m[9]);
    const C d1516 = C(0.5) * (m[14] + m[15]), d1718 = C(0.5) * (m[15] - m[14]);
    f[15] = C(0.5) * (s1516 + d1516);
    f[16] = C(0.5) * (s1516 - d1516);
    f[17] = C(0.5) * (s1718 + d1718);
    f[18] = C(0.5) * (s1718 - d1718);
}

// Eq. (5): equilibrium moments 4..18 (0..3 are rho and rho u).
template <typename C>
__device__ __forceinline__ void equilibrium19(C rho, C ux, C uy, C uz, C *meq) {
    constexpr C cs2 = C(1.0 / 3.0);
    const C ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
    const C usq = ux2 + uy2 + uz2;
    const C varphi = rho * C(1.0 / 9.0) * (C(1) - C(1.5) * usq);
    meq[0] = rho;
    meq[1] = rho * ux;
    meq[2] = rho * uy;
    meq[3] = rho * uz;
    meq[4] = rho + rho * usq;
    meq[5] = rho * (C(2) * ux2 - uy2 - uz2);
    meq[6] = rho * (uy2 - uz2);
    meq[7] = rho * ux * uy;
    meq[8] = rho * ux * uz;
    meq[9] = rho * uy * uz;
    meq[10] = rho * uy * (cs2 + ux2);
    meq[11] = rho * ux * (cs2 + uy2);
    meq[12] = rho * uz * (cs2 + ux2);
    meq[13] = rho * ux * (cs2 + uz2);
    meq[14] = rho * uz * (cs2 + uy2);
    meq[15] = rho * uy * (cs2 + uz2);
    meq[16] = varphi + rho * cs2 * (ux2 + uy2);
    meq[17] = varphi + rho * cs2 * (ux2 + uz2);
    meq[18] = varphi + rho * cs2 * (uy2 + uz2);
}

// a * b + c rounded once (the library is built without automatic contraction,
// so every fused operation is one of these and the rounding is fixed).
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The word holding a pair of T, and packing/unpacking of its halves.
template <typename T>
using PairWord = std::conditional_t<sizeof(T) == 2, unsigned, unsigned long long>;
template <typename T>
__device__ __forceinline__ PairWord<T> pack_pair(T lo, T hi) {
    using H = std::conditional_t<sizeof(T) == 2, unsigned short, unsigned>;
    return (PairWord<T>)__builtin_bit_cast(H, lo) | ((PairWord<T>)__builtin_bit_cast(H, hi) << (8 * sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T pair_half(PairWord<T> w, int h) {
    using H = std::conditional_t<sizeof(T) == 2, unsigned short, unsigned>;
    return __builtin_bit_cast(T, (H)(h ? w >> (8 * sizeof(T)) : w));
}

// ---------------------------------------------------------------------------
// Storage formats of the populations.
// ---------------------------------------------------------------------------

// Each format: T = stored population element, R = stored reference element,
// C = compute type, kDev = deviation encoding against per-node references,
// kScale = factor K of the stored deviations (keeps FP16 deviations above the
// subnormal range).  dec/enc are plain conversions between T and C: the step
// kernel works on K-scaled deviations throughout.  rdec/renc convert the
// (unscaled) references; ddec/denc give the unscaled value in FP64 for the
// helper kernels.
//
// References: FP16 stores them as FP16.  rho - rho_r (up to rho 2^-12) then
// enters every deviation as a node-to-node irregular offset w (rho - rho_r),
// which keeps the FP16 rounding errors of neighbouring nodes uncorrelated.
// With exact (FP32) references the deviations of a smooth region are smooth
// too, their rounding errors line up, and the bias shows as a systematic
// drift (measured: a 5x larger error of the D^2 slope of an evaporating
// droplet).  BF16 keeps FP32 references: its 8-bit rounding of the reference
// would put offsets of up to w rho 2^-9 into every deviation.
struct StoreF32 {
    using T = float;
    using R = float;
    using C = float;
    static constexpr bool kDev = false;
    static constexpr float kScale = 1.0f;
    __device__ static C dec(T v) { return v; }
    __device__ static T enc(C v) { return v; }
    __device__ static C rdec(T v) { return v; }
    __device__ static T renc(C v) { return v; }
    __device__ static double ddec(T v) { return v; }
    __device__ static T denc(double v) { return (T)v; }
};
struct StoreF64 {
    using T = double;
    using R = double;
    using C = double;
    static constexpr bool kDev = false;
    static constexpr double kScale = 1.0;
    __device__ static C dec(T v) { return v; }
    __device__ static T enc(C v) { return v; }
    __device__ static C rdec(T v) { return v; }
    __device__ static T renc(C v) { return v; }
    __device__ static double ddec(T v) { return v; }
    __device__ static T denc(double v) { return v; }
};
struct StoreF32Dev {
    using T = float;
    using R = float;
    using C = float;
    static constexpr bool kDev = true;
    static constexpr float kScale = 1.0f;
    __device__ static C dec(T v) { return v; }
    __device__ static T enc(C v) { return v; }
    __device__ static C rdec(T v) { return v; }
    __device__ static T renc(C v) { return v; }
    __device__ static double ddec(T v) { return v; }
    __device__ static T denc(double v) { return (T)v; }
};
struct StoreF16 {
    using T = _Float16;
    using R = _Float16;
    using C = float;
    static constexpr bool kDev = true;
    static constexpr float kScale = 1024.0f;
    __device__ static C dec(T v) { return (float)v; }
    __device__ static T enc(C v) { return (T)v; }
    // Stochastic rounding (Forsythe, 1959) of a deviation to FP16: the 13
    // bits of the FP32 significand below the FP16 one are raised by `r`
    // (uniform in [0, 2^13)) and the conversion rounds toward zero, so the
    // result is the FP16 neighbour above |v| with the probability of the
    // cut-off fraction, and the rounding is unbiased in the normal range.
    // Round-to-nearest errors of a slowly changing field stay correlated
    // from step to step and add up: measured on the 100^3 D^2 test, a 10%
    // error in the late slope that this removes.  One packing conversion
    // (v_cvt_pkrtz_f16_f32) rounds two values.
    static constexpr int kSrBits = 13;
    __device__ static unsigned enc_pair_sr(C v0, unsigned r0, C v1, unsigned r1) {
        const float u0 = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, v0) + r0);
        const float u1 = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, v1) + r1);
        return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(u0, u1));
    }
    __device__ static T enc_sr(C v, unsigned r) {
        return __builtin_bit_cast(T, (unsigned short)enc_pair_sr(v, r, v, r));
    }
    __device__ static C rdec(R v) { return (float)v; }
    __device__ static R renc(C v) { return (R)v; }
    __device__ static double ddec(T v) { return (double)(float)v * (1.0 / 1024.0); }
    __device__ static T denc(double v) { return (T)(float)(v * 1024.0); }
};
struct StoreBF16 {  // conversions round to nearest even (v_cvt_pk_bf16_f32 on gfx950)
    using T = __bf16;
    using R = float;
    using C = float;
    static constexpr bool kDev = true;
    static constexpr float kScale = 1.0f;
    __device__ static C dec(T v) { return (float)v; }
    __device__ static T enc(C v) { return (T)v; }
    // Stochastic rounding as for FP16, on the 16 bits below the BF16
    // significand (r uniform in [0, 2^16)); the BF16 value is the upper half
    // of the raised FP32 bits.
    static constexpr int kSrBits = 16;
    __device__ static unsigned enc_pair_sr(C v0, unsigned r0, C v1, unsigned r1) {
        const unsigned u0 = __builtin_bit_cast(unsigned, v0) + r0, u1 = __builtin_bit_cast(unsigned, v1) + r1;
        return (u0 >> 16) | (u1 & 0xFFFF0000u);
    }
    __device__ static T enc_sr(C v, unsigned r) {
        return __builtin_bit_cast(T, (unsigned short)((__builtin_bit_cast(unsigned, v) + r) >> 16));
    }
    __device__ static C rdec(R v) { return v; }
    __device__ static R renc(C v) { return v; }
    __device__ static double ddec(T v) { return (double)(float)v; }
    __device__ static T denc(double v) { return (T)(float)v; }
};

// A storage format for a temperature lattice of QT = 7 (D3Q7, Sec. III B) or
// QT = 19 (D3Q19 with the standard weights) velocities.
template <typename S, typename = void>
struct HasStochasticRounding : std::false_type {};
template <typename S>
struct HasStochasticRounding<S, std::void_t<decltype(S::enc_sr(typename S::C(0), 0u))>> : std::true_type {};

template <typename Base, int QT>
struct Fmt : Base {
    static_assert(QT == 7 || QT == 19, "temperature lattice");
    static constexpr int kQT = QT;
    // Encode a value the step stores, with random bits r (uniform in
    // [0, 2^kSrBits)) for formats that round stochastically (FP16, BF16),
    // round-to-nearest otherwise; enc_pair_r encodes the two halves of a
    // word of the paired layout.
    __device__ static typename Base::T enc_r(typename Base::C v, unsigned r) {
        if constexpr (HasStochasticRounding<Base>::value) return Base::enc_sr(v, r);
        else return Base::enc(v);
    }
    __device__ static auto enc_pair_r(typename Base::C v0, unsigned r0, typename Base::C v1, unsigned r1) {
        if constexpr (HasStochasticRounding<Base>::value) return Base::enc_pair_sr(v0, r0, v1, r1);
        else return pack_pair<typename Base::T>(Base::enc(v0), Base::enc(v1));
    }
};

// Loads/stores of a 2-, 4- or 8-byte element through a buffer resource.
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    if constexpr (sizeof(T) == 2) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
    else if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
}
template <typename T>
__device__ __forceinline__ void buf_st(T x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    if constexpr (sizeof(T) == 2) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, 0);
    } else if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, 0);
    } else {
        typedef unsigned v2u __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, x), r, v, s, 0);
    }
}

constexpr int kBufferFlags = 0x00020000;  // raw dword buffer; the record count of each resource is the byte
                                          // size of the planes behind it

// Access to the planes of the two ping-pong copies.
//
// Plain layout (8-byte elements): the kPop = 19 + QT population planes of T,
// `stride` elements apart, then (deviation formats) the rho_r and T_r planes
// of R.
//
// Paired layout (2- and 4-byte elements): two populations share one plane of
// words twice their width, so a node's values arrive in kPop / 2 wide loads
// (the step kernel is limited by how many loads it keeps in flight).  The
// pairs are chosen for the push stores (PopLayout): f_a and g_a of the same
// velocity go to the same neighbour and are written as one word.  16-bit
// references (rho_r, T_r) form the last pair; 32-bit references (BF16)
// follow the kPop / 2 pair planes.
//
// Every access names a population (or reference) index, a per-thread byte
// offset `v` (the node's place inside an x-y plane) and a workgroup-uniform
// byte offset `s` (the z plane), both counted in node strides of the layout
// (two elements per node in a pair plane).
//  BUF = true: two buffer resources per copy (planes below byte offset
//  kSplit * stride * sizeof(T), and the rest); plane and z offsets go into
//  the scalar offset, the x-y offset is the one vector offset and the half of
//  a word a constant, so loads and stores cost no vector address arithmetic.
//  Needs each half to span less than 4 GiB.
//  BUF = false: plain global pointers (any size).
template <typename T>
constexpr bool paired_layout() { return sizeof(T) == 2 || sizeof(T) == 4; }

// Population planes of a copy for a temperature lattice of QT = 7 (D3Q7) or
// 19 (D3Q19) velocities: f_0..f_18 are planes 0..18, g_0..g_{QT-1} follow
// from plane 19, and the references rho_r, T_r are the planes kPop, kPop + 1.
// In the paired layout pair plane p holds populations member(p, 0) (low
// half) and member(p, 1); population a sits in pair pair_of(a), half
// half_of(a).  The last pair holds references as wide as the populations.
//  D3Q7: f_a with g_a for a = 0..6; the diagonal f pair with a partner of
//   the same e_z, whose half is written in the same z-plane pass.
//  D3Q19: f_a with g_a for every a, so each push store writes a whole word.
// Two buffer resources cover a copy: planes [0, kSplit) (pairs
// [0, kSplit / 2)) behind the first, the rest and the references behind the
// second.
template <int QT>
struct PopLayout;

template <>
struct PopLayout<7> {
    static constexpr int kQT = 7, kPop = 26, kPairs = 14, kSplit = 14;
    static constexpr int kMember[14][2] = {{0, 19}, {1, 20}, {2, 21}, {3, 22}, {4, 23}, {5, 24}, {6, 25},
                                           {7, 8},  {9, 10}, {11, 14}, {15, 18}, {12, 13}, {16, 17}, {26, 27}};
    static constexpr int kPairOf[28] = {0, 1, 2, 3, 4, 5, 6, 7, 7, 8, 8, 9, 11, 11, 9, 10, 12, 12, 10,
                                        0, 1, 2, 3, 4, 5, 6, 13, 13};
    static constexpr int kHalfOf[28] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 1, 0, 0, 1, 1, 0, 0, 1, 1,
                                        1, 1, 1, 1, 1, 1, 1, 0, 1};
    __host__ __device__ static constexpr int member(int p, int h) { return kMember[p][h]; }
    __host__ __device__ static constexpr int pair_of(int a) { return kPairOf[a]; }
    __host__ __device__ static constexpr int half_of(int a) { return kHalfOf[a]; }
};

template <>
struct PopLayout<19> {
    static constexpr int kQT = 19, kPop = 38, kPairs = 20, kSplit = 20;
    __host__ __device__ static constexpr int member(int p, int h) { return p < 19 ? p + 19 * h : 38 + h; }
    __host__ __device__ static constexpr int pair_of(int a) { return a < 19 ? a : (a < 38 ? a - 19 : 19); }
    __host__ __device__ static constexpr int half_of(int a) { return a < 19 ? 0 : (a < 38 ? 1 : a - 38); }
};

template <int QT>
constexpr bool pair_tables_consistent() {
    using L = PopLayout<QT>;
    for (int p = 0; p < L::kPairs; ++p)
        for (int h = 0; h < 2; ++h)
            if (L::pair_of(L::member(p, h)) != p || L::half_of(L::member(p, h)) != h) return false;
    return L::kPairs == L::kPop / 2 + 1 && L::kSplit % 2 == 0;
}
static_assert(pair_tables_consistent<7>() && pair_tables_consistent<19>(), "pair tables disagree");

template <typename T, typename R, bool BUF, int QT>
struct PopIO;

template <typename T, typename R, int QT>
struct PopIO<T, R, true, QT> {
    using L = PopLayout<QT>;
    static constexpr int kSplitPlane = L::kSplit, kPairSplit = L::kSplit / 2, kPopPlanes = L::kPop;
    static constexpr bool PAIR = paired_layout<T>();
    __amdgpu_buffer_rsrc_t in_lo, in_hi, out_lo, out_hi;
    unsigned sb;   // population plane stride in bytes (plain layout) or pair plane stride / 2
    unsigned rsb;  // reference plane stride in bytes
    // lo_bytes, hi_bytes: the byte sizes of the planes below and above the
    // split (each under 4 GiB on this path).
    __device__ PopIO(const T *pin, T *pout, size_t stride, unsigned lo_bytes, unsigned hi_bytes) {
        sb = (unsigned)(stride * sizeof(T));
        rsb = (unsigned)(stride * sizeof(R));
        in_lo = __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(pin), 0, (int)lo_bytes, kBufferFlags);
        in_hi = __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(pin) + kSplitPlane * stride, 0, (int)hi_bytes,
                                                  kBufferFlags);
        out_lo = __builtin_amdgcn_make_buffer_rsrc(pout, 0, (int)lo_bytes, kBufferFlags);
        out_hi = __builtin_amdgcn_make_buffer_rsrc(pout + kSplitPlane * stride, 0, (int)hi_bytes, kBufferFlags);
    }
    // Whether population a sits behind the low resource, and the byte offset
    // of its plane from that resource's base (pair plane pair_of(a), 2 sb
    // bytes wide, in the paired layout).
    __device__ static constexpr bool low(int a) { return PAIR ? L::pair_of(a) < kPairSplit : a < kSplitPlane; }
    __device__ unsigned plane_off(int a) const {
        if constexpr (PAIR) {
            const int p = L::pair_of(a);
            return (unsigned)(p < kPairSplit ? p : p - kPairSplit) * 2u * sb;
        } else {
            return (unsigned)(a < kSplitPlane ? a : a - kSplitPlane) * sb;
        }
    }
    __device__ static constexpr unsigned half_off(int a) { return PAIR ? (unsigned)(L::half_of(a) * sizeof(T)) : 0u; }
    __device__ T load(int a, unsigned v, unsigned s) const {
        return low(a) ? buf_ld<T>(in_lo, v + half_off(a), plane_off(a) + s)
                      : buf_ld<T>(in_hi, v + half_off(a), plane_off(a) + s);
    }
    // Both halves of pair plane p (paired layout only).
    __device__ PairWord<T> load_pair(int p, unsigned v, unsigned s) const {
        const int a = L::member(p, 0);
        return low(a) ? buf_ld<PairWord<T>>(in_lo, v, plane_off(a) + s) : buf_ld<PairWord<T>>(in_hi, v, plane_off(a) + s);
    }
    __device__ void store(int a, unsigned v, unsigned s, T x) const {
        if (low(a)) buf_st<T>(x, out_lo, v + half_off(a), plane_off(a) + s);
        else buf_st<T>(x, out_hi, v + half_off(a), plane_off(a) + s);
    }
    __device__ void store_pair(int p, unsigned v, unsigned s, PairWord<T> w) const {
        const int a = L::member(p, 0);
        if (low(a)) buf_st<PairWord<T>>(w, out_lo, v, plane_off(a) + s);
        else buf_st<PairWord<T>>(w, out_hi, v, plane_off(a) + s);
    }
    // Reference plane k (0: rho_r, 1: T_r).  References as wide as the
    // populations are the halves of the last pair plane; wider ones follow
    // the population planes with offsets counted in sizeof(R).
    __device__ R load_ref(int k, unsigned v, unsigned s) const {
        if constexpr (PAIR && sizeof(R) == sizeof(T)) return __builtin_bit_cast(R, load(kPopPlanes + k, v, s));
        else return buf_ld<R>(in_hi, v, (unsigned)(kPopPlanes - kSplitPlane) * sb + (unsigned)k * rsb + s);
    }
    __device__ void store_ref(int k, unsigned v, unsigned s, R x) const {
        if constexpr (PAIR && sizeof(R) == sizeof(T)) store(kPopPlanes + k, v, s, __builtin_bit_cast(T, x));
        else buf_st<R>(x, out_hi, v, (unsigned)(kPopPlanes - kSplitPlane) * sb + (unsigned)k * rsb + s);
    }
};

// Plain global pointers: the z offset `s` is a 64-bit byte count, since a
// copy of a grid that needs this path spans more than 4 GiB.
template <typename T, typename R, int QT>
struct PopIO<T, R, false, QT> {
    using L = PopLayout<QT>;
    static constexpr int kPopPlanes = L::kPop;
    static constexpr bool PAIR = paired_layout<T>();
    const T *in;
    T *out;
    size_t st;
    __device__ PopIO(const T *pin, T *pout, size_t stride, unsigned, unsigned) : in(pin), out(pout), st(stride) {}
    __device__ size_t plane_elems(int a) const {
        return PAIR ? (size_t)L::pair_of(a) * 2 * st + L::half_of(a) : a * st;
    }
    __device__ T load(int a, unsigned v, size_t s) const {
        return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(in + plane_elems(a)) + s + v);
    }
    __device__ PairWord<T> load_pair(int p, unsigned v, size_t s) const {
        return *reinterpret_cast<const PairWord<T> *>(reinterpret_cast<const char *>(in + (size_t)p * 2 * st) + s + v);
    }
    __device__ void store(int a, unsigned v, size_t s, T x) const {
        *reinterpret_cast<T *>(reinterpret_cast<char *>(out + plane_elems(a)) + s + v) = x;
    }
    __device__ void store_pair(int p, unsigned v, size_t s, PairWord<T> w) const {
        *reinterpret_cast<PairWord<T> *>(reinterpret_cast<char *>(out + (size_t)p * 2 * st) + s + v) = w;
    }
    __device__ R load_ref(int k, unsigned v, size_t s) const {
        if constexpr (PAIR && sizeof(R) == sizeof(T)) return __builtin_bit_cast(R, load(kPopPlanes + k, v, s));
        const R *base = reinterpret_cast<const R *>(in + kPopPlanes * st) + k * st;
        return *reinterpret_cast<const R *>(reinterpret_cast<const char *>(base) + s + v);
    }
    __device__ void store_ref(int k, unsigned v, size_t s, R x) const {
        if constexpr (PAIR && sizeof(R) == sizeof(T)) {
            store(kPopPlanes + k, v, s, __builtin_bit_cast(T, x));
        } else {
            R *base = reinterpret_cast<R *>(out + kPopPlanes * st) + k * st;
            *reinterpret_cast<R *>(reinterpret_cast<char *>(base) + s + v) = x;
        }
    }
};

// Element index of population a (or reference plane kPop + k) of node i in
// a copy, for the one-thread-per-node helper kernels.
template <typename T, int QT>
__host__ __device__ inline size_t element_index(int a, size_t st, size_t i) {
    using L = PopLayout<QT>;
    if constexpr (paired_layout<T>()) return (size_t)L::pair_of(a) * 2 * st + 2 * i + L::half_of(a);
    else return (size_t)a * st + i;
}

template <typename ST>
struct StepArgs {
    const typename ST::T *__restrict__ pop_in;  // planes of the current state, `stride` elements apart
    typename ST::T *__restrict__ pop_out;
    typename ST::C *__restrict__ phi;
    const double *__restrict__ rho_ave;
    // walls with the virtual-density scheme: rho_w (nx*ny values) then psi_w
    // (nx*ny) of the solid layer below z = 0, written by k_wall_density
    const double *__restrict__ wall;
    double *__restrict__ partials;  // per-workgroup sum of rho (when gravity is on)
    unsigned *__restrict__ status;
    size_t stride;                  // elements between population planes
    unsigned buf_lo_bytes, buf_hi_bytes;  // bytes of a copy below and above the buffer-resource split
                                          // (the record counts of the two resources; buffer path only)
    // u(t) of Eq. (10) at every node, component planes `unn` values apart
    // (finite-difference divergence only): written by the velocity pass
    // (uout), read by the step (ustage)
    const typename ST::C *__restrict__ ustage;
    typename ST::C *__restrict__ uout;
    size_t unn;
    int nx, ny, nz;
    int ntx, nty, cz;               // tiles in x, y; planes per chunk
    int tile_x, tile_y;             // the tile shape (read by kernels built for fitted tiles)
    Phys<typename ST::C> P;
};

// Fitted tiles (the batch kernel): each lattice has its own tile shape
// tile_x x tile_y of at most the workgroup's threads, whose extended tile
// (tile_x + 2)(tile_y + 2) fits the LDS ring of kFitNodes nodes.
constexpr int kFitNodes = 700;


// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b mod 8).  Give each XCD a contiguous range of logical tiles, so that
// workgroups sharing halo rows share an L2.
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, xcd = b & 7;
    return xcd * q + (xcd < r ? xcd : r) + (b >> 3);
}

// One node's loaded state in the compute type: e, r = stored f and g values
// (K-scaled deviations for the deviation formats), br/bt = references
// (0 for plain storage).
template <typename C, int QT>
struct NodePops {
    C e[19], r[QT], br, bt;
};

// A node's state as it arrives from memory in the paired layout: the pair
// words (kPop / 2 of population pairs, one more of 16-bit references) and,
// for 32-bit references, the references in the compute type.  Planes in flight
// are kept in this form and decoded where they are used, which halves the
// registers they occupy.
template <typename C, typename W, int WORDS>
struct NodeWords {
    W w[WORDS];
    C br, bt;
};

// One workgroup's share of a time step: the x-y tile and z chunk with index
// `logical` (x fastest, then y, then the chunk), for the lattice described by
// A.  `slot` is the workgroup's entry in A.partials (gravity runs only).
// DFD: the velocity divergence by finite differences of A.ustage at interior
// nodes instead of Eq. (48).  VEL: the velocity pass that precedes such a
// step -- the same march over the planes (rho, T, psi and the LDS ring), but
// each tile node only writes u(t) of Eq. (10) to A.uout.
// FIT: the tile is A.tile_x x A.tile_y (at most TX * TY nodes, the
// workgroup's threads; threads beyond the tile only help with the halo),
// instead of TX x TY.  A fitted tile exactly as wide as the lattice spans
// whole x rows: the columns left and right of it are its own last and first
// columns (periodic in x), so its halo is only the rows below and above it,
// and a node of its first or last column also writes its LDS entries into
// the opposite halo column.
template <typename ST, int TX, int TY, bool WALLS, bool BUF, bool DFD = false, bool VEL = false, bool FIT = false>
__device__ __forceinline__ void step_tile(const StepArgs<ST> &A, int logical, int slot) {
    using E = typename ST::T;  // stored element
    using C = typename ST::C;
    constexpr bool DEV = ST::kDev;
    constexpr C K = ST::kScale, IK = C(1) / ST::kScale;
    constexpr int NT = TX * TY;  // threads of the workgroup
    static_assert(FIT || (TX + 2) * (TY + 2) - NT <= NT, "halo must not exceed the tile");
    // LDS nodes of a plane of the ring (the tile and its halo)
    constexpr int NE = FIT ? kFitNodes : (TX + 2) * (TY + 2);
    static_assert(!FIT || NE - 256 <= NT, "fitted tiles keep at least 256 nodes, so their halo fits the threads");
    static_assert(!FIT || (!WALLS && !DFD && !VEL), "fitted tiles are built for the periodic batch step");
    const int tile_x = FIT ? A.tile_x : TX, tile_y = FIT ? A.tile_y : TY;
    const bool wrapx = FIT && tile_x == A.nx && A.nx >= 2;  // a whole-row fitted tile
    const int EX = tile_x + 2, NTL = tile_x * tile_y;
    const int NH = wrapx ? 2 * tile_x : EX * (tile_y + 2) - NTL;
    constexpr int QT = ST::kQT;  // velocities of the temperature lattice
    using LY = PopLayout<QT>;
    constexpr bool PAIR = paired_layout<E>();
    constexpr unsigned NS = PAIR ? 2 * sizeof(E) : sizeof(E);  // bytes between neighbouring nodes of a plane
    // Byte offset of a z plane: 32 bits on the buffer-resource path (the
    // scalar offset of the instruction), 64 bits with plain pointers.
    using ZOff = std::conditional_t<BUF, unsigned, size_t>;
    constexpr int G0 = 19;  // first temperature plane
    constexpr unsigned RSZ = sizeof(typename ST::R);
    // node stride of the reference planes: 16-bit references share a pair plane
    constexpr bool REF_IN_PAIR = ST::kDev && sizeof(typename ST::R) == sizeof(E) && paired_layout<E>();
    constexpr unsigned RU = REF_IN_PAIR ? 2 * sizeof(E) : RSZ;
    // References in the compute type need no LDS copy of rho of their own.
    constexpr bool OWN_RREF = DEV && sizeof(typename ST::R) != sizeof(C);
    constexpr int RS = OWN_RREF ? 4 : 1, RN = OWN_RREF ? NE : 1;
    constexpr int TS = DEV ? 4 : 1, TN = DEV ? NE : 1;
    __shared__ C s_psi[4][NE];
    __shared__ C s_rho[4][NE];
    __shared__ C s_rref[RS][RN];  // rho and T as stored in the reference planes:
    __shared__ C s_tref[TS][TN];  // the references every node writes for itself
    __shared__ double s_red[NT / 64];

    // STASH: the tile node's words of plane z+1 wait in LDS from its moments
    // until its collision (each thread reads back only its own entries, so
    // no barrier guards them), and the words of plane z+2 load straight into
    // the registers they left, after the barrier: no register copy of words
    // in flight, which would wait for every load and store of the wave.
    // Measured: FP32 512^3 7.66 -> 6.47 ms, pool grid -5%; 16-bit periodic
    // grids with 64x8 tiles -2% (512^3, against 128x4 without) and -3%
    // (128^3), the FP16 batch -3%; 16-bit walls +4% and the D3Q19
    // temperature lattice in FP32 +15% (128^3), so those keep their words in
    // registers.
    constexpr bool STASH = paired_layout<E>() && ST::kQT == 7 && (sizeof(E) == 4 || FIT || !WALLS);
    // The float constants of the model are read by vector instructions in
    // every iteration; held in scalar registers they exceed the scalar
    // register file and are spilled to vector lanes, costing one read per use.
    // Keeping them in vector registers from the start (the empty asm only
    // tells the compiler they live there) avoids that.  With the stash only
    // the constants of the temperature lattice (divu_a .. gam_pi, bits 12-20
    // of the mask below) are pinned; pinning all of them then costs more
    // registers than the spills it saves (measured: FP32 64x8 tiles).
    constexpr unsigned kConstInVgpr = STASH ? 0x1FF000u : 0x1FFFFFFu;
    Phys<C> P = A.P;
    if constexpr (sizeof(C) == 4) {
        C *v[] = {&P.a, &P.b, &P.R, &P.kap, &P.inv_Tc, &P.two_over_Gc2, &P.negG, &P.sig6, &P.lam_e, &P.lam_v,
                  &P.lam_q, &P.lam_pi, &P.divu_a, &P.divu_b, &P.inv_cV, &P.wT0, &P.wT1, &P.inv_csT2, &P.kappa,
                  &P.gam_q, &P.gam_pi, &P.gx, &P.gy, &P.gz, &P.T_shell};
#pragma unroll
        for (int i = 0; i < 25; ++i)
            if ((kConstInVgpr >> i) & 1) asm("" : "+v"(*v[i]));
    }
    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const PopIO<E, typename ST::R, BUF, QT> io(A.pop_in, A.pop_out, A.stride, A.buf_lo_bytes, A.buf_hi_bytes);

    const int itx = logical % A.ntx;
    const int rest = logical / A.ntx;
    const int ity = rest % A.nty;
    const int izc = rest / A.nty;
    const int x0 = itx * tile_x, y0 = ity * tile_y, z0 = izc * A.cz;
    const int zend = min(z0 + A.cz, nz);

    const int tid = threadIdx.x;
    const int tx = tid % tile_x, ty = tid / tile_x;
    const int x = x0 + tx, y = y0 + ty;
    // in_tile: the thread owns a tile node (all threads unless FIT)
    const bool in_tile = !FIT || tid < NTL;
    const bool active = in_tile && x < nx && y < ny;
    const int xw = x % nx, yw = y % ny;
    const int li = (ty + 1) * EX + (tx + 1);
    const unsigned irow = (unsigned)yw * nx + xw;
    // Whole-row tile: offset of the second LDS entry of a first- or last-column node.
    auto wrap_copy = [&](int ex) -> int {
        return !wrapx ? 0 : (ex == 0 ? tile_x : (ex == tile_x - 1 ? -tile_x : 0));
    };
    const int ldup = wrap_copy(tx);

    // Halo position owned by this thread (tid < NH): the rows below and above
    // the tile, then (not for whole-row tiles) the columns left and right of it.
    const bool has_halo = tid < NH;
    unsigned hrow = 0;
    int hli = 0, hdup = 0;
    if (has_halo) {
        int ex, ey;
        if (wrapx) {
            ey = tid < tile_x ? -1 : tile_y;
            ex = tid < tile_x ? tid : tid - tile_x;
        }
        else if (tid < EX) { ex = tid - 1; ey = -1; }
        else if (tid < 2 * EX) { ex = tid - EX - 1; ey = tile_y; }
        else if (tid < 2 * EX + tile_y) { ex = -1; ey = tid - 2 * EX; }
        else { ex = tile_x; ey = tid - 2 * EX - tile_y; }
        const int hx = ((x0 + ex) % nx + nx) % nx;
        const int hy = ((y0 + ey) % ny + ny) % ny;
        hrow = (unsigned)hy * nx + hx;
        hli = (ey + 1) * EX + (ex + 1);
        hdup = wrap_copy(ex);
    }

    auto zmap = [&](int zp) -> int {
        if (WALLS) return zp < 0 ? 0 : (zp > nz - 1 ? nz - 1 : zp);
        int zz = zp % nz;
        return zz < 0 ? zz + nz : zz;
    };

    // kPop / 2 words hold f_0..f_18, g_0..g_{QT-1}; references of the
    // element's width are one more.
    constexpr int WORDS = REF_IN_PAIR ? LY::kPairs : LY::kPairs - 1;
    using Pops = NodePops<C, QT>;
    using Node = std::conditional_t<PAIR, NodeWords<C, PairWord<E>, WORDS>, Pops>;
    // The node's values in the compute type.
    auto decode = [&](const Node &n) -> Pops {
        if constexpr (PAIR) {
            Pops d;
#pragma unroll
            for (int p = 0; p < WORDS; ++p) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int a = LY::member(p, h);
                    const E x = pair_half<E>(n.w[p], h);
                    if (a < 19) {
                        d.e[a] = ST::dec(x);
                    } else if (a < LY::kPop) {
                        d.r[a - 19] = ST::dec(x);
                    } else if constexpr (REF_IN_PAIR) {
                        const C ref = ST::rdec(__builtin_bit_cast(typename ST::R, x));
                        if (a == LY::kPop) d.br = ref;
                        else d.bt = ref;
                    }
                }
            }
            if constexpr (!REF_IN_PAIR) {
                d.br = n.br;
                d.bt = n.bt;
            }
            return d;
        } else {
            return n;
        }
    };
    // Node `row` (index inside an x-y plane) of the plane starting at node zoff.
    auto load_node = [&](unsigned row, unsigned zoff, Node &n) {
        if constexpr (PAIR) {
#pragma unroll
            for (int p = 0; p < WORDS; ++p) n.w[p] = io.load_pair(p, row * NS, (ZOff)zoff * NS);
            if constexpr (DEV && !REF_IN_PAIR) {
                n.br = ST::rdec(io.load_ref(0, row * RSZ, (ZOff)zoff * RSZ));
                n.bt = ST::rdec(io.load_ref(1, row * RSZ, (ZOff)zoff * RSZ));
            } else if constexpr (!DEV) {
                n.br = C(0);
                n.bt = C(0);
            }
        } else {
#pragma unroll
            for (int a = 0; a < 19; ++a) n.e[a] = ST::dec(io.load(a, row * NS, (ZOff)zoff * NS));
#pragma unroll
            for (int a = 0; a < QT; ++a) n.r[a] = ST::dec(io.load(G0 + a, row * NS, (ZOff)zoff * NS));
            if constexpr (DEV) {
                n.br = ST::rdec(io.load_ref(0, row * RSZ, (ZOff)zoff * RSZ));
                n.bt = ST::rdec(io.load_ref(1, row * RSZ, (ZOff)zoff * RSZ));
            } else {
                n.br = C(0);
                n.bt = C(0);
            }
        }
    };
    // Plane buffers of the software pipeline (below): plane z, plane z+1
    // (tile, halo node), plane z+2 (tile node; halo node where it is loaded
    // before the barrier).  Where the loads of the halo node of plane z+2 are
    // issued (measured per format and lattice, see the pipeline):
    //   1: inside the collision of plane z, before its streaming stores;
    //   2: after the collision (FP16 with the D3Q19 temperature lattice).
    Node cur, nxt, nxh, nq;
    constexpr int HALO_AT = (QT == 19 && sizeof(E) == 2) ? 2 : 1;
    __shared__ PairWord<E> s_node[STASH ? WORDS : 1][STASH ? NT : 1];
    __shared__ C s_nref[STASH && !REF_IN_PAIR && DEV ? 2 : 1][STASH ? NT : 1];
    auto stash_store = [&](const Node &n) {
        if constexpr (STASH) {
#pragma unroll
            for (int p = 0; p < WORDS; ++p) s_node[p][tid] = n.w[p];
            if constexpr (!REF_IN_PAIR && DEV) {
                s_nref[0][tid] = n.br;
                s_nref[1][tid] = n.bt;
            }
        }
    };
    auto stash_load = [&](Node &n) {
        if constexpr (STASH) {
#pragma unroll
            for (int p = 0; p < WORDS; ++p) n.w[p] = s_node[p][tid];
            if constexpr (!REF_IN_PAIR && DEV) {
                n.br = s_nref[0][tid];
                n.bt = s_nref[1][tid];
            } else {
                n.br = C(0);
                n.bt = C(0);
            }
        }
    };
    // State of plane zp for this thread's tile node and its halo node.
    auto load_plane = [&](int zp, Node &k, Node &h) {
        const unsigned zoff = (unsigned)zmap(zp) * plane;
        if (in_tile) load_node(irow, zoff, k);
        if (has_halo) load_node(hrow, zoff, h);
    };

    // rho = rho_r + sum e / K and T = T_r + sum r / K of a loaded node.
    auto node_rho = [&](const Pops &n) -> C {
        if constexpr (DEV) return fmad(sum19(n.e), IK, n.br);
        else return sum19(n.e);
    };
    auto node_T = [&](const Pops &n) -> C {
        if constexpr (DEV) return fmad(sum_T<QT>(n.r), IK, n.bt);
        else return sum_T<QT>(n.r);
    };
    // rho, T, psi (and the rounded references) of a loaded plane, tile node
    // and halo node, into LDS slot `slot`.
    // u of the tile and halo nodes of plane zp into ring slot `slot`
    // (finite-difference divergence only).
    __shared__ C s_u[DFD ? 4 : 1][3][DFD ? NE : 1];
    auto plane_velocity = [&](int slot, int zp) {
        const size_t zoff = (size_t)zmap(zp) * plane;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (in_tile) s_u[slot][c][li] = A.ustage[c * A.unn + zoff + irow];
            if (has_halo) s_u[slot][c][hli] = A.ustage[c * A.unn + zoff + hrow];
        }
    };
    // One node's entries of LDS ring slot `slot`.
    auto ring_put = [&](int slot, int i, C psi, C rho, C T) {
        s_psi[slot][i] = psi;
        s_rho[slot][i] = rho;
        if constexpr (OWN_RREF) s_rref[slot][i] = ST::rdec(ST::renc(rho));
        if constexpr (DEV) s_tref[slot][i] = ST::rdec(ST::renc(T));
    };
    auto plane_moments = [&](int slot, const Node &kraw, const Node &hraw, C &krho, C &kT, C &kpsi) {
        bool bad = false;
        krho = kT = kpsi = C(0);
        if (in_tile) {
            const Pops k = decode(kraw);
            const C rho = node_rho(k), T = node_T(k);
            const C p2 = psi_squared(P, rho, T);
            // Unstable node (rho <= 0, psi^2 < 0 or NaN): one flag update per wave.
            bad = active && (!(rho > C(0)) || !(p2 >= C(0)));
            const C psi = Num<C>::sqrt(p2 > C(0) ? p2 : C(0));
            ring_put(slot, li, psi, rho, T);
            if (FIT && ldup) ring_put(slot, li + ldup, psi, rho, T);
            krho = rho;
            kT = T;
            kpsi = psi;
        }
        const unsigned long long badmask = __ballot(bad);
        if (badmask && __lane_id() == (unsigned)(__ffsll(badmask) - 1)) atomicOr(A.status, 1u);
        if (has_halo) {
            const Pops h = decode(hraw);
            const C hr = node_rho(h), hT = node_T(h);
            const C hp2 = psi_squared(P, hr, hT);
            const C hpsi = Num<C>::sqrt(hp2 > C(0) ? hp2 : C(0));
            ring_put(slot, hli, hpsi, hr, hT);
            if (FIT && hdup) ring_put(slot, hli + hdup, hpsi, hr, hT);
        }
    };

    // Streaming byte offsets inside a plane (periodic in x and y).
    const int xm = xw == 0 ? nx - 1 : xw - 1, xp = xw == nx - 1 ? 0 : xw + 1;
    const int ym = yw == 0 ? ny - 1 : yw - 1, yp = yw == ny - 1 ? 0 : yw + 1;
    const unsigned Xo[3] = {(unsigned)xm * NS, (unsigned)xw * NS, (unsigned)xp * NS};
    const unsigned Yo[3] = {(unsigned)ym * nx * NS, (unsigned)yw * nx * NS, (unsigned)yp * nx * NS};
    C T_bottom = C(0);
    if (WALLS) {
        const double dx = xw - P.cx, dy = yw - P.cy;
        T_bottom = (C)(dx * dx + dy * dy <= P.patch_r2 ? P.T_patch : P.T_wall);
    }
    const C rho_ave = (C)(*A.rho_ave);
    double rho_sum = 0.0;

    // Collision and streaming of the tile node at plane z (slot s of the ring
    // holds plane z; s-1 and s+1 its neighbours).  All population-space
    // quantities (moments, equilibria, sources, post-collision values) are
    // carried K-scaled, so the stored values convert without a multiply.
    auto collide_stream = [&](int z, int s, const Node &ndraw, C rho, C T, C psi) {
        const Pops nd = decode(ndraw);
        const int sm = (s + 3) & 3, s0 = s & 3, sp = (s + 1) & 3;
        const int sl[3] = {sm, s0, sp};
        // Eq. (7) and the isotropic gradient: omega(1) = 1/6, omega(2) = 1/12.
#define NB(arr, sl, dx, dy) arr[sl][li + (dy) * EX + (dx)]
#define STENCIL(arr, OX, OY, OZ)                                                                                    \
    {                                                                                                               \
        const C xy = NB(arr, s0, 1, 1) - NB(arr, s0, -1, -1), xmy = NB(arr, s0, 1, -1) - NB(arr, s0, -1, 1);        \
        const C xz = NB(arr, sp, 1, 0) - NB(arr, sm, -1, 0), xmz = NB(arr, sm, 1, 0) - NB(arr, sp, -1, 0);          \
        const C yz = NB(arr, sp, 0, 1) - NB(arr, sm, 0, -1), ymz = NB(arr, sm, 0, 1) - NB(arr, sp, 0, -1);          \
        OX = fmad(C(1.0 / 6.0), NB(arr, s0, 1, 0) - NB(arr, s0, -1, 0), C(1.0 / 12.0) * ((xy + xmy) + (xz + xmz))); \
        OY = fmad(C(1.0 / 6.0), NB(arr, s0, 0, 1) - NB(arr, s0, 0, -1), C(1.0 / 12.0) * ((xy - xmy) + (yz + ymz))); \
        OZ = fmad(C(1.0 / 6.0), NB(arr, sp, 0, 0) - NB(arr, sm, 0, 0), C(1.0 / 12.0) * ((xz - xmz) + (yz - ymz))); \
    }
        C Spx, Spy, Spz, grx, gry, grz;
        STENCIL(s_psi, Spx, Spy, Spz)
        STENCIL(s_rho, grx, gry, grz)
#undef STENCIL
#undef NB
        const C inv_rho = Num<C>::rcp(rho);
        const C gpsi = P.negG * psi;
        const C fmx = gpsi * Spx, fmy = gpsi * Spy, fmz = gpsi * Spz;
        C Fx = fmx, Fy = fmy, Fz = fmz;
        if (P.gravity) {
            const C drho = rho - rho_ave;
            Fx = fmad(drho, P.gx, Fx);
            Fy = fmad(drho, P.gy, Fy);
            Fz = fmad(drho, P.gz, Fz);
        }
        // K-scaled force and density (K = 1 for the plain formats).
        const C FxK = K * Fx, FyK = K * Fy, FzK = K * Fz, rhoK = K * rho, inv_rhoK = IK * inv_rho;
        // Moments as deviations from the rest equilibrium w rho.  The rest
        // part is conserved by the collision (Lambda_0 = 1, S_0 = 0, and
        // m_eq(rho, 0) relaxes onto itself), so it is added back to f* at the
        // end instead of being carried through O(rho) sums.  With e the
        // stored values K (f - w rho_r), K (rho - rho_r) = sum e plays the
        // role of rho in the rest-part subtraction.
        C m[19];
        moments19<C, true>(nd.e, m, K * (rho - nd.br));
        // Eq. (10)
        const C ux = fmad(C(0.5), FxK, m[1]) * inv_rhoK;
        const C uy = fmad(C(0.5), FyK, m[2]) * inv_rhoK;
        const C uz = fmad(C(0.5), FzK, m[3]) * inv_rhoK;
        // Eq. (5) for m5..m15, and the deviations from m_eq(rho, 0) of m4
        // and m16..m18 (m4 - rho, m16..18 - rho/9).
        constexpr C cs2 = C(1.0 / 3.0);
        const C rux = rhoK * ux, ruy = rhoK * uy, ruz = rhoK * uz;
        const C r3 = rhoK * cs2;
        const C rxx = rux * ux, ryy = ruy * uy, rzz = ruz * uz;  // rho u_i^2
        const C r6 = C(0.5) * cs2 * (rxx + ryy + rzz);           // rho |u|^2 / 6
        C meq[19];
        meq[4] = rxx + ryy + rzz;
        meq[5] = C(2) * rxx - ryy - rzz;
        meq[6] = ryy - rzz;
        meq[7] = rux * uy;
        meq[8] = rux * uz;
        meq[9] = ruy * uz;
        meq[10] = fmad(rxx, uy, r3 * uy);
        meq[11] = fmad(ryy, ux, r3 * ux);
        meq[12] = fmad(rxx, uz, r3 * uz);
        meq[13] = fmad(rzz, ux, r3 * ux);
        meq[14] = fmad(ryy, uz, r3 * uz);
        meq[15] = fmad(rzz, uy, r3 * uy);
        meq[16] = fmad(cs2, rxx + ryy, -r6);
        meq[17] = fmad(cs2, rxx + rzz, -r6);
        meq[18] = fmad(cs2, ryy + rzz, -r6);
        // Eq. (9)
        const C xFx = ux * FxK, yFy = uy * FyK, zFz = uz * FzK;
        const C Fu = xFx + yFy + zFz;
        const C fm2 = fmad(fmx, fmx, fmad(fmy, fmy, fmz * fmz));
        const C S4 = fmad(P.sig6 * K * fm2, Num<C>::rcp(psi * psi), C(2) * Fu);
        // Eq. (3): m* = m + Lambda (m_eq - m) + (I - Lambda/2) S
        C ms[19];
        ms[0] = C(0);
        ms[1] = m[1] + FxK;
        ms[2] = m[2] + FyK;
        ms[3] = m[3] + FzK;
        ms[4] = fmad(P.lam_e, meq[4] - m[4], fmad(C(1) - C(0.5) * P.lam_e, S4, m[4]));
        const C hv = C(1) - C(0.5) * P.lam_v;
        ms[5] = fmad(P.lam_v, meq[5] - m[5], fmad(hv * C(2), C(2) * xFx - yFy - zFz, m[5]));
        ms[6] = fmad(P.lam_v, meq[6] - m[6], fmad(hv * C(2), yFy - zFz, m[6]));
        ms[7] = fmad(P.lam_v, meq[7] - m[7], fmad(hv, fmad(FxK, uy, FyK * ux), m[7]));
        ms[8] = fmad(P.lam_v, meq[8] - m[8], fmad(hv, fmad(FxK, uz, FzK * ux), m[8]));
        ms[9] = fmad(P.lam_v, meq[9] - m[9], fmad(hv, fmad(FyK, uz, FzK * uy), m[9]));
        const C hq = (C(1) - C(0.5) * P.lam_q) * cs2;
        ms[10] = fmad(P.lam_q, meq[10] - m[10], fmad(hq, FyK, m[10]));
        ms[11] = fmad(P.lam_q, meq[11] - m[11], fmad(hq, FxK, m[11]));
        ms[12] = fmad(P.lam_q, meq[12] - m[12], fmad(hq, FzK, m[12]));
        ms[13] = fmad(P.lam_q, meq[13] - m[13], fmad(hq, FxK, m[13]));
        ms[14] = fmad(P.lam_q, meq[14] - m[14], fmad(hq, FzK, m[14]));
        ms[15] = fmad(P.lam_q, meq[15] - m[15], fmad(hq, FyK, m[15]));
        const C hp = (C(1) - C(0.5) * P.lam_pi) * C(2) * cs2;
        ms[16] = fmad(P.lam_pi, meq[16] - m[16], fmad(hp, xFx + yFy, m[16]));
        ms[17] = fmad(P.lam_pi, meq[17] - m[17], fmad(hp, xFx + zFz, m[17]));
        ms[18] = fmad(P.lam_pi, meq[18] - m[18], fmad(hp, yFy + zFz, m[18]));
        C fs[19];  // K (f* - w rho)
        populations19(ms, fs);

        // ---- temperature lattice ----
        // Equilibrium weight of g_a: Eq. (22) on D3Q7, the standard D3Q19
        // weights (the same as those of f) on D3Q19.
        auto wg = [&](int a) -> C {
            if constexpr (QT == 7) return a == 0 ? P.wT0 : P.wT1;
            else return C(w19(a));
        };
        C gs[QT];  // K (g+ - w T_emit)
        const unsigned own = (unsigned)z * plane + irow;
        // Constant-temperature boundary (Sec. IV A): the outer layer of nodes
        // is a reservoir at T_shell.  It emits w T_shell without collision,
        // and every population streamed into it is replaced by w T_shell.
        bool xs[3] = {false, false, false}, ys[3] = {false, false, false}, zs[3] = {false, false, false};
        bool own_shell = false;
        if (!WALLS && P.shell) {
            const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
            xs[0] = xm == 0 || xm == nx - 1;
            xs[1] = xw == 0 || xw == nx - 1;
            xs[2] = xp == 0 || xp == nx - 1;
            ys[0] = ym == 0 || ym == ny - 1;
            ys[1] = yw == 0 || yw == ny - 1;
            ys[2] = yp == 0 || yp == ny - 1;
            zs[0] = zm == 0 || zm == nz - 1;
            zs[1] = z == 0 || z == nz - 1;
            zs[2] = zp == 0 || zp == nz - 1;
            own_shell = xs[1] || ys[1] || zs[1];
        }
        const C T_emit = own_shell ? P.T_shell : T;
        if (own_shell) {
#pragma unroll
            for (int a = 0; a < QT; ++a) gs[a] = C(0);
        } else if (P.thermal) {
            // Eq. (48): local velocity divergence (pre-collision m_4).
            C divu = fmad(P.divu_b, S4, -fmad(P.divu_a, m[4] - meq[4], C(2) * Fu)) * (C(1.5) * inv_rhoK);
            if (DFD && (!WALLS || (z > 0 && z < nz - 1))) {
                // The practice Eq. (48) replaces: sum omega(|e|^2) e . u(x + e)
                // over the 18 neighbours at interior nodes.
#define NU(c, sl, dx, dy) s_u[sl][c][li + (dy) * EX + (dx)]
                const C ax = (NU(0, s0, 1, 0) - NU(0, s0, -1, 0)) + (NU(1, s0, 0, 1) - NU(1, s0, 0, -1)) +
                             (NU(2, sp, 0, 0) - NU(2, sm, 0, 0));
                const C dxy = ((NU(0, s0, 1, 1) + NU(1, s0, 1, 1)) - (NU(0, s0, -1, -1) + NU(1, s0, -1, -1))) +
                              ((NU(0, s0, 1, -1) - NU(1, s0, 1, -1)) - (NU(0, s0, -1, 1) - NU(1, s0, -1, 1)));
                const C dxz = ((NU(0, sp, 1, 0) + NU(2, sp, 1, 0)) - (NU(0, sm, -1, 0) + NU(2, sm, -1, 0))) +
                              ((NU(0, sm, 1, 0) - NU(2, sm, 1, 0)) - (NU(0, sp, -1, 0) - NU(2, sp, -1, 0)));
                const C dyz = ((NU(1, sp, 0, 1) + NU(2, sp, 0, 1)) - (NU(1, sm, 0, -1) + NU(2, sm, 0, -1))) +
                              ((NU(1, sm, 0, 1) - NU(2, sm, 0, 1)) - (NU(1, sp, 0, -1) - NU(2, sp, 0, -1)));
#undef NU
                divu = fmad(C(1.0 / 6.0), ax, C(1.0 / 12.0) * ((dxy + dxz) + dyz));
            }
            // First moments sum e g (the reference part w T_r cancels): n1..n3
            // of Eq. (38) on D3Q7, the same sums over the 19 velocities on D3Q19.
            C n1, n2, n3, n5 = C(0), n6 = C(0);
            if constexpr (QT == 7) {
                n1 = nd.r[1] - nd.r[2];
                n2 = nd.r[3] - nd.r[4];
                n3 = nd.r[5] - nd.r[6];
                const C a12 = nd.r[1] + nd.r[2], a34 = nd.r[3] + nd.r[4], a56 = nd.r[5] + nd.r[6];
                n5 = a12 - a34;
                n6 = a12 - a56;
            } else {
                C mt[19];
                moments19<C, false>(nd.r, mt);
                n1 = mt[1];
                n2 = mt[2];
                n3 = mt[3];
            }
            const C chi = P.kappa_mode ? P.kappa : P.kappa * inv_rho * P.inv_cV;
            const C inv_vsT = Num<C>::rcp(fmad(chi, P.inv_csT2, C(0.5)));
            // Eq. (45) (D3Q7 MRT) or Eq. (36) (BGK, tau_g = varsigma_T): local
            // temperature gradient (n is K-scaled).
            const C kgr = -inv_vsT * (P.inv_csT2 * IK);
            const C dTx = kgr * n1, dTy = kgr * n2, dTz = kgr * n3;
            // Eq. (18) with (dp/dT)_rho = rho R/(1 - b rho), constant c_V.
            const C cr = chi * inv_rho;
            const C adv = fmad(fmad(cr, grx, -ux), dTx, fmad(fmad(cr, gry, -uy), dTy, fmad(cr, grz, -uz) * dTz));
            const C phis = fmad(-T * P.R * P.inv_cV, Num<C>::rcp(fmad(-P.b, rho, C(1))) * divu, adv);
            // Eqs. (23)-(24): Q = w (1.5 phi_s - 0.5 phi_s(t-1))
            C *phi_own = A.phi + own;
            const C qs = fmad(C(1.5), phis, C(-0.5) * *phi_own);
            const C keep = C(1) - inv_vsT;
            if constexpr (QT == 7) {
                // Eq. (39) with Eq. (42)-(43); n4 is carried as its deviation
                // n4 - d T = (1 - d) T - g0 = w0 (T - T_r) - (g0 - w0 T_r).
                const C s1 = n1 * keep, s2 = n2 * keep, s3 = n3 * keep;
                // The BGK collision of Eq. (19) is the MRT one with every rate 1/tau_g = 1/varsigma_T.
                const C gq = P.thermal_bgk ? inv_vsT : P.gam_q, gp = P.thermal_bgk ? inv_vsT : P.gam_pi;
                const C s4 = fmad(K * P.wT0, T - nd.bt, -nd.r[0]) * (C(1) - gq);
                const C s5 = n5 * (C(1) - gp), s6 = n6 * (C(1) - gp);
                const C Q0 = (K * P.wT0) * qs, Q1 = (K * P.wT1) * qs;
                // Eq. (40)-(41): g+ = N^-1 n* + Q = w T + N^-1 (n* - n_eq) + Q
                const C c456 = (s4 + s5 + s6) * C(1.0 / 6.0);
                const C c3 = (s4 - C(2) * s5 + s6) * C(1.0 / 6.0), c5 = (s4 + s5 - C(2) * s6) * C(1.0 / 6.0);
                gs[0] = Q0 - s4;
                gs[1] = fmad(C(0.5), s1, c456) + Q1;
                gs[2] = fmad(C(-0.5), s1, c456) + Q1;
                gs[3] = fmad(C(0.5), s2, c3) + Q1;
                gs[4] = fmad(C(-0.5), s2, c3) + Q1;
                gs[5] = fmad(C(0.5), s3, c5) + Q1;
                gs[6] = fmad(C(-0.5), s3, c5) + Q1;
            } else {
                // Eq. (19) with g_eq = w T: K (g+ - w T) = K (g - w T)(1 - 1/tau_g) + K w Q,
                // where K (g - w T) = r - K w (T - T_r) (T_r = 0 for plain storage).
                const C dT = T - nd.bt;
#pragma unroll
                for (int a = 0; a < 19; ++a) {
                    const C wK = C(K * w19(a));
                    gs[a] = fmad(fmad(-wK, dT, nd.r[a]), keep, wK * qs);
                }
            }
            *phi_own = phis;
        }

        if constexpr (HALO_AT == 1) {
            // the halo node of plane z+2 (nxh was consumed by the moments of z+1)
            if (z + 2 <= zend && has_halo) load_node(hrow, (unsigned)zmap(z + 2) * plane, nxh);
        }
        // ---- streaming (push), Eq. (4) and Eq. (40) ----
        const ZOff PB = (ZOff)plane * NS;
        const ZOff Zc = (ZOff)z * PB;
        ZOff Zo[3];
        if (WALLS) {
            Zo[0] = z > 0 ? Zc - PB : ZOff(0);
            Zo[1] = Zc;
            Zo[2] = z < nz - 1 ? Zc + PB : ZOff(0);
        } else {
            Zo[0] = (ZOff)(z == 0 ? nz - 1 : z - 1) * PB;
            Zo[1] = Zc;
            Zo[2] = (ZOff)(z == nz - 1 ? 0 : z + 1) * PB;
        }
        const unsigned rowb = irow * NS;
        // Values stored for the D3Q19 population a bound for the node in ring
        // slot `slot` at offset (dx, dy).  Plain storage keeps f* (the rest
        // part r0 closes the sum exactly: the rounded 1/3 + 6/18 + 12/36 is
        // not 1).  Deviation storage encodes K (f* - w rho_r(dest)) as
        // A_a + K w (rho_r(own) - rho_r(dest)) with A_a = K (f* - w rho_r(own)),
        // so that A_a carries no O(rho) part.  (The one-FMA form
        // fs_a + K w (rho - rho_r(dest)) has fewer instructions but makes the
        // batch kernel spill scalar registers: measured 7% slower there.)
        auto rref = [&](int slot, int idx) -> C {
            if constexpr (OWN_RREF) return s_rref[slot][idx];
            else return s_rho[slot][idx];
        };
        C own_rref = C(0), own_tref = C(0);
        if constexpr (DEV) {
            own_rref = rref(s0, li);
            own_tref = s_tref[s0][li];
        }
        const C r1 = rho * C(1.0 / 18.0), r2 = rho * C(1.0 / 36.0);
        const C r0 = rho - fmad(C(6), r1, C(12) * r2);
        C fa[19];
#pragma unroll
        for (int a = 0; a < 19; ++a) {
            if constexpr (DEV) fa[a] = fmad(C(K * w19(a)), rho - own_rref, fs[a]);
            else fa[a] = fs[a] + (a == 0 ? r0 : (a < 7 ? r1 : r2));
        }
        // Random bits of the stochastic rounding (FP16, BF16): a hash of the
        // node's index in the lattice and of the FP32 bits of its rho and T
        // (which change from step to step wherever the field evolves).  A
        // function of the node's data only, so results do not depend on the
        // launch shape.  The seed's upper half, which depends on every bit
        // of the products, is folded into the lower one; word k = (seed ^ c_k)
        // * m is then a bijection of the seed, so its top and bottom
        // kSrBits-bit fields are independent draws: f_a takes the top field
        // of word a, g_a the bottom one, and the D3Q19 populations without a
        // temperature partner (a >= QT) share words two by two.
        unsigned sr_seed = own;
        if constexpr (sizeof(C) == 4) {
            sr_seed = (own ^ (__builtin_bit_cast(unsigned, rho) * 0x9E3779B1u)) ^
                      (__builtin_bit_cast(unsigned, T) * 0x85EBCA77u);
            sr_seed ^= sr_seed >> 16;
        }
        auto srw = [&](int k) -> unsigned { return (sr_seed ^ (0x9E3779B9u * (unsigned)(k + 1))) * 0x7FEB352Du; };
        auto srr = [&](int a) -> unsigned {
            if constexpr (HasStochasticRounding<ST>::value) {
                constexpr int B = ST::kSrBits;
                constexpr unsigned lo = (1u << B) - 1u;
                if (a >= G0) return srw(a - G0) & lo;
                if (a < QT) return srw(a) >> (32 - B);
                const int k = QT + (a - QT) / 2;
                return ((a - QT) & 1) ? (srw(k) & lo) : (srw(k) >> (32 - B));
            } else {
                return 0u;
            }
        };
        // Value stored for population a at its destination (before encoding).
        auto fdest = [&](int a, int slot, int dx, int dy) -> C {
            if constexpr (DEV) return fmad(C(K * w19(a)), own_rref - rref(slot, li + dy * EX + dx), fa[a]);
            else return fa[a];
        };
        auto fval = [&](int a, int slot, int dx, int dy) -> E { return ST::enc_r(fdest(a, slot, dx, dy), srr(a)); };
        // g+ = w T_emit + gs; the deviation formats encode against the
        // destination's T_r as above.  A destination in the reservoir layer
        // receives w T_shell.  Plain storage forms the rest part as T minus
        // the moving ones, so that the weights sum to 1 exactly.
        auto wtimes = [&](int a, C t) -> C {
            if constexpr (QT == 7) {
                const C w1 = P.wT1 * t;
                return a == 0 ? t - C(6) * w1 : w1;
            } else {
                const C t1 = t * C(1.0 / 18.0), t2 = t * C(1.0 / 36.0);
                return a == 0 ? t - fmad(C(6), t1, C(12) * t2) : (a < 7 ? t1 : t2);
            }
        };
        C ga[QT];
#pragma unroll
        for (int a = 0; a < QT; ++a) {
            if constexpr (DEV) ga[a] = fmad(K * wg(a), T_emit - own_tref, gs[a]);
            else ga[a] = wtimes(a, T_emit) + gs[a];
        }
        auto gval = [&](int a, int slot, int dx, int dy, bool to_shell) -> C {
            if constexpr (DEV) {
                const C bd = s_tref[slot][li + dy * EX + dx];
                const C wK = K * wg(a);
                if (to_shell) return wK * (P.T_shell - bd);
                return fmad(wK, own_tref - bd, ga[a]);
            } else {
                if (to_shell) return wtimes(a, P.T_shell);
                return ga[a];
            }
        };
        bool stored = false;
        if constexpr (PAIR && !WALLS) {
          if (P.thermal) {
            stored = true;
            // f_a and g_a of the same velocity (a < QT) go to the same
            // neighbour and share a word of the paired layout: one store.
#pragma unroll
            for (int a = 0; a < QT; ++a) {
                const int ex = kE19X[a], ey = kE19Y[a], ez = kE19Z[a];
                const bool to_shell = xs[ex + 1] || ys[ey + 1] || zs[ez + 1];
                io.store_pair(LY::pair_of(a), Yo[ey + 1] + Xo[ex + 1], Zo[ez + 1],
                              ST::enc_pair_r(fdest(a, sl[ez + 1], ex, ey), srr(a),
                                             gval(a, sl[ez + 1], ex, ey, to_shell), srr(G0 + a)));
            }
            // The others two at a time (one conversion), stored half by half.
            static_assert((19 - QT) % 2 == 0, "D3Q19 populations without a partner come in pairs");
#pragma unroll
            for (int a = QT; a < 19; a += 2) {
                const int ex = kE19X[a], ey = kE19Y[a], ez = kE19Z[a];
                const int ex1 = kE19X[a + 1], ey1 = kE19Y[a + 1], ez1 = kE19Z[a + 1];
                const PairWord<E> w = ST::enc_pair_r(fdest(a, sl[ez + 1], ex, ey), srr(a),
                                                     fdest(a + 1, sl[ez1 + 1], ex1, ey1), srr(a + 1));
                io.store(a, Yo[ey + 1] + Xo[ex + 1], Zo[ez + 1], pair_half<E>(w, 0));
                io.store(a + 1, Yo[ey1 + 1] + Xo[ex1 + 1], Zo[ez1 + 1], pair_half<E>(w, 1));
            }
            if constexpr (REF_IN_PAIR) {
                io.store_pair(LY::pair_of(LY::kPop), rowb, Zc,
                              pack_pair<E>(__builtin_bit_cast(E, ST::renc(rho)), __builtin_bit_cast(E, ST::renc(T))));
            } else if constexpr (DEV) {
                io.store_ref(0, irow * RU, (ZOff)z * plane * RU, ST::renc(rho));
                io.store_ref(1, irow * RU, (ZOff)z * plane * RU, ST::renc(T));
            }
          }
        }
        if (!stored) {
    #pragma unroll
            for (int a = 0; a < 19; ++a) {
                const int ex = kE19X[a], ey = kE19Y[a], ez = kE19Z[a];
                const unsigned inrow = Yo[ey + 1] + Xo[ex + 1];
                if (WALLS) {
                    if (ez < 0 && z == 0) {  // Eq. (50): halfway bounce-back into the own node
                        io.store(opposite(a), rowb, Zc, ST::enc_r(fa[a], srr(a)));
                        continue;
                    }
                    if (ez > 0 && z == nz - 1) {  // Eq. (50) at a top wall, or out through the open top
                        if (P.top_wall) io.store(opposite(a), rowb, Zc, ST::enc_r(fa[a], srr(a)));
                        continue;
                    }
                    if (ez < 0 && z == nz - 1 && !P.top_wall)  // open top: unknown f copied from below
                        io.store(a, inrow, Zc, fval(a, s0, ex, ey));
                }
                io.store(a, inrow, Zo[ez + 1], fval(a, sl[ez + 1], ex, ey));
            }
            if (P.thermal) {
    #pragma unroll
                for (int a = 0; a < QT; ++a) {
                    const int ex = kE19X[a], ey = kE19Y[a], ez = kE19Z[a];  // Eq. (21) is the first 7 of Eq. (2)
                    if (WALLS) {
                        // Eq. (51): g_opp(x_b) = -g+_a(x_b) + 2 w T_w, into the own node
                        const bool bottom = ez < 0 && z == 0, top = ez > 0 && z == nz - 1;
                        if (bottom || top) {
                            const C Tw = bottom ? T_bottom : (C)P.T_top;
                            const C v = DEV ? fmad(K * wg(a), C(2) * Tw - T - own_tref, -gs[a])
                                            : fmad(C(2) * wg(a), Tw, -ga[a]);
                            io.store(G0 + opposite(a), rowb, Zc, ST::enc_r(v, srr(G0 + a)));
                            continue;
                        }
                    }
                    const bool to_shell = xs[ex + 1] || ys[ey + 1] || zs[ez + 1];
                    io.store(G0 + a, Yo[ey + 1] + Xo[ex + 1], Zo[ez + 1],
                             ST::enc_r(gval(a, sl[ez + 1], ex, ey, to_shell), srr(G0 + a)));
                }
            } else {
                // temperature held fixed: g stays at the node (re-encoded against the new reference)
    #pragma unroll
                for (int a = 0; a < QT; ++a) {
                    const C v = DEV ? fmad(K * wg(a), nd.bt - own_tref, nd.r[a]) : nd.r[a];
                    io.store(G0 + a, rowb, Zc, ST::enc_r(v, srr(G0 + a)));
                }
            }
            if constexpr (DEV) {
                io.store_ref(0, irow * RU, (ZOff)z * plane * RU, ST::renc(rho));
                io.store_ref(1, irow * RU, (ZOff)z * plane * RU, ST::renc(T));
            }
        }
        if (P.gravity) rho_sum += (double)rho;
    };

    // Velocity pass: u(t) of the tile node at plane z (slot s), computed as in
    // collide_stream (Eq. (7), (10)).
    auto velocity_out = [&](int z, int s, const Node &ndraw, C rho, C psi) {
        const Pops nd = decode(ndraw);
        const int sm = (s + 3) & 3, s0 = s & 3, sp = (s + 1) & 3;
#define NB(dx, dy, sl) s_psi[sl][li + (dy) * EX + (dx)]
        const C xy = NB(1, 1, s0) - NB(-1, -1, s0), xmy = NB(1, -1, s0) - NB(-1, 1, s0);
        const C xz = NB(1, 0, sp) - NB(-1, 0, sm), xmz = NB(1, 0, sm) - NB(-1, 0, sp);
        const C yz = NB(0, 1, sp) - NB(0, -1, sm), ymz = NB(0, 1, sm) - NB(0, -1, sp);
        const C Spx = fmad(C(1.0 / 6.0), NB(1, 0, s0) - NB(-1, 0, s0), C(1.0 / 12.0) * ((xy + xmy) + (xz + xmz)));
        const C Spy = fmad(C(1.0 / 6.0), NB(0, 1, s0) - NB(0, -1, s0), C(1.0 / 12.0) * ((xy - xmy) + (yz + ymz)));
        const C Spz = fmad(C(1.0 / 6.0), NB(0, 0, sp) - NB(0, 0, sm), C(1.0 / 12.0) * ((xz - xmz) + (yz - ymz)));
#undef NB
        const C inv_rho = Num<C>::rcp(rho);
        const C gpsi = P.negG * psi;
        C Fx = gpsi * Spx, Fy = gpsi * Spy, Fz = gpsi * Spz;
        if (P.gravity) {
            const C drho = rho - rho_ave;
            Fx = fmad(drho, P.gx, Fx);
            Fy = fmad(drho, P.gy, Fy);
            Fz = fmad(drho, P.gz, Fz);
        }
        const C inv_rhoK = IK * inv_rho;
        C m[19];
        moments19<C, true>(nd.e, m, K * (rho - nd.br));
        const unsigned own = (unsigned)z * plane + irow;
        A.uout[own] = fmad(C(0.5), K * Fx, m[1]) * inv_rhoK;
        A.uout[A.unn + own] = fmad(C(0.5), K * Fy, m[2]) * inv_rhoK;
        A.uout[2 * A.unn + own] = fmad(C(0.5), K * Fz, m[3]) * inv_rhoK;
    };

    // Software pipeline over the planes of the chunk.  At iteration z the
    // states of plane z (collision) and z+1 (moments) are in registers.  The
    // loads of the tile node of plane z+2 are issued right after the moments
    // of z+1, so that their latency overlaps the barrier and the collision of
    // plane z.  The loads of its halo node are issued inside the collision,
    // before the streaming stores, so that the halo words are not held across
    // the whole collision (HALO_AT above).  Against issuing them with the tile
    // loads (measured, 128^3 / 256^3 evaporation): FP16 +5% / +19%, FP32 +6% /
    // same, BF16 +9%; FP16 with the D3Q19 temperature lattice runs best with
    // them after the collision (+11%; inside it: +3%).  Issuing loads earlier
    // would put more memory operations between a load and its use than the
    // vmcnt counter can express, which forces a full drain.
    C c_rho, c_T, c_psi, n_rho, n_T, n_psi;
    {
        Node t0, th0, h0;
        C a0, a1, a2;
        load_plane(z0 - 1, t0, th0);
        load_plane(z0, cur, h0);
        load_plane(z0 + 1, nxt, nxh);
        plane_moments(0, t0, th0, a0, a1, a2);
        if (WALLS && P.wet && z0 == 0) {
            // The solid layer below z = 0 holds the virtual density and its
            // psi (k_wall_density) instead of a copy of the layer above.
            const unsigned nxy = plane;
            if (in_tile) {
                s_rho[0][li] = (C)A.wall[irow];
                s_psi[0][li] = (C)A.wall[nxy + irow];
            }
            if (has_halo) {
                s_rho[0][hli] = (C)A.wall[hrow];
                s_psi[0][hli] = (C)A.wall[nxy + hrow];
            }
        }
        plane_moments(1, cur, h0, c_rho, c_T, c_psi);
        stash_store(cur);
        if constexpr (DFD) {
            plane_velocity(0, z0 - 1);
            plane_velocity(1, z0);
        }
    }
    for (int z = z0; z < zend; ++z) {
        const int s = z - z0 + 1;
        plane_moments((s + 1) & 3, nxt, nxh, n_rho, n_T, n_psi);
        if constexpr (DFD) plane_velocity((s + 1) & 3, z + 1);
        const unsigned zoff2 = (unsigned)zmap(z + 2) * plane;
        if (!STASH && z + 2 <= zend && in_tile) load_node(irow, zoff2, nq);
        __syncthreads();
        if constexpr (STASH) {
            Node cw;
            stash_load(cw);
            stash_store(nxt);
            // the words of plane z + 2 straight into nxt, now parked in LDS
            if (z + 2 <= zend && in_tile) load_node(irow, zoff2, nxt);
            if (active) {
                if constexpr (VEL) velocity_out(z, s, cw, c_rho, c_psi);
                else collide_stream(z, s, cw, c_rho, c_T, c_psi);
            }
        } else {
            if (active) {
                if constexpr (VEL) velocity_out(z, s, cur, c_rho, c_psi);
                else collide_stream(z, s, cur, c_rho, c_T, c_psi);
            }
            cur = nxt;
        }
        if (!STASH) nxt = nq;
        // Halo loads not issued inside a collision: inactive tile threads,
        // the velocity pass, and HALO_AT == 2.
        if ((HALO_AT == 2 || VEL || !active) && z + 2 <= zend && has_halo) load_node(hrow, zoff2, nxh);
        c_rho = n_rho;
        c_T = n_T;
        c_psi = n_psi;
    }

    if (!VEL && P.gravity) {
        // Deterministic per-workgroup partial sum of rho(t) for rho_ave.
        for (int o = 32; o > 0; o >>= 1) rho_sum += __shfl_xor(rho_sum, o, 64);
        if ((tid & 63) == 0) s_red[tid >> 6] = rho_sum;
        __syncthreads();
        if (tid == 0) {
            double acc = 0.0;
            for (int w = 0; w < NT / 64; ++w) acc += s_red[w];
            A.partials[slot] = acc;
        }
    }
}

// One launch per time step: workgroup b takes tile/chunk xcd_logical_block(b).
template <typename ST, int TX, int TY, bool WALLS, bool BUF, bool DFD>
__global__ void __launch_bounds__(TX *TY) k_step(const StepArgs<ST> A) {
    step_tile<ST, TX, TY, WALLS, BUF, DFD>(A, xcd_logical_block(blockIdx.x, gridDim.x), blockIdx.x);
}

// The velocity pass that precedes a step with the finite-difference
// divergence: u(t) of every node into A.uout.
template <typename ST, int TX, int TY, bool WALLS, bool BUF>
__global__ void __launch_bounds__(TX *TY) k_velocity_pass(const StepArgs<ST> A) {
    step_tile<ST, TX, TY, WALLS, BUF, false, true>(A, xcd_logical_block(blockIdx.x, gridDim.x), blockIdx.x);
}

// Work list of a batch of independent lattices advanced by one launch.
// Items are (lattice, tile/chunk) pairs.  The lattices are dealt to the 8 XCDs
// (balanced by work) and the items of the lattices of XCD x are the range
// [bin_start[x], bin_start[x+1]); item_case[i] is the lattice of item i and
// first_item[c] the number of the first item of lattice c.  Counter x of
// `queue` hands out the items of range x; queue[8] counts workgroups that have
// finished, and the last one resets all nine, so the next launch (or graph
// replay) starts from zero without a memset.
constexpr int kXcds = 8;
struct BatchQueue {
    const unsigned *item_case;
    const unsigned *first_item;
    unsigned *queue;
    unsigned bin_start[kXcds + 1];
};

// Persistent batched step: a fixed grid of workgroups takes items from the
// counters until every range is exhausted, so lattices of uneven size share
// the GPU without a launch per lattice.  Workgroup b runs on XCD b mod 8
// (round-robin dispatch) and drains that XCD's range first, so neighbouring
// tiles of a lattice -- which share halo rows and the cache lines at tile
// edges -- meet in one L2; it then helps with the other ranges.  parity = 1
// swaps the two population copies of every lattice.
template <typename ST, int TX, int TY, bool BUF, bool FIT = false>
__global__ void __launch_bounds__(TX *TY) k_step_batch(const StepArgs<ST> *__restrict__ cases, BatchQueue Q,
                                                       int parity) {
    __shared__ unsigned s_item;
    const int home = (int)(blockIdx.x % kXcds);
    for (int k = 0; k < kXcds; ++k) {
        const int bin = (home + k) % kXcds;
        const unsigned begin = Q.bin_start[bin], count = Q.bin_start[bin + 1] - begin;
        for (;;) {
            if (threadIdx.x == 0) s_item = atomicAdd(Q.queue + bin, 1u);
            __syncthreads();
            const unsigned local = s_item;
            __syncthreads();  // every thread has read s_item, and the previous item's LDS reads are done
            if (local >= count) break;
            const unsigned item = begin + local;
            const unsigned c = Q.item_case[item];
            StepArgs<ST> A = cases[c];
            if (parity) {
                typename ST::T *t = const_cast<typename ST::T *>(A.pop_in);
                A.pop_in = A.pop_out;
                A.pop_out = t;
            }
            step_tile<ST, TX, TY, false, BUF, false, false, FIT>(A, (int)(item - Q.first_item[c]), 0);
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(Q.queue + kXcds, 1u) == gridDim.x - 1) {
            for (int k = 0; k <= kXcds; ++k) atomicExch(Q.queue + k, 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// Helper kernels (one thread per node; not on the per-step path).  They read
// the state in FP64: a node's populations are w rho_r + e (e decoded), so
// rho = rho_r + sum e and rho u = sum e_alpha e_alpha exactly.
// ---------------------------------------------------------------------------

template <typename ST>
struct NodeView {
    static constexpr int QT = ST::kQT, kPopPlanes = PopLayout<QT>::kPop;
    const typename ST::T *pop;
    size_t st;
    __device__ double e(int a, size_t i) const { return ST::ddec(pop[element_index<typename ST::T, QT>(a, st, i)]); }
    __device__ double ref(int k, size_t i) const {
        if constexpr (ST::kDev && sizeof(typename ST::R) == sizeof(typename ST::T)) {
            return (double)ST::rdec(__builtin_bit_cast(typename ST::R, pop[element_index<typename ST::T, QT>(kPopPlanes + k, st, i)]));
        } else if constexpr (ST::kDev) {
            const typename ST::R *refs = reinterpret_cast<const typename ST::R *>(pop + kPopPlanes * st);
            return (double)ST::rdec(refs[k * st + i]);
        }
        else return 0.0;
    }
};

// Initial state from FP64 fields: f = M^-1 m_eq(rho, u), g = w T, phi = 0;
// sets status bit 2 where rho <= 0, T <= 0 or psi^2 < 0.
template <typename ST>
__global__ void __launch_bounds__(256) k_init(const double *__restrict__ stage, size_t nn,
                                              typename ST::T *__restrict__ pop, typename ST::C *__restrict__ phi,
                                              size_t st, Phys<double> P, unsigned *__restrict__ status) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const double rho = stage[i], ux = stage[nn + i], uy = stage[2 * nn + i], uz = stage[3 * nn + i],
                 T = stage[4 * nn + i];
    const double p2 = T > 0.0 ? psi_squared(P, rho, T) : -1.0;
    if (!(rho > 0.0) || !(T > 0.0) || !(p2 >= 0.0)) atomicOr(status, 2u);
    double meq[19], fl[19];
    equilibrium19(rho, ux, uy, uz, meq);
    populations19(meq, fl);
    double br = 0.0, bt = 0.0;
    using T_ = typename ST::T;
    using R_ = typename ST::R;
    constexpr int QT = ST::kQT, NP = PopLayout<QT>::kPop;
    if constexpr (ST::kDev) {
        br = (double)ST::rdec(ST::renc((float)rho));
        bt = (double)ST::rdec(ST::renc((float)T));
        if constexpr (sizeof(R_) == sizeof(T_)) {
            pop[element_index<T_, QT>(NP, st, i)] = __builtin_bit_cast(T_, ST::renc((float)rho));
            pop[element_index<T_, QT>(NP + 1, st, i)] = __builtin_bit_cast(T_, ST::renc((float)T));
        } else {
            R_ *refs = reinterpret_cast<R_ *>(pop + NP * st);
            refs[i] = ST::renc((float)rho);
            refs[st + i] = ST::renc((float)T);
        }
    }
#pragma unroll
    for (int a = 0; a < 19; ++a) pop[element_index<T_, QT>(a, st, i)] = ST::denc(fl[a] - w19(a) * br);
#pragma unroll
    for (int a = 0; a < QT; ++a) {
        const double w = QT == 7 ? (a == 0 ? P.wT0 : P.wT1) : w19(a);
        pop[element_index<T_, QT>(19 + a, st, i)] = ST::denc(w * (T - bt));
    }
    phi[i] = typename ST::C(0);
}

// Wettability of the bottom wall: the virtual density of each solid node of
// the layer below z = 0, rho_w = phi rho_ave - drho with rho_ave the weighted
// mean of its five fluid neighbours (e_z = +1; weights 1/18 and 1/36), phi
// and drho those of the centred square or of the rest of the wall, and
// psi_w of Eq. (8) at rho_w and the temperature of the fluid node above it.
// Evaluated in FP64 from the state at time t (before the step, and before
// the readout); sets status bit 1 where rho_w <= 0 or psi_w^2 < 0.  The
// patch (phi_in, drho) is the square of side P.wet_square and the disc of
// squared radius disc_r2 centred at (cx, cy).
template <typename ST>
__global__ void __launch_bounds__(256) k_wall_density(const typename ST::T *__restrict__ pop, size_t st, int nx,
                                                      int ny, Phys<double> P, double disc_r2,
                                                      double *__restrict__ wall, unsigned *__restrict__ status) {
    const size_t nxy = (size_t)nx * ny;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nxy) return;
    const int x = (int)(i % nx), y = (int)(i / nx);
    const NodeView<ST> v{pop, st};
    constexpr int QT = ST::kQT;
    auto rho_at = [&](size_t j) {
        double fl[19];
#pragma unroll
        for (int a = 0; a < 19; ++a) fl[a] = v.e(a, j);
        return v.ref(0, j) + sum19(fl);
    };
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int a = 1; a < 19; ++a) {
        if (kE19Z[a] != 1) continue;
        const double w = (kE19X[a] == 0 && kE19Y[a] == 0) ? 1.0 / 18.0 : 1.0 / 36.0;
        const int xn = (x + kE19X[a] + nx) % nx, yn = (y + kE19Y[a] + ny) % ny;
        num += w * rho_at((size_t)yn * nx + xn);
        den += w;
    }
    double gl[QT];
#pragma unroll
    for (int a = 0; a < QT; ++a) gl[a] = v.e(19 + a, i);
    const double T = v.ref(1, i) + sum_T<QT>(gl);
    const double rho_ave = num / den;
    const double h = 0.5 * P.wet_square, dx = x - P.cx, dy = y - P.cy;
    const bool in_patch = (P.wet_square > 0.0 && fabs(dx) <= h && fabs(dy) <= h) ||
                          (disc_r2 > 0.0 && dx * dx + dy * dy <= disc_r2);
    const double rw = in_patch ? P.wet_phi_in * rho_ave - P.wet_drho : P.wet_phi * rho_ave;
    const double p2 = psi_squared(P, rw, T);
    if (!(rw > 0.0) || !(p2 >= 0.0)) atomicOr(status, 1u);
    wall[i] = rw;
    wall[nxy + i] = ::sqrt(p2 > 0.0 ? p2 : 0.0);
}

// Per-node rho, T (and psi) in FP64 into the staging planes 0, 4, 5.
template <typename ST>
__global__ void __launch_bounds__(256) k_macro(const typename ST::T *__restrict__ pop, size_t st, size_t nn,
                                               Phys<double> P, double *__restrict__ stage) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const NodeView<ST> v{pop, st};
    constexpr int QT = ST::kQT;
    double fl[19], gl[QT];
#pragma unroll
    for (int a = 0; a < 19; ++a) fl[a] = v.e(a, i);
#pragma unroll
    for (int a = 0; a < QT; ++a) gl[a] = v.e(19 + a, i);
    const double rho = v.ref(0, i) + sum19(fl), T = v.ref(1, i) + sum_T<QT>(gl);
    const double p2 = psi_squared(P, rho, T);
    stage[i] = rho;
    stage[4 * nn + i] = T;
    stage[5 * nn + i] = ::sqrt(p2 > 0.0 ? p2 : 0.0);
}

// u of Eq. (10) with the total force, in FP64, into staging planes 1..3.
// With walls, a solid neighbour below z = 0 contributes psi_w from `wall`
// (virtual-density wetting) or, if `wall` is null, the psi of the fluid node
// above it.
template <typename ST>
__global__ void __launch_bounds__(256) k_velocity(const typename ST::T *__restrict__ pop, size_t st, int nx, int ny,
                                                  int nz, int walls, Phys<double> P,
                                                  const double *__restrict__ rho_ave, const double *__restrict__ wall,
                                                  double *__restrict__ stage) {
    const size_t nn = (size_t)nx * ny * nz;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((size_t)nx * ny));
    const double *psi = stage + 5 * nn;
    double Sp[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 1; a < 19; ++a) {
        const int xn = (x + kE19X[a] + nx) % nx, yn = (y + kE19Y[a] + ny) % ny;
        int zn = z + kE19Z[a];
        if (walls) zn = zn < 0 ? 0 : (zn > nz - 1 ? nz - 1 : zn);
        else zn = (zn + nz) % nz;
        const double w = (kE19X[a] * kE19X[a] + kE19Y[a] * kE19Y[a] + kE19Z[a] * kE19Z[a]) == 1 ? 1.0 / 6.0 : 1.0 / 12.0;
        const bool solid_below = walls && wall && z + kE19Z[a] < 0;
        const double val = w * (solid_below ? wall[(size_t)nx * ny + (size_t)yn * nx + xn]
                                            : psi[((size_t)zn * ny + yn) * nx + xn]);
        Sp[0] += val * kE19X[a];
        Sp[1] += val * kE19Y[a];
        Sp[2] += val * kE19Z[a];
    }
    const double rho = stage[i];
    const NodeView<ST> v{pop, st};
    double fl[19], m[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) fl[a] = v.e(a, i);
    moments19(fl, m);  // m1..m3 of e equal those of f: sum e w_alpha = 0
    const double drho = P.gravity ? rho - *rho_ave : 0.0;
    const double F[3] = {P.negG * psi[i] * Sp[0] + drho * P.gx, P.negG * psi[i] * Sp[1] + drho * P.gy,
                         P.negG * psi[i] * Sp[2] + drho * P.gz};
    for (int c = 0; c < 3; ++c) stage[(1 + c) * nn + i] = (m[1 + c] + 0.5 * F[c]) / rho;
}

// FP64 per-workgroup sums of rho and T of the current state.
template <typename ST>
__global__ void __launch_bounds__(256) k_sum(const typename ST::T *__restrict__ pop, size_t st, size_t nn,
                                             double *__restrict__ partials) {
    __shared__ double red[2][4];
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0, t = 0.0;
    if (i < nn) {
        const NodeView<ST> v{pop, st};
        constexpr int QT = ST::kQT;
        double fl[19], gl[QT];
#pragma unroll
        for (int a = 0; a < 19; ++a) fl[a] = v.e(a, i);
#pragma unroll
        for (int a = 0; a < QT; ++a) gl[a] = v.e(19 + a, i);
        r = v.ref(0, i) + sum19(fl);
        t = v.ref(1, i) + sum_T<QT>(gl);
    }
    for (int o = 32; o > 0; o >>= 1) {
        r += __shfl_xor(r, o, 64);
        t += __shfl_xor(t, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = r;
        red[1][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        partials[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// Sum `count` partials (with `pitch` values per entry, summing component
// `comp`) in a fixed order and write sum * scale to *out.
__global__ void __launch_bounds__(256) k_finish(const double *__restrict__ partials, int count, int pitch, int comp,
                                                double scale, double *__restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int k = threadIdx.x; k < count; k += 256) acc += partials[(size_t)k * pitch + comp];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

}  // namespace lbm
