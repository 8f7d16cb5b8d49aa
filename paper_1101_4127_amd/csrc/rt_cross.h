// rt_cross.h -- the arithmetic of one (packet, cell) crossing, shared by the
// per-packet march and the tiled march so that both follow a packet through
// bit-identical values: exact integer choice of the exit face, the chord, the
// per-bin optical depth and Eq. (1) attenuation, the split of the absorbed
// photons among HI, HeI and HeII in proportion to their optical depth, and
// the extinction test (Partl et al. 2011, Sec. 2).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <type_traits>

#include "rt_device.h"

namespace rtk {

template <typename R> struct Vec4;
template <> struct Vec4<float> { using T = float4; };
template <> struct Vec4<double> { using T = double4; };

// Per-bin table of the march precision, [7][MB]: cross-sections of HI, HeI,
// HeII, their heat factors (erg), then E_j - E_th,HI (erg).  The float32
// form's table holds the cross-sections (and the H+He heat factors, which
// carry one) times log2(e), so its optical depths come in units of ln 2 (see
// cross_cell).  Read through the constant address space: the indices are
// uniform, so the values live in scalar registers.
template <typename R> using CTab = const __attribute__((address_space(4))) R *;

constexpr uint32_t kNeg = 0x80000000u;      // sign flag packed above |c| (|c| <= 2^20)
constexpr uint32_t kMag = 0x00ffffffu;

// Per-packet depth state.  float64 form: the accumulated optical depth of
// every bin, T_j (bins the source does not populate start at +inf), exactly
// as the oracle sums it.  float32 form: the column densities N_s = sum l kappa_s
// of the three absorbers; T_j = sum_s sigma_s,j N_s is formed when the
// extinction test needs it (the same quantity, one float32 rounding per
// crossing and absorber instead of one per crossing and bin).
template <typename R, int S, int MB>
struct DepthState {
    static constexpr bool F64 = std::is_same<R, double>::value;
    static constexpr int N = F64 ? MB : (S == 1 ? 1 : 3);
};

// Exit face of the current cell by exact integer comparison of the ray
// parameters d_a / |c_a| (all products < 2^32); ties cross several faces at
// once.  Returns the lowest crossed axis.  The 24-bit multiplies read only the
// magnitude bits of a_a (the sign flag sits above them).  An axis the ray does
// not move along (|c_a| = 0, d_a = 1) never wins: its two comparisons need
// d_a |c_b| <= 0 and d_a |c_c| <= 0, i.e. both other components zero as well.
__device__ __forceinline__ int exit_face(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t a0, uint32_t a1,
                                         uint32_t a2, bool &m0, bool &m1, bool &m2) {
    const uint32_t p01 = __umul24(d0, a1), p10 = __umul24(d1, a0);
    const uint32_t p02 = __umul24(d0, a2), p20 = __umul24(d2, a0);
    const uint32_t p12 = __umul24(d1, a2), p21 = __umul24(d2, a1);
    m0 = p01 <= p10 && p02 <= p20;
    m1 = p10 <= p01 && p12 <= p21;
    m2 = p20 <= p02 && p21 <= p12;
    return m0 ? 0 : (m1 ? 1 : 2);
}

// A per-bin table copied into registers once per kernel: with the bins of a
// crossing in branches of their own, table reads through memory would sit in
// (and wait inside) every branch; the copy keeps them out of the loop.
template <typename R, int N>
struct RegTab {
    R v[N];
    __device__ __forceinline__ R operator[](int i) const { return v[i]; }
};

// The table a march passes to the crossing: registers in the float32 form,
// the constant-address-space pointer in the float64 form (its 7 x 8 doubles
// would not fit the scalar registers).
template <typename R, int MB, bool F64 = std::is_same<R, double>::value>
struct MarchTab {
    using type = RegTab<R, kTabRows * MB>;
    __device__ __forceinline__ static type make(CTab<R> t) {
        type r;
#pragma unroll
        for (int i = 0; i < kTabRows * MB; ++i) r.v[i] = t[i];
        return r;
    }
};
template <typename R, int MB>
struct MarchTab<R, MB, true> {
    using type = CTab<R>;
    __device__ __forceinline__ static type make(CTab<R> t) { return t; }
};

// Bins any lane of the wavefront with lane_on set still carries (bit j: some
// such lane has bit j of `active`).  Wave-uniform.
// With every lane of the wavefront executing, the masks are OR-ed across it
// by DPP moves (within quads, half rows and rows, then row broadcasts into
// the last row) and read from lane 63; otherwise one ballot per bin.
template <int MB>
__device__ __forceinline__ uint32_t wave_bins(bool lane_on, uint32_t active) {
    uint32_t v = lane_on ? active : 0u;
    if (__builtin_amdgcn_read_exec() == ~0ull) {
        v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);    // quad_perm 1,0,3,2
        v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);    // quad_perm 2,3,0,1
        v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);   // row_half_mirror
        v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);   // row_mirror
        v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15
        v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);   // row_bcast:31
        return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    }
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < MB; ++j) m |= (__ballot((v >> j) & 1u) != 0ull) ? (1u << j) : 0u;
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)m);
}

// Depth below which the float32 form keeps computing a bin whatever tau_kill.
constexpr float kDropDepth = 30.0f;

// An optical depth in the float32 form's units (ln 2): tau log2(e), rounded
// once to float32.
__device__ __forceinline__ float depth_threshold(double tau) { return (float)(tau * 1.4426950408889634); }

// Optical depth T = sigma_HI N_HI + sigma_HeI N_HeI + sigma_HeII N_HeII of one
// bin from a packet's column densities (float32 form), in one fixed order of
// operations used by every test that compares it with tau_kill.
template <int S>
__device__ __forceinline__ float column_depth(float sH, float sHe1, float sHe2, const float (&N)[S == 1 ? 1 : 3]) {
    if (S == 1) return sH * N[0];
    return __builtin_fmaf(sHe2, N[2], __builtin_fmaf(sHe1, N[1], sH * N[0]));
}

// Eq. (1) in every bin of one cell of chord length l (float32 form: l in
// 1e18 cm, cross-sections in 1e-18 cm^2), with F the photons carried per bin
// (updated to the transmitted part) and the depth state advanced.  Outputs,
// in the march precision: the photons absorbed over all bins; per absorber,
// kappa_s * sum_j sigma_s,j d_j / K_j (the photons the absorber takes); the
// heat sum_s kappa_s sum_j h_s,j d_j / K_j (pure hydrogen: sum_j h_j d_j), in
// erg per photon of the packet's weight; and, in the float64 form, the
// smallest accumulated optical depth over the bins (those the source does
// not populate hold +inf), which ends the packet once it reaches tau_kill
// (float32 form: see Extinction).
//
// Bins outside `wbins` (wave-uniform; a superset of the bins the wavefront's
// crossing lanes still carry, e.g. from wave_bins) are skipped: every crossing
// lane holds exactly 0 photons in them, so skipping changes nothing.
//
// The float32 form forms each bin's optical depth in units of ln 2 from the
// cell's columns and the table's scaled cross-sections,
// t_j = tau_j log2(e) = sum_s (l kappa_s)(sigma_s,j log2(e)), so e^-tau_j is
// the hardware 2^-t_j.  With q_j = (1 - 2^-t_j) / t_j the absorbed photons
// are d_j = F_j q_j t_j, and d_j / K_j = l log2(e) F_j q_j, so the split among
// absorbers needs no division by K_j: per absorber
// (l kappa_s) sum_j (sigma_s,j log2(e)) F_j q_j.  The H+He heat is the same
// sum written as the energy of the absorbed photons less each absorber's
// threshold times the photons it took, sum_j E_j d_j - sum_s E_th,s n_s (the
// photons of bin j absorbed by all species add up to d_j), one product per
// bin.  q_j comes from its Taylor series below
// t = kSeriesT (tau = 1/8; truncation after the tau^4 term, relative error
// below tau^5/720 = 4.2e-8) and from 1 - 2^-t_j times the hardware
// reciprocal above (relative error a few times 1e-7 just above the switch,
// where 1 - 2^-t_j cancels most, and smaller beyond).  The transmitted part
// is F_j - d_j below the switch and F_j 2^-t_j above it, so an opaque cell's
// remainder keeps its digits.
constexpr float kSeriesT = 0.1803368777036667f;   // tau = 1/8 in units of ln 2

__device__ __forceinline__ float absorbed_over_depth(float t) {
    // ln2 (1 - u/2 + u^2/6 - u^3/24 + u^4/120) with u = t ln2
    float q = __builtin_fmaf(t, 0.0013333557872101665f, -0.009618128649890423f);
    q = __builtin_fmaf(t, q, 0.05550410971045494f);
    q = __builtin_fmaf(t, q, -0.24022650718688965f);
    return __builtin_fmaf(t, q, 0.6931471824645996f);
}

template <int S, bool TH, int MB, int NA, int NB, typename KV, typename TT>
__device__ __forceinline__ void cross_cell_f32(float l, const KV &kap, TT tab, float (&F)[MB],
                                               float (&D)[S == 1 ? 1 : 3], float &absorbed, float &e0,
                                               float &e1, float &e2, float &heat, uint32_t wbins) {
    float kH, kHe1 = 0.0f, kHe2 = 0.0f;
    if constexpr (S == 1) kH = kap;
    else { kH = kap.x; kHe1 = kap.y; kHe2 = kap.z; }
    // column densities through the end of this cell
    D[0] = __builtin_fmaf(l, kH, D[0]);
    if (S == 3) {
        D[1] = __builtin_fmaf(l, kHe1, D[1]);
        D[2] = __builtin_fmaf(l, kHe2, D[2]);
    }
    // the cell's columns l kappa_s
    const float cH = l * kH, cHe1 = S == 3 ? l * kHe1 : 0.0f, cHe2 = S == 3 ? l * kHe2 : 0.0f;
    float ab = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, h0 = 0.0f;
    float dH = 0.0f;                // photons of the bins hydrogen alone absorbs (j < NA)
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        if constexpr (MB > 1) {
            if (!((wbins >> j) & 1u)) continue;
        }
        // helium terms of a bin below a helium threshold are zero: with a bin
        // layout known at compile time (the first NA bins hydrogen only, the
        // next NB without HeII; checked on the table by the host) they are
        // skipped, which adds nothing and changes no bit
        const bool he1 = S == 3 && j >= NA, he2 = S == 3 && j >= NA + NB;   // constant once unrolled
        float t = cH * tab[j];
        if (he1) t = __builtin_fmaf(cHe1, tab[MB + j], t);
        if (he2) t = __builtin_fmaf(cHe2, tab[2 * MB + j], t);
        const float tr = __builtin_amdgcn_exp2f(-t);
        const float qs = absorbed_over_depth(t);
        const bool lo = t < kSeriesT;
        float d;
        if (S == 3 && j >= NA) {
            // several absorbers share the bin: F_j q_j = d_j / t_j weighs them
            const float q = lo ? qs : (1.0f - tr) * __builtin_amdgcn_rcpf(t);
            const float gk = F[j] * q;
            d = gk * t;
            g0 = __builtin_fmaf(tab[j], gk, g0);
            if (he1) g1 = __builtin_fmaf(tab[MB + j], gk, g1);
            if (he2) g2 = __builtin_fmaf(tab[2 * MB + j], gk, g2);
            // photon energy absorbed (the ionisation energies come off below)
            if (TH) h0 = __builtin_fmaf(d, tab[3 * MB + j], h0);
        } else {
            // hydrogen alone absorbs: its share is 1
            d = F[j] * (lo ? qs * t : 1.0f - tr);
            if (S == 3) dH += d;
            // heat E_j - E_th,HI per photon (one absorber); photon energy E_j
            // (several absorbers, S == 3)
            if (TH) h0 = __builtin_fmaf(d, tab[3 * MB + j], h0);
        }
        F[j] = lo ? F[j] - d : F[j] * tr;
        ab += d;
    }
    absorbed = ab;
    if (S == 1) {
        e0 = ab;
        e1 = e2 = 0.0f;
        heat = h0;
    } else {
        e0 = __builtin_fmaf(cH, g0, dH);
        e1 = cHe1 * g1;
        e2 = cHe2 * g2;
        // heat = sum_j E_j d_j - sum_s E_th,s (photons species s absorbed):
        // each absorbed photon leaves E_j minus its absorber's threshold
        heat = TH ? __builtin_fmaf(-tab[4 * MB + 2], e2,
                                   __builtin_fmaf(-tab[4 * MB + 1], e1, __builtin_fmaf(-tab[4 * MB], e0, h0)))
                  : 0.0f;
    }
}

template <typename R, int S, bool TH, int MB, int NA = 0, int NB = 0, typename KV, typename TT>
__device__ __forceinline__ void cross_cell(R l, const KV &kap, TT tab, R (&F)[MB],
                                           R (&D)[DepthState<R, S, MB>::N], R &absorbed, R &e0, R &e1,
                                           R &e2, R &heat, R &tmin, uint32_t wbins = ~0u) {
    if constexpr (!std::is_same<R, double>::value) {
        cross_cell_f32<S, TH, MB, NA, NB>(l, kap, tab, F, D, absorbed, e0, e1, e2, heat, wbins);
        tmin = R(INFINITY);
    } else {
        // float64 form: the oracle's order of operations, no contraction
        R kH, kHe1 = R(0), kHe2 = R(0);
        if constexpr (S == 1) kH = kap;
        else { kH = kap.x; kHe1 = kap.y; kHe2 = kap.z; }
        R ab = R(0), g0 = R(0), g1 = R(0), g2 = R(0), h0 = R(0), h1 = R(0), h2 = R(0);
        R dH = R(0), qH = R(0);     // bins absorbed by hydrogen alone (j < NA): photons, heat
        R tm = R(INFINITY);
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            struct { R x, y, z; } sg = {tab[j], tab[MB + j], tab[2 * MB + j]};
            const bool he1 = S == 3 && j >= NA, he2 = S == 3 && j >= NA + NB;   // constant once unrolled
            R K = kH * sg.x;
            if (S == 3) {
                if (he1) K = K + kHe1 * sg.y;
                if (he2) K = K + kHe2 * sg.z;
            }
            const R tau = l * K;
            // absorbed share 1 - e^-tau and transmitted share e^-tau, each
            // with a few ulp of relative error at every tau (an opaque cell's
            // remainder keeps its digits)
            double em, tr;
            attenuation(tau, em, tr);
            const R d = F[j] * em;
            F[j] = F[j] * tr;
            D[j] = D[j] + tau;
            tm = D[j] < tm ? D[j] : tm;
            ab += d;
            if (S == 3 && j < NA) {
                // hydrogen alone absorbs here: its share is 1, its heat E_j - E_th,HI
                dH += d;
                if (TH) qH += d * tab[6 * MB + j];
            } else if (S == 1) {
                if (TH) h0 += d * tab[3 * MB + j];
            } else {
                const R gk = K > R(0) ? d / K : R(0);
                g0 += sg.x * gk;
                if (he1) g1 += sg.y * gk;
                if (he2) g2 += sg.z * gk;
                if (TH) {
                    h0 += tab[3 * MB + j] * gk;
                    if (he1) h1 += tab[4 * MB + j] * gk;
                    if (he2) h2 += tab[5 * MB + j] * gk;
                }
            }
        }
        absorbed = ab;
        tmin = tm;
        if (S == 1) {
            e0 = ab;
            e1 = e2 = R(0);
            heat = h0;
        } else {
            e0 = kH * g0 + dH;
            e1 = kHe1 * g1;
            e2 = kHe2 * g2;
            heat = TH ? ((kH * h0 + kHe1 * h1) + kHe2 * h2) + qH : R(0);
        }
    }
}

// Float32 form with several bins, when a packet moves from one tile of 8^3
// cells into the next: a bin whose optical depth T_j has reached tau_drop
// leaves the packet (its bit cleared in `active`, its remaining photons
// returned for the truncated ledger).  The caller passes
// tau_drop = depth_threshold(max(tau_kill, kDropDepth)) (depths in units of
// ln 2, as the table's cross-sections): a bin so dropped keeps at most e^-30
// (9.4e-14) of its share.  Decided from the packet's own history at tile
// boundaries, so every march organisation drops the same bins at the same
// cells; T_j is formed as in the extinction test (zero helium cross-sections
// of the layout's hydrogen-only bins add exact zeros).
//
// Bins outside `wbins` (wave-uniform superset of the bins the calling lanes
// carry) are not looked at.
template <int S, int MB, int NA, int NB, typename TT>
__device__ __forceinline__ float drop_exhausted(TT tab, uint32_t &active, float tau_drop,
                                                const float (&N)[S == 1 ? 1 : 3], float (&F)[MB],
                                                uint32_t wbins = ~0u) {
    float drop = 0.0f;
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        if (!((wbins >> j) & 1u)) continue;
        const float sH = tab[j];
        float Tj;
        if constexpr (S == 1) Tj = sH * N[0];
        else if (j < NA) Tj = sH * N[0];
        else if (j < NA + NB) Tj = __builtin_fmaf(tab[MB + j], N[1], sH * N[0]);
        else Tj = column_depth<S>(sH, tab[MB + j], tab[2 * MB + j], N);
        const bool gone = ((active >> j) & 1u) && Tj >= tau_drop;
        drop += gone ? F[j] : 0.0f;
        F[j] = gone ? 0.0f : F[j];
        active = gone ? (active & ~(1u << j)) : active;
    }
    return drop;
}

// Extinction test of the float32 form: a packet ends once every bin the
// source populates has T_j = sum_s sigma_s,j N_s >= tau_kill (both in units
// of ln 2: the table's scaled cross-sections, depth_threshold(tau_kill)).  The packet
// keeps a witness bin whose T_j was below tau_kill at the last full check;
// as long as the witness stays below, some bin is (so the packet lives) and
// one T_j is formed per crossing instead of all of them.  When the witness
// reaches tau_kill the full minimum decides, and a new witness is taken.  The
// decision equals the one of the full minimum at every crossing (T_j only
// grows, and the witness's T_j is formed exactly as in the full minimum).
template <int S, int MB>
struct Extinction {
    float wH = 0.0f, wHe1 = 0.0f, wHe2 = 0.0f;    // cross-sections of the witness bin
    uint32_t jw = 0;                              // the witness bin

    __device__ __forceinline__ static float depth(float sH, float sHe1, float sHe2, const float (&N)[S == 1 ? 1 : 3]) {
        return column_depth<S>(sH, sHe1, sHe2, N);
    }

    // full check: true if extinguished; else the witness is the first bin of
    // smallest depth
    template <typename TT>
    __device__ __forceinline__ bool full(TT tab, uint32_t active, float tau_kill,
                                         const float (&N)[S == 1 ? 1 : 3]) {
        float tm = INFINITY;
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            const float sH = tab[j], sHe1 = S == 1 ? 0.0f : tab[MB + j], sHe2 = S == 1 ? 0.0f : tab[2 * MB + j];
            const float t = depth(sH, sHe1, sHe2, N);
            const bool take = ((active >> j) & 1u) && t < tm;
            tm = take ? t : tm;
            wH = take ? sH : wH;
            wHe1 = take ? sHe1 : wHe1;
            wHe2 = take ? sHe2 : wHe2;
            jw = take ? (uint32_t)j : jw;
        }
        return tm >= tau_kill;
    }

    // resume with a known witness bin (cross-sections from a per-lane table)
    __device__ __forceinline__ void resume(uint32_t j, const float *sig) {
        jw = j;
        wH = sig[j];
        wHe1 = S == 1 ? 0.0f : sig[MB + j];
        wHe2 = S == 1 ? 0.0f : sig[2 * MB + j];
    }

    template <typename TT>
    __device__ __forceinline__ bool extinguished(TT tab, uint32_t active, float tau_kill,
                                                 const float (&N)[S == 1 ? 1 : 3]) {
        if (depth(wH, wHe1, wHe2, N) < tau_kill) return false;
        return full(tab, active, tau_kill, N);
    }
};

// Extinction state of either form: the float64 form tests the minimum of its
// per-bin depths (returned by cross_cell), the float32 form a witness.
template <typename R, int S, int MB>
struct DepthTest {
    static constexpr bool F64 = std::is_same<R, double>::value;
    Extinction<S, MB> ext;
    template <typename TT>
    __device__ __forceinline__ void start(TT tab, uint32_t active, const R (&D)[DepthState<R, S, MB>::N]) {
        if constexpr (!F64) (void)ext.full(tab, active, 0.0f, D);
    }
    template <typename TT>
    __device__ __forceinline__ bool extinguished(TT tab, uint32_t active, double tau_kill, R tmin,
                                                 const R (&D)[DepthState<R, S, MB>::N]) {
        if constexpr (F64) return tmin >= tau_kill;
        else return ext.extinguished(tab, active, depth_threshold(tau_kill), D);
    }
};

// Distance (half cells) from the start point o to the next face along one
// axis, for a packet now in cell k: 1 for an axis the packet does not move
// along; otherwise 2k + 2 - o (c > 0) or o - 2k (c < 0).
__device__ __forceinline__ uint32_t next_face(int k, int32_t o, uint32_t a) {
    if ((a & kMag) == 0u) return 1u;
    return (a & kNeg) ? (uint32_t)(o - 2 * k) : (uint32_t)(2 * k + 2 - o);
}

__device__ __forceinline__ uint32_t pack_dir(int32_t c) {
    return (uint32_t)abs(c) | (c < 0 ? kNeg : 0u);
}

__device__ __forceinline__ int32_t unpack_dir(uint32_t a) {
    return (a & kNeg) ? -(int32_t)(a & kMag) : (int32_t)a;
}

}  // namespace rtk
