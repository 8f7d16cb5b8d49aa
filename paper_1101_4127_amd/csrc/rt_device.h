// rt_device.h -- device helpers of the packet march: counter-based generator,
// isotropic integer directions, brick layout of the cell fields, float32
// attenuation kernel.  Included by the HIP translation units only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_internal.h"

namespace rtk {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round multiplies
// counter words 0 and 2 by fixed odd constants, xors the high halves with the
// other two words and the key, and the key advances by a Weyl increment.
// ---------------------------------------------------------------------------
struct U64x4 { uint64_t v[4]; };

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
#pragma unroll 1
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = 0xD2E7470EE14C6C93ull * c0;
        const uint64_t ah = __umul64hi(0xD2E7470EE14C6C93ull, c0);
        const uint64_t b = 0xCA5A826395121157ull * c2;
        const uint64_t bh = __umul64hi(0xCA5A826395121157ull, c2);
        const uint64_t n0 = bh ^ c1 ^ k0;
        const uint64_t n2 = ah ^ c3 ^ k1;
        c0 = n0; c1 = b; c2 = n2; c3 = a;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    U64x4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// Isotropic integer direction of packet g in sub-step `step`: components are
// the top 21 bits of Philox words 0..2 shifted to [-2^20, 2^20); the first
// attempt whose squared length lies in [2^36, 2^40] is used (uniform on the
// sphere); 64 failed attempts give the diagonal 2^19 (1,1,1).
// Source packets draw from stream word 0 (g = packet id), recombination
// packets from stream word 1 (g = natural index of the emitting cell).
__device__ __forceinline__ void sample_direction(uint64_t seed, uint64_t solve_id, uint64_t g,
                                                 uint64_t step, bool octant, int32_t c[3],
                                                 uint64_t stream = 0ull) {
    for (uint32_t attempt = 0; attempt < 64u; ++attempt) {
        const U64x4 r = philox4x64_10(g, step, attempt, stream, seed, solve_id);
        const int32_t x = (int32_t)(r.v[0] >> 43) - (1 << 20);
        const int32_t y = (int32_t)(r.v[1] >> 43) - (1 << 20);
        const int32_t z = (int32_t)(r.v[2] >> 43) - (1 << 20);
        const int64_t q = (int64_t)x * x + (int64_t)y * y + (int64_t)z * z;
        if (q >= (1ll << 36) && q <= (1ll << 40)) {
            c[0] = octant ? abs(x) : x;
            c[1] = octant ? abs(y) : y;
            c[2] = octant ? abs(z) : z;
            return;
        }
    }
    c[0] = c[1] = c[2] = 1 << 19;
}

// Lane number of the t-th set bit (t < popcount) of a wavefront-wide mask.
__device__ __forceinline__ uint32_t nth_set_bit(uint64_t m, uint32_t t) {
    uint32_t lo = 0, hi = 63;                  // the answer b: popc(m & ((2 << b) - 1)) > t
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint64_t below = mid == 63u ? m : (m & ((2ull << mid) - 1ull));
        if ((uint32_t)__popcll(below) > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// The directions of sample_direction for a wavefront's packets, with the
// attempts shared out among all its lanes: each round, the packets still
// without a direction take every lane, a packet's further attempts going to
// its lanes in increasing order (so the first accepted attempt is found, as
// in the one-lane loop).  The wavefront then waits about three rounds of draws
// instead of its slowest packet's seven or so.  Every lane of the wavefront
// must call it (uniform control flow); lanes with `want` false only help.
// KEYED: the key (seed, solve id) and the sub-step differ between lanes (the
// packets of several solves in one wavefront); else they are the same for all.
template <bool KEYED = false>
__device__ __forceinline__ void sample_direction_wave(uint64_t seed, uint64_t solve_id, uint64_t g,
                                                      uint64_t step, bool octant, bool want, int32_t c[3],
                                                      uint64_t stream = 0ull) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lt = lane == 0u ? 0ull : (~0ull >> (64u - lane));
    bool done = !want;
    uint32_t next = 0;                          // next attempt of this lane's own packet
    int32_t cx = 1 << 19, cy = 1 << 19, cz = 1 << 19;
    for (;;) {
        const uint64_t open = __ballot(!done);
        if (open == 0ull) break;
        const uint32_t k = (uint32_t)__popcll(open);
        const uint32_t rank = (uint32_t)__popcll(open & lt);
        const uint32_t t = lane % k, o = lane / k;
        const uint32_t src = nth_set_bit(open, t);
        const uint64_t gt = (uint64_t)__shfl((long long)g, (int)src);
        const uint32_t at = (uint32_t)__shfl((int)next, (int)src) + o;
        bool ok = false;
        int32_t x = 0, y = 0, z = 0;
        uint64_t st = step, sd = seed, si = solve_id;
        if constexpr (KEYED) {
            st = (uint64_t)__shfl((long long)step, (int)src);
            sd = (uint64_t)__shfl((long long)seed, (int)src);
            si = (uint64_t)__shfl((long long)solve_id, (int)src);
        }
        if (at < 64u) {
            const U64x4 r = philox4x64_10(gt, st, at, stream, sd, si);
            x = (int32_t)(r.v[0] >> 43) - (1 << 20);
            y = (int32_t)(r.v[1] >> 43) - (1 << 20);
            z = (int32_t)(r.v[2] >> 43) - (1 << 20);
            const int64_t q = (int64_t)x * x + (int64_t)y * y + (int64_t)z * z;
            ok = q >= (1ll << 36) && q <= (1ll << 40);
        }
        const uint64_t acc = __ballot(ok);
        uint64_t pat = 0ull;                    // lanes 0, k, 2k, ... (wavefront-uniform)
        for (uint32_t j = 0; j < 64u; j += k) pat |= 1ull << j;
        const uint64_t mine = done ? 0ull : (pat << rank);
        const uint64_t hit = mine & acc;
        const uint32_t first = hit ? (uint32_t)__builtin_ctzll(hit) : lane;
        const int32_t sx = __shfl(x, (int)first), sy = __shfl(y, (int)first), sz = __shfl(z, (int)first);
        if (!done) {
            if (hit) {
                cx = sx;
                cy = sy;
                cz = sz;
                done = true;
            } else {
                next += (uint32_t)__popcll(mine);
                if (next >= 64u) done = true;   // no attempt accepted: the diagonal
            }
        }
    }
    c[0] = octant ? abs(cx) : cx;
    c[1] = octant ? abs(cy) : cy;
    c[2] = octant ? abs(cz) : cz;
}

// ---------------------------------------------------------------------------
// Brick layout: the grid is cut into bricks of 2^b cells per side, stored
// brick after brick (x fastest); inside a brick cells follow the Morton
// (bit-interleaved) order, so a ray's consecutive cells share cache lines for
// any direction.  b = 0 is the natural order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t spread3(uint32_t v) {   // 3 low bits -> every third bit
    return (v & 1u) | ((v & 2u) << 2) | ((v & 4u) << 4);
}

__device__ __forceinline__ uint32_t compact3(uint32_t m) {  // inverse of spread3
    return (m & 1u) | ((m >> 2) & 2u) | ((m >> 4) & 4u);
}

__device__ __forceinline__ uint32_t cell_slot(const GridGeom &G, int i, int j, int k) {
    if (G.bl == 0) return (uint32_t)i + (uint32_t)G.n[0] * ((uint32_t)j + (uint32_t)G.n[1] * (uint32_t)k);
    const uint32_t m = (1u << G.bl) - 1u;
    const uint32_t brick = ((uint32_t)(k >> G.bl) * (uint32_t)G.nb[1] + (uint32_t)(j >> G.bl)) * (uint32_t)G.nb[0]
                         + (uint32_t)(i >> G.bl);
    const uint32_t local = spread3((uint32_t)i & m) | (spread3((uint32_t)j & m) << 1)
                         | (spread3((uint32_t)k & m) << 2);
    return (brick << (3 * G.bl)) | local;
}

// Cell of a slot; returns false for padding slots outside the grid.
__device__ __forceinline__ bool slot_cell(const GridGeom &G, uint32_t slot, int &i, int &j, int &k) {
    if (G.bl == 0) {
        i = (int)(slot % (uint32_t)G.n[0]);
        const uint32_t r = slot / (uint32_t)G.n[0];
        j = (int)(r % (uint32_t)G.n[1]);
        k = (int)(r / (uint32_t)G.n[1]);
        return k < G.n[2];
    }
    const uint32_t local = slot & ((1u << (3 * G.bl)) - 1u);
    const uint32_t brick = slot >> (3 * G.bl);
    const uint32_t bi = brick % (uint32_t)G.nb[0];
    const uint32_t r = brick / (uint32_t)G.nb[0];
    const uint32_t bj = r % (uint32_t)G.nb[1];
    const uint32_t bk = r / (uint32_t)G.nb[1];
    i = (int)((bi << G.bl) | compact3(local));
    j = (int)((bj << G.bl) | compact3(local >> 1));
    k = (int)((bk << G.bl) | compact3(local >> 2));
    return i < G.n[0] && j < G.n[1] && k < G.n[2];
}

// ---------------------------------------------------------------------------
// Attenuation factors of one cell in float64, em = 1 - e^-t and tr = e^-t, both from one
// range reduction (Cody & Waite: -t = k ln2 + r, |r| <= ln2 / 2, ln2 split in
// two parts so k ln2 is exact) and one Taylor polynomial p = e^r - 1 to r^13
// (truncation below 2e-17 relative): tr = 2^k (1 + p) and
// em = (1 - 2^k) - 2^k p, both within a few ulp at every t >= 0, where
// computing either as 1 minus the other would lose the small one's digits.
__device__ __forceinline__ void attenuation(double t, double &em, double &tr) {
    if (!(t < 745.0)) {                       // e^-t below the smallest double
        em = 1.0;
        tr = 0.0;
        return;
    }
    const double x = -t;
    const double k = rint(x * 1.4426950408889634);
    const double r = fma(-k, 1.9082149292705877e-10, fma(-k, 0.69314718036912382, x));
    double p = 1.0 / 6227020800.0;                                   // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = p * r;                                                       // e^r - 1
    const int ki = (int)k;
    const double s = ldexp(1.0, ki);                                 // 2^k, k <= 0
    tr = fma(s, p, s);
    em = fma(-s, p, 1.0 - s);
}

// Error-free sum a + b = s + e (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

// Neumaier-compensated accumulation into (s, c).
__device__ __forceinline__ void acc_comp(double &s, double &c, double v) {
    double t, e;
    two_sum(s, v, t, e);
    s = t;
    c += e;
}

}  // namespace rtk
