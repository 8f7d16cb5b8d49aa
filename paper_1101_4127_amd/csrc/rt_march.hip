// rt_march.hip -- the packet march: emission, exact integer traversal,
// multi-frequency optical depth, Eq. (1) attenuation, split among absorbers,
// deposition into per-cell float64 accumulators, termination and the photon
// ledger (Partl et al. 2011, Sec. 2).
//
// Execution model: a persistent grid sized to the resident capacity of the
// chip.  Every lane of a wavefront carries one packet.  Wavefronts claim
// packet ids in chunks from a global counter; directions for 64 ids at a time
// are drawn by all 64 lanes together (full SIMD width for the Philox rejection
// loop) and kept in lane registers.  When enough lanes have finished their
// packet (ballot), they are refilled from that batch through cross-lane
// shuffles, so lanes never sit idle behind a divergent emission branch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <type_traits>

#include "rt_cross.h"
#include "rt_device.h"
#include "rt_internal.h"

namespace rtk {

struct MarchParams {
    GridGeom geo;
    double half_dl;        // half cell size [cm]
    double len_scale;      // float32 form: lengths in units of 1e18 cm
    const SourceRec *src;
    const double *src_ndot;
    const double *src_sedsum;
    const void *sed;       // [n_src][MB] of R
    const void *tab;       // [2][3][MB] of R: cross-sections, heat factors
    uint32_t n_src, P, q, r;   // q = P / n_src, r = P % n_src
    double dt;
    uint64_t seed, solve_id, step;
    double tau_kill;
    const void *kappa;
    double *acc;
    unsigned long long *queue;
    LedgerSlot *slots;
    int32_t *trace;
    int32_t trace_n, trace_len;
    uint32_t trace_stride;
    uint32_t chunk;
    uint32_t refill_min;
};

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// TwoSum-combine (s, c) pairs across the 64 lanes of a wavefront.
__device__ __forceinline__ void wave_sum_pair(double &s, double &c) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double so = __shfl_xor(s, off), co = __shfl_xor(c, off);
        double t, e;
        two_sum(s, so, t, e);
        s = t;
        c = c + co + e;
    }
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Occupancy target (wavefronts per SIMD) the register allocation is held to:
// the float32 instances trade registers for latency hiding, the float64 ones
// are held to a budget at which they do not spill.
template <typename R, int MB> struct MarchOcc { static constexpr int value = 2; };
template <> struct MarchOcc<float, 1> { static constexpr int value = 4; };
template <> struct MarchOcc<float, 8> { static constexpr int value = 3; };

constexpr int kWaves = kMarchBlock / 64;

template <typename R, int S, bool TH, int MB, int NA, int NB>
__global__ void __launch_bounds__(kMarchBlock, (MarchOcc<R, MB>::value)) k_march(const MarchParams p) {
    constexpr bool F64 = std::is_same<R, double>::value;
    constexpr uint32_t ACC = (S == 1) ? (TH ? 2u : 1u) : 4u;
    using KV = typename std::conditional<S == 1, R, typename Vec4<R>::T>::type;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = threadIdx.x >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64u - lane));

    // per-bin tables shared by all lanes (one 4-vector of cross-sections and
    // one of heat factors per bin), and the wave-private emission batch
    using V4R = typename Vec4<R>::T;
    __shared__ int32_t sb_c[kWaves][3][64];
    __shared__ uint32_t sb_g[kWaves][64], sb_src[kWaves][64];
    __shared__ double sb_w[kWaves][64], sb_L[kWaves][64];
    const CTab<R> tab = (CTab<R>)p.tab;
    __syncthreads();

    // ---- packet state (one per lane; only touched while the lane holds a packet) ----
    bool alive = false;
    int k0 = 0, k1 = 0, k2 = 0;                 // current cell
    uint32_t d0 = 1, d1 = 1, d2 = 1;            // |next face - origin| per axis (half cells)
    uint32_t a0 = 0, a1 = 0, a2 = 0;            // |c| per axis, kNeg set for c < 0
    uint32_t pnum = 0, pden = 1;                // entry parameter of the cell = pnum / pden
    double sprev = 0.0, L = 0.0;                // float64 form: entry parameter, length scale
    float Lf = 0.0f;                            // float32 form: length scale (1e18 cm units)
    double w = 0.0, absd = 0.0;
    float dropf = 0.0f;                         // float32 form: photons of bins dropped so far
    uint32_t slot = 0, count = 0, srcid = 0;
    int32_t tix = -1;                           // trace record of this packet, -1 if untraced
    KV kap{};                                   // absorbers of the current cell
    constexpr int ND = DepthState<R, S, MB>::N;
    R F[MB], D[ND];
    uint32_t active = 0;                        // bins the packet's source populates
    DepthTest<R, S, MB> dtest;
#pragma unroll
    for (int j = 0; j < MB; ++j) F[j] = R(0);
#pragma unroll
    for (int j = 0; j < ND; ++j) D[j] = R(0);

    // ---- ledger partials: updated only where every lane of the wave is active ----
    double l_emit = 0.0, l_abs = 0.0, l_esc = 0.0, l_trunc = 0.0;
    uint32_t n_cross = 0, n_pk = 0, n_esc = 0, n_trunc = 0;

    uint32_t batch_cnt = 0, batch_used = 0;     // wave-uniform
    uint32_t pool_next = 0, pool_end = 0;       // wave-uniform claimed id range
    bool exhausted = false;
    const KV *kappa = reinterpret_cast<const KV *>(p.kappa);
    const R *sedtab = reinterpret_cast<const R *>(p.sed);

    for (;;) {
        uint64_t dead = __ballot(!alive);
        uint32_t ndead = __popcll(dead);
        if (ndead != 0 && (ndead >= p.refill_min || ndead == 64u)) {
            while (ndead != 0) {
                if (batch_used == batch_cnt) {
                    if (pool_next == pool_end) {
                        if (exhausted) break;
                        unsigned long long base = 0;
                        if (lane == 0) base = atomicAdd(p.queue, (unsigned long long)p.chunk);
                        const uint32_t lo = uniform((uint32_t)base), hi = uniform((uint32_t)(base >> 32));
                        const unsigned long long b = ((unsigned long long)hi << 32) | lo;
                        if (b >= p.P) { exhausted = true; break; }
                        pool_next = (uint32_t)b;
                        pool_end = (uint32_t)min(b + p.chunk, (unsigned long long)p.P);
                    }
                    // all 64 lanes draw one packet each: source share, photons, direction
                    batch_cnt = min(64u, pool_end - pool_next);
                    const uint32_t id = pool_next + lane;
                    pool_next += batch_cnt;
                    batch_used = 0;
                    double emit = 0.0;
                    if (lane < batch_cnt) {
                        uint32_t sidx, ns;
                        const uint32_t big = p.r * (p.q + 1u);
                        if (id < big) { sidx = id / (p.q + 1u); ns = p.q + 1u; }
                        else { sidx = p.r + (id - big) / p.q; ns = p.q; }
                        const int32_t oct = (int32_t)(p.src[sidx].flags & kSrcOctant);
                        double ww = p.src_ndot[sidx] * p.dt;
                        ww = ww / (double)ns;
                        if (oct) ww = ww * 0.125;
                        int32_t c[3];
                        sample_direction(p.seed, p.solve_id, id, p.step, oct != 0, c);
                        const int64_t qq = (int64_t)c[0] * c[0] + (int64_t)c[1] * c[1] + (int64_t)c[2] * c[2];
                        sb_c[wv][0][lane] = c[0];
                        sb_c[wv][1][lane] = c[1];
                        sb_c[wv][2][lane] = c[2];
                        sb_g[wv][lane] = id;
                        sb_src[wv][lane] = sidx;
                        sb_w[wv][lane] = ww;
                        sb_L[wv][lane] = sqrt((double)qq) * p.half_dl;
                        emit = ww * p.src_sedsum[sidx];
                    }
                    l_emit += emit;
                    n_pk += (lane < batch_cnt) ? 1u : 0u;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
                // hand batch entries to dead lanes in lane order
                const uint32_t take = min(ndead, batch_cnt - batch_used);
                const uint32_t rank = __popcll(dead & lt_mask);
                if (!alive && rank < take) {
                    const uint32_t e = batch_used + rank;
                    const int32_t c0 = sb_c[wv][0][e], c1 = sb_c[wv][1][e], c2 = sb_c[wv][2][e];
                    const uint32_t g = sb_g[wv][e];
                    tix = (p.trace_n > 0 && g % p.trace_stride == 0u && g / p.trace_stride < (uint32_t)p.trace_n)
                              ? (int32_t)(g / p.trace_stride) : -1;
                    srcid = sb_src[wv][e];
                    w = sb_w[wv][e];
                    const double Ld = sb_L[wv][e];
                    const SourceRec sr = p.src[srcid];
                    if (F64) L = Ld; else Lf = (float)(Ld * p.len_scale);
                    k0 = sr.o[0] >> 1; k1 = sr.o[1] >> 1; k2 = sr.o[2] >> 1;
                    a0 = pack_dir(c0);
                    a1 = pack_dir(c1);
                    a2 = pack_dir(c2);
                    // distance to the first face: 1 from a cell centre, 2 from a corner
                    d0 = next_face(k0, sr.o[0], a0);
                    d1 = next_face(k1, sr.o[1], a1);
                    d2 = next_face(k2, sr.o[2], a2);
                    active = sr.flags >> kSrcMaskShift;
                    const R *sed = sedtab + (size_t)srcid * MB;
#pragma unroll
                    for (int j = 0; j < MB; ++j) F[j] = sed[j];
#pragma unroll
                    for (int j = 0; j < ND; ++j)
                        D[j] = (!DepthState<R, S, MB>::F64 || ((active >> j) & 1u)) ? R(0) : R(INFINITY);
                    dtest.start(tab, active, D);
                    sprev = 0.0; pnum = 0; pden = 1;
                    absd = 0.0;
                    dropf = 0.0f;
                    count = 0;
                    slot = cell_slot(p.geo, k0, k1, k2);
                    kap = kappa[slot];
                    alive = true;
                }
                batch_used += take;
                dead = __ballot(!alive);
                ndead = __popcll(dead);
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (__ballot(alive) == 0) {
            if (exhausted && batch_used == batch_cnt && pool_next == pool_end) break;
            continue;
        }

        // what this iteration adds to the ledger (zero for lanes without a packet)
        double it_abs = 0.0, it_left = 0.0, it_drop = 0.0;
        uint32_t it_cross = 0, it_fate = 0;
        if (alive) {
            // ---- geometry: nearest face by exact integer comparison ----
            bool m0, m1, m2;
            const int ax = exit_face(d0, d1, d2, a0, a1, a2, m0, m1, m2);
            const uint32_t num = ax == 0 ? d0 : (ax == 1 ? d1 : d2);
            const uint32_t den = (ax == 0 ? a0 : (ax == 1 ? a1 : a2)) & kMag;
            R l;
            double snew = 0.0;
            if (F64) {
                snew = (double)num / (double)den;
                l = (snew - sprev) * L;
            } else {
                // exact: num/den - pnum/pden = (num pden - pnum den) / (den pden),
                // num < 2^12, pden < 2^21, both products < 2^32
                const uint32_t diff = __umul24(num, pden) - __umul24(pnum, den);
                l = Lf * (float)diff * __builtin_amdgcn_rcpf((float)den * (float)pden);
            }
            const int here = k0 + p.geo.n[0] * (k1 + p.geo.n[1] * k2);
            const int here_k0 = k0, here_k1 = k1, here_k2 = k2;
            if (m0) { k0 += (a0 & kNeg) ? -1 : 1; d0 += 2u; }
            if (m1) { k1 += (a1 & kNeg) ? -1 : 1; d1 += 2u; }
            if (m2) { k2 += (a2 & kNeg) ? -1 : 1; d2 += 2u; }
            const bool o0 = (uint32_t)k0 >= (uint32_t)p.geo.n[0];
            const bool o1 = (uint32_t)k1 >= (uint32_t)p.geo.n[1];
            const bool o2 = (uint32_t)k2 >= (uint32_t)p.geo.n[2];
            const bool out = o0 | o1 | o2;
            // issue the next cell's gather before this cell's arithmetic (a packet
            // that left re-reads its last cell: the value is unused)
            const uint32_t nslot = out ? slot : cell_slot(p.geo, k0, k1, k2);
            const KV knext = kappa[nslot];

            // ---- Eq. (1) per bin and the split among absorbers ----
            R absorbed, e0, e1, e2, hs, tmin;
            cross_cell<R, S, TH, MB, NA, NB>(l, kap, tab, F, D, absorbed, e0, e1, e2, hs, tmin);

            // ---- deposit: float64 accumulators, hardware atomics at L2 ----
            double *cell = p.acc + (size_t)slot * ACC;
            if (S == 1) {
                const double v = w * (double)absorbed;
                if (v != 0.0) unsafeAtomicAdd(cell, v);
                if (TH) {
                    const double q = w * (double)hs;
                    if (q != 0.0) unsafeAtomicAdd(cell + 1, q);
                }
            } else {
                const double v0 = w * (double)e0;
                const double v1 = w * (double)e1;
                const double v2 = w * (double)e2;
                if (v0 != 0.0) unsafeAtomicAdd(cell, v0);
                if (v1 != 0.0) unsafeAtomicAdd(cell + 1, v1);
                if (v2 != 0.0) unsafeAtomicAdd(cell + 2, v2);
                if (TH) {
                    const double q = w * (double)hs;
                    if (q != 0.0) unsafeAtomicAdd(cell + 3, q);
                }
            }
            absd += (double)absorbed;
            it_cross = 1;
            const bool traced = tix >= 0;
            int32_t *rec = p.trace + (size_t)(traced ? tix : 0) * (RT_TRACE_HDR_DEV + p.trace_len);
            if (traced && count < (uint32_t)p.trace_len) rec[RT_TRACE_HDR_DEV + count] = here;
            ++count;

            // ---- termination: extinguished (checked first) or out of the grid ----
            const uint32_t fate = dtest.extinguished(tab, active, p.tau_kill, tmin, D) ? 1u : (out ? 2u : 0u);
            if constexpr (!F64 && MB > 1) {
                // float32 form: bins exhausted when the packet moves into the next
                // tile of 8^3 cells leave it (as in the tiled march)
                const bool next_tile = ((here_k0 ^ k0) | (here_k1 ^ k1) | (here_k2 ^ k2)) >> 3 != 0;
                if (fate == 0 && next_tile)
                    dropf += drop_exhausted<S, MB, NA, NB>(tab, active, depth_threshold(fmax(p.tau_kill, (double)kDropDepth)), D, F);
            }
            if (fate == 0) {
                slot = nslot;
                kap = knext;
                if (F64) sprev = snew; else { pnum = num; pden = den; }
            } else {
                double left = 0.0;
#pragma unroll
                for (int j = 0; j < MB; ++j) left += (double)F[j];
                it_abs = w * absd;
                it_left = w * left;
                it_drop = w * (double)dropf;
                it_fate = fate;
                if (traced) {
                    const int face = fate == 1 ? 0
                        : ((o0 ? 1 : 0) | (o1 ? 2 : 0) | (o2 ? 4 : 0)
                           | (k0 >= p.geo.n[0] ? 8 : 0) | (k1 >= p.geo.n[1] ? 16 : 0) | (k2 >= p.geo.n[2] ? 32 : 0));
                    rec[0] = (int32_t)count; rec[1] = (int32_t)fate; rec[2] = face; rec[3] = here;
                    rec[4] = unpack_dir(a0);
                    rec[5] = unpack_dir(a1);
                    rec[6] = unpack_dir(a2);
                    rec[7] = (int32_t)srcid;
                }
                alive = false;
            }
        }
        // every lane of the wave executes these updates
        n_cross += it_cross;
        l_abs += it_abs;
        l_esc += (it_fate == 2u) ? it_left : 0.0;
        l_trunc += ((it_fate == 1u) ? it_left : 0.0) + it_drop;
        n_esc += (it_fate == 2u) ? 1u : 0u;
        n_trunc += (it_fate == 1u) ? 1u : 0u;
    }

    // ---- block ledger: TwoSum reduction, one slot per block ----
    double v[8] = {l_emit, 0.0, l_abs, 0.0, l_esc, 0.0, l_trunc, 0.0};
#pragma unroll
    for (int i = 0; i < 4; ++i) wave_sum_pair(v[2 * i], v[2 * i + 1]);
    unsigned long long c[4] = {n_cross, n_pk, n_esc, n_trunc};
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = wave_sum_u64(c[i]);
    __shared__ double sh_s[kWaves][8];
    __shared__ unsigned long long sh_c[kWaves][4];
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) sh_s[wv][i] = v[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) sh_c[wv][i] = c[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        LedgerSlot out;
        for (int i = 0; i < 4; ++i) {
            double s = sh_s[0][2 * i], cc = sh_s[0][2 * i + 1];
            for (int u = 1; u < kWaves; ++u) {
                double t, e;
                two_sum(s, sh_s[u][2 * i], t, e);
                s = t;
                cc += sh_s[u][2 * i + 1] + e;
            }
            out.s[2 * i] = s;
            out.s[2 * i + 1] = cc;
        }
        for (int i = 0; i < 4; ++i) {
            unsigned long long t = 0;
            for (int u = 0; u < kWaves; ++u) t += sh_c[u][i];
            out.c[i] = t;
        }
        p.slots[blockIdx.x] = out;
    }
}

// ---------------------------------------------------------------------------
// host-side dispatch over (precision, species, thermal, bin capacity)
// ---------------------------------------------------------------------------
template <typename R, int S, bool TH, int MB, int NA, int NB>
static hipError_t run(const MarchLaunch &m) {
    MarchParams p;
    constexpr bool F64 = std::is_same<R, double>::value;
    p.geo = m.geo;
    p.half_dl = m.half_dl;
    p.len_scale = F64 ? 1.0 : 1.0e-18;
    p.src = m.src;
    p.src_ndot = m.src_ndot;
    p.src_sedsum = m.src_sedsum;
    p.sed = m.sed;
    p.tab = m.tab;
    p.n_src = (uint32_t)m.n_src;
    p.P = m.packets;
    p.q = m.packets / (uint32_t)m.n_src;
    p.r = m.packets % (uint32_t)m.n_src;
    p.dt = m.dt;
    p.seed = m.seed;
    p.solve_id = m.solve_id;
    p.step = m.step_index;
    p.tau_kill = m.tau_kill;
    p.kappa = m.kappa;
    p.acc = m.acc;
    p.queue = m.queue;
    p.slots = m.slots;
    p.trace = m.trace;
    p.trace_n = m.trace ? m.trace_n : 0;
    p.trace_len = m.trace_len;
    p.trace_stride = (uint32_t)m.trace_stride;
    p.chunk = (uint32_t)m.chunk;
    p.refill_min = (uint32_t)m.refill_min;
    hipLaunchKernelGGL((k_march<R, S, TH, MB, NA, NB>), dim3(m.blocks), dim3(kMarchBlock), 0, m.stream, p);
    return hipGetLastError();
}

template <typename R, int S, bool TH, int MB>
static hipError_t occ(int *n) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        n, reinterpret_cast<const void *>(&k_march<R, S, TH, MB, 0, 0>), kMarchBlock, 0);
}

// Compiled bin capacities: 1 (monochromatic) and 8 (up to 8 bins, unused bins
// carry no photons).
template <typename R, int S, bool TH>
static hipError_t pick_mb(const MarchLaunch *m, int mb, int *occ_out) {
    switch (mb) {
    case 1: return m ? run<R, S, TH, 1, 0, 0>(*m) : occ<R, S, TH, 1>(occ_out);
    case 8:
        if (!m) return occ<R, S, TH, 8>(occ_out);
        if (S == 3 && m->layout == 1) return run<R, S, TH, 8, 3, 2>(*m);
        return run<R, S, TH, 8, 0, 0>(*m);
    default: return hipErrorInvalidValue;
    }
}

static hipError_t dispatch(const MarchLaunch *m, int species, int thermal, int fp64, int mb, int *occ_out) {
    if (fp64) {
        if (species == 1) return thermal ? pick_mb<double, 1, true>(m, mb, occ_out) : pick_mb<double, 1, false>(m, mb, occ_out);
        return thermal ? pick_mb<double, 3, true>(m, mb, occ_out) : pick_mb<double, 3, false>(m, mb, occ_out);
    }
    if (species == 1) return thermal ? pick_mb<float, 1, true>(m, mb, occ_out) : pick_mb<float, 1, false>(m, mb, occ_out);
    return thermal ? pick_mb<float, 3, true>(m, mb, occ_out) : pick_mb<float, 3, false>(m, mb, occ_out);
}

hipError_t launch_march(const MarchLaunch &m) {
    return dispatch(&m, m.species, m.thermal, m.fp64, m.mb, nullptr);
}

hipError_t march_occupancy(int species, int thermal, int fp64, int mb, int *blocks_per_cu) {
    return dispatch(nullptr, species, thermal, fp64, mb, blocks_per_cu);
}

}  // namespace rtk
