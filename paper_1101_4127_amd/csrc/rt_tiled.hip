// rt_tiled.hip -- the packet march organised by tiles of the grid.
//
// The physics per crossing is that of the per-packet march (rt_cross.h); what
// changes is the order in which (packet, cell) pairs are visited.  Deposits of
// many packets land in the same cells, and float64 atomics at L2 sustain only
// ~2e10 updates/s on the whole chip, far below the crossing rate the march can
// reach.  So the grid is cut into tiles of 8^3 cells (the bricks of the field
// layout, contiguous in memory), and the propagation runs in passes:
//
//   emission   every packet of the batch is drawn (Philox direction, SED,
//              weight) into a record of fixed size, and its source's tile
//              counts it;
//   pass       each block claims a run of one tile's packet list, stages the
//              tile's absorbers in LDS, marches every packet of the run until
//              it leaves the tile, dies or escapes, adding its deposits to
//              float64 accumulators in LDS, then adds the tile's accumulators
//              to the grid's once (plain read-add-write when the run is the
//              tile's only one this pass, coalesced atomics otherwise).  A
//              packet that moves on is written back to its record and ranked
//              among the packets of its run bound for the same neighbour;
//   sort       the per-tile counts of the next pass are scanned into list
//              offsets and runs, and the record ids are scattered into the
//              next pass's lists.
//
// The grid's partition into tiles is the GPU counterpart of the domain
// decomposition of Sec. 3.2: a tile plays the part of a subdomain and the
// hand-over of packets between passes that of the exchange between tasks.  A
// ray's tile index changes monotonically along every axis, so a packet
// visits at most tx + ty + tz - 2 tiles and that many passes empty every list.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <type_traits>

#include "rt_cross.h"
#include "rt_device.h"
#include "rt_internal.h"
#include "rt_recomb.h"

namespace rtk {

namespace {

constexpr int kTBlock = 256;              // threads of the emission, march and scatter blocks
constexpr int kTWaves = kTBlock / 64;
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 4;               // tiles per scan thread
constexpr int kScanTiles = kScanBlock * kScanPer;

struct TParams {
    GridGeom geo;
    double half_dl, len_scale;
    const SourceRec *src;
    const double *src_ndot, *src_sedsum;
    const void *sed, *tab;
    uint32_t q, r;                        // packets per source: q (+1 for the first r)
    uint32_t n_src;
    double dt;
    uint64_t seed, solve_id, step;
    double tau_kill;
    const void *kappa;
    double *acc;
    LedgerSlot *slots;
    int32_t *trace;
    int32_t trace_n, trace_len;
    uint32_t trace_stride;
    uint32_t refill_min;
    uint32_t park;                        // park at most this many marching lanes (0: never)
    uint32_t g0, nbatch, capacity, cmax, max_chunks, n_tiles;
    uint32_t periodic;                    // periodic boundaries: neighbour tiles wrap
    uint32_t dmax;                        // periodic: largest next-face distance (half cells)
    void *rec;
    uint32_t *idx0, *idx1, *side, *cnt, *off, *cbase, *bsum;
    TChunk *ch0, *ch1;
    TCtrl *ctrl;
    StepLedger *ledger;
    // fused steps of many solves (the kernels' B instances): the solve table,
    // the round, each fused tile's solve, the first fused packet id of every
    // solve in this round ([n + 1]), march blocks (ledger slots per solve)
    const BatchHead *hd;
    const BatchSolve *tb;
    const uint16_t *tsolve;
    const uint32_t *first;
    int32_t round;
    uint32_t nblocks;
};

// Values of the solve a run belongs to: the kernel's own in a single solve,
// the table entry of the run's solve in a fused step.
template <typename R>
struct RunSolve {
    GridGeom geo;
    const void *kappa;
    double *acc;
    const void *tab;
    double tau_kill;
    uint32_t tile0, n_tiles;
};

template <typename R, bool B>
__device__ __forceinline__ RunSolve<R> run_solve(const TParams &p, uint32_t sid) {
    RunSolve<R> r;
    if constexpr (B) {
        const BatchSolve &sv = p.tb[sid];
        r.geo = sv.geo;
        r.kappa = sv.kappa;
        r.acc = sv.acc;
        r.tab = sv.tab;
        r.tau_kill = sv.tau_kill;
        r.tile0 = sv.tile0;
        r.n_tiles = sv.n_tiles;
    } else {
        r.geo = p.geo;
        r.kappa = p.kappa;
        r.acc = p.acc;
        r.tab = p.tab;
        r.tau_kill = p.tau_kill;
        r.tile0 = 0u;
        r.n_tiles = p.n_tiles;
    }
    return r;
}

// The solve of fused packet id i: the last solve whose first id is <= i.
__device__ __forceinline__ uint32_t solve_of_packet(const uint32_t *first, int n, uint32_t i) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return (uint32_t)lo;
}

// Record of a packet between passes (16-byte units), holding everything the
// march needs to resume it without touching the source tables.  The words a
// crossing changes come first:
//   0    the cell it is in (or about to enter) | axis of the last face crossed
//        (3: none yet) << 30
//   1    next-face distances d0 | d1 << 16 (half cells), with the witness
//        bin of the float32 extinction test in bits 12-15
//   2    d2 | bins the source populates << 16
//   3..  float32 form: the column densities N_s, then the photons per bin F_j;
//        float64 form: F_j, then the optical depths T_j (two words each)
// then, from word MOV, what stays fixed: c[3], the integer direction; the
// packet weight (photons per unit of the SED, float64, two words); the length
// scale |c| dx / 2 of the chord (float32 form: one word, in 1e18 cm; float64
// form: two words, in cm).
// A write-back between passes rewrites whole 64-byte pieces from word 0 (the
// fixed words that share them included): HBM takes a partly written piece
// only as a read-modify-write, which made the float32 emission half again
// slower.
template <typename R, int S, int MB>
struct TRec {
    static constexpr bool F64 = std::is_same<R, double>::value;
    static constexpr int ND = DepthState<R, S, MB>::N;
    static constexpr int MOV = 3 + (F64 ? 4 * MB : ND + MB);
    static constexpr int NWORD = MOV + (F64 ? 7 : 6);
    static constexpr int UNITS = (NWORD + 3) / 4;
    static constexpr int WORDS = 4 * UNITS;
    static constexpr int WHOLE = ((UNITS + 3) / 4) * 4;     // units of the whole 64-byte pieces it touches
    // records sit on a power-of-two stride of at least 64 bytes, so a record
    // read or written back never straddles a 128-byte line it does not fill
    static constexpr int STRIDE = UNITS <= 4 ? 4 : (UNITS <= 8 ? 8 : 16);
    static constexpr int BACK = ((MOV + 15) / 16) * 4 < STRIDE ? ((MOV + 15) / 16) * 4 : STRIDE;
    static_assert(UNITS <= 16 && 4 * BACK >= MOV && WHOLE <= STRIDE, "record layout");
};

// Record ids of a run staged in LDS (the first kMaxRun of the run; a longer
// run reads the rest of its list from memory).
constexpr int kMaxRun = 2048;
static_assert(kMaxRun % kTBlock == 0 && kTileCells % kTBlock == 0, "whole loads per thread");

__device__ __forceinline__ uint32_t pack_cell(int k0, int k1, int k2, uint32_t axis) {
    return (uint32_t)k0 | ((uint32_t)k1 << 10) | ((uint32_t)k2 << 20) | (axis << 30);
}

// Source of packet g under the equal share: the first r sources get q + 1.
__device__ __forceinline__ uint32_t source_of(uint32_t g, uint32_t q, uint32_t r, uint32_t &ns) {
    const uint32_t big = r * (q + 1u);
    if (g < big) { ns = q + 1u; return g / (q + 1u); }
    ns = q;
    return r + (g - big) / q;
}

__device__ __forceinline__ double packet_weight(const TParams &p, uint32_t sidx, uint32_t ns, bool oct) {
    double ww = p.src_ndot[sidx] * p.dt;
    ww = ww / (double)ns;
    if (oct) ww = ww * 0.125;
    return ww;
}

__device__ __forceinline__ int32_t trace_slot(const TParams &p, uint32_t g) {
    if (p.trace_n <= 0) return -1;
    return (g % p.trace_stride == 0u && g / p.trace_stride < (uint32_t)p.trace_n) ? (int32_t)(g / p.trace_stride)
                                                                                 : -1;
}

__device__ __forceinline__ uint32_t tile_of_cell(const GridGeom &G, int k0, int k1, int k2) {
    return ((uint32_t)(k2 >> kTileLog2) * (uint32_t)G.nb[1] + (uint32_t)(k1 >> kTileLog2)) * (uint32_t)G.nb[0]
         + (uint32_t)(k0 >> kTileLog2);
}

// Cell of a tile in LDS: linear order x + 8 y + 64 z (two bit operations per
// crossing); the grid's accumulators and absorbers keep the Morton order of
// the brick, so staging and write-out permute within the tile.
__device__ __forceinline__ uint32_t local_cell(int k0, int k1, int k2) {
    return ((uint32_t)k0 & 7u) | (((uint32_t)k1 & 7u) << 3) | (((uint32_t)k2 & 7u) << 6);
}

__device__ __forceinline__ uint32_t local_to_morton(uint32_t i) {
    return spread3(i & 7u) | (spread3((i >> 3) & 7u) << 1) | (spread3(i >> 6) << 2);
}

// neighbour code (dx+1) + 3 (dy+1) + 9 (dz+1) -> tile id offset
__device__ __forceinline__ int64_t code_offset(const GridGeom &G, uint32_t code) {
    const int dx = (int)(code % 3u) - 1, dy = (int)((code / 3u) % 3u) - 1, dz = (int)(code / 9u) - 1;
    return (int64_t)dx + (int64_t)G.nb[0] * ((int64_t)dy + (int64_t)G.nb[1] * (int64_t)dz);
}

// Tile reached from `tile` by neighbour code `code`; with periodic boundaries
// the tile coordinates wrap.  Out of the grid (non-periodic): a negative or
// too large id, which the callers flag.
__device__ __forceinline__ int64_t neighbour_tile(const GridGeom &G, uint32_t tile, uint32_t code, bool periodic) {
    if (!periodic) return (int64_t)tile + code_offset(G, code);
    const int nx = G.nb[0], ny = G.nb[1], nz = G.nb[2];
    int x = (int)(tile % (uint32_t)nx) + (int)(code % 3u) - 1;
    int y = (int)((tile / (uint32_t)nx) % (uint32_t)ny) + (int)((code / 3u) % 3u) - 1;
    int z = (int)(tile / ((uint32_t)nx * (uint32_t)ny)) + (int)(code / 9u) - 1;
    x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
    y = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    z = z < 0 ? z + nz : (z >= nz ? z - nz : z);
    return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * (int64_t)z);
}

// Periodic boundaries: a step of one cell that left [0, n) comes back through
// the opposite face; the tile offset of that step as a neighbour code digit.
__device__ __forceinline__ int wrap_cell(int k, int n) { return k < 0 ? k + n : (k >= n ? k - n : k); }
__device__ __forceinline__ int wrap_step(int v) { return v > 1 ? -1 : (v < -1 ? 1 : v); }

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

// Add per-lane ledger partials (value, compensation pairs and counters) of the
// whole block to the block's own slot (no other block writes it).
__device__ void block_ledger_add(LedgerSlot *slot, double (&v)[8], unsigned long long (&c)[4]) {
    __shared__ double sh_s[kTWaves][8];
    __shared__ unsigned long long sh_c[kTWaves][4];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 4; ++i) wave_sum_pair(v[2 * i], v[2 * i + 1]);
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = wave_sum_u64(c[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) sh_s[wv][i] = v[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) sh_c[wv][i] = c[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        LedgerSlot o = *slot;
        for (int i = 0; i < 4; ++i) {
            double s = o.s[2 * i], cc = o.s[2 * i + 1];
            for (int u = 0; u < kTWaves; ++u) {
                double t, e;
                two_sum(s, sh_s[u][2 * i], t, e);
                s = t;
                cc += sh_s[u][2 * i + 1] + e;
            }
            o.s[2 * i] = s;
            o.s[2 * i + 1] = cc;
        }
        for (int i = 0; i < 4; ++i)
            for (int u = 0; u < kTWaves; ++u) o.c[i] += sh_c[u][i];
        *slot = o;
    }
}

// The first NU units of a record (layout above); words past its end are zero.
template <typename R, int S, int MB, int NU>
__device__ __forceinline__ void put_record(uint4 *dst, int32_t c0, int32_t c1, int32_t c2, uint32_t kw,
                                           uint32_t d0, uint32_t jw, uint32_t d1, uint32_t d2, uint32_t active,
                                           double w, R len, const R (&F)[MB],
                                           const R (&D)[DepthState<R, S, MB>::N]) {
    using RL = TRec<R, S, MB>;
    constexpr int NW = 4 * NU;
    constexpr int M = RL::MOV;
    uint32_t x[NW];
    // indices are compile-time constants once unrolled: words past NW drop out
    auto put = [&x](int i, uint32_t v) {
        if (i < NW) x[i] = v;
    };
#pragma unroll
    for (int i = 0; i < NW; ++i) x[i] = 0u;
    put(0, kw);
    put(1, d0 | (jw << 12) | (d1 << 16));
    put(2, d2 | (active << 16));
    if constexpr (RL::F64) {
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            put(3 + 2 * j, (uint32_t)__double2loint(F[j]));
            put(4 + 2 * j, (uint32_t)__double2hiint(F[j]));
            put(3 + 2 * MB + 2 * j, (uint32_t)__double2loint(D[j]));
            put(4 + 2 * MB + 2 * j, (uint32_t)__double2hiint(D[j]));
        }
    } else {
#pragma unroll
        for (int j = 0; j < RL::ND; ++j) put(3 + j, __float_as_uint(D[j]));
#pragma unroll
        for (int j = 0; j < MB; ++j) put(3 + RL::ND + j, __float_as_uint(F[j]));
    }
    put(M, (uint32_t)c0);
    put(M + 1, (uint32_t)c1);
    put(M + 2, (uint32_t)c2);
    put(M + 3, (uint32_t)__double2loint(w));
    put(M + 4, (uint32_t)__double2hiint(w));
    if constexpr (RL::F64) {
        put(M + 5, (uint32_t)__double2loint((double)len));
        put(M + 6, (uint32_t)__double2hiint((double)len));
    } else {
        put(M + 5, __float_as_uint((float)len));
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) dst[u] = make_uint4(x[4 * u], x[4 * u + 1], x[4 * u + 2], x[4 * u + 3]);
}

// A new packet's record, padded with zeros to whole 64-byte pieces.
template <typename R, int S, int MB>
__device__ __forceinline__ void store_record(uint4 *dst, int32_t c0, int32_t c1, int32_t c2, uint32_t kw,
                                             uint32_t d0, uint32_t jw, uint32_t d1, uint32_t d2, uint32_t active,
                                             double w, R len, const R (&F)[MB],
                                             const R (&D)[DepthState<R, S, MB>::N]) {
    put_record<R, S, MB, TRec<R, S, MB>::WHOLE>(dst, c0, c1, c2, kw, d0, jw, d1, d2, active, w, len, F, D);
}

// Write-back between passes: the 64-byte pieces that hold what a crossing
// changes (cell, face distances, witness, depth state, photons), written
// whole with the fixed words that fall in them.
template <typename R, int S, int MB>
__device__ __forceinline__ void store_moving(uint4 *dst, int32_t c0, int32_t c1, int32_t c2, uint32_t kw,
                                             uint32_t d0, uint32_t jw, uint32_t d1, uint32_t d2, uint32_t active,
                                             double w, R len, const R (&F)[MB],
                                             const R (&D)[DepthState<R, S, MB>::N]) {
    put_record<R, S, MB, TRec<R, S, MB>::BACK>(dst, c0, c1, c2, kw, d0, jw, d1, d2, active, w, len, F, D);
}

// ---------------------------------------------------------------------------
// Emission of one batch: source share, weight, direction, SED; the packet is
// counted in its source's tile (wavefront-aggregated atomics) and its rank in
// that tile's list kept for the scatter.
// ---------------------------------------------------------------------------
template <typename R, int S, bool TH, int MB>
__global__ void __launch_bounds__(kTBlock) k_temit(const TParams p) {
    using RL = TRec<R, S, MB>;
    constexpr int ND = RL::ND;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64u - lane));
    const uint32_t gw = (blockIdx.x * kTBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * kTWaves;
    double l_emit = 0.0;
    uint32_t n_pk = 0;
    const R *sedtab = reinterpret_cast<const R *>(p.sed);
    uint4 *recs = reinterpret_cast<uint4 *>(p.rec);
    for (uint32_t base = gw * 64u; base < p.nbatch; base += nw * 64u) {
        const uint32_t i = base + lane;
        const bool act = i < p.nbatch;
        uint32_t tile = 0;
        const uint32_t g = p.g0 + i;
        uint32_t ns = 1u, sidx = 0u;
        if (act) sidx = source_of(g, p.q, p.r, ns);
        const SourceRec sr = p.src[sidx];
        const bool oct = (sr.flags & kSrcOctant) != 0u;
        int32_t c[3];
        sample_direction_wave(p.seed, p.solve_id, g, p.step, oct, act, c);
        if (act) {
            const double ww = packet_weight(p, sidx, ns, oct);
            l_emit += ww * p.src_sedsum[sidx];
            n_pk += 1u;
            const int k0 = sr.o[0] >> 1, k1 = sr.o[1] >> 1, k2 = sr.o[2] >> 1;
            const uint32_t active = sr.flags >> kSrcMaskShift;
            R F[MB], D[ND];
            const R *sed = sedtab + (size_t)sidx * MB;
#pragma unroll
            for (int j = 0; j < MB; ++j) F[j] = sed[j];
#pragma unroll
            for (int j = 0; j < ND; ++j) D[j] = (!RL::F64 || ((active >> j) & 1u)) ? R(0) : R(INFINITY);
            const uint32_t a0 = pack_dir(c[0]), a1 = pack_dir(c[1]), a2 = pack_dir(c[2]);
            const int64_t qq = (int64_t)c[0] * c[0] + (int64_t)c[1] * c[1] + (int64_t)c[2] * c[2];
            const double Ld = sqrt((double)qq) * p.half_dl;
            const R len = RL::F64 ? (R)Ld : (R)(Ld * p.len_scale);
            const uint32_t jw = active ? (uint32_t)__builtin_ctz(active) : 0u;   // all depths 0: first bin
            store_record<R, S, MB>(recs + (size_t)i * RL::STRIDE, c[0], c[1], c[2], pack_cell(k0, k1, k2, 3u),
                                   next_face(k0, sr.o[0], a0), jw, next_face(k1, sr.o[1], a1),
                                   next_face(k2, sr.o[2], a2), active, ww, len, F, D);
            tile = tile_of_cell(p.geo, k0, k1, k2);
            const int32_t tix = trace_slot(p, g);
            if (tix >= 0) p.trace[(size_t)tix * (RT_TRACE_HDR_DEV + p.trace_len)] = 0;
        }
        // rank in the tile's list: one atomic per distinct tile of the wavefront
        uint64_t pend = __ballot(act);
        uint32_t rel = 0;
        while (pend != 0ull) {
            const int lead = __ffsll((unsigned long long)pend) - 1;
            const uint32_t lt = (uint32_t)__shfl((int)tile, lead);
            const uint64_t same = __ballot(act && tile == lt) & pend;
            uint32_t b = 0;
            if ((int)lane == lead) b = atomicAdd(p.cnt + lt, (uint32_t)__popcll(same));
            b = (uint32_t)__shfl((int)b, lead);
            if ((same >> lane) & 1ull) rel = b + (uint32_t)__popcll(same & lt_mask);
            pend &= ~same;
        }
        if (act) p.side[i] = rel;
    }
    double v[8] = {l_emit, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    unsigned long long c[4] = {0ull, n_pk, 0ull, 0ull};
    block_ledger_add(p.slots + blockIdx.x, v, c);
}

// Emission of one round of a fused step: packet i of the round belongs to the
// solve whose range [first[s], first[s+1]) holds it and is that solve's
// packet g = i - first[s] of its sub-step, drawn exactly as rt_step draws it
// (equal share among the solve's sources, weight, Philox direction with the
// solve's key and sub-step counter, SED).  Its fused tile is counted (one
// atomic per distinct tile of the wavefront) and kept in list 1, free until
// the first pass, for the scatter.  Emitted photons and packets go to the
// (solve, block) ledger slot.
template <typename R, int S, int MB>
__global__ void __launch_bounds__(kTBlock) k_bemit(const TParams p) {
    using RL = TRec<R, S, MB>;
    constexpr int ND = RL::ND;
    __shared__ uint32_t s_first[kMaxBatch + 1];
    __shared__ double s_le[kMaxBatch];
    __shared__ unsigned long long s_lp[kMaxBatch];
    const int n = p.hd->n;
    for (int i = threadIdx.x; i <= n; i += kTBlock) s_first[i] = p.first[i];
    for (int i = threadIdx.x; i < kMaxBatch; i += kTBlock) {
        s_le[i] = 0.0;
        s_lp[i] = 0ull;
    }
    __syncthreads();
    const uint32_t total = s_first[n];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64u - lane));
    const uint32_t gw = (blockIdx.x * kTBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * kTWaves;
    uint4 *recs = reinterpret_cast<uint4 *>(p.rec);
    for (uint32_t base = gw * 64u; base < total; base += nw * 64u) {
        const uint32_t i = base + lane;
        const bool act = i < total && i < p.capacity;
        uint32_t tile = 0;
        // the packet's solve and source, then its direction (the attempts of the
        // wavefront's packets, of whatever solves, shared out among all lanes)
        const uint32_t sid = act ? solve_of_packet(s_first, n, i) : 0u;
        const BatchSolve &sv = p.tb[sid];
        const uint32_t P = act ? s_first[sid + 1] - s_first[sid] : 1u;
        const uint32_t g = act ? i - s_first[sid] : 0u;
        uint32_t ns = 1u, sidx = 0u;
        if (act) sidx = source_of(g, P / (uint32_t)sv.n_src, P % (uint32_t)sv.n_src, ns);
        const SourceRec sr = act ? sv.src[sidx] : SourceRec{};
        const bool oct = (sr.flags & kSrcOctant) != 0u;
        int32_t c[3];
        sample_direction_wave<true>(sv.seed, sv.solve_id, g, sv.step0 + (uint64_t)p.round, oct, act, c);
        if (act) {
            double ww = sv.src_ndot[sidx] * sv.dt;
            ww = ww / (double)ns;
            if (oct) ww = ww * 0.125;
            atomicAdd(&s_le[sid], ww * sv.src_sedsum[sidx]);
            atomicAdd(&s_lp[sid], 1ull);
            const int k0 = sr.o[0] >> 1, k1 = sr.o[1] >> 1, k2 = sr.o[2] >> 1;
            const uint32_t active = sr.flags >> kSrcMaskShift;
            R F[MB], D[ND];
            const R *sed = reinterpret_cast<const R *>(sv.sed) + (size_t)sidx * MB;
#pragma unroll
            for (int j = 0; j < MB; ++j) F[j] = sed[j];
#pragma unroll
            for (int j = 0; j < ND; ++j) D[j] = (!RL::F64 || ((active >> j) & 1u)) ? R(0) : R(INFINITY);
            const uint32_t a0 = pack_dir(c[0]), a1 = pack_dir(c[1]), a2 = pack_dir(c[2]);
            const int64_t qq = (int64_t)c[0] * c[0] + (int64_t)c[1] * c[1] + (int64_t)c[2] * c[2];
            const double Ld = sqrt((double)qq) * sv.half_dl;
            const R len = RL::F64 ? (R)Ld : (R)(Ld * 1.0e-18);
            const uint32_t jw = active ? (uint32_t)__builtin_ctz(active) : 0u;
            store_record<R, S, MB>(recs + (size_t)i * RL::STRIDE, c[0], c[1], c[2], pack_cell(k0, k1, k2, 3u),
                                   next_face(k0, sr.o[0], a0), jw, next_face(k1, sr.o[1], a1),
                                   next_face(k2, sr.o[2], a2), active, ww, len, F, D);
            tile = sv.tile0 + tile_of_cell(sv.geo, k0, k1, k2);
            p.idx1[i] = tile;
        }
        // rank in the tile's list: one atomic per distinct tile of the wavefront
        uint64_t pend = __ballot(act);
        uint32_t rel = 0;
        while (pend != 0ull) {
            const int lead = __ffsll((unsigned long long)pend) - 1;
            const uint32_t lt = (uint32_t)__shfl((int)tile, lead);
            const uint64_t same = __ballot(act && tile == lt) & pend;
            uint32_t b = 0;
            if ((int)lane == lead) b = atomicAdd(p.cnt + lt, (uint32_t)__popcll(same));
            b = (uint32_t)__shfl((int)b, lead);
            if ((same >> lane) & 1ull) rel = b + (uint32_t)__popcll(same & lt_mask);
            pend &= ~same;
        }
        if (act) p.side[i] = rel;
    }
    __syncthreads();
    for (int sid = threadIdx.x; sid < n; sid += kTBlock) {
        if (s_lp[sid] == 0ull) continue;
        LedgerSlot *slot = p.slots + (size_t)sid * p.nblocks + blockIdx.x;
        double t, e;
        two_sum(slot->s[0], s_le[sid], t, e);
        slot->s[0] = t;
        slot->s[1] += e;
        slot->c[1] += s_lp[sid];
    }
}

// Start of a round of a fused step.  Block 0: the first fused packet id of
// every solve in this round (round_packets summed in table order, one thread
// per solve); a round beyond the records is flagged.  Every block: the ledger
// slots of the call's solves ([solve][march block]) cleared.
__global__ void __launch_bounds__(kMaxBatch) k_bstart(const TParams p) {
    {
        const uint32_t ns = (uint32_t)p.hd->n * p.nblocks;
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
            LedgerSlot &sl = p.slots[i];
            for (int k = 0; k < 8; ++k) sl.s[k] = 0.0;
            for (int k = 0; k < 4; ++k) sl.c[k] = 0ull;
        }
    }
    if (blockIdx.x != 0) return;
    __shared__ unsigned long long s_w[kMaxBatch / 64];
    const int n = p.hd->n;
    const int b = threadIdx.x;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const unsigned long long mine = b < n ? round_packets(p.tb[b], p.round) : 0ull;
    unsigned long long v = mine;                  // inclusive scan over the wavefront
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long u = (unsigned long long)__shfl_up((long long)v, d);
        if (lane >= (uint32_t)d) v += u;
    }
    if (lane == 63u) s_w[wv] = v;
    __syncthreads();
    unsigned long long before = 0ull, total = 0ull;
    for (uint32_t u = 0; u < (uint32_t)(kMaxBatch / 64); ++u) {
        if (u < wv) before += s_w[u];
        total += s_w[u];
    }
    const unsigned long long excl = before + v - mine;
    const bool over = total > p.capacity;
    uint32_t *first = const_cast<uint32_t *>(p.first);
    if (b < n) first[b] = over ? 0u : (uint32_t)excl;
    if (b == 0) {
        first[n] = over ? 0u : (uint32_t)total;
        if (over) p.ctrl->err |= 256u;
    }
}

// Solve of every fused tile (tiles of solve s: [tile0, tile0 + n_tiles)).
__global__ void k_btiles(const TParams p) {
    const int n = p.hd->n;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < p.n_tiles; t += gridDim.x * blockDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (p.tb[mid].tile0 <= t) lo = mid; else hi = mid - 1;
        }
        const_cast<uint16_t *>(p.tsolve)[t] = (uint16_t)lo;
    }
}

// List positions of the emitted packets: offset of the source's tile + rank.
template <bool B>
__global__ void __launch_bounds__(kTBlock) k_tscatter_emit(const TParams p) {
    const uint32_t stride = gridDim.x * kTBlock;
    const uint32_t nb = B ? min(p.first[p.hd->n], p.capacity) : p.nbatch;
    for (uint32_t i = blockIdx.x * kTBlock + threadIdx.x; i < nb; i += stride) {
        uint32_t tile;
        if constexpr (B) {
            tile = p.idx1[i];
        } else {
            uint32_t ns;
            const uint32_t sidx = source_of(p.g0 + i, p.q, p.r, ns);
            const SourceRec sr = p.src[sidx];
            tile = tile_of_cell(p.geo, sr.o[0] >> 1, sr.o[1] >> 1, sr.o[2] >> 1);
        }
        const uint32_t pos = p.off[tile] + p.side[i];
        if (tile < p.n_tiles && pos < p.capacity) p.idx0[pos] = i;
        else atomicOr(&p.ctrl->err, 1u);
    }
}

// ---------------------------------------------------------------------------
// Recombination emission of one sub-step (Sec. 2; Sec. 3: a cell emits when a
// packet crosses it and its count of recombinations has reached f_rec N_a),
// after the sub-step's source packets have been marched and before the cell
// update.  One lane per slot.  A cell the source packets deposited in emits
// when some ion's counter is positive and at least f_rec: those counters give
// counter x atoms x ground-state share photons with the ion's Milne spectrum
// at the cell temperature, and restart from zero.  The packet (isotropic,
// Philox stream word 1 keyed by the cell's natural index, from the cell
// centre) takes the next free record, one atomic per wavefront; its tile
// counts it as for emitted source packets.
// ---------------------------------------------------------------------------
template <typename R, int S, int MB>
__global__ void __launch_bounds__(kTBlock) k_remit(const TParams p, const RecombParams rp) {
    using RL = TRec<R, S, MB>;
    constexpr int ND = RL::ND;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64u - lane));
    const uint32_t gw = (blockIdx.x * kTBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * kTWaves;
    const uint32_t np = p.geo.ncell_pad;
    const R *st = reinterpret_cast<const R *>(rp.state);
    uint4 *recs = reinterpret_cast<uint4 *>(p.rec);
    double l_emit = 0.0;
    uint32_t n_pk = 0;
    for (uint32_t base = gw * 64u; base < np; base += nw * 64u) {
        const uint32_t s = base + lane;
        bool emit = false;
        double ww = 0.0;
        R F[MB];
#pragma unroll
        for (int j = 0; j < MB; ++j) F[j] = R(0);
        int k0 = 0, k1 = 0, k2 = 0;
        if (s < np && slot_cell(p.geo, s, k0, k1, k2)) {
            const double *a = p.acc + (size_t)s * rp.acc_stride;
            const bool crossed = a[0] > 0.0 || (S == 3 && (a[1] > 0.0 || a[2] > 0.0));
            if (crossed) {
                const double T = (double)st[6 * (size_t)np + s];
                const double nh = (double)st[s];
                double pg[3];
                ground_fraction(T, pg);
                const double atoms[3] = {nh * rp.volume, (rp.y_he * nh) * rp.volume, (rp.y_he * nh) * rp.volume};
                double ph[3] = {0.0, 0.0, 0.0};
                bool any = false;
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    double *cp = rp.rc + (size_t)q * np + s;
                    const double r = *cp;
                    if (r > 0.0 && r >= rp.f_rec) {
                        ph[q] = (r * atoms[q]) * pg[q];
                        *cp = 0.0;
                        any = true;
                    }
                }
                const double w = (ph[0] + ph[1]) + ph[2];
                if (any && w > 0.0) {
                    double sed[MB];
#pragma unroll
                    for (int j = 0; j < MB; ++j) sed[j] = 0.0;
#pragma unroll
                    for (int q = 0; q < S; ++q) {
                        if (!(ph[q] > 0.0)) continue;
                        double m[MB];
                        milne_at<MB>(rp, q, T, m);
#pragma unroll
                        for (int j = 0; j < MB; ++j) sed[j] += ph[q] * m[j];
                    }
#pragma unroll
                    for (int j = 0; j < MB; ++j) F[j] = (R)(sed[j] / w);
                    ww = w;
                    emit = true;
                }
            }
        }
        const uint64_t em = __ballot(emit);
        if (em == 0ull) continue;                       // wavefront-uniform
        uint32_t b0 = 0;
        if (lane == 0) b0 = atomicAdd(&p.ctrl->ndiff, (uint32_t)__popcll(em));
        b0 = (uint32_t)__shfl((int)b0, 0);
        const uint32_t idx = b0 + (uint32_t)__popcll(em & lt_mask);
        const bool act = emit && idx < p.capacity;
        if (emit && !act) atomicOr(&p.ctrl->err, 128u);
        uint32_t tile = 0;
        const uint32_t cell = (uint32_t)k0 + (uint32_t)p.geo.n[0] * ((uint32_t)k1 + (uint32_t)p.geo.n[1] * (uint32_t)k2);
        int32_t c[3];
        sample_direction_wave(p.seed, p.solve_id, cell, p.step, false, act, c, 1ull);
        if (act) {
            uint32_t active = 0u;
            double carried = 0.0;
#pragma unroll
            for (int j = 0; j < MB; ++j) {
                if (F[j] > R(0)) active |= 1u << j;
                carried += (double)F[j];
            }
            R D[ND];
#pragma unroll
            for (int j = 0; j < ND; ++j) D[j] = (!RL::F64 || ((active >> j) & 1u)) ? R(0) : R(INFINITY);
            const uint32_t a0 = pack_dir(c[0]), a1 = pack_dir(c[1]), a2 = pack_dir(c[2]);
            const int64_t qq = (int64_t)c[0] * c[0] + (int64_t)c[1] * c[1] + (int64_t)c[2] * c[2];
            const double Ld = sqrt((double)qq) * p.half_dl;
            const R len = RL::F64 ? (R)Ld : (R)(Ld * p.len_scale);
            const uint32_t jw = active ? (uint32_t)__builtin_ctz(active) : 0u;
            store_record<R, S, MB>(recs + (size_t)idx * RL::STRIDE, c[0], c[1], c[2], pack_cell(k0, k1, k2, 3u),
                                   next_face(k0, 2 * k0 + 1, a0), jw, next_face(k1, 2 * k1 + 1, a1),
                                   next_face(k2, 2 * k2 + 1, a2), active, ww, len, F, D);
            l_emit += ww * carried;
            n_pk += 1u;
            tile = tile_of_cell(p.geo, k0, k1, k2);
        }
        // rank in the tile's list: one atomic per distinct tile of the wavefront
        uint64_t pend = __ballot(act);
        uint32_t rel = 0;
        while (pend != 0ull) {
            const int lead = __ffsll((unsigned long long)pend) - 1;
            const uint32_t lt = (uint32_t)__shfl((int)tile, lead);
            const uint64_t same = __ballot(act && tile == lt) & pend;
            uint32_t b = 0;
            if ((int)lane == lead) b = atomicAdd(p.cnt + lt, (uint32_t)__popcll(same));
            b = (uint32_t)__shfl((int)b, lead);
            if ((same >> lane) & 1ull) rel = b + (uint32_t)__popcll(same & lt_mask);
            pend &= ~same;
        }
        if (act) p.side[idx] = rel;
    }
    // the diffuse totals of the step: one float64 atomic per wavefront
    double de = l_emit, dc = 0.0;
    wave_sum_pair(de, dc);
    const unsigned long long dn = wave_sum_u64((unsigned long long)n_pk);
    if (lane == 0 && dn != 0ull) {
        atomicAdd(&rp.ledger->d_emit, de + dc);
        atomicAdd(&rp.ledger->d_packets, dn);
    }
    double v[8] = {l_emit, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    unsigned long long cc[4] = {0ull, n_pk, 0ull, 0ull};
    block_ledger_add(p.slots + blockIdx.x, v, cc);
}

// ---------------------------------------------------------------------------
// Background field (Sec. 2: packets from diffuse fields such as the UV
// background), an isotropic intensity entering through the box faces.
// Packet g of a sub-step starts at the centre of a boundary cell face chosen
// uniformly over all 2 (n1 n2 + n0 n2 + n0 n1) of them (Philox counter
// (g, sub-step, 0, 2), word 0 scaled by a high multiply; faces x-, x+, y-, y+,
// z-, z+, cells x fastest), takes the isotropic direction of stream word 3
// turned inward, and carries w = (ndot dt / P) 2 |c_n| / |c| photons per unit
// of the spectrum (2 cos theta averages 1 over the hemisphere).
// ---------------------------------------------------------------------------
template <typename R, int S, int MB>
__global__ void __launch_bounds__(kTBlock) k_bgemit(const TParams p, const BackgroundParams bp) {
    using RL = TRec<R, S, MB>;
    constexpr int ND = RL::ND;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gw = (blockIdx.x * kTBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * kTWaves;
    const R *sed = reinterpret_cast<const R *>(bp.sed);
    uint4 *recs = reinterpret_cast<uint4 *>(p.rec);
    const int n0 = p.geo.n[0], n1 = p.geo.n[1], n2 = p.geo.n[2];
    const uint64_t fx = (uint64_t)n1 * n2, fy = (uint64_t)n0 * n2, fz = (uint64_t)n0 * n1;
    const uint64_t total = 2ull * (fx + fy + fz);
    double l_emit = 0.0;
    uint32_t n_pk = 0;
    for (uint32_t base = gw * 64u; base < p.nbatch; base += nw * 64u) {
        const uint32_t i = base + lane;
        const bool act = i < p.nbatch;
        uint32_t tile = 0;
        const uint64_t g = (uint64_t)bp.g0 + i;
        int32_t c[3];
        sample_direction_wave(p.seed, p.solve_id, g, p.step, false, act, c, 3ull);
        if (act) {
            const U64x4 r = philox4x64_10(g, p.step, 0ull, 2ull, p.seed, p.solve_id);
            uint64_t idx = __umul64hi(r.v[0], total);
            int axis, plus;
            if (idx < 2ull * fx) { axis = 0; plus = idx >= fx; idx -= plus ? fx : 0ull; }
            else if ((idx -= 2ull * fx) < 2ull * fy) { axis = 1; plus = idx >= fy; idx -= plus ? fy : 0ull; }
            else { idx -= 2ull * fy; axis = 2; plus = idx >= fz; idx -= plus ? fz : 0ull; }
            const int u = axis == 0 ? 1 : 0, v = axis == 2 ? 1 : 2;
            const uint32_t nu = (uint32_t)p.geo.n[u], id = (uint32_t)idx;   // id < n_u n_v <= 2^20
            const int ia = (int)(id % nu), ib = (int)(id / nu);
            int32_t o[3], kk[3];
            o[axis] = plus ? 2 * p.geo.n[axis] : 0;
            kk[axis] = plus ? p.geo.n[axis] - 1 : 0;
            o[u] = 2 * ia + 1;
            kk[u] = ia;
            o[v] = 2 * ib + 1;
            kk[v] = ib;
            int32_t cn = c[axis] < 0 ? -c[axis] : c[axis];
            if (cn == 0) cn = 1;                               // never along the face itself
            c[axis] = plus ? -cn : cn;
            const int64_t qq = (int64_t)c[0] * c[0] + (int64_t)c[1] * c[1] + (int64_t)c[2] * c[2];
            double ww = bp.ndot * p.dt;
            ww = ww / (double)bp.packets;
            ww = ww * (2.0 * (double)cn) / sqrt((double)qq);
            l_emit += ww * bp.carried;
            n_pk += 1u;
            const uint32_t active = bp.active;
            R F[MB], D[ND];
#pragma unroll
            for (int j = 0; j < MB; ++j) F[j] = sed[j];
#pragma unroll
            for (int j = 0; j < ND; ++j) D[j] = (!RL::F64 || ((active >> j) & 1u)) ? R(0) : R(INFINITY);
            const uint32_t a0 = pack_dir(c[0]), a1 = pack_dir(c[1]), a2 = pack_dir(c[2]);
            const double Ld = sqrt((double)qq) * p.half_dl;
            const R len = RL::F64 ? (R)Ld : (R)(Ld * p.len_scale);
            const uint32_t jw = active ? (uint32_t)__builtin_ctz(active) : 0u;
            store_record<R, S, MB>(recs + (size_t)i * RL::STRIDE, c[0], c[1], c[2],
                                   pack_cell(kk[0], kk[1], kk[2], 3u), next_face(kk[0], o[0], a0), jw,
                                   next_face(kk[1], o[1], a1), next_face(kk[2], o[2], a2), active, ww, len, F, D);
            tile = tile_of_cell(p.geo, kk[0], kk[1], kk[2]);
        }
        // rank in the tile's list: the packets of a wavefront start on boundary
        // tiles drawn at random, nearly all different, so one atomic per lane
        // (issued together) rather than one per distinct tile in turn
        uint32_t rel = 0;
        if (act) rel = atomicAdd(p.cnt + tile, 1u);
        if (act) p.side[i] = rel;
    }
    double v[8] = {l_emit, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    unsigned long long cc[4] = {0ull, n_pk, 0ull, 0ull};
    block_ledger_add(p.slots + blockIdx.x, v, cc);
}

__global__ void k_tset_u32(uint32_t *p, uint32_t v) {
    if (threadIdx.x == 0) *p = v;
}

// List positions of the recombination packets: offset of the cell's tile +
// rank (records RS 16-byte units apart; the cell is word 3).
template <int RS>
__global__ void __launch_bounds__(kTBlock) k_tscatter_diffuse(const TParams p) {
    const uint32_t stride = gridDim.x * kTBlock;
    const uint32_t n = min(p.ctrl->ndiff, p.capacity);
    const uint4 *recs = reinterpret_cast<const uint4 *>(p.rec);
    for (uint32_t i = blockIdx.x * kTBlock + threadIdx.x; i < n; i += stride) {
        const uint32_t kw = recs[(size_t)i * RS].x;       // word 0: the cell
        const int k0 = (int)(kw & 1023u), k1 = (int)((kw >> 10) & 1023u), k2 = (int)((kw >> 20) & 1023u);
        const uint32_t tile = tile_of_cell(p.geo, k0, k1, k2);
        const uint32_t pos = tile < p.n_tiles ? p.off[tile] + p.side[i] : 0xffffffffu;
        if (pos < p.capacity) p.idx0[pos] = i;
        else atomicOr(&p.ctrl->err, 1u);
    }
}

// ---------------------------------------------------------------------------
// Scan of the per-tile counts into list offsets and runs of at most cmax
// packets (three launches: block sums, scan of the block sums, local scans).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_scan2(uint32_t &a, uint32_t &b, uint32_t &ta, uint32_t &tb) {
    // exclusive scan of (a, b) over a block of kScanBlock threads; totals in (ta, tb)
    __shared__ uint32_t sa[kScanBlock / 64], sb[kScanBlock / 64];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint32_t ia = a, ib = b;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t ua = (uint32_t)__shfl_up((int)ia, d), ub = (uint32_t)__shfl_up((int)ib, d);
        if (lane >= (uint32_t)d) { ia += ua; ib += ub; }
    }
    if (lane == 63u) { sa[wv] = ia; sb[wv] = ib; }
    __syncthreads();
    uint32_t pa = 0, pb = 0;
    ta = 0; tb = 0;
    for (uint32_t u = 0; u < kScanBlock / 64; ++u) {
        if (u < wv) { pa += sa[u]; pb += sb[u]; }
        ta += sa[u]; tb += sb[u];
    }
    __syncthreads();
    a = pa + ia - a;
    b = pb + ib - b;
}

__device__ __forceinline__ uint32_t runs_of(uint32_t n, uint32_t cmax) { return (n + cmax - 1u) / cmax; }

__global__ void __launch_bounds__(kScanBlock) k_tscan_a(const TParams p) {
    const uint32_t t0 = blockIdx.x * kScanTiles + threadIdx.x * kScanPer;
    uint32_t a = 0, b = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const uint32_t t = t0 + k;
        const uint32_t n = t < p.n_tiles ? p.cnt[t] : 0u;
        a += n;
        b += runs_of(n, p.cmax);
    }
    uint32_t ta, tb;
    block_scan2(a, b, ta, tb);
    if (threadIdx.x == 0) {
        p.bsum[2 * blockIdx.x] = ta;
        p.bsum[2 * blockIdx.x + 1] = tb;
    }
}

// A run's `shared` word: bit 0 the tile has more than one run this pass, bits
// 1 and up the solve of the tile (fused steps; 0 in a single solve).
//
// Every block first forms the pass's totals and its own offsets from the
// block sums of k_tscan_a (nblk of them); block 0 publishes the totals.
template <bool B>
__global__ void __launch_bounds__(kScanBlock) k_tscan_c(const TParams p, uint32_t nblk, int nxt) {
    uint32_t pa = 0, pb = 0, sa = 0, sb = 0;
    for (uint32_t i = threadIdx.x; i < nblk; i += kScanBlock) {
        const uint32_t x = p.bsum[2 * i], y = p.bsum[2 * i + 1];
        sa += x;
        sb += y;
        if (i < blockIdx.x) { pa += x; pb += y; }
    }
    uint32_t base_a, base_b, total_a, total_b;
    block_scan2(pa, pb, base_a, base_b);
    block_scan2(sa, sb, total_a, total_b);
    const bool bad = total_a > p.capacity || total_b > p.max_chunks;
    const uint32_t nch = bad ? 0u : total_b;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (bad) p.ctrl->err |= 2u;
        p.ctrl->total[nxt] = bad ? 0u : total_a;
        p.ctrl->n_chunks[nxt] = nch;
        p.ctrl->claim = 0u;
    }
    const uint32_t t0 = blockIdx.x * kScanTiles + threadIdx.x * kScanPer;
    uint32_t n[kScanPer];
    uint32_t a = 0, b = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const uint32_t t = t0 + k;
        n[k] = t < p.n_tiles ? p.cnt[t] : 0u;
        a += n[k];
        b += runs_of(n[k], p.cmax);
    }
    uint32_t ta, tb;
    block_scan2(a, b, ta, tb);
    a += base_a;
    b += base_b;
    TChunk *out = nxt ? p.ch1 : p.ch0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const uint32_t t = t0 + k;
        if (t >= p.n_tiles) break;
        p.off[t] = a;
        const uint32_t nr = runs_of(n[k], p.cmax);
        for (uint32_t j = 0; j < nr; ++j) {
            if (b + j >= nch) break;
            TChunk c;
            c.tile = t;
            c.start = a + j * p.cmax;
            c.len = min(p.cmax, n[k] - j * p.cmax);
            c.shared = (nr > 1u ? 1u : 0u) | (B ? ((uint32_t)p.tsolve[t] << 1) : 0u);
            out[b + j] = c;
        }
        a += n[k];
        b += nr;
        p.cnt[t] = 0u;
    }
}

// Record ids of the packets that moved on, into the next pass's lists.  The
// run's 27 destination bases (neighbour's list offset + the run's reservation
// in it) are formed once per run in LDS.
template <bool B>
__global__ void __launch_bounds__(kTBlock) k_tscatter(const TParams p, int cur) {
    const uint32_t nch = p.ctrl->n_chunks[cur];
    const TChunk *chs = cur ? p.ch1 : p.ch0;
    const uint32_t *in = cur ? p.idx1 : p.idx0;
    uint32_t *outl = cur ? p.idx0 : p.idx1;
    __shared__ uint32_t s_dst[kCodes];
    for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const TChunk ch = chs[c];
        if (ch.start > p.capacity || ch.len > p.capacity - ch.start) continue;   // flagged by the march
        if (threadIdx.x < kCodes) {
            // bases of codes this run did not use are never read
            const RunSolve<float> rs = run_solve<float, B>(p, ch.shared >> 1);
            const int64_t y = ch.tile >= rs.tile0
                ? neighbour_tile(rs.geo, ch.tile - rs.tile0, threadIdx.x, p.periodic != 0u) : -1;
            s_dst[threadIdx.x] = (y >= 0 && y < (int64_t)rs.n_tiles)
                                     ? p.off[rs.tile0 + y] + p.cbase[(size_t)c * kCodes + threadIdx.x] : 0xffffffffu;
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < ch.len; k += kTBlock) {
            const uint32_t pos = ch.start + k;
            const uint32_t sd = p.side[pos];
            if (sd == kSideDead) continue;
            const uint32_t code = sd & 31u, rank = sd >> 5;
            const uint32_t base = code < (uint32_t)kCodes ? s_dst[code] : 0xffffffffu;
            const uint32_t dst = base + rank;
            if (base != 0xffffffffu && dst < p.capacity) outl[dst] = in[pos];
            else atomicOr(&p.ctrl->err, 4u);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// One pass of the march over the runs of every tile.
// ---------------------------------------------------------------------------
// Occupancy target (wavefronts per SIMD) the register allocation is held to.
template <typename R, int MB> struct TOcc { static constexpr int value = 2; };
template <> struct TOcc<float, 1> { static constexpr int value = 4; };
template <> struct TOcc<float, 8> { static constexpr int value = 4; };

// TR: packets are traced (their cells and fates recorded); the instance
// without tracing carries no trace state.  B: a fused step of many solves
// (each run's solve from the table; ledger per (solve, block) slot).
// FIN: the finishing pass.  Every packet of the lists is marched to its end
// (absorbed, escaped or extinguished) across as many tiles as it takes, with
// the absorbers read from the grid and the deposits added to the grid's
// accumulators by float64 atomics; a packet that enters another tile keeps
// its lane (its exhausted bins are dropped there, as at a hand-over).  It
// replaces the long tail of passes that carry few packets each.
template <typename R, int S, bool TH, int MB, int NA, int NB, bool PER, bool TR, bool B, bool FIN>
__global__ void __launch_bounds__(kTBlock, (TOcc<R, MB>::value)) k_tmarch(const TParams p, int cur) {
    static_assert(!(FIN && TR), "the finishing pass does not trace");
    constexpr bool F64 = std::is_same<R, double>::value;
    constexpr uint32_t ACC = (S == 1) ? (TH ? 2u : 1u) : 4u;
    using KV = typename std::conditional<S == 1, R, typename Vec4<R>::T>::type;
    using V4R = typename Vec4<R>::T;
    using RL = TRec<R, S, MB>;
    constexpr int ND = RL::ND;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64u - lane));

    __shared__ KV s_kap[kTileCells];
    __shared__ double s_acc[kTileCells * ACC];
    __shared__ uint32_t s_cnt[kCodes];
    __shared__ uint32_t s_list[kMaxRun];
    __shared__ uint32_t s_next, s_claim;
    __shared__ float s_sigf[3 * MB];          // float32 form: cross-sections, indexed per lane

    const uint32_t nch = p.ctrl->n_chunks[cur];
    const TChunk *chs = cur ? p.ch1 : p.ch0;
    const uint32_t *list = cur ? p.idx1 : p.idx0;
    uint4 *recs = reinterpret_cast<uint4 *>(p.rec);

    double l_abs = 0.0, l_esc = 0.0, l_trunc = 0.0;
    uint32_t n_cross = 0, n_esc = 0, n_trunc = 0;

    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_claim = atomicAdd(&p.ctrl->claim, 1u);
        __syncthreads();
        const uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_claim);   // block-uniform
        if (c >= nch) break;
        const TChunk ch = chs[c];
        const uint32_t sid = ch.shared >> 1;        // the run's solve (fused steps)
        const RunSolve<R> rs = run_solve<R, B>(p, sid);
        if (ch.tile >= p.n_tiles || ch.tile < rs.tile0 || ch.tile - rs.tile0 >= rs.n_tiles
            || ch.start > p.capacity || ch.len > p.capacity - ch.start || ch.len > p.cmax) {
            if (threadIdx.x == 0) atomicOr(&p.ctrl->err, 8u);
            continue;
        }
        const GridGeom geo = rs.geo;
        const uint32_t tile = ch.tile - rs.tile0;   // the tile within its solve's grid
        const int tx = (int)(tile % (uint32_t)geo.nb[0]);
        const int ty = (int)((tile / (uint32_t)geo.nb[0]) % (uint32_t)geo.nb[1]);
        const int tz = (int)(tile / ((uint32_t)geo.nb[0] * (uint32_t)geo.nb[1]));
        const double tau_kill = rs.tau_kill;
        // float32 form: the extinction and drop depths in units of ln 2
        const float kill_t = depth_threshold(tau_kill);
        const float drop_t = depth_threshold(fmax(tau_kill, (double)kDropDepth));
        const CTab<R> ctab = (CTab<R>)rs.tab;
        const typename MarchTab<R, MB>::type tab = MarchTab<R, MB>::make(ctab);

        // stage the tile's absorbers, clear its accumulators
        const KV *kg = reinterpret_cast<const KV *>(rs.kappa);
        // (each thread issues all its loads before it waits for the first; its
        // index is made opaque here so that the per-thread offsets are formed
        // per run, not kept in registers across the march)
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        {
            constexpr int KPT = FIN ? 1 : kTileCells / kTBlock;
            constexpr int LPT = kMaxRun / kTBlock;
            const uint32_t ns = min(ch.len, (uint32_t)kMaxRun);
            KV kv[KPT];
            uint32_t iv[LPT];
            // float32 form: the run's cross-sections, indexed per lane
            const bool sig_lane = !F64 && tid < 3u * MB;
            const float sg = sig_lane ? (float)ctab[tid] : 0.0f;
            if constexpr (!FIN) {
                const KV *kt = kg + ((size_t)tile << (3 * kTileLog2));
#pragma unroll
                for (int k = 0; k < KPT; ++k) kv[k] = kt[local_to_morton(tid + k * kTBlock)];
            }
#pragma unroll
            for (int k = 0; k < LPT; ++k) {
                const uint32_t i = tid + k * kTBlock;
                iv[k] = i < ns ? list[ch.start + i] : 0u;
            }
            if constexpr (!FIN) {
#pragma unroll
                for (int k = 0; k < KPT; ++k) s_kap[tid + k * kTBlock] = kv[k];
                for (int i = threadIdx.x; i < kTileCells * (int)ACC; i += kTBlock) s_acc[i] = 0.0;
            }
#pragma unroll
            for (int k = 0; k < LPT; ++k) {
                const uint32_t i = tid + k * kTBlock;
                if (i < ns) s_list[i] = iv[k];
            }
            if (sig_lane) s_sigf[tid] = sg;
        }
        if (threadIdx.x < kCodes) s_cnt[threadIdx.x] = 0u;
        if (threadIdx.x == 0) s_next = 0u;
        __syncthreads();

        // ---- packet state (one per lane) ----
        bool alive = false;
        bool pend = false;                       // segment over, fate not yet settled (implies alive)
        bool kill = false;                       // extinction candidate at the last crossing
        bool exhausted = false;                  // wave-uniform
        uint32_t pos = 0, rid = 0;               // list position and record of the lane's packet
        int k0 = 0, k1 = 0, k2 = 0;
        uint32_t d0 = 1, d1 = 1, d2 = 1, a0 = 0, a1 = 0, a2 = 0, pnum = 0, pden = 1;
        uint32_t lax = 3;                        // axis of the last face crossed (3: none)
        int hlast = 0;                           // natural index of the last cell crossed (traces)
        double sprev = 0.0, L = 0.0, w = 0.0, absd = 0.0;
        float Lf = 0.0f;
        float dropf = 0.0f;                      // float32 form: photons of bins dropped in this segment
        uint32_t loc = 0, count = 0, active = 0;
        uint32_t wbins = 0;                      // wave-uniform: bins some crossing lane may carry
        int ltx = tx, lty = ty, ltz = tz;        // finishing pass: the tile the lane's packet is in
        uint32_t gcell = 0;                      // finishing pass: the grid slot of its cell
        DepthTest<R, S, MB> dtest;
        int32_t tix = -1;
        R F[MB], D[ND];
#pragma unroll
        for (int j = 0; j < MB; ++j) F[j] = R(0);
#pragma unroll
        for (int j = 0; j < ND; ++j) D[j] = R(0);

        for (;;) {
            // Lanes whose segment ended wait, like dead lanes, until enough lanes
            // are idle; then the wave settles their fates together (extinction
            // check over every bin, record write-back, ledger) and refills the
            // dead lanes, so that code runs once per refill, not per crossing.
            const uint32_t npend = (uint32_t)__popcll(__ballot(pend));
            const uint32_t nidle = (uint32_t)__popcll(__ballot(!alive)) + npend;
            const bool trigger = nidle != 0u
                && (nidle == 64u || (exhausted ? npend >= p.refill_min : nidle >= p.refill_min));
            // what the settled packets add to the ledger (added below in uniform control flow)
            double st_abs = 0.0, st_esc = 0.0, st_trunc = 0.0;
            uint32_t st_nesc = 0, st_ntrunc = 0;
            if (trigger && npend != 0u && pend) {
                bool ex = kill;
                if constexpr (!F64) ex = kill && dtest.ext.full(tab, active, kill_t, D);
                // (periodic: the cell has been wrapped at the crossing; "out" is
                // the end of the packet's path)
                const bool o0 = !PER && (uint32_t)k0 >= (uint32_t)geo.n[0];
                const bool o1 = !PER && (uint32_t)k1 >= (uint32_t)geo.n[1];
                const bool o2 = !PER && (uint32_t)k2 >= (uint32_t)geo.n[2];
                const bool out = PER ? (d0 > p.dmax || d1 > p.dmax || d2 > p.dmax) : (o0 | o1 | o2);
                int dx = (k0 >> kTileLog2) - tx, dy = (k1 >> kTileLog2) - ty, dz = (k2 >> kTileLog2) - tz;
                if constexpr (PER) {
                    dx = wrap_step(dx);
                    dy = wrap_step(dy);
                    dz = wrap_step(dz);
                }
                const bool leave = !FIN && !out && (dx | dy | dz) != 0;
                const uint32_t fate = ex ? 1u : (out ? 2u : (leave ? 3u : 0u));
                if constexpr (!F64 && MB > 1) {
                    // float32 form: bins exhausted at the tile boundary leave the packet
                    if (fate == 3u)
                        dropf += drop_exhausted<S, MB, NA, NB>(tab, active, drop_t, D, F,
                                                               wbins);
                }
                if (fate != 0u) {                  // fate 0: a new witness bin, the packet marches on
                    const bool traced = TR && tix >= 0;
                    int32_t *rec = p.trace + (size_t)(traced ? tix : 0) * (RT_TRACE_HDR_DEV + p.trace_len);
                    st_abs = w * absd;
                    st_trunc = w * (double)dropf;
                    if (fate == 3u) {
                        // moves on into a neighbour tile: record back, rank among the run's
                        // packets bound for the same tile
                        uint32_t jw = 0;
                        if constexpr (!F64) jw = dtest.ext.jw;
                        store_moving<R, S, MB>(recs + (size_t)rid * RL::STRIDE, unpack_dir(a0), unpack_dir(a1),
                                               unpack_dir(a2), pack_cell(k0, k1, k2, lax), d0, jw, d1, d2, active,
                                               w, F64 ? L : Lf, F, D);
                        const uint32_t code = (uint32_t)((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1));
                        const uint32_t rank = atomicAdd(&s_cnt[code], 1u);
                        p.side[pos] = code | (rank << 5);
                        if (traced) rec[0] = (int32_t)count;
                    } else {
                        R left = R(0);
#pragma unroll
                        for (int j = 0; j < MB; ++j) left += F[j];
                        const double wl = w * (double)left;
                        if (fate == 2u) { st_esc = wl; st_nesc = 1u; } else { st_trunc += wl; st_ntrunc = 1u; }
                        p.side[pos] = kSideDead;
                        if (traced) {
                            const int face = fate == 1u ? 0
                                : ((o0 ? 1 : 0) | (o1 ? 2 : 0) | (o2 ? 4 : 0)
                                   | (k0 >= geo.n[0] ? 8 : 0) | (k1 >= geo.n[1] ? 16 : 0)
                                   | (k2 >= geo.n[2] ? 32 : 0));
                            rec[0] = (int32_t)count; rec[1] = (PER && fate == 2u) ? 3 : (int32_t)fate;
                            rec[2] = face; rec[3] = hlast;
                            rec[4] = unpack_dir(a0);
                            rec[5] = unpack_dir(a1);
                            rec[6] = unpack_dir(a2);
                            uint32_t ns;
                            rec[7] = (int32_t)source_of(p.g0 + rid, p.q, p.r, ns);
                        }
                    }
                    alive = false;
                }
                pend = false;
                kill = false;
            }
            l_abs += st_abs;
            l_esc += st_esc;
            l_trunc += st_trunc;
            n_esc += st_nesc;
            n_trunc += st_ntrunc;
            const uint64_t dead = __ballot(!alive);
            const uint32_t ndead = (uint32_t)__popcll(dead);
            if (trigger && !exhausted && ndead != 0u) {
                uint32_t b0 = 0;
                if (lane == 0) b0 = atomicAdd(&s_next, ndead);
                b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b0);
                if (b0 >= ch.len) {
                    exhausted = true;
                } else {
                    const uint32_t got = min(ndead, ch.len - b0);
                    const uint32_t rank = (uint32_t)__popcll(dead & lt_mask);
                    if (!alive && rank < got) {
                        pos = ch.start + b0 + rank;
                        const uint32_t li = b0 + rank;
                        const uint32_t ri = li < (uint32_t)kMaxRun ? s_list[li] : list[ch.start + li];
                        if (ri >= p.capacity) {
                            atomicOr(&p.ctrl->err, 16u);
                            p.side[pos] = kSideDead;
                        } else {
                            rid = ri;
                            const uint4 *rp = recs + (size_t)ri * RL::STRIDE;
                            uint32_t wd[RL::WORDS];
#pragma unroll
                            for (int u = 0; u < RL::UNITS; ++u) {
                                const uint4 v = rp[u];
                                wd[4 * u] = v.x; wd[4 * u + 1] = v.y; wd[4 * u + 2] = v.z; wd[4 * u + 3] = v.w;
                            }
                            constexpr int M = RL::MOV;
                            const int32_t c0 = (int32_t)wd[M], c1 = (int32_t)wd[M + 1], c2 = (int32_t)wd[M + 2];
                            const uint32_t kw = wd[0];
                            d0 = wd[1] & 0xfffu;
                            const uint32_t jw = (wd[1] >> 12) & 0xfu;
                            d1 = wd[1] >> 16;
                            d2 = wd[2] & 0xffffu;
                            active = wd[2] >> 16;
                            w = __hiloint2double((int)wd[M + 4], (int)wd[M + 3]);
                            if constexpr (F64) L = __hiloint2double((int)wd[M + 6], (int)wd[M + 5]);
                            else Lf = __uint_as_float(wd[M + 5]);
                            if constexpr (F64) {
#pragma unroll
                                for (int j = 0; j < MB; ++j) {
                                    F[j] = __hiloint2double((int)wd[4 + 2 * j], (int)wd[3 + 2 * j]);
                                    D[j] = __hiloint2double((int)wd[4 + 2 * MB + 2 * j], (int)wd[3 + 2 * MB + 2 * j]);
                                }
                            } else {
#pragma unroll
                                for (int j = 0; j < ND; ++j) D[j] = __uint_as_float(wd[3 + j]);
#pragma unroll
                                for (int j = 0; j < MB; ++j) F[j] = __uint_as_float(wd[3 + ND + j]);
                            }
                            k0 = (int)(kw & 1023u);
                            k1 = (int)((kw >> 10) & 1023u);
                            k2 = (int)((kw >> 20) & 1023u);
                            const uint32_t ax = kw >> 30;
                            lax = ax;
                            // a record that is not a packet of this tile is an internal error
                            const bool bad = k0 >= geo.n[0] || k1 >= geo.n[1]
                                || k2 >= geo.n[2] || (k0 >> kTileLog2) != tx || (k1 >> kTileLog2) != ty
                                || (k2 >> kTileLog2) != tz || ((uint32_t)(c0 | c1 | c2) == 0u);
                            if (bad) {
                                atomicOr(&p.ctrl->err, 16u);
                                p.side[pos] = kSideDead;
                            } else {
                                a0 = pack_dir(c0);
                                a1 = pack_dir(c1);
                                a2 = pack_dir(c2);
                                // entry parameter of this cell: the last face crossed
                                if (ax == 3u) { pnum = 0u; pden = 1u; }
                                else {
                                    pnum = (ax == 0u ? d0 : (ax == 1u ? d1 : d2)) - 2u;
                                    pden = (ax == 0u ? a0 : (ax == 1u ? a1 : a2)) & kMag;
                                }
                                sprev = (ax == 3u) ? 0.0 : (double)pnum / (double)pden;
                                if constexpr (!F64) dtest.ext.resume(jw < (uint32_t)MB ? jw : 0u, s_sigf);
                                if constexpr (TR) {
                                    tix = trace_slot(p, p.g0 + ri);
                                    count = tix >= 0 ? (uint32_t)p.trace[(size_t)tix * (RT_TRACE_HDR_DEV + p.trace_len)]
                                                     : 0u;
                                }
                                absd = 0.0;
                                dropf = 0.0f;
                                loc = local_cell(k0, k1, k2);
                                if constexpr (FIN) {
                                    ltx = tx;
                                    lty = ty;
                                    ltz = tz;
                                    gcell = (tile << (3 * kTileLog2)) | local_to_morton(loc);
                                }
                                alive = true;
                            }
                        }
                    }
                }
            }
            if (exhausted && __ballot(alive) == 0ull) break;
            // lanes change packets or bins only at a settle or refill (bins are
            // also dropped while crossing, which only clears bits)
            if constexpr (!F64 && MB > 1) {
                if (trigger) wbins = wave_bins<MB>(alive && !pend, active);
            }

            // (with no lane marching this iteration only settles and refills: one
            // path through the loop body keeps the packet state in its registers)
            uint32_t it_cross = 0;
            if (alive && !pend) {
                // this cell's absorbers (the load runs while the traversal arithmetic does)
                KV kap;
                if constexpr (FIN) kap = kg[gcell];
                else kap = s_kap[loc];
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
                    // exact: num < 2^12, pden < 2^21, both products < 2^32
                    const uint32_t diff = __umul24(num, pden) - __umul24(pnum, den);
                    l = Lf * (float)diff * __builtin_amdgcn_rcpf((float)den * (float)pden);
                }
                int here = 0;                          // natural index, for traces only
                if constexpr (TR) here = k0 + geo.n[0] * (k1 + geo.n[1] * k2);
                // the cell steps along the crossed axes (ties cross several)
                const int s0 = m0 ? ((a0 & kNeg) ? -1 : 1) : 0;
                const int s1 = m1 ? ((a1 & kNeg) ? -1 : 1) : 0;
                const int s2 = m2 ? ((a2 & kNeg) ? -1 : 1) : 0;
                k0 += s0;
                k1 += s1;
                k2 += s2;
                if (m0) d0 += 2u;
                if (m1) d1 += 2u;
                if (m2) d2 += 2u;
                bool out;
                int dx, dy, dz;
                if constexpr (PER) {
                    // Sec. 2, periodic boundaries: back in through the opposite
                    // face; the path ends past dmax half cells along an axis
                    k0 = wrap_cell(k0, geo.n[0]);
                    k1 = wrap_cell(k1, geo.n[1]);
                    k2 = wrap_cell(k2, geo.n[2]);
                    out = d0 > p.dmax || d1 > p.dmax || d2 > p.dmax;
                    dx = wrap_step((k0 >> kTileLog2) - (FIN ? ltx : tx));
                    dy = wrap_step((k1 >> kTileLog2) - (FIN ? lty : ty));
                    dz = wrap_step((k2 >> kTileLog2) - (FIN ? ltz : tz));
                } else {
                    out = (uint32_t)k0 >= (uint32_t)geo.n[0] || (uint32_t)k1 >= (uint32_t)geo.n[1]
                        || (uint32_t)k2 >= (uint32_t)geo.n[2];
                    dx = (k0 >> kTileLog2) - (FIN ? ltx : tx);
                    dy = (k1 >> kTileLog2) - (FIN ? lty : ty);
                    dz = (k2 >> kTileLog2) - (FIN ? ltz : tz);
                }
                const bool leave = !out && (dx | dy | dz) != 0;
                // next cell's index in the tile: one step from this cell's (unused
                // when the packet leaves the tile in a tile pass).  Masked from the
                // cell instead in the finishing pass (the tile the packet enters)
                // and with periodic boundaries (a wrap can stay in the tile when an
                // axis has one tile)
                const uint32_t nloc = (FIN || PER) ? local_cell(k0, k1, k2)
                                                   : (uint32_t)((int)loc + s0 + (s1 << kTileLog2) + (s2 << (2 * kTileLog2)));
                uint32_t ngc = gcell;
                if constexpr (FIN) {
                    // (a packet that left the grid keeps its last cell)
                    if (!out) ngc = (tile_of_cell(geo, k0, k1, k2) << (3 * kTileLog2)) | local_to_morton(nloc);
                }

                R absorbed, e0, e1, e2, hs, tmin;
                cross_cell<R, S, TH, MB, NA, NB>(l, kap, tab, F, D, absorbed, e0, e1, e2, hs, tmin, wbins);

                // ---- deposit into the tile's float64 accumulators in LDS ----
                // (zero deposits are added too: an LDS add is cheaper than the
                // branch; one plane per accumulated value, so the adds of a
                // wavefront spread over the banks)
                if constexpr (FIN) {
                    double *g = rs.acc + (size_t)gcell * ACC;
                    if (S == 1) {
                        unsafeAtomicAdd(g, w * (double)absorbed);
                        if (TH) unsafeAtomicAdd(g + 1, w * (double)hs);
                    } else {
                        unsafeAtomicAdd(g, w * (double)e0);
                        unsafeAtomicAdd(g + 1, w * (double)e1);
                        unsafeAtomicAdd(g + 2, w * (double)e2);
                        if (TH) unsafeAtomicAdd(g + 3, w * (double)hs);
                    }
                } else {
                    double *cell = s_acc + loc;
                    if (S == 1) {
                        atomicAdd(cell, w * (double)absorbed);
                        if (TH) atomicAdd(cell + kTileCells, w * (double)hs);
                    } else {
                        atomicAdd(cell, w * (double)e0);
                        atomicAdd(cell + kTileCells, w * (double)e1);
                        atomicAdd(cell + 2 * kTileCells, w * (double)e2);
                        if (TH) atomicAdd(cell + 3 * kTileCells, w * (double)hs);
                    }
                }
                absd += (double)absorbed;
                it_cross = 1;
                if constexpr (TR) {
                    const bool traced = tix >= 0;
                    int32_t *rec = p.trace + (size_t)(traced ? tix : 0) * (RT_TRACE_HDR_DEV + p.trace_len);
                    if (traced && count < (uint32_t)p.trace_len) rec[RT_TRACE_HDR_DEV + count] = here;
                    ++count;
                }

                // the state moves on to the next cell; a packet that left the tile,
                // the grid, or whose witness depth reached the cut is settled later
                loc = nloc;
                if constexpr (FIN) gcell = ngc;
                lax = (uint32_t)ax;
                if (F64) sprev = snew; else { pnum = num; pden = den; }
                if constexpr (TR) hlast = here;
                if constexpr (F64) kill = tmin >= tau_kill;
                else kill = Extinction<S, MB>::depth(dtest.ext.wH, dtest.ext.wHe1, dtest.ext.wHe2, D)
                            >= kill_t;
                if constexpr (FIN) {
                    // into the next tile without a hand-over: the bins exhausted at
                    // the boundary leave the packet there all the same (the order
                    // against an extinction check at this crossing does not matter:
                    // only bins past the cut are dropped)
                    if (leave) {
                        ltx = k0 >> kTileLog2;
                        lty = k1 >> kTileLog2;
                        ltz = k2 >> kTileLog2;
                        if constexpr (!F64 && MB > 1)
                            dropf += drop_exhausted<S, MB, NA, NB>(tab, active, drop_t, D,
                                                                   F, wbins);
                    }
                    pend = kill || out;
                } else {
                    pend = kill || out || leave;
                }
            }
            n_cross += it_cross;

            // ---- run used up and few lanes left: park them for the next pass ----
            // (every parked packet has crossed a cell in this pass, so it progresses)
            if (!FIN && exhausted && p.park != 0u) {
                const uint64_t am = __ballot(alive && !pend);
                if (am != 0ull && (uint32_t)__popcll(am) <= p.park) {
                    double pk_abs = 0.0, pk_drop = 0.0;
                    if (alive && !pend) {
                        uint32_t jw = 0;
                        if constexpr (!F64) jw = dtest.ext.jw;
                        store_moving<R, S, MB>(recs + (size_t)rid * RL::STRIDE, unpack_dir(a0), unpack_dir(a1),
                                               unpack_dir(a2), pack_cell(k0, k1, k2, lax), d0, jw, d1, d2, active,
                                               w, F64 ? L : Lf, F, D);
                        const uint32_t stay = 13u;                 // code of the tile itself
                        const uint32_t rank = atomicAdd(&s_cnt[stay], 1u);
                        p.side[pos] = stay | (rank << 5);
                        if (TR && tix >= 0) p.trace[(size_t)tix * (RT_TRACE_HDR_DEV + p.trace_len)] = (int32_t)count;
                        pk_abs = w * absd;
                        pk_drop = w * (double)dropf;
                        alive = false;
                    }
                    l_abs += pk_abs;
                    l_trunc += pk_drop;
                }
            }
        }
        __syncthreads();

        // ---- the tile's deposits into the grid's accumulators ----
        // (a run that shares its tile with other runs adds by atomics; the
        // others read a group of their cells' values before the first wait, a
        // cell with nothing to add reading the tile's first value unused, so
        // that every load is issued and one wait covers the group)
        if constexpr (!FIN) {
            double *ga = rs.acc + ((size_t)tile << (3 * kTileLog2)) * ACC;
            uint32_t ftid = threadIdx.x;
            asm volatile("" : "+v"(ftid));
            constexpr int FPT = kTileCells * (int)ACC / kTBlock;
            constexpr int G = FPT < 8 ? FPT : 8;
            static_assert(FPT % G == 0, "flush groups");
#pragma unroll
            for (int k0 = 0; k0 < FPT; k0 += G) {
                double v[G], o[G];
                uint32_t off[G];
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const uint32_t i = ftid + (uint32_t)((k0 + k) * kTBlock);
                    v[k] = s_acc[(i % ACC) * kTileCells + i / ACC];
                    off[k] = local_to_morton(i / ACC) * ACC + i % ACC;
                }
                if (ch.shared & 1u) {
#pragma unroll
                    for (int k = 0; k < G; ++k)
                        if (v[k] != 0.0) unsafeAtomicAdd(ga + off[k], v[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < G; ++k) o[k] = ga[v[k] != 0.0 ? off[k] : 0u];
#pragma unroll
                    for (int k = 0; k < G; ++k)
                        if (v[k] != 0.0) ga[off[k]] = o[k] + v[k];
                }
            }
        }
        // ---- reserve the run's places in the neighbours' next lists ----
        if (!FIN && threadIdx.x < kCodes) {
            const uint32_t n = s_cnt[threadIdx.x];
            if (n != 0u) {
                const int64_t y = neighbour_tile(geo, tile, threadIdx.x, PER);
                if (y >= 0 && y < (int64_t)rs.n_tiles)
                    p.cbase[(size_t)c * kCodes + threadIdx.x] = atomicAdd(p.cnt + rs.tile0 + y, n);
                else atomicOr(&p.ctrl->err, 32u);
            }
        }
        if constexpr (B) {
            // the run's ledger goes to its solve's slot of this block
            double v[8] = {0.0, 0.0, l_abs, 0.0, l_esc, 0.0, l_trunc, 0.0};
            unsigned long long cc[4] = {n_cross, 0ull, n_esc, n_trunc};
            block_ledger_add(p.slots + (size_t)sid * p.nblocks + blockIdx.x, v, cc);
            l_abs = l_esc = l_trunc = 0.0;
            n_cross = n_esc = n_trunc = 0;
        }
    }

    if constexpr (!B) {
        double v[8] = {0.0, 0.0, l_abs, 0.0, l_esc, 0.0, l_trunc, 0.0};
        unsigned long long cc[4] = {n_cross, 0ull, n_esc, n_trunc};
        block_ledger_add(p.slots + blockIdx.x, v, cc);
    }
}

__global__ void k_tslots_zero(LedgerSlot *s, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        LedgerSlot z;
        for (int k = 0; k < 8; ++k) z.s[k] = 0.0;
        for (int k = 0; k < 4; ++k) z.c[k] = 0ull;
        s[i] = z;
    }
}

__global__ void k_tzero_u32(uint32_t *p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// End of a batch: every list must be empty (unless a finishing pass marched
// what was left); errors go to the step ledger
// (fused steps: to every solve's).
__global__ void k_tcheck(TCtrl *ctrl, int cur, StepLedger *l, const BatchHead *hd, const BatchSolve *tb) {
    if (threadIdx.x == 0) {
        uint32_t e = ctrl->err;
        if (cur >= 0 && ctrl->total[cur] != 0u) e |= 64u;      // (cur < 0: a finishing pass ended the lists)
        if (e) {
            if (hd) {
                for (int b = 0; b < hd->n; ++b) tb[b].ledger->errors |= e;
            } else {
                l->errors |= e;
            }
        }
    }
}

TParams make_params(const TiledLaunch &t) {
    const MarchLaunch &m = t.m;
    TParams p;
    const bool f64 = m.fp64 != 0;
    p.geo = m.geo;
    p.half_dl = m.half_dl;
    p.len_scale = f64 ? 1.0 : 1.0e-18;
    p.src = m.src;
    p.src_ndot = m.src_ndot;
    p.src_sedsum = m.src_sedsum;
    p.sed = m.sed;
    p.tab = m.tab;
    p.q = m.n_src > 0 ? m.packets / (uint32_t)m.n_src : 0u;
    p.r = m.n_src > 0 ? m.packets % (uint32_t)m.n_src : 0u;
    p.n_src = (uint32_t)m.n_src;
    p.dt = m.dt;
    p.seed = m.seed;
    p.solve_id = m.solve_id;
    p.step = m.step_index;
    p.tau_kill = m.tau_kill;
    p.kappa = m.kappa;
    p.acc = m.acc;
    p.slots = m.slots;
    p.trace = m.trace;
    p.trace_n = m.trace ? m.trace_n : 0;
    p.trace_len = m.trace_len;
    p.trace_stride = (uint32_t)m.trace_stride;
    p.refill_min = (uint32_t)m.refill_min;
    p.park = 0u;
    p.g0 = t.g0;
    p.nbatch = t.nbatch;
    p.capacity = t.capacity;
    p.cmax = t.cmax;
    p.max_chunks = t.max_chunks;
    p.n_tiles = t.n_tiles;
    p.periodic = t.periodic;
    p.dmax = t.dmax;
    p.rec = t.rec;
    p.idx0 = t.idx[0];
    p.idx1 = t.idx[1];
    p.side = t.side;
    p.cnt = t.cnt;
    p.off = t.off;
    p.cbase = t.cbase;
    p.bsum = t.bsum;
    p.ch0 = t.chunks[0];
    p.ch1 = t.chunks[1];
    p.ctrl = t.ctrl;
    p.ledger = t.ledger;
    return p;
}

template <bool B = false>
void scan_lists(const TParams &p, uint32_t scan_blocks, hipStream_t st, int nxt) {
    hipLaunchKernelGGL(k_tscan_a, dim3(scan_blocks), dim3(kScanBlock), 0, st, p);
    hipLaunchKernelGGL(k_tscan_c<B>, dim3(scan_blocks), dim3(kScanBlock), 0, st, p, scan_blocks, nxt);
}

void scan(const TParams &p, const TiledLaunch &t, int nxt) { scan_lists<false>(p, t.scan_blocks, t.m.stream, nxt); }

template <typename R, int S, bool TH, int MB, int NA, int NB>
void run_passes(const TParams &p, const TiledLaunch &t);

template <typename R, int S, bool TH, int MB, int NA, int NB>
hipError_t run_batch(const TiledLaunch &t) {
    const TParams p = make_params(t);
    const hipStream_t st = t.m.stream;
    const dim3 grid(t.m.blocks), blk(kTBlock);
    hipLaunchKernelGGL((k_temit<R, S, TH, MB>), grid, blk, 0, st, p);
    scan(p, t, 0);
    hipLaunchKernelGGL(k_tscatter_emit<false>, dim3(8 * t.m.blocks), blk, 0, st, p);
    run_passes<R, S, TH, MB, NA, NB>(p, t);
    return hipGetLastError();
}

// The recombination packets of the sub-step, as a batch of their own (not
// traced; record ids from 0).
template <typename R, int S, bool TH, int MB, int NA, int NB>
hipError_t run_reemit(const TiledLaunch &t, const RecombParams &rp) {
    TParams p = make_params(t);
    p.trace_n = 0;
    p.g0 = 0u;
    p.nbatch = 0u;
    const hipStream_t st = t.m.stream;
    const dim3 grid(t.m.blocks), blk(kTBlock);
    hipLaunchKernelGGL(k_tzero_u32, dim3(1), dim3(64), 0, st, &t.ctrl->ndiff, 1u);
    hipLaunchKernelGGL((k_remit<R, S, MB>), grid, blk, 0, st, p, rp);
    scan(p, t, 0);
    hipLaunchKernelGGL((k_tscatter_diffuse<TRec<R, S, MB>::STRIDE>), dim3(8 * t.m.blocks), blk, 0, st, p);
    run_passes<R, S, TH, MB, NA, NB>(p, t);
    return hipGetLastError();
}

// A batch of background packets: records 0..nbatch-1 (not traced).
template <typename R, int S, bool TH, int MB, int NA, int NB>
hipError_t run_background(const TiledLaunch &t, const BackgroundParams &bp) {
    TParams p = make_params(t);
    p.trace_n = 0;
    const hipStream_t st = t.m.stream;
    const dim3 grid(t.m.blocks), blk(kTBlock);
    hipLaunchKernelGGL((k_bgemit<R, S, MB>), grid, blk, 0, st, p, bp);
    scan(p, t, 0);
    hipLaunchKernelGGL(k_tset_u32, dim3(1), dim3(64), 0, st, &t.ctrl->ndiff, t.nbatch);
    hipLaunchKernelGGL((k_tscatter_diffuse<TRec<R, S, MB>::STRIDE>), dim3(8 * t.m.blocks), blk, 0, st, p);
    run_passes<R, S, TH, MB, NA, NB>(p, t);
    return hipGetLastError();
}

template <typename R, int S, bool TH, int MB, int NA, int NB>
void run_passes(const TParams &p, const TiledLaunch &t) {
    const hipStream_t st = t.m.stream;
    const dim3 grid(t.m.blocks), blk(kTBlock);
    int cur = 0;
    TParams pp = p;
    const bool tr = p.trace_n > 0;
    // the finishing pass (not while tracing): after `finish` tile passes
    const uint32_t fin = (!tr && t.finish > 0u && t.finish < t.passes) ? t.finish : t.passes;
    for (uint32_t pass = 0; pass < t.passes; ++pass) {
        pp.park = pass < t.park_passes ? t.park_lanes : 0u;
        const bool timed = t.ev && *t.ev_used < t.ev_cap;
        if (timed) (void)hipEventRecord(t.ev[2 * *t.ev_used], st);
        if (pass == fin) {
            pp.park = 0u;
            if (p.periodic) hipLaunchKernelGGL((k_tmarch<R, S, TH, MB, NA, NB, true, false, false, true>), grid, blk, 0, st, pp, cur);
            else hipLaunchKernelGGL((k_tmarch<R, S, TH, MB, NA, NB, false, false, false, true>), grid, blk, 0, st, pp, cur);
            if (timed) {
                (void)hipEventRecord(t.ev[2 * *t.ev_used + 1], st);
                ++*t.ev_used;
            }
            cur = -1;
            break;
        }
        if (p.periodic) {
            if (tr) hipLaunchKernelGGL((k_tmarch<R, S, TH, MB, NA, NB, true, true, false, false>), grid, blk, 0, st, pp, cur);
            else hipLaunchKernelGGL((k_tmarch<R, S, TH, MB, NA, NB, true, false, false, false>), grid, blk, 0, st, pp, cur);
        } else {
            if (tr) hipLaunchKernelGGL((k_tmarch<R, S, TH, MB, NA, NB, false, true, false, false>), grid, blk, 0, st, pp, cur);
            else hipLaunchKernelGGL((k_tmarch<R, S, TH, MB, NA, NB, false, false, false, false>), grid, blk, 0, st, pp, cur);
        }
        if (timed) {
            (void)hipEventRecord(t.ev[2 * *t.ev_used + 1], st);
            ++*t.ev_used;
        }
        scan(p, t, cur ^ 1);
        // each run's scatter waits on two dependent reads before its copies:
        // many more blocks than the march keep enough runs in flight
        hipLaunchKernelGGL(k_tscatter<false>, dim3(8 * t.m.blocks), blk, 0, st, p, cur);
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_tcheck, dim3(1), dim3(64), 0, st, t.ctrl, cur, t.ledger, (const BatchHead *)nullptr,
                       (const BatchSolve *)nullptr);
}

// Bins of the first NA bins absorbed by hydrogen alone, of the next NB
// without HeII: the threshold-aligned layout every H+He table of several bins
// has in the tiled march (the host refuses others).
template <int S, int MB> struct Layout { static constexpr int NA = 0, NB = 0; };
template <> struct Layout<3, 8> { static constexpr int NA = 3, NB = 2; };

template <typename R, int S, bool TH, int MB>
hipError_t occ(int *n) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        n, reinterpret_cast<const void *>(&k_tmarch<R, S, TH, MB, Layout<S, MB>::NA, Layout<S, MB>::NB, false, false, false, false>),
        kTBlock, 0);
}

// What a launch runs after its packets are drawn: source packets (neither
// pointer), recombination packets (rp) or background packets (bp).
struct Extra {
    const RecombParams *rp;
    const BackgroundParams *bp;
};

template <typename R, int S, bool TH, int MB, int NA, int NB>
hipError_t run(const TiledLaunch &t, Extra x) {
    if (x.rp) return run_reemit<R, S, TH, MB, NA, NB>(t, *x.rp);
    if (x.bp) return run_background<R, S, TH, MB, NA, NB>(t, *x.bp);
    return run_batch<R, S, TH, MB, NA, NB>(t);
}

template <typename R, int S, bool TH>
hipError_t pick_mb(const TiledLaunch *t, Extra x, int mb, int *o) {
    switch (mb) {
    case 1: return t ? run<R, S, TH, 1, 0, 0>(*t, x) : occ<R, S, TH, 1>(o);
    case 8:
        if (!t) return occ<R, S, TH, 8>(o);
        if (S == 3 && t->m.layout != 1) return hipErrorInvalidValue;
        return run<R, S, TH, 8, Layout<S, 8>::NA, Layout<S, 8>::NB>(*t, x);
    default: return hipErrorInvalidValue;
    }
}

hipError_t dispatch(const TiledLaunch *t, Extra x, int species, int thermal, int fp64, int mb, int *o) {
    if (fp64) {
        if (species == 1)
            return thermal ? pick_mb<double, 1, true>(t, x, mb, o) : pick_mb<double, 1, false>(t, x, mb, o);
        return thermal ? pick_mb<double, 3, true>(t, x, mb, o) : pick_mb<double, 3, false>(t, x, mb, o);
    }
    if (species == 1)
        return thermal ? pick_mb<float, 1, true>(t, x, mb, o) : pick_mb<float, 1, false>(t, x, mb, o);
    return thermal ? pick_mb<float, 3, true>(t, x, mb, o) : pick_mb<float, 3, false>(t, x, mb, o);
}

template <typename R, int S, int MB> constexpr size_t rec_bytes() { return 16u * TRec<R, S, MB>::STRIDE; }

// ---------------------------------------------------------------------------
// Fused steps of many solves: one round (every solve's sub-step `round`) of
// the tiled march over the concatenation of the solves' tiles.
// ---------------------------------------------------------------------------
TParams make_bparams(const BatchLaunch &b, int round) {
    TParams p;
    memset(&p, 0, sizeof(p));
    p.refill_min = (uint32_t)b.refill_min;
    p.capacity = b.t.capacity;
    p.cmax = b.t.cmax;
    p.max_chunks = b.t.max_chunks;
    p.n_tiles = b.t.max_tiles;
    p.rec = b.t.rec;
    p.idx0 = b.t.idx[0];
    p.idx1 = b.t.idx[1];
    p.side = b.t.side;
    p.cnt = b.t.cnt;
    p.off = b.t.off;
    p.cbase = b.t.cbase;
    p.bsum = b.t.bsum;
    p.ch0 = b.t.chunks[0];
    p.ch1 = b.t.chunks[1];
    p.ctrl = b.t.ctrl;
    p.slots = b.slots;
    p.hd = b.head;
    p.tb = b.table;
    p.tsolve = b.t.tsolve;
    p.first = b.t.first;
    p.round = round;
    p.nblocks = (uint32_t)b.blocks;
    return p;
}

template <typename R, int S, bool TH, int MB, int NA, int NB>
hipError_t run_bround(const BatchLaunch &b, int round) {
    const TParams p = make_bparams(b, round);
    const hipStream_t st = b.stream;
    const dim3 grid(b.blocks), blk(kTBlock);
    hipLaunchKernelGGL(k_bstart, dim3(256), dim3(kMaxBatch), 0, st, p);
    hipLaunchKernelGGL((k_bemit<R, S, MB>), grid, blk, 0, st, p);
    scan_lists<true>(p, b.t.scan_blocks, st, 0);
    hipLaunchKernelGGL(k_tscatter_emit<true>, dim3(8 * b.blocks), blk, 0, st, p);
    int cur = 0;
    const uint32_t fin = (b.finish > 0u && b.finish < b.passes) ? b.finish : b.passes;
    for (uint32_t pass = 0; pass < b.passes; ++pass) {
        if (pass == fin) {
            hipLaunchKernelGGL((k_tmarch<R, S, TH, MB, NA, NB, false, false, true, true>), grid, blk, 0, st, p, cur);
            cur = -1;
            break;
        }
        hipLaunchKernelGGL((k_tmarch<R, S, TH, MB, NA, NB, false, false, true, false>), grid, blk, 0, st, p, cur);
        scan_lists<true>(p, b.t.scan_blocks, st, cur ^ 1);
        hipLaunchKernelGGL(k_tscatter<true>, dim3(8 * b.blocks), blk, 0, st, p, cur);
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_tcheck, dim3(1), dim3(64), 0, st, b.t.ctrl, cur, (StepLedger *)nullptr, b.head, b.table);
    return hipGetLastError();
}

template <typename R, int S, bool TH>
hipError_t bocc(int mb, int *o) {
    if (mb == 1)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            o, reinterpret_cast<const void *>(&k_tmarch<R, S, TH, 1, 0, 0, false, false, true, false>), kTBlock, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        o, reinterpret_cast<const void *>(&k_tmarch<R, S, TH, 8, Layout<S, 8>::NA, Layout<S, 8>::NB, false, false, true, false>),
        kTBlock, 0);
}

template <typename R, int S, bool TH>
hipError_t bround(const BatchLaunch &b, int round) {
    if (b.mb == 1) return run_bround<R, S, TH, 1, 0, 0>(b, round);
    return run_bround<R, S, TH, 8, Layout<S, 8>::NA, Layout<S, 8>::NB>(b, round);
}

}  // namespace

hipError_t launch_batch_tiles(const BatchLaunch &b) {
    const TParams p = make_bparams(b, 0);
    hipLaunchKernelGGL(k_btiles, dim3((b.t.max_tiles + 255) / 256), dim3(256), 0, b.stream, p);
    hipLaunchKernelGGL(k_tzero_u32, dim3(256), dim3(256), 0, b.stream, b.t.cnt, b.t.max_tiles);
    hipLaunchKernelGGL(k_tzero_u32, dim3(1), dim3(64), 0, b.stream, reinterpret_cast<uint32_t *>(b.t.ctrl),
                       (uint32_t)(sizeof(TCtrl) / sizeof(uint32_t)));
    return hipGetLastError();
}

hipError_t launch_batch_march(const BatchLaunch &b, int round) {
    if (b.fp64) {
        if (b.species == 1) return b.thermal ? bround<double, 1, true>(b, round) : bround<double, 1, false>(b, round);
        return b.thermal ? bround<double, 3, true>(b, round) : bround<double, 3, false>(b, round);
    }
    if (b.species == 1) return b.thermal ? bround<float, 1, true>(b, round) : bround<float, 1, false>(b, round);
    return b.thermal ? bround<float, 3, true>(b, round) : bround<float, 3, false>(b, round);
}

hipError_t batch_march_occupancy(int fp64, int species, int thermal, int mb, int *o) {
    if (fp64) {
        if (species == 1) return thermal ? bocc<double, 1, true>(mb, o) : bocc<double, 1, false>(mb, o);
        return thermal ? bocc<double, 3, true>(mb, o) : bocc<double, 3, false>(mb, o);
    }
    if (species == 1) return thermal ? bocc<float, 1, true>(mb, o) : bocc<float, 1, false>(mb, o);
    return thermal ? bocc<float, 3, true>(mb, o) : bocc<float, 3, false>(mb, o);
}

size_t batch_record_bytes(int fp64, int species, int mb) { return tiled_record_bytes(fp64, species, mb); }

size_t tiled_record_bytes(int fp64, int species, int mb) {
    if (fp64) {
        if (mb == 1) return species == 1 ? rec_bytes<double, 1, 1>() : rec_bytes<double, 3, 1>();
        return species == 1 ? rec_bytes<double, 1, 8>() : rec_bytes<double, 3, 8>();
    }
    if (mb == 1) return species == 1 ? rec_bytes<float, 1, 1>() : rec_bytes<float, 3, 1>();
    return species == 1 ? rec_bytes<float, 1, 8>() : rec_bytes<float, 3, 8>();
}

hipError_t launch_tiled_reset(const TiledLaunch &t) {
    hipLaunchKernelGGL(k_tzero_u32, dim3(256), dim3(256), 0, t.m.stream, t.cnt, t.n_tiles);
    hipLaunchKernelGGL(k_tzero_u32, dim3(1), dim3(64), 0, t.m.stream, reinterpret_cast<uint32_t *>(t.ctrl),
                       (uint32_t)(sizeof(TCtrl) / sizeof(uint32_t)));
    return hipGetLastError();
}

hipError_t launch_tiled_slots_zero(const TiledLaunch &t) {
    hipLaunchKernelGGL(k_tslots_zero, dim3((t.m.blocks + 255) / 256), dim3(256), 0, t.m.stream, t.m.slots,
                       t.m.blocks);
    return hipGetLastError();
}

hipError_t launch_tiled_batch(const TiledLaunch &t) {
    return dispatch(&t, Extra{nullptr, nullptr}, t.m.species, t.m.thermal, t.m.fp64, t.m.mb, nullptr);
}

hipError_t launch_tiled_reemit(const TiledLaunch &t, const RecombParams &r) {
    return dispatch(&t, Extra{&r, nullptr}, t.m.species, t.m.thermal, t.m.fp64, t.m.mb, nullptr);
}

hipError_t launch_tiled_background(const TiledLaunch &t, const BackgroundParams &b) {
    return dispatch(&t, Extra{nullptr, &b}, t.m.species, t.m.thermal, t.m.fp64, t.m.mb, nullptr);
}

hipError_t tiled_occupancy(int species, int thermal, int fp64, int mb, int *blocks_per_cu) {
    return dispatch(nullptr, Extra{nullptr, nullptr}, species, thermal, fp64, mb, blocks_per_cu);
}

}  // namespace rtk
