// rt_internal.h -- launch descriptions shared by the host ABI (rt_abi.cpp) and
// the HIP kernels.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtk {

constexpr int kMaxBins = 16;
constexpr int kMarchBlock = 256;          // threads per march block (4 wavefronts)
constexpr int kTabRows = 7;               // rows of the per-bin march table ([rows][bins])
#define RT_TRACE_HDR_DEV 8                // int32 header words of a trace record

struct GridGeom {
    int32_t n[3];        // cells per axis
    int32_t bl;          // log2 of the brick side (0 = natural order)
    int32_t nb[3];       // bricks per axis
    uint32_t ncell_pad;  // slots, >= cells (bricks are padded)
};

// Per-block partial ledger written by the march (one slot per block).
struct LedgerSlot {
    double s[8];                 // (sum, compensation) of emitted, absorbed, escaped, truncated
    unsigned long long c[4];     // crossings, packets, escaped count, truncated count
};

// Ledger of one rt_step, accumulated over its sub-steps on the device.
struct StepLedger {
    double s[8];
    unsigned long long c[4];
    unsigned long long substeps;
    unsigned int nonfinite;
    unsigned int errors;         // an internal consistency check of the march failed
    double d_emit;               // recombination photons emitted (also in s[0])
    unsigned long long d_packets; // recombination packets (also in c[1])
};

struct SourceRec {
    int32_t o[3];        // start point in half-cell units
    uint32_t flags;      // kSrcOctant | (bins with SED > 0) << kSrcMaskShift
};
constexpr uint32_t kSrcOctant = 1u;       // directions folded into the + octant, 1/8 of L
constexpr int kSrcMaskShift = 8;

// Everything one march launch needs (host side, type erased).
struct MarchLaunch {
    GridGeom geo;
    double half_dl;                 // half the cell size [cm]
    int32_t species;                // 1 (pure H) or 3 (H + He)
    int32_t thermal;                // deposit photo-heating too
    int32_t fp64;                   // plain float64 form
    int32_t n_bins;
    int32_t mb;                     // compiled bin capacity (1 or 8)
    int32_t layout;                 // 1: bins 0-2 hydrogen only, 3-4 without HeII (8 bins, H+He)
    const SourceRec *src;
    const double *src_ndot;         // photons / s
    const double *src_sedsum;       // sum of the source's SED row (float64)
    const void *sed;                // [n_src][mb] float (float32 form) or double
    int32_t n_src;
    uint32_t packets;               // packets of this sub-step
    double dt;                      // sub-step length [s]
    uint64_t seed, solve_id, step_index;
    const void *tab;                // [7][mb] of the march precision: cross-sections,
                                    // heat factors, E_j - E_th,HI (see rt_abi.cpp)
    double tau_kill;
    const void *kappa;              // absorbers per slot: R (pure H) or R4
    double *acc;                    // accumulators per slot
    int32_t acc_stride;             // doubles per slot
    unsigned long long *queue;      // packet counter
    LedgerSlot *slots;              // one per block
    int32_t *trace;
    int32_t trace_n, trace_len, trace_stride;
    int32_t chunk;                  // packets claimed per wavefront grab
    int32_t refill_min;
    int32_t blocks;
    hipStream_t stream;
};

struct CellLaunch {
    GridGeom geo;
    int32_t fp64;        // state stored as double
    int32_t species;
    int32_t thermal;
    void *state;         // [7][ncell_pad]: n_H, x_HI, x_HII, x_HeI, x_HeII, x_HeIII, T
    void *kappa;
    double *acc;
    int32_t acc_stride;
    double y_he, cell_cm, dt, redshift;
    int32_t n_chem;
    unsigned long long *queue;
    StepLedger *ledger;
    double *rc;          // [species][ncell_pad] recombination counters; non-null: case-A
                         // rates and counting (recombination re-emission on)
    hipStream_t stream;
};

hipError_t launch_march(const MarchLaunch &m);

// ---------------------------------------------------------------------------
// Tiled march: the grid is cut into tiles of 8^3 cells (the bricks of the
// layout); packets are propagated pass by pass, each pass carrying every live
// packet through one tile, with the deposits of a tile gathered in LDS.
// ---------------------------------------------------------------------------
constexpr int kTileLog2 = 3;
constexpr int kTileCells = 1 << (3 * kTileLog2);
constexpr int kCodes = 27;                // neighbour tiles a packet can move to (and itself)
constexpr uint32_t kSideDead = 0xffffffffu;

struct TChunk {          // a run of one tile's list of packets, marched by one block
    uint32_t tile, start, len, shared;    // shared: the tile has more than one run this pass
};

struct TCtrl {
    uint32_t n_chunks[2];   // runs in chunk table 0 / 1
    uint32_t total[2];      // packets in list 0 / 1
    uint32_t claim;         // next run of the current pass
    uint32_t err;           // a bounds check failed
    uint32_t ndiff;         // recombination packets of the current sub-step
    uint32_t pad;
};

struct TiledLaunch {
    MarchLaunch m;          // physics, sources, accumulators, ledger slots, trace
    uint32_t g0, nbatch;    // packet ids [g0, g0 + nbatch) of the sub-step
    uint32_t capacity;      // packets in flight (records)
    uint32_t cmax;          // packets per run
    uint32_t max_chunks;
    uint32_t n_tiles, scan_blocks;
    uint32_t passes;        // passes launched per batch
    uint32_t park_passes;   // passes (from the first) in which packets may be parked
    uint32_t park_lanes;    // park when at most this many lanes still march (0: never)
    uint32_t finish;        // tile passes before the finishing pass (0: none)
    uint32_t periodic;      // periodic boundaries
    uint32_t dmax;          // periodic: a packet ends once a next-face distance exceeds this
    void *rec;
    uint32_t *idx[2], *side, *cnt, *off, *cbase, *bsum;
    TChunk *chunks[2];
    TCtrl *ctrl;
    StepLedger *ledger;
    // optional timing of every march-kernel launch: event pairs ev[2i], ev[2i+1]
    hipEvent_t *ev;
    int ev_cap;           // pairs available
    int *ev_used;         // pairs recorded so far (host counter)
};

// Inputs of the recombination emission of one sub-step.
struct RecombParams {
    double *rc;            // [species][ncell_pad] recombinations per atom since the last emission
    const double *milne;   // [3][n_t][mb] photon fraction per bin of each ion's ground-state continuum
    const void *state;     // the frozen state ([7][ncell_pad], march precision)
    int32_t n_t;
    int32_t acc_stride;
    double log10_t0, dlog10_t;
    double f_rec;
    double volume;         // cell volume [cm^3]
    double y_he;
    StepLedger *ledger;
};

// Background packets of one batch of a sub-step (packet ids g0.. of the
// sub-step's `packets`; TiledLaunch.nbatch of them).
struct BackgroundParams {
    double ndot;           // photons / s entering through the boundary
    double carried;        // sum of the spectrum row as stored
    const void *sed;       // [mb] photon fraction per bin, march precision
    uint32_t active;       // bins with photons
    uint32_t g0;           // first packet id of the batch
    uint32_t packets;      // background packets of the sub-step
    uint32_t pad;
};

size_t tiled_record_bytes(int fp64, int species, int mb);
hipError_t launch_tiled_background(const TiledLaunch &t, const BackgroundParams &b);
// Recombination emission of the sub-step and the march of its packets (after
// the sub-step's source batches, before the cell update).
hipError_t launch_tiled_reemit(const TiledLaunch &t, const RecombParams &r);
hipError_t launch_tiled_reset(const TiledLaunch &t);
hipError_t launch_tiled_slots_zero(const TiledLaunch &t);
hipError_t launch_tiled_batch(const TiledLaunch &t);
hipError_t tiled_occupancy(int species, int thermal, int fp64, int mb, int *blocks_per_cu);
hipError_t march_occupancy(int species, int thermal, int fp64, int mb, int *blocks_per_cu);

// ---------------------------------------------------------------------------
// Fused steps of many independent solves.  The solves of one call share the
// march instance (precision, species, bins, thermal) and their cell fields in
// bricks of 8^3; every kernel of a fused sub-step reads the solves from one
// device table, so the launch shapes do not depend on the batch and one
// captured graph serves any set of solves; round r of a call is every
// solve's sub-step r.  The march is the tiled one over the concatenation of
// the solves' tiles: global tile id = the solve's first tile + its own tile
// index; a run of a tile belongs to one solve, whose values (grid, absorbers,
// accumulators, per-bin table) the block reads at the start of the run.
// ---------------------------------------------------------------------------
constexpr int kMaxBatch = 256;             // solves per fused call

struct BatchSolve {
    GridGeom geo;
    double half_dl, dt, tau_kill, y_he, cell_cm, redshift;
    uint64_t seed, solve_id, step0;        // step index of the call's first sub-step
    int64_t packets;                       // packets of the call, split over n_sub as rt_step does
    const SourceRec *src;
    const double *src_ndot, *src_sedsum;
    const void *sed, *tab;
    void *state, *kappa;
    double *acc;
    StepLedger *ledger;
    int32_t n_sub, n_src, n_chem, acc_stride;
    uint64_t cell0;                        // first fused cell index of this solve
    uint32_t tile0, n_tiles;               // first fused tile and tiles of this solve
};

struct BatchHead {
    int32_t n;                             // solves in the table
    int32_t pad;
    uint64_t cells;                        // fused cells: the solves' padded slot counts summed
    uint32_t tiles;                        // fused tiles: the solves' tiles summed
    uint32_t pad2;
};

// Packets of sub-step `round` of a solve (zero once its sub-steps are done).
__host__ __device__ inline uint32_t round_packets(const BatchSolve &s, int round) {
    if (round >= s.n_sub) return 0u;
    const int64_t base = s.packets / s.n_sub, extra = s.packets % s.n_sub;
    return (uint32_t)(base + (round < extra ? 1 : 0));
}

// Lists, records and counters of the fused tiled march (in the batch's workspace).
struct BatchTiles {
    void *rec;
    uint32_t *idx[2], *side, *cnt, *off, *cbase, *bsum;
    uint16_t *tsolve;                      // solve of each fused tile
    uint32_t *first;                       // [kMaxBatch + 1] first fused packet id per solve (this round)
    TChunk *chunks[2];
    TCtrl *ctrl;
    uint32_t capacity, max_tiles, max_chunks, cmax, scan_blocks;
};

struct BatchLaunch {
    const BatchHead *head;
    const BatchSolve *table;
    LedgerSlot *slots;                     // [kMaxBatch][blocks] per-block partial ledgers
    unsigned long long *queue;
    int32_t fp64, thermal, species, mb;    // the march instance of the call
    int32_t blocks, refill_min;            // march grid and refill threshold
    int32_t cell_blocks;                   // grid of the cell kernels
    uint32_t passes;                       // march passes per sub-step
    uint32_t finish;                       // tile passes before the finishing pass (0: none)
    BatchTiles t;
    hipStream_t stream;
};

hipError_t launch_batch_begin(const BatchLaunch &b);
hipError_t launch_batch_tiles(const BatchLaunch &b);
hipError_t launch_batch_prep(const BatchLaunch &b, int round);
hipError_t launch_batch_march(const BatchLaunch &b, int round);
hipError_t launch_batch_ledger(const BatchLaunch &b, int round);
hipError_t launch_batch_update(const BatchLaunch &b, int round);
hipError_t launch_batch_gather(const BatchLaunch &b, StepLedger *out);   // every solve's ledger, table order
hipError_t batch_march_occupancy(int fp64, int species, int thermal, int mb, int *blocks_per_cu);
size_t batch_record_bytes(int fp64, int species, int mb);

hipError_t launch_prep(const CellLaunch &c);
hipError_t launch_update(const CellLaunch &c);
hipError_t launch_import(const CellLaunch &c, const void *nh, const void *x, const void *t,
                         int fields_fp64, int64_t ncell);
hipError_t launch_export(const CellLaunch &c, uint32_t mask, void *dst, int as_fp64, int64_t ncell);
// Counters c.rc ([species][ncell_pad]) from natural order [species][ncell]; src null: zero.
hipError_t launch_import_counters(const CellLaunch &c, const void *src, int src_fp64, int64_t ncell);
hipError_t launch_ledger_zero(StepLedger *l, hipStream_t s);
hipError_t launch_ledger_reduce(const LedgerSlot *slots, int nslots, StepLedger *l, hipStream_t s);
hipError_t launch_trace_rays(const GridGeom &g, int m, const int32_t *o, const int32_t *c,
                             int max_len, int32_t *cells, int32_t *count, int32_t *face,
                             hipStream_t s);

}  // namespace rtk
