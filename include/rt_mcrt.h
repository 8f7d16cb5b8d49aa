/*
 * rt_mcrt.h -- C ABI of the MI355X Monte-Carlo radiative-transfer hot path.
 *
 * Method (Partl et al. 2011, "Enabling parallel computing in CRASH", Sec. 2):
 * point sources emit coloured photon packets in random directions; each packet
 * is followed cell by cell through a Cartesian grid, its optical depth in every
 * crossed cell summed over HI, HeI and HeII, the absorbed photons per frequency
 * bin given by Eq. (1) and shared among the absorbers in proportion to their
 * optical depth; the ionisation fractions and temperature of the cells are then
 * advanced from the absorbed photons.  Here the cell state is frozen while the
 * packets of one sub-step fly and every cell is updated once per sub-step.
 *
 * Conventions shared by every call:
 *  - Cells are addressed (i, j, k), 0 <= i < n[0] etc.; the natural linear
 *    index is i + n[0] * (j + n[1] * k).  Every field passed in or out uses
 *    natural order.  Inside the library the fields live in a brick layout.
 *  - Units are cgs: cm, cm^-3, s, K, erg; photon energies in eV.
 *  - Device pointers are plain HIP device addresses owned by the caller.  The
 *    library never allocates device memory: all of its state lives in the
 *    caller-provided workspace, which must outlive the handle.
 *  - Host pointers are read (or written) during the call only.
 *  - Every call returns RT_OK (0) or a negative status; nothing is thrown.  A
 *    failed call that returns RT_EINVAL or RT_ENOMEM leaves the handle as it
 *    was.  After RT_EDEVICE the handle only accepts rt_release.
 *  - Calls on one handle must not overlap; different handles are independent.
 */
#ifndef RT_MCRT_H
#define RT_MCRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_MAX_BINS 16
#define RT_SUPPORTED_BINS 8
#define RT_MAX_CELLS_PER_AXIS 1024

/* status codes */
#define RT_OK 0
#define RT_EINVAL (-1)      /* invalid argument; nothing changed */
#define RT_ENOMEM (-2)      /* workspace too small, or too many sources */
#define RT_EDEVICE (-3)     /* HIP error; the handle is unusable */
#define RT_ESTATE (-4)      /* call not valid in the handle's state */
#define RT_EOVERFLOW (-5)   /* a size exceeds what the library supports */
#define RT_EINTERNAL (-6)   /* an internal consistency check of the march failed;
                               the handle only accepts rt_release */
#define RT_ESCRATCH (-7)    /* rt_init_grid_static: the solve needs more than
                               RT_STATIC_WORKSPACE_BYTES; nothing changed */

/* Size of the library's static per-device workspace (rt_init_grid_static). */
#define RT_STATIC_WORKSPACE_BYTES (64u << 20)

/* rt_grid_desc.flags */
#define RT_ISOTHERMAL 0x1u  /* temperature held fixed */
#define RT_FP64 0x2u        /* plain form: march, absorber table and stored state
                               in float64 (default: float32 march and state,
                               float64 accumulators and float64 cell update) */
#define RT_TIME_MARCH 0x4u  /* time the march of every sub-step with HIP events
                               on the handle's stream (rt_step_stats.march_ms) */
#define RT_DIRECT_MARCH 0x8u /* per-packet march: every wavefront lane follows
                               one packet from emission to its end and adds its
                               deposits to the grid with float64 atomics.
                               Default: the tiled march (tiles of 8^3 cells,
                               deposits gathered per tile in on-chip memory,
                               packets handed between tiles pass by pass).
                               Both give the same packet histories. */
#define RT_RECOMB 0x10u     /* recombination re-emission (Sec. 2; Sec. 3, pCRASH2):
                               case-A recombination in the cell update, which
                               also counts each cell's recombinations per atom
                               of HII, HeII and HeIII; in every sub-step, after
                               the source packets, each cell they deposited in
                               whose counters have reached the threshold emits
                               one packet of ground-state recombination photons
                               (Milne spectrum), marched before the update.
                               Needs rt_set_recombination before rt_step; not
                               with RT_DIRECT_MARCH.  The workspace then holds
                               one packet record per cell at least. */
#define RT_PERIODIC 0x20u   /* periodic boundaries (Sec. 2): a packet leaving
                               through a face re-enters through the opposite
                               one; it ends when extinguished or once it has
                               crossed more than path_cells cell faces along
                               one axis (its photons then count as escaped).
                               Tiled march only. */

/* rt_add_sources src_flags */
#define RT_SRC_CORNER_OCTANT 0x1u /* source at the lowest corner of its cell,
                                     directions folded into the + octant; the
                                     box receives 1/8 of its luminosity */

/* rt_fetch_fields masks (fields are written in this bit order) */
#define RT_F_NH 0x001u     /* hydrogen number density */
#define RT_F_XHI 0x002u    /* ionisation fractions */
#define RT_F_XHII 0x004u
#define RT_F_XHEI 0x008u
#define RT_F_XHEII 0x010u
#define RT_F_XHEIII 0x020u
#define RT_F_T 0x040u      /* temperature */
#define RT_F_DHI 0x080u    /* photons absorbed by HI in the last sub-step */
#define RT_F_DHEI 0x100u   /* ... by HeI */
#define RT_F_DHEII 0x200u  /* ... by HeII */
#define RT_F_Q 0x400u      /* photo-heating energy [erg] of the last sub-step */
#define RT_F_RHII 0x800u   /* RT_RECOMB: HII recombinations per H atom since the
                              cell last emitted (0 without RT_RECOMB) */
#define RT_F_RHEII 0x1000u /* ... HeII recombinations per He atom */
#define RT_F_RHEIII 0x2000u /* ... HeIII recombinations per He atom */
#define RT_F_ALL 0x3fffu

#define RT_MAX_MILNE_T 512  /* temperature nodes of a recombination spectrum table */
#define RT_MAX_PATH_CELLS 2046 /* largest rt_grid_desc.path_cells */
#define RT_MAX_FINISH_PASS 65535 /* largest rt_grid_desc.finish_pass */

/* trace record: RT_TRACE_HDR int32 words then trace_len cell indices */
#define RT_TRACE_HDR 8
#define RT_FATE_TRUNC 1     /* extinguished: every populated bin reached tau_kill */
#define RT_FATE_ESCAPE 2    /* left the grid (non-periodic boundaries) */
#define RT_FATE_PATH 3      /* periodic: reached the path limit */

typedef struct rt_solve *rt_solve_t;

/* Problem statement of one solve (Sec. 2: a static H/He density on a Cartesian
 * grid, photon packets with N_nu frequency bins, per-species cross-sections). */
typedef struct {
    int32_t n[3];                 /* cells per axis, 1..RT_MAX_CELLS_PER_AXIS */
    double cell_cm;               /* proper cell size */
    double y_he;                  /* n_He / n_H ; 0 = pure hydrogen */
    int32_t n_bins;               /* frequency bins: 1 or RT_SUPPORTED_BINS (arrays
                                     hold RT_MAX_BINS; other counts -> RT_EINVAL).
                                     H+He with 8 bins: the table must be
                                     threshold-aligned (HeI and HeII cross-sections
                                     0 in bins 0-2, HeII 0 in bins 3-4), else
                                     RT_EINVAL, in either march */
    double e_bin_ev[RT_MAX_BINS]; /* photon energy of each bin (heat per absorption
                                     is E_j minus the species' threshold) */
    double sigma_cm2[3][RT_MAX_BINS]; /* HI, HeI, HeII cross-sections per bin;
                                     must be 0 where E_j is below the threshold */
    double redshift;              /* Compton exchange with T_cmb = 2.725 (1+z);
                                     < 0 disables it */
    double tau_kill;              /* a packet ends once every bin it carries has
                                     accumulated optical depth >= tau_kill */
    int32_t n_sub;                /* frozen sub-steps per rt_step */
    int32_t n_chem;               /* fixed chemistry sub-steps per frozen sub-step */
    uint32_t flags;               /* RT_ISOTHERMAL | RT_FP64 */
    uint64_t solve_id;            /* second word of the Philox key */
    uint64_t step_index0;         /* Philox sub-step counter to start from (resume) */
    int32_t brick_log2;           /* brick side 2^b, b in 0..3 (0 = natural order); -1 = default.
                                     The tiled march needs b = 3 (or -1). */
    int32_t wave_chunk;           /* per-packet march: packets a wavefront claims
                                     at a time; 0 = default */
    int32_t refill_min;           /* dead lanes a wavefront gathers before it
                                     refills them; 0 = default */
    int32_t blocks_per_cu;        /* persistent march blocks per compute unit; 0 = default */
    int32_t trace_packets;        /* number of traced packets per sub-step (0 = off):
                                     ids g = r * trace_stride, r < trace_packets,
                                     go to trace record r */
    int32_t trace_len;            /* cells recorded per traced packet */
    int32_t trace_stride;         /* spacing of traced packet ids; 0 = 1 */
    int32_t run_len;              /* tiled march: packets of one tile one block
                                     marches before it writes the tile's deposits
                                     out; 0 = default (4096; 2048 in
                                     rt_step_many), else 64..65536 */
    int32_t park_lanes;           /* tiled march: once a run of a tile is used up,
                                     a wavefront with at most this many packets
                                     still marching writes them back; they resume
                                     in the same tile in the next pass (their
                                     histories do not change).  0..64; 0 = never
                                     (default: march them to the tile's edge) */
    int64_t inflight;             /* tiled march: packets propagated together (the
                                     workspace holds one record each); a sub-step
                                     with more packets runs in batches of this
                                     size.  0 = default (2^24) */
    int32_t path_cells;           /* RT_PERIODIC: cell faces a packet may cross along
                                     one axis, 1..RT_MAX_PATH_CELLS; 0 = the longest
                                     side of the grid */
    int32_t finish_pass;          /* tiled march: tile passes after which one
                                     finishing pass marches every packet still in
                                     flight to its end, reading the grid's
                                     absorbers and adding to its accumulators
                                     directly (float64 atomics); the histories do
                                     not change.  0 = default (never), -1 = never,
                                     else 1..RT_MAX_FINISH_PASS; not used while
                                     tracing */
} rt_grid_desc;

/* Photon ledger and counters of the most recent rt_step (all its sub-steps). */
typedef struct {
    double emitted;     /* photons emitted into the box */
    double absorbed;    /* photons absorbed in cells */
    double escaped;     /* photons that left the grid */
    double truncated;   /* photons still carried by extinguished packets */
    int64_t crossings;  /* (packet, cell) pairs with positive path length */
    int64_t packets;
    int64_t n_escaped;
    int64_t n_truncated;
    int64_t substeps;
    uint32_t nonfinite; /* nonzero if the cell update produced a non-finite value */
    uint32_t errors;    /* nonzero if a consistency check of the march failed
                           (rt_read_stats then returns RT_EINTERNAL) */
    double march_ms;    /* RT_TIME_MARCH: time of the whole march of every sub-step
                           (tiled march: emission, passes, sorts), else 0 */
    double kernel_ms;   /* RT_TIME_MARCH: summed time of the march kernel's own
                           launches (tiled march: one per pass), else 0 */
    int64_t kernel_launches; /* launches timed in kernel_ms */
    double diffuse_emitted; /* RT_RECOMB: recombination photons emitted (part of
                               emitted), else 0 */
    int64_t diffuse_packets; /* RT_RECOMB: recombination packets (part of packets) */
} rt_step_stats;

/* Fill *d with defaults: 1 bin, tau_kill 30, n_sub 1, n_chem 8, redshift -1,
 * tiles chosen by the library, tracing off.  Returns RT_OK or RT_EINVAL. */
int32_t rt_desc_defaults(rt_grid_desc *d);

/* Workspace bytes a solve with this description and at most max_sources
 * sources needs.  Returns RT_EINVAL for an invalid description (including a
 * bin count other than 1 or 8, and an H+He table of 8 bins that the tiled
 * march has no instance for). */
int32_t rt_workspace_bytes(const rt_grid_desc *d, int64_t max_sources, size_t *bytes_out);

/* Create a solve in the caller's device workspace and load its initial state.
 *   d_ws, ws_bytes : device workspace (>= rt_workspace_bytes), 256-byte aligned
 *   d_nh           : [ncell] hydrogen density, > 0
 *   d_x            : [5][ncell] x_HI, x_HII, x_HeI, x_HeII, x_HeIII
 *   d_temp         : [ncell] temperature
 *   fields_fp64    : 1 if the three arrays are float64, 0 if float32
 *   hip_stream     : hipStream_t every call of this handle is ordered on (NULL = default)
 * Sources are added with rt_add_sources.  Stream-ordered; returns after the
 * copies are enqueued. */
int32_t rt_init_grid(const rt_grid_desc *d, void *d_ws, size_t ws_bytes, int64_t max_sources,
                     const void *d_nh, const void *d_x, const void *d_temp, int32_t fields_fp64,
                     void *hip_stream, rt_solve_t *out);

/* rt_init_grid for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same solve, with its workspace in a static array of the library
 * (RT_STATIC_WORKSPACE_BYTES on each device it runs on, held until the
 * process ends) instead of a caller's buffer.  Arguments as rt_init_grid
 * without d_ws / ws_bytes; the description may not ask for RT_TIME_MARCH.
 * Allocates nothing: no hipMalloc, no host heap.
 *   RT_ESCRATCH  the solve's workspace (rt_workspace_bytes) exceeds
 *                RT_STATIC_WORKSPACE_BYTES; nothing changed
 *   RT_ESTATE    a static solve on the current device has not been released
 * One static solve per device at a time: it shares the device's array with
 * every other call (the array keeps the last solve's contents; the call
 * re-initialises all of it that a solve reads).  Calls that overlap on one
 * device race.  rt_release frees the slot for the next static solve. */
int32_t rt_init_grid_static(const rt_grid_desc *d, int64_t max_sources, const void *d_nh, const void *d_x,
                            const void *d_temp, int32_t fields_fp64, void *hip_stream, rt_solve_t *out);

/* Append n point sources (Sec. 2: position, luminosity L_s in photons/s, SED
 * over the bins by photon number).  Host arrays:
 *   h_ijk [3n] cell of each source, h_ndot [n] photons/s (>= 0, finite),
 *   h_sed [n * n_bins] photon fraction per bin (>= 0, row sum > 0).
 * Returns RT_ENOMEM beyond max_sources.  Synchronous. */
int32_t rt_add_sources(rt_solve_t h, int32_t n, const int32_t *h_ijk, const double *h_ndot,
                       const double *h_sed, uint32_t src_flags);

/* Advance the solve by dt_s: n_sub frozen sub-steps of dt_s / n_sub, the
 * n_packets shared evenly among the sub-steps and, within a sub-step, equally
 * among the sources (the first P mod S sources get one more; Sec. 3.2: N_p/N_t
 * packets per source per step).  Each sub-step: absorber densities from the
 * frozen state, the packet march with deposition, then the cell update.
 * Every sub-step must give each source at least one packet (else RT_EINVAL);
 * a solve without sources runs the cell update only.  Stream-ordered and
 * asynchronous; if stats is not NULL the call synchronises and fills it. */
int32_t rt_step(rt_solve_t h, double dt_s, int64_t n_packets, uint64_t seed, rt_step_stats *stats);

/* Recombination re-emission inputs of a solve created with RT_RECOMB (Sec. 2:
 * a cell emits once its recombinations reach f_rec N_a; Sec. 3: on a crossing).
 *   f_rec        threshold in recombinations per atom (>= 0; a counter must
 *                also be positive to emit)
 *   n_t, log10_t0, dlog10_t
 *                temperature nodes of the spectrum table: node k at
 *                log10 T = log10_t0 + k dlog10_t, 2 <= n_t <= RT_MAX_MILNE_T;
 *                the spectrum at T is linear in log10 T between nodes, clamped
 *                to the end nodes
 *   h_milne      host [3][n_t][n_bins]: photon fraction per bin of the ground-
 *                state recombination continuum of HII, HeII, HeIII (each row
 *                >= 0, summing to 1; zero in bins below the ion's threshold)
 *   d_counters   device [species][ncell] initial counters in natural order
 *                (species 1 for pure hydrogen, else 3), float64 or float32 per
 *                counters_fp64; NULL: all zero
 * Each photon packet from a cell carries, for every ion whose counter is
 * positive and >= f_rec, counter x atoms x (alpha_A - alpha_B)/alpha_A photons
 * with that ion's spectrum at the cell temperature; those counters restart at
 * zero.  Its direction is isotropic (Philox stream word 1, counter word 0 the
 * cell's natural index) from the cell centre.  Returns RT_ESTATE for a solve
 * created without RT_RECOMB.  Synchronous. */
int32_t rt_set_recombination(rt_solve_t h, double f_rec, int32_t n_t, double log10_t0, double dlog10_t,
                             const double *h_milne, const void *d_counters, int32_t counters_fp64);

/* Background field of a solve (Sec. 2: packets from diffuse fields such as the
 * UV background), an isotropic intensity entering the box through its faces.
 *   ndot              photons per second through the whole boundary (for an
 *                     intensity J in photons/s/cm^2/sr: pi J times the area)
 *   h_sed             host [n_bins] photon fraction per bin (>= 0, sum > 0)
 *   packets_per_step  background packets per rt_step, shared over the
 *                     sub-steps like source packets; 0 switches the field off
 * In each sub-step, after the source packets, packet g starts at the centre of
 * a boundary cell face chosen uniformly over the boundary (Philox counter
 * (g, sub-step, 0, 2)), moves in the isotropic direction of stream word 3
 * turned inward, and carries (ndot dt_sub / P) 2 cos(theta) photons per unit
 * of the spectrum.  Tiled march only (else RT_ESTATE); solves with a
 * background do not enter rt_step_many.  Synchronous. */
int32_t rt_set_background(rt_solve_t h, double ndot, const double *h_sed, int64_t packets_per_step);

/* Synchronise the handle's stream and return the ledger of the last rt_step. */
int32_t rt_read_stats(rt_solve_t h, rt_step_stats *stats);

/* Copy the fields selected by mask, in bit order, each as ncell values in
 * natural order, into dst (device or host memory; float64 if as_fp64 else
 * float32).  Deposits are those of the last sub-step.  Synchronises. */
int32_t rt_fetch_fields(rt_solve_t h, uint32_t mask, void *dst, int32_t dst_is_device,
                        int32_t as_fp64);

/* Copy count trace records (RT_TRACE_HDR + trace_len int32 each: crossings,
 * fate, exit face, last cell, c[3], source, cells...) of the last sub-step to
 * host memory; cell slots past a record's crossing count are unspecified.
 * Synchronises. */
int32_t rt_fetch_trace(rt_solve_t h, int32_t *h_dst, int64_t count);

/* Cells crossed by m rays through the handle's grid, with the same traversal
 * the march uses.  Device arrays: d_origin [3m] start points in half-cell units
 * (inside or on the boundary), d_dir [3m] integer directions (|c_a| <= 2^20, not
 * all zero), d_cells [m * max_len] natural indices, d_count [m] cells crossed
 * (may exceed max_len), d_face [m] exit face (bit a: left through axis a,
 * bit 3+a: through its + side).  Stream-ordered. */
int32_t rt_trace_rays(rt_solve_t h, int32_t m, const int32_t *d_origin, const int32_t *d_dir,
                      int32_t max_len, int32_t *d_cells, int32_t *d_count, int32_t *d_face);

/* Current Philox sub-step counter (for checkpoint and resume). */
int32_t rt_get_step_index(rt_solve_t h, uint64_t *out);

/* Synchronise and destroy the handle (the workspace may then be freed). */
int32_t rt_release(rt_solve_t h);

/* ---- Fused steps of many independent solves (serving) ----
 * rt_step_many advances n solves by one rt_step each, with the same operation
 * per solve as rt_step (Sec. 2 march and cell update; Sec. 3.2 packet shares)
 * and the same packet ids, Philox counters and crossing arithmetic, so every
 * solve's result is the one rt_step gives alone, up to the order in which
 * float64 deposits are added.  Per sub-step the solves share one tiled march
 * over the concatenation of their tiles (each pass carries every live packet
 * of every solve through one tile, a tile's deposits gathered on chip; the
 * paper's subdomains, Sec. 3.2, here the 8^3 tiles of many grids), plus one
 * launch each for the absorbers, the ledgers and the cell update; with
 * RT_BATCH_GRAPH the whole call is captured once per (sub-step count, march
 * passes) as a hipGraph and replayed (the launches read the solves from a
 * device table, so the graph does not depend on which solves are in it).
 *
 * A batch is created for one march instance, given by a shape description
 * (rt_grid_desc: RT_FP64, RT_ISOTHERMAL, y_he > 0, n_bins; run_len,
 * refill_min and blocks_per_cu tune its march).  Solves of a call must match
 * it (precision, species, bins, thermal), keep their fields in bricks of 8^3
 * (the tiled march, or the per-packet march with brick_log2 = 3), and have no
 * tracing, periodic boundaries, recombination re-emission or background
 * field; they sit on the batch's device, each at most once.  Their own streams
 * are ordered around the call with events, so rt_fetch_fields and rt_read_stats
 * on a solve see its result. */
typedef struct rt_batch *rt_batch_t;

#define RT_MAX_BATCH 256     /* solves per rt_step_many */
#define RT_BATCH_GRAPH 0x1u  /* capture each call shape (sub-step count, march
                                passes) once as a hipGraph and replay it */

/* Device workspace bytes of a batch of at most max_solves (1..RT_MAX_BATCH)
 * solves of the given shape: the solve table, per-(solve, block) ledger
 * slots, and the tiled march's records and lists for max_round_packets
 * packets of one sub-step of all solves together and max_tiles tiles of 8^3
 * cells of all solves together.  RT_EINVAL for an invalid shape or size. */
int32_t rt_batch_workspace_bytes(int32_t max_solves, const rt_grid_desc *shape, int64_t max_round_packets,
                                 int64_t max_tiles, size_t *bytes_out);

/* Create a batch in the caller's device workspace (256-byte aligned, at least
 * rt_batch_workspace_bytes for the same arguments).  hip_stream: the stream
 * the fused launches go to; it must not be NULL with RT_BATCH_GRAPH (the
 * legacy stream cannot be captured).  Allocates pinned host memory for the
 * table it stages. */
int32_t rt_batch_init(int32_t max_solves, const rt_grid_desc *shape, int64_t max_round_packets, int64_t max_tiles,
                      void *d_ws, size_t ws_bytes, void *hip_stream, uint32_t flags, rt_batch_t *out);

/* Advance solves[0..n) by one step each: solve i by dt_s[i] with n_packets[i]
 * packets and Philox seed seeds[i], exactly as rt_step(solves[i], ...) would
 * (its n_sub sub-steps; the call runs max n_sub fused rounds).  Returns
 * RT_EINVAL (nothing enqueued) if a solve breaks the rules above or a step
 * argument would be rejected by rt_step, RT_ENOMEM if the solves' tiles or one
 * round's packets exceed the batch's.  Stream-ordered: the host may go on
 * (open the next solves, say) while the call runs; a solve's own stream is
 * ordered after the call when the solve is next used (by its own calls or by
 * a call of another batch).  If stats is not NULL
 * (n entries) the call waits for itself and fills each solve's ledger, as
 * rt_batch_wait does. */
int32_t rt_step_many(rt_batch_t b, const rt_solve_t *solves, int32_t n, const double *dt_s,
                     const int64_t *n_packets, const uint64_t *seeds, rt_step_stats *stats);

/* Wait for the batch's last rt_step_many call and fill the ledgers of its n
 * solves (n: the call's solve count; stats[i] for its solves[i]; march_ms and
 * kernel_ms are 0).  RT_EINVAL if n differs from the call's count; RT_EINTERNAL
 * if a solve's consistency check failed (that solve is then unusable, as
 * after rt_read_stats).  The call's solves must not be released before. */
int32_t rt_batch_wait(rt_batch_t b, int32_t n, rt_step_stats *stats);

/* Synchronise the batch's stream, destroy its graphs and events and free its
 * pinned staging memory (the workspace may then be freed). */
int32_t rt_batch_release(rt_batch_t b);

/* Static description of a status code. */
const char *rt_strerror(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* RT_MCRT_H */
