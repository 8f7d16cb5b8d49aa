// rt_abi.cpp -- host side of the C ABI declared in include/rt_mcrt.h: argument
// validation, workspace layout, and the order of kernels in a step
// (absorbers -> march -> ledger -> cell update, once per frozen sub-step).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "rt_internal.h"
#include "rt_mcrt.h"

namespace {

constexpr uint64_t kMagic = 0x52544d4352543031ull;   // handle tag
constexpr int kMaxMarchBlocks = 8192;                // ledger slots reserved in the workspace
constexpr size_t kAlign = 256;
const double kThresholdEv[3] = {13.598434, 24.587387, 54.417760};
const double kEvErg = 1.602176634e-12;
const double kLog2e = 1.4426950408889634;            // log2(e)

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

constexpr int kMaxSupportedBins = 8;   // widest compiled march instance

int bin_capacity(int n_bins) { return n_bins <= 1 ? 1 : 8; }

constexpr int64_t kDefaultInflight = (int64_t)1 << 24;   // packets in flight in the tiled march
constexpr int kDefaultRun = 4096;                         // packets per tile run (single solve)
constexpr int kDefaultBatchRun = 2048;                    // packets per tile run (fused steps)
constexpr int kMaxRunLen = 1 << 16;                       // longest run a description may ask for

struct Plan {
    int species, thermal, fp64, mb, acc_stride, bl;
    bool tiled;
    rtk::GridGeom geo;
    int64_t ncell;
    size_t real;
    size_t off_state, off_kappa, off_acc, off_src, off_ndot, off_sedsum, off_sed, off_tab, off_slots,
        off_ledger, off_queue, off_trace, off_stage, total;
    bool recomb;            // recombination photons re-emitted as packets
    size_t off_rc, off_milne;
    size_t off_bg;          // background spectrum row
    // tiled march
    uint32_t capacity, cmax, max_chunks, n_tiles, scan_blocks, passes, park_passes, park_lanes;
    uint32_t finish;        // tile passes before the finishing pass (0: none)
    uint32_t periodic, dmax;
    size_t rec_bytes;
    size_t off_rec, off_idx0, off_idx1, off_side, off_cnt, off_off, off_cbase, off_bsum, off_ch0, off_ch1,
        off_ctrl;
};

bool finite_nonneg(double v) { return isfinite(v) && v >= 0.0; }

int32_t validate_desc(const rt_grid_desc *d) {
    if (!d) return RT_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (d->n[a] < 1 || d->n[a] > RT_MAX_CELLS_PER_AXIS) return RT_EINVAL;
    if (!(isfinite(d->cell_cm) && d->cell_cm > 0.0)) return RT_EINVAL;
    if (!finite_nonneg(d->y_he)) return RT_EINVAL;
    // one bin or the full eight: the eight-wide instances are the only
    // multi-bin ones run against the oracle (counts in between are refused)
    if (d->n_bins != 1 && d->n_bins != kMaxSupportedBins) return RT_EINVAL;
    for (int j = 0; j < d->n_bins; ++j) {
        if (!finite_nonneg(d->e_bin_ev[j])) return RT_EINVAL;
        for (int s = 0; s < 3; ++s) {
            if (!finite_nonneg(d->sigma_cm2[s][j])) return RT_EINVAL;
            if (d->sigma_cm2[s][j] > 0.0 && d->e_bin_ev[j] < kThresholdEv[s]) return RT_EINVAL;
        }
    }
    if (!isfinite(d->redshift)) return RT_EINVAL;
    if (!(isfinite(d->tau_kill) && d->tau_kill > 0.0)) return RT_EINVAL;
    if (d->n_sub < 1 || d->n_chem < 1) return RT_EINVAL;
    if (d->flags & ~(RT_ISOTHERMAL | RT_FP64 | RT_TIME_MARCH | RT_DIRECT_MARCH | RT_RECOMB | RT_PERIODIC))
        return RT_EINVAL;
    // periodic boundaries are marched by the tiled march only
    if ((d->flags & RT_PERIODIC) && (d->flags & RT_DIRECT_MARCH)) return RT_EINVAL;
    if (d->path_cells < 0 || d->path_cells > RT_MAX_PATH_CELLS) return RT_EINVAL;
    if (d->finish_pass < -1 || d->finish_pass > RT_MAX_FINISH_PASS) return RT_EINVAL;
    // recombination packets are marched by the tiled march only
    if ((d->flags & RT_RECOMB) && (d->flags & RT_DIRECT_MARCH)) return RT_EINVAL;
    if (d->brick_log2 < -1 || d->brick_log2 > 3) return RT_EINVAL;
    // the tiled march's tiles are the bricks of side 8
    if (!(d->flags & RT_DIRECT_MARCH) && d->brick_log2 != -1 && d->brick_log2 != 3) return RT_EINVAL;
    if (d->run_len < 0 || d->run_len > kMaxRunLen || (d->run_len > 0 && d->run_len < 64)) return RT_EINVAL;
    if (d->inflight < 0 || d->inflight > ((int64_t)1 << 31) - 1) return RT_EINVAL;
    if (d->park_lanes < 0 || d->park_lanes > 64) return RT_EINVAL;
    if (d->wave_chunk < 0 || d->wave_chunk % 64 != 0 || d->wave_chunk > (1 << 20)) return RT_EINVAL;
    if (d->refill_min < 0 || d->refill_min > 64) return RT_EINVAL;
    if (d->blocks_per_cu < 0 || d->blocks_per_cu > 32) return RT_EINVAL;
    if (d->trace_packets < 0 || d->trace_len < 0) return RT_EINVAL;
    if (d->trace_packets > 0 && d->trace_len < 1) return RT_EINVAL;
    if (d->trace_stride < 0) return RT_EINVAL;
    return RT_OK;
}

int32_t make_plan(const rt_grid_desc *d, int64_t max_sources, Plan *p) {
    const int32_t v = validate_desc(d);
    if (v != RT_OK) return v;
    *p = Plan{};
    if (max_sources < 0 || max_sources > (int64_t)1 << 30) return RT_EINVAL;
    p->species = d->y_he > 0.0 ? 3 : 1;
    // H+He tables of several bins: the threshold-aligned layout only (helium
    // cross-sections zero in bins 0-2, HeII zero in bins 3-4), the one both
    // marches have a tested instance for; the generic instance stays unused
    // while the fault of an earlier generic-layout instance is unexplained
    if (p->species == 3 && d->n_bins > 1) {
        for (int j = 0; j < 5; ++j)
            if (d->sigma_cm2[2][j] != 0.0 || (j < 3 && d->sigma_cm2[1][j] != 0.0)) return RT_EINVAL;
    }
    p->thermal = (d->flags & RT_ISOTHERMAL) ? 0 : 1;
    p->fp64 = (d->flags & RT_FP64) ? 1 : 0;
    p->mb = bin_capacity(d->n_bins);
    p->acc_stride = p->species == 1 ? (p->thermal ? 2 : 1) : 4;
    p->tiled = !(d->flags & RT_DIRECT_MARCH);
    p->bl = p->tiled ? 3 : (d->brick_log2 < 0 ? 1 : d->brick_log2);
    rtk::GridGeom &g = p->geo;
    uint64_t np = 1;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = d->n[a];
        g.nb[a] = (d->n[a] + (1 << p->bl) - 1) >> p->bl;
        np *= (uint64_t)g.nb[a] << p->bl;
    }
    g.bl = p->bl;
    if (p->bl == 0) np = (uint64_t)d->n[0] * d->n[1] * d->n[2];
    if (np >= (1ull << 32)) return RT_EOVERFLOW;
    g.ncell_pad = (uint32_t)np;
    p->ncell = (int64_t)d->n[0] * d->n[1] * d->n[2];
    p->real = p->fp64 ? sizeof(double) : sizeof(float);
    const size_t kap_vec = p->species == 1 ? 1 : 4;
    size_t o = 0;
    p->off_state = o; o = align_up(o + 7 * np * p->real);
    p->off_kappa = o; o = align_up(o + kap_vec * np * p->real);
    p->off_acc = o; o = align_up(o + (size_t)p->acc_stride * np * sizeof(double));
    const size_t ms = (size_t)(max_sources > 0 ? max_sources : 1);
    p->off_src = o; o = align_up(o + ms * sizeof(rtk::SourceRec));
    p->off_ndot = o; o = align_up(o + ms * sizeof(double));
    p->off_sedsum = o; o = align_up(o + ms * sizeof(double));
    p->off_sed = o; o = align_up(o + ms * p->mb * p->real);
    p->off_tab = o; o = align_up(o + rtk::kTabRows * (size_t)p->mb * p->real);
    p->off_slots = o; o = align_up(o + kMaxMarchBlocks * sizeof(rtk::LedgerSlot));
    p->off_ledger = o; o = align_up(o + sizeof(rtk::StepLedger));
    p->off_queue = o; o = align_up(o + sizeof(unsigned long long));
    p->off_trace = o;
    o = align_up(o + (size_t)d->trace_packets * (RT_TRACE_HDR + (size_t)d->trace_len) * sizeof(int32_t));
    p->off_stage = o; o = align_up(o + (size_t)p->ncell * sizeof(double));
    p->off_bg = o; o = align_up(o + (size_t)p->mb * p->real);
    p->recomb = (d->flags & RT_RECOMB) != 0;
    p->off_rc = p->off_milne = 0;
    if (p->recomb) {
        p->off_rc = o; o = align_up(o + (size_t)p->species * np * sizeof(double));
        p->off_milne = o; o = align_up(o + 3 * (size_t)RT_MAX_MILNE_T * p->mb * sizeof(double));
    }
    p->capacity = p->cmax = p->max_chunks = p->n_tiles = p->scan_blocks = p->passes = 0;
    p->park_passes = p->park_lanes = 0;
    p->finish = 0;
    p->periodic = p->dmax = 0;
    p->rec_bytes = 0;
    p->off_rec = p->off_idx0 = p->off_idx1 = p->off_side = p->off_cnt = p->off_off = p->off_cbase = p->off_bsum =
        p->off_ch0 = p->off_ch1 = p->off_ctrl = 0;
    if (p->tiled) {
        uint64_t cap = (uint64_t)(d->inflight > 0 ? d->inflight : kDefaultInflight);
        // a sub-step's recombination packets (at most one per cell) form one batch
        if (p->recomb && cap < (uint64_t)p->ncell) cap = (uint64_t)p->ncell;
        const uint64_t nt = (uint64_t)g.nb[0] * g.nb[1] * g.nb[2];
        p->capacity = (uint32_t)cap;
        p->cmax = (uint32_t)(d->run_len > 0 ? d->run_len : kDefaultRun);
        const uint64_t mc = nt + cap / p->cmax + 1;
        if (mc >= (1ull << 31)) return RT_EOVERFLOW;
        p->max_chunks = (uint32_t)mc;
        p->n_tiles = (uint32_t)nt;
        p->scan_blocks = (uint32_t)((nt + 4095) / 4096);
        // a packet visits at most tx + ty + tz - 2 tiles.  Parking is allowed in
        // that many passes and the same number follow without it, so a packet
        // parked in the last parking pass still reaches the end of its path.
        uint32_t visits = (uint32_t)(g.nb[0] + g.nb[1] + g.nb[2] - 2);
        p->periodic = (d->flags & RT_PERIODIC) ? 1u : 0u;
        p->dmax = 0;
        if (p->periodic) {
            // at most path_cells faces along an axis: a path of L cells spans at most
            // (L / n + 2) periods of that axis's nb tiles
            int lmax = d->path_cells;
            if (lmax == 0) lmax = d->n[0] > d->n[1] ? (d->n[0] > d->n[2] ? d->n[0] : d->n[2])
                                                   : (d->n[1] > d->n[2] ? d->n[1] : d->n[2]);
            if (lmax > RT_MAX_PATH_CELLS) lmax = RT_MAX_PATH_CELLS;
            p->dmax = 2u * (uint32_t)lmax + 2u;
            visits = 0;
            for (int a = 0; a < 3; ++a) visits += (uint32_t)((lmax / d->n[a] + 2) * g.nb[a] + 1);
            visits -= 2u;
        }
        p->park_lanes = (uint32_t)d->park_lanes;
        p->park_passes = p->park_lanes ? visits : 0u;
        p->passes = visits + p->park_passes;
        p->finish = d->finish_pass > 0 ? (uint32_t)d->finish_pass : 0u;
        p->rec_bytes = rtk::tiled_record_bytes(p->fp64, p->species, p->mb);
        p->off_rec = o; o = align_up(o + cap * p->rec_bytes);
        p->off_idx0 = o; o = align_up(o + cap * sizeof(uint32_t));
        p->off_idx1 = o; o = align_up(o + cap * sizeof(uint32_t));
        p->off_side = o; o = align_up(o + cap * sizeof(uint32_t));
        p->off_cnt = o; o = align_up(o + nt * sizeof(uint32_t));
        p->off_off = o; o = align_up(o + nt * sizeof(uint32_t));
        p->off_cbase = o; o = align_up(o + mc * rtk::kCodes * sizeof(uint32_t));
        p->off_bsum = o; o = align_up(o + 2 * (size_t)p->scan_blocks * sizeof(uint32_t));
        p->off_ch0 = o; o = align_up(o + mc * sizeof(rtk::TChunk));
        p->off_ch1 = o; o = align_up(o + mc * sizeof(rtk::TChunk));
        p->off_ctrl = o; o = align_up(o + sizeof(rtk::TCtrl));
    }
    p->total = o;
    return RT_OK;
}

// Per-bin march table, [kTabRows][mb] in the march precision, into t (returns
// the number of values).  Rows 0-2: the cross-sections of HI, HeI, HeII
// (float32 form: in units of 1e-18 cm^2, lengths then in 1e18 cm, so optical
// depths stay far from the float32 range limits; times log2(e), formed in
// float64, since its optical depths come in units of ln 2).  Heat, in erg:
// pure hydrogen, row 3 E_j - E_th,HI.  H+He, float64 form: rows 3-5
// sigma_s,j (E_j - E_th,s), row 6 E_j - E_th,HI.  H+He, float32 form: row 3
// the photon energy E_j, row 4 the thresholds E_th,s (first three entries):
// it forms the heat as the energy of the absorbed photons less the
// thresholds of the photons each species absorbed, one product per bin.
int march_table(const rt_grid_desc *d, const Plan &p, double *t) {
    const int n = rtk::kTabRows * p.mb;
    for (int i = 0; i < n; ++i) t[i] = 0.0;
    const double scale = p.fp64 ? 1.0 : 1.0e18;
    const bool energies = !p.fp64 && p.species == 3;
    for (int s = 0; s < 3; ++s)
        for (int j = 0; j < d->n_bins; ++j) {
            const double sig = d->sigma_cm2[s][j];
            // heat per absorbed photon, in erg (so the march's heat needs no
            // conversion where it is deposited)
            const double de = sig > 0.0 ? (d->e_bin_ev[j] - kThresholdEv[s]) * kEvErg : 0.0;
            t[(size_t)s * p.mb + j] = sig * scale * (p.fp64 ? 1.0 : kLog2e);
            if (energies) continue;
            t[(size_t)(3 + s) * p.mb + j] = p.species == 1 ? de : sig * scale * de;
            if (s == 0) t[(size_t)6 * p.mb + j] = de;
        }
    if (energies) {
        for (int j = 0; j < d->n_bins; ++j) t[(size_t)3 * p.mb + j] = d->e_bin_ev[j] * kEvErg;
        for (int s = 0; s < 3; ++s) t[(size_t)4 * p.mb + s] = kThresholdEv[s] * kEvErg;
    }
    return n;
}

// 1 when the 8-bin H+He table has the threshold-aligned layout the tiled
// march has a specialisation for: HeI and HeII cross-sections zero in bins
// 0-2, HeII zero in bins 3-4.
int32_t bin_layout(const rt_grid_desc *d, const Plan &p) {
    if (p.species != 3 || p.mb != 8) return 0;
    for (int j = 0; j < 5 && j < d->n_bins; ++j) {
        if (d->sigma_cm2[2][j] != 0.0) return 0;
        if (j < 3 && d->sigma_cm2[1][j] != 0.0) return 0;
    }
    return 1;
}

}  // namespace

struct rt_solve {
    uint64_t magic;
    bool is_static;         // lives in the library's per-device static storage
    rt_grid_desc d;
    Plan plan;
    hipStream_t stream;
    int device;
    char *ws;
    int64_t max_src, n_src;
    uint64_t step_index;
    int blocks, chunk, refill_min;
    bool dead;
    // march timing (RT_TIME_MARCH): one event pair per timed sub-step of the last rt_step,
    // and one per launch of the march kernel itself (tiled march: one per pass)
    std::vector<hipEvent_t> ev;
    int timed;
    std::vector<hipEvent_t> kev;
    int ktimed;
    // recombination re-emission (RT_RECOMB), set by rt_set_recombination
    bool recomb_set;
    double f_rec, log10_t0, dlog10_t;
    int32_t n_t;
    // background field (rt_set_background)
    double bg_ndot, bg_carried;
    int64_t bg_packets;
    uint32_t bg_active;
    // end of the last fused call (rt_step_many) the solve was in, recorded on
    // that batch's stream (after_stream); the solve's stream waits for it
    // before its next own work or a call of another batch
    hipEvent_t after;
    hipStream_t after_stream;
    bool after_pending;
};

namespace {
constexpr int kMaxTimedSubsteps = 1024;
constexpr int kMaxTimedKernels = 16384;

// Workspace of rt_init_grid_static: a file-scope device array, one copy per
// device the library runs on, held until the process ends.  Host code uses
// the per-device address hipGetSymbolAddress returns, never the name.
constexpr size_t kStaticBytes = (size_t)RT_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices];
rt_solve g_static_solve[kMaxDevices];
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

bool valid(rt_solve_t h) { return h && h->magic == kMagic; }

int32_t fail(rt_solve_t h) {
    if (h) h->dead = true;
    return RT_EDEVICE;
}

rtk::MarchLaunch tiled_base(rt_solve_t h) {
    rtk::MarchLaunch m;
    memset(&m, 0, sizeof(m));
    m.blocks = h->blocks;
    m.stream = h->stream;
    return m;
}

rtk::TiledLaunch tiled_launch(rt_solve_t h, const rtk::MarchLaunch &m) {
    const Plan &p = h->plan;
    rtk::TiledLaunch t;
    memset(&t, 0, sizeof(t));
    t.m = m;
    t.capacity = p.capacity;
    t.cmax = p.cmax;
    t.max_chunks = p.max_chunks;
    t.n_tiles = p.n_tiles;
    t.scan_blocks = p.scan_blocks;
    t.passes = p.passes;
    t.park_passes = p.park_passes;
    t.park_lanes = p.park_lanes;
    t.finish = p.finish;
    t.periodic = p.periodic;
    t.dmax = p.dmax;
    t.rec = h->ws + p.off_rec;
    t.idx[0] = reinterpret_cast<uint32_t *>(h->ws + p.off_idx0);
    t.idx[1] = reinterpret_cast<uint32_t *>(h->ws + p.off_idx1);
    t.side = reinterpret_cast<uint32_t *>(h->ws + p.off_side);
    t.cnt = reinterpret_cast<uint32_t *>(h->ws + p.off_cnt);
    t.off = reinterpret_cast<uint32_t *>(h->ws + p.off_off);
    t.cbase = reinterpret_cast<uint32_t *>(h->ws + p.off_cbase);
    t.bsum = reinterpret_cast<uint32_t *>(h->ws + p.off_bsum);
    t.chunks[0] = reinterpret_cast<rtk::TChunk *>(h->ws + p.off_ch0);
    t.chunks[1] = reinterpret_cast<rtk::TChunk *>(h->ws + p.off_ch1);
    t.ctrl = reinterpret_cast<rtk::TCtrl *>(h->ws + p.off_ctrl);
    t.ledger = reinterpret_cast<rtk::StepLedger *>(h->ws + p.off_ledger);
    return t;
}

rtk::CellLaunch cell_launch(rt_solve_t h, double dt) {
    const Plan &p = h->plan;
    rtk::CellLaunch c;
    c.geo = p.geo;
    c.fp64 = p.fp64;
    c.species = p.species;
    c.thermal = p.thermal;
    c.state = h->ws + p.off_state;
    c.kappa = h->ws + p.off_kappa;
    c.acc = reinterpret_cast<double *>(h->ws + p.off_acc);
    c.acc_stride = p.acc_stride;
    c.y_he = h->d.y_he;
    c.cell_cm = h->d.cell_cm;
    c.dt = dt;
    c.redshift = h->d.redshift;
    c.n_chem = h->d.n_chem;
    c.queue = reinterpret_cast<unsigned long long *>(h->ws + p.off_queue);
    c.ledger = reinterpret_cast<rtk::StepLedger *>(h->ws + p.off_ledger);
    c.rc = p.recomb ? reinterpret_cast<double *>(h->ws + p.off_rc) : nullptr;
    c.stream = h->stream;
    return c;
}

rtk::RecombParams recomb_params(rt_solve_t h) {
    const Plan &p = h->plan;
    rtk::RecombParams r;
    r.rc = reinterpret_cast<double *>(h->ws + p.off_rc);
    r.milne = reinterpret_cast<const double *>(h->ws + p.off_milne);
    r.state = h->ws + p.off_state;
    r.n_t = h->n_t;
    r.acc_stride = p.acc_stride;
    r.log10_t0 = h->log10_t0;
    r.dlog10_t = h->dlog10_t;
    r.f_rec = h->f_rec;
    r.volume = h->d.cell_cm * h->d.cell_cm * h->d.cell_cm;
    r.y_he = h->d.y_he;
    r.ledger = reinterpret_cast<rtk::StepLedger *>(h->ws + p.off_ledger);
    return r;
}

// Fill the handle h and load the initial state into the workspace ws (a plan
// already validated and the arguments checked).  No device memory is
// allocated; events are created only for RT_TIME_MARCH.
// Order the solve's stream after the last fused call it was in (if not yet).
bool order_after_batch(rt_solve *h) {
    if (!h->after_pending) return true;
    h->after_pending = false;
    return hipStreamWaitEvent(h->stream, h->after, 0) == hipSuccess;
}

int32_t init_solve(rt_solve *h, const rt_grid_desc *d, const Plan &p, char *ws, int64_t max_sources,
                   const void *d_nh, const void *d_x, const void *d_temp, int32_t fields_fp64, void *hip_stream) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RT_EDEVICE;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return RT_EDEVICE;
    int bpcu = d->blocks_per_cu;
    if (bpcu == 0) {
        const hipError_t e = p.tiled ? rtk::tiled_occupancy(p.species, p.thermal, p.fp64, p.mb, &bpcu)
                                     : rtk::march_occupancy(p.species, p.thermal, p.fp64, p.mb, &bpcu);
        if (e != hipSuccess) return RT_EDEVICE;
        if (bpcu < 1) bpcu = 1;
    }
    int blocks = cus * bpcu;
    if (blocks > kMaxMarchBlocks) blocks = kMaxMarchBlocks;

    h->magic = kMagic;
    h->d = *d;
    h->plan = p;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->device = dev;
    h->ws = ws;
    h->max_src = max_sources;
    h->n_src = 0;
    h->step_index = d->step_index0;
    h->blocks = blocks;
    h->chunk = d->wave_chunk > 0 ? d->wave_chunk : 256;
    h->refill_min = d->refill_min > 0 ? d->refill_min : (p.tiled ? 32 : 8);
    h->dead = false;
    h->timed = 0;
    h->ktimed = 0;
    h->recomb_set = false;
    h->f_rec = h->log10_t0 = h->dlog10_t = 0.0;
    h->n_t = 0;
    h->bg_ndot = h->bg_carried = 0.0;
    h->bg_packets = 0;
    h->bg_active = 0u;
    h->ev.clear();
    h->kev.clear();
    h->after = nullptr;
    h->after_stream = nullptr;
    h->after_pending = false;
    auto destroy_events = [h] {
        for (hipEvent_t e : h->ev) if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : h->kev) if (e) (void)hipEventDestroy(e);
        h->ev.clear();
        h->kev.clear();
        if (h->after) (void)hipEventDestroy(h->after);
        h->after = nullptr;
    };
    if (hipEventCreateWithFlags(&h->after, hipEventDisableTiming) != hipSuccess) {
        h->after = nullptr;
        return RT_EDEVICE;
    }
    if (d->flags & RT_TIME_MARCH) {
        h->ev.assign(2 * kMaxTimedSubsteps, nullptr);
        h->kev.assign(p.tiled ? 2 * kMaxTimedKernels : 0, nullptr);
        bool ok = true;
        for (size_t i = 0; i < h->ev.size() && ok; ++i) ok = hipEventCreate(&h->ev[i]) == hipSuccess;
        for (size_t i = 0; i < h->kev.size() && ok; ++i) ok = hipEventCreate(&h->kev[i]) == hipSuccess;
        if (!ok) {
            destroy_events();
            return RT_EDEVICE;
        }
    }

    rtk::CellLaunch c = cell_launch(h, 0.0);
    // the per-bin march table in the march precision
    double tab[rtk::kTabRows * kMaxSupportedBins];
    float tab_f[rtk::kTabRows * kMaxSupportedBins];
    const int ntab = march_table(d, p, tab);
    for (int i = 0; i < ntab; ++i) tab_f[i] = (float)tab[i];
    const void *tab_src = p.fp64 ? (const void *)tab : (const void *)tab_f;
    if (hipMemcpyAsync(ws + p.off_tab, tab_src, (size_t)ntab * p.real, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess ||
        rtk::launch_import(c, d_nh, d_x, d_temp, fields_fp64, p.ncell) != hipSuccess ||
        rtk::launch_ledger_zero(c.ledger, h->stream) != hipSuccess ||
        (p.recomb && rtk::launch_import_counters(c, nullptr, 1, p.ncell) != hipSuccess) ||
        (p.tiled && rtk::launch_tiled_reset(tiled_launch(h, tiled_base(h))) != hipSuccess)) {
        destroy_events();
        return RT_EDEVICE;
    }
    return RT_OK;
}

}  // namespace

extern "C" {

int32_t rt_desc_defaults(rt_grid_desc *d) {
    if (!d) return RT_EINVAL;
    memset(d, 0, sizeof(*d));
    d->n[0] = d->n[1] = d->n[2] = 1;
    d->cell_cm = 1.0;
    d->n_bins = 1;
    d->e_bin_ev[0] = 13.6;
    d->redshift = -1.0;
    d->tau_kill = 30.0;
    d->n_sub = 1;
    d->n_chem = 8;
    d->brick_log2 = -1;
    return RT_OK;
}

int32_t rt_workspace_bytes(const rt_grid_desc *d, int64_t max_sources, size_t *bytes_out) {
    if (!bytes_out) return RT_EINVAL;
    Plan p{};
    const int32_t r = make_plan(d, max_sources, &p);
    if (r != RT_OK) return r;
    *bytes_out = p.total;
    return RT_OK;
}

int32_t rt_init_grid(const rt_grid_desc *d, void *d_ws, size_t ws_bytes, int64_t max_sources,
                     const void *d_nh, const void *d_x, const void *d_temp, int32_t fields_fp64,
                     void *hip_stream, rt_solve_t *out) {
    if (!out) return RT_EINVAL;
    *out = nullptr;
    Plan p{};
    const int32_t r = make_plan(d, max_sources, &p);
    if (r != RT_OK) return r;
    if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0) return RT_EINVAL;
    if (!d_nh || !d_x || !d_temp || (fields_fp64 != 0 && fields_fp64 != 1)) return RT_EINVAL;
    if (ws_bytes < p.total) return RT_ENOMEM;
    rt_solve *h = new (std::nothrow) rt_solve;
    if (!h) return RT_ENOMEM;
    h->is_static = false;
    const int32_t st = init_solve(h, d, p, reinterpret_cast<char *>(d_ws), max_sources, d_nh, d_x, d_temp,
                                  fields_fp64, hip_stream);
    if (st != RT_OK) {
        delete h;
        return st;
    }
    *out = h;
    return RT_OK;
}

int32_t rt_init_grid_static(const rt_grid_desc *d, int64_t max_sources, const void *d_nh, const void *d_x,
                            const void *d_temp, int32_t fields_fp64, void *hip_stream, rt_solve_t *out) {
    if (!out) return RT_EINVAL;
    *out = nullptr;
    Plan p{};
    const int32_t r = make_plan(d, max_sources, &p);
    if (r != RT_OK) return r;
    if (!d_nh || !d_x || !d_temp || (fields_fp64 != 0 && fields_fp64 != 1)) return RT_EINVAL;
    if (d->flags & RT_TIME_MARCH) return RT_EINVAL;         // its events would be allocated
    if (p.total > kStaticBytes) return RT_ESCRATCH;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RT_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return RT_EINVAL;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        // the array's device address on this device (the name itself is a
        // host-side stand-in): once per device, with that device current
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RT_EDEVICE;
        g_static_ptr[dev] = ptr;
    }
    rt_solve *h = &g_static_solve[dev];
    if (h->magic == kMagic) return RT_ESTATE;                // the last static solve was not released
    h->is_static = true;
    const int32_t st = init_solve(h, d, p, reinterpret_cast<char *>(g_static_ptr[dev]), max_sources, d_nh, d_x,
                                  d_temp, fields_fp64, hip_stream);
    if (st != RT_OK) {
        h->magic = 0;
        return st;
    }
    *out = h;
    return RT_OK;
}

int32_t rt_add_sources(rt_solve_t h, int32_t n, const int32_t *h_ijk, const double *h_ndot,
                       const double *h_sed, uint32_t src_flags) {
    if (!valid(h)) return RT_EINVAL;
    if (h->dead) return RT_ESTATE;
    if (!order_after_batch(h)) return fail(h);
    if (n < 0 || (src_flags & ~RT_SRC_CORNER_OCTANT)) return RT_EINVAL;
    if (n == 0) return RT_OK;
    if (!h_ijk || !h_ndot || !h_sed) return RT_EINVAL;
    if (h->n_src + n > h->max_src) return RT_ENOMEM;
    const Plan &p = h->plan;
    const int nb = h->d.n_bins, mb = p.mb;
    const bool oct = (src_flags & RT_SRC_CORNER_OCTANT) != 0;
    std::vector<rtk::SourceRec> rec(n);
    std::vector<double> sedsum(n), sed_d((size_t)n * mb, 0.0);
    std::vector<float> sed_f((size_t)n * mb, 0.0f);
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            const int32_t v = h_ijk[3 * i + a];
            if (v < 0 || v >= h->d.n[a]) return RT_EINVAL;
            rec[i].o[a] = 2 * v + (oct ? 0 : 1);
        }
        rec[i].flags = oct ? rtk::kSrcOctant : 0u;
        if (!finite_nonneg(h_ndot[i])) return RT_EINVAL;
        double s = 0.0;
        for (int j = 0; j < nb; ++j) {
            const double v = h_sed[(size_t)i * nb + j];
            if (!finite_nonneg(v)) return RT_EINVAL;
            if (v > 0.0) rec[i].flags |= 1u << (rtk::kSrcMaskShift + j);
            s += v;
            sed_d[(size_t)i * mb + j] = v;
            sed_f[(size_t)i * mb + j] = (float)v;
        }
        if (!(s > 0.0)) return RT_EINVAL;
        sedsum[i] = s;
    }
    const size_t k = (size_t)h->n_src;
    hipStream_t st = h->stream;
    if (hipMemcpyAsync(h->ws + p.off_src + k * sizeof(rtk::SourceRec), rec.data(), n * sizeof(rtk::SourceRec),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h->ws + p.off_ndot + k * sizeof(double), h_ndot, n * sizeof(double),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h->ws + p.off_sedsum + k * sizeof(double), sedsum.data(), n * sizeof(double),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(h);
    const void *sed = p.fp64 ? (const void *)sed_d.data() : (const void *)sed_f.data();
    if (hipMemcpyAsync(h->ws + p.off_sed + k * mb * p.real, sed, (size_t)n * mb * p.real,
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(h);
    h->n_src += n;
    return RT_OK;
}

int32_t rt_read_stats(rt_solve_t h, rt_step_stats *stats) {
    if (!valid(h) || !stats) return RT_EINVAL;
    if (h->dead) return RT_ESTATE;
    if (!order_after_batch(h)) return fail(h);
    rtk::StepLedger l;
    if (hipMemcpyAsync(&l, h->ws + h->plan.off_ledger, sizeof(l), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return fail(h);
    stats->emitted = l.s[0] + l.s[1];
    stats->absorbed = l.s[2] + l.s[3];
    stats->escaped = l.s[4] + l.s[5];
    stats->truncated = l.s[6] + l.s[7];
    stats->crossings = (int64_t)l.c[0];
    stats->packets = (int64_t)l.c[1];
    stats->n_escaped = (int64_t)l.c[2];
    stats->n_truncated = (int64_t)l.c[3];
    stats->substeps = (int64_t)l.substeps;
    stats->nonfinite = l.nonfinite;
    stats->errors = l.errors;
    stats->diffuse_emitted = l.d_emit;
    stats->diffuse_packets = (int64_t)l.d_packets;
    stats->march_ms = 0.0;
    for (int i = 0; i < h->timed; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]) != hipSuccess) return fail(h);
        stats->march_ms += ms;
    }
    stats->kernel_ms = 0.0;
    stats->kernel_launches = 0;
    if (h->plan.tiled) {
        for (int i = 0; i < h->ktimed; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, h->kev[2 * i], h->kev[2 * i + 1]) != hipSuccess) return fail(h);
            stats->kernel_ms += ms;
        }
        stats->kernel_launches = h->ktimed;
    } else {
        stats->kernel_ms = stats->march_ms;      // one march launch per sub-step
        stats->kernel_launches = h->timed;
    }
    if (l.errors) {
        h->dead = true;
        return RT_EINTERNAL;
    }
    return RT_OK;
}

int32_t rt_step(rt_solve_t h, double dt_s, int64_t n_packets, uint64_t seed, rt_step_stats *stats) {
    if (!valid(h)) return RT_EINVAL;
    if (h->dead) return RT_ESTATE;
    if (!order_after_batch(h)) return fail(h);
    if (!(isfinite(dt_s) && dt_s > 0.0) || n_packets < 0) return RT_EINVAL;
    const int32_t nsub = h->d.n_sub;
    const int64_t base = n_packets / nsub, extra = n_packets % nsub;
    if (h->n_src > 0 && base < h->n_src) return RT_EINVAL;
    if (h->plan.recomb && !h->recomb_set) return RT_ESTATE;
    if (base + 1 > ((int64_t)1 << 31)) return RT_EOVERFLOW;
    const Plan &p = h->plan;
    const double dts = dt_s / nsub;
    rtk::CellLaunch c = cell_launch(h, dts);
    if (rtk::launch_ledger_zero(c.ledger, h->stream) != hipSuccess) return fail(h);

    rtk::MarchLaunch m;
    memset(&m, 0, sizeof(m));
    m.geo = p.geo;
    m.half_dl = 0.5 * h->d.cell_cm;
    m.species = p.species;
    m.thermal = p.thermal;
    m.fp64 = p.fp64;
    m.n_bins = h->d.n_bins;
    m.mb = p.mb;
    m.layout = bin_layout(&h->d, p);
    m.src = reinterpret_cast<const rtk::SourceRec *>(h->ws + p.off_src);
    m.src_ndot = reinterpret_cast<const double *>(h->ws + p.off_ndot);
    m.src_sedsum = reinterpret_cast<const double *>(h->ws + p.off_sedsum);
    m.sed = h->ws + p.off_sed;
    m.n_src = (int32_t)h->n_src;
    m.dt = dts;
    m.seed = seed;
    m.solve_id = h->d.solve_id;
    m.tab = h->ws + p.off_tab;
    m.tau_kill = h->d.tau_kill;
    m.kappa = c.kappa;
    m.acc = c.acc;
    m.acc_stride = p.acc_stride;
    m.queue = c.queue;
    m.slots = reinterpret_cast<rtk::LedgerSlot *>(h->ws + p.off_slots);
    m.trace = h->d.trace_packets > 0 ? reinterpret_cast<int32_t *>(h->ws + p.off_trace) : nullptr;
    m.trace_n = h->d.trace_packets;
    m.trace_len = h->d.trace_len;
    m.trace_stride = h->d.trace_stride > 0 ? h->d.trace_stride : 1;
    m.chunk = h->chunk;
    m.refill_min = h->refill_min;
    m.blocks = h->blocks;
    m.stream = h->stream;

    h->timed = 0;
    h->ktimed = 0;
    for (int32_t i = 0; i < nsub; ++i) {
        const int64_t Pi = base + (i < extra ? 1 : 0);
        if (rtk::launch_prep(c) != hipSuccess) return fail(h);
        const bool sources = h->n_src > 0 && Pi > 0;
        const int64_t Pb = h->bg_packets / nsub + (i < h->bg_packets % nsub ? 1 : 0);
        const bool march = sources || Pb > 0;
        if (march) {
            m.packets = (uint32_t)Pi;
            m.step_index = h->step_index;
            const bool timed = !h->ev.empty() && h->timed < kMaxTimedSubsteps;
            if (timed && hipEventRecord(h->ev[2 * h->timed], h->stream) != hipSuccess) return fail(h);
            if (p.tiled) {
                rtk::TiledLaunch t = tiled_launch(h, m);
                if (!h->kev.empty()) {
                    t.ev = h->kev.data();
                    t.ev_cap = kMaxTimedKernels;
                    t.ev_used = &h->ktimed;
                }
                if (rtk::launch_tiled_slots_zero(t) != hipSuccess) return fail(h);
                for (int64_t g0 = 0; sources && g0 < Pi; g0 += p.capacity) {
                    t.g0 = (uint32_t)g0;
                    t.nbatch = (uint32_t)(Pi - g0 < (int64_t)p.capacity ? Pi - g0 : p.capacity);
                    if (rtk::launch_tiled_batch(t) != hipSuccess) return fail(h);
                }
                if (Pb > 0) {
                    rtk::BackgroundParams bp;
                    bp.ndot = h->bg_ndot;
                    bp.carried = h->bg_carried;
                    bp.sed = h->ws + p.off_bg;
                    bp.active = h->bg_active;
                    bp.packets = (uint32_t)Pb;
                    bp.pad = 0;
                    for (int64_t g0 = 0; g0 < Pb; g0 += p.capacity) {
                        bp.g0 = (uint32_t)g0;
                        t.g0 = 0;
                        t.nbatch = (uint32_t)(Pb - g0 < (int64_t)p.capacity ? Pb - g0 : p.capacity);
                        if (rtk::launch_tiled_background(t, bp) != hipSuccess) return fail(h);
                    }
                }
                if (p.recomb && rtk::launch_tiled_reemit(t, recomb_params(h)) != hipSuccess) return fail(h);
            } else if (rtk::launch_march(m) != hipSuccess) {
                return fail(h);
            }
            if (timed) {
                if (hipEventRecord(h->ev[2 * h->timed + 1], h->stream) != hipSuccess) return fail(h);
                ++h->timed;
            }
        }
        if (rtk::launch_ledger_reduce(m.slots, march ? h->blocks : 0, c.ledger, h->stream) != hipSuccess)
            return fail(h);
        if (rtk::launch_update(c) != hipSuccess) return fail(h);
        h->step_index += 1;
    }
    if (stats) return rt_read_stats(h, stats);
    return RT_OK;
}

int32_t rt_fetch_fields(rt_solve_t h, uint32_t mask, void *dst, int32_t dst_is_device, int32_t as_fp64) {
    if (!valid(h)) return RT_EINVAL;
    if (h->dead) return RT_ESTATE;
    if (!order_after_batch(h)) return fail(h);
    if (!dst || mask == 0 || (mask & ~RT_F_ALL) || (as_fp64 != 0 && as_fp64 != 1) ||
        (dst_is_device != 0 && dst_is_device != 1))
        return RT_EINVAL;
    const Plan &p = h->plan;
    rtk::CellLaunch c = cell_launch(h, 0.0);
    const size_t esz = as_fp64 ? sizeof(double) : sizeof(float);
    if (dst_is_device) {
        if (rtk::launch_export(c, mask, dst, as_fp64, p.ncell) != hipSuccess) return fail(h);
    } else {
        void *stage = h->ws + p.off_stage;
        char *out = reinterpret_cast<char *>(dst);
        for (int f = 0; f < 14; ++f) {
            if (!(mask & (1u << f))) continue;
            if (rtk::launch_export(c, 1u << f, stage, as_fp64, p.ncell) != hipSuccess ||
                hipMemcpyAsync(out, stage, (size_t)p.ncell * esz, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
                hipStreamSynchronize(h->stream) != hipSuccess)
                return fail(h);
            out += (size_t)p.ncell * esz;
        }
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h);
    return RT_OK;
}

int32_t rt_set_recombination(rt_solve_t h, double f_rec, int32_t n_t, double log10_t0, double dlog10_t,
                             const double *h_milne, const void *d_counters, int32_t counters_fp64) {
    if (!valid(h)) return RT_EINVAL;
    if (h->dead) return RT_ESTATE;
    if (!order_after_batch(h)) return fail(h);
    const Plan &p = h->plan;
    if (!p.recomb) return RT_ESTATE;
    if (!(isfinite(f_rec) && f_rec >= 0.0) || n_t < 2 || n_t > RT_MAX_MILNE_T || !isfinite(log10_t0) ||
        !(isfinite(dlog10_t) && dlog10_t > 0.0) || !h_milne || (counters_fp64 != 0 && counters_fp64 != 1))
        return RT_EINVAL;
    const int nb = h->d.n_bins, mb = p.mb;
    std::vector<double> tab(3 * (size_t)n_t * mb, 0.0);
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < n_t; ++k) {
            double sum = 0.0;
            for (int j = 0; j < nb; ++j) {
                const double v = h_milne[((size_t)a * n_t + k) * nb + j];
                if (!finite_nonneg(v)) return RT_EINVAL;
                // no photons of an ion in a bin that is not above its threshold
                if (v > 0.0 && h->d.e_bin_ev[j] < kThresholdEv[a] && nb > 1) return RT_EINVAL;
                tab[((size_t)a * n_t + k) * mb + j] = v;
                sum += v;
            }
            if (!(fabs(sum - 1.0) <= 1.0e-9)) return RT_EINVAL;
        }
    rtk::CellLaunch c = cell_launch(h, 0.0);
    if (hipMemcpyAsync(h->ws + p.off_milne, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        rtk::launch_import_counters(c, d_counters, counters_fp64, p.ncell) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return fail(h);
    h->f_rec = f_rec;
    h->n_t = n_t;
    h->log10_t0 = log10_t0;
    h->dlog10_t = dlog10_t;
    h->recomb_set = true;
    return RT_OK;
}

int32_t rt_set_background(rt_solve_t h, double ndot, const double *h_sed, int64_t packets_per_step) {
    if (!valid(h)) return RT_EINVAL;
    if (h->dead) return RT_ESTATE;
    if (!order_after_batch(h)) return fail(h);
    const Plan &p = h->plan;
    if (!p.tiled) return RT_ESTATE;
    if (!finite_nonneg(ndot) || packets_per_step < 0) return RT_EINVAL;
    if (packets_per_step / h->d.n_sub + 1 > ((int64_t)1 << 31)) return RT_EOVERFLOW;
    if (packets_per_step == 0) {
        h->bg_packets = 0;
        return RT_OK;
    }
    if (!h_sed) return RT_EINVAL;
    const int nb = h->d.n_bins, mb = p.mb;
    std::vector<double> sd(mb, 0.0);
    std::vector<float> sf(mb, 0.0f);
    double carried = 0.0, sum = 0.0;
    uint32_t active = 0u;
    for (int j = 0; j < nb; ++j) {
        const double v = h_sed[j];
        if (!finite_nonneg(v)) return RT_EINVAL;
        sd[j] = v;
        sf[j] = (float)v;
        sum += v;
        carried += v;                       // as for source rows: the float64 spectrum's sum
        if (v > 0.0) active |= 1u << j;
    }
    if (!(sum > 0.0)) return RT_EINVAL;
    const void *src = p.fp64 ? (const void *)sd.data() : (const void *)sf.data();
    if (hipMemcpyAsync(h->ws + p.off_bg, src, (size_t)mb * p.real, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return fail(h);
    h->bg_ndot = ndot;
    h->bg_carried = carried;
    h->bg_active = active;
    h->bg_packets = packets_per_step;
    return RT_OK;
}

int32_t rt_fetch_trace(rt_solve_t h, int32_t *h_dst, int64_t count) {
    if (!valid(h)) return RT_EINVAL;
    if (h->dead) return RT_ESTATE;
    if (!order_after_batch(h)) return fail(h);
    if (count < 0 || count > h->d.trace_packets || (count > 0 && !h_dst)) return RT_EINVAL;
    const size_t bytes = (size_t)count * (RT_TRACE_HDR + (size_t)h->d.trace_len) * sizeof(int32_t);
    if (bytes == 0) return RT_OK;
    if (hipMemcpyAsync(h_dst, h->ws + h->plan.off_trace, bytes, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return fail(h);
    return RT_OK;
}

int32_t rt_trace_rays(rt_solve_t h, int32_t m, const int32_t *d_origin, const int32_t *d_dir, int32_t max_len,
                      int32_t *d_cells, int32_t *d_count, int32_t *d_face) {
    if (!valid(h)) return RT_EINVAL;
    if (h->dead) return RT_ESTATE;
    if (!order_after_batch(h)) return fail(h);
    if (m < 0 || max_len < 0) return RT_EINVAL;
    if (m == 0) return RT_OK;
    if (!d_origin || !d_dir || !d_count || !d_face || (max_len > 0 && !d_cells)) return RT_EINVAL;
    if (rtk::launch_trace_rays(h->plan.geo, m, d_origin, d_dir, max_len, d_cells, d_count, d_face, h->stream) !=
        hipSuccess)
        return fail(h);
    return RT_OK;
}

int32_t rt_get_step_index(rt_solve_t h, uint64_t *out) {
    if (!valid(h) || !out) return RT_EINVAL;
    *out = h->step_index;
    return RT_OK;
}

int32_t rt_release(rt_solve_t h) {
    if (!valid(h)) return RT_EINVAL;
    const bool ok = h->dead || (order_after_batch(h) && hipStreamSynchronize(h->stream) == hipSuccess);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->kev) (void)hipEventDestroy(e);
    h->ev.clear();
    h->kev.clear();
    if (h->after) (void)hipEventDestroy(h->after);
    h->after = nullptr;
    if (h->is_static) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        h->magic = 0;                     // the device's static storage is free again
    } else {
        h->magic = 0;
        delete h;
    }
    return ok ? RT_OK : RT_EDEVICE;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Fused steps of many solves
// ---------------------------------------------------------------------------
namespace {

constexpr uint64_t kBatchMagic = 0x52544d4342415443ull;
constexpr int kMaxBatchBlocks = 2048;     // march blocks the ledger slots are sized for

// The march instance the solves of a batch share, from its shape description.
struct BatchShape {
    int fp64, species, mb, thermal, refill_min, cmax, bpcu;
    uint32_t finish;
    size_t rec_bytes;
};

int32_t batch_shape(const rt_grid_desc *d, BatchShape *s) {
    Plan p{};
    const int32_t r = make_plan(d, 1, &p);
    if (r != RT_OK) return r;
    s->fp64 = p.fp64;
    s->species = p.species;
    s->mb = p.mb;
    s->thermal = p.thermal;
    s->refill_min = d->refill_min > 0 ? d->refill_min : 32;
    s->cmax = d->run_len > 0 ? d->run_len : kDefaultBatchRun;
    s->bpcu = d->blocks_per_cu;
    s->finish = d->finish_pass > 0 ? (uint32_t)d->finish_pass : 0u;
    s->rec_bytes = rtk::batch_record_bytes(p.fp64, p.species, p.mb);
    return RT_OK;
}

struct BatchLayout {
    size_t off_head, off_table, off_slots, off_queue, off_rec, off_idx0, off_idx1, off_side, off_cnt, off_off,
        off_tsolve, off_cbase, off_bsum, off_ch0, off_ch1, off_ctrl, off_first, off_ledgers, total;
    uint32_t capacity, max_tiles, max_chunks, scan_blocks;
};

int32_t batch_layout(int32_t max_solves, const BatchShape &sh, int64_t max_round_packets, int64_t max_tiles,
                     BatchLayout *l) {
    if (max_solves < 1 || max_solves > RT_MAX_BATCH || max_round_packets < 1 || max_tiles < 1) return RT_EINVAL;
    if (max_round_packets > ((int64_t)1 << 31) - 1 || max_tiles > ((int64_t)1 << 26)) return RT_EOVERFLOW;
    const uint64_t cap = (uint64_t)max_round_packets, nt = (uint64_t)max_tiles;
    const uint64_t mc = nt + cap / (uint64_t)sh.cmax + 1;
    if (mc >= (1ull << 31)) return RT_EOVERFLOW;
    l->capacity = (uint32_t)cap;
    l->max_tiles = (uint32_t)nt;
    l->max_chunks = (uint32_t)mc;
    l->scan_blocks = (uint32_t)((nt + 4095) / 4096);
    size_t o = 0;
    // the table follows the head directly, as in the staging memory it is copied from
    l->off_head = o;
    l->off_table = o + sizeof(rtk::BatchHead);
    o = align_up(l->off_table + (size_t)max_solves * sizeof(rtk::BatchSolve));
    l->off_slots = o; o = align_up(o + (size_t)max_solves * kMaxBatchBlocks * sizeof(rtk::LedgerSlot));
    l->off_queue = o; o = align_up(o + sizeof(unsigned long long));
    l->off_rec = o; o = align_up(o + cap * sh.rec_bytes);
    l->off_idx0 = o; o = align_up(o + cap * sizeof(uint32_t));
    l->off_idx1 = o; o = align_up(o + cap * sizeof(uint32_t));
    l->off_side = o; o = align_up(o + cap * sizeof(uint32_t));
    l->off_cnt = o; o = align_up(o + nt * sizeof(uint32_t));
    l->off_off = o; o = align_up(o + nt * sizeof(uint32_t));
    l->off_tsolve = o; o = align_up(o + nt * sizeof(uint16_t));
    l->off_cbase = o; o = align_up(o + mc * rtk::kCodes * sizeof(uint32_t));
    l->off_bsum = o; o = align_up(o + 2 * (size_t)l->scan_blocks * sizeof(uint32_t));
    l->off_ch0 = o; o = align_up(o + mc * sizeof(rtk::TChunk));
    l->off_ch1 = o; o = align_up(o + mc * sizeof(rtk::TChunk));
    l->off_ctrl = o; o = align_up(o + sizeof(rtk::TCtrl));
    l->off_first = o; o = align_up(o + (rtk::kMaxBatch + 1) * sizeof(uint32_t));
    l->off_ledgers = o; o = align_up(o + (size_t)max_solves * sizeof(rtk::StepLedger));
    l->total = o;
    return RT_OK;
}

struct BatchGraph {
    int rounds;
    uint32_t passes;
    hipGraphExec_t exec;
};

}  // namespace

struct rt_batch {
    uint64_t magic;
    int32_t max_solves;
    uint32_t flags;
    hipStream_t stream;
    int device, cus;
    char *ws;
    BatchShape shape;
    BatchLayout lay;
    int blocks;                    // march blocks
    void *staging;                 // pinned: head then table
    hipEvent_t staged;             // the last table copy has been read
    bool staged_pending;
    hipEvent_t done;               // end of the last fused call (its ledgers copied out)
    std::vector<hipEvent_t> ev_in; // one per distinct solve stream of a call: its work before the call
    std::vector<BatchGraph> graphs;
    rtk::StepLedger *ledgers;      // pinned: the solves' ledgers after the last call
    std::vector<rt_solve_t> last;  // the solves of the last call, in its order
};

namespace {

bool batch_valid(rt_batch_t b) { return b && b->magic == kBatchMagic; }

rtk::BatchLaunch batch_launch(rt_batch_t b, uint32_t passes) {
    rtk::BatchLaunch l;
    memset(&l, 0, sizeof(l));
    char *ws = b->ws;
    const BatchLayout &y = b->lay;
    l.head = reinterpret_cast<const rtk::BatchHead *>(ws + y.off_head);
    l.table = reinterpret_cast<const rtk::BatchSolve *>(ws + y.off_table);
    l.slots = reinterpret_cast<rtk::LedgerSlot *>(ws + y.off_slots);
    l.queue = reinterpret_cast<unsigned long long *>(ws + y.off_queue);
    l.fp64 = b->shape.fp64;
    l.thermal = b->shape.thermal;
    l.species = b->shape.species;
    l.mb = b->shape.mb;
    l.blocks = b->blocks;
    l.refill_min = b->shape.refill_min;
    l.cell_blocks = b->cus * 8;
    l.passes = passes;
    l.finish = b->shape.finish;
    rtk::BatchTiles &t = l.t;
    t.rec = ws + y.off_rec;
    t.idx[0] = reinterpret_cast<uint32_t *>(ws + y.off_idx0);
    t.idx[1] = reinterpret_cast<uint32_t *>(ws + y.off_idx1);
    t.side = reinterpret_cast<uint32_t *>(ws + y.off_side);
    t.cnt = reinterpret_cast<uint32_t *>(ws + y.off_cnt);
    t.off = reinterpret_cast<uint32_t *>(ws + y.off_off);
    t.cbase = reinterpret_cast<uint32_t *>(ws + y.off_cbase);
    t.bsum = reinterpret_cast<uint32_t *>(ws + y.off_bsum);
    t.tsolve = reinterpret_cast<uint16_t *>(ws + y.off_tsolve);
    t.first = reinterpret_cast<uint32_t *>(ws + y.off_first);
    t.chunks[0] = reinterpret_cast<rtk::TChunk *>(ws + y.off_ch0);
    t.chunks[1] = reinterpret_cast<rtk::TChunk *>(ws + y.off_ch1);
    t.ctrl = reinterpret_cast<rtk::TCtrl *>(ws + y.off_ctrl);
    t.capacity = y.capacity;
    t.max_tiles = y.max_tiles;
    t.max_chunks = y.max_chunks;
    t.cmax = (uint32_t)b->shape.cmax;
    t.scan_blocks = y.scan_blocks;
    l.stream = b->stream;
    return l;
}

// Every launch of one call: ledgers cleared, each fused tile's solve, then per
// round absorbers, the tiled march, ledger reduction and cell update of every
// solve that still has sub-steps.
hipError_t batch_enqueue(const rtk::BatchLaunch &l, int rounds) {
    hipError_t e = rtk::launch_batch_begin(l);
    if (e == hipSuccess) e = rtk::launch_batch_tiles(l);
    for (int r = 0; r < rounds && e == hipSuccess; ++r) {
        e = rtk::launch_batch_prep(l, r);
        if (e == hipSuccess) e = rtk::launch_batch_march(l, r);
        if (e == hipSuccess) e = rtk::launch_batch_ledger(l, r);
        if (e == hipSuccess) e = rtk::launch_batch_update(l, r);
    }
    return e;
}

hipError_t batch_graph(rt_batch_t b, const rtk::BatchLaunch &l, int rounds, hipGraphExec_t *out) {
    for (const BatchGraph &g : b->graphs)
        if (g.rounds == rounds && g.passes == l.passes) {
            *out = g.exec;
            return hipSuccess;
        }
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t el = batch_enqueue(l, rounds);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->stream, &graph);
    if (el != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return el != hipSuccess ? el : e;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    b->graphs.push_back(BatchGraph{rounds, l.passes, exec});
    *out = exec;
    return hipSuccess;
}

void batch_destroy(rt_batch_t b) {
    for (BatchGraph &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    for (hipEvent_t e : b->ev_in) if (e) (void)hipEventDestroy(e);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->staging) (void)hipHostFree(b->staging);
    if (b->ledgers) (void)hipHostFree(b->ledgers);
    b->magic = 0;
    delete b;
}

}  // namespace

extern "C" {

int32_t rt_batch_workspace_bytes(int32_t max_solves, const rt_grid_desc *shape, int64_t max_round_packets,
                                 int64_t max_tiles, size_t *bytes_out) {
    if (!bytes_out || !shape) return RT_EINVAL;
    BatchShape sh;
    int32_t r = batch_shape(shape, &sh);
    if (r != RT_OK) return r;
    BatchLayout l;
    r = batch_layout(max_solves, sh, max_round_packets, max_tiles, &l);
    if (r != RT_OK) return r;
    *bytes_out = l.total;
    return RT_OK;
}

int32_t rt_batch_init(int32_t max_solves, const rt_grid_desc *shape, int64_t max_round_packets, int64_t max_tiles,
                      void *d_ws, size_t ws_bytes, void *hip_stream, uint32_t flags, rt_batch_t *out) {
    if (!out) return RT_EINVAL;
    *out = nullptr;
    if (!shape || (flags & ~RT_BATCH_GRAPH)) return RT_EINVAL;
    if ((flags & RT_BATCH_GRAPH) && !hip_stream) return RT_EINVAL;
    if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) % kAlign) != 0) return RT_EINVAL;
    BatchShape sh;
    int32_t r = batch_shape(shape, &sh);
    if (r != RT_OK) return r;
    BatchLayout lay;
    r = batch_layout(max_solves, sh, max_round_packets, max_tiles, &lay);
    if (r != RT_OK) return r;
    if (ws_bytes < lay.total) return RT_ENOMEM;
    rt_batch *b = new (std::nothrow) rt_batch;
    if (!b) return RT_ENOMEM;
    b->magic = kBatchMagic;
    b->max_solves = max_solves;
    b->flags = flags;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->ws = reinterpret_cast<char *>(d_ws);
    b->shape = sh;
    b->lay = lay;
    b->staging = nullptr;
    b->staged = nullptr;
    b->done = nullptr;
    b->staged_pending = false;
    b->ledgers = nullptr;
    int occ = 0;
    bool ok = hipGetDevice(&b->device) == hipSuccess &&
              hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess;
    if (ok && sh.bpcu == 0) ok = rtk::batch_march_occupancy(sh.fp64, sh.species, sh.thermal, sh.mb, &occ) == hipSuccess;
    if (sh.bpcu > 0) occ = sh.bpcu;
    if (occ < 1) occ = 1;
    b->blocks = b->cus * occ;
    if (b->blocks > kMaxBatchBlocks) b->blocks = kMaxBatchBlocks;
    if (b->blocks < 1) b->blocks = 1;
    ok = ok && hipHostMalloc(&b->staging, sizeof(rtk::BatchHead) + (size_t)max_solves * sizeof(rtk::BatchSolve),
                             hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void **>(&b->ledgers), (size_t)max_solves * sizeof(rtk::StepLedger),
                             hipHostMallocDefault) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->done, hipEventDisableTiming) == hipSuccess;
    b->ev_in.assign(max_solves, nullptr);
    for (int i = 0; i < max_solves && ok; ++i)
        ok = hipEventCreateWithFlags(&b->ev_in[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        batch_destroy(b);
        return RT_EDEVICE;
    }
    *out = b;
    return RT_OK;
}

int32_t rt_step_many(rt_batch_t b, const rt_solve_t *solves, int32_t n, const double *dt_s,
                     const int64_t *n_packets, const uint64_t *seeds, rt_step_stats *stats) {
    if (!batch_valid(b) || !solves || !dt_s || !n_packets || !seeds) return RT_EINVAL;
    if (n < 1 || n > b->max_solves) return RT_EINVAL;
    const BatchShape &sh = b->shape;
    int rounds = 0;
    uint64_t tiles = 0;
    uint32_t passes = 1;
    for (int i = 0; i < n; ++i) {
        const rt_solve_t h = solves[i];
        if (!valid(h)) return RT_EINVAL;
        if (h->dead) return RT_ESTATE;
        for (int k = 0; k < i; ++k)
            if (solves[k] == h) return RT_EINVAL;
        const Plan &p = h->plan;
        // the batch's march instance, cells in bricks of 8^3 (the tiles)
        if (h->device != b->device || p.bl != 3 || p.species != sh.species || p.mb != sh.mb || p.fp64 != sh.fp64 ||
            p.thermal != sh.thermal || h->d.trace_packets > 0 || p.recomb || h->bg_packets > 0 ||
            (h->d.flags & RT_PERIODIC) || (p.species == 3 && p.mb > 1 && bin_layout(&h->d, p) != 1))
            return RT_EINVAL;
        if (!(isfinite(dt_s[i]) && dt_s[i] > 0.0) || n_packets[i] < 0) return RT_EINVAL;
        const int64_t base = n_packets[i] / h->d.n_sub;
        if (h->n_src > 0 && base < h->n_src) return RT_EINVAL;
        if (base + 1 > ((int64_t)1 << 31)) return RT_EOVERFLOW;
        if (h->d.n_sub > rounds) rounds = h->d.n_sub;
        tiles += (uint64_t)p.geo.nb[0] * p.geo.nb[1] * p.geo.nb[2];
        const uint32_t v = (uint32_t)(p.geo.nb[0] + p.geo.nb[1] + p.geo.nb[2] - 2);
        if (v > passes) passes = v;
    }
    if (tiles > b->lay.max_tiles) return RT_ENOMEM;
    // records: the packets of every round must fit those in flight
    for (int r = 0; r < rounds; ++r) {
        uint64_t tot = 0;
        for (int i = 0; i < n; ++i) {
            const rt_solve_t h = solves[i];
            if (h->n_src == 0 || r >= h->d.n_sub) continue;
            const int64_t base = n_packets[i] / h->d.n_sub, extra = n_packets[i] % h->d.n_sub;
            tot += (uint64_t)(base + (r < extra ? 1 : 0));
        }
        if (tot > b->lay.capacity) return RT_ENOMEM;
    }
    const rtk::BatchLaunch l = batch_launch(b, passes);

    // the table: the previous copy out of the staging memory must have happened
    if (b->staged_pending && hipEventSynchronize(b->staged) != hipSuccess) return RT_EDEVICE;
    rtk::BatchHead *hd = reinterpret_cast<rtk::BatchHead *>(b->staging);
    rtk::BatchSolve *tb = reinterpret_cast<rtk::BatchSolve *>(hd + 1);
    uint64_t cells = 0;
    uint32_t tile0 = 0;
    for (int i = 0; i < n; ++i) {
        const rt_solve_t h = solves[i];
        const Plan &p = h->plan;
        rtk::BatchSolve &t = tb[i];
        memset(&t, 0, sizeof(t));
        t.geo = p.geo;
        t.half_dl = 0.5 * h->d.cell_cm;
        t.dt = dt_s[i] / h->d.n_sub;
        t.tau_kill = h->d.tau_kill;
        t.y_he = h->d.y_he;
        t.cell_cm = h->d.cell_cm;
        t.redshift = h->d.redshift;
        t.seed = seeds[i];
        t.solve_id = h->d.solve_id;
        t.step0 = h->step_index;
        t.packets = h->n_src > 0 ? n_packets[i] : 0;     // without sources only the update runs
        t.src = reinterpret_cast<const rtk::SourceRec *>(h->ws + p.off_src);
        t.src_ndot = reinterpret_cast<const double *>(h->ws + p.off_ndot);
        t.src_sedsum = reinterpret_cast<const double *>(h->ws + p.off_sedsum);
        t.sed = h->ws + p.off_sed;
        t.tab = h->ws + p.off_tab;
        t.state = h->ws + p.off_state;
        t.kappa = h->ws + p.off_kappa;
        t.acc = reinterpret_cast<double *>(h->ws + p.off_acc);
        t.ledger = reinterpret_cast<rtk::StepLedger *>(h->ws + p.off_ledger);
        t.n_sub = h->d.n_sub;
        t.n_src = (int32_t)h->n_src;
        t.n_chem = h->d.n_chem;
        t.acc_stride = p.acc_stride;
        t.cell0 = cells;
        t.tile0 = tile0;
        t.n_tiles = (uint32_t)p.geo.nb[0] * p.geo.nb[1] * p.geo.nb[2];
        cells += p.geo.ncell_pad;
        tile0 += t.n_tiles;
    }
    memset(hd, 0, sizeof(*hd));
    hd->n = n;
    hd->cells = cells;
    hd->tiles = tile0;

    // a solve last stepped by another batch: its stream first waits for that
    // call (this batch's own earlier calls are ordered by its stream)
    for (int i = 0; i < n; ++i) {
        rt_solve_t h = solves[i];
        if (h->after_pending && h->after_stream != b->stream && !order_after_batch(h)) return fail(h);
    }
    // order: each solve's earlier work, the table copy, the fused launches
    // (one event per distinct stream: solves opened on one stream share it)
    int n_in = 0;
    for (int i = 0; i < n; ++i) {
        const hipStream_t s = solves[i]->stream;
        if (s == b->stream) continue;
        bool seen = false;
        for (int k = 0; k < i && !seen; ++k) seen = solves[k]->stream == s;
        if (seen) continue;
        if (hipEventRecord(b->ev_in[n_in], s) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->ev_in[n_in], 0) != hipSuccess)
            return RT_EDEVICE;
        ++n_in;
    }
    if (hipMemcpyAsync(b->ws + b->lay.off_head, b->staging,
                       sizeof(rtk::BatchHead) + (size_t)n * sizeof(rtk::BatchSolve), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess)
        return RT_EDEVICE;
    static_assert(sizeof(rtk::BatchHead) % alignof(rtk::BatchSolve) == 0, "table after the head is misaligned");
    if (hipEventRecord(b->staged, b->stream) != hipSuccess) return RT_EDEVICE;
    b->staged_pending = true;
    if (b->flags & RT_BATCH_GRAPH) {
        hipGraphExec_t exec = nullptr;
        if (batch_graph(b, l, rounds, &exec) != hipSuccess || hipGraphLaunch(exec, b->stream) != hipSuccess)
            return RT_EDEVICE;
    } else if (batch_enqueue(l, rounds) != hipSuccess) {
        return RT_EDEVICE;
    }
    // every solve's ledger, in call order, copied out at once
    rtk::StepLedger *gathered = reinterpret_cast<rtk::StepLedger *>(b->ws + b->lay.off_ledgers);
    if (rtk::launch_batch_gather(l, gathered) != hipSuccess ||
        hipMemcpyAsync(b->ledgers, gathered, (size_t)n * sizeof(rtk::StepLedger), hipMemcpyDeviceToHost,
                       b->stream) != hipSuccess ||
        hipEventRecord(b->done, b->stream) != hipSuccess)
        return RT_EDEVICE;
    b->last.assign(solves, solves + n);
    for (int i = 0; i < n; ++i) {
        rt_solve_t h = solves[i];
        h->step_index += (uint64_t)h->d.n_sub;
        h->timed = 0;
        h->ktimed = 0;
        // the solve's own stream is ordered after the call only when it is next used
        if (h->stream != b->stream) {
            if (hipEventRecord(h->after, b->stream) != hipSuccess) return fail(h);
            h->after_stream = b->stream;
            h->after_pending = true;
        }
    }
    return stats ? rt_batch_wait(b, n, stats) : RT_OK;
}

int32_t rt_batch_wait(rt_batch_t b, int32_t n, rt_step_stats *stats) {
    if (!batch_valid(b) || !stats || n < 0 || (size_t)n != b->last.size()) return RT_EINVAL;
    if (hipEventSynchronize(b->done) != hipSuccess) return RT_EDEVICE;
    int32_t status = RT_OK;
    for (int i = 0; i < n; ++i) {
        const rtk::StepLedger &l = b->ledgers[i];
        rt_step_stats &st = stats[i];
        memset(&st, 0, sizeof(st));
        st.emitted = l.s[0] + l.s[1];
        st.absorbed = l.s[2] + l.s[3];
        st.escaped = l.s[4] + l.s[5];
        st.truncated = l.s[6] + l.s[7];
        st.crossings = (int64_t)l.c[0];
        st.packets = (int64_t)l.c[1];
        st.n_escaped = (int64_t)l.c[2];
        st.n_truncated = (int64_t)l.c[3];
        st.substeps = (int64_t)l.substeps;
        st.nonfinite = l.nonfinite;
        st.errors = l.errors;
        st.diffuse_emitted = l.d_emit;
        st.diffuse_packets = (int64_t)l.d_packets;
        if (l.errors) {
            // (as rt_read_stats: a failed consistency check ends the solve)
            rt_solve_t h = b->last[i];
            if (valid(h)) h->dead = true;
            status = RT_EINTERNAL;
        }
    }
    return status;
}

int32_t rt_batch_release(rt_batch_t b) {
    if (!batch_valid(b)) return RT_EINVAL;
    const bool ok = hipStreamSynchronize(b->stream) == hipSuccess;
    batch_destroy(b);
    return ok ? RT_OK : RT_EDEVICE;
}

const char *rt_strerror(int32_t status) {
    switch (status) {
    case RT_OK: return "ok";
    case RT_EINVAL: return "invalid argument";
    case RT_ENOMEM: return "workspace too small or too many sources";
    case RT_EDEVICE: return "HIP device error; the handle is unusable";
    case RT_ESTATE: return "call not valid in the handle's state";
    case RT_EOVERFLOW: return "size beyond what the library supports";
    case RT_EINTERNAL: return "internal consistency check of the march failed; the handle is unusable";
    case RT_ESCRATCH: return "the solve needs more than the static workspace (RT_STATIC_WORKSPACE_BYTES)";
    default: return "unknown status";
    }
}

}  // extern "C"
