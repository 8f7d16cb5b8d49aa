/*
 * rt_oracle.c -- plain float64 CPU oracle of the Monte-Carlo radiative-transfer
 * hot path (CRASH2 / pCRASH2, Partl et al. 2011, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines what the GPU library must
 * compute; it is slow on purpose and shares no code with the HIP path.  Only
 * the test-suite, the smoke check and the benchmark's CPU-baseline leg may
 * build, load or call it.
 *
 * Within one frozen sub-step (cell state held fixed while packets fly):
 *   1. absorber densities kappa_s per cell from the frozen state (Sec. 2: the
 *      cell optical depth sums the HI, HeI and HeII contributions);
 *   2. every source emits its equal share of the step's packets, each carrying
 *      w photons split over the frequency bins by the source SED (Sec. 2,
 *      coloured packets; Sec. 3.2, N_p/N_t packets per source per step);
 *   3. each packet gets an isotropic direction from a counter-based generator
 *      (Philox4x64-10 replaces the paper's per-CPU SPRNG streams, Sec. 3.3);
 *   4. the packet is followed cell by cell (Sec. 2: path length inside every
 *      crossed cell), using an exact integer traversal;
 *   5. per bin, Eq. (1): the absorbed photons are the transmitted ones times
 *      1 - exp(-tau); they are shared among the species in proportion to
 *      their part of tau (Sec. 2) and added to per-cell accumulators;
 *   6. the packet ends when it leaves the box or is extinguished (Sec. 2),
 *      here: every populated bin has tau >= tau_kill; with periodic boundaries
 *      it re-enters through the opposite face instead of leaving and ends
 *      after a set number of cell faces along one axis;
 *   7. after all packets, every cell's ionisation fractions and temperature
 *      are advanced from the accumulated photons (Sec. 2's network, applied
 *      once per cell per sub-step instead of once per crossing).
 * The physics rates (recombination, collisional, cooling) are a stated
 * reading (the paper lists the processes but gives no rates), pinned by the
 * tests against physical identities, constants and published tables.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_BINS 16

/* thresholds of HI, HeI, HeII (eV) and cgs constants */
static const double ORC_ETH_EV[3] = {13.598434, 24.587387, 54.417760};
static const double ORC_EV = 1.602176634e-12;
static const double ORC_KB = 1.380649e-16;

enum { ORC_ISOTHERMAL = 1, ORC_PERIODIC = 2 };
enum { ORC_SRC_OCTANT = 1 };
enum { ORC_FATE_TRUNC = 1, ORC_FATE_ESCAPE = 2, ORC_FATE_PATH = 3 };

typedef struct {
    int32_t n[3];
    double cell_cm;
    double y_he;                       /* n_He / n_H ; 0 => pure hydrogen */
    int32_t n_bins;
    double e_ev[ORC_MAX_BINS];
    double sigma[3][ORC_MAX_BINS];     /* HI, HeI, HeII cross-sections per bin */
    double redshift;                   /* < 0: no Compton coupling */
    double tau_kill;
    int32_t n_chem;
    uint32_t flags;
    int32_t path_cells;                /* periodic: a packet ends once it has crossed more
                                          than this many cell faces along one axis */
} orc_grid;

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw 2011, SC'11): 10 rounds of     */
/* two 64x64->128 multiplies with a Weyl-sequence key schedule.              */
/* ------------------------------------------------------------------------ */
static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(M0, c[0], &hi0, &lo0);
        mul128(M1, c[2], &hi1, &lo1);
        uint64_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Isotropic integer direction (Sec. 2: emission direction from the source's
 * angular PDF, isotropic here).  Each attempt draws one Philox block keyed by
 * (seed, solve id) at counter (packet id, sub-step index, attempt, stream); the top
 * 21 bits of the first three words give components in [-2^20, 2^20).  The
 * vector is kept if 2^36 <= |c|^2 <= 2^40 (a spherical shell: uniform
 * direction).  After 64 rejections the diagonal (2^19, 2^19, 2^19) is used.
 * A corner (octant) source folds the direction into the positive octant.
 * Returns the number of attempts made. */
int orc_direction_ex(uint64_t seed, uint64_t solve_id, uint64_t g, uint64_t step_index,
                     int octant, uint64_t stream, int32_t c[3])
{
    const uint64_t key[2] = {seed, solve_id};
    for (int attempt = 0; attempt < 64; ++attempt) {
        uint64_t ctr[4] = {g, step_index, (uint64_t)attempt, stream};
        uint64_t r[4];
        orc_philox4x64_10(ctr, key, r);
        int64_t v[3], q = 0;
        for (int a = 0; a < 3; ++a) {
            v[a] = (int64_t)(r[a] >> 43) - (int64_t)(1 << 20);
            q += v[a] * v[a];
        }
        if (q >= ((int64_t)1 << 36) && q <= ((int64_t)1 << 40)) {
            for (int a = 0; a < 3; ++a)
                c[a] = (int32_t)(octant ? llabs(v[a]) : v[a]);
            return attempt + 1;
        }
    }
    c[0] = c[1] = c[2] = 1 << 19;
    return 64;
}

/* Source packets use stream word 0 with their packet id as g; a diffuse
 * (recombination) packet uses stream word 1 with its cell's natural index. */
int orc_direction(uint64_t seed, uint64_t solve_id, uint64_t g, uint64_t step_index,
                  int octant, int32_t c[3])
{
    return orc_direction_ex(seed, solve_id, g, step_index, octant, 0, c);
}

/* ------------------------------------------------------------------------ */
/* Exact integer traversal.  Positions are in half-cell units: cell k spans  */
/* [2k, 2k+2] on each axis; a ray is o + t c, t >= 0.  The next face on axis */
/* a is at t_a = dist_a / |c_a|; axis a is hit before axis b exactly when    */
/* dist_a |c_b| < dist_b |c_a| (integers, exact).  Axes tied at the minimum  */
/* step together, so cells touched with zero length are never visited.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t k[3];      /* current cell */
    int64_t dist[3];   /* |next boundary - o| on each axis (half-cells) */
    int64_t ac[3];     /* |c_a| */
    int sg[3];         /* sign of c_a */
} orc_ray;

static void ray_start(orc_ray *r, const int32_t o[3], const int32_t c[3])
{
    for (int a = 0; a < 3; ++a) {
        r->sg[a] = (c[a] > 0) - (c[a] < 0);
        r->ac[a] = llabs((int64_t)c[a]);
        int64_t oa = o[a];
        /* the cell the ray occupies just after leaving o */
        if (oa % 2 != 0) r->k[a] = (oa - 1) / 2;
        else r->k[a] = (c[a] >= 0) ? oa / 2 : oa / 2 - 1;
        if (c[a] > 0) r->dist[a] = 2 * (r->k[a] + 1) - oa;
        else if (c[a] < 0) r->dist[a] = oa - 2 * r->k[a];
        else r->dist[a] = 0;
    }
}

/* Axis mask of the nearest face(s); *num / *den is its ray parameter. */
static int ray_exit_axes(const orc_ray *r, int64_t *num, int64_t *den)
{
    int best = -1, mask = 0;
    for (int a = 0; a < 3; ++a) {
        if (r->ac[a] == 0) continue;
        if (best < 0) { best = a; mask = 1 << a; continue; }
        uint64_t lhs = (uint64_t)r->dist[a] * (uint64_t)r->ac[best];
        uint64_t rhs = (uint64_t)r->dist[best] * (uint64_t)r->ac[a];
        if (lhs < rhs) { best = a; mask = 1 << a; }
        else if (lhs == rhs) mask |= 1 << a;
    }
    *num = r->dist[best];
    *den = r->ac[best];
    return mask;
}

/* Move across the faces in mask.  Returns 0 inside the grid, otherwise the
 * exit-face code: bit a = left through axis a, bit 3+a = through its + side. */
static int ray_step(orc_ray *r, int mask, const int32_t n[3])
{
    int face = 0;
    for (int a = 0; a < 3; ++a) {
        if (!(mask & (1 << a))) continue;
        r->k[a] += r->sg[a];
        r->dist[a] += 2;
        if (r->k[a] < 0) face |= 1 << a;
        if (r->k[a] >= n[a]) face |= (1 << a) | (8 << a);
    }
    return face;
}

static int64_t cell_index(const int64_t k[3], const int32_t n[3])
{
    return k[0] + (int64_t)n[0] * (k[1] + (int64_t)n[1] * k[2]);
}

/* Cells crossed by one ray; records at most max_len cell indices and exit
 * parameters.  Returns the number of crossed cells; *face gets the exit code.
 * The start point must lie inside the grid or on its boundary. */
int64_t orc_trace_ray(const int32_t n[3], const int32_t o[3], const int32_t c[3],
                      int64_t max_len, int64_t *cells, double *s_exit, int32_t *face)
{
    orc_ray r;
    ray_start(&r, o, c);
    for (int a = 0; a < 3; ++a)
        if (r.k[a] < 0 || r.k[a] >= n[a]) { *face = -1; return 0; }
    int64_t count = 0;
    for (;;) {
        int64_t num, den;
        int mask = ray_exit_axes(&r, &num, &den);
        if (count < max_len) {
            cells[count] = cell_index(r.k, n);
            if (s_exit) s_exit[count] = (double)num / (double)den;
        }
        ++count;
        int f = ray_step(&r, mask, n);
        if (f) { *face = f; return count; }
    }
}

/* ------------------------------------------------------------------------ */
/* Compensated (Neumaier) summation for the photon ledgers.                  */
/* ------------------------------------------------------------------------ */
static void nsum(double *s, double *cmp, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *cmp += (*s - t) + v;
    else *cmp += (v - t) + *s;
    *s = t;
}

/* ledger layout (doubles) */
enum {
    L_EMIT = 0, L_ABS = 2, L_ESC = 4, L_TRUNC = 6,   /* (sum, compensation) pairs */
    L_CROSS = 8, L_NESC = 9, L_NTRUNC = 10, L_PACKETS = 11,
    L_DEMIT = 12,                                    /* diffuse photons emitted (pair, in L_EMIT too) */
    L_DPACKETS = 14, L_SIZE = 16
};

/* Source of packet g when P packets are shared equally by S sources: the first
 * P mod S sources get one packet more (Sec. 2: a source's emission in a step is
 * split over its packets; Sec. 3.2: N_p/N_t packets per source per step). */
static int64_t source_of(int64_t g, int64_t P, int64_t S, int64_t *n_s)
{
    int64_t q = P / S, rem = P % S, s;
    if (g < rem * (q + 1)) s = g / (q + 1);
    else s = rem + (g - rem * (q + 1)) / q;
    *n_s = q + (s < rem ? 1 : 0);
    return s;
}

/* Heat per absorbed photon of bin j by species s [erg]. */
static void heat_table(const orc_grid *G, double heat_ev[3][ORC_MAX_BINS])
{
    for (int s = 0; s < 3; ++s)
        for (int j = 0; j < G->n_bins; ++j)
            heat_ev[s][j] = (G->e_ev[j] - ORC_ETH_EV[s]) * ORC_EV;
}

/*
 * Follow one packet of w photons per unit of sed, starting at o (half-cell
 * units) in direction c, until it is extinguished or leaves the box; deposits
 * go to acc, the packet's end to the ledger (its emission is the caller's).
 * rec, when not NULL, receives the crossed cells and the end (words 0-6).
 */
static void march_packet(const orc_grid *G, const double *kappa, const double heat_ev[3][ORC_MAX_BINS],
                         double w, const double *sed, const int32_t o[3], const int32_t c[3],
                         double *acc, double *ledger, int32_t trace_len, int32_t *rec)
{
    const int64_t ncell = (int64_t)G->n[0] * G->n[1] * G->n[2];
    const int nb = G->n_bins;
    const int pure_h = !(G->y_he > 0.0);
    const int periodic = (G->flags & ORC_PERIODIC) != 0;
    double f[ORC_MAX_BINS], T[ORC_MAX_BINS];
    for (int j = 0; j < nb; ++j) { f[j] = 1.0; T[j] = 0.0; }
    const double len_scale =
        sqrt((double)((int64_t)c[0] * c[0] + (int64_t)c[1] * c[1] + (int64_t)c[2] * c[2]))
        * (0.5 * G->cell_cm);

    orc_ray r;
    ray_start(&r, o, c);
    double s_prev = 0.0;
    int64_t count = 0;
    int fate = 0, face = 0;
    int64_t last = -1;

    for (;;) {
        int64_t num, den;
        int mask = ray_exit_axes(&r, &num, &den);
        const double s_new = (double)num / (double)den;
        const double l = (s_new - s_prev) * len_scale;     /* chord in this cell [cm] */
        const int64_t cell = cell_index(r.k, G->n);
        const double kap[3] = {kappa[cell], pure_h ? 0.0 : kappa[ncell + cell],
                               pure_h ? 0.0 : kappa[2 * ncell + cell]};

        /* Eq. (1) per bin and the split among absorbers */
        double dep[3] = {0.0, 0.0, 0.0}, heat = 0.0, absorbed = 0.0;
        for (int j = 0; j < nb; ++j) {
            if (!(sed[j] > 0.0)) continue;
            double part[3];
            for (int s = 0; s < 3; ++s) part[s] = kap[s] * G->sigma[s][j];
            const double ksum = (part[0] + part[1]) + part[2];
            const double tau = l * ksum;
            /* Eq. (1): absorbed f (1 - e^-tau), transmitted f e^-tau; each
               from its own function (f - d would leave an opaque cell's
               transmitted remainder without a correct digit) */
            const double d = f[j] * (-expm1(-tau));
            f[j] = f[j] * exp(-tau);
            T[j] = T[j] + tau;
            const double nabs = sed[j] * d;
            absorbed += nabs;
            if (ksum > 0.0) {
                for (int s = 0; s < 3; ++s) {
                    const double share = part[s] / ksum;
                    dep[s] += nabs * share;
                    heat += nabs * share * heat_ev[s][j];
                }
            }
        }
        for (int s = 0; s < 3; ++s) acc[s * ncell + cell] += w * dep[s];
        acc[3 * ncell + cell] += w * heat;
        nsum(&ledger[L_ABS], &ledger[L_ABS + 1], w * absorbed);
        ledger[L_CROSS] += 1.0;
        if (rec && count < trace_len) rec[8 + count] = (int32_t)cell;
        ++count;
        last = cell;

        /* extinguished: every populated bin has accumulated tau >= tau_kill */
        double tmin = INFINITY;
        for (int j = 0; j < nb; ++j)
            if (sed[j] > 0.0 && T[j] < tmin) tmin = T[j];
        if (tmin >= G->tau_kill) { fate = ORC_FATE_TRUNC; break; }

        face = ray_step(&r, mask, G->n);
        if (periodic) {
            /* Sec. 2: with periodic boundaries a packet leaving through a face
               comes back through the opposite one; it ends (its photons counted
               as escaped) once it has crossed more than path_cells faces along
               some axis */
            for (int a = 0; a < 3; ++a) {
                if (r.k[a] < 0) r.k[a] += G->n[a];
                else if (r.k[a] >= G->n[a]) r.k[a] -= G->n[a];
            }
            face = 0;
            const int64_t dmax = 2 * (int64_t)G->path_cells + 2;
            if (r.dist[0] > dmax || r.dist[1] > dmax || r.dist[2] > dmax) { fate = ORC_FATE_PATH; break; }
        } else if (face) {
            fate = ORC_FATE_ESCAPE;
            break;
        }
        s_prev = s_new;
    }
    double left = 0.0;
    for (int j = 0; j < nb; ++j) left += sed[j] * f[j];
    if (fate == ORC_FATE_TRUNC) {
        nsum(&ledger[L_TRUNC], &ledger[L_TRUNC + 1], w * left);
        ledger[L_NTRUNC] += 1.0;
    } else {
        nsum(&ledger[L_ESC], &ledger[L_ESC + 1], w * left);
        ledger[L_NESC] += 1.0;
    }
    if (rec) {
        rec[0] = (int32_t)count; rec[1] = fate; rec[2] = face; rec[3] = (int32_t)last;
        rec[4] = c[0]; rec[5] = c[1]; rec[6] = c[2];
    }
}

/*
 * March packets g in [g_begin, g_end) of one frozen sub-step.
 *   kappa : [3][ncell] absorber densities (HI, HeI, HeII), natural order
 *   acc   : [4][ncell] accumulators D_HI, D_HeI, D_HeII (photons), Q (erg)
 *   ledger: see enum above (accumulated, not cleared)
 *   trace : optional, trace_n records of (8 + trace_len) int32; packet ids
 *           g = r * trace_stride (r < trace_n) fill record r: count, fate, face,
 *           last cell, c[3], source, then the crossed cells
 */
void orc_march(const orc_grid *G, const double *kappa,
               int32_t n_src, const int32_t *src_ijk, const double *src_ndot,
               const double *src_sed, uint32_t src_flags,
               double dt, int64_t P, uint64_t seed, uint64_t solve_id, uint64_t step_index,
               int64_t g_begin, int64_t g_end, double *acc, double *ledger,
               int32_t trace_n, int32_t trace_len, int32_t trace_stride, int32_t *trace)
{
    const int nb = G->n_bins;
    const int octant = (src_flags & ORC_SRC_OCTANT) != 0;
    double heat_ev[3][ORC_MAX_BINS];
    heat_table(G, heat_ev);

    for (int64_t g = g_begin; g < g_end; ++g) {
        /* --- emission --- */
        int64_t n_s;
        int64_t src = source_of(g, P, n_src, &n_s);
        double w = src_ndot[src] * dt;
        w = w / (double)n_s;
        if (octant) w = w * 0.125;
        const double *sed = src_sed + src * nb;
        int32_t c[3], o[3];
        orc_direction(seed, solve_id, (uint64_t)g, step_index, octant, c);
        for (int a = 0; a < 3; ++a)
            o[a] = octant ? 2 * src_ijk[3 * src + a] : 2 * src_ijk[3 * src + a] + 1;
        double emitted = 0.0;
        for (int j = 0; j < nb; ++j) emitted += sed[j];
        nsum(&ledger[L_EMIT], &ledger[L_EMIT + 1], w * emitted);
        ledger[L_PACKETS] += 1.0;

        const int64_t stride = trace_stride > 0 ? trace_stride : 1;
        int32_t *rec = (trace && g % stride == 0 && g / stride < trace_n)
                     ? trace + (g / stride) * (8 + trace_len) : NULL;
        march_packet(G, kappa, heat_ev, w, sed, o, c, acc, ledger, trace_len, rec);
        if (rec) rec[7] = (int32_t)src;
    }
}

/* ------------------------------------------------------------------------ */
/* Cell update: ionisation network and temperature (Sec. 2), once per cell   */
/* per frozen sub-step.  Rates follow published fits; see the rates table of */
/* the design notes (case-B recombination of Hui & Gnedin 1997, dielectronic */
/* HeII recombination, collisional ionisation and cooling fits of Cen 1992,  */
/* bremsstrahlung with a temperature-dependent Gaunt factor, Compton         */
/* exchange with the CMB).                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    double a_hii, a_heii, a_heiii;     /* recombination coefficients [cm^3/s] */
    double b_hi, b_hei, b_heii;        /* collisional ionisation [cm^3/s] */
} orc_rates;

void orc_rates_at(double T, orc_rates *r);

static double hg97_hydrogenic(double T, double t_th)
{
    const double lam = 2.0 * t_th / T;
    return 2.753e-14 * pow(lam, 1.5) / pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
}

/* Case A of the same fits: every recombination counted, ground state included. */
static double hg97_hydrogenic_a(double T, double t_th)
{
    const double lam = 2.0 * t_th / T;
    return 1.269e-13 * pow(lam, 1.503) / pow(1.0 + pow(lam / 0.522, 0.470), 1.923);
}

static double heii_dielectronic(double T)
{
    return 1.9e-3 * pow(T, -1.5) * exp(-470000.0 / T) * (1.0 + 0.3 * exp(-94000.0 / T));
}

/* Rates with case-A recombination (used when recombination photons are
 * followed as packets instead of being absorbed on the spot). */
void orc_rates_case_a(double T, orc_rates *r)
{
    orc_rates_at(T, r);
    r->a_hii = hg97_hydrogenic_a(T, 157807.0);
    r->a_heiii = 2.0 * hg97_hydrogenic_a(T, 631515.0);
    r->a_heii = 3.0e-14 * pow(2.0 * 285335.0 / T, 0.654) + heii_dielectronic(T);
}

/* Share of each ion's recombinations that go directly to the ground state and
 * so emit an ionising photon: (alpha_A - alpha_B) / alpha_A of the radiative
 * rates (HeII: over the total with the dielectronic part), at least 0.
 * p = HII, HeII, HeIII. */
void orc_ground_fraction(double T, double p[3])
{
    const double ah_a = hg97_hydrogenic_a(T, 157807.0), ah_b = hg97_hydrogenic(T, 157807.0);
    const double ahe_a = hg97_hydrogenic_a(T, 631515.0), ahe_b = hg97_hydrogenic(T, 631515.0);
    const double r_a = 3.0e-14 * pow(2.0 * 285335.0 / T, 0.654);
    const double r_b = 1.26e-14 * pow(2.0 * 285335.0 / T, 0.750);
    p[0] = (ah_a - ah_b) / ah_a;
    p[1] = (r_a - r_b) / (r_a + heii_dielectronic(T));
    p[2] = (ahe_a - ahe_b) / ahe_a;
    /* the HeII power laws cross below ~70 K, outside the fits' range: no
       ground-state share there */
    for (int i = 0; i < 3; ++i) p[i] = p[i] > 0.0 ? p[i] : 0.0;
}

void orc_rates_at(double T, orc_rates *r)
{
    const double f5 = 1.0 / (1.0 + sqrt(T / 1.0e5));
    r->a_hii = hg97_hydrogenic(T, 157807.0);
    r->a_heiii = 2.0 * hg97_hydrogenic(T, 631515.0);
    r->a_heii = 1.26e-14 * pow(2.0 * 285335.0 / T, 0.750)
              + 1.9e-3 * pow(T, -1.5) * exp(-470000.0 / T) * (1.0 + 0.3 * exp(-94000.0 / T));
    r->b_hi = 5.85e-11 * sqrt(T) * exp(-157809.1 / T) * f5;
    r->b_hei = 2.38e-11 * sqrt(T) * exp(-285335.4 / T) * f5;
    r->b_heii = 5.68e-12 * sqrt(T) * exp(-631515.0 / T) * f5;
}

/* The processes of the cooling function one by one [erg cm^-3 s^-1]:
 *  0 collisional excitation of HI       1 collisional excitation of HeII
 *  2 collisional ionisation of HI       3 ... of HeI       4 ... of HeII
 *  5 recombination of HII               6 ... of HeII      7 ... of HeIII
 *  8 dielectronic recombination of HeII 9 bremsstrahlung (free-free) */
void orc_cooling_terms(double T, double ne, double n_hi, double n_hii,
                       double n_hei, double n_heii, double n_heiii, double t[10])
{
    const double f5 = 1.0 / (1.0 + sqrt(T / 1.0e5));
    const double sT = sqrt(T);
    /* collisional excitation */
    t[0] = 7.50e-19 * exp(-118348.0 / T) * f5 * ne * n_hi;
    t[1] = 5.54e-17 * pow(T, -0.397) * exp(-473638.0 / T) * f5 * ne * n_heii;
    /* collisional ionisation */
    t[2] = 1.27e-21 * sT * exp(-157809.1 / T) * f5 * ne * n_hi;
    t[3] = 9.38e-22 * sT * exp(-285335.4 / T) * f5 * ne * n_hei;
    t[4] = 4.95e-22 * sT * exp(-631515.0 / T) * f5 * ne * n_heii;
    /* recombination */
    const double t3 = pow(T / 1.0e3, -0.2), t6 = 1.0 / (1.0 + pow(T / 1.0e6, 0.7));
    t[5] = 8.70e-27 * sT * t3 * t6 * ne * n_hii;
    t[6] = 1.55e-26 * pow(T, 0.3647) * ne * n_heii;
    t[7] = 3.48e-26 * sT * t3 * t6 * ne * n_heiii;
    /* dielectronic recombination */
    t[8] = 1.24e-13 * pow(T, -1.5) * exp(-470000.0 / T) * (1.0 + 0.3 * exp(-94000.0 / T)) * ne * n_heii;
    /* bremsstrahlung */
    const double lt = log10(T);
    const double gff = 1.1 + 0.34 * exp(-(5.5 - lt) * (5.5 - lt) / 3.0);
    t[9] = 1.42e-27 * gff * sT * (n_hii + n_heii + 4.0 * n_heiii) * ne;
}

/* Radiative and collisional cooling [erg cm^-3 s^-1], Compton excluded: the
 * sum of the terms above in their order. */
double orc_cooling(double T, double ne, double n_hi, double n_hii,
                   double n_hei, double n_heii, double n_heiii)
{
    double t[10];
    orc_cooling_terms(T, ne, n_hi, n_hii, n_hei, n_heii, n_heiii, t);
    double lam = 0.0;
    for (int i = 0; i < 10; ++i) lam += t[i];
    return lam;
}

/* Compton coefficient C(z): Lambda_C = C n_e (T - T_cmb), C = 4 sigma_T a k T_cmb^4 / (m_e c). */
double orc_compton_coeff(double z)
{
    const double sigma_t = 6.6524587321e-25, a_rad = 7.5657e-15;
    const double me_c = 9.1093837015e-28 * 2.99792458e10;
    const double tc = 2.725 * (1.0 + z);
    return 4.0 * sigma_t * a_rad * ORC_KB * tc * tc * tc * tc / me_c;
}

/* Two-level hydrogen with fixed ionisation rate I and recombination rate R
 * over time h: exact exponential approach to I/(I+R).  Each of x_HI, x_HII is
 * advanced from its own value. */
static void solve_h(double *xhi, double *xhii, double I, double R, double h)
{
    const double lam = I + R;
    if (!(lam > 0.0)) return;
    const double e = exp(-lam * h);
    const double hi_eq = R / lam, hii_eq = I / lam;
    *xhi = hi_eq + (*xhi - hi_eq) * e;
    *xhii = hii_eq + (*xhii - hii_eq) * e;
}

/* Three-level helium chain HeI <-> HeII <-> HeIII with fixed rates, exact
 * solution.  Generator M (x' = M x, x = (HeI, HeII, HeIII)):
 *   [ -I1      R2        0  ]
 *   [  I1  -(R2+I2)     R3  ]
 *   [  0      I2       -R3  ]
 * Its non-zero eigenvalues l1, l2 are the roots of l^2 - tr l + det with
 * tr = -(I1+R2+I2+R3) and det = I1 I2 + I1 R3 + R2 R3 (real for a chain).
 * On the zero-sum subspace exp(M h) = c0 + c1 M, so
 *   x(h) = (1 - c0) x_eq + c0 x0 + c1 M x0,
 * with x_eq = (R2 R3, I1 R3, I1 I2) / det the stationary state. */
static void solve_he(double x[3], double I1, double R2, double I2, double R3, double h)
{
    const double tr = -(I1 + R2 + I2 + R3);
    if (!(tr < 0.0)) return;
    const double det = I1 * I2 + I1 * R3 + R2 * R3;
    const double m = 0.5 * tr;
    const double q = sqrt(fmax(m * m - det, 0.0));
    const double l2 = m - q;                 /* most negative */
    const double l1 = det / l2;              /* other root, without cancellation */
    const double e1 = exp(l1 * h);
    const double dl = l1 - l2;
    double c1;
    if (dl * h > 1.0e-3) c1 = (e1 - exp(l2 * h)) / dl;
    else {
        const double u = dl * h;
        c1 = h * exp(0.5 * (l1 + l2) * h) * (1.0 + u * u / 24.0);
    }
    const double c0 = e1 - c1 * l1;
    double eq[3] = {0.0, 0.0, 0.0};
    if (det > 0.0) { eq[0] = R2 * R3 / det; eq[1] = I1 * R3 / det; eq[2] = I1 * I2 / det; }
    const double mx[3] = {-I1 * x[0] + R2 * x[1],
                          I1 * x[0] - (R2 + I2) * x[1] + R3 * x[2],
                          I2 * x[1] - R3 * x[2]};
    for (int i = 0; i < 3; ++i) x[i] = (1.0 - c0) * eq[i] + c0 * x[i] + c1 * mx[i];
}

static double electrons(double nh, double nhe, const double x[5])
{
    return nh * x[1] + nhe * (x[3] + 2.0 * x[4]);
}

static double particles(double nh, double nhe, const double x[5])
{
    return nh * (1.0 + x[1]) + nhe * (1.0 + x[3] + 2.0 * x[4]);
}

static void advance_fractions(double xo[5], const double x[5], const orc_rates *R,
                              const double gam[3], double ne, double h, int he)
{
    for (int i = 0; i < 5; ++i) xo[i] = x[i];
    solve_h(&xo[0], &xo[1], gam[0] + R->b_hi * ne, R->a_hii * ne, h);
    if (he) solve_he(&xo[2], gam[1] + R->b_hei * ne, R->a_heii * ne,
                     gam[2] + R->b_heii * ne, R->a_heiii * ne, h);
}

/* Time integral over h of x_HII along the two-level solution (rates I, R)
 * that took it from x0 to xh: h x_eq + (x0 - xh) / (I + R). */
double orc_hii_time(double x0, double xh, double I, double R, double h)
{
    const double lam = I + R;
    if (!(lam > 0.0)) return h * x0;
    const double v = h * (I / lam) + (x0 - xh) / lam;
    return v > 0.0 ? v : 0.0;
}

/* Time integrals over h of x_HeII and x_HeIII along the chain's solution
 * from x0 to xh (x = HeI, HeII, HeIII): h x_eq + z, where z is the zero-sum
 * solution of M z = xh - x0 (M the generator of solve_he), i.e.
 * z_HeII = (R3 d0 + I1 d2) / det, z_HeIII = (I2 d0 - (I1 + R2) d2) / det. */
void orc_he_ion_time(const double x0[3], const double xh[3], double I1, double R2, double I2,
                     double R3, double h, double out[2])
{
    const double det = I1 * I2 + I1 * R3 + R2 * R3;
    if (!(det > 0.0)) { out[0] = h * x0[1]; out[1] = h * x0[2]; return; }
    const double d0 = xh[0] - x0[0], d2 = xh[2] - x0[2];
    const double z1 = (R3 * d0 + I1 * d2) / det;
    const double z2 = (I2 * d0 - (I1 + R2) * d2) / det;
    const double v1 = h * (I1 * R3 / det) + z1, v2 = h * (I1 * I2 / det) + z2;
    out[0] = v1 > 0.0 ? v1 : 0.0;
    out[1] = v2 > 0.0 ? v2 : 0.0;
}

static void renormalise(double *a, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) { if (a[i] < 0.0) a[i] = 0.0; s += a[i]; }
    if (s > 0.0) for (int i = 0; i < n; ++i) a[i] = a[i] / s;
}

/*
 * One cell, one frozen sub-step of length dt.
 *   acc = (D_HI, D_HeI, D_HeII, Q): photons absorbed by each species and heat.
 * Photo-ionisation rate per absorber: Gamma_s = D_s / (n_s V dt) (rate form).
 * n_chem fixed sub-steps h = dt / n_chem; each: electrons from the current
 * fractions, a predictor with them, a corrector with the mean of the start and
 * predicted electron densities; then the temperature by a linearised implicit
 * energy balance
 *   1.5 k n_tot' T' = 1.5 k n_tot T + h (H + C n_e T_cmb - (Lambda(T)/T) T' - C n_e T'),
 * with H = Q/(V dt) held fixed, Lambda evaluated with the new fractions.
 * fixed != NULL replaces the temperature-dependent rates, no_cool drops
 * every cooling and Compton term (both used only by closed-form tests).
 */
void orc_update_cell_rx(const orc_grid *G, double dt, double nh, double x[5], double *T,
                        const double acc[4], const orc_rates *fixed, int no_cool, int case_a,
                        double rc[3])
{
    const int he = G->y_he > 0.0;
    const double nhe = he ? G->y_he * nh : 0.0;
    const double V = G->cell_cm * G->cell_cm * G->cell_cm;
    const double nabs[3] = {nh * x[0], nhe * x[2], nhe * x[3]};
    double gam[3];
    for (int s = 0; s < 3; ++s)
        gam[s] = (acc[s] > 0.0 && nabs[s] > 0.0) ? acc[s] / (nabs[s] * V * dt) : 0.0;
    const double heat = acc[3] / (V * dt);
    const int iso = (G->flags & ORC_ISOTHERMAL) != 0;
    const int compton = !no_cool && G->redshift >= 0.0;
    const double ccomp = compton ? orc_compton_coeff(G->redshift) : 0.0;
    const double tcmb = 2.725 * (1.0 + (G->redshift > 0.0 ? G->redshift : 0.0));
    const double h = dt / G->n_chem;

    orc_rates R;
    if (fixed) R = *fixed; else if (case_a) orc_rates_case_a(*T, &R); else orc_rates_at(*T, &R);
    for (int m = 0; m < G->n_chem; ++m) {
        if (m > 0 && !fixed && !iso) {                        /* T moved: new rates */
            if (case_a) orc_rates_case_a(*T, &R); else orc_rates_at(*T, &R);
        }
        const double ne0 = electrons(nh, nhe, x);
        double xp[5], xn[5];
        advance_fractions(xp, x, &R, gam, ne0, h, he);
        const double ne_bar = 0.5 * (ne0 + electrons(nh, nhe, xp));
        advance_fractions(xn, x, &R, gam, ne_bar, h, he);
        if (rc) {
            /* recombinations per atom over h (Sec. 2: N_rec is recorded by the
             * network): rate coefficient times the time integral of the ion
             * fraction along the corrector's solution */
            const double rh = R.a_hii * ne_bar;
            rc[0] += rh * orc_hii_time(x[1], xn[1], gam[0] + R.b_hi * ne_bar, rh, h);
            if (he) {
                const double r2 = R.a_heii * ne_bar, r3 = R.a_heiii * ne_bar;
                double tm[2];
                orc_he_ion_time(&x[2], &xn[2], gam[1] + R.b_hei * ne_bar, r2, gam[2] + R.b_heii * ne_bar,
                            r3, h, tm);
                rc[1] += r2 * tm[0];
                rc[2] += r3 * tm[1];
            }
        }
        renormalise(&xn[0], 2);
        if (he) renormalise(&xn[2], 3);
        if (!iso) {
            const double n0 = particles(nh, nhe, x), n1 = particles(nh, nhe, xn);
            const double ne1 = electrons(nh, nhe, xn);
            const double lam = no_cool ? 0.0
                : orc_cooling(*T, ne1, nh * xn[0], nh * xn[1], nhe * xn[2], nhe * xn[3], nhe * xn[4]);
            const double cne = ccomp * ne1;
            double tn = (1.5 * ORC_KB * n0 * (*T) + h * (heat + cne * tcmb))
                      / (1.5 * ORC_KB * n1 + h * (lam / (*T) + cne));
            if (tn < tcmb) tn = tcmb;
            *T = tn;
        }
        for (int i = 0; i < 5; ++i) x[i] = xn[i];
    }
}

void orc_update_cell_ex(const orc_grid *G, double dt, double nh, double x[5], double *T,
                        const double acc[4], const orc_rates *fixed, int no_cool)
{
    orc_update_cell_rx(G, dt, nh, x, T, acc, fixed, no_cool, 0, NULL);
}

void orc_update_cell(const orc_grid *G, double dt, double nh, double x[5], double *T,
                     const double acc[4])
{
    orc_update_cell_ex(G, dt, nh, x, T, acc, NULL, 0);
}

/* Update cells listed in idx (or all cells when idx is NULL) of fields laid
 * out [5][ncell] (fractions) and [ncell] (T), reading acc [4][ncell]. */
void orc_update_cells(const orc_grid *G, double dt, const double *nh, double *x, double *T,
                      const double *acc, int64_t count, const int64_t *idx)
{
    const int64_t ncell = (int64_t)G->n[0] * G->n[1] * G->n[2];
    for (int64_t i = 0; i < count; ++i) {
        const int64_t c = idx ? idx[i] : i;
        double xc[5], a[4];
        for (int f = 0; f < 5; ++f) xc[f] = x[f * ncell + c];
        for (int f = 0; f < 4; ++f) a[f] = acc[f * ncell + c];
        orc_update_cell(G, dt, nh[c], xc, &T[c], a);
        for (int f = 0; f < 5; ++f) x[f * ncell + c] = xc[f];
    }
}

/* Absorber densities of the frozen state: kappa = (n_H x_HI, y n_H x_HeI, y n_H x_HeII). */
void orc_absorbers(const orc_grid *G, const double *nh, const double *x, double *kappa)
{
    const int64_t ncell = (int64_t)G->n[0] * G->n[1] * G->n[2];
    const double y = G->y_he > 0.0 ? G->y_he : 0.0;
    for (int64_t c = 0; c < ncell; ++c) {
        kappa[c] = nh[c] * x[c];
        kappa[ncell + c] = (y * nh[c]) * x[2 * ncell + c];
        kappa[2 * ncell + c] = (y * nh[c]) * x[3 * ncell + c];
    }
}

/* Update with case-A rates and recombination counters rc [3][ncell]
 * (recombinations per atom of HII, HeII, HeIII since the cell last emitted). */
void orc_update_cells_rx(const orc_grid *G, double dt, const double *nh, double *x, double *T,
                         const double *acc, double *rc)
{
    const int64_t ncell = (int64_t)G->n[0] * G->n[1] * G->n[2];
    for (int64_t c = 0; c < ncell; ++c) {
        double xc[5], a[4], r[3];
        for (int f = 0; f < 5; ++f) xc[f] = x[f * ncell + c];
        for (int f = 0; f < 4; ++f) a[f] = acc[f * ncell + c];
        for (int f = 0; f < 3; ++f) r[f] = rc[f * ncell + c];
        orc_update_cell_rx(G, dt, nh[c], xc, &T[c], a, NULL, 0, 1, r);
        for (int f = 0; f < 5; ++f) x[f * ncell + c] = xc[f];
        for (int f = 0; f < 3; ++f) rc[f * ncell + c] = r[f];
    }
}

/* ------------------------------------------------------------------------ */
/* Recombination re-emission (Sec. 2; Sec. 3: pCRASH2 emits when a packet    */
/* crosses a cell whose recombination count has reached f_rec N_a).          */
/* ------------------------------------------------------------------------ */
typedef struct {
    double f_rec;              /* threshold, recombinations per atom */
    int32_t n_t;               /* temperature nodes of the spectrum table (>= 2) */
    double log10_t0, dlog10_t; /* node m sits at log10 T = log10_t0 + m dlog10_t */
    const double *milne;       /* [3][n_t][n_bins] photon fraction per bin of the
                                  ground-state recombination continuum (Milne
                                  spectrum) of HII, HeII, HeIII */
} orc_reemit;

/* Spectrum of ion `ion` at T: linear in log10 T between the table's nodes,
 * clamped to the end nodes. */
void orc_milne_at(const orc_reemit *E, int nb, int ion, double T, double *out)
{
    double u = (log10(T) - E->log10_t0) / E->dlog10_t;
    const double top = (double)(E->n_t - 1);
    if (!(u > 0.0)) u = 0.0;
    if (u > top) u = top;
    int m = (int)floor(u);
    if (m > E->n_t - 2) m = E->n_t - 2;
    const double f = u - (double)m;
    const double *a = E->milne + ((size_t)ion * E->n_t + m) * nb, *b = a + nb;
    for (int j = 0; j < nb; ++j) out[j] = (1.0 - f) * a[j] + f * b[j];
}

/*
 * One sub-step's recombination emission, after the source packets have been
 * marched (their deposits in acc, the crossing test) and before the cell
 * update.  A cell crossed by a source or background packet in this sub-step
 * (some photons deposited in it) emits one diffuse packet holding, for every ion whose
 * counter is positive and at least f_rec, counter x atoms x ground-state share
 * photons with that ion's Milne spectrum at the cell's temperature; those
 * counters restart from zero.  The packet leaves the cell centre in an
 * isotropic direction (stream word 1, g = the cell's natural index) and is
 * marched like a source packet.  Returns the number of diffuse packets.
 */
int64_t orc_reemit_substep(const orc_grid *G, const orc_reemit *E, const double *nh, const double *T,
                           const double *kappa, double *rc, uint64_t seed, uint64_t solve_id,
                           uint64_t step_index, double *acc, double *ledger)
{
    const int64_t ncell = (int64_t)G->n[0] * G->n[1] * G->n[2];
    const int nb = G->n_bins;
    const int ions = G->y_he > 0.0 ? 3 : 1;
    const double y = G->y_he > 0.0 ? G->y_he : 0.0;
    const double V = G->cell_cm * G->cell_cm * G->cell_cm;
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    double *wl = (double *)malloc(sizeof(double) * (size_t)(ncell > 0 ? ncell : 1));
    double *sl = (double *)malloc(sizeof(double) * (size_t)(ncell > 0 ? ncell : 1) * nb);
    int64_t ne = 0;
    /* first every emitter, from the source packets' deposits alone */
    for (int64_t c = 0; c < ncell; ++c) {
        if (!(acc[c] > 0.0 || acc[ncell + c] > 0.0 || acc[2 * ncell + c] > 0.0)) continue;
        double p[3], ph[3] = {0.0, 0.0, 0.0};
        int any = 0;
        orc_ground_fraction(T[c], p);
        const double atoms[3] = {nh[c] * V, (y * nh[c]) * V, (y * nh[c]) * V};
        for (int a = 0; a < ions; ++a) {
            const double r = rc[a * ncell + c];
            if (r > 0.0 && r >= E->f_rec) {
                ph[a] = (r * atoms[a]) * p[a];
                rc[a * ncell + c] = 0.0;
                any = 1;
            }
        }
        const double w = (ph[0] + ph[1]) + ph[2];
        if (!any || !(w > 0.0)) continue;         /* no ionising photon among them: no packet */
        double *sed = sl + ne * nb;
        for (int j = 0; j < nb; ++j) sed[j] = 0.0;
        for (int a = 0; a < ions; ++a) {
            if (!(ph[a] > 0.0)) continue;
            double m[ORC_MAX_BINS];
            orc_milne_at(E, nb, a, T[c], m);
            for (int j = 0; j < nb; ++j) sed[j] += ph[a] * m[j];
        }
        for (int j = 0; j < nb; ++j) sed[j] = sed[j] / w;
        list[ne] = c;
        wl[ne] = w;
        ++ne;
    }
    /* then their packets */
    double heat_ev[3][ORC_MAX_BINS];
    heat_table(G, heat_ev);
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t c = list[e];
        const int64_t k0 = c % G->n[0], k1 = (c / G->n[0]) % G->n[1], k2 = c / ((int64_t)G->n[0] * G->n[1]);
        const int32_t o[3] = {(int32_t)(2 * k0 + 1), (int32_t)(2 * k1 + 1), (int32_t)(2 * k2 + 1)};
        int32_t dir[3];
        orc_direction_ex(seed, solve_id, (uint64_t)c, step_index, 0, 1, dir);
        const double *sed = sl + e * nb;
        double carried = 0.0;
        for (int j = 0; j < nb; ++j) carried += sed[j];
        nsum(&ledger[L_EMIT], &ledger[L_EMIT + 1], wl[e] * carried);
        nsum(&ledger[L_DEMIT], &ledger[L_DEMIT + 1], wl[e] * carried);
        ledger[L_PACKETS] += 1.0;
        ledger[L_DPACKETS] += 1.0;
        march_packet(G, kappa, heat_ev, wl[e], sed, o, dir, acc, ledger, 0, NULL);
    }
    free(list);
    free(wl);
    free(sl);
    return ne;
}

/* ------------------------------------------------------------------------ */
/* Background field (Sec. 2: packets from diffuse fields such as the UV      */
/* background): photons entering the box through its faces.                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double ndot;               /* photons per second entering through the whole boundary */
    const double *sed;         /* [n_bins] photon fraction per bin */
    int64_t packets;           /* packets per step (shared over the sub-steps like source packets) */
} orc_background;

/*
 * Background packet b of a sub-step.  Its boundary cell face is uniform over
 * all 2 (n1 n2 + n0 n2 + n0 n1) faces of boundary cells: Philox block at
 * counter (b, sub-step, 0, 2), word 0 scaled to that count by a 64x64 -> high
 * 64 multiply; faces in the order x-, x+, y-, y+, z-, z+, cells x fastest.
 * It starts at the centre of that face, its direction is the isotropic one of
 * stream word 3 turned inward along the face normal, and, the field being
 * isotropic, its weight carries the cosine to the normal:
 * w = (ndot dt / P) 2 |c_n| / |c| (2 cos theta averages 1 over the hemisphere).
 */
static double background_packet(const orc_grid *G, const orc_background *B, double dt, int64_t P,
                                uint64_t seed, uint64_t solve_id, uint64_t step_index, uint64_t b,
                                int32_t o[3], int32_t c[3])
{
    const int64_t n0 = G->n[0], n1 = G->n[1], n2 = G->n[2];
    const uint64_t faces[6] = {(uint64_t)(n1 * n2), (uint64_t)(n1 * n2), (uint64_t)(n0 * n2),
                               (uint64_t)(n0 * n2), (uint64_t)(n0 * n1), (uint64_t)(n0 * n1)};
    const uint64_t total = 2 * (faces[0] + faces[2] + faces[4]);
    const uint64_t key[2] = {seed, solve_id};
    const uint64_t ctr[4] = {b, step_index, 0, 2};
    uint64_t r[4], hi, lo;
    orc_philox4x64_10(ctr, key, r);
    mul128(r[0], total, &hi, &lo);
    uint64_t idx = hi;
    int f = 0;
    while (idx >= faces[f]) { idx -= faces[f]; ++f; }
    const int axis = f / 2, plus = f % 2;
    const int u = axis == 0 ? 1 : 0, v = axis == 2 ? 1 : 2;       /* the face's two in-plane axes */
    const int64_t a = (int64_t)(idx % (uint64_t)G->n[u]), bb = (int64_t)(idx / (uint64_t)G->n[u]);
    o[axis] = plus ? 2 * G->n[axis] : 0;
    o[u] = (int32_t)(2 * a + 1);
    o[v] = (int32_t)(2 * bb + 1);
    orc_direction_ex(seed, solve_id, b, step_index, 0, 3, c);
    int32_t cn = c[axis] < 0 ? -c[axis] : c[axis];
    if (cn == 0) cn = 1;                        /* never along the face itself */
    c[axis] = plus ? -cn : cn;
    const double q = (double)((int64_t)c[0] * c[0] + (int64_t)c[1] * c[1] + (int64_t)c[2] * c[2]);
    double w = B->ndot * dt;
    w = w / (double)P;
    return w * (2.0 * (double)cn) / sqrt(q);
}

/* Background packet b of a sub-step (start point o in half cells, direction
 * c); returns its weight. */
double orc_background_packet(const orc_grid *G, const orc_background *B, double dt, int64_t P, uint64_t seed,
                             uint64_t solve_id, uint64_t step_index, uint64_t b, int32_t o[3], int32_t c[3])
{
    return background_packet(G, B, dt, P, seed, solve_id, step_index, b, o, c);
}

/* March background packets [0, P) of one sub-step. */
void orc_march_background(const orc_grid *G, const double *kappa, const orc_background *B, double dt,
                          int64_t P, uint64_t seed, uint64_t solve_id, uint64_t step_index,
                          double *acc, double *ledger)
{
    const int nb = G->n_bins;
    double heat_ev[3][ORC_MAX_BINS];
    heat_table(G, heat_ev);
    double carried = 0.0;
    for (int j = 0; j < nb; ++j) carried += B->sed[j];
    for (int64_t b = 0; b < P; ++b) {
        int32_t o[3], c[3];
        const double w = background_packet(G, B, dt, P, seed, solve_id, step_index, (uint64_t)b, o, c);
        nsum(&ledger[L_EMIT], &ledger[L_EMIT + 1], w * carried);
        ledger[L_PACKETS] += 1.0;
        march_packet(G, kappa, heat_ev, w, B->sed, o, c, acc, ledger, 0, NULL);
    }
}

/*
 * One call = n_sub frozen sub-steps of dt / n_sub, the packets shared as
 * evenly as possible (the first P mod n_sub sub-steps get one more).  Each
 * sub-step: absorbers, zeroed accumulators, march of every packet in id order,
 * [with B: the background packets of the sub-step,] [with E: recombination
 * emission, decided from all deposits so far, and the march of its packets,] cell update
 * (with E: case-A rates and the counters rc [3][ncell]).  *step_index is the
 * Philox sub-step counter, advanced once per sub-step.  acc holds the last
 * sub-step's deposits on return; ledger accumulates over all sub-steps; trace
 * (if given) records the last sub-step's source packets.
 * Returns 0, or -1 if some sub-step has fewer packets than sources.
 */
int orc_step_rx(const orc_grid *G, const double *nh, double *x, double *T,
                int32_t n_src, const int32_t *src_ijk, const double *src_ndot,
                const double *src_sed, uint32_t src_flags,
                double dt, int64_t P, int32_t n_sub, uint64_t seed, uint64_t solve_id,
                uint64_t *step_index, double *acc, double *kappa, double *ledger,
                int32_t trace_n, int32_t trace_len, int32_t trace_stride, int32_t *trace,
                const orc_reemit *E, double *rc, const orc_background *B)
{
    const int64_t ncell = (int64_t)G->n[0] * G->n[1] * G->n[2];
    if (n_src > 0 && P / n_sub < n_src) return -1;
    const double dts = dt / n_sub;
    for (int32_t i = 0; i < n_sub; ++i) {
        const int64_t Pi = P / n_sub + (i < P % n_sub ? 1 : 0);
        orc_absorbers(G, nh, x, kappa);
        memset(acc, 0, sizeof(double) * 4 * ncell);
        if (n_src > 0)
            orc_march(G, kappa, n_src, src_ijk, src_ndot, src_sed, src_flags, dts, Pi,
                      seed, solve_id, *step_index, 0, Pi, acc, ledger, trace_n, trace_len,
                      trace_stride, trace);
        if (B && B->packets > 0) {
            const int64_t Pb = B->packets / n_sub + (i < B->packets % n_sub ? 1 : 0);
            if (Pb > 0)
                orc_march_background(G, kappa, B, dts, Pb, seed, solve_id, *step_index, acc, ledger);
        }
        if (E) {
            orc_reemit_substep(G, E, nh, T, kappa, rc, seed, solve_id, *step_index, acc, ledger);
            orc_update_cells_rx(G, dts, nh, x, T, acc, rc);
        } else {
            orc_update_cells(G, dts, nh, x, T, acc, ncell, NULL);
        }
        *step_index += 1;
    }
    return 0;
}

int orc_step(const orc_grid *G, const double *nh, double *x, double *T,
             int32_t n_src, const int32_t *src_ijk, const double *src_ndot,
             const double *src_sed, uint32_t src_flags,
             double dt, int64_t P, int32_t n_sub, uint64_t seed, uint64_t solve_id,
             uint64_t *step_index, double *acc, double *kappa, double *ledger,
             int32_t trace_n, int32_t trace_len, int32_t trace_stride, int32_t *trace)
{
    return orc_step_rx(G, nh, x, T, n_src, src_ijk, src_ndot, src_sed, src_flags, dt, P, n_sub, seed,
                       solve_id, step_index, acc, kappa, ledger, trace_n, trace_len, trace_stride, trace,
                       NULL, NULL, NULL);
}
