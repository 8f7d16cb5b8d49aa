// rt_cells.hip -- per-cell kernels around the packet march: the frozen-state
// absorber table, the float64 ionisation/temperature update (Partl et al.
// 2011, Sec. 2: network for HI, HeI, HeII and the temperature with
// photo-heating and the change in free particles), layout conversion between
// natural order and bricks, the photon ledger and a geometric ray tracer.
#include <hip/hip_runtime.h>
#include <math.h>
#include <type_traits>

#include "rt_device.h"
#include "rt_internal.h"
#include "rt_recomb.h"

namespace rtk {

constexpr int kCellBlock = 256;

template <typename R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };

static inline int cell_blocks(uint64_t n) {
    const uint64_t b = (n + kCellBlock - 1) / kCellBlock;
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

// ---------------------------------------------------------------------------
// Absorber densities of the frozen state, accumulators cleared, march queue
// reset: kappa = (n_H x_HI, (y n_H) x_HeI, (y n_H) x_HeII).
// ---------------------------------------------------------------------------
template <typename R, int S>
__device__ __forceinline__ void prep_slot(uint32_t np, const R *__restrict__ st, void *__restrict__ kappa,
                                          double *__restrict__ acc, int acc_stride, double y_he, uint32_t s) {
    const double nh = (double)st[s];
    const double xhi = (double)st[(size_t)np + s];
    if (S == 1) {
        reinterpret_cast<R *>(kappa)[s] = (R)(nh * xhi);
    } else {
        const double yn = y_he * nh;
        typename V4<R>::T v;
        v.x = (R)(nh * xhi);
        v.y = (R)(yn * (double)st[3 * (size_t)np + s]);
        v.z = (R)(yn * (double)st[4 * (size_t)np + s]);
        v.w = R(0);
        reinterpret_cast<typename V4<R>::T *>(kappa)[s] = v;
    }
    double *a = acc + (size_t)s * acc_stride;
    for (int i = 0; i < acc_stride; ++i) a[i] = 0.0;
}

template <typename R, int S>
__global__ void __launch_bounds__(kCellBlock) k_prep(GridGeom G, const R *__restrict__ st,
                                                     void *__restrict__ kappa, double *__restrict__ acc,
                                                     int acc_stride, double y_he, unsigned long long *queue) {
    const uint32_t np = G.ncell_pad;
    const uint32_t step = gridDim.x * blockDim.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0ull;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < np; s += step)
        prep_slot<R, S>(np, st, kappa, acc, acc_stride, y_he, s);
}

// ---------------------------------------------------------------------------
// Rates (cgs).  Recombination: case B of Hui & Gnedin (1997) for HII and
// HeIII (the hydrogenic form scaled by Z = 2), their HeII fit plus dielectronic
// recombination (case A of the same fits when recombination photons are
// followed as packets); collisional ionisation and cooling after Cen (1992);
// bremsstrahlung with a temperature-dependent Gaunt factor; Compton exchange
// with the CMB.
// ---------------------------------------------------------------------------
struct Rates {
    double rec_hii, rec_heii, rec_heiii;   // cm^3 / s
    double col_hi, col_hei, col_heii;      // cm^3 / s
};

// Factors of T that the rates and the cooling of one chemistry sub-step share
// (evaluated once; each rate multiplies them in the order its formula is
// written).  Powers of T: where the update counts recombinations (`exact`,
// case-A rates) pow, as the formulas are written -- the counters' time
// integral of x_HII cancels strongly in some cells, and pow keeps them equal
// to the plain formulas' to the last bit; otherwise exp(a ln T) from one ln T,
// within 5e-15 of pow at half the update's cost (pow is two float64
// transcendentals in one).
struct TFac {
    double damp, rt, e_hi, e_hei, e_heii;   // 1/(1+sqrt(T/1e5)), sqrt(T), exp(-T_X/T)
    double p15, e470, e94;                  // T^-1.5, exp(-470000/T), 1 + 0.3 exp(-94000/T)
    double lt;                              // ln T (not formed when EXACT)
};

// HE false (pure hydrogen): the helium factors are not formed (left 0).
template <bool EXACT, bool HE = true>
__device__ __forceinline__ TFac tfac(double T) {
    TFac f;
    f.lt = EXACT ? 0.0 : log(T);
    f.damp = 1.0 / (1.0 + sqrt(T * 1.0e-5));
    f.rt = sqrt(T);
    f.e_hi = exp(-157809.1 / T);
    f.e_hei = f.e_heii = f.p15 = f.e470 = f.e94 = 0.0;
    if constexpr (HE) {
        f.e_hei = exp(-285335.4 / T);
        f.e_heii = exp(-631515.0 / T);
        f.p15 = EXACT ? pow(T, -1.5) : exp(-1.5 * f.lt);
        f.e470 = exp(-470000.0 / T);
        f.e94 = 1.0 + 0.3 * exp(-94000.0 / T);
    }
    return f;
}

// Case A with pow (recombination counting, EXACT) or case B from ln T.  HE
// false (pure hydrogen): the helium rates are not formed (left 0).
template <bool EXACT, bool HE = true>
__device__ Rates rates_at(double T, const TFac &f) {
    constexpr bool case_a = EXACT;
    Rates r;
    const double damp = f.damp;
    const double rt = f.rt;
    r.rec_heii = r.rec_heiii = r.col_hei = r.col_heii = 0.0;
    const double diel = HE ? 1.9e-3 * f.p15 * f.e470 * f.e94 : 0.0;
    if (case_a) {
        r.rec_hii = hydrogenic_casea(T, 157807.0);
        if constexpr (HE) {
            r.rec_heiii = 2.0 * hydrogenic_casea(T, 631515.0);
            r.rec_heii = heii_rad_casea(T) + diel;
        }
    } else {
        // lambda^1.5 / (1 + (lambda / 2.740)^0.407)^2.242 with ln lambda = ln 2 T_ion - ln T
        const double lh = 12.662275226919286 - f.lt, lhe = 14.049024154019651 - f.lt;   // ln 2 x 157807, 631515
        r.rec_hii = 2.753e-14 * exp(1.5 * lh - 2.242 * log1p(exp(0.407 * (lh - 1.007957920399979))));  // ln 2.740
        if constexpr (HE) {
            r.rec_heiii = 2.0 * (2.753e-14 * exp(1.5 * lhe - 2.242 * log1p(exp(0.407 * (lhe - 1.007957920399979)))));
            r.rec_heii = 1.26e-14 * exp(0.750 * (13.254566388120152 - f.lt)) + diel;                     // ln 570670
        }
    }
    r.col_hi = 5.85e-11 * rt * f.e_hi * damp;
    if constexpr (HE) {
        r.col_hei = 2.38e-11 * rt * f.e_hei * damp;
        r.col_heii = 5.68e-12 * rt * f.e_heii * damp;
    }
    return r;
}

// Cooling [erg cm^-3 s^-1] without the Compton term.  HE false: no helium
// (its densities are 0, and the terms proportional to them are left out).
template <bool EXACT, bool HE = true>
__device__ double cooling_rate(double T, const TFac &f, double ne, double n_hi, double n_hii, double n_hei,
                               double n_heii, double n_heiii) {
    const double damp = f.damp;
    const double rt = f.rt;
    const double e_hi = f.e_hi, e_hei = f.e_hei, e_heii = f.e_heii;
    constexpr bool ex = EXACT;
    const double t3 = ex ? pow(T * 1.0e-3, -0.2) : exp(-0.2 * (f.lt - 6.907755278982137));          // ln 1e3
    const double t6 = 1.0 / (1.0 + (ex ? pow(T * 1.0e-6, 0.7) : exp(0.7 * (f.lt - 13.815510557964274))));  // ln 1e6
    const double lg = ex ? log10(T) : f.lt * 0.43429448190325176;                                      // 1 / ln 10
    const double gaunt = 1.1 + 0.34 * exp(-(5.5 - lg) * (5.5 - lg) / 3.0);
    double per_ne_hi = 7.50e-19 * exp(-118348.0 / T) * damp      // excitation
                     + 1.27e-21 * rt * e_hi * damp;              // ionisation
    if constexpr (!HE) {
        // the sum below without its helium terms (their densities are 0)
        return ne * (per_ne_hi * n_hi + 8.70e-27 * rt * t3 * t6 * n_hii + 1.42e-27 * gaunt * rt * n_hii);
    }
    double per_ne_heii = 5.54e-17 * (ex ? pow(T, -0.397) : exp(-0.397 * f.lt)) * exp(-473638.0 / T) * damp
                       + 4.95e-22 * rt * e_heii * damp
                       + 1.55e-26 * (ex ? pow(T, 0.3647) : exp(0.3647 * f.lt))                // recombination
                       + 1.24e-13 * f.p15 * f.e470 * f.e94;
    double lam = ne * (per_ne_hi * n_hi + per_ne_heii * n_heii
                       + 9.38e-22 * rt * e_hei * damp * n_hei
                       + 8.70e-27 * rt * t3 * t6 * n_hii
                       + 3.48e-26 * rt * t3 * t6 * n_heiii
                       + 1.42e-27 * gaunt * rt * (n_hii + n_heii + 4.0 * n_heiii));
    return lam;
}

// Ionisation fractions over time h with fixed rates.  Hydrogen: exact two-level
// exponential (each fraction from its own value).  Helium: the three-level
// chain's exact solution, x(h) = (1-c0) x_eq + c0 x0 + c1 M x0, where c0, c1
// come from the two non-zero eigenvalues of the generator M.
struct Frac { double hi, hii, hei, heii, heiii; };

// EXACT (recombination counting): the divisions as the formulas write them
// (the counters' integrals cancel strongly and follow these values to the
// last bit); else one reciprocal per denominator.
template <bool EXACT>
__device__ void evolve(Frac &x, const Frac &x0, const Rates &r, const double gam[3], double ne,
                       double h, bool he) {
    {
        const double ion = gam[0] + r.col_hi * ne, rec = r.rec_hii * ne;
        const double lam = ion + rec;
        if (lam > 0.0) {
            const double e = exp(-lam * h);
            double eq_hi, eq_hii;
            if constexpr (EXACT) {
                eq_hi = rec / lam;
                eq_hii = ion / lam;
            } else {
                const double il = 1.0 / lam;
                eq_hi = rec * il;
                eq_hii = ion * il;
            }
            x.hi = eq_hi + (x0.hi - eq_hi) * e;
            x.hii = eq_hii + (x0.hii - eq_hii) * e;
        } else {
            x.hi = x0.hi;
            x.hii = x0.hii;
        }
    }
    x.hei = x0.hei; x.heii = x0.heii; x.heiii = x0.heiii;
    if (!he) return;
    const double i1 = gam[1] + r.col_hei * ne, r2 = r.rec_heii * ne;
    const double i2 = gam[2] + r.col_heii * ne, r3 = r.rec_heiii * ne;
    const double sum = i1 + r2 + i2 + r3;
    if (!(sum > 0.0)) return;
    const double det = i1 * i2 + i1 * r3 + r2 * r3;
    const double half = -0.5 * sum;
    const double disc = half * half - det;
    const double lb = half - sqrt(disc > 0.0 ? disc : 0.0);   // most negative eigenvalue
    const double la = det / lb;                              // the other one
    const double ea = exp(la * h);
    const double gap = la - lb;
    double c1;
    if (gap * h > 1.0e-3) {
        c1 = (ea - exp(lb * h)) / gap;
    } else {
        const double u = gap * h;
        c1 = h * exp(0.5 * (la + lb) * h) * (1.0 + u * u / 24.0);
    }
    const double c0 = ea - c1 * la;
    double q1 = 0.0, q2 = 0.0, q3 = 0.0;
    if (det > 0.0) {
        if constexpr (EXACT) {
            q1 = r2 * r3 / det; q2 = i1 * r3 / det; q3 = i1 * i2 / det;
        } else {
            const double id = 1.0 / det;
            q1 = r2 * r3 * id; q2 = i1 * r3 * id; q3 = i1 * i2 * id;
        }
    }
    const double m1 = -i1 * x0.hei + r2 * x0.heii;
    const double m2 = i1 * x0.hei - (r2 + i2) * x0.heii + r3 * x0.heiii;
    const double m3 = i2 * x0.heii - r3 * x0.heiii;
    x.hei = (1.0 - c0) * q1 + c0 * x0.hei + c1 * m1;
    x.heii = (1.0 - c0) * q2 + c0 * x0.heii + c1 * m2;
    x.heiii = (1.0 - c0) * q3 + c0 * x0.heiii + c1 * m3;
}

// Constants of one solve's cell update for a sub-step of length dt.
struct UpdateConst {
    double V, kb, tcmb, ccomp, h;
    __device__ __forceinline__ UpdateConst(double cell_cm, double dt, double redshift, int n_chem) {
        V = cell_cm * cell_cm * cell_cm;
        kb = 1.380649e-16;
        const bool compton = redshift >= 0.0;
        tcmb = 2.725 * (1.0 + (redshift > 0.0 ? redshift : 0.0));
        // 4 sigma_T a_rad k T_cmb^4 / (m_e c)
        ccomp = compton ? 4.0 * 6.6524587321e-25 * 7.5657e-15 * kb * (tcmb * tcmb) * (tcmb * tcmb)
                              / (9.1093837015e-28 * 2.99792458e10)
                        : 0.0;
        h = dt / n_chem;
    }
};

// Rates of the last temperature a thread evaluated them at (isothermal
// updates: they depend on T alone, so a thread's next cell at the same T
// takes them as they are, bit for bit).
struct RateCache {
    double T = -1.0;
    Rates r;
};

// The update of slot s (padding slots outside the grid are left alone); bad is
// set when a result is not finite.  rc non-null: case-A rates, and the
// recombinations per atom of each ion over the sub-step are added to its
// counters (rate times the time integral of the ion fraction along the
// corrector's solution).
// CNT: count the recombinations into rc (re-emission; case-A rates, pow).
template <typename R, int S, bool TH, bool CNT>
__device__ __forceinline__ void update_slot(const GridGeom &G, R *__restrict__ st, const double *__restrict__ acc,
                                            int acc_stride, double y_he, double dt, int n_chem,
                                            const UpdateConst &u, uint32_t s, unsigned int &bad,
                                            RateCache &cache, double *__restrict__ rc = nullptr) {
    constexpr bool he = (S == 3);
    const uint32_t np = G.ncell_pad;
    const double V = u.V, kb = u.kb, tcmb = u.tcmb, ccomp = u.ccomp, h = u.h;
    {
        int i, j, k;
        if (!slot_cell(G, s, i, j, k)) return;
        const double nh = (double)st[s];
        const double nhe = he ? y_he * nh : 0.0;
        Frac x;
        x.hi = (double)st[(size_t)np + s];
        x.hii = (double)st[2 * (size_t)np + s];
        x.hei = (double)st[3 * (size_t)np + s];
        x.heii = (double)st[4 * (size_t)np + s];
        x.heiii = (double)st[5 * (size_t)np + s];
        double T = (double)st[6 * (size_t)np + s];
        const double *a = acc + (size_t)s * acc_stride;
        const double dep[3] = {a[0], he ? a[1] : 0.0, he ? a[2] : 0.0};
        const double qheat = TH ? a[he ? 3 : 1] : 0.0;
        const double absorbers[3] = {nh * x.hi, nhe * x.hei, nhe * x.heii};
        double gam[3];
        for (int q = 0; q < 3; ++q)
            gam[q] = (dep[q] > 0.0 && absorbers[q] > 0.0) ? dep[q] / (absorbers[q] * V * dt) : 0.0;
        const double heat = qheat / (V * dt);
        constexpr bool count = CNT;
        double n_rec[3] = {0.0, 0.0, 0.0};
        if (count)
            for (int q = 0; q < S; ++q) n_rec[q] = rc[(size_t)q * np + s];
        TFac tf;
        Rates r;
        if constexpr (TH) {
            tf = tfac<CNT, he>(T);
            r = rates_at<CNT, he>(T, tf);
        } else {
            if (!(T == cache.T)) {
                cache.r = rates_at<CNT, he>(T, tfac<CNT, he>(T));
                cache.T = T;
            }
            r = cache.r;
        }
        for (int m = 0; m < n_chem; ++m) {
            if (TH && m > 0) {
                tf = tfac<CNT, he>(T);
                r = rates_at<CNT, he>(T, tf);
            }
            const double ne0 = nh * x.hii + nhe * (x.heii + 2.0 * x.heiii);
            Frac xp, xn;
            evolve<CNT>(xp, x, r, gam, ne0, h, he);
            const double ne_bar = 0.5 * (ne0 + (nh * xp.hii + nhe * (xp.heii + 2.0 * xp.heiii)));
            evolve<CNT>(xn, x, r, gam, ne_bar, h, he);
            if (count) {
                const double rh = r.rec_hii * ne_bar;
                n_rec[0] += rh * hii_time(x.hii, xn.hii, gam[0] + r.col_hi * ne_bar, rh, h);
                if (he) {
                    const double r2 = r.rec_heii * ne_bar, r3 = r.rec_heiii * ne_bar;
                    double t2, t3;
                    he_ion_time(x.hei, x.heii, x.heiii, xn.hei, xn.heii, xn.heiii, gam[1] + r.col_hei * ne_bar, r2,
                                gam[2] + r.col_heii * ne_bar, r3, h, t2, t3);
                    n_rec[1] += r2 * t2;
                    n_rec[2] += r3 * t3;
                }
            }
            // clamp and renormalise each element's fractions
            xn.hi = fmax(xn.hi, 0.0); xn.hii = fmax(xn.hii, 0.0);
            const double sh = xn.hi + xn.hii;
            if (sh > 0.0) {
                if constexpr (CNT) {
                    xn.hi = xn.hi / sh; xn.hii = xn.hii / sh;
                } else {
                    const double is = 1.0 / sh;
                    xn.hi = xn.hi * is; xn.hii = xn.hii * is;
                }
            }
            if (he) {
                xn.hei = fmax(xn.hei, 0.0); xn.heii = fmax(xn.heii, 0.0); xn.heiii = fmax(xn.heiii, 0.0);
                const double she = (xn.hei + xn.heii) + xn.heiii;
                if (she > 0.0) {
                    if constexpr (CNT) {
                        xn.hei = xn.hei / she; xn.heii = xn.heii / she; xn.heiii = xn.heiii / she;
                    } else {
                        const double is = 1.0 / she;
                        xn.hei = xn.hei * is; xn.heii = xn.heii * is; xn.heiii = xn.heiii * is;
                    }
                }
            }
            if (TH) {
                const double ntot0 = nh * (1.0 + x.hii) + nhe * (1.0 + x.heii + 2.0 * x.heiii);
                const double ntot1 = nh * (1.0 + xn.hii) + nhe * (1.0 + xn.heii + 2.0 * xn.heiii);
                const double ne1 = nh * xn.hii + nhe * (xn.heii + 2.0 * xn.heiii);
                const double lam = cooling_rate<CNT, he>(T, tf, ne1, nh * xn.hi, nh * xn.hii, nhe * xn.hei,
                                                nhe * xn.heii, nhe * xn.heiii);
                const double cne = ccomp * ne1;
                double tn = (1.5 * kb * ntot0 * T + h * (heat + cne * tcmb))
                          / (1.5 * kb * ntot1 + h * (lam / T + cne));
                T = tn < tcmb ? tcmb : tn;
            }
            x = xn;
        }
        const double vals[6] = {x.hi, x.hii, x.hei, x.heii, x.heiii, T};
        for (int q = 0; q < 6; ++q) {
            if (!isfinite(vals[q])) bad = 1;
            st[(size_t)(q + 1) * np + s] = (R)vals[q];
        }
        if (count)
            for (int q = 0; q < S; ++q) {
                if (!isfinite(n_rec[q])) bad = 1;
                rc[(size_t)q * np + s] = n_rec[q];
            }
    }
}

template <typename R, int S, bool TH>
__global__ void __launch_bounds__(kCellBlock, (TH ? 3 : 4)) k_update(GridGeom G, R *__restrict__ st, const double *__restrict__ acc,
                                                       int acc_stride, double y_he, double cell_cm, double dt,
                                                       double redshift, int n_chem, StepLedger *ledger,
                                                       double *__restrict__ rc) {
    const uint32_t np = G.ncell_pad;
    const uint32_t stride = gridDim.x * blockDim.x;
    const UpdateConst u(cell_cm, dt, redshift, n_chem);
    unsigned int bad = 0;
    RateCache cache;
    if (rc != nullptr) {
        for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < np; s += stride)
            update_slot<R, S, TH, true>(G, st, acc, acc_stride, y_he, dt, n_chem, u, s, bad, cache, rc);
    } else {
        for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < np; s += stride)
            update_slot<R, S, TH, false>(G, st, acc, acc_stride, y_he, dt, n_chem, u, s, bad, cache);
    }
    if (bad) atomicOr(&ledger->nonfinite, 1u);
}

// ---------------------------------------------------------------------------
// Layout conversion (natural order <-> bricks)
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_fill_zero(R *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = R(0);
}

template <typename R, typename In>
__global__ void __launch_bounds__(kCellBlock) k_import(GridGeom G, R *__restrict__ st, const In *__restrict__ nh,
                                                       const In *__restrict__ x, const In *__restrict__ t,
                                                       uint32_t ncell) {
    const uint32_t np = G.ncell_pad;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
        const int i = (int)(c % (uint32_t)G.n[0]);
        const int j = (int)((c / (uint32_t)G.n[0]) % (uint32_t)G.n[1]);
        const int k = (int)(c / ((uint32_t)G.n[0] * (uint32_t)G.n[1]));
        const uint32_t s = cell_slot(G, i, j, k);
        st[s] = (R)nh[c];
        for (int f = 0; f < 5; ++f) st[(size_t)(f + 1) * np + s] = (R)x[(size_t)f * ncell + c];
        st[6 * (size_t)np + s] = (R)t[c];
    }
}

// Recombination counters from natural order (src null: all zero).
template <typename In>
__global__ void __launch_bounds__(kCellBlock) k_import_rc(GridGeom G, double *__restrict__ rc,
                                                          const In *__restrict__ src, int species, uint32_t ncell) {
    const uint32_t np = G.ncell_pad;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
        const int i = (int)(c % (uint32_t)G.n[0]);
        const int j = (int)((c / (uint32_t)G.n[0]) % (uint32_t)G.n[1]);
        const int k = (int)(c / ((uint32_t)G.n[0] * (uint32_t)G.n[1]));
        const uint32_t s = cell_slot(G, i, j, k);
        for (int q = 0; q < species; ++q) rc[(size_t)q * np + s] = src ? (double)src[(size_t)q * ncell + c] : 0.0;
    }
}

template <typename R, typename Out>
__global__ void __launch_bounds__(kCellBlock) k_export(GridGeom G, const R *__restrict__ st,
                                                       const double *__restrict__ acc, int acc_stride,
                                                       int species, int thermal, uint32_t mask,
                                                       Out *__restrict__ dst, uint32_t ncell,
                                                       const double *__restrict__ rc) {
    const uint32_t np = G.ncell_pad;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x) {
        const int i = (int)(c % (uint32_t)G.n[0]);
        const int j = (int)((c / (uint32_t)G.n[0]) % (uint32_t)G.n[1]);
        const int k = (int)(c / ((uint32_t)G.n[0] * (uint32_t)G.n[1]));
        const uint32_t s = cell_slot(G, i, j, k);
        int out = 0;
        for (int f = 0; f < 14; ++f) {
            if (!(mask & (1u << f))) continue;
            double v;
            if (f < 7) {
                v = (double)st[(size_t)f * np + s];
            } else if (f >= 11) {
                v = (rc && f - 11 < species) ? rc[(size_t)(f - 11) * np + s] : 0.0;
            } else {
                const double *a = acc + (size_t)s * acc_stride;
                if (species == 3) v = (f < 10 || thermal) ? a[f - 7] : 0.0;
                else v = (f == 7) ? a[0] : ((f == 10 && thermal) ? a[1] : 0.0);
            }
            dst[(size_t)out * ncell + c] = (Out)v;
            ++out;
        }
    }
}

// ---------------------------------------------------------------------------
// Ledger: per-block slots of the march summed (TwoSum) into the step ledger.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void zero_ledger(StepLedger *l) {
    StepLedger z;
    for (int i = 0; i < 8; ++i) z.s[i] = 0.0;
    for (int i = 0; i < 4; ++i) z.c[i] = 0ull;
    z.substeps = 0ull;
    z.nonfinite = 0u;
    z.errors = 0u;
    z.d_emit = 0.0;
    z.d_packets = 0ull;
    *l = z;
}

__global__ void k_ledger_zero(StepLedger *l) {
    if (threadIdx.x == 0) zero_ledger(l);
}

// One wavefront adds n per-block slots into a step ledger: lane-strided
// partial sums, then a TwoSum tree; the sub-step counter moves by one.
__device__ __forceinline__ void reduce_slots(const LedgerSlot *slots, int n, StepLedger *l) {
    const int lane = threadIdx.x & 63;
    double s[8];
    unsigned long long c[4] = {0, 0, 0, 0};
    for (int i = 0; i < 8; ++i) s[i] = 0.0;
    for (int b = lane; b < n; b += 64) {
        for (int i = 0; i < 4; ++i) {
            double t, e;
            two_sum(s[2 * i], slots[b].s[2 * i], t, e);
            s[2 * i] = t;
            s[2 * i + 1] += slots[b].s[2 * i + 1] + e;
        }
        for (int i = 0; i < 4; ++i) c[i] += slots[b].c[i];
    }
    for (int off = 32; off >= 1; off >>= 1) {
        for (int i = 0; i < 4; ++i) {
            const double so = __shfl_xor(s[2 * i], off), co = __shfl_xor(s[2 * i + 1], off);
            double t, e;
            two_sum(s[2 * i], so, t, e);
            s[2 * i] = t;
            s[2 * i + 1] += co + e;
        }
        for (int i = 0; i < 4; ++i) c[i] += __shfl_xor(c[i], off);
    }
    if (lane == 0) {
        for (int i = 0; i < 4; ++i) {
            double t, e;
            two_sum(l->s[2 * i], s[2 * i], t, e);
            l->s[2 * i] = t;
            l->s[2 * i + 1] += s[2 * i + 1] + e;
            l->c[i] += c[i];
        }
        l->substeps += 1ull;
    }
}

__global__ void __launch_bounds__(64) k_ledger_reduce(const LedgerSlot *slots, int n, StepLedger *l) {
    reduce_slots(slots, n, l);
}

// Sub-step without packets: only the sub-step counter of the ledger moves.
__global__ void k_ledger_tick(StepLedger *l) {
    if (threadIdx.x == 0) l->substeps += 1ull;
}

// ---------------------------------------------------------------------------
// Geometric ray tracer: the march's traversal without the physics.
// ---------------------------------------------------------------------------
__global__ void k_trace_rays(GridGeom G, int m, const int32_t *o, const int32_t *c, int max_len,
                             int32_t *cells, int32_t *count, int32_t *face) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    int k[3];
    uint32_t d[3], a[3];
    int sg[3];
    bool bad = false;
    for (int ax = 0; ax < 3; ++ax) {
        const int oa = o[3 * r + ax], ca = c[3 * r + ax];
        sg[ax] = (ca > 0) - (ca < 0);
        a[ax] = (uint32_t)abs(ca);
        k[ax] = (oa & 1) ? (oa - 1) / 2 : (ca >= 0 ? oa / 2 : oa / 2 - 1);
        d[ax] = ca > 0 ? (uint32_t)(2 * (k[ax] + 1) - oa) : (ca < 0 ? (uint32_t)(oa - 2 * k[ax]) : 1u);
        if (k[ax] < 0 || k[ax] >= G.n[ax]) bad = true;
    }
    if (bad || (a[0] | a[1] | a[2]) == 0u) { count[r] = 0; face[r] = -1; return; }
    int n = 0;
    for (;;) {
        const uint32_t p01 = __umul24(d[0], a[1]), p10 = __umul24(d[1], a[0]);
        const uint32_t p02 = __umul24(d[0], a[2]), p20 = __umul24(d[2], a[0]);
        const uint32_t p12 = __umul24(d[1], a[2]), p21 = __umul24(d[2], a[1]);
        const bool m0 = a[0] != 0u && p01 <= p10 && p02 <= p20;
        const bool m1 = a[1] != 0u && p10 <= p01 && p12 <= p21;
        const bool m2 = a[2] != 0u && p20 <= p02 && p21 <= p12;
        if (n < max_len) cells[(size_t)r * max_len + n] = k[0] + G.n[0] * (k[1] + G.n[1] * k[2]);
        ++n;
        if (m0) { k[0] += sg[0]; d[0] += 2u; }
        if (m1) { k[1] += sg[1]; d[1] += 2u; }
        if (m2) { k[2] += sg[2]; d[2] += 2u; }
        int f = 0;
        for (int ax = 0; ax < 3; ++ax) {
            if (k[ax] < 0) f |= 1 << ax;
            if (k[ax] >= G.n[ax]) f |= (1 << ax) | (8 << ax);
        }
        if (f) { face[r] = f; break; }
    }
    count[r] = n;
}

// ---------------------------------------------------------------------------
// Fused sub-steps of many solves: the cell kernels walk the concatenation of
// the solves' slots; each thread finds its solve in the table (first slots
// ascending, staged in LDS).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int batch_solve_of(const uint64_t *first, int n, uint64_t g) {
    int lo = 0, hi = n - 1;                 // the last solve whose first slot is <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(64) k_bbegin(const BatchHead *hd, const BatchSolve *tb) {
    if (threadIdx.x == 0 && (int)blockIdx.x < hd->n) zero_ledger(tb[blockIdx.x].ledger);
}

template <typename R, int S>
__global__ void __launch_bounds__(kCellBlock) k_bprep(const BatchHead *hd, const BatchSolve *tb, int round,
                                                      unsigned long long *queue) {
    __shared__ uint64_t s_first[kMaxBatch];
    const int n = hd->n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s_first[i] = tb[i].cell0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0ull;
    __syncthreads();
    const uint64_t total = hd->cells;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const int b = batch_solve_of(s_first, n, g);
        const BatchSolve &sv = tb[b];
        if (round >= sv.n_sub) continue;
        prep_slot<R, S>(sv.geo.ncell_pad, reinterpret_cast<const R *>(sv.state), sv.kappa, sv.acc, sv.acc_stride,
                        sv.y_he, (uint32_t)(g - s_first[b]));
    }
}

__global__ void __launch_bounds__(64) k_bledger(const BatchHead *hd, const BatchSolve *tb, int round,
                                                const LedgerSlot *slots, int nslots) {
    const int b = blockIdx.x;
    if (b >= hd->n || round >= tb[b].n_sub) return;
    reduce_slots(slots + (size_t)b * nslots, nslots, tb[b].ledger);
}

template <typename R, int S, bool TH>
__global__ void __launch_bounds__(kCellBlock) k_bupdate(const BatchHead *hd, const BatchSolve *tb, int round) {
    __shared__ uint64_t s_first[kMaxBatch];
    RateCache cache;
    const int n = hd->n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s_first[i] = tb[i].cell0;
    __syncthreads();
    const uint64_t total = hd->cells;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const int b = batch_solve_of(s_first, n, g);
        const BatchSolve &sv = tb[b];
        if (round >= sv.n_sub) continue;
        const UpdateConst u(sv.cell_cm, sv.dt, sv.redshift, sv.n_chem);
        unsigned int bad = 0;
        update_slot<R, S, TH, false>(sv.geo, reinterpret_cast<R *>(sv.state), sv.acc, sv.acc_stride, sv.y_he, sv.dt,
                              sv.n_chem, u, (uint32_t)(g - s_first[b]), bad, cache);
        if (bad) atomicOr(&sv.ledger->nonfinite, 1u);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_batch_begin(const BatchLaunch &b) {
    hipLaunchKernelGGL(k_bbegin, dim3(kMaxBatch), dim3(64), 0, b.stream, b.head, b.table);
    return hipGetLastError();
}

template <typename R, int S>
static void bprep(const BatchLaunch &b, int round) {
    hipLaunchKernelGGL((k_bprep<R, S>), dim3(b.cell_blocks), dim3(kCellBlock), 0, b.stream, b.head, b.table, round,
                       b.queue);
}

hipError_t launch_batch_prep(const BatchLaunch &b, int round) {
    if (b.fp64) {
        if (b.species == 1) bprep<double, 1>(b, round); else bprep<double, 3>(b, round);
    } else {
        if (b.species == 1) bprep<float, 1>(b, round); else bprep<float, 3>(b, round);
    }
    return hipGetLastError();
}

hipError_t launch_batch_ledger(const BatchLaunch &b, int round) {
    hipLaunchKernelGGL(k_bledger, dim3(kMaxBatch), dim3(64), 0, b.stream, b.head, b.table, round, b.slots, b.blocks);
    return hipGetLastError();
}

template <typename R, int S>
static void bupdate(const BatchLaunch &b, int round) {
    const dim3 g(b.cell_blocks), t(kCellBlock);
    if (b.thermal) hipLaunchKernelGGL((k_bupdate<R, S, true>), g, t, 0, b.stream, b.head, b.table, round);
    else hipLaunchKernelGGL((k_bupdate<R, S, false>), g, t, 0, b.stream, b.head, b.table, round);
}

hipError_t launch_batch_update(const BatchLaunch &b, int round) {
    if (b.fp64) {
        if (b.species == 1) bupdate<double, 1>(b, round); else bupdate<double, 3>(b, round);
    } else {
        if (b.species == 1) bupdate<float, 1>(b, round); else bupdate<float, 3>(b, round);
    }
    return hipGetLastError();
}
// Each solve's step ledger into out[solve] (table order), for one copy to the host.
__global__ void k_bgather(const BatchHead *hd, const BatchSolve *tb, StepLedger *out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < hd->n) out[b] = *tb[b].ledger;
}

hipError_t launch_batch_gather(const BatchLaunch &b, StepLedger *out) {
    hipLaunchKernelGGL(k_bgather, dim3(kMaxBatch / 64), dim3(64), 0, b.stream, b.head, b.table, out);
    return hipGetLastError();
}

hipError_t launch_prep(const CellLaunch &c) {
    const int nb = cell_blocks(c.geo.ncell_pad);
    if (c.fp64) {
        if (c.species == 1)
            hipLaunchKernelGGL((k_prep<double, 1>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (const double *)c.state, c.kappa, c.acc, c.acc_stride, c.y_he, c.queue);
        else
            hipLaunchKernelGGL((k_prep<double, 3>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (const double *)c.state, c.kappa, c.acc, c.acc_stride, c.y_he, c.queue);
    } else {
        if (c.species == 1)
            hipLaunchKernelGGL((k_prep<float, 1>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (const float *)c.state, c.kappa, c.acc, c.acc_stride, c.y_he, c.queue);
        else
            hipLaunchKernelGGL((k_prep<float, 3>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (const float *)c.state, c.kappa, c.acc, c.acc_stride, c.y_he, c.queue);
    }
    return hipGetLastError();
}

template <typename R, int S, bool TH>
static void upd(const CellLaunch &c, int nb) {
    hipLaunchKernelGGL((k_update<R, S, TH>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo, (R *)c.state,
                       c.acc, c.acc_stride, c.y_he, c.cell_cm, c.dt, c.redshift, c.n_chem, c.ledger, c.rc);
}

hipError_t launch_update(const CellLaunch &c) {
    const int nb = cell_blocks(c.geo.ncell_pad);
    if (c.fp64) {
        if (c.species == 1) { if (c.thermal) upd<double, 1, true>(c, nb); else upd<double, 1, false>(c, nb); }
        else { if (c.thermal) upd<double, 3, true>(c, nb); else upd<double, 3, false>(c, nb); }
    } else {
        if (c.species == 1) { if (c.thermal) upd<float, 1, true>(c, nb); else upd<float, 1, false>(c, nb); }
        else { if (c.thermal) upd<float, 3, true>(c, nb); else upd<float, 3, false>(c, nb); }
    }
    return hipGetLastError();
}

hipError_t launch_import(const CellLaunch &c, const void *nh, const void *x, const void *t,
                         int fields_fp64, int64_t ncell) {
    const size_t nst = 7 * (size_t)c.geo.ncell_pad;
    const int nb = cell_blocks((uint64_t)ncell);
    if (c.fp64) {
        hipLaunchKernelGGL((k_fill_zero<double>), dim3(cell_blocks(nst)), dim3(kCellBlock), 0, c.stream,
                           (double *)c.state, nst);
        if (fields_fp64)
            hipLaunchKernelGGL((k_import<double, double>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (double *)c.state, (const double *)nh, (const double *)x, (const double *)t,
                               (uint32_t)ncell);
        else
            hipLaunchKernelGGL((k_import<double, float>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (double *)c.state, (const float *)nh, (const float *)x, (const float *)t,
                               (uint32_t)ncell);
    } else {
        hipLaunchKernelGGL((k_fill_zero<float>), dim3(cell_blocks(nst)), dim3(kCellBlock), 0, c.stream,
                           (float *)c.state, nst);
        if (fields_fp64)
            hipLaunchKernelGGL((k_import<float, double>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (float *)c.state, (const double *)nh, (const double *)x, (const double *)t,
                               (uint32_t)ncell);
        else
            hipLaunchKernelGGL((k_import<float, float>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (float *)c.state, (const float *)nh, (const float *)x, (const float *)t,
                               (uint32_t)ncell);
    }
    // accumulators start at zero so a fetch before the first step is defined
    hipLaunchKernelGGL((k_fill_zero<double>), dim3(cell_blocks((size_t)c.geo.ncell_pad * c.acc_stride)),
                       dim3(kCellBlock), 0, c.stream, c.acc, (size_t)c.geo.ncell_pad * c.acc_stride);
    return hipGetLastError();
}

hipError_t launch_export(const CellLaunch &c, uint32_t mask, void *dst, int as_fp64, int64_t ncell) {
    const int nb = cell_blocks((uint64_t)ncell);
    if (c.fp64) {
        if (as_fp64)
            hipLaunchKernelGGL((k_export<double, double>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (const double *)c.state, c.acc, c.acc_stride, c.species, c.thermal, mask,
                               (double *)dst, (uint32_t)ncell, c.rc);
        else
            hipLaunchKernelGGL((k_export<double, float>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (const double *)c.state, c.acc, c.acc_stride, c.species, c.thermal, mask,
                               (float *)dst, (uint32_t)ncell, c.rc);
    } else {
        if (as_fp64)
            hipLaunchKernelGGL((k_export<float, double>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (const float *)c.state, c.acc, c.acc_stride, c.species, c.thermal, mask,
                               (double *)dst, (uint32_t)ncell, c.rc);
        else
            hipLaunchKernelGGL((k_export<float, float>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo,
                               (const float *)c.state, c.acc, c.acc_stride, c.species, c.thermal, mask,
                               (float *)dst, (uint32_t)ncell, c.rc);
    }
    return hipGetLastError();
}

hipError_t launch_import_counters(const CellLaunch &c, const void *src, int src_fp64, int64_t ncell) {
    const int nb = cell_blocks((uint64_t)ncell);
    if (src_fp64 || !src)
        hipLaunchKernelGGL((k_import_rc<double>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo, c.rc,
                           (const double *)src, c.species, (uint32_t)ncell);
    else
        hipLaunchKernelGGL((k_import_rc<float>), dim3(nb), dim3(kCellBlock), 0, c.stream, c.geo, c.rc,
                           (const float *)src, c.species, (uint32_t)ncell);
    return hipGetLastError();
}

hipError_t launch_ledger_zero(StepLedger *l, hipStream_t s) {
    hipLaunchKernelGGL(k_ledger_zero, dim3(1), dim3(64), 0, s, l);
    return hipGetLastError();
}

hipError_t launch_ledger_reduce(const LedgerSlot *slots, int nslots, StepLedger *l, hipStream_t s) {
    if (nslots > 0) hipLaunchKernelGGL(k_ledger_reduce, dim3(1), dim3(64), 0, s, slots, nslots, l);
    else hipLaunchKernelGGL(k_ledger_tick, dim3(1), dim3(64), 0, s, l);
    return hipGetLastError();
}

hipError_t launch_trace_rays(const GridGeom &g, int m, const int32_t *o, const int32_t *c, int max_len,
                             int32_t *cells, int32_t *count, int32_t *face, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_trace_rays, dim3((m + 255) / 256), dim3(256), 0, s, g, m, o, c, max_len, cells, count,
                       face);
    return hipGetLastError();
}

}  // namespace rtk
