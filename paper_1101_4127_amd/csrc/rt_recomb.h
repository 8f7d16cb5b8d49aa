// rt_recomb.h -- device helpers of recombination re-emission (Partl et al.
// 2011, Sec. 2: the network records the recombinations N_rec of a cell; once
// N_rec >= f_rec N_a the cell emits a packet of recombination photons with a
// Milne spectrum; Sec. 3: pCRASH2 emits when a packet crosses such a cell).
// Rate fits: Hui & Gnedin (1997), case A and case B.  Included by the HIP
// translation units only.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rt_internal.h"

namespace rtk {

// Hydrogenic radiative recombination, lambda = 2 T_ion / T.
__device__ __forceinline__ double hydrogenic_caseb(double T, double t_ion) {
    const double lam = 2.0 * t_ion / T;
    return 2.753e-14 * pow(lam, 1.5) / pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
}

__device__ __forceinline__ double hydrogenic_casea(double T, double t_ion) {
    const double lam = 2.0 * t_ion / T;
    return 1.269e-13 * pow(lam, 1.503) / pow(1.0 + pow(lam / 0.522, 0.470), 1.923);
}

// HeII -> HeI radiative part (case A / case B) and the dielectronic part.
__device__ __forceinline__ double heii_rad_casea(double T) { return 3.0e-14 * pow(570670.0 / T, 0.654); }
__device__ __forceinline__ double heii_rad_caseb(double T) { return 1.26e-14 * pow(570670.0 / T, 0.750); }
__device__ __forceinline__ double heii_dielectronic(double T) {
    return 1.9e-3 * pow(T, -1.5) * exp(-470000.0 / T) * (1.0 + 0.3 * exp(-94000.0 / T));
}

// Share of each ion's recombinations that go directly to the ground state,
// (alpha_A - alpha_B) / alpha_A of the radiative rates (HeII over the total
// with its dielectronic part), never below 0 (the HeII power laws cross below
// ~70 K).  p = HII, HeII, HeIII.
__device__ __forceinline__ void ground_fraction(double T, double p[3]) {
    const double ah_a = hydrogenic_casea(T, 157807.0), ah_b = hydrogenic_caseb(T, 157807.0);
    const double ahe_a = hydrogenic_casea(T, 631515.0), ahe_b = hydrogenic_caseb(T, 631515.0);
    const double r_a = heii_rad_casea(T), r_b = heii_rad_caseb(T);
    p[0] = (ah_a - ah_b) / ah_a;
    p[1] = (r_a - r_b) / (r_a + heii_dielectronic(T));
    p[2] = (ahe_a - ahe_b) / ahe_a;
    for (int i = 0; i < 3; ++i) p[i] = p[i] > 0.0 ? p[i] : 0.0;
}

// Time integral over h of x_HII along the two-level solution with rates I, R
// that took it from x0 to xh: h x_eq + (x0 - xh) / (I + R).
__device__ __forceinline__ double hii_time(double x0, double xh, double I, double R, double h) {
    const double lam = I + R;
    if (!(lam > 0.0)) return h * x0;
    const double v = h * (I / lam) + (x0 - xh) / lam;
    return v > 0.0 ? v : 0.0;
}

// Time integrals over h of x_HeII and x_HeIII along the helium chain's
// solution from (a0, b0, c0) to (ah, bh, ch) (HeI, HeII, HeIII): h x_eq + z
// with z the zero-sum solution of M z = xh - x0 for the chain's generator M.
__device__ __forceinline__ void he_ion_time(double a0, double b0, double c0, double ah, double bh, double ch,
                                            double I1, double R2, double I2, double R3, double h, double &t_heii,
                                            double &t_heiii) {
    (void)bh;
    const double det = I1 * I2 + I1 * R3 + R2 * R3;
    if (!(det > 0.0)) { t_heii = h * b0; t_heiii = h * c0; return; }
    const double d0 = ah - a0, d2 = ch - c0;
    const double z1 = (R3 * d0 + I1 * d2) / det;
    const double z2 = (I2 * d0 - (I1 + R2) * d2) / det;
    const double v1 = h * (I1 * R3 / det) + z1, v2 = h * (I1 * I2 / det) + z2;
    t_heii = v1 > 0.0 ? v1 : 0.0;
    t_heiii = v2 > 0.0 ? v2 : 0.0;
}

// Spectrum of ion `ion` at T: linear in log10 T between the table's nodes,
// clamped to the end nodes; m[j] for j < mb.
template <int MB>
__device__ __forceinline__ void milne_at(const RecombParams &r, int ion, double T, double (&m)[MB]) {
    double u = (log10(T) - r.log10_t0) / r.dlog10_t;
    const double top = (double)(r.n_t - 1);
    if (!(u > 0.0)) u = 0.0;
    if (u > top) u = top;
    int k = (int)floor(u);
    if (k > r.n_t - 2) k = r.n_t - 2;
    const double f = u - (double)k;
    const double *a = r.milne + ((size_t)ion * r.n_t + k) * MB, *b = a + MB;
#pragma unroll
    for (int j = 0; j < MB; ++j) m[j] = (1.0 - f) * a[j] + f * b[j];
}

}  // namespace rtk
