// conv_physics.hpp -- device-side thermodynamics and per-level building blocks of the convection
// scheme for gfx950 (FP64 throughout).
//
// The scheme is the written reading of the paper's deep and shallow convection (arXiv:1711.00289,
// Background and Algorithms 2-3): steps C0-C1 (grid, thermodynamics), D1-D10 (deep) and S1-S9
// (shallow).  `tsat` is the saturated inversion that plays the role of the paper's iterative
// `ientropy` (Algorithm 2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "conv.h"

namespace cvk {

constexpr double CP = 1004.64;
constexpr double RD = 287.04;
constexpr double RV = 461.5;
constexpr double LV = 2.501e6;
constexpr double GRAV = 9.80616;
constexpr double EPSV = RD / RV;
constexpr double CVIR = 1.0 / EPSV - 1.0;
constexpr double OMEPS = 1.0 - EPSV;
constexpr double T_ES_MIN = 40.0;
constexpr double SQRT_2PI = 2.5066282746310002;
constexpr double ES_SLOPE = 17.67 * 243.5;

struct Sat {
    double qs, dqs;
};

// Saturation specific humidity and its temperature derivative at (T, p) (C1): Bolton's es over
// liquid, qs capped at 1 where es >= p, es := 0 at or below T_ES_MIN.  Two reciprocals and one
// exp per call; the Newton solver calls this once per iteration.
__device__ __forceinline__ Sat sat_eval(double T, double p) {
    if (T <= T_ES_MIN) return Sat{0.0, 0.0};
    const double rb = 1.0 / (T - 29.65);
    const double e = 611.2 * exp(17.67 * (T - 273.15) * rb);
    if (e >= p) return Sat{1.0, 0.0};
    const double rd = 1.0 / (p - OMEPS * e);
    const double qs = EPSV * e * rd;
    return Sat{qs, qs * ES_SLOPE * (rb * rb) * (p * rd)};
}

__device__ __forceinline__ double qsat(double T, double p) { return sat_eval(T, p).qs; }

__device__ __forceinline__ double tv(double T, double q) { return T * (1.0 + CVIR * q); }

// Safeguarded Newton for the root of G(T) = cp*T + Lv*qs(T,p) - H inside the bracket [lo, hi]
// that holds it, starting from T with G = G(T), Gp = G'(T) already evaluated.  Stops once a step
// is below 4e-12*T (quadratic convergence puts the iterate at the root to rounding).  Returns the
// root; `s` holds qs and dqs/dT there.
__device__ __forceinline__ double newton_root(double H, double p, double T, double G, double Gp,
                                              double lo, double hi, Sat &s) {
    for (int it = 0; it < 80; ++it) {
        if (G == 0.0) break;
        if (G > 0.0) hi = T; else lo = T;
        double Tn = T - G / Gp;
        if (!(Tn >= lo && Tn <= hi)) Tn = 0.5 * (lo + hi);
        const double dT = Tn - T;
        T = Tn;
        s = sat_eval(T, p);
        G = CP * T + LV * s.qs - H;
        Gp = CP + LV * s.dqs;
        if (fabs(dT) <= 4e-12 * T) break;
    }
    return T;
}

// tsat(H, p): the saturated temperature of moist static energy H at pressure p (C1).
__device__ __forceinline__ double tsat(double H, double p, double Tguess, Sat &s) {
    const double hi = H * (1.0 / CP);
    if (hi <= T_ES_MIN) {
        s = Sat{0.0, 0.0};
        return hi;
    }
    double T = fmin(fmax(Tguess, T_ES_MIN), hi);
    s = sat_eval(T, p);
    return newton_root(H, p, T, CP * T + LV * s.qs - H, CP + LV * s.dqs, T_ES_MIN, hi, s);
}

struct Lifted {
    double T, qv, dqs;
    bool sat;
};

// A parcel of energy H (= h - g*z - phis) and total water qt at pressure p: unsaturated if
// qt <= qs(T_dry), else at saturation (C1).  The saturation test's evaluation is the first Newton
// iterate (G(T_dry) = Lv*(qs(T_dry) - qt) < 0 when saturated, so T_dry bounds the root below).
__device__ __forceinline__ Lifted lift(double H, double qt, double p) {
    const double Tdry = (H - LV * qt) * (1.0 / CP);
    Sat s = sat_eval(Tdry, p);
    if (qt <= s.qs) return Lifted{Tdry, qt, s.dqs, false};
    const double hi = H * (1.0 / CP);
    const double T = newton_root(H, p, Tdry, CP * Tdry + LV * s.qs - H, CP + LV * s.dqs, Tdry,
                                 hi, s);
    return Lifted{T, s.qs, s.dqs, true};
}

}  // namespace cvk
