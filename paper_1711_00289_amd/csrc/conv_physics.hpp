// conv_physics.hpp -- device-side thermodynamics and per-level building blocks of the convection
// scheme for gfx950 (FP64 throughout).
//
// The scheme is the written reading of the paper's deep and shallow convection (arXiv:1711.00289,
// Background and Algorithms 2-3): steps C0-C1 (grid, thermodynamics), D1-D10 (deep) and S1-S9
// (shallow).  `tsat` is the saturated inversion that plays the role of the paper's iterative
// `ientropy` (Algorithm 2), the loop the paper singles out as convergence-tested and hard to
// vectorise.  Here it costs about two exp evaluations per saturated level: each solve starts from
// a first-order prediction off the previous level's root, takes Halley steps until a step is below
// 1e-4 K (the next error is then below one ulp of T), and carries the saturation humidity to the
// root by its Taylor series instead of evaluating it again.
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
constexpr double RCP_CP = 1.0 / CP;
constexpr double HALLEY_DONE = 1e-4;  // K

// 1/x to about one ulp: the hardware reciprocal estimate refined by two Newton-Raphson steps
// (not correctly rounded; used where the scheme's result does not depend on the last bit).
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

struct Sat {
    double qs;    // saturation specific humidity
    double dqs;   // d qs / dT
    double d2qs;  // d2 qs / dT2
    double qs_p;  // -d qs / dp = qs / (p - (1-eps) es)
};

// qs(T, p) and its derivatives (C1): Bolton's es over liquid, qs capped at 1 where es >= p, es := 0
// at or below T_ES_MIN.  One exp and two reciprocals.  With A = 17.67*243.5/(T-29.65)^2 and
// d = p - (1-eps) es:  qs' = qs A p / d,  qs'' = qs' (A (p + (1-eps) es)/d - 2/(T-29.65)).
__device__ __forceinline__ Sat sat_eval(double T, double p) {
    if (T <= T_ES_MIN) return Sat{0.0, 0.0, 0.0, 0.0};
    const double rb = frcp(T - 29.65);
    const double e = 611.2 * exp(17.67 * (T - 273.15) * rb);
    if (e >= p) return Sat{1.0, 0.0, 0.0, 0.0};
    const double rd = frcp(p - OMEPS * e);
    const double A = ES_SLOPE * (rb * rb);
    const double qs = EPSV * e * rd;
    const double dqs = qs * A * (p * rd);
    const double d2qs = dqs * (A * (p + OMEPS * e) * rd - 2.0 * rb);
    return Sat{qs, dqs, d2qs, qs * rd};
}

__device__ __forceinline__ double tv(double T, double q) { return T * (1.0 + CVIR * q); }

// Root of G(T) = cp*T + Lv*qs(T,p) - H inside [lo, hi], from T with s = sat_eval(T, p).  Halley
// steps dT = -(G/G') / (1 - G G'' / (2 G'^2)) (cubic convergence, G'' = Lv qs'' is a by-product of
// sat_eval), bisecting whenever a step leaves the bracket.  Once a step is below HALLEY_DONE the
// next error is below K*dT^3 with K ~ 4e-3 K^-2, i.e. under one ulp of T, so T + dT is the root to
// rounding and `s` is carried there by its Taylor series (qs to second order, qs' to first).
__device__ __forceinline__ double solve_sat(double H, double p, double T, double lo, double hi,
                                           Sat &s) {
    for (int it = 0; it < 100; ++it) {
        const double G = CP * T + LV * s.qs - H;
        if (G > 0.0) hi = T;
        else if (G < 0.0) lo = T;
        else return T;
        const double rGp = frcp(CP + LV * s.dqs);
        const double nstep = G * rGp;
        const double dT = -nstep * frcp(1.0 - 0.5 * nstep * (LV * s.d2qs) * rGp);
        const double Tn = T + dT;
        if (Tn >= lo && Tn <= hi) {
            if (fabs(dT) <= HALLEY_DONE) {
                s.qs = fma(dT, fma(0.5 * dT, s.d2qs, s.dqs), s.qs);
                s.dqs = fma(s.d2qs, dT, s.dqs);
                return Tn;
            }
            T = Tn;
        } else {
            T = 0.5 * (lo + hi);
        }
        s = sat_eval(T, p);
    }
    return T;
}

// tsat(H, p) from an initial guess (C1).
__device__ __forceinline__ double tsat(double H, double p, double Tguess, Sat &s) {
    const double hi = H * RCP_CP;
    if (hi <= T_ES_MIN) {
        s = Sat{0.0, 0.0, 0.0, 0.0};
        return hi;
    }
    const double T = fmin(fmax(Tguess, T_ES_MIN), hi);
    s = sat_eval(T, p);
    return solve_sat(H, p, T, T_ES_MIN, hi, s);
}

// The last saturated solution along a rising or sinking parcel, from which the next level's root
// is predicted to first order: dT = (dH + Lv*(qs/d)*dp) / G'.
struct Hint {
    bool ok;
    double T, H, p, rGp, qs_p;
    __device__ void clear() { ok = false; }
    __device__ void set(double T_, double H_, double p_, const Sat &s) {
        ok = true;
        T = T_;
        H = H_;
        p = p_;
        rGp = frcp(CP + LV * s.dqs);
        qs_p = s.qs_p;
    }
    __device__ double predict(double H_, double p_) const {
        return T + ((H_ - H) + LV * qs_p * (p_ - p)) * rGp;
    }
};

// tsat with a prediction from the hint when it has one; updates the hint.
__device__ __forceinline__ double tsat_h(double H, double p, double Tguess, Sat &s, Hint &h) {
    const double T = tsat(H, p, h.ok ? h.predict(H, p) : Tguess, s);
    h.set(T, H, p, s);
    return T;
}

struct Lifted {
    double T, qv, dqs;
    bool sat;
};

// A parcel of energy H (= h - g*z - phis) and total water qt at pressure p (C1): unsaturated
// (T = T_dry) if qt <= qs(T_dry), else at saturation.  One solver path for every lane: without a
// hint the first evaluation is at T_dry and doubles as the saturation test (G(T_dry) < 0 when
// saturated, so T_dry bounds the root from below); with a hint it is at the prediction and the test
// is read off the root (saturated iff the root lies above T_dry, G being increasing), made directly
// within 1e-12 relative of T_dry so the decision is the direct comparison's.
__device__ __forceinline__ Lifted lift(double H, double qt, double p, Hint &h) {
    const double Tdry = (H - LV * qt) * RCP_CP;
    const double hi = H * RCP_CP;
    const bool pred = h.ok && hi > T_ES_MIN;
    const double T0 = pred ? fmin(fmax(h.predict(H, p), T_ES_MIN), hi) : Tdry;
    Sat s = sat_eval(T0, p);
    bool sat = pred || qt > s.qs;
    double T = Tdry;
    if (sat) {
        T = solve_sat(H, p, T0, pred ? T_ES_MIN : Tdry, hi, s);
        if (pred) {
            if (T > Tdry * (1.0 + 1e-12)) sat = true;
            else if (T < Tdry * (1.0 - 1e-12)) sat = false;
            else sat = qt > sat_eval(Tdry, p).qs;
        }
    }
    if (!sat) {
        h.clear();
        return Lifted{Tdry, qt, 0.0, false};
    }
    h.set(T, H, p, s);
    return Lifted{T, s.qs, s.dqs, true};
}

}  // namespace cvk
