/*
 * conv_oracle.cpp -- plain single-threaded FP64 CPU oracle of the convection scheme.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, by the smoke check and by the benchmark's CPU-baseline
 * leg.  The product library never links or calls it and the two share no code.
 *
 * The paper (arXiv:1711.00289) names the deep scheme (Zhang-McFarlane) and the shallow scheme
 * (University of Washington, Park-Bretherton) in its Background section and gives only their loop
 * skeletons: the deep scheme's entrainment loop and precipitation loop over columns x levels,
 * each calling an iterative inversion `ientropy` (Algorithm 2), and the shallow scheme's column
 * loop whose repeated thermodynamic checks send a column to an exit that zeroes its outputs
 * (Algorithm 3).  The physics filling those skeletons is a written reading in steps C0-C1 (grid,
 * thermodynamics), D1-D10 (deep) and S1-S9 (shallow), stated in the comments where each step is
 * computed below.  The code follows the steps in order, with no
 * blocking or reordering, so it can be checked against the written steps by eye.
 *
 * Compiled with -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 *
 * Scalar type R is double for the plain run, or Dual (value + one tangent) for the forward-mode
 * derivative used to check the hand-written adjoint.  Branches always test the value part, so the
 * tangent is the derivative with every branch (indices, saturation flags, limiters) held fixed.
 */
#include "conv_oracle.h"

#include <cmath>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

/* ---------------------------------------------------------------- scalar types */
struct Dual {
    double v, d;
    Dual() : v(0.0), d(0.0) {}
    Dual(double x) : v(x), d(0.0) {}  // NOLINT: implicit on purpose (constants)
    Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline Dual sqrt(Dual a) { double r = std::sqrt(a.v); return Dual(r, a.d / (2.0 * r)); }
inline double val(double x) { return x; }
inline double val(const Dual &x) { return x.v; }

/* Counted: a double that counts the arithmetic done on it (the algorithmic operation count of the
 * scheme, for the roofline): +, -, *, / and sqrt count 1, exp and log count 1 (no fused
 * multiply-add occurs: the oracle is built without contraction).  Only operations with a state- or
 * parameter-dependent operand run in this type; the grid's own arithmetic (interface heights,
 * layer thicknesses, log-pressure widths: 6 per layer) is added by the caller. */
thread_local long long g_ops = 0;
struct Counted {
    double v;
    Counted() : v(0.0) {}
    Counted(double x) : v(x) {}  // NOLINT: implicit on purpose (constants)
};
inline Counted operator+(Counted a, Counted b) { ++g_ops; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { ++g_ops; return Counted(a.v - b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline Counted operator*(Counted a, Counted b) { ++g_ops; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { ++g_ops; return Counted(a.v / b.v); }
inline Counted exp(Counted a) { ++g_ops; return Counted(std::exp(a.v)); }
inline Counted log(Counted a) { ++g_ops; return Counted(std::log(a.v)); }
inline Counted sqrt(Counted a) { ++g_ops; return Counted(std::sqrt(a.v)); }
inline double val(const Counted &x) { return x.v; }
using std::exp;
using std::log;
using std::sqrt;

/* ---------------------------------------------------------------- C0: constants (SI) */
constexpr double CP = 1004.64;        // J kg^-1 K^-1
constexpr double RD = 287.04;         // J kg^-1 K^-1
constexpr double RV = 461.5;          // J kg^-1 K^-1
constexpr double LV = 2.501e6;        // J kg^-1
constexpr double GRAV = 9.80616;      // m s^-2
constexpr double EPSV = RD / RV;      // Rd/Rv
constexpr double CVIR = 1.0 / EPSV - 1.0;
constexpr double ONE_MINUS_EPSV = 1.0 - EPSV;
constexpr double T_ES_MIN = 40.0;     // es := 0 at or below (keeps clear of the pole at 29.65 K)
constexpr double SQRT_2PI = 2.5066282746310002;

/* ---------------------------------------------------------------- C1: thermodynamics */
// Saturation vapour pressure over liquid (Bolton 1980), Pa.
template <class R> R es_(const R &T) {
    if (val(T) <= T_ES_MIN) return R(0.0);
    return 611.2 * exp(17.67 * (T - 273.15) / (T - 29.65));
}

// Saturation specific humidity, capped at 1 where es >= p.
template <class R> R qs_(const R &T, double p) {
    R e = es_(T);
    if (val(e) >= p) return R(1.0);
    R d = p - ONE_MINUS_EPSV * e;
    return EPSV * e / d;
}

// d qs / d T at fixed p (0 where qs is capped or es is cut to 0).
template <class R> R dqsdT_(const R &T, double p) {
    if (val(T) <= T_ES_MIN) return R(0.0);
    R e = es_(T);
    if (val(e) >= p) return R(0.0);
    R d = p - ONE_MINUS_EPSV * e;
    R q = EPSV * e / d;
    R b = T - 29.65;
    return q * (17.67 * 243.5 / (b * b)) * p / d;
}

// Saturated inversion (the analogue of the paper's `ientropy`): the unique root T of
// G(T) = cp*T + Lv*qs(T, p) - H on [T_ES_MIN, H/cp].  Newton, safeguarded by bisection inside the
// bracket, iterated until |dT| <= 1e-12*T and then one more step.
template <class R> R tsat_(const R &H, double p, const R &Tguess, int *iters) {
    R hi = H / CP;
    if (val(hi) <= T_ES_MIN) {
        if (iters) *iters = 0;
        return hi;
    }
    R lo = R(T_ES_MIN);
    R T = Tguess;
    if (val(T) < val(lo)) T = lo;
    if (val(T) > val(hi)) T = hi;
    bool last = false;
    int it = 0;
    for (; it < 200; ++it) {
        R G = CP * T + LV * qs_(T, p) - H;
        if (val(G) == 0.0) break;
        if (val(G) > 0.0) hi = T; else lo = T;
        R Gp = CP + LV * dqsdT_(T, p);
        R Tn = T - G / Gp;
        if (!(val(Tn) >= val(lo) && val(Tn) <= val(hi))) Tn = 0.5 * (lo + hi);
        R dT = Tn - T;
        T = Tn;
        if (last) break;
        if (std::fabs(val(dT)) <= 1e-12 * val(T)) last = true;
    }
    if (iters) *iters = it;
    return T;
}

template <class R> R tv_(const R &T, const R &q) { return T * (1.0 + CVIR * q); }

// A parcel of moist static energy H (= h - g*z - phis) and total water qt placed at pressure p:
// unsaturated if qt <= qs(T_dry), else brought to saturation by tsat (C1, D2, D5, S2, S7).
template <class R> struct Lifted {
    R T, qv;
    bool sat;
};
template <class R> Lifted<R> lift_(const R &H, const R &qt, double p) {
    R Tdry = (H - LV * qt) / CP;
    if (val(qt) <= val(qs_(Tdry, p))) return Lifted<R>{Tdry, qt, false};
    R T = tsat_(H, p, Tdry, nullptr);
    return Lifted<R>{T, qs_(T, p), true};
}

/* ---------------------------------------------------------------- column validity */
// A column the scheme can run on: finite inputs, 100 K < T < 400 K, 0 <= q < 1, interface
// pressures increasing downward with each mid-layer pressure strictly inside its layer, heights
// strictly decreasing downward and positive.  Anything else is reported as an invalid column.
template <class R>
bool column_valid(int L, const R *T, const R *q, const double *pm, const double *pi, const double *z,
                  double phis) {
    if (!std::isfinite(phis)) return false;
    if (!(std::isfinite(pi[0]) && pi[0] > 0.0)) return false;
    for (int k = 0; k < L; ++k) {
        double t = val(T[k]), w = val(q[k]);
        if (!(std::isfinite(t) && std::isfinite(w) && std::isfinite(pm[k]) && std::isfinite(z[k]) &&
              std::isfinite(pi[k + 1])))
            return false;
        if (!(t > 100.0 && t < 400.0)) return false;
        if (!(w >= 0.0 && w < 1.0)) return false;
        if (!(pi[k] < pm[k] && pm[k] < pi[k + 1])) return false;
        if (k < L - 1 && !(z[k] > z[k + 1])) return false;
    }
    return z[L - 1] > 0.0;
}

/* ---------------------------------------------------------------- C0: grid */
struct Grid {
    std::vector<double> zi, dz, dp, lam;
};
Grid make_grid(int L, const double *pi, const double *z) {
    Grid g;
    g.zi.assign(L + 1, 0.0);
    g.dz.assign(L, 0.0);
    g.dp.assign(L, 0.0);
    g.lam.assign(L, 0.0);
    g.zi[L] = 0.0;
    for (int i = 1; i <= L - 1; ++i) g.zi[i] = 0.5 * (z[i - 1] + z[i]);
    g.zi[0] = 2.0 * z[0] - g.zi[1];
    for (int k = 0; k < L; ++k) {
        g.dz[k] = g.zi[k] - g.zi[k + 1];
        g.dp[k] = pi[k + 1] - pi[k];
        g.lam[k] = std::log(pi[k + 1] / pi[k]);
    }
    return g;
}

/* ---------------------------------------------------------------- deep scheme (D1-D10) */
template <class R> struct DeepRes {
    std::vector<R> dTdt, dqdt, mu, md, eta, etad;
    R prec, cape, F, Mc, Mlim, Mb, alpha, C1, E1, P1;
    int kb, kt, kd, klim, trig, status;
};

template <class R>
void deep_column(int L, const oracle_params_t &P, const R &tau, const R &epsd, const R *T,
                 const R *q, const double *pm, const double *pi, const double *z, double phis,
                 double dt, DeepRes<R> &o) {
    o.dTdt.assign(L, R(0.0));
    o.dqdt.assign(L, R(0.0));
    o.mu.assign(L + 1, R(0.0));
    o.md.assign(L + 1, R(0.0));
    o.eta.assign(L + 1, R(0.0));
    o.etad.assign(L + 1, R(0.0));
    o.prec = o.cape = o.F = o.Mc = o.Mb = o.alpha = o.C1 = o.E1 = o.P1 = R(0.0);
    o.Mlim = R(std::numeric_limits<double>::infinity());
    o.kb = o.kt = o.kd = o.klim = -1;
    o.trig = 0;
    if (!column_valid(L, T, q, pm, pi, z, phis)) {
        o.status = 3;
        return;
    }
    const Grid g = make_grid(L, pi, z);
    std::vector<R> s(L), h(L);
    for (int k = 0; k < L; ++k) {
        s[k] = CP * T[k] + GRAV * z[k] + phis;  // dry static energy
        h[k] = s[k] + LV * q[k];                // moist static energy
    }

    // D1: launch layer = argmax h over layers with p_mid >= p_launch_min; the lower layer wins a tie.
    int kb = -1;
    for (int k = L - 1; k >= 0; --k)
        if (pm[k] >= P.p_launch_min && (kb < 0 || val(h[k]) > val(h[kb]))) kb = k;
    // D3 (limit): highest layer the cloud top may reach.
    int klim = -1;
    for (int k = 0; k < L; ++k)
        if (pm[k] >= P.p_top_min) {
            klim = k;
            break;
        }
    o.kb = kb;
    o.klim = klim;
    if (kb < 0 || klim < 0) {
        o.status = 1;
        return;
    }

    // D2: pseudo-adiabatic parcel from layer kb, lifted layer by layer upward.  Undilute by
    // default; with eps_cape > 0 it entrains environmental air on the way up (dilute CAPE): its
    // mass grows by eps_cape per metre of mid-level height and h and the total water mix in as
    // conserved quantities.  The condensate stays in the mixed water (not in the buoyancy), so
    // eps_cape = 0 is exactly the undilute parcel of every layer lifted from kb's h and q.
    std::vector<R> Tp(L, R(0.0)), qp(L, R(0.0)), B(L, R(0.0));
    std::vector<char> sat(L, 0);
    {
        R hmix = h[kb], qmix = q[kb];
        for (int k = kb - 1; k >= klim; --k) {
            const double mix = P.eps_cape * (z[k] - z[k + 1]);
            hmix = (hmix + mix * h[k]) / (1.0 + mix);
            qmix = (qmix + mix * q[k]) / (1.0 + mix);
            R H = hmix - GRAV * z[k] - phis;
            Lifted<R> pt = lift_(H, qmix, pm[k]);
            Tp[k] = pt.T;
            qp[k] = pt.qv;
            sat[k] = pt.sat;
            B[k] = tv_(pt.T, pt.qv) - tv_(T[k], q[k]);
        }
    }
    // D3: cloud top = highest layer in [klim, kb) with positive buoyancy.
    int kt = -1;
    for (int k = klim; k < kb; ++k)
        if (val(B[k]) > 0.0) {
            kt = k;
            break;
        }
    o.kt = kt;
    if (kt < 0) {
        o.status = 1;
        return;
    }
    // D4: CAPE = max(0, signed sum of Rd*B*dlnp over [kt, kb)), summed upward; trigger.
    R sum = R(0.0);
    for (int k = kb - 1; k >= kt; --k) sum = sum + RD * B[k] * g.lam[k];
    o.cape = val(sum) > 0.0 ? sum : R(0.0);
    o.trig = val(o.cape) > P.cape_threshold ? 1 : 0;
    if (!o.trig) {
        o.status = 1;
        return;
    }

    // D5: entraining updraft, unit base mass flux at interface kb, detraining in layer kt.
    std::vector<R> eta(L + 1, R(0.0)), su(L + 1, R(0.0)), qu(L + 1, R(0.0)), c(L, R(0.0));
    eta[kb] = R(1.0);
    R hu = h[kb];
    {
        R H = h[kb] - GRAV * g.zi[kb] - phis;
        Lifted<R> pt = lift_(H, q[kb], pi[kb]);
        su[kb] = CP * pt.T + GRAV * g.zi[kb] + phis;
        qu[kb] = pt.qv;
        c[kb] = eta[kb] * (q[kb] - pt.qv);
    }
    for (int k = kb - 1; k >= kt + 1; --k) {
        R E = epsd * eta[k + 1] * g.dz[k];
        eta[k] = eta[k + 1] + E;
        R hm = (eta[k + 1] * hu + E * h[k]) / eta[k];
        R qm = (eta[k + 1] * qu[k + 1] + E * q[k]) / eta[k];
        R H = hm - GRAV * g.zi[k] - phis;
        Lifted<R> pt = lift_(H, qm, pi[k]);
        su[k] = CP * pt.T + GRAV * g.zi[k] + phis;
        qu[k] = pt.qv;
        c[k] = eta[k] * (qm - pt.qv);
        hu = hm;
    }
    R C1 = R(0.0);
    for (int k = kt + 1; k <= kb; ++k) C1 = C1 + c[k];

    // D6: saturated entraining downdraft from the layer of minimum h between top and base.
    std::vector<R> etad(L + 1, R(0.0)), sd(L + 1, R(0.0)), qd(L + 1, R(0.0)), e1(L, R(0.0));
    R alpha = R(0.0), E1 = R(0.0);
    int kd = -1;
    if (kb - kt >= 2) {
        kd = kt + 1;
        for (int k = kt + 2; k <= kb - 1; ++k)
            if (val(h[k]) < val(h[kd])) kd = k;
        R ad = R(1.0);  // |eta_d| at the current interface
        R hd = h[kd];
        {
            int i = kd + 1;
            R H = hd - GRAV * g.zi[i] - phis;
            R Td = tsat_(H, pi[i], R((H - LV * q[kd]) / CP), nullptr);
            R qdv = qs_(Td, pi[i]);
            etad[i] = -ad;
            sd[i] = CP * Td + GRAV * g.zi[i] + phis;
            qd[i] = qdv;
            e1[kd] = qdv - q[kd];
        }
        for (int k = kd + 1; k <= kb - 1; ++k) {
            R Ed = epsd * ad * g.dz[k];
            R adn = ad + Ed;
            hd = (ad * hd + Ed * h[k]) / adn;
            int i = k + 1;
            R H = hd - GRAV * g.zi[i] - phis;
            R Td = tsat_(H, pi[i], R((H - LV * q[k]) / CP), nullptr);
            R qdn = qs_(Td, pi[i]);
            e1[k] = adn * qdn - ad * qd[k] - Ed * q[k];
            etad[i] = -adn;
            sd[i] = CP * Td + GRAV * g.zi[i] + phis;
            qd[i] = qdn;
            ad = adn;
        }
        for (int k = kd; k <= kb - 1; ++k) E1 = E1 + e1[k];
        alpha = R(P.alpha_dd);
        if (P.alpha_dd * val(E1) > P.evap_max_frac * val(C1)) alpha = P.evap_max_frac * C1 / E1;
    }

    // D7: flux-form unit tendencies with upwind environment values in the compensating flow.
    std::vector<R> Fs(L + 1, R(0.0)), Fq(L + 1, R(0.0));
    for (int i = kt + 1; i <= kb; ++i) {
        R m = eta[i] + alpha * etad[i];
        int up = val(m) >= 0.0 ? i - 1 : i;
        Fs[i] = eta[i] * (su[i] - s[up]) + alpha * etad[i] * (sd[i] - s[up]);
        Fq[i] = eta[i] * (qu[i] - q[up]) + alpha * etad[i] * (qd[i] - q[up]);
    }
    std::vector<R> dT1(L, R(0.0)), dq1(L, R(0.0));
    R P1 = R(0.0);
    for (int k = kt; k <= kb; ++k) {
        R net = c[k] - alpha * e1[k];
        dT1[k] = (Fs[k + 1] - Fs[k] + LV * net) * GRAV / (CP * g.dp[k]);
        dq1[k] = (Fq[k + 1] - Fq[k] - net) * GRAV / g.dp[k];
        P1 = P1 + net;
    }

    // D8: closure.  F = -(d CAPE) along the unit tendencies with kb, kt and the saturation flags
    // fixed, then M_c = CAPE / (tau * F).  The undilute parcel is perturbed through its
    // launch-layer state; a dilute one also through the air it entrained on the way up.
    R dh = CP * dT1[kb] + LV * dq1[kb];
    R Fsum = R(0.0);
    if (P.eps_cape > 0.0) {
        R dhm = dh, dqm = dq1[kb];
        for (int k = kb - 1; k >= kt; --k) {
            const double mix = P.eps_cape * (z[k] - z[k + 1]);
            dhm = (dhm + mix * (CP * dT1[k] + LV * dq1[k])) / (1.0 + mix);
            dqm = (dqm + mix * dq1[k]) / (1.0 + mix);
            R dTp, dqp;
            if (sat[k]) {
                R qsp = dqsdT_(Tp[k], pm[k]);
                dTp = dhm / (CP + LV * qsp);
                dqp = qsp * dTp;
            } else {
                dTp = (dhm - LV * dqm) / CP;
                dqp = dqm;
            }
            R dTvp = (1.0 + CVIR * qp[k]) * dTp + CVIR * Tp[k] * dqp;
            R dTve = (1.0 + CVIR * q[k]) * dT1[k] + CVIR * T[k] * dq1[k];
            Fsum = Fsum + g.lam[k] * (dTvp - dTve);
        }
    }
    for (int k = kt; k <= kb - 1 && !(P.eps_cape > 0.0); ++k) {
        R dTp, dqp;
        if (sat[k]) {
            R qsp = dqsdT_(Tp[k], pm[k]);
            dTp = dh / (CP + LV * qsp);
            dqp = qsp * dTp;
        } else {
            dTp = dT1[kb];
            dqp = dq1[kb];
        }
        R dTvp = (1.0 + CVIR * qp[k]) * dTp + CVIR * Tp[k] * dqp;
        R dTve = (1.0 + CVIR * q[k]) * dT1[k] + CVIR * T[k] * dq1[k];
        Fsum = Fsum + g.lam[k] * (dTvp - dTve);
    }
    R F = -RD * Fsum;
    o.kd = kd;
    o.F = F;
    o.alpha = alpha;
    o.C1 = C1;
    o.E1 = E1;
    o.P1 = P1;
    if (!(val(F) > 0.0)) {
        o.status = 2;
        return;
    }
    R Mc = o.cape / (tau * F);

    // D9: limiter keeping q >= 0 after one step dt.
    R Mlim = R(std::numeric_limits<double>::infinity());
    for (int k = kt; k <= kb; ++k)
        if (val(dq1[k]) < 0.0) {
            R m = q[k] / (-dt * dq1[k]);
            if (val(m) < val(Mlim)) Mlim = m;
        }
    R Mb = val(Mc) <= val(Mlim) ? Mc : Mlim;

    // D10: outputs.
    for (int k = kt; k <= kb; ++k) {
        o.dTdt[k] = Mb * dT1[k];
        o.dqdt[k] = Mb * dq1[k];
    }
    for (int i = kt + 1; i <= kb; ++i) {
        o.mu[i] = Mb * eta[i];
        o.md[i] = Mb * (alpha * etad[i]);
    }
    o.prec = Mb * P1;
    o.eta = eta;
    o.etad = etad;
    o.Mc = Mc;
    o.Mlim = Mlim;
    o.Mb = Mb;
    o.status = 0;
}

/* ---------------------------------------------------------------- shallow scheme (S1-S9) */
template <class R> struct ShallowRes {
    std::vector<R> dTdt, dqdt, mu, eta;
    R prec, cin, hs, qsrc, rho_s, sigw2, Mclos, Mlim, Mb, P1;
    int ks, klcl, klfc, kt, status;
};

// `state_checked`: the column's validity (C0) was already decided on the input state of the step;
// the deep-updated state of a valid column is not re-validated (its humidity can sit a rounding
// error below zero where the deep limiter binds).
// The mixing rates eps_sh and delta_sh are passed separately (as R) so that the forward-mode
// derivative can carry tangents along them.
template <class R>
void shallow_column(int L, const oracle_params_t &P, const R &eps_sh, const R &delta_sh,
                    const R *T, const R *q, const double *pm, const double *pi, const double *z,
                    double phis, double pblh, double tke, double dt, ShallowRes<R> &o,
                    bool state_checked = false) {
    o.dTdt.assign(L, R(0.0));
    o.dqdt.assign(L, R(0.0));
    o.mu.assign(L + 1, R(0.0));
    o.eta.assign(L + 1, R(0.0));
    o.prec = o.cin = o.hs = o.qsrc = o.rho_s = o.sigw2 = o.Mclos = o.Mb = o.P1 = R(0.0);
    o.Mlim = R(std::numeric_limits<double>::infinity());
    o.ks = o.klcl = o.klfc = o.kt = -1;
    if ((!state_checked && !column_valid(L, T, q, pm, pi, z, phis)) || !std::isfinite(pblh) ||
        !std::isfinite(tke)) {
        o.status = 6;
        return;
    }
    const Grid g = make_grid(L, pi, z);
    std::vector<R> s(L), h(L);
    for (int k = 0; k < L; ++k) {
        s[k] = CP * T[k] + GRAV * z[k] + phis;
        h[k] = s[k] + LV * q[k];
    }

    // S1: source = pressure-weighted mean over the boundary-layer layers (z <= pblh, always
    // including the lowest layer); the plume starts at the top interface of the highest one.
    int ks = L - 1;
    while (ks > 0 && z[ks - 1] <= pblh) --ks;
    R hsum = R(0.0), qsum = R(0.0);
    double wsum = 0.0;
    for (int k = L - 1; k >= ks; --k) {
        hsum = hsum + g.dp[k] * h[k];
        qsum = qsum + g.dp[k] * q[k];
        wsum = wsum + g.dp[k];
    }
    R hs = hsum / wsum, qsrc = qsum / wsum;
    o.ks = ks;
    o.hs = hs;
    o.qsrc = qsrc;

    // S2-S5: undilute parcel from the source, upward: lifting condensation level, level of free
    // convection, convective inhibition below it.
    int klcl = -1, klfc = -1;
    R cin = R(0.0);
    for (int k = ks - 1; k >= 0; --k) {
        if (klcl < 0 && pm[k] < P.p_lcl_min) break;
        if (klcl >= 0 && pm[k] < P.p_sh_top_min) break;
        R H = hs - GRAV * z[k] - phis;
        Lifted<R> pt = lift_(H, qsrc, pm[k]);
        R Bk = tv_(pt.T, pt.qv) - tv_(T[k], q[k]);
        if (klcl < 0 && pt.sat) klcl = k;
        if (klcl >= 0 && val(Bk) > 0.0 && pm[k] >= P.p_sh_top_min) {
            klfc = k;
            break;
        }
        if (val(Bk) < 0.0) cin = cin + RD * (-Bk) * g.lam[k];
    }
    o.klcl = klcl;
    o.klfc = klfc;
    if (klcl < 0) {
        o.status = 1;
        return;
    }
    if (klfc < 0) {
        o.status = 2;
        return;
    }
    o.cin = cin;
    if (val(cin) > P.cin_max) {
        o.status = 3;
        return;
    }
    // S6: cloud-base mass flux from the boundary-layer vertical-velocity spread and CIN.
    double sigw2 = P.c_tke * tke;
    o.sigw2 = R(sigw2);
    if (!(sigw2 > 0.0)) {
        o.status = 4;
        return;
    }
    R rho_s = pi[ks] / (RD * tv_(T[ks], q[ks]));
    double sigw = std::sqrt(sigw2);
    R Mclos = rho_s * sigw / SQRT_2PI * exp(-P.a_buoy * cin / sigw2);
    o.rho_s = rho_s;
    o.Mclos = Mclos;

    // S7: entraining-detraining plume with vertical-velocity equation and rain-out above qlcrit.
    std::vector<R> eta(L + 1, R(0.0)), slu(L + 1, R(0.0)), qtu(L + 1, R(0.0)), pr(L, R(0.0));
    eta[ks] = R(1.0);
    R hu = hs;
    {
        R H = hs - GRAV * g.zi[ks] - phis;
        Lifted<R> pt = lift_(H, qsrc, pi[ks]);
        R ql = qsrc - pt.qv;
        R r = val(ql) - P.qlcrit_sh > 0.0 ? ql - P.qlcrit_sh : R(0.0);
        pr[ks] = eta[ks] * r;
        qtu[ks] = qsrc - r;
        slu[ks] = CP * pt.T + GRAV * g.zi[ks] + phis - LV * (ql - r);
    }
    R w2 = sigw2 + 2.0 * P.a_buoy * cin;
    int kt = -1;
    for (int k = ks - 1; k >= 0; --k) {
        R E = eps_sh * eta[k + 1] * g.dz[k];
        R D = delta_sh * eta[k + 1] * g.dz[k];
        R en = eta[k + 1] + E - D;
        if (pi[k] < P.p_sh_top_min || k == 0 || !(val(en) > 0.0)) {
            kt = k;
            break;
        }
        R hm = ((eta[k + 1] - D) * hu + E * h[k]) / en;
        R qm = ((eta[k + 1] - D) * qtu[k + 1] + E * q[k]) / en;
        R H = hm - GRAV * g.zi[k] - phis;
        Lifted<R> pt = lift_(H, qm, pi[k]);
        R ql = qm - pt.qv;
        R r = val(ql) - P.qlcrit_sh > 0.0 ? ql - P.qlcrit_sh : R(0.0);
        R Trho = pt.T * (1.0 + CVIR * pt.qv - (ql - r));
        R Tve = tv_(T[k], q[k]);
        R Bk = GRAV * (Trho - Tve) / Tve;
        R w2n = w2 + 2.0 * g.dz[k] * (P.a_buoy * Bk - P.b_drag * eps_sh * w2);
        if (!(val(w2n) > 0.0)) {
            kt = k;
            break;
        }
        eta[k] = en;
        hu = hm;
        qtu[k] = qm - r;
        pr[k] = en * r;
        slu[k] = CP * pt.T + GRAV * g.zi[k] + phis - LV * (ql - r);
        w2 = w2n;
    }
    o.kt = kt;
    if (kt == ks - 1) {
        o.status = 5;
        return;
    }

    // S8: flux-form unit tendencies (updraft only; environment values from the layer above).
    std::vector<R> Fs(L + 1, R(0.0)), Fq(L + 1, R(0.0));
    for (int i = kt + 1; i <= ks; ++i) {
        Fs[i] = eta[i] * (slu[i] - s[i - 1]);
        Fq[i] = eta[i] * (qtu[i] - q[i - 1]);
    }
    std::vector<R> dT1(L, R(0.0)), dq1(L, R(0.0));
    R P1 = R(0.0);
    for (int k = kt; k <= ks; ++k) {
        dT1[k] = (Fs[k + 1] - Fs[k] + LV * pr[k]) * GRAV / (CP * g.dp[k]);
        dq1[k] = (Fq[k + 1] - Fq[k] - pr[k]) * GRAV / g.dp[k];
        P1 = P1 + pr[k];
    }
    // S9: limiter and outputs.
    R Mlim = R(std::numeric_limits<double>::infinity());
    for (int k = kt; k <= ks; ++k)
        if (val(dq1[k]) < 0.0) {
            R m = q[k] / (-dt * dq1[k]);
            if (val(m) < val(Mlim)) Mlim = m;
        }
    R Mb = val(Mclos) <= val(Mlim) ? Mclos : Mlim;
    for (int k = kt; k <= ks; ++k) {
        o.dTdt[k] = Mb * dT1[k];
        o.dqdt[k] = Mb * dq1[k];
    }
    for (int i = kt + 1; i <= ks; ++i) o.mu[i] = Mb * eta[i];
    o.eta = eta;
    o.prec = Mb * P1;
    o.Mlim = Mlim;
    o.Mb = Mb;
    o.P1 = P1;
    o.status = 0;
}

/* ---------------------------------------------------------------- convective tracer transport
 * A passive tracer C (mixing ratio per unit mass of air) is carried by the plumes exactly as the
 * schemes carry moist static energy: each plume mixes in environmental air where it entrains, the
 * updraft starts from the air of its source, the deep downdraft from layer k_d's air, and the
 * tendencies are the flux divergences of the plume-minus-environment fluxes with the same upwind
 * environmental values (D7, S8).  No sources or sinks: the column integral of the tendency,
 * weighted by dp/g, is zero.
 *
 * Momentum (a wind component) is carried the same way plus the convective pressure-gradient term
 * of Gregory, Kershaw & Inness (1997): the cloud-scale pressure gradient pulls the plume's wind
 * towards the environment's as the plume crosses environmental shear, so crossing a layer adds
 * cpgf times the plume's mass flux times the change of the environmental wind from the layer the
 * plume comes from to the layer it crosses (the layer below for an updraft, the layer above for
 * the downdraft).  cpgf = 0 is the passive tracer; cpgf = 1 makes the plume follow the
 * environment's shear exactly.  The tendency stays a flux divergence, so column momentum is
 * conserved. */
void deep_tracer(int L, const oracle_params_t &P, const DeepRes<double> &d, const Grid &g,
                 const double *C, double *out, double cpgf = 0.0) {
    for (int k = 0; k < L; ++k) out[k] = 0.0;
    if (d.status != 0) return;
    const int kb = d.kb, kt = d.kt, kd = d.kd;
    const std::vector<double> &eta = d.eta, &etad = d.etad;
    // Updraft (D5's mixing): the launch layer's air at interface kb, entraining layer k's air
    // between interfaces k+1 and k.
    std::vector<double> Cu(L + 1, 0.0), Cd(L + 1, 0.0);
    Cu[kb] = C[kb];
    for (int k = kb - 1; k >= kt + 1; --k) {
        const double E = P.eps_deep * eta[k + 1] * g.dz[k];
        Cu[k] = (eta[k + 1] * Cu[k + 1] + E * C[k] + cpgf * eta[k + 1] * (C[k] - C[k + 1])) /
                eta[k];
    }
    // Downdraft (D6's mixing): layer k_d's air at interface k_d+1, entraining layer k's air
    // between interfaces k and k+1.
    if (kd >= 0) {
        double ad = 1.0;
        Cd[kd + 1] = C[kd];
        for (int k = kd + 1; k <= kb - 1; ++k) {
            const double Ed = P.eps_deep * ad * g.dz[k];
            const double adn = ad + Ed;
            Cd[k + 1] = (ad * Cd[k] + Ed * C[k] + cpgf * ad * (C[k] - C[k - 1])) / adn;
            ad = adn;
        }
    }
    // D7's fluxes and their divergence, scaled by the base mass flux.
    std::vector<double> F(L + 1, 0.0);
    for (int i = kt + 1; i <= kb; ++i) {
        const double m = eta[i] + d.alpha * etad[i];
        const int up = m >= 0.0 ? i - 1 : i;
        F[i] = eta[i] * (Cu[i] - C[up]) + d.alpha * etad[i] * (Cd[i] - C[up]);
    }
    for (int k = kt; k <= kb; ++k) out[k] = d.Mb * (F[k + 1] - F[k]) * GRAV / g.dp[k];
}

void shallow_tracer(int L, const oracle_params_t &P, const ShallowRes<double> &o, const Grid &g,
                    const double *C, double *out, double cpgf = 0.0) {
    for (int k = 0; k < L; ++k) out[k] = 0.0;
    if (o.status != 0) return;
    const int ks = o.ks, kt = o.kt;
    const std::vector<double> &eta = o.eta;
    // S1's source: the pressure-weighted mean over the source layers.
    double csum = 0.0, wsum = 0.0;
    for (int k = L - 1; k >= ks; --k) {
        csum = csum + g.dp[k] * C[k];
        wsum = wsum + g.dp[k];
    }
    // S7's mixing: entrainment of layer k's air and detrainment of plume air.
    std::vector<double> Cu(L + 1, 0.0);
    Cu[ks] = csum / wsum;
    for (int k = ks - 1; k >= kt + 1; --k) {
        const double E = P.eps_sh * eta[k + 1] * g.dz[k];
        const double D = P.delta_sh * eta[k + 1] * g.dz[k];
        Cu[k] = ((eta[k + 1] - D) * Cu[k + 1] + E * C[k] + cpgf * eta[k + 1] * (C[k] - C[k + 1])) /
                eta[k];
    }
    // S8's fluxes (environment from the layer above) and their divergence.
    std::vector<double> F(L + 1, 0.0);
    for (int i = kt + 1; i <= ks; ++i) F[i] = eta[i] * (Cu[i] - C[i - 1]);
    for (int k = kt; k <= ks; ++k) out[k] = o.Mb * (F[k + 1] - F[k]) * GRAV / g.dp[k];
}

/* ---------------------------------------------------------------- level-major helpers */
struct ColIn {
    std::vector<double> T, q, pm, pi, z;
    double phis, pblh, tke;
};
void gather(const oracle_state_t *s, int L, int64_t c, ColIn &col) {
    const int64_t ld = s->ld;
    col.T.resize(L);
    col.q.resize(L);
    col.pm.resize(L);
    col.z.resize(L);
    col.pi.resize(L + 1);
    for (int k = 0; k < L; ++k) {
        col.T[k] = s->T[k * ld + c];
        col.q[k] = s->q[k * ld + c];
        col.pm[k] = s->p_mid[k * ld + c];
        col.z[k] = s->z[k * ld + c];
    }
    for (int k = 0; k <= L; ++k) col.pi[k] = s->p_int[k * ld + c];
    col.phis = s->phis ? s->phis[c] : 0.0;
    col.pblh = s->pblh ? s->pblh[c] : 0.0;
    col.tke = s->tke ? s->tke[c] : 0.0;
}

void scatter_deep(const DeepRes<double> &r, int L, int64_t ld, int64_t c, oracle_deep_out_t *o) {
    for (int k = 0; k < L; ++k) {
        o->dTdt[k * ld + c] = r.dTdt[k];
        o->dqdt[k * ld + c] = r.dqdt[k];
    }
    for (int k = 0; k <= L; ++k) {
        o->mu[k * ld + c] = r.mu[k];
        o->md[k * ld + c] = r.md[k];
    }
    o->prec[c] = r.prec;
    o->cape[c] = r.cape;
    o->klaunch[c] = r.kb;
    o->ktop[c] = r.kt;
    o->trig[c] = r.trig;
    o->status[c] = r.status;
}

void scatter_shallow(const ShallowRes<double> &r, int L, int64_t ld, int64_t c,
                     oracle_shallow_out_t *o) {
    for (int k = 0; k < L; ++k) {
        o->dTdt[k * ld + c] = r.dTdt[k];
        o->dqdt[k * ld + c] = r.dqdt[k];
    }
    for (int k = 0; k <= L; ++k) o->mu[k * ld + c] = r.mu[k];
    o->prec[c] = r.prec;
    // CIN is reported where it was completed (statuses 0, 3, 4, 5); kbase wherever the column is
    // valid; ktop only where the plume ran (statuses 0 and 5).
    const int st = r.status;
    o->cin[c] = (st == 0 || st == 3 || st == 4 || st == 5) ? r.cin : 0.0;
    o->kbase[c] = (st == 6) ? -1 : r.ks;
    o->ktop[c] = (st == 0 || st == 5) ? r.kt : -1;
    o->status[c] = st;
}

bool args_ok(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s) {
    return ncol >= 0 && nlev >= 2 && p && s && s->ld >= ncol && s->T && s->q && s->p_mid &&
           s->z && s->p_int;
}

void step_one(int L, const oracle_params_t *p, const oracle_state_t *s, int64_t c,
              oracle_deep_out_t *od, oracle_shallow_out_t *os) {
    ColIn col;
    gather(s, L, c, col);
    DeepRes<double> d;
    deep_column<double>(L, *p, p->tau, p->eps_deep, col.T.data(), col.q.data(), col.pm.data(),
                        col.pi.data(), col.z.data(), col.phis, s->dt, d);
    scatter_deep(d, L, s->ld, c, od);
    // Algorithm 1 order: the shallow scheme sees the state updated by the deep scheme.
    std::vector<double> T2(L), q2(L);
    for (int k = 0; k < L; ++k) {
        T2[k] = col.T[k] + s->dt * d.dTdt[k];
        q2[k] = col.q[k] + s->dt * d.dqdt[k];
    }
    // Validity is a property of the input column: an invalid one (deep status 3) is invalid for
    // the shallow scheme too; a valid one stays valid after the deep update.
    ShallowRes<double> sh;
    if (d.status == 3)
        shallow_column<double>(L, *p, p->eps_sh, p->delta_sh, col.T.data(), col.q.data(),
                               col.pm.data(), col.pi.data(), col.z.data(), col.phis, col.pblh,
                               col.tke, s->dt, sh);
    else
        shallow_column<double>(L, *p, p->eps_sh, p->delta_sh, T2.data(), q2.data(), col.pm.data(),
                               col.pi.data(), col.z.data(), col.phis, col.pblh, col.tke, s->dt, sh,
                               true);
    scatter_shallow(sh, L, s->ld, c, os);
}

// The step of one column (as step_one) with every state-dependent operation counted; returns the
// count including the two grids' own arithmetic (6 operations per layer each).
long long step_one_ops(int L, const oracle_params_t *p, const oracle_state_t *s, int64_t c) {
    ColIn col;
    gather(s, L, c, col);
    std::vector<Counted> T(L), q(L);
    for (int k = 0; k < L; ++k) {
        T[k] = col.T[k];
        q[k] = col.q[k];
    }
    g_ops = 0;
    DeepRes<Counted> d;
    deep_column<Counted>(L, *p, p->tau, p->eps_deep, T.data(), q.data(), col.pm.data(),
                         col.pi.data(), col.z.data(), col.phis, s->dt, d);
    std::vector<Counted> T2(L), q2(L);
    for (int k = 0; k < L; ++k) {
        T2[k] = T[k] + s->dt * d.dTdt[k];
        q2[k] = q[k] + s->dt * d.dqdt[k];
    }
    ShallowRes<Counted> sh;
    if (d.status == 3)
        shallow_column<Counted>(L, *p, p->eps_sh, p->delta_sh, T.data(), q.data(), col.pm.data(),
                                col.pi.data(), col.z.data(), col.phis, col.pblh, col.tke, s->dt,
                                sh);
    else
        shallow_column<Counted>(L, *p, p->eps_sh, p->delta_sh, T2.data(), q2.data(),
                                col.pm.data(), col.pi.data(), col.z.data(), col.phis, col.pblh,
                                col.tke, s->dt, sh, true);
    return g_ops + 2LL * 6 * L;
}

}  // namespace

/* ---------------------------------------------------------------- C entry points */
extern "C" {

int oracle_deep(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                oracle_deep_out_t *o) {
    if (!args_ok(ncol, nlev, p, s) || !o) return -1;
    ColIn col;
    for (int64_t c = 0; c < ncol; ++c) {
        gather(s, nlev, c, col);
        DeepRes<double> d;
        deep_column<double>(nlev, *p, p->tau, p->eps_deep, col.T.data(), col.q.data(),
                            col.pm.data(), col.pi.data(), col.z.data(), col.phis, s->dt, d);
        scatter_deep(d, nlev, s->ld, c, o);
    }
    return 0;
}

int oracle_shallow(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                   oracle_shallow_out_t *o) {
    if (!args_ok(ncol, nlev, p, s) || !o) return -1;
    ColIn col;
    for (int64_t c = 0; c < ncol; ++c) {
        gather(s, nlev, c, col);
        ShallowRes<double> r;
        shallow_column<double>(nlev, *p, p->eps_sh, p->delta_sh, col.T.data(), col.q.data(),
                               col.pm.data(), col.pi.data(), col.z.data(), col.phis, col.pblh,
                               col.tke, s->dt, r);
        scatter_shallow(r, nlev, s->ld, c, o);
    }
    return 0;
}

int oracle_step(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                oracle_deep_out_t *od, oracle_shallow_out_t *os) {
    if (!args_ok(ncol, nlev, p, s) || !od || !os) return -1;
    for (int64_t c = 0; c < ncol; ++c) step_one(nlev, p, s, c, od, os);
    return 0;
}

int oracle_tracers(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                   int ntr, const double *tracers, double *tend, double *deep_tend) {
    return oracle_transport(ncol, nlev, p, s, ntr, tracers, 0.0, tend, deep_tend);
}

int oracle_momentum(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                    const double *wind, double cpgf, double *tend, double *deep_tend) {
    if (!wind || !tend) return -1;
    return oracle_transport(ncol, nlev, p, s, 2, wind, cpgf, tend, deep_tend);
}

int oracle_transport(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                     int ntr, const double *tracers, double cpgf, double *tend, double *deep_tend) {
    if (!args_ok(ncol, nlev, p, s) || ntr < 0 || (ntr > 0 && (!tracers || !tend))) return -1;
    const int L = nlev;
    const int64_t ld = s->ld, plane = (int64_t)L * ld;
    ColIn col;
    std::vector<double> C(L), Cd(L), Cs(L), C2(L), T2(L), q2(L);
    for (int64_t c = 0; c < ncol; ++c) {
        gather(s, L, c, col);
        // The step (Algorithm 1): deep, the update, shallow on the updated state.
        DeepRes<double> d;
        deep_column<double>(L, *p, p->tau, p->eps_deep, col.T.data(), col.q.data(), col.pm.data(),
                            col.pi.data(), col.z.data(), col.phis, s->dt, d);
        for (int k = 0; k < L; ++k) {
            T2[k] = col.T[k] + s->dt * d.dTdt[k];
            q2[k] = col.q[k] + s->dt * d.dqdt[k];
        }
        ShallowRes<double> sh;
        if (d.status == 3)
            shallow_column<double>(L, *p, p->eps_sh, p->delta_sh, col.T.data(), col.q.data(),
                                   col.pm.data(), col.pi.data(), col.z.data(), col.phis,
                                   col.pblh, col.tke, s->dt, sh);
        else
            shallow_column<double>(L, *p, p->eps_sh, p->delta_sh, T2.data(), q2.data(),
                                   col.pm.data(), col.pi.data(), col.z.data(), col.phis,
                                   col.pblh, col.tke, s->dt, sh, true);
        const Grid g = make_grid(L, col.pi.data(), col.z.data());
        for (int t = 0; t < ntr; ++t) {
            for (int k = 0; k < L; ++k) C[k] = tracers[t * plane + k * ld + c];
            deep_tracer(L, *p, d, g, C.data(), Cd.data(), cpgf);
            // The shallow scheme transports the tracer updated by the deep transport.
            for (int k = 0; k < L; ++k) C2[k] = C[k] + s->dt * Cd[k];
            shallow_tracer(L, *p, sh, g, C2.data(), Cs.data(), cpgf);
            for (int k = 0; k < L; ++k) {
                tend[t * plane + k * ld + c] = Cd[k] + Cs[k];
                if (deep_tend) deep_tend[t * plane + k * ld + c] = Cd[k];
            }
        }
    }
    return 0;
}

int oracle_step_ops(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                    double *ops) {
    if (!args_ok(ncol, nlev, p, s) || !ops) return -1;
    for (int64_t c = 0; c < ncol; ++c) ops[c] = (double)step_one_ops(nlev, p, s, c);
    return 0;
}

int oracle_step_omp(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                    oracle_deep_out_t *od, oracle_shallow_out_t *os, int chunk, int nthreads) {
    if (!args_ok(ncol, nlev, p, s) || !od || !os || chunk < 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, chunk)
#endif
    for (int64_t c = 0; c < ncol; ++c) step_one(nlev, p, s, c, od, os);
    (void)nthreads;
    return 0;
}

int oracle_deep_column(int nlev, const oracle_params_t *p, const double *T, const double *q,
                       const double *p_mid, const double *p_int, const double *z, double phis,
                       double dt, double *dTdt, double *dqdt, double *mu, double *md, double *prec,
                       oracle_deep_diag_t *diag, double *eta, double *eta_d) {
    if (nlev < 2 || !p) return -1;
    DeepRes<double> d;
    deep_column<double>(nlev, *p, p->tau, p->eps_deep, T, q, p_mid, p_int, z, phis, dt, d);
    for (int k = 0; k < nlev; ++k) {
        if (dTdt) dTdt[k] = d.dTdt[k];
        if (dqdt) dqdt[k] = d.dqdt[k];
    }
    for (int k = 0; k <= nlev; ++k) {
        if (mu) mu[k] = d.mu[k];
        if (md) md[k] = d.md[k];
        if (eta) eta[k] = d.eta[k];
        if (eta_d) eta_d[k] = d.etad[k];
    }
    if (prec) *prec = d.prec;
    if (diag) {
        diag->kb = d.kb;
        diag->kt = d.kt;
        diag->kd = d.kd;
        diag->klim = d.klim;
        diag->status = d.status;
        diag->cape = d.cape;
        diag->F = d.F;
        diag->Mc = d.Mc;
        diag->Mlim = d.Mlim;
        diag->Mb = d.Mb;
        diag->alpha = d.alpha;
        diag->C1 = d.C1;
        diag->E1 = d.E1;
        diag->P1 = d.P1;
    }
    return 0;
}

int oracle_shallow_column(int nlev, const oracle_params_t *p, const double *T, const double *q,
                          const double *p_mid, const double *p_int, const double *z, double phis,
                          double pblh, double tke, double dt, double *dTdt, double *dqdt,
                          double *mu, double *prec, oracle_shallow_diag_t *diag) {
    if (nlev < 2 || !p) return -1;
    ShallowRes<double> r;
    shallow_column<double>(nlev, *p, p->eps_sh, p->delta_sh, T, q, p_mid, p_int, z, phis, pblh,
                           tke, dt, r);
    for (int k = 0; k < nlev; ++k) {
        if (dTdt) dTdt[k] = r.dTdt[k];
        if (dqdt) dqdt[k] = r.dqdt[k];
    }
    for (int k = 0; k <= nlev; ++k)
        if (mu) mu[k] = r.mu[k];
    if (prec) *prec = r.prec;
    if (diag) {
        diag->ks = r.ks;
        diag->klcl = r.klcl;
        diag->klfc = r.klfc;
        diag->kt = r.kt;
        diag->status = r.status;
        diag->hs = r.hs;
        diag->qs = r.qsrc;
        diag->cin = r.cin;
        diag->rho_s = r.rho_s;
        diag->sigw2 = r.sigw2;
        diag->Mclos = r.Mclos;
        diag->Mlim = r.Mlim;
        diag->Mb = r.Mb;
        diag->P1 = r.P1;
    }
    return 0;
}

int oracle_deep_parcel(int nlev, const oracle_params_t *p, const double *T, const double *q,
                       const double *p_mid, const double *p_int, const double *z, double phis,
                       double *B, int32_t *sat, double *Tp, double *qp) {
    if (nlev < 2 || !p) return -1;
    (void)p_int;
    std::vector<double> h(nlev);
    for (int k = 0; k < nlev; ++k) h[k] = CP * T[k] + GRAV * z[k] + phis + LV * q[k];
    int kb = -1;
    for (int k = nlev - 1; k >= 0; --k)
        if (p_mid[k] >= p->p_launch_min && (kb < 0 || h[k] > h[kb])) kb = k;
    for (int k = 0; k < nlev; ++k) {
        B[k] = 0.0;
        sat[k] = 0;
        Tp[k] = 0.0;
        qp[k] = 0.0;
    }
    if (kb < 0) return 0;
    for (int k = 0; k < kb; ++k) {
        double H = h[kb] - GRAV * z[k] - phis;
        Lifted<double> pt = lift_(H, q[kb], p_mid[k]);
        Tp[k] = pt.T;
        qp[k] = pt.qv;
        sat[k] = pt.sat;
        B[k] = tv_(pt.T, pt.qv) - tv_(T[k], q[k]);
    }
    return 0;
}

int oracle_deep_column_jvp(int nlev, const oracle_params_t *p, const double *T, const double *q,
                           const double *p_mid, const double *p_int, const double *z, double phis,
                           double dt, const double *dT, const double *dq, double dtau, double deps,
                           double *t_dTdt, double *t_dqdt, double *t_prec) {
    if (nlev < 2 || !p) return -1;
    std::vector<Dual> Td(nlev), qd(nlev);
    for (int k = 0; k < nlev; ++k) {
        Td[k] = Dual(T[k], dT ? dT[k] : 0.0);
        qd[k] = Dual(q[k], dq ? dq[k] : 0.0);
    }
    DeepRes<Dual> d;
    deep_column<Dual>(nlev, *p, Dual(p->tau, dtau), Dual(p->eps_deep, deps), Td.data(), qd.data(),
                      p_mid, p_int, z, phis, dt, d);
    for (int k = 0; k < nlev; ++k) {
        t_dTdt[k] = d.dTdt[k].d;
        t_dqdt[k] = d.dqdt[k].d;
    }
    *t_prec = d.prec.d;
    return d.status;
}

int oracle_shallow_column_jvp(int nlev, const oracle_params_t *p, const double *T,
                              const double *q, const double *p_mid, const double *p_int,
                              const double *z, double phis, double pblh, double tke, double dt,
                              const double *dT, const double *dq, double deps_sh,
                              double ddelta_sh, double *t_dTdt, double *t_dqdt, double *t_prec) {
    if (nlev < 2 || !p) return -1;
    std::vector<Dual> Td(nlev), qd(nlev);
    for (int k = 0; k < nlev; ++k) {
        Td[k] = Dual(T[k], dT ? dT[k] : 0.0);
        qd[k] = Dual(q[k], dq ? dq[k] : 0.0);
    }
    ShallowRes<Dual> r;
    shallow_column<Dual>(nlev, *p, Dual(p->eps_sh, deps_sh), Dual(p->delta_sh, ddelta_sh),
                         Td.data(), qd.data(), p_mid, p_int, z, phis, pblh, tke, dt, r);
    for (int k = 0; k < nlev; ++k) {
        t_dTdt[k] = r.dTdt[k].d;
        t_dqdt[k] = r.dqdt[k].d;
    }
    *t_prec = r.prec.d;
    return r.status;
}

// One column of the step (deep, the state update T + dt dTdt, q + dt dqdt, shallow on the
// updated state: Algorithm 1 order) with the tangent carried through all three.
int oracle_step_column_jvp(int nlev, const oracle_params_t *p, const double *T, const double *q,
                           const double *p_mid, const double *p_int, const double *z, double phis,
                           double pblh, double tke, double dt, const double *dT, const double *dq,
                           const double *dpar, double *t_deep, double *t_shallow,
                           int32_t *status) {
    if (nlev < 2 || !p || !dpar || !t_deep || !t_shallow || !status) return -1;
    const int L = nlev;
    std::vector<Dual> Td(L), qd(L);
    for (int k = 0; k < L; ++k) {
        Td[k] = Dual(T[k], dT ? dT[k] : 0.0);
        qd[k] = Dual(q[k], dq ? dq[k] : 0.0);
    }
    DeepRes<Dual> d;
    deep_column<Dual>(L, *p, Dual(p->tau, dpar[0]), Dual(p->eps_deep, dpar[1]), Td.data(),
                      qd.data(), p_mid, p_int, z, phis, dt, d);
    std::vector<Dual> T2(L), q2(L);
    for (int k = 0; k < L; ++k) {
        T2[k] = Td[k] + dt * d.dTdt[k];
        q2[k] = qd[k] + dt * d.dqdt[k];
    }
    ShallowRes<Dual> sh;
    const Dual es(p->eps_sh, dpar[2]), ds(p->delta_sh, dpar[3]);
    if (d.status == 3)
        shallow_column<Dual>(L, *p, es, ds, Td.data(), qd.data(), p_mid, p_int, z, phis, pblh,
                             tke, dt, sh);
    else
        shallow_column<Dual>(L, *p, es, ds, T2.data(), q2.data(), p_mid, p_int, z, phis, pblh,
                             tke, dt, sh, true);
    for (int k = 0; k < L; ++k) {
        t_deep[k] = d.dTdt[k].d;
        t_deep[L + k] = d.dqdt[k].d;
        t_shallow[k] = sh.dTdt[k].d;
        t_shallow[L + k] = sh.dqdt[k].d;
    }
    t_deep[2 * L] = d.prec.d;
    t_shallow[2 * L] = sh.prec.d;
    status[0] = d.status;
    status[1] = sh.status;
    return 0;
}

double oracle_es(double T) { return es_(T); }
double oracle_qs(double T, double p) { return qs_(T, p); }
double oracle_dqsdT(double T, double p) { return dqsdT_(T, p); }
double oracle_tsat(double H, double p, double T_guess, int *iterations) {
    return tsat_(H, p, T_guess, iterations);
}

}  // extern "C"
