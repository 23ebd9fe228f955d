// conv_adjoint.hip -- hand-written adjoint (reverse mode) of the deep convection scheme, D1-D10 of
// the written reading of the paper's deep convection (arXiv:1711.00289, Background and Algorithm
// 2: an entrainment loop and a precipitation loop around an iterative inversion).
//
// The derivative is taken through the branch the forward run took: launch layer kb, cloud top kt,
// downdraft start kd, every saturation flag, every upwind choice, the downdraft-strength branch
// (alpha_dd or the evaporation cap) and the base-flux branch (closure M_c or the humidity limiter,
// with its limiting layer) are held fixed.  It is checkpointed: from the inputs and the forward
// run's status / launch / top outputs, each active column recomputes its parcel, updraft,
// downdraft, tendencies and closure (storing the per-level values the reverse sweep needs in a
// per-thread scratch region of the caller's workspace), then runs the reverse sweep:
//   base flux -> closure F (with the parcel sensitivities, which need qs'') and CAPE -> parcel
//   (implicit derivative of the saturated inversion, dT/dH = 1/(cp + Lv qs')) -> flux-form
//   tendencies -> downdraft strength alpha -> downdraft recurrence -> updraft recurrence -> h.
// Outputs: dL/dT, dL/dq per level and dL/dtau, dL/deps_deep summed over columns in a fixed order.
//
// The shallow scheme (S1-S9, Algorithm 3) has an adjoint of the same shape (k_shallow_adjoint),
// and the two compose into the adjoint of a whole step (Algorithm 1: deep, the state update
// T' = T + dt dTdt, shallow on T'): the shallow adjoint runs first and yields dL/dT', which the
// deep adjoint then carries through the update, as the identity plus dt times an extra cotangent
// of the deep tendencies.
#include "conv_internal.hpp"

using namespace cvk;

namespace {

// Per-level scratch arrays (index = level or interface).
enum : int {
    P_TP = 0, P_QP, P_Q1, P_Q2, P_SAT,                      // parcel, layers kt..kb-1
    U_ETA, U_HM, U_QM, U_TU, U_QU, U_Q1, U_SAT, U_E, U_C,   // updraft (U_E, U_C per layer)
    D_AD, D_HD, D_TD, D_QD, D_Q1, D_ED, D_E1,               // downdraft (D_ED, D_E1 per layer)
    X_DT1, X_DQ1, X_UPW,                                    // unit tendencies, upwind flags
    G_T, G_Q, G_ETA, G_TU, G_QU, G_AD, G_TD, G_QD, G_C, G_E1, G_DT1, G_DQ1,
    GD_T, GD_Q,                                             // the downdraft's part of G_T, G_Q
    G2_T, G2_Q,                                             // the lower interfaces' part
    N_ADJ
};

struct AdjWork {
    int *cnt;
    int *list;
    double *pgrad;  // [2][ld]: per-column dL/dtau, dL/deps
    double *scr;
    int64_t stride;
    int lmax;
    const double *cT, *cq, *cP;  // cotangents of dTdt, dqdt [nlev][ld] and prec [ld] (may be NULL)
    double *gT, *gq;             // [nlev][ld]
    // Step mode: dL/dT', dL/dq' of the shallow scheme at the updated state (may alias gT, gq; NULL
    // outside step mode).  They add dt*x to the tendencies' cotangents and x to the gradients.
    const double *xT, *xq;
};

// Active (status 0) columns into a list, and zero parameter-gradient rows.  The gradients of the
// other columns are written by k_deep_adjoint's blocks that hold no chunk of the list, while the
// rest run their chains: as a pass of its own here, before the adjoint, the 27 MB took about
// 6 us of the backward's 0.122 ms.
__global__ __launch_bounds__(BLOCK) void k_adj_compact(Member M, AdjWork w) {
    const int64_t col = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool live = col < M.ncol;
    const int64_t ld = M.ld;
    const bool act = live && M.dout.status[col] == 0;
    if (live) {
        w.pgrad[col] = 0.0;
        w.pgrad[ld + col] = 0.0;
    }
    const int slot = wave_append(act, &w.cnt[0]);
    if (slot >= 0) w.list[slot] = (int)col;
}

constexpr int AB = 4;  // levels per batch of loads in the reverse sweeps

// The deep adjoint runs as blocks of four wavefronts on the same 64 columns (lane l of each on
// column l), which take the independent chains of a column in parallel and meet at block
// barriers:
//   phase 1  wavefront 0: updraft (D5); wavefronts 1 and 3: parcel, CAPE and the closure's parcel
//            sums (D2-D4), alternate layers each; wavefront 2: downdraft start and recurrence (D6);
//   phase 2  all four: alpha and the unit tendencies (D6-D7), a quarter of the layers each;
//            then wavefront 0: closure and limiter (D8-D9), the start of the reverse sweep (D10,
//            D9/D8) and the environment's terms of the closure's adjoint;
//   phase 3  wavefronts 0 and 2: adjoint of the tendencies (the net sources, and a third and two
//            thirds of the interfaces' fluxes); wavefronts 1 and 3: adjoint of the parcel's terms
//            (into the launch layer's h and q), on the layers they lifted;
//   phase 4  wavefronts 0 and 2: adjoint of alpha; then wavefront 0: updraft recurrence in
//            reverse, the launch layer; wavefront 2: downdraft recurrence in reverse (into its own
//            accumulators and its own part of dL/deps);
//   phase 5  all four: dL/dT, dL/dq out (a quarter of the levels each); the parameter gradients.
// The four share the column's scratch slot.  Values that cross wavefronts go through LDS.
constexpr int ADJ_WAVES = 4;

__global__ __launch_bounds__(ADJ_WAVES * WAVE) void k_deep_adjoint(Member M, AdjWork w) {
    const int n = w.cnt[0];
    const int lane = threadIdx.x % WAVE;
    const int role = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int64_t sid = (int64_t)blockIdx.x * WAVE + lane;  // the column's scratch slot
    const int L = M.nlev;
    const int64_t ld = M.ld;
    const conv_params_t &P = M.P;
    const double tau = P.tau, epsd = P.eps_deep, beta = P.evap_max_frac, dt = M.dt;
    double *scr = w.scr;
#define S(arr, lev) scr[((int64_t)(arr) * (w.lmax + 1) + (lev)) * w.stride + sid]
    __shared__ double x_cape[2][WAVE], x_SA[2][WAVE], x_SB[2][WAVE], x_E1[WAVE], x_gF[WAVE],
        x_gcape[WAVE], x_dT1b[WAVE], x_dq1b[WAVE], x_ghkb[2][WAVE], x_gqkb[2][WAVE], x_geps[WAVE];
    __shared__ double x_C1[WAVE], x_P1[ADJ_WAVES][WAVE], x_Fenv[ADJ_WAVES][WAVE],
        x_Mlim[ADJ_WAVES][WAVE];
    __shared__ double x_galpha[2][WAVE], x_gMb[ADJ_WAVES][WAVE];
    __shared__ int x_kd[WAVE], x_skip[WAVE], x_klim[ADJ_WAVES][WAVE];

    for (int64_t base = (int64_t)blockIdx.x * WAVE; base < n; base += (int64_t)gridDim.x * WAVE) {
        const int64_t slot = base + lane;
        const bool act = slot < n;
        const int64_t col = act ? w.list[slot] : 0;
        const int kb = act ? M.dout.klaunch[col] : 0, kt = act ? M.dout.ktop[col] : 0;
        const double phis = act ? M.phis[col] : 0.0;
        auto Tk = [&](int k) { return AT(M.T, k); };
        auto qk = [&](int k) { return AT(M.q, k); };
        auto hk = [&](int k) { return (CP * AT(M.T, k) + GRAV * AT(M.z, k) + phis) + LV * AT(M.q, k); };
        auto zi = [&](int i) { return 0.5 * (AT(M.z, i - 1) + AT(M.z, i)); };
        const double hkb = act ? hk(kb) : 0.0, qkb = act ? qk(kb) : 0.0;
        // Carried from one phase to the next by the wavefront that computes them.
        double C1 = 0.0, gtau = 0.0, geps = 0.0, gepsd = 0.0, gF = 0.0, gcape = 0.0;
        double dT1b = 0.0, dq1b = 0.0, ghkb = 0.0, gqkb = 0.0, gP1 = 0.0;
        int kd = -1;
        double alpha = 0.0, E1 = 0.0;
        bool capped = false, skip = false;

        // ============================================ phase 1: forward recomputation
        if (act && (role == 1 || role == 3)) {
            // D2-D4: parcel over [kt, kb), CAPE and the closure's parcel sensitivities; wavefront 1
            // takes layers kb-1, kb-3, .., wavefront 3 layers kb-2, kb-4, .. (each lift starts from
            // the previous one of its own wavefront), each its own part of the three sums.
            const int half = role == 1 ? 0 : 1;
            double cape = 0.0, SA = 0.0, SB = 0.0;
            {
                Hint hp;
                hp.clear();
                // The next layer's inputs are loaded one iteration ahead (clamped at kt).
                struct PL {
                    double z, pm, T, q, pt, pb;
                };
                auto pload = [&](int k) {
                    PL v;
                    const int kk = max(k, kt);
                    v.z = AT(M.z, kk);
                    v.pm = AT(M.pm, kk);
                    v.T = Tk(kk);
                    v.q = qk(kk);
                    v.pt = AT(M.pi, kk);
                    v.pb = AT(M.pi, kk + 1);
                    return v;
                };
                PL nx = pload(kb - 1 - half);
                for (int k = kb - 1 - half; k >= kt; k -= 2) {
                    const PL v = nx;
                    nx = pload(k - 2);
                    const Lifted r = lift(hkb - GRAV * v.z - phis, qkb, v.pm, hp);
                    // The closure's parcel sensitivity needs qs' and qs'' at the root itself (the
                    // solver carries qs'' only to zeroth order), so they are evaluated there.
                    const Sat sr = r.sat ? sat_eval(r.T, v.pm) : Sat{0.0, 0.0, 0.0, 0.0};
                    S(P_TP, k) = r.T;
                    S(P_QP, k) = r.qv;
                    S(P_Q1, k) = sr.dqs;
                    S(P_Q2, k) = sr.d2qs;
                    S(P_SAT, k) = r.sat ? 1.0 : 0.0;
                    const double lam = log(v.pb / v.pt);
                    cape += RD * (tv(r.T, r.qv) - tv(v.T, v.q)) * lam;
                    double ca, cb;
                    if (r.sat) {
                        const double c = (1.0 + CVIR * r.qv) + CVIR * r.T * sr.dqs;
                        const double rden = frcp(CP + LV * sr.dqs);
                        ca = c * CP * rden;
                        cb = c * LV * rden;
                    } else {
                        ca = 1.0 + CVIR * r.qv;
                        cb = CVIR * r.T;
                    }
                    SA += lam * ca;
                    SB += lam * cb;
                }
            }
            x_cape[half][lane] = cape;
            x_SA[half][lane] = SA;
            x_SB[half][lane] = SB;
            // The reverse sweep's accumulators start at zero (the parcel is the shortest chain of
            // this phase): alternate levels of kt .. kb+1 each.
            for (int lev = kt + half; lev <= kb + 1; lev += 2)
                for (int a = G_T; a < N_ADJ; ++a) S(a, lev) = 0.0;
        } else if (act && role == 0) {
            // D5: updraft.
            {
                Hint hu;
                hu.clear();
                double zlo = zi(kb);
                const Lifted r0 = lift(hkb - GRAV * zlo - phis, qkb, AT(M.pi, kb), hu);
                S(U_ETA, kb) = 1.0;
                S(U_HM, kb) = hkb;
                S(U_QM, kb) = qkb;
                S(U_TU, kb) = r0.T;
                S(U_QU, kb) = r0.qv;
                S(U_Q1, kb) = r0.dqs;
                S(U_SAT, kb) = r0.sat ? 1.0 : 0.0;
                C1 = qkb - r0.qv;
                S(U_C, kb) = C1;
                double eta = 1.0, hum = hkb, qup = r0.qv;
                struct UL {
                    double za, z, T, q, p;  // heights of layers k-1 and k, T, q, top pressure of k
                };
                auto uload = [&](int k) {
                    UL v;
                    const int kk = max(k, kt + 1);
                    v.za = AT(M.z, kk - 1);
                    v.z = AT(M.z, kk);
                    v.T = Tk(kk);
                    v.q = qk(kk);
                    v.p = AT(M.pi, kk);
                    return v;
                };
                UL nx = uload(kb - 1);
                for (int k = kb - 1; k >= kt + 1; --k) {
                    const UL v = nx;
                    nx = uload(k - 1);
                    const double zk = 0.5 * (v.za + v.z);
                    const double E = epsd * eta * (zk - zlo);
                    const double etan = eta + E;
                    const double hm = (eta * hum + E * ((CP * v.T + GRAV * v.z + phis) + LV * v.q)) / etan;
                    const double qm = (eta * qup + E * v.q) / etan;
                    const Lifted r = lift(hm - GRAV * zk - phis, qm, v.p, hu);
                    const double c = etan * (qm - r.qv);
                    S(U_ETA, k) = etan;
                    S(U_HM, k) = hm;
                    S(U_QM, k) = qm;
                    S(U_TU, k) = r.T;
                    S(U_QU, k) = r.qv;
                    S(U_Q1, k) = r.dqs;
                    S(U_SAT, k) = r.sat ? 1.0 : 0.0;
                    S(U_E, k) = E;
                    S(U_C, k) = c;
                    C1 += c;
                    eta = etan;
                    hum = hm;
                    qup = r.qv;
                    zlo = zk;
                }
            }
            x_C1[lane] = C1;
        } else if (act) {
            // D6: downdraft.
            if (kb - kt >= 2) {
                kd = kt + 1;
                double hkd = hk(kd);
                for (int k = kt + 2; k <= kb - 1; ++k) {
                    const double h = hk(k);
                    if (h < hkd) {
                        kd = k;
                        hkd = h;
                    }
                }
                Hint hdn;
                hdn.clear();
                double ad = 1.0, hd = hkd, zii = zi(kd + 1);
                Sat s;
                double H = hd - GRAV * zii - phis;
                double Td = tsat_h(H, AT(M.pi, kd + 1), (H - LV * qk(kd)) * RCP_CP, s, hdn);
                double qd = s.qs;
                S(D_AD, kd + 1) = 1.0;
                S(D_HD, kd + 1) = hd;
                S(D_TD, kd + 1) = Td;
                S(D_QD, kd + 1) = qd;
                S(D_Q1, kd + 1) = s.dqs;
                E1 = qd - qk(kd);
                S(D_E1, kd) = E1;
                struct DL {
                    double z, zb, T, q, pb;  // heights of layers k and k+1, T, q, bottom pressure of k
                };
                auto dload = [&](int k) {
                    DL v;
                    const int kk = min(k, kb - 1);
                    v.z = AT(M.z, kk);
                    v.zb = AT(M.z, kk + 1);
                    v.T = Tk(kk);
                    v.q = qk(kk);
                    v.pb = AT(M.pi, kk + 1);
                    return v;
                };
                DL nx = dload(kd + 1);
                for (int k = kd + 1; k <= kb - 1; ++k) {
                    const DL v = nx;
                    nx = dload(k + 1);
                    const double zlow = 0.5 * (v.z + v.zb);
                    const double Ed = epsd * ad * (zii - zlow);
                    const double adn = ad + Ed;
                    hd = (ad * hd + Ed * ((CP * v.T + GRAV * v.z + phis) + LV * v.q)) / adn;
                    H = hd - GRAV * zlow - phis;
                    Td = tsat_h(H, v.pb, (H - LV * v.q) * RCP_CP, s, hdn);
                    const double e1 = adn * s.qs - ad * qd - Ed * v.q;
                    S(D_ED, k) = Ed;
                    S(D_E1, k) = e1;
                    S(D_AD, k + 1) = adn;
                    S(D_HD, k + 1) = hd;
                    S(D_TD, k + 1) = Td;
                    S(D_QD, k + 1) = s.qs;
                    S(D_Q1, k + 1) = s.dqs;
                    E1 += e1;
                    ad = adn;
                    qd = s.qs;
                    zii = zlow;
                }
            }
            x_kd[lane] = kd;
            x_E1[lane] = E1;
        }
        __syncthreads();

        // ============================================ phase 2a: alpha and the tendencies (all four)
        // Every wavefront derives alpha (the same arithmetic), then takes a quarter of the layers
        // kt..kb; a range that starts below kt first recomputes the flux at its top interface.
        if (act) {
            kd = x_kd[lane];
            E1 = x_E1[lane];
            const double C1u = x_C1[lane];
            if (kd >= 0) {
                alpha = P.alpha_dd;
                if (P.alpha_dd * E1 > beta * C1u) {
                    alpha = beta * C1u / E1;
                    capped = true;
                }
            }
            const int len = (kb - kt + ADJ_WAVES) / ADJ_WAVES;
            const int ks = kt + role * len, ke = min(ks + len - 1, kb);
            // D7-D9: unit tendencies, F, limiter.
            double P1 = 0.0, Fenv = 0.0, Mlim = __builtin_inf();
            int klim_at = -1;
            if (ks <= kb) {
                double Fs_top = 0.0, Fq_top = 0.0;
                // Layers k0 .. k0+AB-1 and their bottom interfaces, loaded together (levels clamped
                // to kb; the upwind candidates of both sides are loaded, the choice made after).
                for (int k0 = ks > kt ? ks - 1 : kt; k0 <= ke; k0 += AB) {
                    struct V {
                        double T, q, z, pt, pb, Tb, qb, zb, et, ad, tu, qu, td, qd, c, e1;
                    } v[AB];
#pragma unroll
                    for (int j = 0; j < AB; ++j) {
                        const int k = min(k0 + j, kb), i = min(k + 1, kb);
                        v[j].T = Tk(k);
                        v[j].q = qk(k);
                        v[j].z = AT(M.z, k);
                        v[j].pt = AT(M.pi, k);
                        v[j].pb = AT(M.pi, k + 1);
                        v[j].Tb = Tk(i);
                        v[j].qb = qk(i);
                        v[j].zb = AT(M.z, i);
                        v[j].et = S(U_ETA, i);
                        v[j].ad = S(D_AD, i);
                        v[j].tu = S(U_TU, i);
                        v[j].qu = S(U_QU, i);
                        v[j].td = S(D_TD, i);
                        v[j].qd = S(D_QD, i);
                        v[j].c = S(U_C, k);
                        v[j].e1 = S(D_E1, k);
                    }
#pragma unroll
                    for (int j = 0; j < AB; ++j) {
                        const int k = k0 + j;
                        if (k > ke) break;
                        const bool own = k >= ks;  // else only the flux at the range's top
                        double Fs = 0.0, Fq = 0.0;
                        const int i = k + 1;
                        if (i <= kb) {
                            const double et = v[j].et;
                            const bool dn = kd >= 0 && i >= kd + 1;
                            const double ed = dn ? -v[j].ad : 0.0;
                            const bool upw = et + alpha * ed >= 0.0;  // upwind layer i-1 = k, else i
                            const double s_up = upw ? CP * v[j].T + GRAV * v[j].z + phis
                                                    : CP * v[j].Tb + GRAV * v[j].zb + phis;
                            const double q_up = upw ? v[j].q : v[j].qb;
                            const double zii = 0.5 * (v[j].z + v[j].zb);
                            Fs = et * ((CP * v[j].tu + GRAV * zii + phis) - s_up);
                            Fq = et * (v[j].qu - q_up);
                            if (dn) {
                                Fs += alpha * ed * ((CP * v[j].td + GRAV * zii + phis) - s_up);
                                Fq += alpha * ed * (v[j].qd - q_up);
                            }
                            if (own) S(X_UPW, i) = upw ? 1.0 : 0.0;
                        }
                        if (!own) {
                            Fs_top = Fs;
                            Fq_top = Fq;
                            continue;
                        }
                        const double c = (k >= kt + 1) ? v[j].c : 0.0;
                        const double e1 = (kd >= 0 && k >= kd && k <= kb - 1) ? v[j].e1 : 0.0;
                        const double net = c - alpha * e1;
                        const double dp = v[j].pb - v[j].pt;
                        const double dT1 = (Fs - Fs_top + LV * net) * GRAV / (CP * dp);
                        const double dq1 = (Fq - Fq_top - net) * GRAV / dp;
                        S(X_DT1, k) = dT1;
                        S(X_DQ1, k) = dq1;
                        P1 += net;
                        if (k <= kb - 1)
                            Fenv += log(v[j].pb / v[j].pt) *
                                    ((1.0 + CVIR * v[j].q) * dT1 + CVIR * v[j].T * dq1);
                        if (dq1 < 0.0) {
                            const double m = v[j].q / (-dt * dq1);
                            if (m < Mlim) {
                                Mlim = m;
                                klim_at = k;
                            }
                        }
                        Fs_top = Fs;
                        Fq_top = Fq;
                    }
                }
            }
            x_P1[role][lane] = P1;
            x_Fenv[role][lane] = Fenv;
            x_Mlim[role][lane] = Mlim;
            x_klim[role][lane] = klim_at;
        }
        __syncthreads();

        // ============================================ phase 2b: closure and the reverse sweep's start
        // Every wavefront combines the ranges' sums (in order; the limiter's first smallest ratio,
        // as over one sweep) and derives the closure (the same arithmetic); D10 takes a quarter of
        // the layers each.
        bool closure = false;
        double Mc = 0.0, Mb = 0.0, Mlim = __builtin_inf(), P1 = 0.0, F = 0.0;
        int klim_at = -1;
        double SA = 0.0, SB = 0.0;
        if (act) {
            const double cape = x_cape[0][lane] + x_cape[1][lane];
            SA = x_SA[0][lane] + x_SA[1][lane];
            SB = x_SB[0][lane] + x_SB[1][lane];
            double Fenv = 0.0;
            for (int r = 0; r < ADJ_WAVES; ++r) {
                P1 += x_P1[r][lane];
                Fenv += x_Fenv[r][lane];
                if (x_Mlim[r][lane] < Mlim) {
                    Mlim = x_Mlim[r][lane];
                    klim_at = x_klim[r][lane];
                }
            }
            dT1b = S(X_DT1, kb);
            dq1b = S(X_DQ1, kb);
            F = -RD * (dT1b * SA + dq1b * SB - Fenv);
            skip = !(F > 0.0);
            if (skip && role == 0) {
                // Not reachable for a status-0 column; no derivative there.
                for (int k = 0; k < L; ++k) {
                    AT(w.gT, k) = w.xT ? AT(w.xT, k) : 0.0;
                    AT(w.gq, k) = w.xq ? AT(w.xq, k) : 0.0;
                }
                w.pgrad[col] = 0.0;
                w.pgrad[ld + col] = 0.0;
            }
            if (role == 0) x_skip[lane] = skip ? 1 : 0;
            Mc = cape / (tau * F);
            closure = Mc <= Mlim;
            Mb = closure ? Mc : Mlim;
        }
        if (act && !skip) {
            // ============================================ reverse sweep (accumulators zeroed in 1)
            // The reverse sweep's loops load AB levels at a time (levels clamped to the loop's
            // range, so every load is in range; values past the end are not used), then compute
            // those levels in order: one memory round trip per AB levels instead of one per level.
            // A loop that adds into a neighbouring level's accumulator keeps the batch's
            // accumulators in registers.
            // D10: outputs = M_b * unit profiles.
            const int len = (kb - kt + ADJ_WAVES) / ADJ_WAVES;
            const int k0a = kt + role * len, k1a = min(k0a + len - 1, kb);
            double gMb = 0.0;
            for (int k0 = k0a; k0 <= k1a; k0 += AB) {
                double cT[AB], cq[AB], d1[AB], q1[AB];
#pragma unroll
                for (int j = 0; j < AB; ++j) {
                    const int k = min(k0 + j, k1a);
                    cT[j] = (w.cT ? AT(w.cT, k) : 0.0) + (w.xT ? dt * AT(w.xT, k) : 0.0);
                    cq[j] = (w.cq ? AT(w.cq, k) : 0.0) + (w.xq ? dt * AT(w.xq, k) : 0.0);
                    d1[j] = S(X_DT1, k);
                    q1[j] = S(X_DQ1, k);
                }
#pragma unroll
                for (int j = 0; j < AB; ++j) {
                    const int k = k0 + j;
                    if (k > k1a) break;
                    gMb += cT[j] * d1[j] + cq[j] * q1[j];
                    S(G_DT1, k) = cT[j] * Mb;
                    S(G_DQ1, k) = cq[j] * Mb;
                }
            }
            x_gMb[role][lane] = gMb;
        }
        __syncthreads();
        if (act && role == 0 && !skip) {
            double gMb = 0.0;
            for (int r = 0; r < ADJ_WAVES; ++r) gMb += x_gMb[r][lane];
            const double cPc = w.cP ? w.cP[col] : 0.0;
            gMb += cPc * P1;
            gP1 = cPc * Mb;
            // D9/D8: base-flux branch.
            if (closure) {
                gcape = gMb / (tau * F);
                gF = -gMb * Mc / F;
                gtau = -gMb * Mc / tau;
            } else {
                const double dq1m = S(X_DQ1, klim_at);
                S(G_Q, klim_at) += gMb / (-dt * dq1m);
                S(G_DQ1, klim_at) += gMb * (-Mlim / dq1m);
            }
            S(G_DT1, kb) += -RD * gF * SA;
            S(G_DQ1, kb) += -RD * gF * SB;
            x_gF[lane] = gF;
            x_gcape[lane] = gcape;
            x_dT1b[lane] = dT1b;
            x_dq1b[lane] = dq1b;
        }
        __syncthreads();
        if (act && !skip) {
            // D8 closure F and D4 CAPE: the environment's terms, a quarter of the layers each (the
            // parcel's go to hkb, qkb: the parcel wavefronts, next phase).
            gF = x_gF[lane];
            gcape = x_gcape[lane];
            const int len = (kb - kt - 1 + ADJ_WAVES) / ADJ_WAVES;
            const int k0b = kt + role * len, k1b = min(k0b + len - 1, kb - 1);
            for (int k0 = k0b; k0 <= k1b; k0 += AB) {
              struct V {
                  double pt, pb, T, q, dT1, dq1, gdt, gdq, gT, gq;
              } v[AB];
#pragma unroll
              for (int j = 0; j < AB; ++j) {
                  const int k = min(k0 + j, k1b);
                  v[j].pt = AT(M.pi, k);
                  v[j].pb = AT(M.pi, k + 1);
                  v[j].T = Tk(k);
                  v[j].q = qk(k);
                  v[j].dT1 = S(X_DT1, k);
                  v[j].dq1 = S(X_DQ1, k);
                  v[j].gdt = S(G_DT1, k);
                  v[j].gdq = S(G_DQ1, k);
                  v[j].gT = S(G_T, k);
                  v[j].gq = S(G_Q, k);
              }
#pragma unroll
              for (int j = 0; j < AB; ++j) {
                const int k = k0 + j;
                if (k > k1b) break;
                const double lam = log(v[j].pb / v[j].pt), T = v[j].T, q = v[j].q;
                const double dT1 = v[j].dT1, dq1 = v[j].dq1;
                S(G_DT1, k) = v[j].gdt + RD * gF * lam * (1.0 + CVIR * q);
                S(G_DQ1, k) = v[j].gdq + RD * gF * lam * CVIR * T;
                double gTk = RD * gF * lam * CVIR * dq1;
                double gqk = RD * gF * lam * CVIR * dT1;
                const double gB = RD * lam * gcape;
                gTk -= gB * (1.0 + CVIR * q);
                gqk -= gB * CVIR * T;
                S(G_T, k) = v[j].gT + gTk;
                S(G_Q, k) = v[j].gq + gqk;
              }
            }
        }
        __syncthreads();

        // ============================================ phase 3
        // Wavefront 0: net sources of every layer and the fluxes of interfaces kt+1 .. im;
        // wavefront 2: the fluxes of interfaces im+1 .. kb, adding into its own layer accumulators
        // (G2_T, G2_Q: the layer between the two ranges can take both).
        const int im = kt + (kb - kt) / 3;
        if (act && (role == 0 || role == 2) && x_skip[lane] == 0) {
            // D7 tendencies: net sources per layer, fluxes per interface.
            double galpha = 0.0;
            const int iA = role == 0 ? kt + 1 : im + 1, iB = role == 0 ? im : kb;
            const int aT = role == 0 ? G_T : G2_T, aQ = role == 0 ? G_Q : G2_Q;
            if (role == 0) {
            for (int k0 = kt; k0 <= kb; k0 += AB) {
                double pt[AB], pb[AB], gdt[AB], gdq[AB], gc[AB], ge[AB], e1[AB];
#pragma unroll
                for (int j = 0; j < AB; ++j) {
                    const int k = min(k0 + j, kb);
                    pt[j] = AT(M.pi, k);
                    pb[j] = AT(M.pi, k + 1);
                    gdt[j] = S(G_DT1, k);
                    gdq[j] = S(G_DQ1, k);
                    gc[j] = S(G_C, k);
                    ge[j] = S(G_E1, k);
                    e1[j] = S(D_E1, k);
                }
#pragma unroll
                for (int j = 0; j < AB; ++j) {
                    const int k = k0 + j;
                    if (k > kb) break;
                    const double dp = pb[j] - pt[j];
                    const double gnet = LV * GRAV / (CP * dp) * gdt[j] - GRAV / dp * gdq[j] + gP1;
                    if (k >= kt + 1) S(G_C, k) = gc[j] + gnet;
                    if (kd >= 0 && k >= kd && k <= kb - 1) {
                        S(G_E1, k) = ge[j] + -alpha * gnet;
                        galpha -= gnet * e1[j];
                    }
                }
            }
            }
            // Interfaces i0 .. i0+AB-1 touch the layer accumulators of layers i0-1 .. i0+AB-1 (the
            // upwind layer of interface i is i-1 or i): those are held in registers for the batch
            // and stored once, each layer by the batch that last adds to it before the next loads it.
            for (int i0 = iA; i0 <= iB; i0 += AB) {
                struct V {
                    double pa, pm, pb, gdta, gdtb, gdqa, gdqb, et, upw, Ta, za, qa, Tb, zb, qb, tu, qu, ad,
                        td, qd, geta, gtu, gqu, gad, gtd, gqd;
                } v[AB];
                double gT[AB + 1], gq[AB + 1];
#pragma unroll
                for (int j = 0; j <= AB; ++j) {
                    const int k = min(i0 - 1 + j, iB);
                    gT[j] = S(aT, k);
                    gq[j] = S(aQ, k);
                }
#pragma unroll
                for (int j = 0; j < AB; ++j) {
                    const int i = min(i0 + j, iB);
                    v[j].pa = AT(M.pi, i - 1);
                    v[j].pm = AT(M.pi, i);
                    v[j].pb = AT(M.pi, i + 1);
                    v[j].gdta = S(G_DT1, i - 1);
                    v[j].gdtb = S(G_DT1, i);
                    v[j].gdqa = S(G_DQ1, i - 1);
                    v[j].gdqb = S(G_DQ1, i);
                    v[j].et = S(U_ETA, i);
                    v[j].upw = S(X_UPW, i);
                    v[j].Ta = Tk(i - 1);
                    v[j].za = AT(M.z, i - 1);
                    v[j].qa = qk(i - 1);
                    v[j].Tb = Tk(i);
                    v[j].zb = AT(M.z, i);
                    v[j].qb = qk(i);
                    v[j].tu = S(U_TU, i);
                    v[j].qu = S(U_QU, i);
                    v[j].ad = S(D_AD, i);
                    v[j].td = S(D_TD, i);
                    v[j].qd = S(D_QD, i);
                    v[j].geta = S(G_ETA, i);
                    v[j].gtu = S(G_TU, i);
                    v[j].gqu = S(G_QU, i);
                    v[j].gad = S(G_AD, i);
                    v[j].gtd = S(G_TD, i);
                    v[j].gqd = S(G_QD, i);
                }
#pragma unroll
                for (int j = 0; j < AB; ++j) {
                    const int i = i0 + j;
                    if (i > iB) break;
                    const double dpa = v[j].pm - v[j].pa, dpb = v[j].pb - v[j].pm;
                    const double gPs = GRAV / (CP * dpa) * v[j].gdta - GRAV / (CP * dpb) * v[j].gdtb;
                    const double gPq = GRAV / dpa * v[j].gdqa - GRAV / dpb * v[j].gdqb;
                    const double et = v[j].et;
                    const bool upw = v[j].upw != 0.0;  // upwind layer i-1, else i
                    const double s_up = upw ? CP * v[j].Ta + GRAV * v[j].za + phis
                                            : CP * v[j].Tb + GRAV * v[j].zb + phis;
                    const double q_up = upw ? v[j].qa : v[j].qb;
                    const double zii = 0.5 * (v[j].za + v[j].zb);
                    const double su = CP * v[j].tu + GRAV * zii + phis, qu = v[j].qu;
                    const bool dn = kd >= 0 && i >= kd + 1;
                    const double ed = dn ? -v[j].ad : 0.0;
                    const double m = et + alpha * ed;
                    S(G_ETA, i) = v[j].geta + (gPs * (su - s_up) + gPq * (qu - q_up));
                    S(G_TU, i) = v[j].gtu + CP * gPs * et;
                    S(G_QU, i) = v[j].gqu + gPq * et;
                    if (upw) {
                        gT[j] += -CP * gPs * m;
                        gq[j] += -gPq * m;
                    } else {
                        gT[j + 1] += -CP * gPs * m;
                        gq[j + 1] += -gPq * m;
                    }
                    if (dn) {
                        const double sd = CP * v[j].td + GRAV * zii + phis, qd = v[j].qd;
                        galpha += gPs * ed * (sd - s_up) + gPq * ed * (qd - q_up);
                        S(G_AD, i) = v[j].gad + -alpha * (gPs * (sd - s_up) + gPq * (qd - q_up));
                        S(G_TD, i) = v[j].gtd + CP * alpha * ed * gPs;
                        S(G_QD, i) = v[j].gqd + alpha * ed * gPq;
                    }
                }
#pragma unroll
                for (int j = 0; j <= AB; ++j) {
                    const int k = i0 - 1 + j;
                    if (k > iB) break;
                    S(aT, k) = gT[j];
                    S(aQ, k) = gq[j];
                }
            }
            x_galpha[role / 2][lane] = galpha;
        }
        if (act && (role == 1 || role == 3) && x_skip[lane] == 0) {
            const int half = role == 1 ? 0 : 1;
            gF = x_gF[lane];
            gcape = x_gcape[lane];
            dT1b = x_dT1b[lane];
            dq1b = x_dq1b[lane];
            // D8 closure F and D4 CAPE through the parcel (D2): the parcel's terms, into hkb, qkb
            // (each wavefront over the layers whose lifts it recomputed).
            for (int k0 = kb - 1 - half; k0 >= kt; k0 -= 2 * AB) {
              struct V {
                  double pt, pb, Tp, qp, sat, Q1, Q2;
              } v[AB];
#pragma unroll
              for (int j = 0; j < AB; ++j) {
                  const int k = max(k0 - 2 * j, kt);
                  v[j].pt = AT(M.pi, k);
                  v[j].pb = AT(M.pi, k + 1);
                  v[j].Tp = S(P_TP, k);
                  v[j].qp = S(P_QP, k);
                  v[j].sat = S(P_SAT, k);
                  v[j].Q1 = S(P_Q1, k);
                  v[j].Q2 = S(P_Q2, k);
              }
#pragma unroll
              for (int j = 0; j < AB; ++j) {
                const int k = k0 - 2 * j;
                if (k < kt) break;
                const double lam = log(v[j].pb / v[j].pt);
                const double ga = -RD * gF * lam * dT1b, gb = -RD * gF * lam * dq1b;
                const double gB = RD * lam * gcape;
                const double Tp = v[j].Tp, qp = v[j].qp;
                double gTp = gB * (1.0 + CVIR * qp), gqp = gB * CVIR * Tp;
                if (v[j].sat != 0.0) {
                    const double Q1 = v[j].Q1, Q2 = v[j].Q2;
                    const double c = (1.0 + CVIR * qp) + CVIR * Tp * Q1;
                    const double den = CP + LV * Q1;
                    const double dc = CVIR * (2.0 * Q1 + Tp * Q2), dden = LV * Q2;
                    const double dq = (dc * den - c * dden) / (den * den);
                    gTp += ga * CP * dq + gb * LV * dq;
                    ghkb += (gTp + gqp * Q1) / den;
                } else {
                    gqp += ga * CVIR;
                    gTp += gb * CVIR;
                    ghkb += gTp / CP;
                    gqkb += -LV * gTp / CP + gqp;
                }
              }
            }
            x_ghkb[half][lane] = ghkb;
            x_gqkb[half][lane] = gqkb;
        }
        __syncthreads();

        // ============================================ phase 4
        // D6 downdraft strength when capped by the evaporation limit: its adjoint goes into the
        // condensation sources (wavefront 0, for the updraft) and the evaporation sources
        // (wavefront 2, for the downdraft).
        const double galpha = x_galpha[0][lane] + x_galpha[1][lane];
        if (act && role == 0 && !skip && capped) {
            const double gC1 = galpha * beta / E1;
            for (int k0 = kt + 1; k0 <= kb; k0 += AB) {
                double g[AB];
#pragma unroll
                for (int j = 0; j < AB; ++j) g[j] = S(G_C, min(k0 + j, kb));
#pragma unroll
                for (int j = 0; j < AB; ++j)
                    if (k0 + j <= kb) S(G_C, k0 + j) = g[j] + gC1;
            }
        } else if (act && role == 2 && x_skip[lane] == 0 && capped) {
            const double gE1 = -galpha * alpha / E1;
            for (int k0 = kd; k0 <= kb - 1; k0 += AB) {
                double g[AB];
#pragma unroll
                for (int j = 0; j < AB; ++j) g[j] = S(G_E1, min(k0 + j, kb - 1));
#pragma unroll
                for (int j = 0; j < AB; ++j)
                    if (k0 + j <= kb - 1) S(G_E1, k0 + j) = g[j] + gE1;
            }
        }
        if (act && role == 0 && !skip) {
            // D5 updraft recurrence, in reverse (top interface first), carrying what an iteration adds
            // to the adjoints of the interface below it (eta, h_u, q_u) in registers.
            double ceta = 0.0, chu = 0.0, cqu = 0.0;  // recurrence parts at interface k
            ghkb = x_ghkb[0][lane] + x_ghkb[1][lane];  // the parcel's part
            gqkb = x_gqkb[0][lane] + x_gqkb[1][lane];
            {
                double eta = S(U_ETA, kt + 1), zk = zi(kt + 1);
                for (int k0 = kt + 1; k0 <= kb - 1; k0 += AB) {
                  struct V {
                      double etan1, hm, hu1, qm, qu, qu1, E, Q1, zlo, gc, geta, gqu, gTu, sat, h, q, gT,
                          gq;
                  } v[AB];
#pragma unroll
                  for (int j = 0; j < AB; ++j) {
                      const int k = min(k0 + j, kb - 1);
                      v[j].etan1 = S(U_ETA, k + 1);
                      v[j].hm = S(U_HM, k);
                      v[j].hu1 = S(U_HM, k + 1);
                      v[j].qm = S(U_QM, k);
                      v[j].qu = S(U_QU, k);
                      v[j].qu1 = S(U_QU, k + 1);
                      v[j].E = S(U_E, k);
                      v[j].Q1 = S(U_Q1, k);
                      v[j].zlo = zi(k + 1);
                      v[j].gc = S(G_C, k);
                      v[j].geta = S(G_ETA, k);
                      v[j].gqu = S(G_QU, k);
                      v[j].gTu = S(G_TU, k);
                      v[j].sat = S(U_SAT, k);
                      v[j].h = hk(k);
                      v[j].q = qk(k);
                      v[j].gT = S(G_T, k);
                      v[j].gq = S(G_Q, k);
                  }
#pragma unroll
                  for (int j = 0; j < AB; ++j) {
                    const int k = k0 + j;
                    if (k > kb - 1) break;
                    const double etan1 = v[j].etan1;
                    const double hm = v[j].hm, hu1 = v[j].hu1;
                    const double qm = v[j].qm, qu = v[j].qu, qu1 = v[j].qu1;
                    const double E = v[j].E, Q1 = v[j].Q1, zlo = v[j].zlo;
                    const double gc = v[j].gc;
                    double geta = v[j].geta + ceta + gc * (qm - qu);
                    double gqm = gc * eta;
                    const double gqu = v[j].gqu + cqu - gc * eta;
                    double ghm = chu;
                    const double gTu = v[j].gTu;
                    if (v[j].sat != 0.0) {
                        ghm += (gTu + gqu * Q1) / (CP + LV * Q1);
                    } else {
                        ghm += gTu / CP;
                        gqm += -LV * gTu / CP + gqu;
                    }
                    const double reta = 1.0 / eta;
                    double geta1 = (ghm * hu1 + gqm * qu1) * reta;
                    chu = ghm * etan1 * reta;
                    cqu = gqm * etan1 * reta;
                    double gE = (ghm * v[j].h + gqm * v[j].q) * reta;
                    const double gh = ghm * E * reta;
                    S(G_T, k) = v[j].gT + CP * gh;
                    S(G_Q, k) = v[j].gq + (LV * gh + gqm * E * reta);
                    geta += -(ghm * hm + gqm * qm) * reta;
                    geta1 += geta;
                    gE += geta;
                    const double dz = zk - zlo;
                    geps += gE * etan1 * dz;
                    geta1 += gE * epsd * dz;
                    ceta = geta1;
                    eta = etan1;
                    zk = zlo;
                  }
                }
            }
            {
                // Launch interface kb: h_u = h_kb, q_m = q_kb, c_kb = q_kb - q_u(kb).
                const double gc = S(G_C, kb);
                const double gqu = S(G_QU, kb) + cqu - gc;
                double ghm = chu;
                const double gTu = S(G_TU, kb), Q1 = S(U_Q1, kb);
                double gqm = 0.0;
                if (S(U_SAT, kb) != 0.0) {
                    ghm += (gTu + gqu * Q1) / (CP + LV * Q1);
                } else {
                    ghm += gTu / CP;
                    gqm = -LV * gTu / CP + gqu;
                }
                ghkb += ghm;
                gqkb += gqm + gc;
            }
            S(G_T, kb) += CP * ghkb;
            S(G_Q, kb) += LV * ghkb + gqkb;

        } else if (act && role == 2 && x_skip[lane] == 0) {
            // D6 downdraft recurrence, in reverse (bottom layer first), into GD_T, GD_Q and its own
            // part of dL/deps.  What an iteration adds to the
            // adjoints of the interface above it (ad, q_d, h_d) is carried in registers to the next
            // iteration, not written back to the scratch.
            if (kd >= 0) {
                double cad = 0.0, cqd = 0.0, chd = 0.0;  // recurrence parts at interface k+1
                double adk1 = S(D_AD, kb), hdk1 = S(D_HD, kb), qdk1 = S(D_QD, kb), zlo = zi(kb);
                for (int k0 = kb - 1; k0 >= kd + 1; k0 -= AB) {
                  struct V {
                      double ad, hd, qd, Ed, Q1, q, h, ge1, zk, gad1, gqd1, gtd1, gT, gq;
                  } v[AB];
#pragma unroll
                  for (int j = 0; j < AB; ++j) {
                      const int k = max(k0 - j, kd + 1);
                      v[j].ad = S(D_AD, k);
                      v[j].hd = S(D_HD, k);
                      v[j].qd = S(D_QD, k);
                      v[j].Ed = S(D_ED, k);
                      v[j].Q1 = S(D_Q1, k + 1);
                      v[j].q = qk(k);
                      v[j].h = hk(k);
                      v[j].ge1 = S(G_E1, k);
                      v[j].zk = zi(k);
                      v[j].gad1 = S(G_AD, k + 1);
                      v[j].gqd1 = S(G_QD, k + 1);
                      v[j].gtd1 = S(G_TD, k + 1);
                      v[j].gT = S(GD_T, k);
                      v[j].gq = S(GD_Q, k);
                  }
#pragma unroll
                  for (int j = 0; j < AB; ++j) {
                    const int k = k0 - j;
                    if (k < kd + 1) break;
                    const double adk = v[j].ad, hdk = v[j].hd, qdk = v[j].qd;
                    const double Ed = v[j].Ed, Q1 = v[j].Q1, q = v[j].q, h = v[j].h;
                    const double ge1 = v[j].ge1, zk = v[j].zk;
                    double gad1 = v[j].gad1 + cad + ge1 * qdk1;
                    const double gqd1 = v[j].gqd1 + cqd + ge1 * adk1;
                    double gad0 = -ge1 * qdk;
                    double gEd = -ge1 * q;
                    const double gq = -ge1 * Ed;
                    const double gTd1 = v[j].gtd1 + gqd1 * Q1;
                    const double ghd1 = chd + gTd1 / (CP + LV * Q1);
                    const double rad1 = 1.0 / adk1;
                    gad0 += ghd1 * hdk * rad1;
                    gEd += ghd1 * h * rad1;
                    const double gh = ghd1 * Ed * rad1;
                    gad1 += -ghd1 * hdk1 * rad1;
                    gad0 += gad1;
                    gEd += gad1;
                    const double dz = zk - zlo;
                    gepsd += gEd * adk * dz;
                    gad0 += gEd * epsd * dz;
                    cad = gad0;
                    cqd = -ge1 * adk;
                    chd = ghd1 * adk * rad1;
                    S(GD_T, k) = v[j].gT + CP * gh;
                    S(GD_Q, k) = v[j].gq + (LV * gh + gq);
                    adk1 = adk;
                    hdk1 = hdk;
                    qdk1 = qdk;
                    zlo = zk;
                  }
                }
                // Start: h_d = h of layer kd at interface kd+1; e1_kd = q_d(kd+1) - q_kd.
                const double ge1 = S(G_E1, kd);
                const double gqd1 = S(G_QD, kd + 1) + cqd + ge1;
                const double Q1 = S(D_Q1, kd + 1);
                const double gTd1 = S(G_TD, kd + 1) + gqd1 * Q1;
                const double ghd1 = chd + gTd1 / (CP + LV * Q1);
                S(GD_T, kd) += CP * ghd1;
                S(GD_Q, kd) += LV * ghd1 - ge1;
            }
            x_geps[lane] = gepsd;
        }
        __syncthreads();

        // ============================================ phase 5: the gradients out (all four)
        if (act && x_skip[lane] == 0) {
            // All levels, a quarter each: the pass-through gradient (if any) plus the scheme's on
            // the plume's levels.  (x may be the output itself: a batch reads all its levels
            // before it writes them.)
            const int len = (L + ADJ_WAVES - 1) / ADJ_WAVES;
            const int k1 = min((role + 1) * len, L);
            for (int k0 = role * len; k0 < k1; k0 += AB) {
                double xt[AB], xq[AB], gt[AB], gq[AB];
#pragma unroll
                for (int j = 0; j < AB; ++j) {
                    const int k = min(k0 + j, k1 - 1);
                    xt[j] = w.xT ? AT(w.xT, k) : 0.0;
                    xq[j] = w.xq ? AT(w.xq, k) : 0.0;
                    gt[j] = S(G_T, k) + S(G2_T, k) + S(GD_T, k);
                    gq[j] = S(G_Q, k) + S(G2_Q, k) + S(GD_Q, k);
                }
#pragma unroll
                for (int j = 0; j < AB; ++j) {
                    const int k = k0 + j;
                    if (k >= k1) break;
                    const bool in = k >= kt && k <= kb;
                    AT(w.gT, k) = xt[j] + (in ? gt[j] : 0.0);
                    AT(w.gq, k) = xq[j] + (in ? gq[j] : 0.0);
                }
            }
            if (role == 0) {
                w.pgrad[col] = gtau;
                w.pgrad[ld + col] = geps + x_geps[lane];
            }
        }
    }

    // The columns without deep convection: their gradients are the pass-through (or zero).  The
    // blocks that hold no chunk of the list write them while the others run their chains (if
    // every block holds one, all blocks do after their chunks); with the pass-through in place
    // there is nothing to write.
    if (w.xT == w.gT && w.xq == w.gq) return;
    const int64_t nchunk = ((int64_t)n + WAVE - 1) / WAVE;
    const int64_t nidle = (int64_t)gridDim.x - nchunk;
    if (nidle > 0 && (int64_t)blockIdx.x < nchunk) return;
    const int64_t fi = nidle > 0 ? (int64_t)blockIdx.x - nchunk : (int64_t)blockIdx.x;
    const int64_t nf = nidle > 0 ? nidle : (int64_t)gridDim.x;
    for (int64_t c0 = fi * (ADJ_WAVES * WAVE); c0 < M.ncol; c0 += nf * (ADJ_WAVES * WAVE)) {
        const int64_t col = c0 + threadIdx.x;
        if (col >= M.ncol || M.dout.status[col] == 0) continue;
        for (int k = 0; k < L; ++k) {
            AT(w.gT, k) = w.xT ? AT(w.xT, k) : 0.0;
            AT(w.gq, k) = w.xq ? AT(w.xq, k) : 0.0;
        }
    }
#undef S
}

// ------------------------------------------------------------------ shallow scheme (S1-S9)
// Per-level scratch of the shallow adjoint (index = level or interface).
enum : int {
    C_TP = 0, C_QP, C_Q1, C_FL,                            // S2-S5 scan levels: parcel, flags
    W_ETA, W_HM, W_QM, W_QTU, W_TP, W_QP, W_Q1, W_FL,      // plume interfaces kt+1 .. ks
    W_DT1, W_DQ1, W_GDT1, W_GDQ1,                          // unit tendencies and their adjoints
    W_GT, W_GQ,                                            // dL/dT, dL/dq accumulators
    N_SADJ
};
constexpr int FL_SAT = 1;   // the parcel is saturated
constexpr int FL_AUX = 2;   // scan level: counted in CIN (B < 0); plume interface: rains out

struct SAdjWork {
    int *cnt;
    int *list;
    double *pgrad;  // [2][ld]: per-column dL/deps_sh, dL/ddelta_sh
    double *scr;
    int64_t stride;
    int lmax;
    const double *cT, *cq, *cP;  // cotangents of the shallow dTdt, dqdt, prec (may be NULL)
    double *gT, *gq;             // dL/dT, dL/dq of the state the scheme saw [nlev][ld]
    int upd;                     // the scheme saw T + dt*dTdt, q + dt*dqdt of M.dout (step)
};

// Shallow-active (status 0) columns into a list, and zero parameter-gradient rows; the other
// columns' gradients are written by k_shallow_adjoint's blocks that hold no list entries.
__global__ __launch_bounds__(BLOCK) void k_sadj_compact(Member M, SAdjWork w) {
    const int64_t col = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool live = col < M.ncol;
    const int64_t ld = M.ld;
    const bool act = live && M.sout.status[col] == 0;
    if (live) {
        w.pgrad[col] = 0.0;
        w.pgrad[ld + col] = 0.0;
    }
    const int slot = wave_append(act, &w.cnt[1]);
    if (slot >= 0) w.list[slot] = (int)col;
}

// Adjoint of the parcel lift (C1) at a stored solution: with H the parcel's energy and qt its
// water, a saturated parcel has cp T + Lv qs(T) = H (dT/dH = 1/(cp + Lv qs')), q_v = qs(T); an
// unsaturated one T = (H - Lv qt)/cp, q_v = qt.  Adds to gH and gqt.
__device__ __forceinline__ void lift_adjoint(bool sat, double Q1, double gTp, double gqv, double &gH,
                                             double &gqt) {
    if (sat) {
        gH += (gTp + gqv * Q1) / (CP + LV * Q1);
    } else {
        gH += gTp * RCP_CP;
        gqt += -LV * RCP_CP * gTp + gqv;
    }
}

// Persistent over the shallow list.  Per column: recompute S1-S9 from the (possibly updated)
// state with the forward run's source layer and plume top, storing what the reverse sweep needs;
// then the reverse sweep: base flux (closure M_c or the humidity limiter) -> flux-form tendencies
// -> plume recurrence (top interface first) -> the source's parcel -> M_c through rho_s and CIN ->
// the source means.  The vertical-velocity equation only decides the plume top, which is held
// fixed, so it carries no derivative.
__global__ __launch_bounds__(WAVE) void k_shallow_adjoint(Member M, SAdjWork w) {
    const int n = w.cnt[1];
    const int64_t gtid = (int64_t)blockIdx.x * WAVE + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * WAVE;
    const int L = M.nlev;
    const int64_t ld = M.ld;
    const conv_params_t &P = M.P;
    const double dt = M.dt;
    double *scr = w.scr;
#define S(arr, lev) scr[((int64_t)(arr) * (w.lmax + 1) + (lev)) * w.stride + gtid]

    for (int64_t slot = gtid; slot < n; slot += nthreads) {
        const int64_t col = w.list[slot];
        const int ks = M.sout.kbase[col], kt = M.sout.ktop[col];
        const double phis = M.phis[col], tke = M.tke[col];
        auto Tk = [&](int k) { return w.upd ? AT(M.T, k) + dt * AT(M.dout.dTdt, k) : AT(M.T, k); };
        auto qk = [&](int k) { return w.upd ? AT(M.q, k) + dt * AT(M.dout.dqdt, k) : AT(M.q, k); };
        auto sk = [&](int k) { return CP * Tk(k) + GRAV * AT(M.z, k) + phis; };
        auto hk = [&](int k) { return (CP * Tk(k) + GRAV * AT(M.z, k) + phis) + LV * qk(k); };
        auto zi = [&](int i) { return 0.5 * (AT(M.z, i - 1) + AT(M.z, i)); };
        auto dpk = [&](int k) { return AT(M.pi, k + 1) - AT(M.pi, k); };
        auto zero_column = [&]() {
            for (int k = 0; k < L; ++k) {
                AT(w.gT, k) = 0.0;
                AT(w.gq, k) = 0.0;
            }
            w.pgrad[col] = 0.0;
            w.pgrad[ld + col] = 0.0;
        };
        if (ks < 1 || kt < 0 || kt >= ks - 1) {  // not a status-0 column of this state
            zero_column();
            continue;
        }

        // ============================================ forward recomputation
        // S1: pressure-weighted means over the source layers, summed bottom-up.
        double hsum = 0.0, qsum = 0.0, wsum = 0.0;
        for (int k = L - 1; k >= ks; --k) {
            const double dp = dpk(k);
            hsum += dp * hk(k);
            qsum += dp * qk(k);
            wsum += dp;
        }
        const double hs = hsum / wsum, qsrc = qsum / wsum;
        // S2-S5: the undilute scan up to the level of free convection, and CIN.
        double cin = 0.0;
        int klcl = -1, klfc = -1;
        {
            Hint hint;
            hint.clear();
            for (int k = ks - 1; k >= 0; --k) {
                const double pm = AT(M.pm, k);
                if ((klcl < 0 && pm < P.p_lcl_min) || (klcl >= 0 && pm < P.p_sh_top_min)) break;
                const Lifted r = lift(hs - GRAV * AT(M.z, k) - phis, qsrc, pm, hint);
                const double B = tv(r.T, r.qv) - tv(Tk(k), qk(k));
                if (klcl < 0 && r.sat) klcl = k;
                S(C_TP, k) = r.T;
                S(C_QP, k) = r.qv;
                S(C_Q1, k) = r.sat ? sat_eval(r.T, pm).dqs : 0.0;
                int fl = r.sat ? FL_SAT : 0;
                if (klcl >= 0 && B > 0.0 && pm >= P.p_sh_top_min) {
                    S(C_FL, k) = fl;
                    klfc = k;
                    break;
                }
                if (B < 0.0) {
                    cin += RD * (-B) * log(AT(M.pi, k + 1) / AT(M.pi, k));
                    fl |= FL_AUX;
                }
                S(C_FL, k) = fl;
            }
        }
        if (klfc < 0) {  // not reachable for a status-0 column
            zero_column();
            continue;
        }
        // S6: closure.
        const double sigw2 = P.c_tke * tke, sigw = sqrt(sigw2);
        const double tvs = tv(Tk(ks), qk(ks));
        const double rho_s = AT(M.pi, ks) / (RD * tvs);
        const double Mclos = rho_s * sigw / SQRT_2PI * exp(-P.a_buoy * cin / sigw2);
        // S7-S8: plume from interface ks up to kt+1, and the unit tendencies of layers ks .. kt.
        double Mlim = __builtin_inf(), P1;
        int klim = -1;
        {
            Hint hp;
            hp.clear();
            double eta = 1.0, hu = hs, qtu, Fs_lo, Fq_lo;
            double zlo = zi(ks);
            {
                const Lifted r = lift(hs - GRAV * zlo - phis, qsrc, AT(M.pi, ks), hp);
                const double ql = qsrc - r.qv;
                const bool rain = ql - P.qlcrit_sh > 0.0;
                const double rr = rain ? ql - P.qlcrit_sh : 0.0;
                qtu = qsrc - rr;
                const double slu = CP * r.T + GRAV * zlo + phis - LV * (ql - rr);
                const double Fs = slu - sk(ks - 1), Fq = qtu - qk(ks - 1);
                const double dp = dpk(ks);
                const double dT1 = (0.0 - Fs + LV * rr) * GRAV / (CP * dp);
                const double dq1 = (0.0 - Fq - rr) * GRAV / dp;
                S(W_ETA, ks) = 1.0;
                S(W_HM, ks) = hs;
                S(W_QM, ks) = qsrc;
                S(W_QTU, ks) = qtu;
                S(W_TP, ks) = r.T;
                S(W_QP, ks) = r.qv;
                S(W_Q1, ks) = r.sat ? sat_eval(r.T, AT(M.pi, ks)).dqs : 0.0;
                S(W_FL, ks) = (r.sat ? FL_SAT : 0) | (rain ? FL_AUX : 0);
                S(W_DT1, ks) = dT1;
                S(W_DQ1, ks) = dq1;
                P1 = rr;
                if (dq1 < 0.0) {
                    const double m = qk(ks) / (-dt * dq1);
                    if (m < Mlim) {
                        Mlim = m;
                        klim = ks;
                    }
                }
                Fs_lo = Fs;
                Fq_lo = Fq;
            }
            for (int k = ks - 1; k >= kt + 1; --k) {
                const double zk = zi(k);
                const double dz = zk - zlo;
                const double E = P.eps_sh * eta * dz, D = P.delta_sh * eta * dz;
                const double en = eta + E - D;
                const double Tkk = Tk(k), qkk = qk(k);
                const double hm =
                    ((eta - D) * hu + E * ((CP * Tkk + GRAV * AT(M.z, k) + phis) + LV * qkk)) / en;
                const double qm = ((eta - D) * qtu + E * qkk) / en;
                const Lifted r = lift(hm - GRAV * zk - phis, qm, AT(M.pi, k), hp);
                const double ql = qm - r.qv;
                const bool rain = ql - P.qlcrit_sh > 0.0;
                const double rr = rain ? ql - P.qlcrit_sh : 0.0;
                const double qtn = qm - rr;
                const double slu = CP * r.T + GRAV * zk + phis - LV * (ql - rr);
                const double Fs = en * (slu - sk(k - 1)), Fq = en * (qtn - qk(k - 1));
                const double pr = en * rr;
                const double dp = dpk(k);
                const double dT1 = (Fs_lo - Fs + LV * pr) * GRAV / (CP * dp);
                const double dq1 = (Fq_lo - Fq - pr) * GRAV / dp;
                S(W_ETA, k) = en;
                S(W_HM, k) = hm;
                S(W_QM, k) = qm;
                S(W_QTU, k) = qtn;
                S(W_TP, k) = r.T;
                S(W_QP, k) = r.qv;
                S(W_Q1, k) = r.sat ? sat_eval(r.T, AT(M.pi, k)).dqs : 0.0;
                S(W_FL, k) = (r.sat ? FL_SAT : 0) | (rain ? FL_AUX : 0);
                S(W_DT1, k) = dT1;
                S(W_DQ1, k) = dq1;
                P1 += pr;
                if (dq1 < 0.0) {
                    const double m = qkk / (-dt * dq1);
                    if (m < Mlim) {
                        Mlim = m;
                        klim = k;
                    }
                }
                eta = en;
                hu = hm;
                qtu = qtn;
                zlo = zk;
                Fs_lo = Fs;
                Fq_lo = Fq;
            }
            // The top layer kt: only the flux through its bottom interface.
            const double dp = dpk(kt);
            const double dT1 = Fs_lo * GRAV / (CP * dp);
            const double dq1 = Fq_lo * GRAV / dp;
            S(W_DT1, kt) = dT1;
            S(W_DQ1, kt) = dq1;
            if (dq1 < 0.0) {
                const double m = qk(kt) / (-dt * dq1);
                if (m < Mlim) {
                    Mlim = m;
                    klim = kt;
                }
            }
        }
        const bool closure = Mclos <= Mlim || klim < 0;  // (klim < 0 only if M_c is not finite)
        const double Mb = closure ? Mclos : Mlim;
        // Highest level with a derivative: the plume top, or a CIN level above it when the
        // entraining plume stops below the level of free convection.
        const int kmin = min(kt, klfc + 1);

        // ============================================ reverse sweep
        for (int lev = kmin; lev < L; ++lev) {
            S(W_GT, lev) = 0.0;
            S(W_GQ, lev) = 0.0;
        }
        // S9 outputs = M_b * unit profiles (AB levels loaded at a time, as in the deep adjoint).
        double gMb = 0.0;
        for (int k0 = kt; k0 <= ks; k0 += AB) {
            double cT[AB], cq[AB], d1[AB], q1[AB];
#pragma unroll
            for (int j = 0; j < AB; ++j) {
                const int k = min(k0 + j, ks);
                cT[j] = w.cT ? AT(w.cT, k) : 0.0;
                cq[j] = w.cq ? AT(w.cq, k) : 0.0;
                d1[j] = S(W_DT1, k);
                q1[j] = S(W_DQ1, k);
            }
#pragma unroll
            for (int j = 0; j < AB; ++j) {
                const int k = k0 + j;
                if (k > ks) break;
                gMb += cT[j] * d1[j] + cq[j] * q1[j];
                S(W_GDT1, k) = cT[j] * Mb;
                S(W_GDQ1, k) = cq[j] * Mb;
            }
        }
        const double cPc = w.cP ? w.cP[col] : 0.0;
        gMb += cPc * P1;
        const double gP1 = cPc * Mb;
        double gMclos = 0.0;
        if (closure) {
            gMclos = gMb;
        } else {
            const double dq1m = S(W_DQ1, klim);
            S(W_GQ, klim) += gMb / (-dt * dq1m);
            S(W_GDQ1, klim) += gMb * (-Mlim / dq1m);
        }
        // S8 and S7 in reverse, top interface first.  (ceta, chu, cqtu): what the step at
        // interface k adds to the adjoints of the plume state at interface k+1.
        double ceta = 0.0, chu = 0.0, cqtu = 0.0, geps = 0.0, gdel = 0.0, ghs = 0.0, gqs = 0.0;
        for (int k = kt + 1; k <= ks; ++k) {
            const double dpa = dpk(k - 1), dpb = dpk(k);
            // Flux at interface k: the top of layer k, the bottom of layer k-1.
            const double gFs = GRAV / (CP * dpa) * S(W_GDT1, k - 1) - GRAV / (CP * dpb) * S(W_GDT1, k);
            const double gFq = GRAV / dpa * S(W_GDQ1, k - 1) - GRAV / dpb * S(W_GDQ1, k);
            const double gpr = LV * GRAV / (CP * dpb) * S(W_GDT1, k) - GRAV / dpb * S(W_GDQ1, k) + gP1;
            const double en = S(W_ETA, k), hm = S(W_HM, k), qm = S(W_QM, k), qtuk = S(W_QTU, k);
            const double Tp = S(W_TP, k), qvp = S(W_QP, k), Q1 = S(W_Q1, k);
            const int fl = (int)S(W_FL, k);
            const double ql = qm - qvp;
            const double rr = (fl & FL_AUX) ? ql - P.qlcrit_sh : 0.0;
            const double zk = zi(k);
            const double slu = CP * Tp + GRAV * zk + phis - LV * (ql - rr);
            const double s_up = sk(k - 1), q_up = qk(k - 1);
            double gen = gFs * (slu - s_up) + gFq * (qtuk - q_up) + ceta;
            const double gslu = gFs * en;
            const double gqtu = gFq * en + cqtu;
            S(W_GT, k - 1) -= CP * gFs * en;
            S(W_GQ, k - 1) -= gFq * en;
            gen += rr * gpr;
            double grr = en * gpr + LV * gslu - gqtu;
            const double gTp = CP * gslu;
            double gql = -LV * gslu;
            double gqm = gqtu;
            if (fl & FL_AUX) gql += grr;
            gqm += gql;
            const double gqv = -gql;
            double gH = 0.0;
            lift_adjoint((fl & FL_SAT) != 0, Q1, gTp, gqv, gH, gqm);
            const double ghm = gH + chu;
            if (k == ks) {  // the source interface: h_u = hs, q_m = q_src, eta = 1
                ghs += ghm;
                gqs += gqm;
                break;
            }
            // The recurrence step from interface k+1 to k.
            const double eta1 = S(W_ETA, k + 1), hu1 = S(W_HM, k + 1), qtu1 = S(W_QTU, k + 1);
            const double dz = zk - zi(k + 1);
            const double E = P.eps_sh * eta1 * dz, D = P.delta_sh * eta1 * dz;
            const double a = eta1 - D;
            const double ren = 1.0 / en;
            const double ga = (ghm * hu1 + gqm * qtu1) * ren;
            chu = ghm * a * ren;
            cqtu = gqm * a * ren;
            double gE = (ghm * hk(k) + gqm * qk(k)) * ren;
            const double gh = ghm * E * ren;
            S(W_GT, k) += CP * gh;
            S(W_GQ, k) += LV * gh + gqm * E * ren;
            gen -= (ghm * hm + gqm * qm) * ren;
            double geta1 = gen + ga;
            gE += gen;
            const double gD = -gen - ga;
            geta1 += gE * P.eps_sh * dz + gD * P.delta_sh * dz;
            geps += gE * eta1 * dz;
            gdel += gD * eta1 * dz;
            ceta = geta1;
        }
        // S6: M_c = rho_s sigma_w / sqrt(2 pi) exp(-a CIN / sigma_w^2).
        const double gcin = -gMclos * Mclos * P.a_buoy / sigw2;
        {
            const double grho = gMclos * Mclos / rho_s;
            const double gtv = -grho * rho_s / tvs;
            S(W_GT, ks) += gtv * (1.0 + CVIR * qk(ks));
            S(W_GQ, ks) += gtv * CVIR * Tk(ks);
        }
        // S5: CIN over the scan levels with negative buoyancy.
        for (int k = ks - 1; k > klfc; --k) {
            const int fl = (int)S(C_FL, k);
            if (!(fl & FL_AUX)) continue;
            const double gB = -RD * log(AT(M.pi, k + 1) / AT(M.pi, k)) * gcin;
            const double Tp = S(C_TP, k), qvp = S(C_QP, k);
            S(W_GT, k) -= gB * (1.0 + CVIR * qk(k));
            S(W_GQ, k) -= gB * CVIR * Tk(k);
            lift_adjoint((fl & FL_SAT) != 0, S(C_Q1, k), gB * (1.0 + CVIR * qvp), gB * CVIR * Tp,
                         ghs, gqs);
        }
        // S1: the source means.
        for (int k0 = ks; k0 < L; k0 += AB) {
            double pt[AB], pb[AB], gt[AB], gq[AB];
#pragma unroll
            for (int j = 0; j < AB; ++j) {
                const int k = min(k0 + j, L - 1);
                pt[j] = AT(M.pi, k);
                pb[j] = AT(M.pi, k + 1);
                gt[j] = S(W_GT, k);
                gq[j] = S(W_GQ, k);
            }
#pragma unroll
            for (int j = 0; j < AB; ++j) {
                const int k = k0 + j;
                if (k >= L) break;
                const double f = (pb[j] - pt[j]) / wsum;
                S(W_GT, k) = gt[j] + CP * ghs * f;
                S(W_GQ, k) = gq[j] + (LV * ghs + gqs) * f;
            }
        }
        for (int k0 = 0; k0 < L; k0 += AB) {
            double gt[AB], gq[AB];
#pragma unroll
            for (int j = 0; j < AB; ++j) {
                const int k = min(k0 + j, L - 1);
                gt[j] = S(W_GT, k);
                gq[j] = S(W_GQ, k);
            }
#pragma unroll
            for (int j = 0; j < AB; ++j) {
                const int k = k0 + j;
                if (k >= L) break;
                const bool in = k >= kmin;
                AT(w.gT, k) = in ? gt[j] : 0.0;
                AT(w.gq, k) = in ? gq[j] : 0.0;
            }
        }
        w.pgrad[col] = geps;
        w.pgrad[ld + col] = gdel;
    }

    // The columns without shallow convection get zero gradients, written by the blocks that hold
    // no list entries while the others run their chains (if every block holds some, by all of
    // them after their entries), as in k_deep_adjoint.
    const int64_t nchunk = ((int64_t)n + WAVE - 1) / WAVE;
    const int64_t nidle = (int64_t)gridDim.x - nchunk;
    if (nidle > 0 && (int64_t)blockIdx.x < nchunk) return;
    const int64_t fi = nidle > 0 ? (int64_t)blockIdx.x - nchunk : (int64_t)blockIdx.x;
    const int64_t nf = nidle > 0 ? nidle : (int64_t)gridDim.x;
    for (int64_t c0 = fi * WAVE; c0 < M.ncol; c0 += nf * WAVE) {
        const int64_t col = c0 + threadIdx.x;
        if (col >= M.ncol || M.sout.status[col] == 0) continue;
        for (int k = 0; k < L; ++k) {
            AT(w.gT, k) = 0.0;
            AT(w.gq, k) = 0.0;
        }
    }
#undef S
}

// dL/dtau and dL/deps: sums of the per-column values over columns 0..ncol-1 in a fixed order, so
// the result is reproducible bit for bit.  Stage 1: block b sums the b-th of NPART contiguous
// column ranges (each thread a strided subset in order, then a fixed-shape tree); stage 2 sums the
// NPART partials with the same tree.  (One kernel whose last block does stage 2 was no faster: its
// device-scope fence writes back the L2 full of the gradients just stored.)
constexpr int NPART = BLOCK;

__device__ void block_tree_sum(double a, double b, double *out0, double *out1) {
    __shared__ double s0[BLOCK], s1[BLOCK];
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out0 = s0[0];
        *out1 = s1[0];
    }
}

__global__ __launch_bounds__(BLOCK) void k_adj_partial(const double *pgrad, int64_t ld, int64_t ncol,
                                                       double *part) {
    const int64_t chunk = (ncol + NPART - 1) / NPART;
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = c0 + chunk < ncol ? c0 + chunk : ncol;
    double a = 0.0, b = 0.0;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += BLOCK) {
        a += pgrad[c];
        b += pgrad[ld + c];
    }
    block_tree_sum(a, b, &part[blockIdx.x], &part[NPART + blockIdx.x]);
}

__global__ __launch_bounds__(BLOCK) void k_adj_final(const double *part, double *out) {
    block_tree_sum(part[threadIdx.x], part[NPART + threadIdx.x], &out[0], &out[1]);
}

__global__ void k_adj_zero2(double *out) {
    if (threadIdx.x < 2) out[threadIdx.x] = 0.0;
}

struct AdjLayout {
    size_t cnt, part, list, slist, pgrad, scr, total;
    int64_t threads;
};
constexpr int NPGRAD = 4;  // per-column parameter-gradient rows: tau, eps_deep, eps_sh, delta_sh

AdjLayout adj_layout(int64_t ncol, int nlev, int cus) {
    AdjLayout l{};
    const int64_t n = ncol > 0 ? ncol : 1;
    const int64_t tiles = (n + BLOCK - 1) / BLOCK;
    const int64_t cap = (int64_t)cus;  // one persistent block per compute unit
    l.threads = (tiles < cap ? tiles : cap) * BLOCK;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~size_t(255);
        return o;
    };
    l.cnt = take(NCOUNTERS * sizeof(int));
    l.part = take(2 * NPART * sizeof(double));
    l.list = take(n * sizeof(int));
    l.slist = take(n * sizeof(int));
    l.pgrad = 0;  // per-column values live in a [NPGRAD][ld] region sized at call time
    const int nscr = N_ADJ > N_SADJ ? N_ADJ : N_SADJ;  // the two adjoints run one after the other
    l.scr = take((size_t)nscr * (nlev + 1) * l.threads * sizeof(double));
    l.total = off;
    return l;
}

__global__ void k_adj_reset(int *cnt) {
    if (threadIdx.x < NCOUNTERS) cnt[threadIdx.x] = 0;
}

}  // namespace

namespace {

bool backward_state_ok(const conv_ctx_t *ctx, const conv_state_t *s, bool shallow) {
    if (ctx->ncol == 0) return true;  // nothing is read: the arrays may be NULL
    if (!s->T || !s->q || !s->p_mid || !s->z || !s->p_int || !s->phis || s->ld < ctx->ncol ||
        !(s->dt > 0.0))
        return false;
    return !shallow || (s->pblh && s->tke);
}

// Sums rows r and r+1 of the per-column parameter gradients into out[0], out[1] (fixed order).
void param_sums(const double *pgrad, int64_t ld, int64_t ncol, double *part, double *out,
                hipStream_t st) {
    hipLaunchKernelGGL(k_adj_partial, dim3(NPART), dim3(BLOCK), 0, st, pgrad, ld, ncol, part);
    hipLaunchKernelGGL(k_adj_final, dim3(1), dim3(BLOCK), 0, st, (const double *)part, out);
}

AdjWork deep_work(char *b, const AdjLayout &l, const conv_ctx_t *ctx, const conv_deep_cot_t *cot,
                  double *gT, double *gq, double *pgrad) {
    AdjWork w;
    w.cnt = (int *)(b + l.cnt);
    w.list = (int *)(b + l.list);
    w.scr = (double *)(b + l.scr);
    w.pgrad = pgrad;
    w.stride = l.threads;
    w.lmax = ctx->nlev;
    w.cT = cot ? cot->g_dTdt : nullptr;
    w.cq = cot ? cot->g_dqdt : nullptr;
    w.cP = cot ? cot->g_prec : nullptr;
    w.gT = gT;
    w.gq = gq;
    w.xT = nullptr;
    w.xq = nullptr;
    return w;
}

SAdjWork shallow_work(char *b, const AdjLayout &l, const conv_ctx_t *ctx,
                      const conv_shallow_cot_t *cot, double *gT, double *gq, double *pgrad,
                      int upd) {
    SAdjWork w;
    w.cnt = (int *)(b + l.cnt);
    w.list = (int *)(b + l.slist);
    w.scr = (double *)(b + l.scr);
    w.pgrad = pgrad;
    w.stride = l.threads;
    w.lmax = ctx->nlev;
    w.cT = cot ? cot->g_dTdt : nullptr;
    w.cq = cot ? cot->g_dqdt : nullptr;
    w.cP = cot ? cot->g_prec : nullptr;
    w.gT = gT;
    w.gq = gq;
    w.upd = upd;
    return w;
}

}  // namespace

extern "C" {

size_t conv_backward_workspace_bytes(int64_t ncol, int32_t nlev, int64_t ld) {
    if (ncol < 0 || ncol > INT32_MAX || nlev < 2 || nlev > 256 || ld < ncol) return 0;
    const AdjLayout l = adj_layout(ncol, nlev, device_cus());
    return l.total + (size_t)NPGRAD * (ld > 0 ? ld : 1) * sizeof(double) + 256;
}

int conv_deep_backward(conv_ctx_t *ctx, const conv_state_t *state, const conv_deep_out_t *fwd,
                       const conv_deep_cot_t *cot, conv_deep_grad_t *grad, void *workspace,
                       size_t ws_bytes, void *stream) {
    if (!ctx || !state || !fwd || !cot || !grad || !workspace) return CONV_EINVAL;
    if (!backward_state_ok(ctx, state, false)) return CONV_EINVAL;
    if (!grad->g_params ||
        (ctx->ncol > 0 && (!fwd->status || !fwd->klaunch || !fwd->ktop || !grad->g_T || !grad->g_q)))
        return CONV_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return CONV_EINVAL;
    if (ctx->P.eps_cape != 0.0) return CONV_EUNSUPPORTED;  // the adjoint is of the undilute parcel
    const AdjLayout l = adj_layout(ctx->ncol, ctx->nlev, ctx->cus);
    const int64_t ld = state->ld;
    if (ws_bytes < l.total + (size_t)2 * ld * sizeof(double)) return CONV_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (ctx->ncol == 0) {
        hipLaunchKernelGGL(k_adj_zero2, dim3(1), dim3(64), 0, st, grad->g_params);
        return check_launch();
    }
    char *b = (char *)workspace;
    const Member M = make_member(ctx->ncol, ctx->nlev, ctx->P, state, fwd, nullptr, 0);
    const AdjWork w = deep_work(b, l, ctx, cot, grad->g_T, grad->g_q, (double *)(b + l.total));
    const unsigned gcols = (unsigned)((ctx->ncol + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_adj_reset, dim3(1), dim3(NCOUNTERS), 0, st, w.cnt);
    hipLaunchKernelGGL(k_adj_compact, dim3(gcols), dim3(BLOCK), 0, st, M, w);
    hipLaunchKernelGGL(k_deep_adjoint, dim3((unsigned)(l.threads / WAVE)), dim3(ADJ_WAVES * WAVE), 0,
                       st, M, w);
    param_sums(w.pgrad, ld, ctx->ncol, (double *)(b + l.part), grad->g_params, st);
    return check_launch();
}

int conv_shallow_backward(conv_ctx_t *ctx, const conv_state_t *state,
                          const conv_shallow_out_t *fwd, const conv_shallow_cot_t *cot,
                          conv_shallow_grad_t *grad, void *workspace, size_t ws_bytes,
                          void *stream) {
    if (!ctx || !state || !fwd || !cot || !grad || !workspace) return CONV_EINVAL;
    if (!backward_state_ok(ctx, state, true)) return CONV_EINVAL;
    if (!grad->g_params ||
        (ctx->ncol > 0 && (!fwd->status || !fwd->kbase || !fwd->ktop || !grad->g_T || !grad->g_q)))
        return CONV_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return CONV_EINVAL;
    const AdjLayout l = adj_layout(ctx->ncol, ctx->nlev, ctx->cus);
    const int64_t ld = state->ld;
    if (ws_bytes < l.total + (size_t)2 * ld * sizeof(double)) return CONV_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (ctx->ncol == 0) {
        hipLaunchKernelGGL(k_adj_zero2, dim3(1), dim3(64), 0, st, grad->g_params);
        return check_launch();
    }
    char *b = (char *)workspace;
    const Member M = make_member(ctx->ncol, ctx->nlev, ctx->P, state, nullptr, fwd, 0);
    const SAdjWork w =
        shallow_work(b, l, ctx, cot, grad->g_T, grad->g_q, (double *)(b + l.total), 0);
    const unsigned gcols = (unsigned)((ctx->ncol + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_adj_reset, dim3(1), dim3(NCOUNTERS), 0, st, w.cnt);
    hipLaunchKernelGGL(k_sadj_compact, dim3(gcols), dim3(BLOCK), 0, st, M, w);
    hipLaunchKernelGGL(k_shallow_adjoint, dim3((unsigned)(l.threads / WAVE)), dim3(WAVE), 0, st,
                       M, w);
    param_sums(w.pgrad, ld, ctx->ncol, (double *)(b + l.part), grad->g_params, st);
    return check_launch();
}

int conv_step_backward(conv_ctx_t *ctx, const conv_state_t *state, const conv_deep_out_t *dfwd,
                       const conv_shallow_out_t *sfwd, const conv_deep_cot_t *dcot,
                       const conv_shallow_cot_t *scot, conv_step_grad_t *grad, void *workspace,
                       size_t ws_bytes, void *stream) {
    if (!ctx || !state || !dfwd || !sfwd || !grad || !workspace) return CONV_EINVAL;
    if (!backward_state_ok(ctx, state, true)) return CONV_EINVAL;
    if (!grad->g_params ||
        (ctx->ncol > 0 && (!dfwd->status || !dfwd->klaunch || !dfwd->ktop || !dfwd->dTdt ||
                           !dfwd->dqdt || !sfwd->status || !sfwd->kbase || !sfwd->ktop ||
                           !grad->g_T || !grad->g_q)))
        return CONV_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return CONV_EINVAL;
    if (ctx->P.eps_cape != 0.0) return CONV_EUNSUPPORTED;  // the deep adjoint is undilute
    const AdjLayout l = adj_layout(ctx->ncol, ctx->nlev, ctx->cus);
    const int64_t ld = state->ld;
    if (ws_bytes < l.total + (size_t)NPGRAD * ld * sizeof(double)) return CONV_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    if (ctx->ncol == 0) {
        hipLaunchKernelGGL(k_adj_zero2, dim3(1), dim3(64), 0, st, grad->g_params);
        hipLaunchKernelGGL(k_adj_zero2, dim3(1), dim3(64), 0, st, grad->g_params + 2);
        return check_launch();
    }
    char *b = (char *)workspace;
    double *pgrad = (double *)(b + l.total);
    const Member M = make_member(ctx->ncol, ctx->nlev, ctx->P, state, dfwd, sfwd, 0);
    const unsigned gcols = (unsigned)((ctx->ncol + BLOCK - 1) / BLOCK);
    const unsigned gpers = (unsigned)(l.threads / WAVE);  // one wavefront per block
    // Shallow adjoint at the updated state: dL/dT', dL/dq' into g_T, g_q.
    const SAdjWork sw = shallow_work(b, l, ctx, scot, grad->g_T, grad->g_q, pgrad + 2 * ld, 1);
    hipLaunchKernelGGL(k_adj_reset, dim3(1), dim3(NCOUNTERS), 0, st, sw.cnt);
    hipLaunchKernelGGL(k_sadj_compact, dim3(gcols), dim3(BLOCK), 0, st, M, sw);
    hipLaunchKernelGGL(k_shallow_adjoint, dim3(gpers), dim3(WAVE), 0, st, M, sw);
    // Deep adjoint with the update's chain rule, in place on g_T, g_q.
    AdjWork dw = deep_work(b, l, ctx, dcot, grad->g_T, grad->g_q, pgrad);
    dw.xT = grad->g_T;
    dw.xq = grad->g_q;
    hipLaunchKernelGGL(k_adj_compact, dim3(gcols), dim3(BLOCK), 0, st, M, dw);
    hipLaunchKernelGGL(k_deep_adjoint, dim3(gpers), dim3(ADJ_WAVES * WAVE), 0, st, M, dw);
    double *part = (double *)(b + l.part);
    param_sums(pgrad, ld, ctx->ncol, part, grad->g_params, st);
    param_sums(pgrad + 2 * ld, ld, ctx->ncol, part, grad->g_params + 2, st);
    return check_launch();
}

}  // extern "C"
