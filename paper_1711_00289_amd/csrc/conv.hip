// conv.hip -- gfx950 kernels and the C ABI (include/conv.h) of the FP64 deep + shallow convection
// library.
//
// Pipeline of one step (the paper's Algorithm 1 order: deep, then shallow on the updated state):
//   k_reset         zero the on-device list counters (a fill kernel, so the step stays capturable)
//   k_trigger       one lane per column over all columns, one bottom-up sweep: validity, moist
//                   static energy, launch layer (D1), the undilute parcel with CAPE and the closure's
//                   parcel sensitivities (D2-D4), and the shallow source and parcel (S1-S6).  Columns
//                   that do not convect get their exact-zero outputs here; columns that do are
//                   compacted into on-device lists by wavefront ballot + popcount + one atomic per
//                   wavefront, so the imbalance between convecting and quiet columns (the paper's
//                   Methodology, "Load Balancing Convections") is removed by compaction rather than by
//                   scheduling.
//   k_deep_plume    persistent over the deep list: updraft (D5), downdraft (D6), flux-form unit
//                   tendencies (D7), closure (D8), limiter (D9), outputs (D10); in a full step also the
//                   shallow trigger on the deep-updated state.
//   k_shallow_plume persistent over the shallow list: plume, tendencies, limiter (S7-S9).
// Per-level plume profiles live in a per-thread scratch region of the caller's workspace laid out
// [array][level][thread], so a wavefront's accesses to one level are contiguous.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include "conv.h"
#include "conv_physics.hpp"

using namespace cvk;

namespace {

constexpr int BLOCK = 256;
constexpr int WAVE = 64;
constexpr int PLUME_BLOCKS_PER_CU = 4;
constexpr int NCOUNTERS = 64;
constexpr int DEEP_SCR = 8;     // su, qu, c->dT1, sd, qd, e1->dq1, eta_d, eta
constexpr int SHALLOW_SCR = 3;  // eta, dT1, dq1

struct Work {
    int *cnt;  // [0] deep list length, [1] shallow list length
    int *dlist, *dkb, *dkt;
    double *dcape, *dSA, *dSB;
    int *slist, *sks, *sflag;
    double *shs, *sqs, *scin, *sMc, *ssig2;
    double *dscr, *sscr;
    int64_t scr_stride;  // threads of the persistent grid
};

struct Args {
    const double *T, *q, *pm, *pi, *z, *phis, *pblh, *tke;
    int64_t ld;
    double dt;
    int64_t ncol;
    int nlev;
    conv_params_t P;
    conv_deep_out_t dout;
    conv_shallow_out_t sout;
    Work w;
};

#define AT(arr, k) (arr)[(int64_t)(k) * ld + col]

// ------------------------------------------------------------------ wavefront compaction
// Appends the lanes with `pred` set to the list counted by *counter: one ballot, one popcount and
// one atomicAdd per wavefront.  Must be reached by every lane of the wavefront.
__device__ __forceinline__ int wave_append(bool pred, int *counter) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, leader);
    return pred ? base + (int)__popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// ------------------------------------------------------------------ shallow trigger (S1-S6)
struct ShallowTrigger {
    int ks, klcl, klfc;
    bool inpbl, act;
    double hsum, qsum, wsum, hs, qs, cin;

    __device__ void init(int L) {
        ks = L - 1;
        inpbl = true;
        hsum = qsum = wsum = 0.0;
        klcl = klfc = -1;
        cin = 0.0;
        act = false;
    }
    // S1, called bottom-up for k = L-1, L-2, ...: the contiguous run of layers with z <= pblh.
    __device__ void pbl(int k, int L, double z, double pblh, double h, double q, double dp) {
        if (k == L - 1 || (inpbl && z <= pblh)) {
            if (k < L - 1) ks = k;
            hsum += dp * h;
            qsum += dp * q;
            wsum += dp;
        } else {
            inpbl = false;
        }
    }
    __device__ void start() {
        hs = hsum / wsum;
        qs = qsum / wsum;
        act = ks >= 1;
    }
    // Whether layer k is examined by the S2-S5 scan (which also ends the scan where it must).
    __device__ bool wants(int k, double pm, const conv_params_t &P) {
        if (!act || k >= ks) return false;
        if ((klcl < 0 && pm < P.p_lcl_min) || (klcl >= 0 && pm < P.p_sh_top_min)) {
            act = false;
            return false;
        }
        return true;
    }
    __device__ void level(int k, const Lifted &r, double tve, double pm, double lam,
                          const conv_params_t &P) {
        const double B = tv(r.T, r.qv) - tve;
        if (klcl < 0 && r.sat) klcl = k;
        if (klcl >= 0 && B > 0.0 && pm >= P.p_sh_top_min) {
            klfc = k;
            act = false;
        } else if (B < 0.0) {
            cin += RD * (-B) * lam;
        }
    }
    // Status after S3-S6 (-1 = passes, the plume must run).
    __device__ int status(double tke, const conv_params_t &P) const {
        if (klcl < 0) return 1;
        if (klfc < 0) return 2;
        if (cin > P.cin_max) return 3;
        if (!(P.c_tke * tke > 0.0)) return 4;
        return -1;
    }
};

__device__ void write_shallow_zero(const Args &a, int64_t col, int st, double cin, int ks) {
    const int L = a.nlev;
    const int64_t ld = a.ld;
    for (int k = 0; k < L; ++k) {
        AT(a.sout.dTdt, k) = 0.0;
        AT(a.sout.dqdt, k) = 0.0;
    }
    for (int k = 0; k <= L; ++k) AT(a.sout.mu, k) = 0.0;
    a.sout.prec[col] = 0.0;
    a.sout.cin[col] = (st == 3 || st == 4) ? cin : 0.0;
    a.sout.kbase[col] = (st == 6) ? -1 : ks;
    a.sout.ktop[col] = -1;
    a.sout.status[col] = st;
}

__device__ void write_deep_zero(const Args &a, int64_t col) {
    const int L = a.nlev;
    const int64_t ld = a.ld;
    for (int k = 0; k < L; ++k) {
        AT(a.dout.dTdt, k) = 0.0;
        AT(a.dout.dqdt, k) = 0.0;
    }
    for (int k = 0; k <= L; ++k) {
        AT(a.dout.mu, k) = 0.0;
        AT(a.dout.md, k) = 0.0;
    }
    a.dout.prec[col] = 0.0;
}

// Stores the closure inputs of a shallow column that passed S1-S6 and appends it to the list.
__device__ void shallow_enqueue(const Args &a, int slot, int64_t col, const ShallowTrigger &s,
                                double rho_s, double tke, int updated) {
    const double sigw2 = a.P.c_tke * tke;
    const double sigw = sqrt(sigw2);
    a.w.slist[slot] = (int)col;
    a.w.sks[slot] = s.ks;
    a.w.sflag[slot] = updated;
    a.w.shs[slot] = s.hs;
    a.w.sqs[slot] = s.qs;
    a.w.scin[slot] = s.cin;
    a.w.ssig2[slot] = sigw2;
    a.w.sMc[slot] = rho_s * sigw / SQRT_2PI * exp(-a.P.a_buoy * s.cin / sigw2);
}

// ------------------------------------------------------------------ kernels
__global__ void k_reset(int *cnt) {
    if (threadIdx.x < NCOUNTERS) cnt[threadIdx.x] = 0;
}

template <bool DEEP, bool SHALLOW>
__global__ __launch_bounds__(BLOCK) void k_trigger(Args a) {
    const int64_t col = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool live = col < a.ncol;
    const int L = a.nlev;
    const int64_t ld = a.ld;
    const conv_params_t &P = a.P;

    bool valid = live;
    double phis = 0.0, pblh = 0.0, tke = 0.0;
    int kb = -1, klim = -1;
    double hkb = 0.0, qkb = 0.0;
    ShallowTrigger sh;
    sh.init(L);

    // Sweep 1 (bottom-up, every level): validity, h, launch layer, top limit, boundary layer.
    if (live) {
        phis = a.phis[col];
        if (SHALLOW) {
            pblh = a.pblh[col];
            tke = a.tke[col];
        }
        valid = isfinite(phis);
        double pbot = AT(a.pi, L);
        double zbelow = 0.0;
        for (int k = L - 1; k >= 0; --k) {
            const double T = AT(a.T, k), q = AT(a.q, k), pm = AT(a.pm, k), z = AT(a.z, k);
            const double pt = AT(a.pi, k);
            valid = valid && isfinite(T) && isfinite(q) && isfinite(pm) && isfinite(z) &&
                    isfinite(pbot) && T > 100.0 && T < 400.0 && q >= 0.0 && q < 1.0 && pt < pm &&
                    pm < pbot && (k == L - 1 ? z > 0.0 : z > zbelow);
            const double h = (CP * T + GRAV * z + phis) + LV * q;
            if (DEEP && pm >= P.p_launch_min && (kb < 0 || h > hkb)) {
                kb = k;
                hkb = h;
                qkb = q;
            }
            if (pm >= P.p_top_min) klim = k;
            if (SHALLOW) sh.pbl(k, L, z, pblh, h, q, pbot - pt);
            zbelow = z;
            pbot = pt;
        }
        valid = valid && isfinite(pbot) && pbot > 0.0;
    }
    const bool svalid = valid && (!SHALLOW || (isfinite(pblh) && isfinite(tke)));

    // Sweep 2 (bottom-up): deep parcel from kb (D2-D4) and shallow parcel from the source
    // (S2-S5), both evaluated at each layer they need.
    const bool dscan = DEEP && valid && kb >= 0 && klim >= 0 && klim < kb;
    int kt = -1;
    double S = 0.0, SA = 0.0, SB = 0.0, Skt = 0.0, SAkt = 0.0, SBkt = 0.0;
    if (SHALLOW && svalid) sh.start();
    if (dscan || (SHALLOW && sh.act)) {
        for (int k = L - 2; k >= 0; --k) {
            const bool dd = dscan && k < kb && k >= klim;
            const double pm = AT(a.pm, k);
            const bool ss = SHALLOW && sh.wants(k, pm, P);
            if (!dd && !ss) {
                if ((!dscan || k < klim) && !(SHALLOW && sh.act)) break;
                continue;
            }
            const double T = AT(a.T, k), q = AT(a.q, k), z = AT(a.z, k);
            const double lam = log(AT(a.pi, k + 1) / AT(a.pi, k));
            const double tve = tv(T, q);
            if (dd) {
                const Lifted r = lift(hkb - GRAV * z - phis, qkb, pm);
                const double B = tv(r.T, r.qv) - tve;
                S += RD * B * lam;
                double ca, cb;
                if (r.sat) {
                    const double c = (1.0 + CVIR * r.qv) + CVIR * r.T * r.dqs;
                    const double rden = 1.0 / (CP + LV * r.dqs);
                    ca = c * CP * rden;
                    cb = c * LV * rden;
                } else {
                    ca = 1.0 + CVIR * r.qv;
                    cb = CVIR * r.T;
                }
                SA += lam * ca;
                SB += lam * cb;
                if (B > 0.0) {
                    kt = k;
                    Skt = S;
                    SAkt = SA;
                    SBkt = SB;
                }
            }
            if (ss) {
                const Lifted r = lift(sh.hs - GRAV * z - phis, sh.qs, pm);
                sh.level(k, r, tve, pm, lam, P);
            }
        }
    }

    // Deep epilogue (D4): trigger; quiet columns get their zeros, triggered ones are compacted.
    bool trig = false;
    if (DEEP) {
        double cape = 0.0;
        int st = 1;
        if (!valid) {
            st = 3;
            kb = -1;
            kt = -1;
        } else if (dscan && kt >= 0) {
            cape = Skt > 0.0 ? Skt : 0.0;
            trig = cape > P.cape_threshold;
            st = trig ? 0 : 1;
        }
        if (live) {
            a.dout.cape[col] = cape;
            a.dout.klaunch[col] = kb;
            a.dout.ktop[col] = dscan ? kt : -1;
            a.dout.trig[col] = trig ? 1 : 0;
            a.dout.status[col] = st;
            if (!trig) write_deep_zero(a, col);
        }
        const int slot = wave_append(live && trig, &a.w.cnt[0]);
        if (slot >= 0) {
            a.w.dlist[slot] = (int)col;
            a.w.dkb[slot] = kb;
            a.w.dkt[slot] = kt;
            a.w.dcape[slot] = cape;
            a.w.dSA[slot] = SAkt;
            a.w.dSB[slot] = SBkt;
        }
    }

    // Shallow epilogue (S3-S6) for columns whose state the deep scheme leaves unchanged.
    if (SHALLOW) {
        const bool mine = live && !(DEEP && trig);
        int st = -1;
        double rho_s = 0.0;
        if (mine) {
            st = svalid ? sh.status(tke, P) : 6;
            if (st < 0) rho_s = AT(a.pi, sh.ks) / (RD * tv(AT(a.T, sh.ks), AT(a.q, sh.ks)));
            else write_shallow_zero(a, col, st, sh.cin, sh.ks);
        }
        const int slot = wave_append(mine && st < 0, &a.w.cnt[1]);
        if (slot >= 0) shallow_enqueue(a, slot, col, sh, rho_s, tke, 0);
    }
}

template <bool SHALLOW>
__global__ __launch_bounds__(BLOCK) void k_deep_plume(Args a) {
    const int n = a.w.cnt[0];
    const int L = a.nlev;
    const int64_t ld = a.ld;
    const conv_params_t &P = a.P;
    const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * BLOCK;
    const int64_t stride = a.w.scr_stride;
    double *scr = a.w.dscr;
#define SCR(arr, lev) scr[((int64_t)(arr) * (L + 1) + (lev)) * stride + tid]

    // Wavefront-uniform loop: every lane of a wavefront iterates together (for the ballot).
    const int64_t wave0 = tid - (threadIdx.x % WAVE);
    for (int64_t base = wave0; base < n; base += nthreads) {
        const int64_t slot = base + (threadIdx.x % WAVE);
        const bool act = slot < n;
        int64_t col = 0;
        int st = 0, kb = 0, kt = 0;
        double Mb = 0.0;
        if (act) {
            col = a.w.dlist[slot];
            kb = a.w.dkb[slot];
            kt = a.w.dkt[slot];
            const double cape = a.w.dcape[slot];
            const double SA = a.w.dSA[slot], SB = a.w.dSB[slot];
            const double phis = a.phis[col];
            const double epsd = P.eps_deep;
            auto zi = [&](int i) { return 0.5 * (AT(a.z, i - 1) + AT(a.z, i)); };
            auto hk = [&](int k) {
                return (CP * AT(a.T, k) + GRAV * AT(a.z, k) + phis) + LV * AT(a.q, k);
            };

            // D5: updraft, interfaces kb .. kt+1.
            const double qkb = AT(a.q, kb);
            double hu = hk(kb);
            double eta = 1.0, C1;
            {
                const double zb = zi(kb);
                const Lifted r = lift(hu - GRAV * zb - phis, qkb, AT(a.pi, kb));
                SCR(0, kb) = CP * r.T + GRAV * zb + phis;
                SCR(1, kb) = r.qv;
                C1 = qkb - r.qv;
                SCR(2, kb) = C1;
                SCR(7, kb) = 1.0;
            }
            double qup = SCR(1, kb);
            double zlo = zi(kb);
            for (int k = kb - 1; k >= kt + 1; --k) {
                const double zk = zi(k);
                const double E = epsd * eta * (zk - zlo);
                const double etan = eta + E;
                const double hm = (eta * hu + E * hk(k)) / etan;
                const double qm = (eta * qup + E * AT(a.q, k)) / etan;
                const Lifted r = lift(hm - GRAV * zk - phis, qm, AT(a.pi, k));
                const double c = etan * (qm - r.qv);
                SCR(0, k) = CP * r.T + GRAV * zk + phis;
                SCR(1, k) = r.qv;
                SCR(2, k) = c;
                SCR(7, k) = etan;
                C1 += c;
                eta = etan;
                hu = hm;
                qup = r.qv;
                zlo = zk;
            }

            // D6: downdraft from the minimum-h layer between top and base.
            int kd = -1;
            double alpha = 0.0;
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
                double ad = 1.0, hd = hkd;
                int i = kd + 1;
                double zii = zi(i);
                Sat s;
                double H = hd - GRAV * zii - phis;
                double Td = tsat(H, AT(a.pi, i), (H - LV * AT(a.q, kd)) * (1.0 / CP), s);
                double qd = s.qs;
                SCR(3, i) = CP * Td + GRAV * zii + phis;
                SCR(4, i) = qd;
                SCR(6, i) = -ad;
                double E1 = qd - AT(a.q, kd);
                SCR(5, kd) = E1;
                for (int k = kd + 1; k <= kb - 1; ++k) {
                    const double zlow = zi(k + 1);
                    const double Ed = epsd * ad * (zii - zlow);
                    const double adn = ad + Ed;
                    const double qk = AT(a.q, k);
                    hd = (ad * hd + Ed * hk(k)) / adn;
                    H = hd - GRAV * zlow - phis;
                    Td = tsat(H, AT(a.pi, k + 1), (H - LV * qk) * (1.0 / CP), s);
                    const double e1 = adn * s.qs - ad * qd - Ed * qk;
                    SCR(5, k) = e1;
                    SCR(3, k + 1) = CP * Td + GRAV * zlow + phis;
                    SCR(4, k + 1) = s.qs;
                    SCR(6, k + 1) = -adn;
                    E1 += e1;
                    ad = adn;
                    qd = s.qs;
                    zii = zlow;
                }
                alpha = P.alpha_dd;
                if (P.alpha_dd * E1 > P.evap_max_frac * C1) alpha = P.evap_max_frac * C1 / E1;
            }

            // D7 + D8/D9 accumulations: top-down over layers kt .. kb.
            double Fs_top = 0.0, Fq_top = 0.0, P1 = 0.0, Fenv = 0.0;
            double Mlim = __builtin_inf();
            double dT1 = 0.0, dq1 = 0.0;
            for (int k = kt; k <= kb; ++k) {
                double Fs = 0.0, Fq = 0.0;
                const int i = k + 1;
                if (i <= kb) {
                    const double et = SCR(7, i);
                    const bool dn = kd >= 0 && i >= kd + 1;
                    const double ed = dn ? SCR(6, i) : 0.0;
                    const int up = (et + alpha * ed >= 0.0) ? i - 1 : i;
                    const double s_up = CP * AT(a.T, up) + GRAV * AT(a.z, up) + phis;
                    const double q_up = AT(a.q, up);
                    Fs = et * (SCR(0, i) - s_up);
                    Fq = et * (SCR(1, i) - q_up);
                    if (dn) {
                        Fs += alpha * ed * (SCR(3, i) - s_up);
                        Fq += alpha * ed * (SCR(4, i) - q_up);
                    }
                }
                const double c = (k >= kt + 1) ? SCR(2, k) : 0.0;
                const double e1 = (kd >= 0 && k >= kd && k <= kb - 1) ? SCR(5, k) : 0.0;
                const double net = c - alpha * e1;
                const double dp = AT(a.pi, k + 1) - AT(a.pi, k);
                dT1 = (Fs - Fs_top + LV * net) * GRAV / (CP * dp);
                dq1 = (Fq - Fq_top - net) * GRAV / dp;
                SCR(2, k) = dT1;
                SCR(5, k) = dq1;
                P1 += net;
                const double Tk = AT(a.T, k), qk = AT(a.q, k);
                if (k <= kb - 1) {
                    const double lam = log(AT(a.pi, k + 1) / AT(a.pi, k));
                    Fenv += lam * ((1.0 + CVIR * qk) * dT1 + CVIR * Tk * dq1);
                }
                if (dq1 < 0.0) Mlim = fmin(Mlim, qk / (-a.dt * dq1));
                Fs_top = Fs;
                Fq_top = Fq;
            }
            // D8: F from the launch-layer tendencies and the parcel sensitivities of the trigger.
            const double F = -RD * (dT1 * SA + dq1 * SB - Fenv);
            if (!(F > 0.0)) {
                st = 2;
            } else {
                const double Mc = cape / (P.tau * F);
                Mb = Mc <= Mlim ? Mc : Mlim;
            }
            // D10: write every level of this column.
            for (int k = 0; k < L; ++k) {
                const bool in = st == 0 && k >= kt && k <= kb;
                AT(a.dout.dTdt, k) = in ? Mb * SCR(2, k) : 0.0;
                AT(a.dout.dqdt, k) = in ? Mb * SCR(5, k) : 0.0;
            }
            for (int i = 0; i <= L; ++i) {
                const bool in = st == 0 && i >= kt + 1 && i <= kb;
                const bool dn = in && kd >= 0 && i >= kd + 1;
                AT(a.dout.mu, i) = in ? Mb * SCR(7, i) : 0.0;
                AT(a.dout.md, i) = dn ? Mb * (alpha * SCR(6, i)) : 0.0;
            }
            a.dout.prec[col] = st == 0 ? Mb * P1 : 0.0;
            a.dout.status[col] = st;
        }

        if (SHALLOW) {
            // Shallow trigger on the deep-updated state T' = T + dt*dTdt, q' = q + dt*dqdt.
            ShallowTrigger sh;
            sh.init(L);
            int sst = -1;
            double rho_s = 0.0, tke = 0.0;
            if (act) {
                const double phis = a.phis[col];
                const double pblh = a.pblh[col];
                tke = a.tke[col];
                const bool conv = st == 0;
                auto Tn = [&](int k) {
                    return (conv && k >= kt && k <= kb) ? AT(a.T, k) + a.dt * (Mb * SCR(2, k))
                                                        : AT(a.T, k);
                };
                auto qn = [&](int k) {
                    return (conv && k >= kt && k <= kb) ? AT(a.q, k) + a.dt * (Mb * SCR(5, k))
                                                        : AT(a.q, k);
                };
                const bool svalid = isfinite(pblh) && isfinite(tke);
                if (svalid) {
                    double pbot = AT(a.pi, L);
                    for (int k = L - 1; k >= 0 && (k == L - 1 || sh.inpbl); --k) {
                        const double pt = AT(a.pi, k), z = AT(a.z, k), q = qn(k);
                        sh.pbl(k, L, z, pblh, (CP * Tn(k) + GRAV * z + phis) + LV * q, q,
                               pbot - pt);
                        pbot = pt;
                    }
                    sh.start();
                    for (int k = sh.ks - 1; k >= 0; --k) {
                        const double pm = AT(a.pm, k);
                        if (!sh.wants(k, pm, P)) break;
                        const double z = AT(a.z, k);
                        const double lam = log(AT(a.pi, k + 1) / AT(a.pi, k));
                        const Lifted r = lift(sh.hs - GRAV * z - phis, sh.qs, pm);
                        sh.level(k, r, tv(Tn(k), qn(k)), pm, lam, P);
                    }
                    sst = sh.status(tke, P);
                } else {
                    sst = 6;
                }
                if (sst < 0)
                    rho_s = AT(a.pi, sh.ks) / (RD * tv(Tn(sh.ks), qn(sh.ks)));
                else
                    write_shallow_zero(a, col, sst, sh.cin, sh.ks);
            }
            const int sslot = wave_append(act && sst < 0, &a.w.cnt[1]);
            if (sslot >= 0) shallow_enqueue(a, sslot, col, sh, rho_s, tke, 1);
        }
    }
#undef SCR
}

__global__ __launch_bounds__(BLOCK) void k_shallow_plume(Args a) {
    const int n = a.w.cnt[1];
    const int L = a.nlev;
    const int64_t ld = a.ld;
    const conv_params_t &P = a.P;
    const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * BLOCK;
    const int64_t stride = a.w.scr_stride;
    double *scr = a.w.sscr;
#define SCR(arr, lev) scr[((int64_t)(arr) * (L + 1) + (lev)) * stride + tid]

    for (int64_t slot = tid; slot < n; slot += nthreads) {
        const int64_t col = a.w.slist[slot];
        const int ks = a.w.sks[slot];
        const bool upd = a.w.sflag[slot] != 0;
        const double hs = a.w.shs[slot], qsrc = a.w.sqs[slot], cin = a.w.scin[slot];
        const double Mclos = a.w.sMc[slot], sigw2 = a.w.ssig2[slot];
        const double phis = a.phis[col];
        auto Tn = [&](int k) {
            return upd ? AT(a.T, k) + a.dt * AT(a.dout.dTdt, k) : AT(a.T, k);
        };
        auto qn = [&](int k) {
            return upd ? AT(a.q, k) + a.dt * AT(a.dout.dqdt, k) : AT(a.q, k);
        };
        auto zi = [&](int i) { return 0.5 * (AT(a.z, i - 1) + AT(a.z, i)); };

        double Mlim = __builtin_inf();
        double P1;
        // Source interface ks (S7 start).
        double Fs_lo, Fq_lo;  // fluxes at the interface below the current layer
        double eta = 1.0, hu = hs, qtu;
        {
            const double zs = zi(ks);
            const Lifted r = lift(hs - GRAV * zs - phis, qsrc, AT(a.pi, ks));
            const double ql = qsrc - r.qv;
            const double rr = ql - P.qlcrit_sh > 0.0 ? ql - P.qlcrit_sh : 0.0;
            qtu = qsrc - rr;
            const double slu = CP * r.T + GRAV * zs + phis - LV * (ql - rr);
            const double Tup = Tn(ks - 1), qupk = qn(ks - 1);
            const double s_up = CP * Tup + GRAV * AT(a.z, ks - 1) + phis;
            const double Fs = slu - s_up, Fq = qtu - qupk;
            const double dp = AT(a.pi, ks + 1) - AT(a.pi, ks);
            const double dT1 = (0.0 - Fs + LV * rr) * GRAV / (CP * dp);
            const double dq1 = (0.0 - Fq - rr) * GRAV / dp;
            SCR(0, ks) = 1.0;
            SCR(1, ks) = dT1;
            SCR(2, ks) = dq1;
            P1 = rr;
            if (dq1 < 0.0) Mlim = fmin(Mlim, qn(ks) / (-a.dt * dq1));
            Fs_lo = Fs;
            Fq_lo = Fq;
        }
        double w2 = sigw2 + 2.0 * P.a_buoy * cin;
        int kt = -1;
        double zlo = zi(ks);
        for (int k = ks - 1; k >= 0; --k) {
            bool stop = AT(a.pi, k) < P.p_sh_top_min || k == 0;
            double zk = 0.0, E = 0.0, D = 0.0, en = 0.0;
            if (!stop) {
                zk = zi(k);
                const double dz = zk - zlo;
                E = P.eps_sh * eta * dz;
                D = P.delta_sh * eta * dz;
                en = eta + E - D;
                stop = !(en > 0.0);
            }
            double Fs = 0.0, Fq = 0.0, rr = 0.0, w2n = 0.0, hm = 0.0, qtn = 0.0;
            if (!stop) {
                const double Tk = Tn(k), qk = qn(k);
                hm = ((eta - D) * hu + E * ((CP * Tk + GRAV * AT(a.z, k) + phis) + LV * qk)) / en;
                const double qm = ((eta - D) * qtu + E * qk) / en;
                const Lifted r = lift(hm - GRAV * zk - phis, qm, AT(a.pi, k));
                const double ql = qm - r.qv;
                rr = ql - P.qlcrit_sh > 0.0 ? ql - P.qlcrit_sh : 0.0;
                const double Trho = r.T * (1.0 + CVIR * r.qv - (ql - rr));
                const double Tve = tv(Tk, qk);
                const double B = GRAV * (Trho - Tve) / Tve;
                w2n = w2 + 2.0 * (zk - zlo) * (P.a_buoy * B - P.b_drag * P.eps_sh * w2);
                stop = !(w2n > 0.0);
                if (!stop) {
                    qtn = qm - rr;
                    const double slu = CP * r.T + GRAV * zk + phis - LV * (ql - rr);
                    const double s_up = CP * Tn(k - 1) + GRAV * AT(a.z, k - 1) + phis;
                    Fs = en * (slu - s_up);
                    Fq = en * (qtn - qn(k - 1));
                }
            }
            const double pr = stop ? 0.0 : en * rr;
            const double dp = AT(a.pi, k + 1) - AT(a.pi, k);
            const double dT1 = (Fs_lo - Fs + LV * pr) * GRAV / (CP * dp);
            const double dq1 = (Fq_lo - Fq - pr) * GRAV / dp;
            SCR(1, k) = dT1;
            SCR(2, k) = dq1;
            P1 += pr;
            if (dq1 < 0.0) Mlim = fmin(Mlim, qn(k) / (-a.dt * dq1));
            if (stop) {
                kt = k;
                break;
            }
            SCR(0, k) = en;
            eta = en;
            hu = hm;
            qtu = qtn;
            w2 = w2n;
            zlo = zk;
            Fs_lo = Fs;
            Fq_lo = Fq;
        }
        const int st = (kt == ks - 1) ? 5 : 0;
        const double Mb = Mclos <= Mlim ? Mclos : Mlim;
        for (int k = 0; k < L; ++k) {
            const bool in = st == 0 && k >= kt && k <= ks;
            AT(a.sout.dTdt, k) = in ? Mb * SCR(1, k) : 0.0;
            AT(a.sout.dqdt, k) = in ? Mb * SCR(2, k) : 0.0;
        }
        for (int i = 0; i <= L; ++i) {
            const bool in = st == 0 && i >= kt + 1 && i <= ks;
            AT(a.sout.mu, i) = in ? Mb * SCR(0, i) : 0.0;
        }
        a.sout.prec[col] = st == 0 ? Mb * P1 : 0.0;
        a.sout.cin[col] = cin;
        a.sout.kbase[col] = ks;
        a.sout.ktop[col] = kt;
        a.sout.status[col] = st;
    }
#undef SCR
}

#undef AT

// ------------------------------------------------------------------ host side
thread_local int g_last_hip = 0;

struct Layout {
    size_t cnt, dlist, dkb, dkt, dcape, dSA, dSB, slist, sks, sflag, shs, sqs, scin, sMc, ssig2;
    size_t dscr, sscr, total;
    int64_t plume_threads;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

Layout make_layout(int64_t ncol, int nlev, int cus) {
    Layout l{};
    const int64_t n = ncol > 0 ? ncol : 1;
    const int64_t rounded = (n + BLOCK - 1) / BLOCK * BLOCK;
    const int64_t cap = (int64_t)cus * PLUME_BLOCKS_PER_CU * BLOCK;
    l.plume_threads = rounded < cap ? rounded : cap;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    l.cnt = take(NCOUNTERS * sizeof(int));
    l.dlist = take(n * sizeof(int));
    l.dkb = take(n * sizeof(int));
    l.dkt = take(n * sizeof(int));
    l.dcape = take(n * sizeof(double));
    l.dSA = take(n * sizeof(double));
    l.dSB = take(n * sizeof(double));
    l.slist = take(n * sizeof(int));
    l.sks = take(n * sizeof(int));
    l.sflag = take(n * sizeof(int));
    l.shs = take(n * sizeof(double));
    l.sqs = take(n * sizeof(double));
    l.scin = take(n * sizeof(double));
    l.sMc = take(n * sizeof(double));
    l.ssig2 = take(n * sizeof(double));
    l.dscr = take((size_t)DEEP_SCR * (nlev + 1) * l.plume_threads * sizeof(double));
    l.sscr = take((size_t)SHALLOW_SCR * (nlev + 1) * l.plume_threads * sizeof(double));
    l.total = off;
    return l;
}

}  // namespace

constexpr int NSTAGES = 4;  // reset, trigger, deep plume, shallow plume

struct conv_ctx {
    int64_t ncol;
    int nlev;
    conv_params_t P;
    char *ws;
    size_t ws_bytes;
    Layout lay;
    // Optional per-kernel timing: NSTAGES+1 events per recorded call.
    hipEvent_t *ev;
    int ev_cap, ev_used;
};

namespace {

Work make_work(conv_ctx *c) {
    Work w;
    char *b = c->ws;
    const Layout &l = c->lay;
    w.cnt = (int *)(b + l.cnt);
    w.dlist = (int *)(b + l.dlist);
    w.dkb = (int *)(b + l.dkb);
    w.dkt = (int *)(b + l.dkt);
    w.dcape = (double *)(b + l.dcape);
    w.dSA = (double *)(b + l.dSA);
    w.dSB = (double *)(b + l.dSB);
    w.slist = (int *)(b + l.slist);
    w.sks = (int *)(b + l.sks);
    w.sflag = (int *)(b + l.sflag);
    w.shs = (double *)(b + l.shs);
    w.sqs = (double *)(b + l.sqs);
    w.scin = (double *)(b + l.scin);
    w.sMc = (double *)(b + l.sMc);
    w.ssig2 = (double *)(b + l.ssig2);
    w.dscr = (double *)(b + l.dscr);
    w.sscr = (double *)(b + l.sscr);
    w.scr_stride = l.plume_threads;
    return w;
}

bool state_ok(const conv_ctx *c, const conv_state_t *s, bool shallow) {
    if (!s || !s->T || !s->q || !s->p_mid || !s->z || !s->p_int || !s->phis) return false;
    if (shallow && (!s->pblh || !s->tke)) return false;
    if (s->ld < c->ncol || !(s->dt > 0.0)) return false;
    return true;
}

bool deep_ok(const conv_deep_out_t *o) {
    return o && o->dTdt && o->dqdt && o->mu && o->md && o->prec && o->cape && o->klaunch &&
           o->ktop && o->trig && o->status;
}

bool shallow_ok(const conv_shallow_out_t *o) {
    return o && o->dTdt && o->dqdt && o->mu && o->prec && o->cin && o->kbase && o->ktop &&
           o->status;
}

Args make_args(conv_ctx *c, const conv_state_t *s, const conv_deep_out_t *d,
               const conv_shallow_out_t *sh) {
    Args a;
    memset(&a, 0, sizeof(a));
    a.T = s->T;
    a.q = s->q;
    a.pm = s->p_mid;
    a.pi = s->p_int;
    a.z = s->z;
    a.phis = s->phis;
    a.pblh = s->pblh;
    a.tke = s->tke;
    a.ld = s->ld;
    a.dt = s->dt;
    a.ncol = c->ncol;
    a.nlev = c->nlev;
    a.P = c->P;
    if (d) a.dout = *d;
    if (sh) a.sout = *sh;
    a.w = make_work(c);
    return a;
}

int finish() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        return CONV_EHIP;
    }
    return CONV_OK;
}

template <bool DEEP, bool SHALLOW>
int run(conv_ctx *c, const Args &a, hipStream_t st) {
    const unsigned grid_cols = (unsigned)((c->ncol + BLOCK - 1) / BLOCK);
    const unsigned grid_plume = (unsigned)(c->lay.plume_threads / BLOCK);
    hipEvent_t *ev = nullptr;
    if (c->ev && c->ev_used < c->ev_cap) ev = c->ev + (size_t)(c->ev_used++) * (NSTAGES + 1);
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(NCOUNTERS), 0, st, a.w.cnt);
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL((k_trigger<DEEP, SHALLOW>), dim3(grid_cols), dim3(BLOCK), 0, st, a);
    if (ev) (void)hipEventRecord(ev[2], st);
    if (DEEP) hipLaunchKernelGGL((k_deep_plume<SHALLOW>), dim3(grid_plume), dim3(BLOCK), 0, st, a);
    if (ev) (void)hipEventRecord(ev[3], st);
    if (SHALLOW) hipLaunchKernelGGL(k_shallow_plume, dim3(grid_plume), dim3(BLOCK), 0, st, a);
    if (ev) (void)hipEventRecord(ev[4], st);
    return finish();
}

void free_events(conv_ctx *c) {
    if (c->ev) {
        for (int i = 0; i < c->ev_cap * (NSTAGES + 1); ++i) (void)hipEventDestroy(c->ev[i]);
        delete[] c->ev;
    }
    c->ev = nullptr;
    c->ev_cap = c->ev_used = 0;
}

}  // namespace

extern "C" {

size_t conv_workspace_bytes(int64_t ncol, int32_t nlev) {
    if (ncol < 0 || nlev < 2 || nlev > 256) return 0;
    return make_layout(ncol, nlev, device_cus()).total;
}

int conv_create(int64_t ncol, int32_t nlev, const conv_params_t *params, void *workspace,
                size_t ws_bytes, conv_ctx_t **out) {
    // Argument checks come first and make no HIP call.
    if (!out || !params || !workspace || ncol < 0 || ncol > INT32_MAX || nlev < 2 || nlev > 256)
        return CONV_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return CONV_EINVAL;
    const Layout l = make_layout(ncol, nlev, device_cus());
    if (ws_bytes < l.total) return CONV_EINVAL;
    conv_ctx *c = new conv_ctx;
    c->ncol = ncol;
    c->nlev = nlev;
    c->P = *params;
    c->ws = (char *)workspace;
    c->ws_bytes = ws_bytes;
    c->lay = l;
    c->ev = nullptr;
    c->ev_cap = c->ev_used = 0;
    *out = c;
    return CONV_OK;
}

int conv_set_params(conv_ctx_t *ctx, const conv_params_t *params) {
    if (!ctx || !params) return CONV_EINVAL;
    ctx->P = *params;
    return CONV_OK;
}

void conv_destroy(conv_ctx_t *ctx) {
    if (!ctx) return;
    free_events(ctx);
    delete ctx;
}

int conv_timing_start(conv_ctx_t *ctx, int max_calls) {
    if (!ctx || max_calls < 0) return CONV_EINVAL;
    free_events(ctx);
    if (max_calls == 0) return CONV_OK;
    ctx->ev = new hipEvent_t[(size_t)max_calls * (NSTAGES + 1)];
    for (int i = 0; i < max_calls * (NSTAGES + 1); ++i) {
        if (hipEventCreate(&ctx->ev[i]) != hipSuccess) {
            ctx->ev_cap = i / (NSTAGES + 1);
            free_events(ctx);
            return CONV_EHIP;
        }
    }
    ctx->ev_cap = max_calls;
    ctx->ev_used = 0;
    return CONV_OK;
}

int conv_timing_read(conv_ctx_t *ctx, double *ms, int *ncalls) {
    if (!ctx || !ms || !ncalls) return CONV_EINVAL;
    for (int s = 0; s < NSTAGES; ++s) ms[s] = 0.0;
    *ncalls = ctx->ev_used;
    for (int i = 0; i < ctx->ev_used; ++i) {
        hipEvent_t *ev = ctx->ev + (size_t)i * (NSTAGES + 1);
        if (hipEventSynchronize(ev[NSTAGES]) != hipSuccess) return CONV_EHIP;
        for (int s = 0; s < NSTAGES; ++s) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[s], ev[s + 1]) != hipSuccess) return CONV_EHIP;
            ms[s] += t;
        }
    }
    return CONV_OK;
}

int conv_deep_forward(conv_ctx_t *ctx, const conv_state_t *state, conv_deep_out_t *out,
                      void *stream) {
    if (!ctx || !state_ok(ctx, state, false) || !deep_ok(out)) return CONV_EINVAL;
    if (ctx->ncol == 0) return CONV_OK;
    const Args a = make_args(ctx, state, out, nullptr);
    return run<true, false>(ctx, a, (hipStream_t)stream);
}

int conv_shallow_forward(conv_ctx_t *ctx, const conv_state_t *state, conv_shallow_out_t *out,
                         void *stream) {
    if (!ctx || !state_ok(ctx, state, true) || !shallow_ok(out)) return CONV_EINVAL;
    if (ctx->ncol == 0) return CONV_OK;
    const Args a = make_args(ctx, state, nullptr, out);
    return run<false, true>(ctx, a, (hipStream_t)stream);
}

int conv_step(conv_ctx_t *ctx, const conv_state_t *state, conv_deep_out_t *deep,
              conv_shallow_out_t *shallow, void *stream) {
    if (!ctx || !state_ok(ctx, state, true) || !deep_ok(deep) || !shallow_ok(shallow))
        return CONV_EINVAL;
    if (ctx->ncol == 0) return CONV_OK;
    const Args a = make_args(ctx, state, deep, shallow);
    return run<true, true>(ctx, a, (hipStream_t)stream);
}

const char *conv_strerror(int code) {
    switch (code) {
        case CONV_OK: return "ok";
        case CONV_EINVAL: return "invalid argument";
        case CONV_EUNSUPPORTED: return "unsupported";
        case CONV_EHIP: return "HIP launch failure";
        default: return "unknown error";
    }
}

int conv_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
