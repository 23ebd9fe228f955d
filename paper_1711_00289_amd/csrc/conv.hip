// conv.hip -- gfx950 kernels and the C ABI (include/conv.h) of the FP64 deep + shallow convection
// library.
//
// One physics step (the paper's Algorithm 1 order: deep, then shallow on the updated state):
//   k_reset          zero the on-device counters (a fill kernel, so a captured step replays).
//   k_trigger        one lane per column, one bottom-up sweep over every level: validity, moist
//                    static energy, the launch layer (D1), then the undilute parcel with CAPE and
//                    the closure's parcel sensitivities (D2-D4) and the shallow source, parcel and
//                    CIN (S1-S6).  Quiet columns get their exact-zero outputs at once; triggered
//                    ones are compacted into an on-device list by wavefront ballot + popcount + one
//                    atomic per wavefront, so the imbalance between convecting and quiet columns
//                    (the paper's Methodology, "Load Balancing Convections") is removed by
//                    compaction rather than by scheduling individual columns.
//   k_deep_plume     persistent; wavefronts claim 64 consecutive slots of the deep list at a time:
//                    updraft (D5), downdraft (D6), flux-form tendencies (D7), closure (D8),
//                    limiter (D9), outputs (D10).
//   k_shallow_retrigger  the shallow trigger (S1-S6) of the deep columns on the deep-updated
//                    state, with the plume, tendencies and limiter (S7-S9) of those that pass in
//                    the same lane; then the plumes of the columns the trigger listed.
//   k_shallow_plume  persistent over the shallow list: S7-S9 (the shallow scheme alone).
// Per-level plume profiles live in a per-thread scratch region of the caller's workspace laid out
// [array][level][thread], so a wavefront's accesses to one level are contiguous; the deep plume
// keeps its unit tendencies in LDS when the grid has at most 31 levels.  Level loops load
// the next level's inputs before working on the current level.  Kernels are generic over a member
// source: one grid (kernel argument) or an ensemble table of grids with their own level counts,
// parameters and arrays (device memory) covered by the same launches.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "conv.h"
#include "conv_internal.hpp"

using namespace cvk;

thread_local int g_last_hip = 0;

namespace cvk {

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

int check_launch() {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        return CONV_EHIP;
    }
    return CONV_OK;
}

}  // namespace cvk

namespace {

constexpr int DEEP_SCR = 7;     // deep plume profiles (enum DeepScr)
constexpr int SHALLOW_SCR = 3;  // eta, dT1, dq1
constexpr int CNT_DEEP = 0;
constexpr int CNT_SHALLOW = 1;
constexpr int CNT_DGRAB = 2;  // deep-list slots claimed by the deep plume past its first round

struct Work {
    int *cnt;
    int *dlist, *dmem, *dkb, *dkt, *dkd;
    double *dcape, *dSA, *dSB;
    int *slist, *smem, *sks, *sflag;
    double *shs, *sqs, *scin, *sMc, *ssig2;
    double *dscr, *sscr;
    int64_t dstride, sstride;  // threads of the deep-plume / shallow-plume persistent grids
    int64_t rstride;           // threads of the shallow re-trigger grid
    int lmax;                  // level capacity of the scratch
    int cus;                   // compute units of the device
};

constexpr int RETRIGGER_BPC = 3;  // 256-thread units per compute unit of the shallow re-trigger

// The deep plume keeps its unit tendencies (the last two of its DEEP_SCR profiles) of the XW
// layers from the launch layer up in LDS: 31 KB per wavefront, so that its default five
// wavefronts per CU stay resident (32 KB each left room for four).  Grids of at most XW levels
// never need more, and the workspace then holds only the other profiles; deeper plumes keep
// their upper layers' tendencies in the workspace.
constexpr int XW = 31;
constexpr size_t DEEP_X_LDS = (size_t)2 * XW * WAVE * sizeof(double);
inline bool deep_xg(int lmax) { return lmax > XW; }
inline int deep_scr_global(int lmax) { return deep_xg(lmax) ? DEEP_SCR : DEEP_SCR - 2; }


// The inputs of one level of one column (pt = p_int at the level's top interface).
struct Lev {
    double T, q, pm, z, pt;
};

// The trigger's sweep streams every input once: non-temporal loads, which keep the rest of the
// grid's lines from displacing what the plume passes re-read.
__device__ __forceinline__ void load_lev(Lev &v, const Member &M, int64_t ld, int64_t col, int k) {
    v.T = __builtin_nontemporal_load(&AT(M.T, k));
    v.q = __builtin_nontemporal_load(&AT(M.q, k));
    v.pm = __builtin_nontemporal_load(&AT(M.pm, k));
    v.z = __builtin_nontemporal_load(&AT(M.z, k));
    v.pt = __builtin_nontemporal_load(&AT(M.pi, k));
}

// ------------------------------------------------------------------ shallow trigger (S1-S6)
struct ShallowTrigger {
    int ks, klcl, klfc;
    bool inpbl, act;
    double hsum, qsum, wsum, hs, qs, cin;
    Hint hint;

    __device__ void init(int L) {
        ks = L - 1;
        inpbl = true;
        hsum = qsum = wsum = 0.0;
        klcl = klfc = -1;
        cin = 0.0;
        act = false;
        hint.clear();
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
    __device__ void level(int k, double z, double phis, double tve, double pm, double lam,
                          const conv_params_t &P) {
        const Lifted r = lift(hs - GRAV * z - phis, qs, pm, hint);
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

// Scalar outputs of a column the shallow scheme leaves alone (its arrays were zeroed in sweep 1).
__device__ void write_shallow_quiet(const Member &M, int64_t col, int st, double cin, int ks) {
    M.sout.prec[col] = 0.0;
    M.sout.cin[col] = (st == 3 || st == 4) ? cin : 0.0;
    M.sout.kbase[col] = (st == 6) ? -1 : ks;
    M.sout.ktop[col] = -1;
    M.sout.status[col] = st;
}

// Zero every output array of level k (and of interface k) of a column: the exact-zero outputs of
// quiet columns, written while the sweep's loads are in flight; the plume passes overwrite only
// the levels a plume touches.  Non-temporal stores: these lines are not read again in the step
// (step 0.948 -> 0.924 ms with the non-temporal loads above, the trigger and the plume both
// faster).
template <bool DEEP, bool SHALLOW>
__device__ __forceinline__ void zero_level(const Member &M, int64_t ld, int64_t col, int k) {
    if (DEEP) {
        __builtin_nontemporal_store(0.0, &AT(M.dout.dTdt, k));
        __builtin_nontemporal_store(0.0, &AT(M.dout.dqdt, k));
        __builtin_nontemporal_store(0.0, &AT(M.dout.mu, k));
        __builtin_nontemporal_store(0.0, &AT(M.dout.md, k));
    }
    if (SHALLOW) {
        __builtin_nontemporal_store(0.0, &AT(M.sout.dTdt, k));
        __builtin_nontemporal_store(0.0, &AT(M.sout.dqdt, k));
        __builtin_nontemporal_store(0.0, &AT(M.sout.mu, k));
    }
}

// M_c of S8 from the closure inputs of a column that passed S1-S6.
__device__ __forceinline__ double shallow_closure(const Member &M, const ShallowTrigger &s,
                                                  double rho_s, double sigw2) {
    const double sigw = sqrt(sigw2);
    return rho_s * sigw / SQRT_2PI * exp(-M.P.a_buoy * s.cin / sigw2);
}

// Stores the closure inputs of a shallow column that passed S1-S6 in list slot `slot`.
__device__ void shallow_enqueue(const Member &M, const Work &w, int slot, int mi, int64_t col,
                                const ShallowTrigger &s, double rho_s, double tke, int updated) {
    const double sigw2 = M.P.c_tke * tke;
    w.slist[slot] = (int)col;
    w.smem[slot] = mi;
    w.sks[slot] = s.ks;
    w.sflag[slot] = updated;
    w.shs[slot] = s.hs;
    w.sqs[slot] = s.qs;
    w.scin[slot] = s.cin;
    w.ssig2[slot] = sigw2;
    w.sMc[slot] = shallow_closure(M, s, rho_s, sigw2);
}

// ------------------------------------------------------------------ kernels
__global__ void k_reset(int *cnt) {
    if (threadIdx.x < NCOUNTERS) cnt[threadIdx.x] = 0;
}

// Trigger pass: one lane per column; block b covers tile b of the launch's tile space.  Every
// level loop loads the next level's inputs before working on the current one, so the loads of a
// level are in flight during the previous level's Newton solves.
template <class Src, bool DEEP, bool SHALLOW>
__global__ __launch_bounds__(BLOCK) void k_trigger(Src src, Work w) {
    const int64_t tile = blockIdx.x;
    const int mi = src.find(tile);
    const Member M = src.at(mi);  // a copy: loaded once (through a reference into the member
                                  // table every use would be reloaded after each store)
    const int L = M.nlev;
    const int64_t ld = M.ld;
    const conv_params_t &P = M.P;
    const int64_t col = (tile - M.tile0) * BLOCK + threadIdx.x;
    const bool live = col < M.ncol;

    bool valid = live;
    double phis = 0.0, pblh = 0.0, tke = 0.0;
    int kb = -1;
    double hkb = 0.0;
    double hmix = 0.0, qmix = 0.0;  // the (dilute) parcel's h and total water
    const bool dilute = P.eps_cape > 0.0;
    ShallowTrigger sh;
    sh.init(L);
    bool sstarted = false;
    int kt = -1;
    double S = 0.0, SA = 0.0, SB = 0.0, Skt = 0.0, SAkt = 0.0, SBkt = 0.0;
    Hint hd;
    hd.clear();
    // Downdraft start (D6): argmin h over the parcel's layers passed so far (kt+1 .. kb-1 once kt
    // is fixed); scanning upward, a tie goes to the upper layer.
    double hmin = 0.0;
    int kmin = -1, kdkt = -1;

    // One bottom-up sweep reads every level once: validity (C0), zero outputs, h, the launch
    // layer (D1), the undilute parcel with CAPE and the closure's parcel sensitivities (D2-D4),
    // the boundary-layer source (S1) and the shallow parcel (S2-S5).  The deep parcel rises from
    // the best launch layer found so far and restarts whenever a higher-h layer of the launch
    // region appears below it (a level the parcel has passed is never needed again: the parcel
    // of the final launch layer starts above it).
    if (live) {
        phis = M.phis[col];
        if (SHALLOW) {
            pblh = M.pblh[col];
            tke = M.tke[col];
        }
        valid = isfinite(phis);
        double pbot = AT(M.pi, L);
        double zbelow = 0.0;
        if (DEEP) {
            AT(M.dout.mu, L) = 0.0;
            AT(M.dout.md, L) = 0.0;
        }
        if (SHALLOW) AT(M.sout.mu, L) = 0.0;
        auto step = [&](const Lev &v, int k) {
            zero_level<DEEP, SHALLOW>(M, ld, col, k);
            valid = valid && isfinite(v.T) && isfinite(v.q) && isfinite(v.pm) && isfinite(v.z) &&
                    isfinite(pbot) && v.T > 100.0 && v.T < 400.0 && v.q >= 0.0 && v.q < 1.0 &&
                    v.pt < v.pm && v.pm < pbot && (k == L - 1 ? v.z > 0.0 : v.z > zbelow);
            const double h = (CP * v.T + GRAV * v.z + phis) + LV * v.q;
            bool dd = false;
            if (DEEP) {
                if (v.pm >= P.p_launch_min && (kb < 0 || h > hkb)) {
                    kb = k;  // a new launch layer: the parcel restarts above it
                    hkb = h;
                    hmix = h;
                    qmix = v.q;
                    kt = -1;
                    S = SA = SB = Skt = SAkt = SBkt = 0.0;
                    hd.clear();
                    kmin = kdkt = -1;
                } else {
                    dd = kb >= 0 && v.pm >= P.p_top_min;
                }
            }
            bool ss = false;
            if (SHALLOW) {
                if (!sstarted) {
                    sh.pbl(k, L, v.z, pblh, h, v.q, pbot - v.pt);
                    if (!sh.inpbl) {
                        sh.start();
                        sstarted = true;
                    }
                }
                ss = sstarted && sh.wants(k, v.pm, P);
            }
            if (dd || ss) {
                const double lam = log(pbot / v.pt);
                const double tve = tv(v.T, v.q);
                if (dd) {
                    if (dilute) {  // entrain layer k's air over the rise from layer k+1
                        const double mix = P.eps_cape * (v.z - zbelow);
                        hmix = (hmix + mix * h) / (1.0 + mix);
                        qmix = (qmix + mix * v.q) / (1.0 + mix);
                    }
                    const Lifted r = lift(hmix - GRAV * v.z - phis, qmix, v.pm, hd);
                    const double B = tv(r.T, r.qv) - tve;
                    S += RD * B * lam;
                    double ca, cb;
                    if (r.sat) {
                        const double c = (1.0 + CVIR * r.qv) + CVIR * r.T * r.dqs;
                        const double rden = frcp(CP + LV * r.dqs);
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
                        kdkt = kmin;
                    }
                    if (kmin < 0 || h <= hmin) {
                        kmin = k;
                        hmin = h;
                    }
                }
                if (ss) sh.level(k, v.z, phis, tve, v.pm, lam, P);
            }
            zbelow = v.z;
            pbot = v.pt;
        };
        // Two level buffers: level k-1 loads while level k is worked on (a third buffer costs the
        // registers of a third resident wavefront per SIMD).  Loads are unconditional (level
        // index clamped at 0) so the wait counts stay exact.
        Lev b0, b1;
        load_lev(b0, M, ld, col, L - 1);
        for (int k = L - 1; k >= 0; k -= 2) {
            load_lev(b1, M, ld, col, max(k - 1, 0));
            step(b0, k);
            if (k - 1 < 0) break;
            load_lev(b0, M, ld, col, max(k - 2, 0));
            step(b1, k - 1);
        }
        valid = valid && isfinite(pbot) && pbot > 0.0;
        if (SHALLOW && !sstarted) sh.start();  // the boundary layer reaches the model top
    }
    const bool svalid = valid && (!SHALLOW || (isfinite(pblh) && isfinite(tke)));
    // (A column with no parcel layer at or below p_top_min above kb keeps kt = -1: not triggered.)
    const bool dscan = DEEP && valid && kb >= 0;

    // Deep epilogue (D4): quiet columns get their zeros; triggered ones are compacted into the
    // deep list with what the plume pass needs.
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
            M.dout.cape[col] = cape;
            M.dout.klaunch[col] = kb;
            M.dout.ktop[col] = dscan ? kt : -1;
            M.dout.trig[col] = trig ? 1 : 0;
            M.dout.status[col] = st;
            if (!trig) M.dout.prec[col] = 0.0;
        }
        const int slot = wave_append(live && trig, &w.cnt[CNT_DEEP]);
        if (slot >= 0) {
            w.dlist[slot] = (int)col;
            w.dmem[slot] = mi;
            w.dkb[slot] = kb;
            w.dkt[slot] = kt;
            w.dkd[slot] = kdkt;
            w.dcape[slot] = cape;
            w.dSA[slot] = SAkt;
            w.dSB[slot] = SBkt;
        }
    }

    // Shallow epilogue (S3-S6) for columns whose state the deep scheme leaves unchanged.
    if (SHALLOW) {
        const bool mine = live && !(DEEP && trig);
        int st = -1;
        double rho_s = 0.0;
        if (mine) {
            st = svalid ? sh.status(tke, P) : 6;
            if (st < 0)
                rho_s = AT(M.pi, sh.ks) / (RD * tv(AT(M.T, sh.ks), AT(M.q, sh.ks)));
            else
                write_shallow_quiet(M, col, st, sh.cin, sh.ks);
        }
        const int slot = wave_append(mine && st < 0, &w.cnt[CNT_SHALLOW]);
        if (slot >= 0) shallow_enqueue(M, w, slot, mi, col, sh, rho_s, tke, 0);
    }
}

// Per-thread plume scratch of the deep pass ([profile][level][thread]).  Only the last three are
// kept for every level of the plume; the others only for the downdraft region kd .. kb.
enum DeepScr : int {
    U_SU = 0, U_QU, U_C,   // updraft s, q_v and condensation at interfaces kd+1 .. kb
    D_ED,                  // downdraft eta_d (< 0) at interfaces kd+1 .. kb
    U_ETA,                 // updraft mass flux at interfaces kt+1 .. kb
    X_DT1, X_DQ1,          // unit tendencies in layers kt .. kb (last: in LDS up to XW layers)
};

// Deep plume pass, persistent over the deep list.  Per column: the entraining updraft (D5) from
// the base to the top, which also completes the fluxes and tendencies (D7) of the layers above the
// downdraft, where the downdraft strength alpha does not enter; then one top-down sweep from the
// trigger's k_d to the base that carries the saturated downdraft (D6) and, at each of its
// interfaces, the fluxes and tendencies of the layer above; then the closure (D8), limiter (D9)
// and outputs (D10).  The updraft finishes an interface one level after computing it, when the
// upwind layer's values (the next level up) have arrived.  The downdraft sweep takes alpha at its
// uncapped value; alpha is capped by the updraft's condensation only when the downdraft's total
// evaporation, known at the end of the sweep, exceeds the allowed fraction of it, and then the
// sweep runs again with the capped alpha (its contributions are accumulated apart for this).
// The unit tendencies live in the block's LDS (one wavefront per block, [array][kb - level]
// [lane]) instead of the global scratch: they are written once per layer and read back by the
// closure and the output stores, and in LDS they leave the caches to the inputs and the other
// profiles.  With XG, layers more than XW above the launch layer use the global scratch.
template <class Src, bool XG>
__global__ __launch_bounds__(WAVE) void k_deep_plume(Src src, Work w) {
    const int n = w.cnt[CNT_DEEP];
    const int64_t gtid = (int64_t)blockIdx.x * WAVE + threadIdx.x;
    const int lane = threadIdx.x % WAVE;
    double *scr = w.dscr;
#define SCR(arr, lev) scr[((int64_t)(arr) * (w.lmax + 1) + (lev)) * w.dstride + gtid]
    extern __shared__ double xlds[];

    // Wavefront g takes slots 64g .. 64g+63 of the deep list, then claims the next 64 unclaimed
    // slots past the grid's first round until the list runs out (list order keeps a wavefront's
    // columns close in memory).  Lane 0 holds the smallest slot, so it is active whenever any
    // lane is.
    const int64_t first_round = (int64_t)gridDim.x * WAVE;
    for (int64_t slot0 = gtid - lane;;) {
        const int64_t slot = slot0 + lane;
        if (slot >= n) break;
        const Member M = src.at(w.dmem[slot]);  // a copy: the fields stay in registers
        const int64_t ld = M.ld;
        const conv_params_t &P = M.P;
        const int64_t col = w.dlist[slot];
        const int kb = w.dkb[slot], kt = w.dkt[slot], kd = w.dkd[slot];
        const double cape = w.dcape[slot];
        const double SA = w.dSA[slot], SB = w.dSB[slot];
        const double phis = M.phis[col];
        const double epsd = P.eps_deep;
        const double dt = M.dt;
        // Unit tendency a (0: dT1, 1: dq1) of layer k (kt <= k <= kb).
        auto xput = [&](int a, int k, double v) {
            const int r = kb - k;
            if (!XG || r < XW)
                xlds[(a * XW + r) * WAVE + lane] = v;
            else
                SCR(X_DT1 + a, k) = v;
        };
        auto xget = [&](int a, int k) {
            const int r = kb - k;
            return (!XG || r < XW) ? xlds[(a * XW + r) * WAVE + lane] : SCR(X_DT1 + a, k);
        };

        // Accumulations of D7-D9: the layers the updraft sweep completes, and the downdraft
        // region (kept apart, since it is recomputed when alpha is capped).
        struct Acc {
            double P1, Fenv, Mlim;
        };
        Acc up = {0.0, 0.0, __builtin_inf()}, dn = {0.0, 0.0, __builtin_inf()};
        double dT1kb = 0.0, dq1kb = 0.0;
        // One layer's unit tendencies from the fluxes at its top and bottom interfaces.
        auto layer = [&](Acc &a, int k, double Fs_top, double Fq_top, double Fs_bot, double Fq_bot,
                         double net, double T, double q, double p_top, double p_bot) {
            const double dp = p_bot - p_top;
            const double dT1 = (Fs_bot - Fs_top + LV * net) * GRAV / (CP * dp);
            const double dq1 = (Fq_bot - Fq_top - net) * GRAV / dp;
            xput(0, k, dT1);
            xput(1, k, dq1);
            a.P1 += net;
            if (k <= kb - 1) {
                a.Fenv += log(p_bot / p_top) * ((1.0 + CVIR * q) * dT1 + CVIR * T * dq1);
            } else {
                dT1kb = dT1;
                dq1kb = dq1;
            }
            if (dq1 < 0.0) a.Mlim = fmin(a.Mlim, q / (-dt * dq1));
        };

        // D5 + the alpha-free part of D7: updraft from the base (interface kb) to interface kt+1.
        // `u_*` hold the updraft at interface i+1, `e_*` the environment of layer i+1, `p_top` and
        // `p_bot` its interface pressures, `Fs_b`/`Fq_b` the flux at interface i+2.
        double C1;
        double Fs_kd = 0.0, Fq_kd = 0.0, c_kd = 0.0;  // interface kd, for the downdraft region
        {
            Hint hu;
            hu.clear();
            const double qkb = AT(M.q, kb), Tkb = AT(M.T, kb), zkb = AT(M.z, kb);
            double zup = AT(M.z, kb - 1);
            double hu_m = (CP * Tkb + GRAV * zkb + phis) + LV * qkb;
            double zlo = 0.5 * (zup + zkb);
            double u_eta = 1.0, u_su, u_qu, u_c;
            {
                const Lifted r = lift(hu_m - GRAV * zlo - phis, qkb, AT(M.pi, kb), hu);
                u_su = CP * r.T + GRAV * zlo + phis;
                u_qu = r.qv;
                u_c = qkb - r.qv;
            }
            C1 = u_c;
            SCR(U_ETA, kb) = 1.0;
            if (kd >= 0) {
                SCR(U_SU, kb) = u_su;
                SCR(U_QU, kb) = u_qu;
                SCR(U_C, kb) = u_c;
            }
            double e_T = Tkb, e_q = qkb, p_top = AT(M.pi, kb), p_bot = AT(M.pi, kb + 1);
            double Fs_b = 0.0, Fq_b = 0.0;
            // Interface i+1 and layer i+1, with the environment of layer i (the upwind layer:
            // the compensating flow points up where there is no downdraft).
            auto finish = [&](int i, double Ti, double qi, double zi_) {
                const int j = i + 1;
                if (kd >= 0 && j >= kd + 1) return;  // downdraft region: after alpha
                const double s_up = CP * Ti + GRAV * zi_ + phis;
                const double Fs = u_eta * (u_su - s_up);
                const double Fq = u_eta * (u_qu - qi);
                if (kd < 0 || j <= kd - 1) {
                    layer(up, j, Fs, Fq, Fs_b, Fq_b, u_c, e_T, e_q, p_top, p_bot);
                } else {  // j == kd
                    Fs_kd = Fs;
                    Fq_kd = Fq;
                    c_kd = u_c;
                }
                Fs_b = Fs;
                Fq_b = Fq;
            };
            // Layer k needs T, q and the top-interface pressure of layer k and the height of the
            // layer above.  Two level buffers: the loads of layer k-2 are issued while layer k is
            // worked on (indices clamped at 0; values past the top are not used).
            struct UpLev {
                double T, q, zab, p;
            };
            auto upload = [&](int k) {
                UpLev v;
                const int kk = max(k, 0);
                v.T = AT(M.T, kk);
                v.q = AT(M.q, kk);
                v.zab = AT(M.z, max(k - 1, 0));
                v.p = AT(M.pi, kk);
                return v;
            };
            double zcur = zup;  // height of the layer being worked on
            auto uplevel = [&](const UpLev &v, int k) {
                const double Tk = v.T, qk = v.q, zkk = zcur, zabove = v.zab, pik = v.p;
                zcur = zabove;
                finish(k, Tk, qk, zkk);
                const double zk = 0.5 * (zabove + zkk);
                const double hkk = (CP * Tk + GRAV * zkk + phis) + LV * qk;
                const double E = epsd * u_eta * (zk - zlo);
                const double etan = u_eta + E;
                const double hm = (u_eta * hu_m + E * hkk) / etan;
                const double qm = (u_eta * u_qu + E * qk) / etan;
                const Lifted r = lift(hm - GRAV * zk - phis, qm, pik, hu);
                u_eta = etan;
                u_su = CP * r.T + GRAV * zk + phis;
                u_qu = r.qv;
                u_c = etan * (qm - r.qv);
                C1 += u_c;
                SCR(U_ETA, k) = etan;
                if (kd >= 0 && k >= kd + 1) {
                    SCR(U_SU, k) = u_su;
                    SCR(U_QU, k) = u_qu;
                    SCR(U_C, k) = u_c;
                }
                hu_m = hm;
                zlo = zk;
                e_T = Tk;
                e_q = qk;
                p_bot = p_top;
                p_top = pik;
            };
            UpLev u0 = upload(kb - 1), u1 = upload(kb - 2);
            bool top_in_u1 = false;  // which buffer holds layer kt when the sweep ends
            for (int k = kb - 1; k >= kt + 1; k -= 2) {
                uplevel(u0, k);
                u0 = upload(k - 2);
                if (k - 1 < kt + 1) {
                    top_in_u1 = true;
                    break;
                }
                uplevel(u1, k - 1);
                u1 = upload(k - 3);
            }
            const double tT = top_in_u1 ? u1.T : u0.T, tq = top_in_u1 ? u1.q : u0.q,
                         tp = top_in_u1 ? u1.p : u0.p;
            // Interface kt+1 and layer kt+1 with layer kt's environment (loaded ahead), then the
            // top layer kt, whose upper flux is zero and which has no source.
            finish(kt, tT, tq, zcur);
            layer(up, kt, 0.0, 0.0, Fs_b, Fq_b, 0.0, tT, tq, tp, p_top);
        }

        // D6 with the downdraft region's part of D7: layers kd .. kb, top down.
        double alpha = 0.0;
        if (kd >= 0) {
            // What layer k needs from memory: the environment of layer k+1 and the pressure of
            // the interface between them (which the downdraft reaches next), and the updraft at
            // that interface and its condensation in layer k.  Two level buffers: the loads of
            // layer k+2 are issued while layer k is worked on (levels clamped, so every load is in
            // range; values past the base are not used).
            struct FLev {
                double Tb, qb, zb, pb, et, su, qu, c;
            };
            auto fload = [&](int k) {
                FLev v;
                const int i = min(k + 1, kb), kk = min(k, kb);
                v.Tb = AT(M.T, i);
                v.qb = AT(M.q, i);
                v.zb = AT(M.z, i);
                v.pb = AT(M.pi, min(k + 1, kb + 1));
                v.et = SCR(U_ETA, i);
                v.su = SCR(U_SU, i);
                v.qu = SCR(U_QU, i);
                v.c = SCR(U_C, kk);
                return v;
            };
            const double T_kd = AT(M.T, kd), q_kd = AT(M.q, kd), z_kd = AT(M.z, kd),
                         p_kd = AT(M.pi, kd);
            alpha = P.alpha_dd;
            for (int pass = 0;; ++pass) {
                Hint hdn;
                hdn.clear();
                Sat s;
                dn = {0.0, 0.0, __builtin_inf()};
                double E1 = 0.0, hd = 0.0, ad = 1.0, qd = 0.0, zii = 0.0;
                double Fs_t = Fs_kd, Fq_t = Fq_kd;
                double Tk = T_kd, qk = q_kd, zk = z_kd, pt = p_kd;
                auto flevel = [&](const FLev &v, int k) {
                    const int i = k + 1;  // the layer's bottom interface
                    double Fs = 0.0, Fq = 0.0, e1 = 0.0;
                    if (i <= kb) {
                        // The downdraft from interface k down to i: it starts saturated at the
                        // interface below k_d with layer k_d's h; below, it entrains each layer's
                        // air in proportion to its mass flux and the distance.
                        const double zlow = 0.5 * (zk + v.zb);
                        double adn, Ed = 0.0;
                        if (k == kd) {
                            hd = (CP * Tk + GRAV * zk + phis) + LV * qk;
                            adn = 1.0;
                        } else {
                            const double hk = (CP * Tk + GRAV * zk + phis) + LV * qk;
                            Ed = epsd * ad * (zii - zlow);
                            adn = ad + Ed;
                            hd = (ad * hd + Ed * hk) / adn;
                        }
                        const double H = hd - GRAV * zlow - phis;
                        const double Td = tsat_h(H, v.pb, (H - LV * qk) * RCP_CP, s, hdn);
                        if (k == kd) {
                            e1 = s.qs - qk;
                        } else {
                            e1 = adn * s.qs - ad * qd - Ed * qk;
                        }
                        const double sd = CP * Td + GRAV * zlow + phis;
                        ad = adn;
                        qd = s.qs;
                        zii = zlow;
                        // The fluxes at interface i, upwind in the net environmental flow.
                        const double et = v.et, ed = -adn;
                        SCR(D_ED, i) = ed;
                        const bool upw = et + alpha * ed >= 0.0;
                        const double s_up = upw ? CP * Tk + GRAV * zk + phis
                                                : CP * v.Tb + GRAV * v.zb + phis;
                        const double q_up = upw ? qk : v.qb;
                        Fs = et * (v.su - s_up) + alpha * ed * (sd - s_up);
                        Fq = et * (v.qu - q_up) + alpha * ed * (qd - q_up);
                        E1 += e1;
                    }
                    const double c = k == kd ? c_kd : v.c;
                    layer(dn, k, Fs_t, Fq_t, Fs, Fq, c - alpha * e1, Tk, qk, pt, v.pb);
                    Fs_t = Fs;
                    Fq_t = Fq;
                    Tk = v.Tb;
                    qk = v.qb;
                    zk = v.zb;
                    pt = v.pb;
                };
                FLev v0 = fload(kd), v1 = fload(kd + 1);
                for (int k = kd; k <= kb; k += 2) {
                    flevel(v0, k);
                    v0 = fload(k + 2);
                    if (k + 1 > kb) break;
                    flevel(v1, k + 1);
                    v1 = fload(k + 3);
                }
                // D6's strength: capped so that the downdraft evaporates at most the allowed
                // fraction of the updraft's condensation.
                if (pass > 0 || !(P.alpha_dd * E1 > P.evap_max_frac * C1)) break;
                alpha = P.evap_max_frac * C1 / E1;
            }
        }
        const double P1 = up.P1 + dn.P1, Fenv = up.Fenv + dn.Fenv, Mlim = fmin(up.Mlim, dn.Mlim);

        // D8: F from the launch-layer tendencies and the trigger's parcel sensitivities; D9, D10.
        // A dilute parcel is also moved by the air it entrained: its sensitivity is swept up from
        // the launch layer along the unit tendencies, the parcel recomputed on the way.
        double F = -RD * (dT1kb * SA + dq1kb * SB - Fenv);
        if (P.eps_cape > 0.0) {
            Hint hp;
            hp.clear();
            double hmix = (CP * AT(M.T, kb) + GRAV * AT(M.z, kb) + phis) + LV * AT(M.q, kb);
            double qmix = AT(M.q, kb);
            double dhm = CP * dT1kb + LV * dq1kb, dqm = dq1kb, Fsum = 0.0;
            double zb = AT(M.z, kb);
            // Layer k's state, unit tendencies and interface pressures, loaded one layer ahead
            // (levels clamped at kt: every load is in range, values past the top unused).
            struct XLev {
                double T, q, z, pm, dT1, dq1, pt, pb;
            };
            auto xload = [&](int k) {
                XLev v;
                const int kk = max(k, kt);
                v.T = AT(M.T, kk);
                v.q = AT(M.q, kk);
                v.z = AT(M.z, kk);
                v.pm = AT(M.pm, kk);
                v.dT1 = xget(0, kk);
                v.dq1 = xget(1, kk);
                v.pt = AT(M.pi, kk);
                v.pb = AT(M.pi, kk + 1);
                return v;
            };
            XLev nx = xload(kb - 1);
            for (int k = kb - 1; k >= kt; --k) {
                const XLev v = nx;
                nx = xload(k - 1);
                const double Tk = v.T, qk = v.q, zk = v.z, pm = v.pm;
                const double dT1 = v.dT1, dq1 = v.dq1;
                const double mix = P.eps_cape * (zk - zb);
                hmix = (hmix + mix * ((CP * Tk + GRAV * zk + phis) + LV * qk)) / (1.0 + mix);
                qmix = (qmix + mix * qk) / (1.0 + mix);
                dhm = (dhm + mix * (CP * dT1 + LV * dq1)) / (1.0 + mix);
                dqm = (dqm + mix * dq1) / (1.0 + mix);
                const Lifted r = lift(hmix - GRAV * zk - phis, qmix, pm, hp);
                double dTp, dqp;
                if (r.sat) {
                    const double Q1 = sat_eval(r.T, pm).dqs;  // qs' at the root itself
                    dTp = dhm / (CP + LV * Q1);
                    dqp = Q1 * dTp;
                } else {
                    dTp = (dhm - LV * dqm) * RCP_CP;
                    dqp = dqm;
                }
                const double dTvp = (1.0 + CVIR * r.qv) * dTp + CVIR * r.T * dqp;
                const double dTve = (1.0 + CVIR * qk) * dT1 + CVIR * Tk * dq1;
                Fsum += log(v.pb / v.pt) * (dTvp - dTve);
                zb = zk;
            }
            F = -RD * Fsum;
        }
        int st = 0;
        double Mb = 0.0;
        if (!(F > 0.0)) {
            st = 2;
        } else {
            const double Mc = cape / (P.tau * F);
            Mb = Mc <= Mlim ? Mc : Mlim;
        }
        if (st == 0) {  // the trigger pass zeroed the whole column
            // Layers kt..kb and interfaces kt+1..kb, OUTC levels at a time: the scratch loads of
            // a batch are issued together (levels clamped to kb, so every load is in range), then
            // the stores, instead of one load round trip per stored value.
            constexpr int OUTC = 8;
            const bool dd = kd >= 0;
            for (int k0 = kt; k0 <= kb; k0 += OUTC) {
                double a[OUTC], b[OUTC], e[OUTC], d[OUTC];
#pragma unroll
                for (int j = 0; j < OUTC; ++j) {
                    const int k = min(k0 + j, kb);
                    a[j] = xget(0, k);
                    b[j] = xget(1, k);
                    e[j] = SCR(U_ETA, max(k, kt + 1));
                    d[j] = SCR(D_ED, dd ? max(k, kd + 1) : k);
                }
#pragma unroll
                for (int j = 0; j < OUTC; ++j) {
                    const int k = k0 + j;
                    if (k > kb) break;
                    AT(M.dout.dTdt, k) = Mb * a[j];
                    AT(M.dout.dqdt, k) = Mb * b[j];
                    if (k >= kt + 1) AT(M.dout.mu, k) = Mb * e[j];
                    if (dd && k >= kd + 1) AT(M.dout.md, k) = Mb * (alpha * d[j]);
                }
            }
        }
        M.dout.prec[col] = st == 0 ? Mb * P1 : 0.0;
        M.dout.status[col] = st;

        int claim = 0;
        if (lane == 0) claim = atomicAdd(&w.cnt[CNT_DGRAB], WAVE);
        slot0 = first_round + __builtin_amdgcn_readfirstlane(claim);
    }
#undef SCR
}

// S7-S9 of one shallow column that passed S1-S6: the plume from the source interface ks with
// its closure inputs (from the trigger or the re-trigger), the tendencies and the limiter; writes
// the column's shallow outputs.  `upd`: the plume sees the deep-updated state T + dt*dTdt,
// q + dt*dqdt.  The per-level profiles go to the thread's scratch column `tid` of `stride`.
__device__ void shallow_plume_column(const Member &M, int64_t col, int ks, bool upd, double hs,
                                     double qsrc, double cin, double Mclos, double sigw2,
                                     double *scr, int64_t stride, int64_t tid, int lmax) {
    const int64_t ld = M.ld;
    const conv_params_t &P = M.P;
#define SCR(arr, lev) scr[((int64_t)(arr) * (lmax + 1) + (lev)) * stride + tid]
    const double phis = M.phis[col];
    auto Tn = [&](int k) { return upd ? AT(M.T, k) + M.dt * AT(M.dout.dTdt, k) : AT(M.T, k); };
    auto qn = [&](int k) { return upd ? AT(M.q, k) + M.dt * AT(M.dout.dqdt, k) : AT(M.q, k); };
    auto zi = [&](int i) { return 0.5 * (AT(M.z, i - 1) + AT(M.z, i)); };

    Hint hp;
    hp.clear();
    double Mlim = __builtin_inf();
    double P1;
    double Fs_lo, Fq_lo;  // fluxes at the interface below the current layer
    double eta = 1.0, hu = hs, qtu;
    // S7 start: thermodynamics at the source interface ks.
    {
        const double zs = zi(ks);
        const Lifted r = lift(hs - GRAV * zs - phis, qsrc, AT(M.pi, ks), hp);
        const double ql = qsrc - r.qv;
        const double rr = ql - P.qlcrit_sh > 0.0 ? ql - P.qlcrit_sh : 0.0;
        qtu = qsrc - rr;
        const double slu = CP * r.T + GRAV * zs + phis - LV * (ql - rr);
        const double s_up = CP * Tn(ks - 1) + GRAV * AT(M.z, ks - 1) + phis;
        const double Fs = slu - s_up, Fq = qtu - qn(ks - 1);
        const double dp = AT(M.pi, ks + 1) - AT(M.pi, ks);
        const double dT1 = (0.0 - Fs + LV * rr) * GRAV / (CP * dp);
        const double dq1 = (0.0 - Fq - rr) * GRAV / dp;
        SCR(0, ks) = 1.0;
        SCR(1, ks) = dT1;
        SCR(2, ks) = dq1;
        P1 = rr;
        if (dq1 < 0.0) Mlim = fmin(Mlim, qn(ks) / (-M.dt * dq1));
        Fs_lo = Fs;
        Fq_lo = Fq;
    }
    double w2 = sigw2 + 2.0 * P.a_buoy * cin;
    int kt = -1;
    double zlo = zi(ks);
    for (int k = ks - 1; k >= 0; --k) {
        bool stop = AT(M.pi, k) < P.p_sh_top_min || k == 0;
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
            hm = ((eta - D) * hu + E * ((CP * Tk + GRAV * AT(M.z, k) + phis) + LV * qk)) / en;
            const double qm = ((eta - D) * qtu + E * qk) / en;
            const Lifted r = lift(hm - GRAV * zk - phis, qm, AT(M.pi, k), hp);
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
                const double s_up = CP * Tn(k - 1) + GRAV * AT(M.z, k - 1) + phis;
                Fs = en * (slu - s_up);
                Fq = en * (qtn - qn(k - 1));
            }
        }
        const double pr = stop ? 0.0 : en * rr;
        const double dp = AT(M.pi, k + 1) - AT(M.pi, k);
        const double dT1 = (Fs_lo - Fs + LV * pr) * GRAV / (CP * dp);
        const double dq1 = (Fq_lo - Fq - pr) * GRAV / dp;
        SCR(1, k) = dT1;
        SCR(2, k) = dq1;
        P1 += pr;
        if (dq1 < 0.0) Mlim = fmin(Mlim, qn(k) / (-M.dt * dq1));
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
    if (st == 0) {  // the trigger pass zeroed the column; write the plume's levels
        // OUTC levels at a time, loads first (levels clamped to ks), as in the deep plume.
        constexpr int OUTC = 4;
        for (int k0 = kt; k0 <= ks; k0 += OUTC) {
            double a[OUTC], b[OUTC], e[OUTC];
#pragma unroll
            for (int j = 0; j < OUTC; ++j) {
                const int k = min(k0 + j, ks);
                a[j] = SCR(1, k);
                b[j] = SCR(2, k);
                e[j] = SCR(0, k);
            }
#pragma unroll
            for (int j = 0; j < OUTC; ++j) {
                const int k = k0 + j;
                if (k > ks) break;
                AT(M.sout.dTdt, k) = Mb * a[j];
                AT(M.sout.dqdt, k) = Mb * b[j];
                if (k >= kt + 1) AT(M.sout.mu, k) = Mb * e[j];
            }
        }
    }
    M.sout.prec[col] = st == 0 ? Mb * P1 : 0.0;
    M.sout.cin[col] = cin;
    M.sout.kbase[col] = ks;
    M.sout.ktop[col] = kt;
    M.sout.status[col] = st;
#undef SCR
}

// The shallow plume pass over the list the trigger filled (columns without deep convection).
template <class Src>
__global__ __launch_bounds__(WAVE) void k_shallow_plume(Src src, Work w) {
    const int n = w.cnt[CNT_SHALLOW];
    const int64_t gtid = (int64_t)blockIdx.x * WAVE + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * WAVE;
    for (int64_t slot = gtid; slot < n; slot += nthreads) {
        const Member M = src.at(w.smem[slot]);  // a copy: the fields stay in registers
        shallow_plume_column(M, w.slist[slot], w.sks[slot], w.sflag[slot] != 0, w.shs[slot],
                             w.sqs[slot], w.scin[slot], w.sMc[slot], w.ssig2[slot], w.sscr,
                             w.sstride, gtid, w.lmax);
    }
}

// The shallow scheme after the deep one: the shallow trigger (S1-S6) on the deep-updated state
// T' = T + dt*dTdt, q' = q + dt*dqdt of every column of the deep list, and the plume (S7-S9) of
// each column that passes it, in the same lane; then the plumes of the columns the trigger listed
// (no deep convection there).  Persistent over the deep list.  Its own kernel (not the tail of
// the deep plume pass) so that it runs at the occupancy its registers allow; the plumes run
// inline because most of the columns that pass S1-S6 after deep convection stop at their first
// level, which a separate pass would pay a list round trip and a launch for.  On one grid it is
// held to three wavefronts per SIMD (at most 168 registers, a few spilled; the inline plume wants
// more), the occupancy its launch of 12 wavefronts per CU needs.  An ensemble's lanes also hold
// their member's fields: there two wavefronts per SIMD without spills run faster (2.18 -> 2.13 ms
// per ensemble step; the single grid's re-trigger 0.077 -> 0.081 ms).
template <class Src>
struct RetriggerOccupancy {
    static constexpr int waves_per_simd = 3;
};
template <>
struct RetriggerOccupancy<Many> {
    static constexpr int waves_per_simd = 2;
};
template <class Src>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(RetriggerOccupancy<Src>::waves_per_simd)))
void k_shallow_retrigger(Src src, Work w) {
    const int n = w.cnt[CNT_DEEP];
    const int64_t gtid = (int64_t)blockIdx.x * WAVE + threadIdx.x;  // one wavefront per block
    const int64_t nthreads = (int64_t)gridDim.x * WAVE;
    const int64_t wave0 = gtid - (threadIdx.x % WAVE);
    for (int64_t base = wave0; base < n; base += nthreads) {
        const int64_t slot = base + (threadIdx.x % WAVE);
        const bool act = slot < n;
        const int mi = act ? w.dmem[slot] : 0;
        const Member M = src.at(mi);  // a copy: the fields stay in registers
        const int L = M.nlev;
        const int64_t ld = M.ld;
        const conv_params_t &P = M.P;
        const int64_t col = act ? w.dlist[slot] : 0;
        // Shallow trigger on the deep-updated state T' = T + dt*dTdt, q' = q + dt*dqdt.
        ShallowTrigger sh;
        sh.init(L);
        int sst = -1;
        double rho_s = 0.0, tke = 0.0;
        if (act) {
            const double phis = M.phis[col];
            const double pblh = M.pblh[col];
            tke = M.tke[col];
            // The deep outputs were zeroed outside the plume's levels, so the updated state is
            // T + dt*dTdt at every level (unconditional loads keep the wait counts exact).
            auto Tn = [&](int k) { return AT(M.T, k) + M.dt * AT(M.dout.dTdt, k); };
            auto qn = [&](int k) { return AT(M.q, k) + M.dt * AT(M.dout.dqdt, k); };
            if (isfinite(pblh) && isfinite(tke)) {
                constexpr int PBLC = 4;  // levels of the boundary-layer scan loaded at once
                double pbot = AT(M.pi, L);
                for (int k0 = L - 1; k0 >= 0 && (k0 == L - 1 || sh.inpbl); k0 -= PBLC) {
                    double pt[PBLC], z[PBLC], T[PBLC], q[PBLC];
#pragma unroll
                    for (int j = 0; j < PBLC; ++j) {
                        const int kk = max(k0 - j, 0);
                        pt[j] = AT(M.pi, kk);
                        z[j] = AT(M.z, kk);
                        T[j] = Tn(kk);
                        q[j] = qn(kk);
                    }
#pragma unroll
                    for (int j = 0; j < PBLC; ++j) {
                        const int k = k0 - j;
                        if (k < 0 || !(k == L - 1 || sh.inpbl)) break;
                        sh.pbl(k, L, z[j], pblh, (CP * T[j] + GRAV * z[j] + phis) + LV * q[j], q[j],
                               pbot - pt[j]);
                        pbot = pt[j];
                    }
                }
                sh.start();
                int k = sh.ks - 1;
                const int k0 = max(k, 0);
                double pmn = AT(M.pm, k0), zn = AT(M.z, k0), Tnn = Tn(k0), qnn = qn(k0),
                       ptn = AT(M.pi, k0), pbn = AT(M.pi, k0 + 1);
                for (; k >= 0; --k) {
                    const double pm = pmn, z = zn, Tk = Tnn, qk = qnn, pt = ptn, pb = pbn;
                    if (!sh.wants(k, pm, P)) break;
                    const int kn = max(k - 1, 0);
                    pmn = AT(M.pm, kn);
                    zn = AT(M.z, kn);
                    Tnn = Tn(kn);
                    qnn = qn(kn);
                    ptn = AT(M.pi, kn);
                    pbn = pt;
                    sh.level(k, z, phis, tv(Tk, qk), pm, log(pb / pt), P);
                }
                sst = sh.status(tke, P);
            } else {
                sst = 6;
            }
            if (sst < 0) {
                rho_s = AT(M.pi, sh.ks) / (RD * tv(Tn(sh.ks), qn(sh.ks)));
                const double sigw2 = P.c_tke * tke;
                shallow_plume_column(M, col, sh.ks, true, sh.hs, sh.qs, sh.cin,
                                     shallow_closure(M, sh, rho_s, sigw2), sigw2, w.sscr, nthreads,
                                     gtid, w.lmax);
            } else {
                write_shallow_quiet(M, col, sst, sh.cin, sh.ks);
            }
        }
    }
    const int ns = w.cnt[CNT_SHALLOW];
    for (int64_t slot = gtid; slot < ns; slot += nthreads) {
        const Member M = src.at(w.smem[slot]);
        shallow_plume_column(M, w.slist[slot], w.sks[slot], w.sflag[slot] != 0, w.shs[slot],
                             w.sqs[slot], w.scin[slot], w.sMc[slot], w.ssig2[slot], w.sscr,
                             nthreads, gtid, w.lmax);
    }
}


#undef AT

// ------------------------------------------------------------------ host side
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace layout for `ncol` columns (all members together) of at most `lmax` levels and `nmem`
// ensemble members.  `thread_cap` > 0 limits the persistent grids the plume scratch is sized for.
Layout make_layout(int64_t ncol, int lmax, int nmem, int cus, int64_t thread_cap = 0) {
    Layout l{};
    const int64_t n = ncol > 0 ? ncol : 1;
    const int64_t tiles = (n + BLOCK - 1) / BLOCK;
    const int64_t cap = (int64_t)cus * MAX_BPC;
    l.threads = (tiles < cap ? tiles : cap) * BLOCK;
    if (thread_cap > 0 && thread_cap < l.threads) l.threads = thread_cap;
    l.lmax = lmax;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    l.cnt = take(NCOUNTERS * sizeof(int));
    l.dlist = take(n * sizeof(int));
    l.dmem = take(n * sizeof(int));
    l.dkb = take(n * sizeof(int));
    l.dkt = take(n * sizeof(int));
    l.dkd = take(n * sizeof(int));
    l.dcape = take(n * sizeof(double));
    l.dSA = take(n * sizeof(double));
    l.dSB = take(n * sizeof(double));
    l.slist = take(n * sizeof(int));
    l.smem = take(n * sizeof(int));
    l.sks = take(n * sizeof(int));
    l.sflag = take(n * sizeof(int));
    l.shs = take(n * sizeof(double));
    l.sqs = take(n * sizeof(double));
    l.scin = take(n * sizeof(double));
    l.sMc = take(n * sizeof(double));
    l.ssig2 = take(n * sizeof(double));
    l.members = take((size_t)(nmem > 0 ? nmem : 1) * sizeof(Member));
    l.dscr = take((size_t)deep_scr_global(lmax) * (lmax + 1) * l.threads * sizeof(double));
    l.sscr = take((size_t)SHALLOW_SCR * (lmax + 1) * l.threads * sizeof(double));
    l.total = off;
    return l;
}

}  // namespace

namespace {

Work make_work(char *b, const Layout &l, const Launch &launch, int cus) {
    Work w;
    w.cnt = (int *)(b + l.cnt);
    w.dlist = (int *)(b + l.dlist);
    w.dmem = (int *)(b + l.dmem);
    w.dkb = (int *)(b + l.dkb);
    w.dkt = (int *)(b + l.dkt);
    w.dkd = (int *)(b + l.dkd);
    w.dcape = (double *)(b + l.dcape);
    w.dSA = (double *)(b + l.dSA);
    w.dSB = (double *)(b + l.dSB);
    w.slist = (int *)(b + l.slist);
    w.smem = (int *)(b + l.smem);
    w.sks = (int *)(b + l.sks);
    w.sflag = (int *)(b + l.sflag);
    w.shs = (double *)(b + l.shs);
    w.sqs = (double *)(b + l.sqs);
    w.scin = (double *)(b + l.scin);
    w.sMc = (double *)(b + l.sMc);
    w.ssig2 = (double *)(b + l.ssig2);
    w.dscr = (double *)(b + l.dscr);
    w.sscr = (double *)(b + l.sscr);
    const int64_t fd = (int64_t)cus * launch.fused_wpc * WAVE;
    const int64_t sh = (int64_t)cus * launch.shallow_wpc * WAVE;
    w.dstride = fd < l.threads ? fd : l.threads;
    w.sstride = sh < l.threads ? sh : l.threads;
    const int64_t rt = (int64_t)cus * RETRIGGER_BPC * BLOCK;
    w.rstride = rt < l.threads ? rt : l.threads;
    w.lmax = l.lmax;
    w.cus = cus;
    return w;
}

bool state_ok(int64_t ncol, const conv_state_t *s, bool shallow) {
    if (!s || !s->T || !s->q || !s->p_mid || !s->z || !s->p_int || !s->phis) return false;
    if (shallow && (!s->pblh || !s->tke)) return false;
    if (s->ld < ncol || !(s->dt > 0.0)) return false;
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

int finish() { return check_launch(); }

// The step's launches on `st`; `ev` (CONV_NSTAGES+1 events, may be null) brackets each stage.
template <class Src, bool DEEP, bool SHALLOW>
int launch_step(const Src &src, const Work &w, hipStream_t st, hipEvent_t *ev) {
    const unsigned gt = (unsigned)src.ntiles;
    // The plume passes run one wavefront per block: a short list then spreads over as many
    // compute units as it has wavefronts instead of filling a few (the wavefronts of one CU share
    // its load pipeline and L1).
    const unsigned gd = (unsigned)(w.dstride / WAVE);
    const unsigned gs = (unsigned)(w.sstride / WAVE);
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(NCOUNTERS), 0, st, w.cnt);
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL((k_trigger<Src, DEEP, SHALLOW>), dim3(gt), dim3(BLOCK), 0, st, src, w);
    if (ev) (void)hipEventRecord(ev[2], st);
    if (DEEP) {
        if (deep_xg(w.lmax))
            hipLaunchKernelGGL((k_deep_plume<Src, true>), dim3(gd), dim3(WAVE), DEEP_X_LDS, st, src, w);
        else
            hipLaunchKernelGGL((k_deep_plume<Src, false>), dim3(gd), dim3(WAVE), DEEP_X_LDS, st, src,
                               w);
    }
    if (ev) (void)hipEventRecord(ev[3], st);
    if (DEEP && SHALLOW) {
        // one-wavefront blocks, RETRIGGER_BPC x 256 threads per CU (78 -> 69 us against
        // 256-thread blocks on the 884,736-column grid); the shallow plumes run inside
        const unsigned gr = (unsigned)(w.rstride / WAVE);
        hipLaunchKernelGGL((k_shallow_retrigger<Src>), dim3(gr), dim3(WAVE), 0, st, src, w);
    }
    if (ev) (void)hipEventRecord(ev[4], st);
    if (SHALLOW && !DEEP)
        hipLaunchKernelGGL((k_shallow_plume<Src>), dim3(gs), dim3(WAVE), 0, st, src, w);
    if (ev) (void)hipEventRecord(ev[5], st);
    return finish();
}

template <bool DEEP, bool SHALLOW>
int run_one(conv_ctx *c, const conv_state_t *s, const conv_deep_out_t *d,
            const conv_shallow_out_t *sh, hipStream_t st) {
    One src;
    src.m = make_member(c->ncol, c->nlev, c->P, s, d, sh, 0);
    src.ntiles = (c->ncol + BLOCK - 1) / BLOCK;
    const Work w = make_work(c->ws, c->lay, c->launch, c->cus);
    hipEvent_t *ev = nullptr;
    if (c->ev && c->ev_used < c->ev_cap) ev = c->ev + (size_t)(c->ev_used++) * (CONV_NSTAGES + 1);
    return launch_step<One, DEEP, SHALLOW>(src, w, st, ev);
}

// ------------------------------------------------------------------ launch-shape autotuner
// Candidate persistent-grid sizes (wavefronts per compute unit) for the deep-plume and
// shallow-plume kernels; the trigger launch is one block per tile and has no shape to tune.  The
// deep plume's candidates are fine around one and two wavefronts per SIMD: its end is set by how
// many 64-column passes its busiest wavefronts take (on the 884,736-column grid, 5 per CU:
// 0.255 -> 0.233 ms against 4).
// Deep-plume shapes the autotuners try (its LDS leaves room for five resident wavefronts per CU;
// a larger grid queues blocks, which helped the ensemble a little); the step does not launch the
// shallow plume kernel (its re-trigger runs the shallow plumes), whose shape keeps its default.
constexpr int TUNE_FUSED[] = {4, 5, 6, 8};
constexpr int NTUNE = sizeof(TUNE_FUSED) / sizeof(TUNE_FUSED[0]);

struct TuneResult {
    Launch launch;
    float ms;
};

std::mutex g_tune_mu;
std::map<std::string, TuneResult> g_tune_cache;  // per process, keyed by device and shapes

// Times `run(shape)` (which enqueues one step on `st`) for every candidate shape: one untimed
// call, then `reps` calls each bracketed by events; the score is the median, the lower of two
// sweeps (the first can run while the clocks still rise).  Waits on the host.
template <class Run>
int tune(hipStream_t st, int reps, Run run, TuneResult *best) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        g_last_hip = (int)hipGetLastError();
        return CONV_EHIP;
    }
    std::vector<float> t((size_t)reps);
    float score[NTUNE];
    for (float &x : score) x = __builtin_inff();
    auto body = [&]() -> int {
        for (int sweep = 0; sweep < 2; ++sweep) {
            for (int i = 0; i < NTUNE; ++i) {
                const Launch L{TUNE_FUSED[i], DEFAULT_LAUNCH.shallow_wpc};
                int rc = run(L);
                if (rc != CONV_OK) return rc;
                for (int r = 0; r < reps; ++r) {
                    if (hipEventRecord(e0, st) != hipSuccess) return CONV_EHIP;
                    rc = run(L);
                    if (rc != CONV_OK) return rc;
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t[(size_t)r], e0, e1) != hipSuccess)
                        return CONV_EHIP;
                }
                std::sort(t.begin(), t.end());
                const float med = t[(size_t)reps / 2];
                if (med < score[i]) score[i] = med;
            }
        }
        return CONV_OK;
    };
    const int rc = body();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == CONV_EHIP) g_last_hip = (int)hipGetLastError();
    if (rc == CONV_OK) {
        TuneResult b{DEFAULT_LAUNCH, __builtin_inff()};
        for (int i = 0; i < NTUNE; ++i)
            if (score[i] < b.ms)
                b = TuneResult{Launch{TUNE_FUSED[i], DEFAULT_LAUNCH.shallow_wpc}, score[i]};
        *best = b;
    }
    return rc;
}

std::string tune_key(const char *kind, int cus, const std::vector<std::pair<int64_t, int>> &shapes) {
    int dev = -1;
    (void)hipGetDevice(&dev);
    std::string k = std::string(kind) + ":" + std::to_string(dev) + ":" + std::to_string(cus);
    for (const auto &p : shapes) k += ":" + std::to_string(p.first) + "x" + std::to_string(p.second);
    return k;
}

// Cached or freshly tuned shape for `key`.
template <class Run>
int tune_cached(const std::string &key, int force, hipStream_t st, int reps, Run run, TuneResult *out) {
    if (!force) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second;
            return CONV_OK;
        }
    }
    TuneResult r;
    const int rc = tune(st, reps, run, &r);
    if (rc != CONV_OK) return rc;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = r;
    }
    *out = r;
    return CONV_OK;
}

void free_events(conv_ctx *c) {
    if (c->ev) {
        for (int i = 0; i < c->ev_cap * (CONV_NSTAGES + 1); ++i) (void)hipEventDestroy(c->ev[i]);
        delete[] c->ev;
    }
    c->ev = nullptr;
    c->ev_cap = c->ev_used = 0;
}

}  // namespace

// An ensemble: several grids (members) with their own column and level counts, parameters and
// arrays, stepped by the same launches.  The member table lives in the workspace.
struct conv_ens {
    int nm;
    int64_t ncol;  // all members
    int64_t ntiles;
    int lmax;
    char *ws;
    size_t ws_bytes;
    cvk::Layout lay;
    cvk::Launch launch;
    int cus;
    std::vector<std::pair<int64_t, int>> shapes;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

bool member_ok(const conv_member_t &m) {
    if (m.ncol < 0 || m.ncol > INT32_MAX || m.nlev < 2 || m.nlev > 256) return false;
    if (m.ncol == 0) return true;
    return state_ok(m.ncol, &m.state, true) && deep_ok(&m.deep) && shallow_ok(&m.shallow);
}

// Totals of a member list; false if any member is malformed or the total is too large.
bool ens_totals(int n, const conv_member_t *ms, int64_t *ncol, int64_t *ntiles, int *lmax) {
    if (n < 1 || n > 4096 || !ms) return false;
    int64_t c = 0, t = 0;
    int l = 2;
    for (int i = 0; i < n; ++i) {
        if (!member_ok(ms[i])) return false;
        c += ms[i].ncol;
        t += (ms[i].ncol + BLOCK - 1) / BLOCK;
        l = ms[i].nlev > l ? ms[i].nlev : l;
    }
    if (c > INT32_MAX) return false;
    *ncol = c;
    *ntiles = t;
    *lmax = l;
    return true;
}

int ens_launch(const conv_ens *e, const Launch &launch, hipStream_t st) {
    if (e->ntiles == 0) return CONV_OK;
    Many src;
    src.ms = (const Member *)(e->ws + e->lay.members);
    src.nm = e->nm;
    src.ntiles = e->ntiles;
    const Work w = make_work(e->ws, e->lay, launch, e->cus);
    return launch_step<Many, true, true>(src, w, st, nullptr);
}

void ens_drop_graph(conv_ens *e) {
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->exec = nullptr;
    e->graph = nullptr;
}

int hip_fail() {
    g_last_hip = (int)hipGetLastError();
    return CONV_EHIP;
}

}  // namespace

extern "C" {

size_t conv_workspace_bytes(int64_t ncol, int32_t nlev) {
    if (ncol < 0 || ncol > INT32_MAX || nlev < 2 || nlev > 256) return 0;
    return make_layout(ncol, nlev, 1, device_cus()).total;
}

int conv_create(int64_t ncol, int32_t nlev, const conv_params_t *params, void *workspace,
                size_t ws_bytes, conv_ctx_t **out) {
    // Argument checks come first and make no HIP call.
    if (!out || !params || !workspace || ncol < 0 || ncol > INT32_MAX || nlev < 2 || nlev > 256)
        return CONV_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return CONV_EINVAL;
    const int cus = device_cus();
    const Layout l = make_layout(ncol, nlev, 1, cus);
    if (ws_bytes < l.total) return CONV_EINVAL;
    conv_ctx *c = new conv_ctx;
    c->ncol = ncol;
    c->nlev = nlev;
    c->P = *params;
    c->ws = (char *)workspace;
    c->ws_bytes = ws_bytes;
    c->lay = l;
    c->launch = DEFAULT_LAUNCH;
    c->cus = cus;
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

int conv_set_launch(conv_ctx_t *ctx, int fused_waves_per_cu, int shallow_waves_per_cu) {
    if (!ctx || fused_waves_per_cu < 1 || fused_waves_per_cu > MAX_WPC ||
        shallow_waves_per_cu < 1 || shallow_waves_per_cu > MAX_WPC)
        return CONV_EINVAL;
    ctx->launch = Launch{fused_waves_per_cu, shallow_waves_per_cu};
    return CONV_OK;
}

int conv_get_launch(conv_ctx_t *ctx, int *fused_waves_per_cu, int *shallow_waves_per_cu) {
    if (!ctx || !fused_waves_per_cu || !shallow_waves_per_cu) return CONV_EINVAL;
    *fused_waves_per_cu = ctx->launch.fused_wpc;
    *shallow_waves_per_cu = ctx->launch.shallow_wpc;
    return CONV_OK;
}

void conv_destroy(conv_ctx_t *ctx) {
    if (!ctx) return;
    free_events(ctx);
    delete ctx;
}

int conv_deep_forward(conv_ctx_t *ctx, const conv_state_t *state, conv_deep_out_t *out,
                      void *stream) {
    if (!ctx || !state || !out) return CONV_EINVAL;
    if (ctx->ncol == 0) return CONV_OK;  // nothing to read or write: the arrays may be NULL
    if (!state_ok(ctx->ncol, state, false) || !deep_ok(out)) return CONV_EINVAL;
    return run_one<true, false>(ctx, state, out, nullptr, (hipStream_t)stream);
}

int conv_shallow_forward(conv_ctx_t *ctx, const conv_state_t *state, conv_shallow_out_t *out,
                         void *stream) {
    if (!ctx || !state || !out) return CONV_EINVAL;
    if (ctx->ncol == 0) return CONV_OK;
    if (!state_ok(ctx->ncol, state, true) || !shallow_ok(out)) return CONV_EINVAL;
    return run_one<false, true>(ctx, state, nullptr, out, (hipStream_t)stream);
}

int conv_step(conv_ctx_t *ctx, const conv_state_t *state, conv_deep_out_t *deep,
              conv_shallow_out_t *shallow, void *stream) {
    if (!ctx || !state || !deep || !shallow) return CONV_EINVAL;
    if (ctx->ncol == 0) return CONV_OK;
    if (!state_ok(ctx->ncol, state, true) || !deep_ok(deep) || !shallow_ok(shallow))
        return CONV_EINVAL;
    return run_one<true, true>(ctx, state, deep, shallow, (hipStream_t)stream);
}

// ------------------------------------------------------------------ conv_step_static
// The workspace of conv_step_static: a static device array, one per GPU, held until the process
// ends.  Host code never uses its name as an address (the name is a host-side stand-in): the
// device address is looked up once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
static __device__ __align__(256) char scratch[CONV_STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's `scratch` (looked up on the first call on a device).
int static_scratch(char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail();
    if (dev < 0 || dev >= MAX_DEVICES) return CONV_EUNSUPPORTED;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_last_hip = (int)(e != hipSuccess ? e : hipErrorInvalidSymbol);
            (void)hipGetLastError();
            return CONV_EHIP;
        }
        g_scratch_ptr[dev] = (char *)p;
    }
    *out = g_scratch_ptr[dev];
    return CONV_OK;
}
}  // namespace

int conv_step_static(int64_t ncol, int32_t nlev, const conv_params_t *params,
                     const conv_state_t *state, conv_deep_out_t *deep,
                     conv_shallow_out_t *shallow, void *stream) {
    if (!params || !state || !deep || !shallow || ncol < 0 || ncol > INT32_MAX || nlev < 2 ||
        nlev > 256)
        return CONV_EINVAL;
    if (ncol == 0) return CONV_OK;
    if (!state_ok(ncol, state, true) || !deep_ok(deep) || !shallow_ok(shallow)) return CONV_EINVAL;
    // The widest plume grids (5, 4, ... 1 wavefronts per CU) whose workspace fits the array.
    const int cus = device_cus();
    Layout l{};
    int wpc = DEFAULT_LAUNCH.fused_wpc;
    for (; wpc >= 1; --wpc) {
        l = make_layout(ncol, nlev, 1, cus, (int64_t)cus * wpc * WAVE);
        if (l.total <= CONV_STATIC_SCRATCH_BYTES) break;
    }
    if (wpc < 1) return CONV_ERANGE;
    char *ws = nullptr;
    const int rc = static_scratch(&ws);
    if (rc != CONV_OK) return rc;
    One src;
    src.m = make_member(ncol, nlev, *params, state, deep, shallow, 0);
    src.ntiles = (ncol + BLOCK - 1) / BLOCK;
    const Work w = make_work(ws, l, Launch{wpc, wpc}, cus);
    return launch_step<One, true, true>(src, w, (hipStream_t)stream, nullptr);
}

int conv_timing_start(conv_ctx_t *ctx, int max_calls) {
    if (!ctx || max_calls < 0) return CONV_EINVAL;
    free_events(ctx);
    if (max_calls == 0) return CONV_OK;
    ctx->ev = new hipEvent_t[(size_t)max_calls * (CONV_NSTAGES + 1)];
    for (int i = 0; i < max_calls * (CONV_NSTAGES + 1); ++i) {
        if (hipEventCreate(&ctx->ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(ctx->ev[j]);
            delete[] ctx->ev;
            ctx->ev = nullptr;
            return CONV_EHIP;
        }
    }
    ctx->ev_cap = max_calls;
    ctx->ev_used = 0;
    return CONV_OK;
}

int conv_timing_read(conv_ctx_t *ctx, double *ms, int *ncalls) {
    if (!ctx || !ms || !ncalls) return CONV_EINVAL;
    for (int s = 0; s < CONV_NSTAGES; ++s) ms[s] = 0.0;
    *ncalls = ctx->ev_used;
    for (int i = 0; i < ctx->ev_used; ++i) {
        hipEvent_t *ev = ctx->ev + (size_t)i * (CONV_NSTAGES + 1);
        if (hipEventSynchronize(ev[CONV_NSTAGES]) != hipSuccess) return CONV_EHIP;
        for (int s = 0; s < CONV_NSTAGES; ++s) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[s], ev[s + 1]) != hipSuccess) return CONV_EHIP;
            ms[s] += t;
        }
    }
    return CONV_OK;
}

const char *conv_strerror(int code) {
    switch (code) {
        case CONV_OK: return "ok";
        case CONV_EINVAL: return "invalid argument";
        case CONV_EUNSUPPORTED: return "unsupported";
        case CONV_EHIP: return "HIP launch failure";
        case CONV_ERANGE: return "size beyond the static scratch of conv_step_static";
        default: return "unknown error";
    }
}

int conv_last_hip_error(void) { return g_last_hip; }

int conv_autotune(conv_ctx_t *ctx, const conv_state_t *state, conv_deep_out_t *deep,
                  conv_shallow_out_t *shallow, void *stream, int reps, int force,
                  int *fused_waves_per_cu, int *shallow_waves_per_cu, float *ms) {
    if (!ctx || !state_ok(ctx->ncol, state, true) || !deep_ok(deep) || !shallow_ok(shallow) ||
        reps < 1 || reps > 1000)
        return CONV_EINVAL;
    if (ctx->ncol == 0) return CONV_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    auto run = [&](const Launch &L) {
        One src;
        src.m = make_member(ctx->ncol, ctx->nlev, ctx->P, state, deep, shallow, 0);
        src.ntiles = (ctx->ncol + BLOCK - 1) / BLOCK;
        return launch_step<One, true, true>(src, make_work(ctx->ws, ctx->lay, L, ctx->cus), st,
                                            nullptr);
    };
    TuneResult r;
    const int rc = tune_cached(tune_key("step", ctx->cus, {{ctx->ncol, ctx->nlev}}), force, st, reps,
                               run, &r);
    if (rc != CONV_OK) return rc;
    ctx->launch = r.launch;
    if (fused_waves_per_cu) *fused_waves_per_cu = r.launch.fused_wpc;
    if (shallow_waves_per_cu) *shallow_waves_per_cu = r.launch.shallow_wpc;
    if (ms) *ms = r.ms;
    return CONV_OK;
}

size_t conv_ensemble_workspace_bytes(int n_members, const conv_member_t *members) {
    int64_t ncol, ntiles;
    int lmax;
    if (!ens_totals(n_members, members, &ncol, &ntiles, &lmax)) return 0;
    return make_layout(ncol, lmax, n_members, device_cus()).total;
}

int conv_ensemble_create(int n_members, const conv_member_t *members, void *workspace,
                         size_t ws_bytes, conv_ens_t **out) {
    int64_t ncol, ntiles;
    int lmax;
    if (!out || !workspace || !ens_totals(n_members, members, &ncol, &ntiles, &lmax))
        return CONV_EINVAL;
    if (((uintptr_t)workspace & 255u) != 0) return CONV_EINVAL;
    const int cus = device_cus();
    const Layout l = make_layout(ncol, lmax, n_members, cus);
    if (ws_bytes < l.total) return CONV_EINVAL;
    // Tiles go to the members with the most levels first: their columns then enter the active
    // lists first, and the plume passes, which claim the lists in order, start on the longest
    // plumes and end on short ones (largest jobs first) instead of finishing on a deep member.
    // The table order is internal: every member's results go to its own arrays.
    std::vector<int> order((size_t)n_members);
    for (int i = 0; i < n_members; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return members[a].nlev > members[b].nlev; });
    std::vector<Member> tab((size_t)n_members);
    int64_t tile0 = 0;
    for (int j = 0; j < n_members; ++j) {
        const conv_member_t &m = members[order[(size_t)j]];
        tab[(size_t)j] = make_member(m.ncol, m.nlev, m.params, &m.state, &m.deep, &m.shallow, tile0);
        tile0 += (m.ncol + BLOCK - 1) / BLOCK;
    }
    if (hipMemcpy((char *)workspace + l.members, tab.data(), tab.size() * sizeof(Member),
                  hipMemcpyHostToDevice) != hipSuccess)
        return hip_fail();
    conv_ens *e = new conv_ens;
    e->nm = n_members;
    e->ncol = ncol;
    e->ntiles = ntiles;
    e->lmax = lmax;
    e->ws = (char *)workspace;
    e->ws_bytes = ws_bytes;
    e->lay = l;
    e->launch = DEFAULT_LAUNCH;
    e->cus = cus;
    for (int i = 0; i < n_members; ++i) e->shapes.emplace_back(members[i].ncol, members[i].nlev);
    e->graph = nullptr;
    e->exec = nullptr;
    *out = e;
    return CONV_OK;
}

void conv_ensemble_destroy(conv_ens_t *e) {
    if (!e) return;
    ens_drop_graph(e);
    delete e;
}

int conv_ensemble_step(conv_ens_t *e, void *stream) {
    if (!e) return CONV_EINVAL;
    return ens_launch(e, e->launch, (hipStream_t)stream);
}

int conv_ensemble_set_launch(conv_ens_t *e, int fused_waves_per_cu, int shallow_waves_per_cu) {
    if (!e || fused_waves_per_cu < 1 || fused_waves_per_cu > MAX_WPC || shallow_waves_per_cu < 1 ||
        shallow_waves_per_cu > MAX_WPC)
        return CONV_EINVAL;
    e->launch = Launch{fused_waves_per_cu, shallow_waves_per_cu};
    ens_drop_graph(e);
    return CONV_OK;
}

int conv_ensemble_get_launch(conv_ens_t *e, int *fused_waves_per_cu, int *shallow_waves_per_cu) {
    if (!e || !fused_waves_per_cu || !shallow_waves_per_cu) return CONV_EINVAL;
    *fused_waves_per_cu = e->launch.fused_wpc;
    *shallow_waves_per_cu = e->launch.shallow_wpc;
    return CONV_OK;
}

int conv_ensemble_autotune(conv_ens_t *e, void *stream, int reps, int force,
                           int *fused_waves_per_cu, int *shallow_waves_per_cu, float *ms) {
    if (!e || reps < 1 || reps > 1000 || e->ntiles == 0) return CONV_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    auto run = [&](const Launch &L) { return ens_launch(e, L, st); };
    TuneResult r;
    const int rc = tune_cached(tune_key("ensemble", e->cus, e->shapes), force, st, reps, run, &r);
    if (rc != CONV_OK) return rc;
    if (r.launch.fused_wpc != e->launch.fused_wpc || r.launch.shallow_wpc != e->launch.shallow_wpc)
        ens_drop_graph(e);
    e->launch = r.launch;
    if (fused_waves_per_cu) *fused_waves_per_cu = r.launch.fused_wpc;
    if (shallow_waves_per_cu) *shallow_waves_per_cu = r.launch.shallow_wpc;
    if (ms) *ms = r.ms;
    return CONV_OK;
}

int conv_ensemble_capture(conv_ens_t *e, void *stream) {
    if (!e || !stream) return CONV_EINVAL;
    ens_drop_graph(e);
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return hip_fail();
    const int rc = ens_launch(e, e->launch, st);
    hipGraph_t g = nullptr;
    const hipError_t end = hipStreamEndCapture(st, &g);
    if (rc != CONV_OK || end != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc != CONV_OK ? rc : hip_fail();
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail();
    }
    e->graph = g;
    e->exec = x;
    return CONV_OK;
}

int conv_ensemble_replay(conv_ens_t *e, void *stream) {
    if (!e || !e->exec) return CONV_EINVAL;
    if (hipGraphLaunch(e->exec, (hipStream_t)stream) != hipSuccess) return hip_fail();
    return CONV_OK;
}

}  // extern "C"
