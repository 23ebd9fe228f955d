// conv_tracers.hip -- convective transport of passive tracers by the plumes of one step (the
// convection schemes the paper accelerates move heat and water; the same mass fluxes move every
// other constituent), and convective momentum transport: the wind components carried the same way
// plus the pressure-gradient term of Gregory, Kershaw & Inness (1997), which pulls a plume's wind
// towards the environment's as it crosses shear (coefficient c_pgf; 0 = a passive tracer).
//
// A tracer is mixed by the plumes exactly as moist static energy is (D5-D7 deep, S7-S8 shallow):
// the deep updraft starts from the launch layer's air and entrains layer k's air between
// interfaces k+1 and k; the downdraft starts from layer k_d's air and entrains on its way down; the
// shallow updraft starts from the source layers' pressure-weighted mean, entrains and detrains at
// its rates eps_sh, delta_sh.  Tendencies are the flux divergences of the plume-minus-environment
// fluxes with the schemes' upwind environment values.  Everything comes from the step's outputs:
// the deep mass fluxes mu, md (their differences are the entrained mass), the shallow mu (with the
// mixing rates), the status and index outputs; the plumes are not run again.  The shallow scheme
// transports the tracer already updated by the deep transport (Algorithm 1 order).
//
// One wavefront per block, one lane per column, two tracers per wavefront (one where the LDS of two
// would pass 64 KiB, nlev > 64): the plumes' mass fluxes, pressures and indices are then loaded
// once for both, and each load batch carries both tracers' values (8 tracers on the
// 884,736-column grid: 0.537 -> 0.495 ms; u and v: 0.120 -> 0.114 ms).  Block b takes tracer
// pair b % npairs of column block b / npairs, so the tracers of one column block are dispatched
// together, and the slow convecting blocks spread over the run instead of piling up at its end.
// The tendencies are written once and not read again here: non-temporal stores (0.58 -> 0.52 ms
// for 8 tracers on the 884,736-column grid).  A lane accumulates its column's tendencies in LDS
// ([tracer][level][lane]); then the wavefront stores level by level with every lane active, so
// each store covers whole 128-byte lines (stores that cover only part of a line, as a wavefront
// mixing quiet and convecting columns would issue, run at a fraction of the bandwidth on this
// part).  Quiet columns contribute zeros.
#include <cmath>
#include <mutex>
#include <set>

#include "conv_internal.hpp"

using namespace cvk;

namespace {

constexpr int TW = WAVE;  // threads per block
constexpr int TB = 8;     // levels whose loads are issued together in the plume sweeps

struct TrArgs {
    Member M;          // state, both schemes' outputs and parameters of the step
    double pgf;        // pressure-gradient coefficient (0 for passive tracers)
    int ntr;
    const double *C;   // tracers [ntr][nlev][ld]
    double *tend;      // deep + shallow tendency [ntr][nlev][ld]
    double *dtend;     // deep tendency alone (may be NULL)
};

// TPW tracers per wavefront (tracers t0 .. t0 + nt - 1; with nt < TPW the missing ones repeat the
// last, which is computed again but not stored).
template <int TPW>
__global__ __launch_bounds__(TW) void k_tracers(TrArgs a) {
    extern __shared__ double sh[];  // [TPW][nlev][TW]
    const Member &M = a.M;
    const int lane = threadIdx.x;
    const int ngr = (a.ntr + TPW - 1) / TPW;
    const int t0 = (int)(blockIdx.x % (unsigned)ngr) * TPW;
    const int nt = min(TPW, a.ntr - t0);  // tracers of this block (a missing one repeats the last)
    const int64_t col = (int64_t)(blockIdx.x / (unsigned)ngr) * TW + lane;
    const bool live = col < M.ncol;
    const int64_t ld = M.ld;
    const int L = M.nlev;
    const int64_t plane = (int64_t)L * ld;
    const conv_params_t &P = M.P;
    const double *C[TPW];
    double *out[TPW];
    double *dout[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
        const int tj = t0 + min(j, nt - 1);
        C[j] = a.C + (int64_t)tj * plane;
        out[j] = a.tend + (int64_t)tj * plane;
        dout[j] = a.dtend ? a.dtend + (int64_t)tj * plane : nullptr;
    }
#define SH(j, k) sh[((j) * L + (k)) * TW + lane]

    bool deep = false, shal = false;
    int kb = 0, kt = 0, ks = 0, kts = 0;
    if (live) {
        kb = M.dout.klaunch[col];
        kt = M.dout.ktop[col];
        ks = M.sout.kbase[col];
        kts = M.sout.ktop[col];
        deep = M.dout.status[col] == 0 && kb >= 1 && kb < L && kt >= 0 && kt < kb &&
               AT(M.dout.mu, kb) > 0.0;
        shal = M.sout.status[col] == 0 && ks >= 1 && ks < L && kts >= 0 && kts < ks - 1 &&
               AT(M.sout.mu, ks) > 0.0;
    }
    auto dp = [&](int k) { return AT(M.pi, k + 1) - AT(M.pi, k); };

    if (__ballot(deep || shal) == 0ull) {
        if (live) {
#pragma unroll
            for (int j = 0; j < TPW; ++j) {
                if (j >= nt) break;
                for (int k = 0; k < L; ++k) {
                    __builtin_nontemporal_store(0.0, &AT(out[j], k));
                    if (dout[j]) __builtin_nontemporal_store(0.0, &AT(dout[j], k));
                }
            }
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < TPW; ++j)
        for (int k = 0; k < L; ++k) SH(j, k) = 0.0;

    const bool pgf = a.pgf != 0.0;
    if (deep) {
        double Cu[TPW], Fb[TPW], Cbel[TPW], mu1 = 0.0;
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            Cu[j] = AT(C[j], kb);
            Fb[j] = 0.0;
            Cbel[j] = 0.0;
        }
        int i0 = kb + 1;
        for (int b = kb; b >= kt + 1; b -= TB) {
            double mu[TB], md[TB], Ci[TPW][TB + 1], pt[TB + 1];
#pragma unroll
            for (int jj = 0; jj <= TB; ++jj) {
                const int i = max(b - jj, kt);
#pragma unroll
                for (int j = 0; j < TPW; ++j) Ci[j][jj] = AT(C[j], i);
                pt[jj] = AT(M.pi, i);
            }
            const double pbot0 = AT(M.pi, b + 1);
#pragma unroll
            for (int jj = 0; jj < TB; ++jj) {
                const int i = max(b - jj, kt + 1);
                mu[jj] = AT(M.dout.mu, i);
                md[jj] = AT(M.dout.md, i);
            }
#pragma unroll
            for (int jj = 0; jj < TB; ++jj) {
                const int i = b - jj;
                if (i < kt + 1) break;
                if (md[jj] != 0.0) i0 = i;
                const double pbot = jj == 0 ? pbot0 : pt[jj - 1];
                const bool upw = mu[jj] + md[jj] >= 0.0;
#pragma unroll
                for (int j = 0; j < TPW; ++j) {
                    if (i < kb) {
                        double num = mu1 * Cu[j] + (mu[jj] - mu1) * Ci[j][jj];
                        if (pgf) num += a.pgf * mu1 * (Ci[j][jj] - Cbel[j]);
                        Cu[j] = num / mu[jj];
                    }
                    Cbel[j] = Ci[j][jj];
                    const double F = mu[jj] * (Cu[j] - (upw ? Ci[j][jj + 1] : Ci[j][jj]));
                    SH(j, i) = (Fb[j] - F) * GRAV / (pbot - pt[jj]);
                    Fb[j] = F;
                }
                mu1 = mu[jj];
            }
        }
#pragma unroll
        for (int j = 0; j < TPW; ++j) SH(j, kt) = Fb[j] * GRAV / dp(kt);
        if (i0 <= kb) {
            double Cd[TPW], Cabv[TPW], ad1 = 0.0;
#pragma unroll
            for (int j = 0; j < TPW; ++j) {
                Cd[j] = AT(C[j], i0 - 1);
                Cabv[j] = 0.0;
            }
            for (int b = i0; b <= kb; b += TB) {
                double mu[TB], md[TB], Cl[TPW][TB + 1], pl[TB + 2];
#pragma unroll
                for (int jj = 0; jj < TB; ++jj) {
                    const int i = min(b + jj, kb);
                    mu[jj] = AT(M.dout.mu, i);
                    md[jj] = AT(M.dout.md, i);
                }
#pragma unroll
                for (int jj = 0; jj <= TB; ++jj)
#pragma unroll
                    for (int j = 0; j < TPW; ++j) Cl[j][jj] = AT(C[j], min(b - 1 + jj, kb));
#pragma unroll
                for (int jj = 0; jj <= TB + 1; ++jj) pl[jj] = AT(M.pi, min(b - 1 + jj, kb + 1));
#pragma unroll
                for (int jj = 0; jj < TB; ++jj) {
                    const int i = b + jj;
                    if (i > kb) break;
                    const double ad = -md[jj];
                    const bool upw = mu[jj] + md[jj] >= 0.0;
#pragma unroll
                    for (int j = 0; j < TPW; ++j) {
                        if (i > i0) {
                            double num = ad1 * Cd[j] + (ad - ad1) * Cl[j][jj];
                            if (pgf) num += a.pgf * ad1 * (Cl[j][jj] - Cabv[j]);
                            Cd[j] = num / ad;
                        }
                        Cabv[j] = Cl[j][jj];
                        const double F = md[jj] * (Cd[j] - (upw ? Cl[j][jj] : Cl[j][jj + 1]));
                        SH(j, i - 1) += F * GRAV / (pl[jj + 1] - pl[jj]);
                        SH(j, i) -= F * GRAV / (pl[jj + 2] - pl[jj + 1]);
                    }
                    ad1 = ad;
                }
            }
        }
    }
    if (dout[0]) {
        __builtin_amdgcn_wave_barrier();
        if (live)
#pragma unroll
            for (int j = 0; j < TPW; ++j) {
                if (j >= nt) break;
                for (int k = 0; k < L; ++k) __builtin_nontemporal_store(SH(j, k), &AT(dout[j], k));
            }
    }
    if (shal) {
        double csum[TPW], wsum = 0.0;
#pragma unroll
        for (int j = 0; j < TPW; ++j) csum[j] = 0.0;
        for (int b = L - 1; b >= ks; b -= TB) {
            double Ck[TPW][TB], pt[TB], pb[TB];
#pragma unroll
            for (int jj = 0; jj < TB; ++jj) {
                const int k = max(b - jj, ks);
#pragma unroll
                for (int j = 0; j < TPW; ++j) Ck[j][jj] = AT(C[j], k);
                pt[jj] = AT(M.pi, k);
                pb[jj] = AT(M.pi, k + 1);
            }
#pragma unroll
            for (int jj = 0; jj < TB; ++jj) {
                const int k = b - jj;
                if (k < ks) break;
                const double dpk = pb[jj] - pt[jj];
#pragma unroll
                for (int j = 0; j < TPW; ++j) csum[j] += dpk * (Ck[j][jj] + M.dt * SH(j, k));
                wsum += dpk;
            }
        }
        double Cu[TPW], Fb[TPW], C2bel[TPW], mu1 = 0.0;
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            Cu[j] = csum[j] / wsum;
            Fb[j] = 0.0;
            C2bel[j] = 0.0;
        }
        for (int b = ks; b >= kts + 1; b -= TB) {
            double mu[TB], Cl[TPW][TB + 1], zl[TB + 2], pl[TB + 1];
#pragma unroll
            for (int jj = 0; jj < TB; ++jj) mu[jj] = AT(M.sout.mu, max(b - jj, kts + 1));
#pragma unroll
            for (int jj = 0; jj <= TB; ++jj)
#pragma unroll
                for (int j = 0; j < TPW; ++j) Cl[j][jj] = AT(C[j], max(b - jj, kts));
#pragma unroll
            for (int jj = 0; jj <= TB + 1; ++jj) zl[jj] = AT(M.z, min(max(b + 1 - jj, 0), L - 1));
#pragma unroll
            for (int jj = 0; jj <= TB; ++jj) pl[jj] = AT(M.pi, max(b + 1 - jj, 0));
#pragma unroll
            for (int jj = 0; jj < TB; ++jj) {
                const int i = b - jj;
                if (i < kts + 1) break;
                double E = 0.0, D = 0.0;
                if (i < ks) {
                    const double dz = 0.5 * (zl[jj + 2] + zl[jj + 1]) - 0.5 * (zl[jj + 1] + zl[jj]);
                    E = P.eps_sh * mu1 * dz;
                    D = P.delta_sh * mu1 * dz;
                }
#pragma unroll
                for (int j = 0; j < TPW; ++j) {
                    const double Cim1 = Cl[j][jj + 1] + M.dt * SH(j, i - 1);
                    const double C2i = Cl[j][jj] + M.dt * SH(j, i);
                    if (i < ks) {
                        double num = (mu1 - D) * Cu[j] + E * C2i;
                        if (pgf) num += a.pgf * mu1 * (C2i - C2bel[j]);
                        Cu[j] = num / mu[jj];
                    }
                    C2bel[j] = C2i;
                    const double F = mu[jj] * (Cu[j] - Cim1);
                    SH(j, i) += (Fb[j] - F) * GRAV / (pl[jj] - pl[jj + 1]);
                    Fb[j] = F;
                }
                mu1 = mu[jj];
            }
        }
#pragma unroll
        for (int j = 0; j < TPW; ++j) SH(j, kts) += Fb[j] * GRAV / dp(kts);
    }
    __builtin_amdgcn_wave_barrier();
    if (live)
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            if (j >= nt) break;
            for (int k = 0; k < L; ++k) __builtin_nontemporal_store(SH(j, k), &AT(out[j], k));
        }
#undef SH
}

}  // namespace

extern "C" {

namespace {
int transport(conv_ctx_t *ctx, const conv_state_t *state, const conv_deep_out_t *dfwd,
              const conv_shallow_out_t *sfwd, int32_t ntr, const double *tracers, double pgf,
              double *tend, double *deep_tend, void *stream);
}  // namespace

int conv_tracer_transport(conv_ctx_t *ctx, const conv_state_t *state, const conv_deep_out_t *dfwd,
                          const conv_shallow_out_t *sfwd, int32_t ntr, const double *tracers,
                          double *tend, double *deep_tend, void *stream) {
    return transport(ctx, state, dfwd, sfwd, ntr, tracers, 0.0, tend, deep_tend, stream);
}

int conv_momentum_transport(conv_ctx_t *ctx, const conv_state_t *state,
                            const conv_deep_out_t *dfwd, const conv_shallow_out_t *sfwd,
                            const double *wind, double c_pgf, double *tend, double *deep_tend,
                            void *stream) {
    if (!std::isfinite(c_pgf)) return CONV_EINVAL;
    if (ctx && ctx->ncol > 0 && (!wind || !tend)) return CONV_EINVAL;
    return transport(ctx, state, dfwd, sfwd, 2, wind, c_pgf, tend, deep_tend, stream);
}

}  // extern "C"

namespace {
int transport(conv_ctx_t *ctx, const conv_state_t *state, const conv_deep_out_t *dfwd,
              const conv_shallow_out_t *sfwd, int32_t ntr, const double *tracers, double pgf,
              double *tend, double *deep_tend, void *stream) {
    if (!ctx || !state || !dfwd || !sfwd || ntr < 0 || ntr > 65535) return CONV_EINVAL;
    if (ctx->ncol == 0) return CONV_OK;  // nothing to read or write: the arrays may be NULL
    if (!state->z || !state->p_int || state->ld < ctx->ncol || !(state->dt > 0.0)) return CONV_EINVAL;
    if (!dfwd->mu || !dfwd->md || !dfwd->status || !dfwd->klaunch || !dfwd->ktop || !sfwd->mu ||
        !sfwd->status || !sfwd->kbase || !sfwd->ktop)
        return CONV_EINVAL;
    if (ntr > 0 && (!tracers || !tend)) return CONV_EINVAL;
    if (ctx->ncol == 0 || ntr == 0) return CONV_OK;
    TrArgs a;
    a.M = make_member(ctx->ncol, ctx->nlev, ctx->P, state, dfwd, sfwd, 0);
    a.pgf = pgf;
    a.ntr = ntr;
    a.C = tracers;
    a.tend = tend;
    a.dtend = deep_tend;
    // Two tracers per wavefront while their LDS stays within the default 64 KiB (nlev <= 64),
    // else one (at most 128 KiB for nlev <= 256, with the kernel's limit raised).
    const int tpw = (ntr >= 2 && 2 * (size_t)ctx->nlev * TW * sizeof(double) <= 65536) ? 2 : 1;
    const size_t lds = (size_t)tpw * ctx->nlev * TW * sizeof(double);
    if (lds > 65536) {
        static std::mutex mu;
        static std::set<int> done;  // devices with the LDS limit of k_tracers<1> raised
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return CONV_EHIP;
        std::lock_guard<std::mutex> g(mu);
        if (!done.count(dev)) {
            if (hipFuncSetAttribute((const void *)k_tracers<1>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
                hipSuccess)
                return CONV_EHIP;
            done.insert(dev);
        }
    }
    const int64_t blocks = (ctx->ncol + TW - 1) / TW * ((ntr + tpw - 1) / tpw);
    if (blocks > 0x7fffffff) return CONV_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    if (tpw == 2)
        hipLaunchKernelGGL(k_tracers<2>, dim3((unsigned)blocks), dim3(TW), lds, st, a);
    else
        hipLaunchKernelGGL(k_tracers<1>, dim3((unsigned)blocks), dim3(TW), lds, st, a);
    return check_launch();
}
}  // namespace
