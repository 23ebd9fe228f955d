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
// One wavefront per block, one lane per column; block b takes tracer b % ntr of column block
// b / ntr, so the tracers of one column block are dispatched together (they share its mass fluxes
// in L2, and the slow convecting blocks spread over the run instead of piling up at its end).
// The tendencies are written once and not read again here: non-temporal stores (0.58 -> 0.52 ms
// for 8 tracers on the 884,736-column grid).
// A lane accumulates its
// column's tendencies in LDS ([level][lane]); then the wavefront stores level by level with every
// lane active, so each store covers whole 128-byte lines (stores that cover only part of a line,
// as a wavefront mixing quiet and convecting columns would issue, run at a fraction of the
// bandwidth on this part).  Quiet columns contribute zeros.
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

__global__ __launch_bounds__(TW) void k_tracers(TrArgs a) {
    extern __shared__ double sh[];  // [nlev][TW]
    const Member &M = a.M;
    const int lane = threadIdx.x;
    const int t = (int)(blockIdx.x % (unsigned)a.ntr);
    const int64_t col = (int64_t)(blockIdx.x / (unsigned)a.ntr) * TW + lane;
    const bool live = col < M.ncol;
    const int64_t ld = M.ld;
    const int L = M.nlev;
    const int64_t plane = (int64_t)L * ld;
    const conv_params_t &P = M.P;
    const double *C = a.C + (int64_t)t * plane;
    double *out = a.tend + (int64_t)t * plane;
    double *dout = a.dtend ? a.dtend + (int64_t)t * plane : nullptr;
#define SH(k) sh[(k) * TW + lane]

    // Active columns: status 0 with indices a status-0 column has, and a nonzero base mass flux
    // (the shallow closure's exp(-a CIN / sigma_w^2) can underflow to zero; such a plume moves
    // nothing).  Anything else moves nothing.
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

    // A wavefront with nothing convecting stores its zeros directly.
    if (__ballot(deep || shal) == 0ull) {
        if (live) {
            for (int k = 0; k < L; ++k) {
                __builtin_nontemporal_store(0.0, &AT(out, k));
                if (dout) __builtin_nontemporal_store(0.0, &AT(dout, k));
            }
        }
        return;
    }
    for (int k = 0; k < L; ++k) SH(k) = 0.0;

    if (deep) {
        // Updraft, bottom-up: C_u at interface i, its flux, and layer i's tendency from its
        // bottom (Fb) and top fluxes.  The loads of TB interfaces are issued together, then those
        // interfaces are computed (a level's arithmetic is far shorter than a load's latency);
        // indices are clamped, so values loaded past the top are not used.  The downdraft's
        // first interface (the highest one with md != 0) is noted on the way.
        // With a pressure-gradient term, crossing layer i adds pgf * mu[i+1] * (C_i - C_{i+1}):
        // `Cbel` holds C of the layer below the interface being computed.
        double Cu = AT(C, kb), Fb = 0.0, mu1 = 0.0, Cbel = 0.0;
        const bool pgf = a.pgf != 0.0;
        int i0 = kb + 1;
        for (int b = kb; b >= kt + 1; b -= TB) {
            double mu[TB], md[TB], Ci[TB + 1], pt[TB + 1];
#pragma unroll
            for (int j = 0; j <= TB; ++j) {
                const int i = max(b - j, kt);
                Ci[j] = AT(C, i);
                pt[j] = AT(M.pi, i);
            }
            const double pbot0 = AT(M.pi, b + 1);
#pragma unroll
            for (int j = 0; j < TB; ++j) {
                const int i = max(b - j, kt + 1);
                mu[j] = AT(M.dout.mu, i);
                md[j] = AT(M.dout.md, i);
            }
#pragma unroll
            for (int j = 0; j < TB; ++j) {
                const int i = b - j;
                if (i < kt + 1) break;
                // interface i: layer i below (C_i), layer i-1 above (C_{i-1}); layer i spans
                // pressures pt[j] (top) .. its bottom interface (pt[j-1], or pbot0 for j = 0)
                if (md[j] != 0.0) i0 = i;
                if (i < kb) {
                    double num = mu1 * Cu + (mu[j] - mu1) * Ci[j];
                    if (pgf) num += a.pgf * mu1 * (Ci[j] - Cbel);
                    Cu = num / mu[j];
                }
                Cbel = Ci[j];
                const double F = mu[j] * (Cu - (mu[j] + md[j] >= 0.0 ? Ci[j + 1] : Ci[j]));
                const double pbot = j == 0 ? pbot0 : pt[j - 1];
                SH(i) = (Fb - F) * GRAV / (pbot - pt[j]);
                Fb = F;
                mu1 = mu[j];
            }
        }
        SH(kt) = Fb * GRAV / dp(kt);
        // Downdraft, top-down from its first interface: C_d at interface i mixes layer i-1's air
        // into C_d at i-1; its flux enters layer i-1 from below and leaves layer i at the top.
        if (i0 <= kb) {
            // Crossing layer i-1 downward adds pgf * |md[i-1]| * (C_{i-1} - C_{i-2}): `Cabv` holds
            // C of the layer above the one crossed.
            double Cd = AT(C, i0 - 1), ad1 = 0.0, Cabv = 0.0;
            for (int b = i0; b <= kb; b += TB) {
                // interfaces b .. b+TB-1: layers b-1 .. b+TB-1 and their interfaces b-1 .. b+TB
                double mu[TB], md[TB], Cl[TB + 1], pl[TB + 2];
#pragma unroll
                for (int j = 0; j < TB; ++j) {
                    const int i = min(b + j, kb);
                    mu[j] = AT(M.dout.mu, i);
                    md[j] = AT(M.dout.md, i);
                }
#pragma unroll
                for (int j = 0; j <= TB; ++j) Cl[j] = AT(C, min(b - 1 + j, kb));
#pragma unroll
                for (int j = 0; j <= TB + 1; ++j) pl[j] = AT(M.pi, min(b - 1 + j, kb + 1));
#pragma unroll
                for (int j = 0; j < TB; ++j) {
                    const int i = b + j;
                    if (i > kb) break;
                    const double ad = -md[j];
                    if (i > i0) {
                        double num = ad1 * Cd + (ad - ad1) * Cl[j];
                        if (pgf) num += a.pgf * ad1 * (Cl[j] - Cabv);
                        Cd = num / ad;
                    }
                    Cabv = Cl[j];
                    const double F = md[j] * (Cd - (mu[j] + md[j] >= 0.0 ? Cl[j] : Cl[j + 1]));
                    SH(i - 1) += F * GRAV / (pl[j + 1] - pl[j]);
                    SH(i) -= F * GRAV / (pl[j + 2] - pl[j + 1]);
                    ad1 = ad;
                }
            }
        }
    }
    if (dout) {
        __builtin_amdgcn_wave_barrier();
        if (live)
            for (int k = 0; k < L; ++k) __builtin_nontemporal_store(SH(k), &AT(dout, k));
    }
    if (shal) {
        // The tracer the shallow scheme sees: updated by the deep transport (zero where the deep
        // scheme left the column alone).
        // C2(k) = C(k) + dt SH(k): the tracer after the deep transport.  The recursion below adds
        // the shallow part to level i only after reading C2(i) and C2(i - 1), and level i is read
        // by no later step, so SH holds the deep part wherever C2 is evaluated.
        double csum = 0.0, wsum = 0.0;
        for (int b = L - 1; b >= ks; b -= TB) {
            double Ck[TB], pt[TB], pb[TB];
#pragma unroll
            for (int j = 0; j < TB; ++j) {
                const int k = max(b - j, ks);
                Ck[j] = AT(C, k);
                pt[j] = AT(M.pi, k);
                pb[j] = AT(M.pi, k + 1);
            }
#pragma unroll
            for (int j = 0; j < TB; ++j) {
                const int k = b - j;
                if (k < ks) break;
                const double dpk = pb[j] - pt[j];
                csum += dpk * (Ck[j] + M.dt * SH(k));
                wsum += dpk;
            }
        }
        double Cu = csum / wsum, Fb = 0.0, mu1 = 0.0, C2bel = 0.0;
        const bool pgf = a.pgf != 0.0;
        for (int b = ks; b >= kts + 1; b -= TB) {
            // interfaces b .. b-TB+1: layers b .. b-TB, heights b+1 .. b-TB, pressures b+1 .. b-TB+1
            double mu[TB], Cl[TB + 1], zl[TB + 2], pl[TB + 1];
#pragma unroll
            for (int j = 0; j < TB; ++j) mu[j] = AT(M.sout.mu, max(b - j, kts + 1));
#pragma unroll
            for (int j = 0; j <= TB; ++j) Cl[j] = AT(C, max(b - j, kts));
#pragma unroll
            for (int j = 0; j <= TB + 1; ++j) zl[j] = AT(M.z, min(max(b + 1 - j, 0), L - 1));
#pragma unroll
            for (int j = 0; j <= TB; ++j) pl[j] = AT(M.pi, max(b + 1 - j, 0));
#pragma unroll
            for (int j = 0; j < TB; ++j) {
                const int i = b - j;
                if (i < kts + 1) break;
                const double Cim1 = Cl[j + 1] + M.dt * SH(i - 1);
                const double C2i = Cl[j] + M.dt * SH(i);  // before SH(i) takes its shallow part
                if (i < ks) {
                    // zi(i) - zi(i + 1), the interface heights as means of the layers around them
                    const double dz = 0.5 * (zl[j + 2] + zl[j + 1]) - 0.5 * (zl[j + 1] + zl[j]);
                    const double E = P.eps_sh * mu1 * dz, D = P.delta_sh * mu1 * dz;
                    double num = (mu1 - D) * Cu + E * C2i;
                    if (pgf) num += a.pgf * mu1 * (C2i - C2bel);
                    Cu = num / mu[j];
                }
                C2bel = C2i;
                const double F = mu[j] * (Cu - Cim1);
                SH(i) += (Fb - F) * GRAV / (pl[j] - pl[j + 1]);
                Fb = F;
                mu1 = mu[j];
            }
        }
        SH(kts) += Fb * GRAV / dp(kts);
    }
    __builtin_amdgcn_wave_barrier();
    if (live)
        for (int k = 0; k < L; ++k) __builtin_nontemporal_store(SH(k), &AT(out, k));
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
    const size_t lds = (size_t)ctx->nlev * TW * sizeof(double);  // at most 128 KiB (nlev <= 256)
    if (lds > 65536) {
        static std::mutex mu;
        static std::set<int> done;  // devices with the LDS limit of k_tracers raised
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return CONV_EHIP;
        std::lock_guard<std::mutex> g(mu);
        if (!done.count(dev)) {
            if (hipFuncSetAttribute((const void *)k_tracers,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
                hipSuccess)
                return CONV_EHIP;
            done.insert(dev);
        }
    }
    const int64_t blocks = (ctx->ncol + TW - 1) / TW * ntr;
    if (blocks > 0x7fffffff) return CONV_EINVAL;
    hipLaunchKernelGGL(k_tracers, dim3((unsigned)blocks), dim3(TW), lds, (hipStream_t)stream, a);
    return check_launch();
}
}  // namespace
