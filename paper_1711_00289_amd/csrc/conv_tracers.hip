// conv_tracers.hip -- convective transport of passive tracers by the plumes of one step (the
// convection schemes the paper accelerates move heat and water; the same mass fluxes move every
// other constituent).
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
// One lane per column; tracers, then levels, innermost, so that a wavefront's stores of one level
// are one contiguous 512-byte segment.  Quiet columns only store zeros.
#include "conv_internal.hpp"

using namespace cvk;

namespace {

struct TrArgs {
    Member M;          // state, both schemes' outputs and parameters of the step
    int ntr;
    const double *C;   // tracers [ntr][nlev][ld]
    double *tend;      // deep + shallow tendency [ntr][nlev][ld]
    double *dtend;     // deep tendency alone (may be NULL)
};

__global__ __launch_bounds__(BLOCK) void k_tracers(TrArgs a) {
    const Member &M = a.M;
    const int64_t col = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (col >= M.ncol) return;
    const int64_t ld = M.ld;
    const int L = M.nlev;
    const int64_t plane = (int64_t)L * ld;
    const conv_params_t &P = M.P;
    // Active columns: status 0 with indices a status-0 column has, and a nonzero base mass flux
    // (the shallow closure's exp(-a CIN / sigma_w^2) can underflow to zero; such a plume moves
    // nothing).  Anything else moves nothing.
    const int kb = M.dout.klaunch[col], kt = M.dout.ktop[col];
    const int ks = M.sout.kbase[col], kts = M.sout.ktop[col];
    const bool deep = M.dout.status[col] == 0 && kb >= 1 && kb < L && kt >= 0 && kt < kb &&
                      AT(M.dout.mu, kb) > 0.0;
    const bool shal = M.sout.status[col] == 0 && ks >= 1 && ks < L && kts >= 0 && kts < ks - 1 &&
                      AT(M.sout.mu, ks) > 0.0;
    auto dp = [&](int k) { return AT(M.pi, k + 1) - AT(M.pi, k); };
    auto zi = [&](int i) { return 0.5 * (AT(M.z, i - 1) + AT(M.z, i)); };
    // The downdraft starts at the first interface from the top where it carries mass.
    int kd = -1;
    if (deep)
        for (int i = kt + 1; i <= kb; ++i)
            if (AT(M.dout.md, i) != 0.0) {
                kd = i - 1;
                break;
            }

    for (int t = 0; t < a.ntr; ++t) {
        const double *C = a.C + t * plane;
        double *out = a.tend + t * plane;
        double *dout = a.dtend ? a.dtend + t * plane : nullptr;
        for (int k = 0; k < L; ++k) {
            const bool in_d = deep && k >= kt && k <= kb;
            const bool in_s = shal && k >= kts && k <= ks;
            if (!in_d && !in_s) AT(out, k) = 0.0;
            if (dout && !in_d) AT(dout, k) = 0.0;
        }
        if (deep) {
            // Updraft, bottom-up: C_u at interface i, its flux, and layer i's tendency from its
            // bottom (Fb) and top fluxes.
            double Cu = AT(C, kb), Fb = 0.0, mu1 = 0.0;
            for (int i = kb; i >= kt + 1; --i) {
                const double mu = AT(M.dout.mu, i), md = AT(M.dout.md, i);
                if (i < kb) Cu = (mu1 * Cu + (mu - mu1) * AT(C, i)) / mu;
                const double Cup = AT(C, mu + md >= 0.0 ? i - 1 : i);
                const double F = mu * (Cu - Cup);
                AT(out, i) = (Fb - F) * GRAV / dp(i);
                Fb = F;
                mu1 = mu;
            }
            AT(out, kt) = Fb * GRAV / dp(kt);
            // Downdraft, top-down: C_d at interface i mixes layer i-1's air into C_d at i-1; its
            // flux enters layer i-1 from below and leaves layer i at the top.
            if (kd >= 0) {
                double Cd = AT(C, kd), ad1 = 0.0;
                for (int i = kd + 1; i <= kb; ++i) {
                    const double mu = AT(M.dout.mu, i), md = AT(M.dout.md, i);
                    const double ad = -md;
                    if (i > kd + 1) Cd = (ad1 * Cd + (ad - ad1) * AT(C, i - 1)) / ad;
                    const double F = md * (Cd - AT(C, mu + md >= 0.0 ? i - 1 : i));
                    AT(out, i - 1) += F * GRAV / dp(i - 1);
                    AT(out, i) -= F * GRAV / dp(i);
                    ad1 = ad;
                }
            }
            if (dout)
                for (int k = kt; k <= kb; ++k) AT(dout, k) = AT(out, k);
        }
        if (shal) {
            // The tracer the shallow scheme sees: updated by the deep transport.
            auto in_d = [&](int k) { return deep && k >= kt && k <= kb; };
            auto C2 = [&](int k) { return in_d(k) ? AT(C, k) + M.dt * AT(out, k) : AT(C, k); };
            double csum = 0.0, wsum = 0.0;
            for (int k = L - 1; k >= ks; --k) {
                csum += dp(k) * C2(k);
                wsum += dp(k);
            }
            double Cu = csum / wsum, Fb = 0.0, mu1 = 0.0;
            for (int i = ks; i >= kts + 1; --i) {
                const double mu = AT(M.sout.mu, i);
                if (i < ks) {
                    const double dz = zi(i) - zi(i + 1);
                    const double E = P.eps_sh * mu1 * dz, D = P.delta_sh * mu1 * dz;
                    Cu = ((mu1 - D) * Cu + E * C2(i)) / mu;
                }
                const double F = mu * (Cu - C2(i - 1));
                AT(out, i) = (in_d(i) ? AT(out, i) : 0.0) + (Fb - F) * GRAV / dp(i);
                Fb = F;
                mu1 = mu;
            }
            AT(out, kts) = (in_d(kts) ? AT(out, kts) : 0.0) + Fb * GRAV / dp(kts);
        }
    }
}

}  // namespace

extern "C" {

int conv_tracer_transport(conv_ctx_t *ctx, const conv_state_t *state, const conv_deep_out_t *dfwd,
                          const conv_shallow_out_t *sfwd, int32_t ntr, const double *tracers,
                          double *tend, double *deep_tend, void *stream) {
    if (!ctx || !state || !dfwd || !sfwd || ntr < 0) return CONV_EINVAL;
    if (!state->z || !state->p_int || state->ld < ctx->ncol || !(state->dt > 0.0)) return CONV_EINVAL;
    if (!dfwd->mu || !dfwd->md || !dfwd->status || !dfwd->klaunch || !dfwd->ktop || !sfwd->mu ||
        !sfwd->status || !sfwd->kbase || !sfwd->ktop)
        return CONV_EINVAL;
    if (ntr > 0 && (!tracers || !tend)) return CONV_EINVAL;
    if (ctx->ncol == 0 || ntr == 0) return CONV_OK;
    TrArgs a;
    a.M = make_member(ctx->ncol, ctx->nlev, ctx->P, state, dfwd, sfwd, 0);
    a.ntr = ntr;
    a.C = tracers;
    a.tend = tend;
    a.dtend = deep_tend;
    const unsigned g = (unsigned)((ctx->ncol + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_tracers, dim3(g), dim3(BLOCK), 0, (hipStream_t)stream, a);
    return check_launch();
}

}  // extern "C"
