/*
 * conv.h -- C ABI of libconv.so: FP64 deep (Zhang-McFarlane-style) and shallow (UW
 * bulk-plume-style) cumulus convection over many independent columns on one MI355X (gfx950).
 *
 * The paper (Ramesh et al., arXiv:1711.00289) states the problem these calls follow: physics is
 * computed per vertical column, independently across columns, once per time step, deep convection
 * before shallow convection (Background, Algorithm 1); deep convection is an entrainment loop and a
 * precipitation loop over columns x levels around an iterative thermodynamic inversion (Algorithm
 * 2); shallow convection tests thermodynamic conditions at several points and zeroes the outputs of
 * columns that exit early (Algorithm 3); inputs and outputs travel as one structure of arrays with
 * resident parameters and static buffers (Methodology, "Proportional Partitioning": packing,
 * offloading only the needed data, static in/out variables).  The paper gives the loop skeletons but
 * not the physics; the scheme computed is a written reading of ZM-style deep and UW-style shallow
 * convection in steps C0-C1 (grid, thermodynamics), D1-D10 (deep) and S1-S9 (shallow), which the
 * oracle's source (oracle/conv_oracle.cpp) states step by step and the kernels cite.
 *
 * Conventions for every call:
 *  - All array pointers are DEVICE pointers owned by the caller.  The library never allocates or
 *    frees device memory and never synchronises the host: calls only enqueue work on `stream`
 *    (a hipStream_t; NULL = the default stream) and return.  Kernel faults surface at the caller's
 *    next synchronisation.
 *  - Arrays are FP64, level-major: element (k, col) is at [k*ld + col], level 0 is the model top,
 *    the column index is fastest.  Layer arrays have nlev rows, interface arrays nlev+1 rows
 *    (interface i is the top of layer i; interface nlev is the surface).  Per-column arrays have
 *    ld entries.  Only columns 0 .. ncol-1 are read or written; ld >= ncol allows padding.
 *  - Index outputs are 0-based with -1 meaning "undefined".
 *  - Return value: CONV_OK (0) or a negative CONV_E* code.  CONV_EINVAL: a NULL pointer, a bad
 *    size, ld < ncol, dt <= 0 or a workspace that is too small; nothing is enqueued.  CONV_EHIP: a
 *    kernel launch failed (conv_last_hip_error() returns the hipError_t value).
 *  - A context over 0 columns reads and writes no array, so its calls accept NULL array pointers
 *    (the argument structs themselves must be given); they enqueue nothing but the zeroing of the
 *    backward calls' parameter gradients (g_params, which must be given).
 *  - A context is not thread-safe and its workspace is shared by its calls: calls on one context
 *    must be ordered on one stream.
 *  - Per-column physics outcomes are not errors; they are reported in `status`:
 *      deep:    0 convecting, 1 not triggered, 2 closure F <= 0, 3 invalid column
 *      shallow: 0 convecting, 1 no LCL, 2 no LFC, 3 CIN > cin_max, 4 tke <= 0,
 *               5 plume dies in the first layer, 6 invalid column
 *    Every flux, tendency and precipitation output of a non-convecting column is exactly +0.0.
 */
#ifndef CONV_H
#define CONV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CONV_OK 0
#define CONV_EINVAL (-1)
#define CONV_EUNSUPPORTED (-2)
#define CONV_EHIP (-3)
#define CONV_ERANGE (-4) /* conv_step_static: the sizes need more than its static scratch */

/* Size of the static device array conv_step_static uses as its workspace (one per GPU). */
#define CONV_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

typedef struct conv_ctx conv_ctx_t; /* opaque host-side handle */

/* Scheme parameters, SI units (defaults in parentheses). */
typedef struct {
    double cape_threshold; /* trigger: CAPE > threshold (70 J/kg) */
    double tau;            /* deep closure time scale (3600 s) */
    double eps_deep;       /* deep entrainment rate (1e-4 1/m) */
    double alpha_dd;       /* downdraft strength (0.2) */
    double evap_max_frac;  /* downdraft evaporation <= this fraction of condensate (0.9) */
    double p_launch_min;   /* launch layer search: p_mid >= this (60000 Pa) */
    double p_top_min;      /* cloud top: p_mid >= this (4000 Pa) */
    double eps_sh;         /* shallow entrainment rate (1e-3 1/m) */
    double delta_sh;       /* shallow detrainment rate (1e-3 1/m) */
    double qlcrit_sh;      /* shallow rain-out threshold (1e-3 kg/kg) */
    double cin_max;        /* shallow CIN limit (100 J/kg) */
    double a_buoy;         /* buoyancy factor in w^2 (1) */
    double b_drag;         /* drag factor in w^2 (1) */
    double c_tke;          /* sigma_w^2 = c_tke * tke (1) */
    double p_lcl_min;      /* LCL must lie at p_mid >= this (60000 Pa) */
    double p_sh_top_min;   /* shallow LFC and plume top: p >= this (40000 Pa) */
    double eps_cape;       /* entrainment rate of the CAPE parcel (0 1/m: undilute).  > 0: the
                              parcel mixes in environmental air on its way up (dilute CAPE; h and
                              total water mix in, eps_cape per metre of mid-level height) and the
                              closure follows the entrained air too.  The adjoints support 0 only. */
} conv_params_t;

/* Input state (device pointers, read only). */
typedef struct {
    const double *T;     /* [nlev][ld]   temperature, K */
    const double *q;     /* [nlev][ld]   specific humidity, kg/kg */
    const double *p_mid; /* [nlev][ld]   mid-layer pressure, Pa */
    const double *z;     /* [nlev][ld]   mid-layer height above the surface, m */
    const double *p_int; /* [nlev+1][ld] interface pressure, Pa */
    const double *phis;  /* [ld]         surface geopotential, m^2/s^2 */
    const double *pblh;  /* [ld]         boundary-layer height, m (shallow only) */
    const double *tke;   /* [ld]         boundary-layer TKE, m^2/s^2 (shallow only) */
    int64_t ld;          /* leading dimension, >= ncol */
    double dt;           /* physics time step, s (> 0) */
} conv_state_t;

/* Deep-scheme outputs (device pointers, written). */
typedef struct {
    double *dTdt, *dqdt;           /* [nlev][ld]   heating K/s, moistening 1/s */
    double *mu, *md;               /* [nlev+1][ld] updraft / downdraft mass flux kg m^-2 s^-1 */
    double *prec, *cape;           /* [ld]         kg m^-2 s^-1, J/kg */
    int32_t *klaunch, *ktop, *trig, *status; /* [ld] */
} conv_deep_out_t;

/* Shallow-scheme outputs (device pointers, written). */
typedef struct {
    double *dTdt, *dqdt; /* [nlev][ld] */
    double *mu;          /* [nlev+1][ld] */
    double *prec, *cin;  /* [ld] */
    int32_t *kbase, *ktop, *status; /* [ld] */
} conv_shallow_out_t;

/* Device workspace size (bytes) that a context over (ncol, nlev) needs on the current device. */
size_t conv_workspace_bytes(int64_t ncol, int32_t nlev);

/* Create a context for up to `ncol` columns of `nlev` levels (2 <= nlev <= 256) over a
 * caller-owned device workspace of at least conv_workspace_bytes(ncol, nlev) bytes, 256-byte
 * aligned.  `params` is a host pointer and is copied.  The handle is host memory. */
int conv_create(int64_t ncol, int32_t nlev, const conv_params_t *params, void *workspace,
                size_t ws_bytes, conv_ctx_t **out);
/* Replace the parameters (host pointer, copied). */
int conv_set_params(conv_ctx_t *ctx, const conv_params_t *params);
/* Free the host handle (the workspace stays the caller's). */
void conv_destroy(conv_ctx_t *ctx);

/* Deep scheme (steps D1-D10) over columns 0 .. ncol-1. */
int conv_deep_forward(conv_ctx_t *ctx, const conv_state_t *state, conv_deep_out_t *out,
                      void *stream);
/* Shallow scheme (steps S1-S9) on the given state. */
int conv_shallow_forward(conv_ctx_t *ctx, const conv_state_t *state, conv_shallow_out_t *out,
                         void *stream);
/* One physics step of both schemes in the paper's Algorithm 1 order: deep, then the state update
 * T' = T + dt*dTdt, q' = q + dt*dqdt, then shallow on (T', q'). */
int conv_step(conv_ctx_t *ctx, const conv_state_t *state, conv_deep_out_t *deep,
              conv_shallow_out_t *shallow, void *stream);

/* conv_step with no context and no workspace argument, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid allocation.  The
 * kernels are conv_step's and the results bit-identical to it.  Their workspace (counters, active
 * lists, plume scratch) is a static device array of CONV_STATIC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends; its address is looked up once per device,
 * on the first call there.  The plume kernels get the widest persistent grids (5 wavefronts per
 * compute unit down to 1) whose workspace fits the array; sizes for which even one wavefront per
 * compute unit does not fit (on 256 compute units: more than 1,017,088 columns of 30 levels,
 * 726,112 of 46 or 385,344 of 72) return CONV_ERANGE with nothing enqueued.  The call allocates
 * no memory, host or device, and does not synchronise the host; `params` is a host pointer, read
 * during the call.
 * Every call on one GPU shares that GPU's array and leaves its contents behind (the counters are
 * cleared by the call's own first kernel): calls that overlap on one GPU (different streams or
 * threads) race, so the caller must order them. */
int conv_step_static(int64_t ncol, int32_t nlev, const conv_params_t *params,
                     const conv_state_t *state, conv_deep_out_t *deep,
                     conv_shallow_out_t *shallow, void *stream);

/* Cotangents of the deep outputs (device pointers; any may be NULL = zero). */
typedef struct {
    const double *g_dTdt, *g_dqdt; /* [nlev][ld] */
    const double *g_prec;          /* [ld] */
} conv_deep_cot_t;

/* Gradients (device pointers, written). */
typedef struct {
    double *g_T, *g_q; /* [nlev][ld]  dL/dT, dL/dq */
    double *g_params;  /* [2]         dL/dtau, dL/deps_deep summed over columns */
} conv_deep_grad_t;

/* Device workspace (bytes) the backward calls (conv_deep_backward, conv_shallow_backward,
 * conv_step_backward) need for a context over (ncol, nlev) and state
 * arrays of leading dimension ld. */
size_t conv_backward_workspace_bytes(int64_t ncol, int32_t nlev, int64_t ld);

/* Hand-written adjoint of the deep scheme (steps D1-D10): the gradient of
 * L = sum(g_dTdt*dTdt) + sum(g_dqdt*dqdt) + sum(g_prec*prec) with respect to T, q and the
 * parameters tau and eps_deep, through the branch the forward run took (launch and top levels,
 * downdraft start, saturation flags, upwind choices, downdraft-strength and base-flux branches held
 * fixed).  `fwd` must hold the status, klaunch and ktop outputs of conv_deep_forward (or conv_step)
 * on the same state and parameters; everything else is recomputed per column (checkpointing).
 * Columns whose deep status is not 0 get zero gradients.  The parameter gradients are summed in a
 * fixed order (bit-reproducible).  `workspace`: caller-owned, 256-byte aligned, at least
 * conv_backward_workspace_bytes(ncol, nlev, ld) bytes; it may not be the context's forward
 * workspace.  The paper's deep convection (Algorithm 2) is the forward this differentiates.
 * Returns CONV_EUNSUPPORTED when the context's eps_cape is not 0 (the adjoint is of the undilute
 * parcel). */
int conv_deep_backward(conv_ctx_t *ctx, const conv_state_t *state, const conv_deep_out_t *fwd,
                       const conv_deep_cot_t *cot, conv_deep_grad_t *grad, void *workspace,
                       size_t ws_bytes, void *stream);

/* Cotangents of the shallow scheme's outputs (device [nlev][ld] / [ld]; any may be NULL = 0) and
 * the gradients of its adjoint (g_T, g_q [nlev][ld], written for every column 0..ncol-1;
 * g_params: device double[2] = dL/d eps_sh, dL/d delta_sh). */
typedef struct {
    const double *g_dTdt, *g_dqdt, *g_prec;
} conv_shallow_cot_t;
typedef struct {
    double *g_T, *g_q;
    double *g_params;
} conv_shallow_grad_t;

/* Hand-written adjoint of the shallow scheme (steps S1-S9) alone: the gradient of
 * L = sum(g_dTdt*dTdt) + sum(g_dqdt*dqdt) + sum(g_prec*prec) over conv_shallow_forward's outputs with
 * respect to its input T, q and the mixing rates eps_sh, delta_sh, through the branch the forward
 * run took (source layers, lifting-condensation and free-convection levels, the levels counted in
 * CIN, saturation and rain-out flags, plume top, base-flux branch and limiting layer held fixed).
 * `fwd` must hold the status, kbase and ktop outputs of conv_shallow_forward on the same state and
 * parameters; everything else is recomputed per column.  Columns whose shallow status is not 0 get
 * zero gradients.  Workspace as for conv_deep_backward.  The paper's shallow convection
 * (Algorithm 3) is the forward this differentiates. */
int conv_shallow_backward(conv_ctx_t *ctx, const conv_state_t *state,
                          const conv_shallow_out_t *fwd, const conv_shallow_cot_t *cot,
                          conv_shallow_grad_t *grad, void *workspace, size_t ws_bytes,
                          void *stream);

/* Gradients of the adjoint of a whole step: g_T, g_q [nlev][ld] for every column; g_params: device
 * double[4] = dL/d tau, dL/d eps_deep, dL/d eps_sh, dL/d delta_sh. */
typedef struct {
    double *g_T, *g_q;
    double *g_params;
} conv_step_grad_t;

/* Hand-written adjoint of conv_step (Algorithm 1 order: deep, the state update T' = T + dt*dTdt,
 * q' = q + dt*dqdt, shallow on the updated state): the gradient of a loss with cotangents on both
 * schemes' outputs (`dcot`, `scot`; any array may be NULL) with respect to T, q and the four
 * parameters.  The shallow adjoint runs first, at the updated state; its gradient is then carried
 * through the update (identity plus dt times the deep tendencies' cotangent) into the deep
 * adjoint.  Branches are held fixed as for the two schemes' adjoints.  `dfwd` and `sfwd` must hold
 * the outputs of conv_step on the same state and parameters (status, klaunch, ktop, dTdt, dqdt of
 * the deep scheme; status, kbase, ktop of the shallow one).  Workspace as for conv_deep_backward.
 * Returns CONV_EUNSUPPORTED when the context's eps_cape is not 0. */
int conv_step_backward(conv_ctx_t *ctx, const conv_state_t *state, const conv_deep_out_t *dfwd,
                       const conv_shallow_out_t *sfwd, const conv_deep_cot_t *dcot,
                       const conv_shallow_cot_t *scot, conv_step_grad_t *grad, void *workspace,
                       size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- convective tracer transport
 * Transport of ntr passive tracers (mixing ratios, no sources or sinks) by the plumes of one
 * conv_step: each plume mixes a tracer exactly as it mixes moist static energy (deep updraft and
 * downdraft of steps D5-D7, shallow updraft of S7-S8: the same entrainment, detrainment and upwind
 * environment values), and the tendency is the flux divergence.  The shallow scheme transports the
 * tracer updated by the deep transport, C + dt * deep tendency (Algorithm 1 order).  Extends the
 * paper's convection, which moves heat and water, to every other constituent the same mass fluxes
 * carry.
 * `dfwd`, `sfwd`: the outputs of conv_step on `state` with the context's parameters (mu, md,
 * status, klaunch, ktop of the deep scheme; mu, status, kbase, ktop of the shallow one); the
 * plumes are not run again.  tracers, tend, deep_tend: device [ntr][nlev][ld] with the state's ld;
 * tend receives the deep + shallow tendency (s-1), deep_tend (may be NULL) the deep part alone.
 * Columns with neither scheme active get exact zeros.  ntr = 0 does nothing.  Returns CONV_EINVAL
 * for missing arrays or ntr outside 0..65535. */
int conv_tracer_transport(conv_ctx_t *ctx, const conv_state_t *state, const conv_deep_out_t *dfwd,
                          const conv_shallow_out_t *sfwd, int32_t ntr, const double *tracers,
                          double *tend, double *deep_tend, void *stream);

/* Convective momentum transport by the plumes of one conv_step: the two horizontal wind components
 * carried as conv_tracer_transport carries a tracer, plus the convective pressure-gradient term of
 * Gregory, Kershaw & Inness (1997, Q. J. R. Meteorol. Soc. 123): the cloud-scale pressure gradient
 * pulls a plume's wind towards the environment's as the plume crosses environmental shear, so
 * crossing a layer adds c_pgf times the plume's mass flux times the change of the environmental
 * wind from the layer the plume comes from (below for an updraft, above for the downdraft) to the
 * layer it crosses.  c_pgf = 0 is passive transport (the results are then bit-identical to
 * conv_tracer_transport of the two components), 1 makes a plume follow the environment's shear;
 * Gregory et al. use 0.7.  The tendencies are flux divergences, so column momentum is conserved.
 * Extends the paper's convection, which moves heat and water, to the momentum the same mass fluxes
 * carry.
 * `dfwd`, `sfwd`: the outputs of conv_step on `state` with the context's parameters, as for
 * conv_tracer_transport.  wind: device [2][nlev][ld] (u, then v; m/s) with the state's ld; tend
 * (m s^-2) and deep_tend (may be NULL: the deep part alone) likewise.  Columns with neither scheme
 * active get exact zeros.  Returns CONV_EINVAL for missing arrays or a non-finite c_pgf. */
int conv_momentum_transport(conv_ctx_t *ctx, const conv_state_t *state,
                            const conv_deep_out_t *dfwd, const conv_shallow_out_t *sfwd,
                            const double *wind, double c_pgf, double *tend, double *deep_tend,
                            void *stream);

/* ---------------------------------------------------------------- batched ensemble
 * Several grids ("members", e.g. ensemble members of a forecast) with their own column counts,
 * level counts (2..256), parameters and arrays, advanced by one conv_step each in the SAME kernel
 * launches: the trigger launch covers every member's tiles and the plume launches run over one
 * compacted list of active columns drawn from all members.  This is the batching counterpart of
 * the paper's chunked column loop (Methodology, load balancing): uneven members share the GPU
 * instead of running one after the other.  Per-column results are bit-identical to conv_step on
 * each member alone. */
typedef struct conv_ens conv_ens_t; /* opaque host-side handle */

typedef struct {
    int64_t ncol;                /* >= 0; a member with 0 columns may leave its pointers NULL */
    int32_t nlev;                /* 2..256 */
    conv_params_t params;
    conv_state_t state;          /* device pointers, as for conv_step */
    conv_deep_out_t deep;        /* device pointers, written */
    conv_shallow_out_t shallow;  /* device pointers, written */
} conv_member_t;

/* Workspace bytes for these members (0 if any member is malformed). */
size_t conv_ensemble_workspace_bytes(int n_members, const conv_member_t *members);

/* Copies the member table (host array, 1..4096 entries) into the 256-byte aligned, caller-owned
 * device workspace (a synchronous host-to-device copy on the current device) and returns a handle.
 * The members' arrays must stay valid while the handle is used. */
int conv_ensemble_create(int n_members, const conv_member_t *members, void *workspace,
                         size_t ws_bytes, conv_ens_t **out);
void conv_ensemble_destroy(conv_ens_t *e); /* frees the host handle and any captured graph */

/* One step of every member on `stream` (four kernel launches in all, no host synchronisation, no
 * memset nodes: capturable). */
int conv_ensemble_step(conv_ens_t *e, void *stream);

/* Persistent-grid shape of the plume kernels (wavefronts per compute unit, 1..32, as for
 * conv_set_launch).  Changing it drops a captured graph. */
int conv_ensemble_set_launch(conv_ens_t *e, int fused_waves_per_cu, int shallow_waves_per_cu);
int conv_ensemble_get_launch(conv_ens_t *e, int *fused_waves_per_cu, int *shallow_waves_per_cu);

/* Autotuner: times conv_ensemble_step (median of `reps` runs, 1..1000, the lower of two sweeps)
 * for every deep-plume shape in {4,5,6,8} wavefronts per CU and keeps the fastest (the step runs
 * the shallow plumes inside its re-trigger, so the shallow-plume shape keeps its default of 32;
 * it serves conv_shallow alone).  Results are cached per process, keyed by device and member
 * shapes; `force` != 0 re-tunes.  Runs steps (the outputs are overwritten) and waits on the host,
 * so it may not be called during capture.  Outputs may be NULL. */
int conv_ensemble_autotune(conv_ens_t *e, void *stream, int reps, int force,
                           int *fused_waves_per_cu, int *shallow_waves_per_cu, float *ms);

/* Captures one conv_ensemble_step on `stream` (not the null stream) into a HIP graph owned by the
 * handle, replacing any earlier one; conv_ensemble_replay launches it (CONV_EINVAL if there is
 * none).  A replay reads the member table and arrays as they are when it runs. */
int conv_ensemble_capture(conv_ens_t *e, void *stream);
int conv_ensemble_replay(conv_ens_t *e, void *stream);

/* The same autotuner for a single context's conv_step on (state, deep, shallow). */
int conv_autotune(conv_ctx_t *ctx, const conv_state_t *state, conv_deep_out_t *deep,
                  conv_shallow_out_t *shallow, void *stream, int reps, int force,
                  int *fused_waves_per_cu, int *shallow_waves_per_cu, float *ms);

/* Launch shape of the persistent kernels: wavefronts per compute unit for the deep-plume kernel
 * and for the shallow-plume kernel that conv_shallow launches (each 1..32; default 5 and 32),
 * launched as blocks of one 64-thread wavefront each (the deep plume's LDS keeps at most 5 per CU
 * resident; the others queue).  Neither the workspace size nor the results depend on it (the
 * results are bit-identical). */
int conv_set_launch(conv_ctx_t *ctx, int fused_waves_per_cu, int shallow_waves_per_cu);
int conv_get_launch(conv_ctx_t *ctx, int *fused_waves_per_cu, int *shallow_waves_per_cu);

/* Instrumentation: record HIP events on the call's stream around each kernel of the next
 * `max_calls` calls (0 turns recording off).  conv_timing_read() waits for the recorded calls and
 * returns, per stage, the summed milliseconds over those calls in ms[0..4] (counter reset, trigger
 * pass, deep-plume pass, shallow re-trigger of the deep columns with their shallow plumes,
 * shallow-plume pass of the shallow scheme alone; a stage a call does not run reads as the time
 * between its neighbours' events) and the number of recorded calls in *ncalls.
 * Events are host-side handles created here; no device memory is allocated. */
int conv_timing_start(conv_ctx_t *ctx, int max_calls);
int conv_timing_read(conv_ctx_t *ctx, double *ms, int *ncalls);

const char *conv_strerror(int code);
int conv_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif
