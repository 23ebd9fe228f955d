/*
 * conv_oracle.h -- C entry points of the CPU oracle for the deep (Zhang-McFarlane-style) and
 * shallow (UW bulk-plume-style) cumulus convection schemes.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64 reference used by the
 * tests, by the smoke check and by the benchmark's CPU baseline to check the HIP path.  Nothing in
 * the product library links, includes or calls it, and it shares no code with the HIP kernels.
 *
 * The paper (Ramesh et al., "Deep and Shallow convections in Atmosphere Models on Intel Xeon Phi
 * Coprocessor Systems", arXiv:1711.00289) names the two schemes (Background, "Deep Convection" /
 * "Shallow Convection") and gives their loop skeletons (Algorithms 2 and 3) but no physics; the
 * scheme computed here is a written reading in steps C0-C1, D1-D10 and S1-S9, stated step by step
 * in conv_oracle.cpp.  All arrays are host arrays, level-major: element (k, col) at [k*ld + col], level 0 at
 * the model top; interface arrays have nlev+1 rows.
 */
#ifndef CONV_ORACLE_H
#define CONV_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double cape_threshold, tau, eps_deep, alpha_dd, evap_max_frac, p_launch_min, p_top_min;
    double eps_sh, delta_sh, qlcrit_sh, cin_max, a_buoy, b_drag, c_tke, p_lcl_min, p_sh_top_min;
    double eps_cape; /* entrainment rate of the CAPE parcel, 1/m (0: undilute) */
} oracle_params_t;

typedef struct {
    const double *T, *q, *p_mid, *z; /* [nlev][ld] */
    const double *p_int;             /* [nlev+1][ld] */
    const double *phis, *pblh, *tke; /* [ld] */
    int64_t ld;
    double dt;
} oracle_state_t;

typedef struct {
    double *dTdt, *dqdt;   /* [nlev][ld]   K/s, kg/kg/s */
    double *mu, *md;       /* [nlev+1][ld] kg m^-2 s^-1 (md <= 0) */
    double *prec, *cape;   /* [ld] */
    int32_t *klaunch, *ktop, *trig, *status;
} oracle_deep_out_t;

typedef struct {
    double *dTdt, *dqdt;   /* [nlev][ld] */
    double *mu;            /* [nlev+1][ld] */
    double *prec, *cin;    /* [ld] */
    int32_t *kbase, *ktop, *status;
} oracle_shallow_out_t;

/* Per-column diagnostics of the deep scheme (for the pins). */
typedef struct {
    int32_t kb, kt, kd, klim, status;
    double cape, F, Mc, Mlim, Mb, alpha, C1, E1, P1;
} oracle_deep_diag_t;

/* Per-column diagnostics of the shallow scheme. */
typedef struct {
    int32_t ks, klcl, klfc, kt, status;
    double hs, qs, cin, rho_s, sigw2, Mclos, Mlim, Mb, P1;
} oracle_shallow_diag_t;

/* Full column runs over ncol columns (0 on success, -1 on bad arguments). */
int oracle_deep(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                oracle_deep_out_t *o);
int oracle_shallow(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                   oracle_shallow_out_t *o);
/* Deep, then T' = T + dt*dTdt, q' = q + dt*dqdt, then shallow on (T', q') (Algorithm 1 order). */
int oracle_step(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                oracle_deep_out_t *od, oracle_shallow_out_t *os);

/* Algorithmic operation count of oracle_step per column (ops[ncol]): +, -, *, /, sqrt, exp and
 * log count 1 each, over every operation with a state- or parameter-dependent operand, plus the
 * grid's own arithmetic (6 operations per layer for each scheme).  The count follows the oracle's
 * own algorithm (its root finder's iterations included). */
int oracle_step_ops(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                    double *ops);

/* Same as oracle_step with OpenMP dynamic scheduling over columns (CPU baseline only). */
int oracle_step_omp(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                    oracle_deep_out_t *od, oracle_shallow_out_t *os, int chunk, int nthreads);

/* One column (contiguous arrays of length nlev / nlev+1) with diagnostics and the plume profiles
 * (eta, eta_d at interfaces; may be NULL). */
int oracle_deep_column(int nlev, const oracle_params_t *p, const double *T, const double *q,
                       const double *p_mid, const double *p_int, const double *z, double phis,
                       double dt, double *dTdt, double *dqdt, double *mu, double *md, double *prec,
                       oracle_deep_diag_t *diag, double *eta, double *eta_d);
int oracle_shallow_column(int nlev, const oracle_params_t *p, const double *T, const double *q,
                          const double *p_mid, const double *p_int, const double *z, double phis,
                          double pblh, double tke, double dt, double *dTdt, double *dqdt,
                          double *mu, double *prec, oracle_shallow_diag_t *diag);

/* Undilute parcel diagnostics of the deep trigger for one column: B[k], saturation flag, Tp, qp. */
int oracle_deep_parcel(int nlev, const oracle_params_t *p, const double *T, const double *q,
                       const double *p_mid, const double *p_int, const double *z, double phis,
                       double *B, int32_t *sat, double *Tp, double *qp);

/* Forward-mode directional derivative (dual numbers) of the deep scheme of one column along
 * (dT, dq, dtau, deps) with every branch held where the primal run takes it.  Outputs are the
 * tangents of dTdt, dqdt [nlev] and prec. */
int oracle_deep_column_jvp(int nlev, const oracle_params_t *p, const double *T, const double *q,
                           const double *p_mid, const double *p_int, const double *z, double phis,
                           double dt, const double *dT, const double *dq, double dtau, double deps,
                           double *t_dTdt, double *t_dqdt, double *t_prec);

/* Convective transport of ntr passive tracers by one step (deep, update, shallow on the updated
 * state and on the tracer updated by the deep transport): tracers, tend, deep_tend are
 * [ntr][nlev][ld] level-major like the state; tend = deep + shallow tendency; deep_tend (may be
 * NULL) the deep part.  Returns 0, or -1 on bad arguments. */
int oracle_tracers(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                   int ntr, const double *tracers, double *tend, double *deep_tend);

/* Convective momentum transport by one step: the two wind components wind[2][nlev][ld] (u, then v)
 * carried by the plumes as tracers are, plus the pressure-gradient term of Gregory, Kershaw &
 * Inness (1997) with coefficient cpgf (the plume's wind is pulled towards the environment's as it
 * crosses shear; 0 = passive tracers).  tend, deep_tend (may be NULL): [2][nlev][ld], m s^-2. */
int oracle_momentum(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                    const double *wind, double cpgf, double *tend, double *deep_tend);
/* The common transport of ntr fields with pressure-gradient coefficient cpgf. */
int oracle_transport(int64_t ncol, int nlev, const oracle_params_t *p, const oracle_state_t *s,
                     int ntr, const double *tracers, double cpgf, double *tend, double *deep_tend);

/* Forward-mode derivative of the shallow scheme (S1-S9) of one column along (dT, dq, d eps_sh,
 * d delta_sh), with every integer decision of the run held fixed: source layers, lifting
 * condensation and free-convection levels, the levels counted in CIN, saturation and rain-out
 * flags, the plume top and the base-flux branch with its limiting layer.  Returns the status. */
int oracle_shallow_column_jvp(int nlev, const oracle_params_t *p, const double *T,
                              const double *q, const double *p_mid, const double *p_int,
                              const double *z, double phis, double pblh, double tke, double dt,
                              const double *dT, const double *dq, double deps_sh,
                              double ddelta_sh, double *t_dTdt, double *t_dqdt, double *t_prec);

/* Forward-mode derivative of one column of the step: deep scheme, state update, shallow scheme on
 * the updated state (Algorithm 1).  dpar[4] = tangents of (tau, eps_deep, eps_sh, delta_sh);
 * t_deep and t_shallow [2*nlev+1] receive the tangents of (dTdt, dqdt, prec) of each scheme;
 * status[2] the deep and shallow statuses.  Returns 0, or -1 on bad arguments. */
int oracle_step_column_jvp(int nlev, const oracle_params_t *p, const double *T, const double *q,
                           const double *p_mid, const double *p_int, const double *z, double phis,
                           double pblh, double tke, double dt, const double *dT, const double *dq,
                           const double *dpar, double *t_deep, double *t_shallow,
                           int32_t *status);

/* Thermodynamics (C1 of the scheme). */
double oracle_es(double T);
double oracle_qs(double T, double p);
double oracle_dqsdT(double T, double p);
double oracle_tsat(double H, double p, double T_guess, int *iterations);

#ifdef __cplusplus
}
#endif
#endif
