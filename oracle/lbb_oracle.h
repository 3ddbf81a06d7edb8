/*
 * Plain FP64 CPU oracle of the hybrid thermal pseudopotential lattice
 * Boltzmann boiling model (Li, Kang, Francois, He, Luo, arXiv:1501.03857).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * Every routine follows the paper's equations in the paper's order; where the
 * paper is silent the reading adopted is stated next to the code.
 */
#ifndef LBB_ORACLE_H
#define LBB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_COUPLED = 0, ORC_ISOTHERMAL = 1, ORC_THERMAL_ONLY = 2 };

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_ENOMEM = -2,
    ORC_ENONFINITE = -4
};

/* Model parameters, lattice units (Sec. 3.1: c = dx = dt = 1). */
typedef struct orc_params {
    int32_t nx, ny;
    /* Peng-Robinson EOS, Eq. (21) */
    double a, b, R, omega;
    double Ts_over_Tc;      /* saturation temperature T_s / T_c          */
    /* pseudopotential force, Eq. (7), and the improved forcing, Eq. (8) */
    double G, sigma;
    /* relaxation rates of Eq. (4) (the viscous rate follows from nu)     */
    double s_rho, s_e, s_zeta, s_j, s_q;
    double nu_L, nu_V;      /* kinematic viscosities (Sec. 3.1)          */
    double rho_L, rho_V;    /* coexistence densities used for tau(rho)   */
    /* temperature equation, Eq. (18) */
    double cv, cv_chi;      /* c_v and c_v*chi (lambda = rho*c_v*chi)    */
    double g;               /* gravity magnitude, Eq. (9)                */
    double Gw_bottom, Gw_top; /* fluid-solid strength, Eq. (22)          */
    int32_t periodic_y;     /* 1: no walls, periodic in y (test mode)    */
    int32_t thermal_mode;   /* ORC_COUPLED / ORC_ISOTHERMAL / ORC_THERMAL_ONLY */
    int32_t ghost_layer;    /* 1: F_m of Eq. (7) also on the wall rows, with a
                               ghost fluid layer beyond each wall mirroring
                               the first fluid row (Sec. 3.2)              */
} orc_params;

typedef struct orc_state orc_state;

/* ---- EOS utilities (Eq. (21)) ---------------------------------------- */
double orc_Tc(double a, double b, double R);
double orc_kappa(double omega);
double orc_phi(double T, double Tc, double kappa);
double orc_dphi_dT(double T, double Tc, double kappa);
double orc_p_eos(double rho, double T, double a, double b, double R, double Tc, double kappa);
double orc_dp_dT(double rho, double T, double a, double b, double R, double Tc, double kappa);
double orc_dp_drho(double rho, double T, double a, double b, double R, double Tc, double kappa);
/* Maxwell equal-area coexistence at temperature T; returns 0 on success. */
int orc_maxwell(double a, double b, double R, double omega, double T,
                double *rho_V, double *rho_L, double *p_sat);

/* ---- lattice tables (for identity checks) ---------------------------- */
void orc_lattice(int32_t ex[9], int32_t ey[9], double W[9], double wpsi[9], double M[81]);

/* ---- single-site and operator building blocks ------------------------ */
void orc_feq(double rho, double ux, double uy, double feq[9]);
void orc_collide_site(const orc_params *p, const double f[9], double rho, double vx, double vy,
                      double Fx, double Fy, double Q, double fpost[9]);
void orc_forcing_moments(const orc_params *p, double vx, double vy, double Fx, double Fy,
                         double Q, double S[9]);
/* Interaction force and Q = |F_m|^2/psi^2 from a psi field (rows 1..ny-2,
 * or every row when periodic_y).  Arrays are row-major [ny][nx]. */
void orc_interaction_force(const orc_params *p, const double *psi, double *Fx, double *Fy, double *Q);
/* Right-hand side K(T) of Eq. (18) on the interior rows (0 on wall rows). */
void orc_thermal_rhs(const orc_params *p, const double *rho, const double *vx, const double *vy,
                     const double *T, double *K);
void orc_grad_iso(int32_t nx, int32_t ny, int32_t periodic_y, const double *phi,
                  double *dx, double *dy, double *lap);

/* ---- whole-domain time stepping -------------------------------------- */
/* rho0 [ny*nx] is required; ux0/uy0/T0 may be NULL (zero velocity; T = T_s).
 * T_bottom [nx] may be NULL (T_s).  The wall rows of T are set to T_bottom
 * (row 0) and T_s (row ny-1) unless periodic_y. */
int orc_create(const orc_params *p, const double *rho0, const double *ux0, const double *uy0,
               const double *T0, const double *T_bottom, orc_state **out);
void orc_destroy(orc_state *s);
int orc_step(orc_state *s, int64_t n);
int64_t orc_time(const orc_state *s);
/* Macroscopic fields of the current state (any pointer may be NULL). */
void orc_fields(const orc_state *s, double *rho, double *ux, double *uy, double *T, double *f);
void orc_heat_flux(const orc_state *s, double *q_now, double *q_sum, int64_t *n_samples, double *q_local);
void orc_reset_average(orc_state *s);
void orc_set_heater(orc_state *s, const double *T_bottom);
void orc_set_wettability(orc_state *s, double Gw_bottom);
/* Rounding model: 24 rounds the post-collision populations to FP32 each step
 * (FP32 storage of f); 1..52 rounds the post-collision populations, psi and
 * the new T to that many significant bits (about one extra FP64 rounding of
 * each at 52); 0 turns it off (the default).  The arithmetic stays FP64. */
int orc_set_storage_rounding(orc_state *s, int bits);
const char *orc_last_error(void);
int orc_num_threads(void);
void orc_constants(const orc_state *s, double *Tc, double *kappa, double *Ts);
/* ---- discrete adjoint (lbb_oracle_adjoint.c) ------------------------- */
/* J = (1/N) sum_{n=1..N} q^n over N steps from the current state (left
 * unchanged) and dJ/dT_b [nx], dJ/dG_w,bottom; checkpoints every K steps. */
int orc_adjoint(const orc_state *s, int64_t N, int64_t K, double *J, double *dJ_dTb, double *dJ_dGw);
/* One step transposed at the current state: adjoints (lf1 [9n], lT1 [n]) of
 * the next state -> adjoints (lf0, lT0) of the current one; *gGw += dJ/dG_w. */
int orc_step_vjp(const orc_state *s, const double *lf1, const double *lT1, double *lf0, double *lT0,
                 double *gGw);

/* ---- three-dimensional extension on D3Q19 (lbb_oracle3d.c) ----------- */
/* Velocities e[3a..3a+2], weights W[a] and the moment basis M[19k + a]. */
void orc3_lattice(int32_t e[57], double W[19], double M[361]);
void orc3_feq(double rho, const double v[3], double feq[19]);
void orc3_collide_site(const orc_params *p, const double f[19], double rho, const double v[3],
                       const double F[3], double Q, double fpost[19]);
/* isotropic D3Q19 stencils of phi [nz][ny][nx] (0 on wall rows) */
void orc3_grad_iso(int32_t nx, int32_t ny, int32_t nz, int32_t periodic_y, const double *phi, double *dx,
                   double *dy, double *dz, double *lap);
typedef struct orc3_state orc3_state;
/* Arrays are [nz][ny][nx] (x fastest); f is [19][nz][ny][nx]; T_bottom is
 * [nz][nx].  Walls at y = 0 and y = ny-1 unless periodic_y; x and z are
 * periodic.  ghost_layer must be 0. */
int orc3_create(const orc_params *p, int32_t nz, const double *rho0, const double *ux0, const double *uy0,
                const double *uz0, const double *T0, const double *T_bottom, orc3_state **out);
void orc3_destroy(orc3_state *s);
int orc3_step(orc3_state *s, int64_t n);
int64_t orc3_time(const orc3_state *s);
void orc3_fields(const orc3_state *s, double *rho, double *ux, double *uy, double *uz, double *T, double *f);
void orc3_heat_flux(const orc3_state *s, double *q_now, double *q_sum, int64_t *n_samples, double *q_local);
void orc3_reset_average(orc3_state *s);
void orc3_set_heater(orc3_state *s, const double *T_bottom);
int orc3_set_storage_rounding(orc3_state *s, int bits);

/* Copy/restore the full state (f, T, time, heat-flux accumulators). */
int64_t orc_state_size(const orc_state *s);
void orc_save(const orc_state *s, double *buf);
void orc_load(orc_state *s, const double *buf);

#ifdef __cplusplus
}
#endif
#endif
