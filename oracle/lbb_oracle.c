/*
 * Plain FP64 CPU oracle of the hybrid thermal pseudopotential lattice
 * Boltzmann boiling model of Li, Kang, Francois, He and Luo
 * ("Lattice Boltzmann modeling of boiling heat transfer: the boiling curve
 * and the effects of wettability", arXiv:1501.03857).
 *
 * TEST INFRASTRUCTURE ONLY: this is the reference the GPU library is checked
 * against.  Only tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares nothing with the GPU library.
 *
 * It is written for reading, not for speed: every stage of a time step is a
 * separate sweep over the whole lattice that stores its result in a full
 * array, in the order the paper gives them (Sec. 2):
 *
 *   O1  density               rho = sum_a f_a                    Eq. (6)
 *   O2  domain-mean density   rho_ave                            Eq. (9)
 *   O3  pseudopotential       psi from the P-R EOS                Eq. (21), Sec. 2
 *   O4  interaction force     F_m and Q = |F_m|^2/psi^2           Eq. (7), Eq. (8)
 *   O5  fluid-solid force     F_ads                               Eq. (22)
 *   O6  buoyancy              F_b = (rho - rho_ave) g             Eq. (9)
 *   O7  total force           F = F_m + F_ads + F_b
 *   O8  velocity              rho v = sum_a e_a f_a + F/2         Eq. (6)
 *   O9  MRT collision         m* = m - L(m - m_eq) + (I - L/2) S  Eqs. (2), (4), (5), (8)
 *   O10 streaming                                                 Eq. (3)
 *   O11 Zou-He no-slip walls                                      Sec. 3.1
 *   O12 RK4 temperature step  T^{t+1} from K(T), rho, v at t      Eqs. (18)-(20)
 *   O13 wall heat flux        q_w = -lambda dT/dy at y = 0        Sec. 3.2
 *
 * Readings of points the paper leaves open (both this oracle and the GPU
 * library implement the same reading):
 *  - G = -1; pseudopotential weights w = 1/3 (axes), 1/12 (diagonals).
 *  - M is the standard D2Q9 moment basis (rho, e, zeta, jx, qx, jy, qy, pxx,
 *    pxy) with velocities ordered rest, E, N, W, S, NE, NW, SW, SE.
 *  - tau_nu is linear in rho between (rho_V, tau_V) and (rho_L, tau_L).
 *  - Rows 0 and ny-1 are wet wall nodes (Zou-He, zero wall velocity).  No
 *    force acts on them: F_m and Q are zero there as the paper states, and
 *    neither buoyancy nor the fluid-solid force is applied, because a body
 *    force on a Zou-He node turns into a mass flux through the wall.  The
 *    fluid-solid force of Eq. (22) acts on the fluid rows next to the walls
 *    with the wall rows as the solid; this reproduces the contact angles the
 *    paper reports for G_w = 0, 0.065 and 0.105.
 *  - Ghost-layer variant (ghost_layer = 1, Sec. 3.2): F_m and Q of Eq. (7)
 *    are also formed on the wall rows, with a ghost fluid layer beyond each
 *    wall that mirrors the fluid about the wall row, psi(i, -1) = psi(i, 1)
 *    and psi(i, ny) = psi(i, ny-2).  The wall row is then a symmetry line of
 *    psi, so the normal component of F_m vanishes there (up to rounding) and
 *    no body force pushes mass through the no-penetration wall; only the
 *    tangential component acts.  Buoyancy still does not act on the wall
 *    rows, and the fluid-solid force is applied as above.
 *  - rho_ave is recomputed every step over all nodes, wall rows included.
 *  - The temperature equation runs on rows 1..ny-2 with the wall rows held at
 *    their Dirichlet values in every RK stage; the velocity it sees is zero
 *    on the wall rows.  The conduction term is chi (lap T + grad rho . grad T / rho),
 *    i.e. div(lambda grad T)/(rho c_v) with lambda = rho c_v chi.
 *  - The isotropic central stencils on the D2Q9 neighbourhood are the
 *    lattice-weight forms d_x f = 3 sum_a W_a e_ax f(x+e_a),
 *    lap f = 6 sum_a W_a (f(x+e_a) - f(x)).
 *  - q_w uses the second-order one-sided difference at the wall and lambda
 *    of the wall node; it is sampled on the state after each step.
 */
#include "lbb_oracle_internal.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* D2Q9 lattice                                                            */
/* ---------------------------------------------------------------------- */

/* velocities: rest, E, N, W, S, NE, NW, SW, SE */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* lattice weights of the equilibrium (c_s^2 = 1/3) */
static const double WEQ[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* weights w_a of the interaction force, Eq. (7) */
static const double WPSI[9] = {0.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0,
                               1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0};
/* moment basis M (rows: rho, e, zeta, jx, qx, jy, qy, pxx, pxy) */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};
/* squared row norms: M M^T = diag(MNORM), hence M^{-1} = M^T diag(1/MNORM) */
static const double MNORM[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};

#ifdef _OPENMP
#define ORC_PARALLEL_ROWS _Pragma("omp parallel for schedule(static)")
#else
#define ORC_PARALLEL_ROWS
#endif

static _Thread_local char g_err[256];

static void set_err(const char *msg, int64_t t)
{
    snprintf(g_err, sizeof g_err, "%s (step %lld)", msg, (long long)t);
}

const char *orc_last_error(void) { return g_err; }

#ifdef _OPENMP
#include <omp.h>
#endif
/* threads the row loops use (1 without OpenMP) */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_lattice(int32_t ex[9], int32_t ey[9], double W[9], double wpsi[9], double M[81])
{
    for (int a = 0; a < 9; ++a) {
        ex[a] = EX[a];
        ey[a] = EY[a];
        W[a] = WEQ[a];
        wpsi[a] = WPSI[a];
        for (int b = 0; b < 9; ++b) M[9 * a + b] = MM[a][b];
    }
}

/* ---------------------------------------------------------------------- */
/* Peng-Robinson equation of state, Eq. (21)                               */
/* ---------------------------------------------------------------------- */

/* T_c from a = 0.45724 R^2 Tc^2 / p_c and b = 0.0778 R Tc / p_c (Eq. (21)):
 * dividing the two gives a/b = (0.45724/0.0778) R Tc. */
double orc_Tc(double a, double b, double R) { return (a / b) * (0.0778 / 0.45724) / R; }

/* kappa(omega) inside phi(T), Eq. (21) */
double orc_kappa(double omega) { return 0.37464 + 1.54226 * omega - 0.26992 * omega * omega; }

/* phi(T) = [1 + kappa (1 - sqrt(T/Tc))]^2, Eq. (21) */
double orc_phi(double T, double Tc, double kappa)
{
    double s = 1.0 + kappa * (1.0 - sqrt(T / Tc));
    return s * s;
}

/* d phi / dT = -kappa [1 + kappa (1 - sqrt(T/Tc))] / sqrt(T Tc) */
double orc_dphi_dT(double T, double Tc, double kappa)
{
    double s = 1.0 + kappa * (1.0 - sqrt(T / Tc));
    return -kappa * s / sqrt(T * Tc);
}

/* p_EOS = rho R T / (1 - b rho) - a phi(T) rho^2 / (1 + 2 b rho - b^2 rho^2), Eq. (21) */
double orc_p_eos(double rho, double T, double a, double b, double R, double Tc, double kappa)
{
    double phi = orc_phi(T, Tc, kappa);
    return rho * R * T / (1.0 - b * rho) - a * phi * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

/* (dp_EOS/dT)_rho: the coefficient of the pressure-work term of Eq. (18) */
double orc_dp_dT(double rho, double T, double a, double b, double R, double Tc, double kappa)
{
    double dphi = orc_dphi_dT(T, Tc, kappa);
    return rho * R / (1.0 - b * rho) - a * dphi * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

/* (dp_EOS/drho)_T */
double orc_dp_drho(double rho, double T, double a, double b, double R, double Tc, double kappa)
{
    double phi = orc_phi(T, Tc, kappa);
    double den = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    return R * T / ((1.0 - b * rho) * (1.0 - b * rho)) - a * phi * 2.0 * rho * (1.0 + b * rho) / (den * den);
}

/* Antiderivative of p_EOS/rho^2 in rho (used by the equal-area rule):
 *   int rho R T/(1-b rho)/rho^2 = R T ln(rho/(1 - b rho))
 *   int a phi/(2 - (1 - b rho)^2)  = -(a phi/(2 sqrt2 b)) ln((sqrt2 + 1 - b rho)/(sqrt2 - 1 + b rho)) */
static double p_over_rho2_primitive(double rho, double T, double a, double b, double R, double Tc,
                                    double kappa)
{
    const double s2 = sqrt(2.0);
    double phi = orc_phi(T, Tc, kappa);
    double x = 1.0 - b * rho;
    return R * T * log(rho / x) + a * phi / (2.0 * s2 * b) * log((s2 + x) / (s2 - x));
}

/* bisection for g(rho) = 0 on [lo, hi] with g(lo), g(hi) of opposite sign */
typedef double (*orc_fn)(double rho, const double *par);

static double bisect(orc_fn g, const double *par, double lo, double hi)
{
    double glo = g(lo, par);
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double gm = g(mid, par);
        if ((gm < 0) == (glo < 0)) {
            lo = mid;
            glo = gm;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

/* par = {T, a, b, R, Tc, kappa, p0} */
static double g_dpdrho(double rho, const double *q) { return orc_dp_drho(rho, q[0], q[1], q[2], q[3], q[4], q[5]); }
static double g_p_minus(double rho, const double *q) { return orc_p_eos(rho, q[0], q[1], q[2], q[3], q[4], q[5]) - q[6]; }

/* Maxwell construction: rho_V < rho_L with p(rho_V) = p(rho_L) = p_sat and
 * int_{rho_V}^{rho_L} (p - p_sat)/rho^2 d rho = 0 (equal areas in the p-1/rho
 * plane).  Spinodals bracket both branches; the outer bisection is on p_sat,
 * along which the area decreases monotonically. */
int orc_maxwell(double a, double b, double R, double omega, double T, double *rho_V, double *rho_L,
                double *p_sat)
{
    double Tc = orc_Tc(a, b, R), kappa = orc_kappa(omega);
    if (!(T > 0) || !(T < Tc) || !(a > 0) || !(b > 0) || !(R > 0)) return ORC_EINVAL;
    double par[7] = {T, a, b, R, Tc, kappa, 0.0};
    /* locate the two spinodals (sign changes of dp/drho) on a fine scan */
    const int nscan = 200000;
    double rmax = (1.0 / b) * (1.0 - 1e-9);
    double sp[2];
    int nsp = 0;
    double prev_r = rmax / nscan, prev = g_dpdrho(prev_r, par);
    for (int k = 2; k <= nscan && nsp < 2; ++k) {
        double r = rmax * k / nscan, d = g_dpdrho(r, par);
        if ((d < 0) != (prev < 0)) sp[nsp++] = bisect(g_dpdrho, par, prev_r, r);
        prev_r = r;
        prev = d;
    }
    if (nsp != 2) return ORC_EINVAL;
    double p_hi = orc_p_eos(sp[0], T, a, b, R, Tc, kappa); /* local maximum */
    double p_lo = orc_p_eos(sp[1], T, a, b, R, Tc, kappa); /* local minimum */
    if (p_lo < 1e-14 * p_hi) p_lo = 1e-14 * p_hi;
    double lo = p_lo, hi = p_hi, rv = 0, rl = 0;
    for (int it = 0; it < 200; ++it) {
        double p0 = 0.5 * (lo + hi);
        if (p0 <= lo || p0 >= hi) break;
        par[6] = p0;
        rv = bisect(g_p_minus, par, 1e-300, sp[0]);
        rl = bisect(g_p_minus, par, sp[1], rmax);
        double area = (p_over_rho2_primitive(rl, T, a, b, R, Tc, kappa) + p0 / rl) -
                      (p_over_rho2_primitive(rv, T, a, b, R, Tc, kappa) + p0 / rv);
        if (area > 0) lo = p0; else hi = p0;
    }
    *p_sat = 0.5 * (lo + hi);
    *rho_V = rv;
    *rho_L = rl;
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Single-site pieces                                                      */
/* ---------------------------------------------------------------------- */

/* f_eq_a = W_a rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2] (its moments are Eq. (5)) */
void orc_feq(double rho, double ux, double uy, double feq[9])
{
    double u2 = ux * ux + uy * uy;
    for (int a = 0; a < 9; ++a) {
        double eu = EX[a] * ux + EY[a] * uy;
        feq[a] = WEQ[a] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * u2);
    }
}

static double tau_L(const orc_params *p) { return 3.0 * p->nu_L + 0.5; }
static double tau_V(const orc_params *p) { return 3.0 * p->nu_V + 0.5; }

/* relaxation time of the shear moments, linear in rho between the phases */
static double tau_nu(const orc_params *p, double rho)
{
    return tau_V(p) + (rho - p->rho_V) * (tau_L(p) - tau_V(p)) / (p->rho_L - p->rho_V);
}

/* forcing term S of Eq. (8); Q stands for |F_m|^2/psi^2 */
void orc_forcing_moments(const orc_params *p, double vx, double vy, double Fx, double Fy, double Q,
                         double S[9])
{
    double tau_e = 1.0 / p->s_e, tau_z = 1.0 / p->s_zeta;
    double vF = vx * Fx + vy * Fy;
    S[0] = 0.0;
    S[1] = 6.0 * vF + p->sigma * Q / (tau_e - 0.5);
    S[2] = -6.0 * vF - p->sigma * Q / (tau_z - 0.5);
    S[3] = Fx;
    S[4] = -Fx;
    S[5] = Fy;
    S[6] = -Fy;
    S[7] = 2.0 * (vx * Fx - vy * Fy);
    S[8] = vx * Fy + vy * Fx;
}

/* MRT collision at one node, Eqs. (2), (4), (5), (8): f* = M^{-1} m* */
void orc_collide_site(const orc_params *p, const double f[9], double rho, double vx, double vy,
                      double Fx, double Fy, double Q, double fpost[9])
{
    double m[9], meq[9], S[9], ms[9];
    for (int k = 0; k < 9; ++k) {
        m[k] = 0.0;
        for (int a = 0; a < 9; ++a) m[k] += MM[k][a] * f[a];
    }
    double v2 = vx * vx + vy * vy;
    meq[0] = rho;
    meq[1] = rho * (-2.0 + 3.0 * v2);
    meq[2] = rho * (1.0 - 3.0 * v2);
    meq[3] = rho * vx;
    meq[4] = -rho * vx;
    meq[5] = rho * vy;
    meq[6] = -rho * vy;
    meq[7] = rho * (vx * vx - vy * vy);
    meq[8] = rho * vx * vy;
    orc_forcing_moments(p, vx, vy, Fx, Fy, Q, S);
    double s_nu = 1.0 / tau_nu(p, rho);
    double L[9] = {p->s_rho, p->s_e, p->s_zeta, p->s_j, p->s_q, p->s_j, p->s_q, s_nu, s_nu};
    for (int k = 0; k < 9; ++k) ms[k] = m[k] - L[k] * (m[k] - meq[k]) + (1.0 - 0.5 * L[k]) * S[k];
    for (int a = 0; a < 9; ++a) {
        fpost[a] = 0.0;
        for (int k = 0; k < 9; ++k) fpost[a] += MM[k][a] * ms[k] / MNORM[k];
    }
}

/* ---------------------------------------------------------------------- */
/* Stencils                                                                */
/* ---------------------------------------------------------------------- */

static inline int wrap(int i, int n) { return (i % n + n) % n; }

/* isotropic first derivatives and Laplacian on the D2Q9 neighbourhood:
 *   d_x phi = 3 sum_a W_a e_ax phi(x + e_a)
 *   lap phi = 6 sum_a W_a (phi(x + e_a) - phi(x))
 * evaluated where every neighbour exists (interior rows, or every row when
 * periodic_y); other entries are set to 0. */
void orc_grad_iso(int32_t nx, int32_t ny, int32_t periodic_y, const double *phi, double *dx,
                  double *dy, double *lap)
{
    ORC_PARALLEL_ROWS
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            if (!periodic_y && (j == 0 || j == ny - 1)) {
                if (dx) dx[c] = 0.0;
                if (dy) dy[c] = 0.0;
                if (lap) lap[c] = 0.0;
                continue;
            }
            double sx = 0.0, sy = 0.0, sl = 0.0;
            for (int a = 1; a < 9; ++a) {
                int ii = wrap(i + EX[a], nx), jj = periodic_y ? wrap(j + EY[a], ny) : j + EY[a];
                double v = phi[(size_t)jj * nx + ii];
                sx += WEQ[a] * EX[a] * v;
                sy += WEQ[a] * EY[a] * v;
                sl += WEQ[a] * (v - phi[c]);
            }
            if (dx) dx[c] = 3.0 * sx;
            if (dy) dy[c] = 3.0 * sy;
            if (lap) lap[c] = 6.0 * sl;
        }
    }
}

/* O4: F_m = -G psi(x) sum_a w_a psi(x + e_a) e_a (Eq. (7)) and
 * Q = |F_m|^2/psi^2 = G^2 |sum_a w_a psi(x + e_a) e_a|^2 (Eq. (8)); zero on
 * the wall rows, where the paper does not apply the fluid-fluid force,
 * unless ghost_layer is set: then the wall rows get the same sum, with the
 * neighbours beyond the wall taken from the ghost fluid layer, the mirror
 * image of the first fluid row (Sec. 3.2). */
void orc_interaction_force(const orc_params *p, const double *psi, double *Fx, double *Fy, double *Q)
{
    const int nx = p->nx, ny = p->ny;
    ORC_PARALLEL_ROWS
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            if (!p->periodic_y && (j == 0 || j == ny - 1) && !p->ghost_layer) {
                Fx[c] = Fy[c] = Q[c] = 0.0;
                continue;
            }
            double sx = 0.0, sy = 0.0;
            for (int a = 1; a < 9; ++a) {
                int ii = wrap(i + EX[a], nx), jj = p->periodic_y ? wrap(j + EY[a], ny) : j + EY[a];
                if (jj < 0) jj = -jj;                   /* ghost layer below the bottom wall */
                if (jj > ny - 1) jj = 2 * (ny - 1) - jj; /* ghost layer above the top wall */
                double v = psi[(size_t)jj * nx + ii];
                sx += WPSI[a] * v * EX[a];
                sy += WPSI[a] * v * EY[a];
            }
            Fx[c] = -p->G * psi[c] * sx;
            Fy[c] = -p->G * psi[c] * sy;
            Q[c] = p->G * p->G * (sx * sx + sy * sy);
        }
    }
}

/* K(T) of Eq. (18) on the interior rows:
 *   K = -v.grad T + chi (lap T + grad rho . grad T / rho)
 *       - T/(rho c_v) (dp/dT)_rho div v
 * with rho and v frozen at time level t; zero on Dirichlet rows.
 * ws holds 7 scratch arrays of nx*ny doubles. */
static void thermal_rhs_ws(const orc_params *p, const double *rho, const double *vx, const double *vy,
                           const double *T, double *K, double *const ws[7])
{
    const int nx = p->nx, ny = p->ny;
    double Tc = orc_Tc(p->a, p->b, p->R), kappa = orc_kappa(p->omega);
    double chi = p->cv_chi / p->cv;
    double *Tx = ws[0], *Ty = ws[1], *TL = ws[2], *rx = ws[3], *ry = ws[4], *ux_x = ws[5], *uy_y = ws[6];
    orc_grad_iso(nx, ny, p->periodic_y, T, Tx, Ty, TL);
    orc_grad_iso(nx, ny, p->periodic_y, rho, rx, ry, NULL);
    orc_grad_iso(nx, ny, p->periodic_y, vx, ux_x, NULL, NULL);
    orc_grad_iso(nx, ny, p->periodic_y, vy, NULL, uy_y, NULL);
    ORC_PARALLEL_ROWS
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            if (!p->periodic_y && (j == 0 || j == ny - 1)) {
                K[c] = 0.0;
                continue;
            }
            double adv = vx[c] * Tx[c] + vy[c] * Ty[c];
            double cond = chi * (TL[c] + (rx[c] * Tx[c] + ry[c] * Ty[c]) / rho[c]);
            double divv = ux_x[c] + uy_y[c];
            double dpdT = orc_dp_dT(rho[c], T[c], p->a, p->b, p->R, Tc, kappa);
            double work = T[c] / (rho[c] * p->cv) * dpdT * divv;
            K[c] = -adv + cond - work;
        }
    }
}

void orc_thermal_rhs(const orc_params *p, const double *rho, const double *vx, const double *vy,
                     const double *T, double *K)
{
    const size_t n = (size_t)p->nx * p->ny;
    double *ws[7];
    for (int k = 0; k < 7; ++k) ws[k] = malloc(n * sizeof(double));
    thermal_rhs_ws(p, rho, vx, vy, T, K, ws);
    for (int k = 0; k < 7; ++k) free(ws[k]);
}

/* ---------------------------------------------------------------------- */
/* Whole-domain state                                                      */
/* ---------------------------------------------------------------------- */

#define F_AT(s, a, c) ((s)->f[(size_t)(a) * (size_t)(s)->p.nx * (s)->p.ny + (c)])

static int params_ok(const orc_params *p)
{
    if (p->nx < 3) return 0;
    if (p->periodic_y ? p->ny < 3 : p->ny < 4) return 0;
    double v[] = {p->a, p->b, p->R, p->omega, p->Ts_over_Tc, p->G, p->sigma, p->s_rho, p->s_e,
                  p->s_zeta, p->s_j, p->s_q, p->nu_L, p->nu_V, p->rho_L, p->rho_V, p->cv,
                  p->cv_chi, p->g, p->Gw_bottom, p->Gw_top};
    for (size_t k = 0; k < sizeof v / sizeof v[0]; ++k)
        if (!isfinite(v[k])) return 0;
    if (!(p->a > 0 && p->b > 0 && p->R > 0 && p->Ts_over_Tc > 0 && p->cv > 0)) return 0;
    if (!(p->G < 0)) return 0;
    if (!(p->rho_L != p->rho_V)) return 0;
    if (!(p->s_e > 0 && p->s_zeta > 0 && p->s_e != 2.0 && p->s_zeta != 2.0)) return 0;
    if (p->thermal_mode < ORC_COUPLED || p->thermal_mode > ORC_THERMAL_ONLY) return 0;
    if (p->ghost_layer != 0 && p->ghost_layer != 1) return 0;
    return 1;
}

static void heat_flux_sample(orc_state *s, double *q_local);

int orc_create(const orc_params *p, const double *rho0, const double *ux0, const double *uy0,
               const double *T0, const double *T_bottom, orc_state **out)
{
    *out = NULL;
    if (!p || !rho0 || !params_ok(p)) {
        set_err("invalid parameters", 0);
        return ORC_EINVAL;
    }
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    orc_state *s = calloc(1, sizeof *s);
    if (!s) return ORC_ENOMEM;
    s->p = *p;
    s->Tc = orc_Tc(p->a, p->b, p->R);
    s->kappa = orc_kappa(p->omega);
    s->Ts = p->Ts_over_Tc * s->Tc;
    s->f = malloc(9 * n * sizeof(double));
    s->fpost = malloc(9 * n * sizeof(double));
    s->T = malloc(n * sizeof(double));
    s->Tb = malloc((size_t)nx * sizeof(double));
    double **work[] = {&s->rho, &s->psi, &s->Fx, &s->Fy, &s->Q, &s->vx, &s->vy, &s->vTx, &s->vTy,
                       &s->Tst, &s->h, &s->acc};
    int ok = s->f && s->fpost && s->T && s->Tb;
    for (size_t k = 0; k < sizeof work / sizeof work[0]; ++k) {
        *work[k] = malloc(n * sizeof(double));
        ok = ok && *work[k];
    }
    for (int k = 0; k < 7; ++k) {
        s->ws[k] = malloc(n * sizeof(double));
        ok = ok && s->ws[k];
    }
    if (!ok) {
        orc_destroy(s);
        return ORC_ENOMEM;
    }
    for (int i = 0; i < nx; ++i) s->Tb[i] = T_bottom ? T_bottom[i] : s->Ts;
    for (size_t c = 0; c < n; ++c) {
        double feq[9];
        if (!(rho0[c] > 0) || !isfinite(rho0[c]) || p->b * rho0[c] >= 1.0) {
            orc_destroy(s);
            set_err("invalid initial density", 0);
            return ORC_EINVAL;
        }
        orc_feq(rho0[c], ux0 ? ux0[c] : 0.0, uy0 ? uy0[c] : 0.0, feq);
        for (int a = 0; a < 9; ++a) F_AT(s, a, c) = feq[a];
        s->T[c] = T0 ? T0[c] : s->Ts;
    }
    if (!p->periodic_y) {
        for (int i = 0; i < nx; ++i) {
            s->T[i] = s->Tb[i];
            s->T[(size_t)(ny - 1) * nx + i] = s->Ts;
        }
    }
    for (size_t c = 0; c < n; ++c) {
        if (!(s->T[c] > 0) || !isfinite(s->T[c])) {
            orc_destroy(s);
            set_err("invalid initial temperature", 0);
            return ORC_EINVAL;
        }
    }
    heat_flux_sample(s, NULL);
    *out = s;
    return ORC_OK;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    free(s->f); free(s->fpost); free(s->T); free(s->Tb);
    free(s->rho); free(s->psi); free(s->Fx); free(s->Fy); free(s->Q); free(s->vx); free(s->vy);
    free(s->vTx); free(s->vTy); free(s->Tst); free(s->h); free(s->acc);
    for (int k = 0; k < 7; ++k) free(s->ws[k]);
    free(s);
}

int64_t orc_time(const orc_state *s) { return s->t; }

void orc_constants(const orc_state *s, double *Tc, double *kappa, double *Ts)
{
    if (Tc) *Tc = s->Tc;
    if (kappa) *kappa = s->kappa;
    if (Ts) *Ts = s->Ts;
}

/* O1 density, Eq. (6) */
static int density(orc_state *s)
{
    const size_t n = (size_t)s->p.nx * s->p.ny;
    int bad = 0;
    for (size_t c = 0; c < n; ++c) {
        double r = 0.0;
        for (int a = 0; a < 9; ++a) r += F_AT(s, a, c);
        s->rho[c] = r;
        if (!(r > 0) || !isfinite(r)) bad = 1;
    }
    return bad ? ORC_ENONFINITE : ORC_OK;
}

/* O3 psi = sqrt(2 (p_EOS - rho c_s^2) / (G c^2)) (Sec. 2, Eq. (21)) */
static double round_storage(int bits, double x)
{
    if (bits == 0) return x;
    if (bits == 24) return (double)(float)x;
    const double c = ldexp(1.0, 53 - bits) + 1.0;
    const double y = c * x;
    return y - (y - x);
}

static int pseudopotential(orc_state *s)
{
    const orc_params *p = &s->p;
    const size_t n = (size_t)p->nx * p->ny;
    int bad = 0;
    for (size_t c = 0; c < n; ++c) {
        double pe = orc_p_eos(s->rho[c], s->T[c], p->a, p->b, p->R, s->Tc, s->kappa);
        double r = 2.0 * (pe - s->rho[c] / 3.0) / p->G;
        if (!(r >= 0) || !isfinite(r)) bad = 1;
        s->psi[c] = sqrt(r);
        if (s->store_bits != 24) s->psi[c] = round_storage(s->store_bits, s->psi[c]);
    }
    return bad ? ORC_ENONFINITE : ORC_OK;
}

/* O5 F_ads = -G_w psi(x) sum_a omega_a S(x + e_a) e_a with S = psi(x) s(x + e_a)
 * and omega_a = w_a/3, Eq. (22).  The wall rows are the solid (s = 1); the
 * force acts on the fluid nodes next to them.  Each wall carries its own G_w. */
static void fluid_solid_force(const orc_state *s, int i, int j, double *fx, double *fy)
{
    const orc_params *p = &s->p;
    *fx = *fy = 0.0;
    if (p->periodic_y || j == 0 || j == p->ny - 1) return;
    double psi = s->psi[(size_t)j * p->nx + i];
    double sx = 0.0, sy = 0.0;
    for (int a = 1; a < 9; ++a) {
        int jj = j + EY[a];
        double Gw_s = 0.0; /* G_w times the switch s of the neighbour */
        if (jj == 0) Gw_s = p->Gw_bottom;
        if (jj == p->ny - 1) Gw_s = p->Gw_top;
        double omega = WPSI[a] / 3.0;
        sx += omega * Gw_s * psi * EX[a];
        sy += omega * Gw_s * psi * EY[a];
    }
    *fx = -psi * sx;
    *fy = -psi * sy;
}

/* O10 + O11: streaming, Eq. (3), then Zou-He with zero wall velocity */
static void stream_and_walls(orc_state *s)
{
    const int nx = s->p.nx, ny = s->p.ny;
    const size_t n = (size_t)nx * ny;
    ORC_PARALLEL_ROWS
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            for (int a = 0; a < 9; ++a) {
                int is = wrap(i - EX[a], nx);
                int js = j - EY[a];
                if (s->p.periodic_y) js = wrap(js, ny);
                if (js < 0 || js > ny - 1) continue; /* unknown: set by the wall rule */
                s->f[(size_t)a * n + c] = s->fpost[(size_t)a * n + (size_t)js * nx + is];
            }
        }
    }
    if (s->p.periodic_y) return;
    for (int i = 0; i < nx; ++i) {
        /* bottom wall, unknowns 2 (N), 5 (NE), 6 (NW) */
        size_t c = (size_t)i;
        double d13 = F_AT(s, 1, c) - F_AT(s, 3, c);
        F_AT(s, 2, c) = F_AT(s, 4, c);
        F_AT(s, 5, c) = F_AT(s, 7, c) - 0.5 * d13;
        F_AT(s, 6, c) = F_AT(s, 8, c) + 0.5 * d13;
        /* top wall, unknowns 4 (S), 7 (SW), 8 (SE) */
        c = (size_t)(ny - 1) * nx + i;
        d13 = F_AT(s, 1, c) - F_AT(s, 3, c);
        F_AT(s, 4, c) = F_AT(s, 2, c);
        F_AT(s, 7, c) = F_AT(s, 5, c) + 0.5 * d13;
        F_AT(s, 8, c) = F_AT(s, 6, c) - 0.5 * d13;
    }
}

/* O12: classical RK4 of Eqs. (19)-(20); rho and v frozen at level t, wall
 * rows held at their Dirichlet values in every stage. */
static int thermal_rk4(orc_state *s)
{
    const orc_params *p = &s->p;
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    const double stage_c[4] = {0.0, 0.5, 0.5, 1.0};
    const double stage_w[4] = {1.0, 2.0, 2.0, 1.0};
    for (size_t c = 0; c < n; ++c) s->acc[c] = 0.0;
    for (int k = 0; k < 4; ++k) {
        for (size_t c = 0; c < n; ++c) s->Tst[c] = s->T[c] + stage_c[k] * (k ? s->h[c] : 0.0);
        thermal_rhs_ws(p, s->rho, s->vTx, s->vTy, s->Tst, s->h, s->ws);
        for (size_t c = 0; c < n; ++c) s->acc[c] += stage_w[k] * s->h[c];
    }
    int bad = 0;
    for (int j = 0; j < ny; ++j) {
        if (!p->periodic_y && (j == 0 || j == ny - 1)) continue;
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            s->T[c] = s->T[c] + s->acc[c] / 6.0;
            if (s->store_bits != 24) s->T[c] = round_storage(s->store_bits, s->T[c]);
            if (!(s->T[c] > 0) || !isfinite(s->T[c])) bad = 1;
        }
    }
    return bad ? ORC_ENONFINITE : ORC_OK;
}

/* O13: q_w(x) = -lambda dT/dy at y = 0 with lambda = rho c_v chi and the
 * second-order one-sided difference; q = mean over x (Sec. 3.2). */
static void heat_flux_sample(orc_state *s, double *q_local)
{
    const orc_params *p = &s->p;
    const int nx = p->nx;
    if (p->periodic_y) {
        s->q_now = 0.0;
        return;
    }
    double sum = 0.0;
    for (int i = 0; i < nx; ++i) {
        double rho0 = 0.0;
        for (int a = 0; a < 9; ++a) rho0 += F_AT(s, a, (size_t)i);
        double dTdy = (-3.0 * s->T[i] + 4.0 * s->T[(size_t)nx + i] - s->T[(size_t)2 * nx + i]) / 2.0;
        double qw = -p->cv_chi * rho0 * dTdy;
        if (q_local) q_local[i] = qw;
        sum += qw;
    }
    s->q_now = sum / nx;
}

static int one_step(orc_state *s)
{
    const orc_params *p = &s->p;
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    int rc;

    /* O1 */
    if ((rc = density(s)) != ORC_OK) {
        set_err("non-positive or non-finite density", s->t);
        return rc;
    }

    if (p->thermal_mode == ORC_THERMAL_ONLY) {
        /* flow frozen: the temperature equation sees rho and sum_a e_a f_a / rho */
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                size_t c = (size_t)j * nx + i;
                double jx = 0.0, jy = 0.0;
                for (int a = 0; a < 9; ++a) {
                    jx += EX[a] * F_AT(s, a, c);
                    jy += EY[a] * F_AT(s, a, c);
                }
                int wall = !p->periodic_y && (j == 0 || j == ny - 1);
                s->vTx[c] = wall ? 0.0 : jx / s->rho[c];
                s->vTy[c] = wall ? 0.0 : jy / s->rho[c];
            }
        }
    } else {
        /* O2 */
        double mass = 0.0;
        for (size_t c = 0; c < n; ++c) mass += s->rho[c];
        double rho_ave = mass / (double)n;
        /* O3 */
        if ((rc = pseudopotential(s)) != ORC_OK) {
            set_err("negative or non-finite pseudopotential radicand", s->t);
            return rc;
        }
        /* O4 */
        orc_interaction_force(p, s->psi, s->Fx, s->Fy, s->Q);
        /* O5-O8 */
        ORC_PARALLEL_ROWS
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                size_t c = (size_t)j * nx + i;
                double fax, fay;
                fluid_solid_force(s, i, j, &fax, &fay);
                int wall = !p->periodic_y && (j == 0 || j == ny - 1);
                /* O6 buoyancy (none on the wall rows: see the file header) */
                double fbx = 0.0, fby = wall ? 0.0 : -(s->rho[c] - rho_ave) * p->g;
                s->Fx[c] += fax + fbx;
                s->Fy[c] += fay + fby;
                double jx = 0.0, jy = 0.0;
                for (int a = 0; a < 9; ++a) {
                    jx += EX[a] * F_AT(s, a, c);
                    jy += EY[a] * F_AT(s, a, c);
                }
                s->vx[c] = (jx + 0.5 * s->Fx[c]) / s->rho[c];
                s->vy[c] = (jy + 0.5 * s->Fy[c]) / s->rho[c];
                s->vTx[c] = wall ? 0.0 : s->vx[c];
                s->vTy[c] = wall ? 0.0 : s->vy[c];
            }
        }
        /* O9 */
        ORC_PARALLEL_ROWS
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                size_t c = (size_t)j * nx + i;
                double fl[9], fp[9];
                for (int a = 0; a < 9; ++a) fl[a] = F_AT(s, a, c);
                orc_collide_site(p, fl, s->rho[c], s->vx[c], s->vy[c], s->Fx[c], s->Fy[c], s->Q[c], fp);
                for (int a = 0; a < 9; ++a) s->fpost[(size_t)a * n + c] = round_storage(s->store_bits, fp[a]);
            }
        }
    }

    /* O12 uses rho and v of level t, so it runs before f is overwritten */
    if (p->thermal_mode != ORC_ISOTHERMAL) {
        if ((rc = thermal_rk4(s)) != ORC_OK) {
            set_err("non-positive or non-finite temperature", s->t);
            return rc;
        }
    }

    /* O10, O11 */
    if (p->thermal_mode != ORC_THERMAL_ONLY) stream_and_walls(s);

    s->t += 1;
    /* O13 */
    heat_flux_sample(s, NULL);
    s->q_sum += s->q_now;
    s->n_samples += 1;
    return ORC_OK;
}

int orc_step(orc_state *s, int64_t n)
{
    if (n < 0) {
        set_err("negative step count", s->t);
        return ORC_EINVAL;
    }
    for (int64_t k = 0; k < n; ++k) {
        int rc = one_step(s);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

/* Macroscopic fields of the current state: rho = sum f, v of Eq. (6) with
 * the force of the current state, T, and f itself. */
void orc_fields(const orc_state *cs, double *rho, double *ux, double *uy, double *T, double *f)
{
    orc_state *s = (orc_state *)cs; /* work arrays only */
    const orc_params *p = &s->p;
    const size_t n = (size_t)p->nx * p->ny;
    density(s);
    if (ux || uy) {
        if (p->thermal_mode == ORC_THERMAL_ONLY) {
            for (size_t c = 0; c < n; ++c) s->Fx[c] = s->Fy[c] = 0.0;
        } else {
            double mass = 0.0;
            for (size_t c = 0; c < n; ++c) mass += s->rho[c];
            double rho_ave = mass / (double)n;
            pseudopotential(s);
            orc_interaction_force(p, s->psi, s->Fx, s->Fy, s->Q);
            for (int j = 0; j < p->ny; ++j) {
                for (int i = 0; i < p->nx; ++i) {
                    size_t c = (size_t)j * p->nx + i;
                    double fax, fay;
                    fluid_solid_force(s, i, j, &fax, &fay);
                    int wall = !p->periodic_y && (j == 0 || j == p->ny - 1);
                    s->Fx[c] += fax;
                    s->Fy[c] += fay - (wall ? 0.0 : (s->rho[c] - rho_ave) * p->g);
                }
            }
        }
        for (size_t c = 0; c < n; ++c) {
            double jx = 0.0, jy = 0.0;
            for (int a = 0; a < 9; ++a) {
                jx += EX[a] * F_AT(s, a, c);
                jy += EY[a] * F_AT(s, a, c);
            }
            if (ux) ux[c] = (jx + 0.5 * s->Fx[c]) / s->rho[c];
            if (uy) uy[c] = (jy + 0.5 * s->Fy[c]) / s->rho[c];
        }
    }
    if (rho) memcpy(rho, s->rho, n * sizeof(double));
    if (T) memcpy(T, s->T, n * sizeof(double));
    if (f) memcpy(f, s->f, 9 * n * sizeof(double));
}

void orc_heat_flux(const orc_state *cs, double *q_now, double *q_sum, int64_t *n_samples, double *q_local)
{
    orc_state *s = (orc_state *)cs;
    double keep = s->q_now;
    if (q_local) heat_flux_sample(s, q_local);
    s->q_now = keep;
    if (q_now) *q_now = s->q_now;
    if (q_sum) *q_sum = s->q_sum;
    if (n_samples) *n_samples = s->n_samples;
}

void orc_reset_average(orc_state *s)
{
    s->q_sum = 0.0;
    s->n_samples = 0;
}

void orc_set_heater(orc_state *s, const double *T_bottom)
{
    for (int i = 0; i < s->p.nx; ++i) {
        s->Tb[i] = T_bottom ? T_bottom[i] : s->Ts;
        if (!s->p.periodic_y) s->T[i] = s->Tb[i];
    }
}

void orc_set_wettability(orc_state *s, double Gw_bottom) { s->p.Gw_bottom = Gw_bottom; }

/* Rounding model (the arithmetic stays FP64).  bits = 24: the post-collision
 * populations are rounded to the nearest float before they stream (FP32
 * storage of f).  1 <= bits <= 52: the post-collision populations, the
 * pseudopotential and the new temperature are rounded to `bits` significant
 * bits by Veltkamp's splitting, x -> c - (c - x) with c = (2^(53-bits) + 1) x:
 * at 52, about one extra FP64 rounding of every quantity a step hands from
 * one stage to the next.  0 turns the model off (the default).  Used to
 * measure how far rounding of that size alone moves the trajectory. */
int orc_set_storage_rounding(orc_state *s, int bits)
{
    if (bits < 0 || bits > 52) return ORC_EINVAL;
    s->store_bits = bits;
    return ORC_OK;
}

int64_t orc_state_size(const orc_state *s) { return (int64_t)10 * s->p.nx * s->p.ny + s->p.nx + 4; }

void orc_save(const orc_state *s, double *buf)
{
    const size_t n = (size_t)s->p.nx * s->p.ny;
    memcpy(buf, s->f, 9 * n * sizeof(double));
    memcpy(buf + 9 * n, s->T, n * sizeof(double));
    memcpy(buf + 10 * n, s->Tb, (size_t)s->p.nx * sizeof(double));
    double *tail = buf + 10 * n + s->p.nx;
    tail[0] = (double)s->t;
    tail[1] = s->q_now;
    tail[2] = s->q_sum;
    tail[3] = (double)s->n_samples;
}

void orc_load(orc_state *s, const double *buf)
{
    const size_t n = (size_t)s->p.nx * s->p.ny;
    memcpy(s->f, buf, 9 * n * sizeof(double));
    memcpy(s->T, buf + 9 * n, n * sizeof(double));
    memcpy(s->Tb, buf + 10 * n, (size_t)s->p.nx * sizeof(double));
    const double *tail = buf + 10 * n + s->p.nx;
    s->t = (int64_t)tail[0];
    s->q_now = tail[1];
    s->q_sum = tail[2];
    s->n_samples = (int64_t)tail[3];
}
